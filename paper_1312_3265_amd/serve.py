"""Continuous-batching solve server over the resident multi-slot CG solver.

Requests (lattice size, formulation, mass, source, tolerance) arrive over
time.  Gauge fields stay resident in HBM, one per lattice size.  Requests that
share a gauge field and formulation form a group; a group's requests run in
solver pools (``Batch``: a multi-slot solver whose every stencil launch serves
all of its running systems).  A request takes a free slot of one of its
group's pools as soon as one frees up, while the other slots keep iterating;
finished systems are harvested between chunks of iterations.  Each pool runs
in its own host thread on its own HIP stream, so the pools' kernels overlap
on the device (the library calls release the GIL).

HBM admission by footprint: the server holds one budget of workspace bytes
for all groups.  A request's footprint is what one more system of its group
adds to a pool's workspace (``solve_workspace_bytes``).  When a group has more
waiting requests than free slots, the scheduler opens a new pool for it with
as many slots as the waiting requests need (at least ``min_pool``, at most
``slots``) and the unused budget allows, but at least one; groups are served
in the order of their longest-waiting request.  A group that cannot open even
a one-slot pool waits; meanwhile the pools of the other groups that have no
request waiting take no new request, close once their running systems have
finished, and return their bytes to the budget, so a lattice size without
traffic lends its memory to a busy one.  Running pools are never preempted:
a group whose queue never empties keeps its pools, and a starved group waits
until the other groups' queues drain.  A request is rejected only if a
one-slot pool of its group exceeds the whole budget, or its lattice is not
resident.

Cancellation: ``cancel(request_id)`` (from any thread, or at a request's
``cancel_at`` time) drops a request that is still queued, and frees the slot
of one that is running at the next chunk boundary; a request that finished
first is delivered as usual.

The arithmetic all happens in the library; this module only schedules.
"""
from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import FEAT_CORNERS, FEAT_EO, FEAT_F32, FEAT_Q16, WILSON, Batch, Gauge, Lattice, \
    SLOT_DONE, SLOT_FAILED, SolveOpts, _torch, solve_opts, solve_workspace_bytes


@dataclass
class Request:
    id: int
    dims: tuple
    formulation: int
    mass: float
    source: object            # canonical complex128 field (numpy or torch)
    tol: float
    arrival: float = 0.0      # seconds after the server's start
    maxiter: int = 100000
    cancel_at: float = None   # seconds after the server's start: cancel then


@dataclass
class Result:
    id: int
    x: object
    info: dict
    arrival: float
    admitted: float
    finished: float

    @property
    def latency(self):
        return self.finished - self.arrival


class Ledger:
    """Workspace bytes handed out against a fixed budget.  ``fit(ws, want)``
    is the largest n <= want with ws(n) within what is left (0 if none)."""

    def __init__(self, budget):
        self.budget = int(budget)
        self.used = 0
        self.peak = 0

    def left(self):
        return self.budget - self.used

    def fit(self, ws, want):
        n = int(want)
        while n > 0 and ws(n) > self.left():
            n -= 1
        return n

    def take(self, nbytes):
        if nbytes > self.left():
            raise ValueError("workspace exceeds the budget")
        self.used += int(nbytes)
        self.peak = max(self.peak, self.used)

    def give(self, nbytes):
        self.used -= int(nbytes)


@dataclass
class _Group:
    key: tuple
    waiting: "collections.deque" = field(default_factory=collections.deque)
    pools: list = field(default_factory=list)


@dataclass
class _Pool:
    group: _Group
    batch: Batch
    stream: object
    nbytes: int
    free: list
    slot_req: dict = field(default_factory=dict)
    retire: bool = False       # set by the scheduler: run nothing new, then exit
    closed: bool = False       # set by the worker when it has exited
    thread: threading.Thread = None


class SolveServer:
    """Serve solve requests on resident gauge fields with continuous batching.

    fields: {dims: canonical gauge field (numpy or torch)}; opts: solver
    options (default FP32 Krylov vectors, 12-real links, FP64 reliable
    updates); mem_budget: bytes of HBM for solver workspaces (all groups);
    slots: upper bound on slots per pool; min_pool: slots a new pool asks for
    at least (when they fit); chunk: iterations per step; evenodd: Wilson
    requests (r = 1) are solved even-odd preconditioned (the gauge fields then
    carry even-odd link copies); every solution still meets eq. (2)'s
    residual.
    """

    def __init__(self, fields, opts=None, mem_budget=8 << 30, slots=16, chunk=16, r=1.0,
                 g55=0, evenodd=False, min_pool=1):
        self.torch = _torch()
        self.opts = opts or solve_opts(precision=1, links=12, poll_interval=chunk)
        self.evenodd = bool(evenodd) and r == 1.0
        self.chunk = chunk
        self.r = r
        self.g55 = g55
        self.max_slots = max(1, int(slots))
        self.min_pool = max(1, min(int(min_pool), self.max_slots))
        self.ledger = Ledger(mem_budget)
        self.mem_budget = self.ledger.budget
        self.lattices = {}
        self.gauges = {}
        for dims, U in fields.items():
            dims = tuple(dims)
            lat = Lattice(dims)
            self.lattices[dims] = lat
            feats = FEAT_CORNERS | FEAT_F32 | FEAT_Q16 | (FEAT_EO if self.evenodd else 0)
            self.gauges[dims] = Gauge(lat, U, feats)
        self.groups = {}
        self.results = []
        self.rejected = []
        self.cancelled = []       # (request id, "queued" or "running", seconds)
        self.pools_opened = 0
        self.pools_closed = 0
        self.pools_lent = 0       # pools closed early to give their memory to another group
        self._cancel = set()
        self._lock = threading.Lock()
        self._t0 = None
        self._stop = False
        self._ws_cache = {}

    # ----------------------------------------------------------- admission
    def opts_for(self, formulation):
        """The solver options of a (dims, formulation) group."""
        if not (self.evenodd and formulation == WILSON):
            return self.opts
        o = SolveOpts.from_buffer_copy(self.opts)
        o.evenodd = 1
        return o

    def pool_bytes(self, dims, formulation, nslots):
        """Workspace bytes of a pool of nslots systems of the group."""
        key = (dims, formulation, nslots)
        if key not in self._ws_cache:
            self._ws_cache[key] = solve_workspace_bytes(self.gauges[dims], formulation,
                                                        self.opts_for(formulation), nslots,
                                                        g55=self.g55)
        return self._ws_cache[key]

    def per_system_bytes(self, dims, formulation):
        """A request's footprint: the bytes one more system adds to a pool."""
        return self.pool_bytes(dims, formulation, 2) - self.pool_bytes(dims, formulation, 1)

    def set_budget(self, nbytes):
        """Change the workspace budget (between runs)."""
        self.ledger.budget = self.mem_budget = int(nbytes)

    @property
    def allocated(self):
        return self.ledger.used

    def _now(self):
        return time.perf_counter() - self._t0

    def _submit(self, req):
        dims = tuple(req.dims)
        if dims not in self.gauges or self.pool_bytes(dims, req.formulation, 1) > self.mem_budget:
            with self._lock:
                self.rejected.append(req.id)
                self._cancel.discard(req.id)
            return
        key = (dims, req.formulation)
        with self._lock:
            g = self.groups.get(key)
            if g is None:
                g = self.groups[key] = _Group(key=key)
            g.waiting.append(req)

    def _open_pool(self, g, nslots):
        dims, formulation = g.key
        nbytes = self.pool_bytes(dims, formulation, nslots)
        stream = self.torch.cuda.Stream()
        with self.torch.cuda.stream(stream):
            b = Batch(self.gauges[dims], formulation, nslots, r=self.r, g55=self.g55,
                      opts=self.opts_for(formulation))
        p = _Pool(group=g, batch=b, stream=stream, nbytes=b.nbytes, free=list(range(nslots)))
        p.thread = threading.Thread(target=self._worker, args=(p,), daemon=True)
        with self._lock:
            self.ledger.take(max(nbytes, b.nbytes))
            p.nbytes = max(nbytes, b.nbytes)
            g.pools.append(p)
            self.pools_opened += 1
        p.thread.start()

    def _schedule(self):
        """One pass of the scheduler: drop cancelled queued requests, close
        retired pools that have exited, open pools where requests wait for
        slots and the budget allows, and retire idle pools when a group is
        short of memory."""
        closed = []
        with self._lock:
            for g in self.groups.values():
                keep = collections.deque()
                for req in g.waiting:
                    if req.id in self._cancel:
                        self._cancel.discard(req.id)
                        self.cancelled.append((req.id, "queued", self._now()))
                    else:
                        keep.append(req)
                g.waiting = keep
                for p in [p for p in g.pools if p.closed]:
                    g.pools.remove(p)
                    self.ledger.give(p.nbytes)
                    self.pools_closed += 1
                    closed.append(p)
            wants = []
            for g in self.groups.values():
                free = sum(len(p.free) for p in g.pools if not p.retire)
                short = len(g.waiting) - free
                if short > 0:
                    wants.append((g.waiting[0].arrival, g, short))
            wants.sort(key=lambda w: w[0])   # the group waiting longest first
        if closed:
            for p in closed:
                p.batch = None
            self.torch.cuda.empty_cache()   # return the retired workspaces to the device
        starved = []
        for _, g, short in wants:
            dims, formulation = g.key
            want = min(self.max_slots, max(short, self.min_pool))
            with self._lock:
                n = self.ledger.fit(lambda k: self.pool_bytes(dims, formulation, k), want)
            if n >= 1:
                self._open_pool(g, n)
            else:
                starved.append(g)
        if starved:
            # lend memory: the pools of every other group with nothing waiting
            # take no new request and close once their running systems finish
            with self._lock:
                for g in self.groups.values():
                    if g.waiting or g in starved:
                        continue
                    for p in g.pools:
                        if not p.retire:
                            p.retire = True
                            self.pools_lent += 1

    # -------------------------------------------------------------- worker
    def _worker(self, p):
        g = p.group
        b = p.batch
        while True:
            loads = []
            with self._lock:
                while p.free and g.waiting and not p.retire:
                    req = g.waiting.popleft()
                    s = p.free.pop(0)
                    p.slot_req[s] = (req, self._now())
                    loads.append((s, req))
            for s, req in loads:
                b.load(s, req.source, req.mass, req.tol, req.maxiter, stream=p.stream)
            if not p.slot_req:
                with self._lock:
                    if p.retire or (self._stop and not g.waiting):
                        b = None        # the scheduler frees the pool's workspace
                        p.closed = True
                        return
                time.sleep(0.0005)
                continue
            states = b.step(self.chunk, stream=p.stream)
            for s, st in enumerate(states):
                if s in p.slot_req and st in (SLOT_DONE, SLOT_FAILED):
                    req, adm = p.slot_req[s]
                    x, info = b.fetch(s, stream=p.stream)
                    with self._lock:
                        del p.slot_req[s]
                        self.results.append(Result(req.id, x, info, req.arrival, adm, self._now()))
                        self._cancel.discard(req.id)   # finished first: a late cancel is void
                        p.free.append(s)
                elif s in p.slot_req and self._take_cancel(p.slot_req[s][0].id, "running"):
                    b.cancel(s, stream=p.stream)
                    with self._lock:
                        del p.slot_req[s]
                        p.free.append(s)

    def _take_cancel(self, rid, phase):
        """True (and recorded) if request rid has been cancelled."""
        with self._lock:
            if rid not in self._cancel:
                return False
            self._cancel.discard(rid)
            self.cancelled.append((rid, phase, self._now()))
            return True

    # ----------------------------------------------------------------- API
    def status(self, request_id):
        """'running' while the request holds a slot, 'queued' while it waits
        for one, 'finished', 'cancelled' or 'rejected' once it is out, else None
        (not yet arrived, or unknown)."""
        with self._lock:
            if any(r.id == request_id for r in self.results):
                return "finished"
            if any(c[0] == request_id for c in self.cancelled):
                return "cancelled"
            if request_id in self.rejected:
                return "rejected"
            for g in self.groups.values():
                for p in g.pools:
                    if any(req.id == request_id for req, _ in p.slot_req.values()):
                        return "running"
                if any(req.id == request_id for req in g.waiting):
                    return "queued"
        return None

    def cancel(self, request_id):
        """Cancel a request: dropped if still queued, its slot freed at the next
        chunk boundary if running; no effect once it has finished."""
        with self._lock:
            if not any(r.id == request_id for r in self.results):
                self._cancel.add(request_id)

    def run(self, requests):
        """Feed requests at their arrival times (seconds from now), schedule
        pools until every request has finished, been cancelled or been
        rejected.  Returns the results in completion order."""
        self._t0 = time.perf_counter()
        self._stop = False
        timers = []
        for req in requests:
            if req.cancel_at is not None:
                t = threading.Timer(req.cancel_at, self.cancel, args=(req.id,))
                t.daemon = True
                t.start()
                timers.append(t)
        order = sorted(requests, key=lambda r: r.arrival)
        ids = {req.id for req in requests}
        nxt = 0
        while True:
            now = self._now()
            while nxt < len(order) and order[nxt].arrival <= now:
                self._submit(order[nxt])
                nxt += 1
            self._schedule()
            with self._lock:
                out = ({r.id for r in self.results} | {c[0] for c in self.cancelled} |
                       set(self.rejected))
                done = nxt == len(order) and ids <= out
                alive = [p for g in self.groups.values() for p in g.pools]
            if done:
                break
            wait = 0.0005
            if nxt < len(order):
                wait = min(wait, max(0.0, order[nxt].arrival - now))
            for p in alive:
                if not p.thread.is_alive() and not p.closed:
                    raise RuntimeError("a solver pool's worker died")
            time.sleep(wait)
        with self._lock:
            self._stop = True
        for g in list(self.groups.values()):
            for p in list(g.pools):
                p.thread.join()
        self._schedule()
        for t in timers:
            t.cancel()
        return self.results

    def report(self):
        lat = np.array([r.latency for r in self.results]) if self.results else np.zeros(1)
        span = max((r.finished for r in self.results), default=0.0)
        ok = sum(1 for r in self.results if r.info["status"] == 0)
        return dict(completed=len(self.results), converged=ok, rejected=len(self.rejected),
                    cancelled=len(self.cancelled),
                    solves_per_s=len(self.results) / span if span > 0 else 0.0,
                    p50_latency_s=float(np.percentile(lat, 50)),
                    p99_latency_s=float(np.percentile(lat, 99)),
                    workspace_bytes=self.ledger.peak, budget_bytes=self.mem_budget,
                    pools_opened=self.pools_opened, pools_closed=self.pools_closed,
                    pools_lent=self.pools_lent)
