"""Continuous-batching solve server over the resident multi-slot CG solver.

Requests (lattice size, formulation, mass, source, tolerance) arrive over
time.  Gauge fields stay resident in HBM, one per lattice size.  Requests that
share a gauge field and formulation share one multi-slot solver (``Batch``):
every stencil launch serves all of its running systems.  A request is admitted
into a free slot as soon as one frees up, while the other slots keep iterating;
finished systems are harvested between chunks of iterations.  Each group runs
in its own host thread on its own HIP stream, so the groups' kernels overlap
on the device (the library calls release the GIL).

HBM admission: every group's solver workspace is allocated when the group is
created, with as many slots as fit into its share of the memory budget; a
request waits in its group's queue until a slot is free.  A request whose
group cannot hold even one system is rejected.

Cancellation: ``cancel(request_id)`` (from any thread, or at a request's
``cancel_at`` time) drops a request that is still queued, and frees the slot
of one that is running at the next chunk boundary; a request that finished
first is delivered as usual.

The arithmetic all happens in the library; this module only schedules.
"""
from __future__ import annotations

import collections
import queue
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


@dataclass
class _Group:
    key: tuple
    batch: Batch
    stream: object
    pending: "queue.Queue" = field(default_factory=queue.Queue)
    waiting: "collections.deque" = field(default_factory=collections.deque)
    slot_req: dict = field(default_factory=dict)
    thread: threading.Thread = None


class SolveServer:
    """Serve solve requests on resident gauge fields with continuous batching.

    fields: {dims: canonical gauge field (numpy or torch)}; opts: solver
    options (default FP32 Krylov vectors, 12-real links, FP64 reliable
    updates); mem_budget: bytes of HBM for solver workspaces (all groups);
    slots: upper bound on slots per group; chunk: iterations per step;
    evenodd: Wilson requests (r = 1) are solved even-odd preconditioned (the
    gauge fields then carry even-odd link copies); every solution still meets
    eq. (2)'s residual.
    """

    def __init__(self, fields, opts=None, mem_budget=8 << 30, slots=16, chunk=16, r=1.0,
                 g55=0, evenodd=False):
        self.torch = _torch()
        self.opts = opts or solve_opts(precision=1, links=12, poll_interval=chunk)
        self.evenodd = bool(evenodd) and r == 1.0
        self.chunk = chunk
        self.r = r
        self.g55 = g55
        self.max_slots = slots
        self.mem_budget = int(mem_budget)
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
        self._cancel = set()
        self._lock = threading.Lock()
        self._t0 = None
        self._stop = threading.Event()
        self.allocated = 0

    # ----------------------------------------------------------- admission
    def opts_for(self, formulation):
        """The solver options of a (dims, formulation) group."""
        if not (self.evenodd and formulation == WILSON):
            return self.opts
        o = SolveOpts.from_buffer_copy(self.opts)
        o.evenodd = 1
        return o

    def per_system_bytes(self, dims, formulation):
        o = self.opts_for(formulation)
        return solve_workspace_bytes(self.gauges[dims], formulation, o, 2, g55=self.g55) - \
            solve_workspace_bytes(self.gauges[dims], formulation, o, 1, g55=self.g55)

    def _group(self, dims, formulation):
        key = (dims, formulation)
        if key in self.groups:
            return self.groups[key]
        # each (dims, formulation) pair gets an equal share of the budget
        share = self.mem_budget // (2 * len(self.gauges))
        per = self.per_system_bytes(dims, formulation)
        nslots = int(min(self.max_slots, max(0, share // max(per, 1))))
        while nslots > 0 and solve_workspace_bytes(self.gauges[dims], formulation,
                                                   self.opts_for(formulation), nslots,
                                                   g55=self.g55) > share:
            nslots -= 1
        if nslots == 0:
            self.groups[key] = None
            return None
        stream = self.torch.cuda.Stream()
        with self.torch.cuda.stream(stream):
            b = Batch(self.gauges[dims], formulation, nslots, r=self.r, g55=self.g55,
                      opts=self.opts_for(formulation))
        self.allocated += b.nbytes
        g = _Group(key=key, batch=b, stream=stream)
        g.thread = threading.Thread(target=self._worker, args=(g,), daemon=True)
        self.groups[key] = g
        g.thread.start()
        return g

    def _now(self):
        return time.perf_counter() - self._t0

    # -------------------------------------------------------------- worker
    def _worker(self, g):
        b = g.batch
        free = list(range(b.nslots))
        torch = self.torch
        while True:
            # take arrivals into the group's waiting line, drop cancelled
            # requests from it whether or not a slot is free, then admit
            while True:
                try:
                    req = g.pending.get_nowait()
                except queue.Empty:
                    break
                with self._lock:
                    g.waiting.append(req)
            with self._lock:
                keep = collections.deque()
                for req in g.waiting:
                    if req.id in self._cancel:
                        self._cancel.discard(req.id)
                        self.cancelled.append((req.id, "queued", self._now()))
                    else:
                        keep.append(req)
                g.waiting = keep
            while free and g.waiting:
                with self._lock:
                    req = g.waiting.popleft()
                s = free.pop(0)
                b.load(s, req.source, req.mass, req.tol, req.maxiter, stream=g.stream)
                g.slot_req[s] = (req, self._now())
            if not g.slot_req:
                if self._stop.is_set() and g.pending.empty() and not g.waiting:
                    return
                time.sleep(0.0005)
                continue
            states = b.step(self.chunk, stream=g.stream)
            for s, st in enumerate(states):
                if s in g.slot_req and st in (SLOT_DONE, SLOT_FAILED):
                    req, adm = g.slot_req.pop(s)
                    x, info = b.fetch(s, stream=g.stream)
                    with self._lock:
                        self.results.append(Result(req.id, x, info, req.arrival, adm, self._now()))
                        self._cancel.discard(req.id)   # finished first: a late cancel is void
                    free.append(s)
                elif s in g.slot_req and self._take_cancel(g.slot_req[s][0].id, "running"):
                    g.slot_req.pop(s)
                    b.cancel(s, stream=g.stream)
                    free.append(s)

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
            for g in list(self.groups.values()):
                if g is None:
                    continue
                if any(req.id == request_id for req, _ in list(g.slot_req.values())):
                    return "running"
                if any(req.id == request_id for req in list(g.waiting)):
                    return "queued"
        return None

    def cancel(self, request_id):
        """Cancel a request: dropped if still queued, its slot freed at the next
        chunk boundary if running; no effect once it has finished."""
        with self._lock:
            if not any(r.id == request_id for r in self.results):
                self._cancel.add(request_id)

    def run(self, requests):
        """Feed requests at their arrival times (seconds from now) and wait
        for all of them.  Returns the results in completion order."""
        self._t0 = time.perf_counter()
        timers = []
        for req in requests:
            if req.cancel_at is not None:
                t = threading.Timer(req.cancel_at, self.cancel, args=(req.id,))
                t.daemon = True
                t.start()
                timers.append(t)
        for req in sorted(requests, key=lambda r: r.arrival):
            delay = req.arrival - self._now()
            if delay > 0:
                time.sleep(delay)
            g = self._group(tuple(req.dims), req.formulation)
            if g is None:
                with self._lock:
                    self.rejected.append(req.id)
                    self._cancel.discard(req.id)
                continue
            g.pending.put(req)
        self._stop.set()
        for g in list(self.groups.values()):
            if g is not None:
                g.thread.join()
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
                    workspace_bytes=self.allocated, budget_bytes=self.mem_budget,
                    groups={f"{k[0]}:{k[1]}": (g.batch.nslots if g else 0)
                            for k, g in self.groups.items()})
