"""The serving scheduler's host logic (admission by footprint against one
shared budget, lending memory between lattice sizes, rejection, cancellation)
on the CPU, with the library's solver pool replaced by a stand-in whose
systems finish after a set number of steps.  The GPU path of the same server
is covered by test_gpu_serving.py."""
import threading
import time

import numpy as np
import pytest

lq = pytest.importorskip("paper_1312_3265_amd")
serve = pytest.importorskip("paper_1312_3265_amd.serve")

PER_SITE = 100       # stand-in footprint: bytes per site and system
FIXED = 1000         # stand-in bytes of a pool besides its systems


class _Lat:
    def __init__(self, dims):
        self.dims = tuple(dims)


class _Gauge:
    def __init__(self, lat, U, feats):
        self.dims = lat.dims


def _ws(gauge, formulation, opts, nslots, g55=0):
    return FIXED + int(np.prod(gauge.dims)) * PER_SITE * nslots


class _Batch:
    """Slots finish after `mass` steps (the request's mass field is the
    stand-in's work count); every step takes a millisecond."""
    live = 0
    peak_live = 0
    lock = threading.Lock()

    def __init__(self, gauge, formulation, nslots, r=1.0, g55=0, opts=None):
        self.nslots = nslots
        self.nbytes = _ws(gauge, formulation, opts, nslots)
        self.left = [None] * nslots
        with _Batch.lock:
            _Batch.live += self.nbytes
            _Batch.peak_live = max(_Batch.peak_live, _Batch.live)
        self.freed = False

    def load(self, slot, chi, mass, tol, maxiter=100000, stream=None):
        assert self.left[slot] is None
        self.left[slot] = int(mass)

    def step(self, iterations, stream=None):
        time.sleep(0.001)
        out = []
        for s, v in enumerate(self.left):
            if v is None:
                out.append(lq.SLOT_EMPTY)
            elif v <= 1:
                self.left[s] = 0
                out.append(lq.SLOT_DONE)
            else:
                self.left[s] = v - 1
                out.append(lq.SLOT_RUNNING)
        return out

    def fetch(self, slot, stream=None):
        assert self.left[slot] == 0
        self.left[slot] = None
        return slot, {"status": 0, "iterations": 1}

    def cancel(self, slot, stream=None):
        assert self.left[slot] is not None
        self.left[slot] = None

    def __del__(self):
        with _Batch.lock:
            _Batch.live -= self.nbytes


class _Cuda:
    class Stream:
        pass

    class stream:
        def __init__(self, s):
            pass

        def __enter__(self):
            return self

        def __exit__(self, *a):
            return False

    @staticmethod
    def empty_cache():
        pass


class _Torch:
    cuda = _Cuda


@pytest.fixture
def fake(monkeypatch):
    monkeypatch.setattr(serve, "Lattice", _Lat)
    monkeypatch.setattr(serve, "Gauge", _Gauge)
    monkeypatch.setattr(serve, "Batch", _Batch)
    monkeypatch.setattr(serve, "solve_workspace_bytes", _ws)
    monkeypatch.setattr(serve, "_torch", lambda: _Torch)
    _Batch.live = 0
    _Batch.peak_live = 0
    return serve


A, B = (4, 4, 4, 4), (8, 8, 8, 8)
SA, SB = 256 * PER_SITE, 4096 * PER_SITE     # one system's footprint


def _req(i, dims, steps, arrival=0.0, form=0):
    return serve.Request(i, dims, form, float(steps), None, 1e-8, arrival=arrival)


def test_one_lattice_size_takes_the_whole_budget(fake):
    """Eight systems' worth of budget, two resident lattices, traffic on one:
    its pools hold up to eight systems at once (a fixed per-group share would
    give it two)."""
    budget = 2 * FIXED + 8 * SA
    srv = fake.SolveServer({A: None, B: None}, mem_budget=budget, slots=4, min_pool=4)
    reqs = [_req(i, A, 30) for i in range(8)]
    res = srv.run(reqs)
    rep = srv.report()
    assert sorted(r.id for r in res) == list(range(8))
    assert rep["pools_opened"] == 2 and rep["workspace_bytes"] == budget
    # all eight were admitted before any finished
    assert max(r.admitted for r in res) < min(r.finished for r in res)


def test_idle_lattice_lends_its_memory(fake):
    """The budget holds one 8^4 system or a pool of 4^4 systems, not both:
    8^4 requests that arrive while 4^4 systems run wait until those finish,
    the 4^4 pool closes, and the 8^4 pool opens in its place; the peak stays
    within the budget."""
    budget = FIXED + SB + SA // 2
    srv = fake.SolveServer({A: None, B: None}, mem_budget=budget, slots=4, min_pool=4)
    reqs = [_req(i, A, 40) for i in range(4)] + [_req(10 + i, B, 5, arrival=0.01) for i in range(2)]
    res = srv.run(reqs)
    rep = srv.report()
    by = {r.id: r for r in res}
    assert sorted(by) == [0, 1, 2, 3, 10, 11]
    assert rep["workspace_bytes"] <= budget and _Batch.peak_live <= budget
    assert rep["pools_lent"] >= 1
    lastA = max(by[i].finished for i in range(4))
    assert min(by[i].admitted for i in (10, 11)) >= lastA - 1e-3


def test_requests_that_cannot_fit_or_have_no_field_are_rejected(fake):
    srv = fake.SolveServer({A: None, B: None}, mem_budget=FIXED + SA, slots=4)
    res = srv.run([_req(0, A, 3), _req(1, B, 3), _req(2, (2, 2, 2, 2), 3)])
    assert [r.id for r in res] == [0]
    assert sorted(srv.rejected) == [1, 2]
    assert srv.status(1) == "rejected" and srv.status(0) == "finished"


def test_cancel_before_arrival_and_while_running(fake):
    """One slot: request 1 runs long and is cancelled once seen running,
    request 2 is cancelled before it arrives, request 3 then runs."""
    srv = fake.SolveServer({A: None}, mem_budget=FIXED + SA, slots=1)
    reqs = [_req(1, A, 100000), _req(2, A, 3), _req(3, A, 3)]
    srv.cancel(2)
    out = {}
    t = threading.Thread(target=lambda: out.setdefault("r", srv.run(reqs)))
    t.start()
    while srv.status(1) != "running":
        time.sleep(0.001)
    assert srv.status(3) == "queued"
    srv.cancel(1)
    t.join(timeout=60)
    assert not t.is_alive()
    assert [r.id for r in out["r"]] == [3]
    assert {rid: ph for rid, ph, _ in srv.cancelled} == {1: "running", 2: "queued"}
    assert srv.report()["pools_opened"] == 1


def test_ledger_fit_and_take():
    led = serve.Ledger(1000)
    ws = lambda n: 100 + 200 * n
    assert led.fit(ws, 10) == 4
    led.take(ws(4))
    assert led.left() == 100 and led.fit(ws, 1) == 0
    with pytest.raises(ValueError):
        led.take(101)
    led.give(ws(4))
    assert led.used == 0 and led.peak == 900
