"""The C-ABI boundary: gauge upload from host or device memory, and the solve
statuses and flags of lq_solve_info; the growth restart of the 16-bit solver
at long reliable-update intervals on the 16^3 x 32 workload."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import solvers

pytestmark = pytest.mark.gpu

lq = pytest.importorskip("paper_1312_3265_amd")
torch = pytest.importorskip("torch")


def test_gauge_from_host_equals_gauge_from_device():
    """A host field is uploaded in chunks of 4096 sites through the staging
    area; 8x8x8x10 (5120 sites) needs a full and a partial chunk.  Both
    uploads must give the same library field: equal plaquettes, bitwise equal
    matvecs in every storage and for both operators."""
    dims = (8, 8, 8, 10)
    U = synth.gauge_field(dims, "haar", 314)
    lat = lq.Lattice(dims)
    feats = lq.FEAT_CORNERS | lq.FEAT_F32 | lq.FEAT_Q16
    gh = lq.Gauge(lat, U, feats)                                  # host pointer
    gd = lq.Gauge(lat, torch.from_numpy(U).cuda(), feats)        # device pointer
    assert gh.plaquette() == gd.plaquette()
    assert gh.su3_deviation() == gd.su3_deviation()
    for form in (synth.WILSON, synth.STAGGERED_WILSON):
        psi = synth.gaussian_field(dims, form, 3)
        for prec in (lq.F64, lq.F32, lq.Q16):
            a = lq.apply(gh, form, 0.1, psi, precision=prec)
            b = lq.apply(gd, form, 0.1, psi, precision=prec)
            assert torch.equal(a, b), (form, prec)


def test_solve_statuses_and_flags():
    dims = (8, 8, 6, 8)
    U = synth.gauge_field(dims, "near_identity", 5, 0.436)
    g = lq.Gauge(lq.Lattice(dims), U)
    chi = synth.point_source(dims, synth.STAGGERED_WILSON, 0)
    x, info = lq.cg_solve(g, synth.STAGGERED_WILSON, -0.35, chi, 1e-8)
    assert info["status"] == lq.OK and info["flags"] == 0
    x, info = lq.cg_solve(g, synth.STAGGERED_WILSON, -0.35, chi, 1e-12, maxiter=7)
    assert info["status"] == lq.NOT_CONVERGED and info["flags"] & lq.FLAG_MAXITER
    assert not info["flags"] & (lq.FLAG_BREAKDOWN | lq.FLAG_STAGNATION)
    # the flags of a running slot are reported by peek without device work
    b = lq.Batch(g, synth.STAGGERED_WILSON, nslots=1)
    b.load(0, chi, -0.35, 1e-12, maxiter=5)
    b.step(8)
    pk = b.peek(0)
    assert pk["status"] == lq.SLOT_FAILED and pk["flags"] & lq.FLAG_MAXITER
    _, inf = b.fetch(0)
    assert inf["status"] == lq.NOT_CONVERGED and inf["flags"] == pk["flags"]


@pytest.mark.parametrize("interval", [400, 1024])
def test_q16_wilson_long_reliable_interval_converges(interval):
    """The 16-bit Wilson solve nearest m_c (delta = 0.02) with reliable updates
    at most every 400 or 1024 iterations: without the restart on 100-fold
    residual growth it diverged; with it the solve converges, and the
    stagnation stop (growth that persists across a restart) does not end it
    early.  The oracle recomputes eq. (2)'s residual in FP64."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "workloads.json")) as f:
        w = json.load(f)
    dims = tuple(w["dims"])
    U = synth.gauge_field(dims, "near_identity", w["seed"], w["eps"])
    g = lq.Gauge(lq.Lattice(dims), U, lq.FEAT_Q16)
    m = w["m_c"]["wilson"] + 0.02
    chi = synth.point_source(dims, synth.WILSON, 0)
    opts = lq.solve_opts(precision=lq.Q16, links=12, reliable_interval=interval)
    x, info = lq.cg_solve(g, synth.WILSON, m, chi, 1e-8, opts=opts)
    print(f"interval {interval}: {info}")
    assert info["status"] == lq.OK, info
    rn, _ = solvers.true_residual(synth.WILSON, U, chi, x.cpu().numpy(), m)
    assert rn <= 1e-8, rn
