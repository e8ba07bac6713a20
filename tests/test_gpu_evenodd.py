"""GPU parity of the even-odd (Schur complement) Wilson path against the oracle
(needs an MI355X).

The oracle's Schur operator is built from its full Wilson matrix by parity
projection (``oracle/evenodd.py``); the library's from half-lattice hop
kernels over checkerboarded links.  Bars as for the full matvecs: FP64
relative error <= 1e-13 (max-norm), FP32 and 16-bit within their roundoff
bounds, and the odd half of the result exactly zero.
"""
import numpy as np
import pytest

import synth
from oracle import evenodd as EO

pytestmark = pytest.mark.gpu

lq = pytest.importorskip("paper_1312_3265_amd")
torch = pytest.importorskip("torch")

FEATURES = lq.FEAT_EO | lq.FEAT_F32 | lq.FEAT_Q16
_GAUGE = {}


def _gauge(dims, kind, seed, bc=(1, 1, 1, 1), eps=None):
    key = (dims, kind, seed, bc, eps)
    if key not in _GAUGE:
        U = synth.gauge_field(dims, kind, seed, eps)
        _GAUGE[key] = (U, lq.Gauge(lq.Lattice(dims, bc), U, FEATURES))
    return _GAUGE[key]


def _relerr(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


CASES = [((4, 4, 4, 4), "haar", (1, 1, 1, 1)),
         ((6, 4, 6, 8), "haar", (1, 1, 1, -1)),          # V/2 = 576: ragged last block
         ((8, 8, 6, 4), "near_identity", (-1, 1, 1, -1))]


@pytest.mark.parametrize("dims,kind,bc", CASES)
@pytest.mark.parametrize("dagger", [False, True])
@pytest.mark.parametrize("links", [0, 18])
def test_fp64_schur_matches_oracle(dims, kind, bc, dagger, links):
    U, g = _gauge(dims, kind, 11, bc, 0.436 if kind != "haar" else None)
    psi = synth.gaussian_field(dims, synth.WILSON, 5)
    m = -0.21
    out = lq.schur_apply(g, m, psi, dagger=dagger, links=links).cpu().numpy()
    ref = EO.schur_apply(U, EO.project(psi, EO.EVEN), m, bc, dagger)
    assert _relerr(out, ref) <= 1e-13
    assert np.abs(EO.project(out, EO.ODD)).max() == 0.0


@pytest.mark.parametrize("precision,links,bound", [(lq.F32, 18, 2e-6), (lq.F32, 12, 4e-6),
                                                  (lq.Q16, 12, 1e-4), (lq.Q16, 18, 1e-4)])
def test_low_precision_schur_within_roundoff(precision, links, bound):
    """Two hop stencils in sequence, the intermediate stored in the working
    precision: the bounds of the single matvec hold with room to spare."""
    dims = (6, 4, 6, 8)
    U, g = _gauge(dims, "near_identity", 21, eps=0.436)
    psi = synth.gaussian_field(dims, synth.WILSON, 7)
    out = lq.schur_apply(g, 0.1, psi, precision=precision, links=links).cpu().numpy()
    ref = EO.schur_apply(U, EO.project(psi, EO.EVEN), 0.1)
    assert _relerr(out, ref) <= bound


def test_schur_needs_the_even_odd_links():
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, "haar", 3)
    g = lq.Gauge(lq.Lattice(dims), U, lq.FEAT_F32)
    with pytest.raises(lq.LQError):
        lq.schur_apply(g, 0.1, synth.gaussian_field(dims, synth.WILSON, 1))


# ------------------------------------------------------------------ solves
def test_fp64_eo_cg_4x4_matches_oracle():
    """The library stops once eq. (2)'s own residual for the whole solution
    is below tol (the oracle's even-odd CG stops on the Schur system, whose
    residual can be smaller): the solution matches the oracle's, and the
    reported residual is the oracle's FP64 recomputation."""
    from oracle import solvers
    dims = (4, 4, 4, 4)
    U, g = _gauge(dims, "haar", 1000)
    chi = synth.point_source(dims, synth.WILSON, 0)
    m, tol = 0.5, 1e-10
    x, info = lq.cg_solve(g, synth.WILSON, m, chi, tol, opts=lq.solve_opts(evenodd=1))
    assert info["status"] == lq.OK
    xo, oinfo = EO.cgnr(U, chi, m, 1e-13, 10000)
    assert oinfo["status"] == solvers.CONVERGED
    x = x.cpu().numpy()
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= 1e-8
    rn, rd = solvers.true_residual(synth.WILSON, U, chi, x, m)
    assert rn <= tol
    assert abs(info["true_residual"] - rn) <= 1e-3 * tol + 1e-15


@pytest.mark.parametrize("precision", [lq.F32, lq.Q16])
def test_mixed_eo_batch_solves_eq2_with_fewer_iterations(precision):
    """Point sources over several masses near m_c on a near-identity field:
    every system's full solution meets eq. (2) (FP64, oracle), and the
    preconditioned iteration count is below half the unpreconditioned one."""
    from oracle import solvers
    dims = (8, 8, 8, 8)
    U, g = _gauge(dims, "near_identity", 2000, eps=0.4359375)
    ms = [-0.30, -0.25, -0.20, -0.30]
    chis = np.stack([synth.point_source(dims, synth.WILSON, a) for a in (0, 5, 7)]
                    + [synth.z2_source(dims, synth.WILSON, 3)])
    tol = 1e-8
    x, infos = lq.cg_solve_batch(g, synth.WILSON, ms, chis, [tol] * 4,
                                 opts=lq.solve_opts(precision=precision, evenodd=1))
    x0, infos0 = lq.cg_solve_batch(g, synth.WILSON, ms, chis, [tol] * 4,
                                   opts=lq.solve_opts(precision=precision))
    for k in range(4):
        assert infos[k]["status"] == lq.OK
        rn, _ = solvers.true_residual(synth.WILSON, U, chis[k], x[k].cpu().numpy(), ms[k])
        assert rn <= tol
        assert abs(infos[k]["true_residual"] - rn) <= 1e-3 * tol
        assert infos[k]["iterations"] < 0.5 * infos0[k]["iterations"]


def test_eo_batch_result_is_bitwise_the_single_result():
    dims = (8, 8, 8, 8)
    U, g = _gauge(dims, "near_identity", 2000, eps=0.4359375)
    ms = [-0.25, -0.1, -0.3]
    chis = np.stack([synth.point_source(dims, synth.WILSON, a) for a in (1, 4, 11)])
    opts = lq.solve_opts(precision=lq.Q16, evenodd=1, reliable_interval=40)
    xb, ib = lq.cg_solve_batch(g, synth.WILSON, ms, chis, [1e-8, 1e-9, 1e-7], opts=opts)
    for k, t in enumerate([1e-8, 1e-9, 1e-7]):
        xs, is_ = lq.cg_solve(g, synth.WILSON, ms[k], chis[k], t, opts=opts)
        assert is_["iterations"] == ib[k]["iterations"]
        assert torch.equal(xs, xb[k])


def test_eo_refused_outside_wilson_r1():
    dims = (4, 4, 4, 4)
    U, g = _gauge(dims, "haar", 1000)
    opts = lq.solve_opts(evenodd=1)
    with pytest.raises(lq.LQError):
        lq.cg_solve(g, synth.STAGGERED_WILSON, 0.5, synth.point_source(dims, synth.STAGGERED_WILSON, 0),
                    1e-8, opts=opts)
    with pytest.raises(lq.LQError):
        lq.cg_solve(g, synth.WILSON, 0.5, synth.point_source(dims, synth.WILSON, 0), 1e-8, opts=opts,
                    r=0.7)


def test_eo_continuous_batching_alone_vs_in_the_mix():
    """Requests admitted into free slots while others iterate (even-odd,
    16-bit) give bitwise the result they give alone."""
    dims = (8, 8, 8, 8)
    U, g = _gauge(dims, "near_identity", 2000, eps=0.4359375)
    opts = lq.solve_opts(precision=lq.Q16, evenodd=1, reliable_interval=48, poll_interval=8)
    reqs = [(synth.point_source(dims, synth.WILSON, a), m, t)
            for a, m, t in ((0, -0.3, 1e-8), (5, -0.25, 1e-7), (7, -0.2, 1e-9), (2, -0.28, 1e-8))]
    alone = [lq.cg_solve(g, synth.WILSON, m, c, t, opts=opts) for c, m, t in reqs]
    b = lq.Batch(g, synth.WILSON, nslots=2, opts=opts)
    pending = list(range(len(reqs)))
    slot_of, results, free = {}, {}, [0, 1]
    guard = 0
    while pending or slot_of:
        while pending and free:
            k = pending.pop(0)
            s = free.pop(0)
            c, m, t = reqs[k]
            b.load(s, c, m, t)
            slot_of[s] = k
        for s, st in enumerate(b.step(16)):
            if s in slot_of and st in (lq.SLOT_DONE, lq.SLOT_FAILED):
                results[slot_of.pop(s)] = b.fetch(s)
                free.append(s)
        guard += 1
        assert guard < 10000
    for k in range(len(reqs)):
        xm, im = results[k]
        xa, ia = alone[k]
        assert im["status"] == lq.OK and im["iterations"] == ia["iterations"]
        assert torch.equal(xm, xa)


def test_eo_pair_timing_modes():
    dims = (8, 8, 8, 8)
    U, g = _gauge(dims, "near_identity", 2000, eps=0.4359375)
    for kern in (3, 4):
        ms = lq.time_dslash(g, synth.WILSON, -0.3, precision=lq.Q16, links=12, nrhs=5, reps=4,
                            rhs_per_thread=2, window=-3, kernel=kern)
        assert 0.0 < ms < 100.0
    with pytest.raises(lq.LQError):
        lq.time_dslash(g, synth.STAGGERED_WILSON, -0.3, kernel=3)


def test_full_size_16x32_schur_and_eo_batch():
    """The 16^3 x 32 workload field: M^ and M^dag in FP64 against the oracle over
    the whole field, 16-bit M^ within its roundoff bound, and a 16-bit even-odd
    batch of the 12 point sources at m_c + 0.1 (the Wilson batch of the
    benchmark's even-odd comparison, one mass): every full solution meets
    eq. (2) in the oracle's FP64 recomputation."""
    from oracle import solvers
    import json
    import os
    wl = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "workloads.json")))
    dims = tuple(wl["dims"])
    U, g = _gauge(dims, "near_identity", wl["seed"], eps=wl["eps"])
    m = wl["m_c"]["wilson"] + 0.1
    psi = synth.gaussian_field(dims, synth.WILSON, 5)
    pe = EO.project(psi, EO.EVEN)
    for dagger in (False, True):
        out = lq.schur_apply(g, m, psi, dagger=dagger).cpu().numpy()
        ref = EO.schur_apply(U, pe, m, dagger=dagger)
        assert _relerr(out, ref) <= 1e-13
        assert np.abs(EO.project(out, EO.ODD)).max() == 0.0
    out = lq.schur_apply(g, m, psi, precision=lq.Q16).cpu().numpy()
    assert _relerr(out, EO.schur_apply(U, pe, m)) <= 1e-4
    chis = np.stack([synth.point_source(dims, synth.WILSON, a) for a in range(12)])
    tol = 1e-8
    x, infos = lq.cg_solve_batch(g, synth.WILSON, [m] * 12, chis, [tol] * 12,
                                 opts=lq.solve_opts(precision=lq.Q16, evenodd=1))
    for k in range(12):
        assert infos[k]["status"] == lq.OK
        rn, _ = solvers.true_residual(synth.WILSON, U, chis[k], x[k].cpu().numpy(), m)
        assert rn <= tol
        assert abs(infos[k]["true_residual"] - rn) <= 1e-3 * tol
