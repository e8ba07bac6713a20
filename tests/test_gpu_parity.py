"""GPU parity of the HIP path against the FP64 oracle (needs an MI355X).

Inputs are seeded synthetic fields from ``synth``; the oracle and the library
share nothing else.  Bars: FP64 matvec relative error <= 1e-13 (max-norm over
the field); FP32 and 16-bit fixed-point stencils within bounds derived from their unit
roundoff times the operator's term count; solves judged by the FP64 true
residual recomputed by the oracle, which must be <= the requested tolerance.
"""
import numpy as np
import pytest

import synth
from oracle import gauge as ogauge
from oracle import solvers
from oracle import staggered_wilson as SW
from oracle import wilson as W

pytestmark = pytest.mark.gpu

lq = pytest.importorskip("paper_1312_3265_amd")
torch = pytest.importorskip("torch")

FORMS = [synth.WILSON, synth.STAGGERED_WILSON]


def _oracle_apply(formulation, U, psi, m, op, r=1.0, bc=(1, 1, 1, 1)):
    mod = W if formulation == synth.WILSON else SW
    if op == lq.OP_M:
        return mod.apply(U, psi, m, r, bc)
    if op == lq.OP_MDAG:
        return mod.apply(U, psi, m, r, bc, dagger=True)
    return mod.apply(U, mod.apply(U, psi, m, r, bc), m, r, bc, dagger=True)


def _relerr(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


_GAUGE_CACHE = {}


def _gauge(dims, kind, seed, bc=(1, 1, 1, 1), eps=None,
           features=lq.FEAT_CORNERS | lq.FEAT_F32 | lq.FEAT_Q16):
    key = (dims, kind, seed, bc, eps, features)
    if key not in _GAUGE_CACHE:
        U = synth.gauge_field(dims, kind, seed, eps)
        lat = lq.Lattice(dims, bc)
        _GAUGE_CACHE[key] = (U, lat, lq.Gauge(lat, U, features))
    return _GAUGE_CACHE[key]


# ------------------------------------------------------------------ gauge
@pytest.mark.parametrize("dims,kind,eps", [((4, 4, 4, 4), "haar", None),
                                           ((8, 6, 4, 10), "near_identity", 0.436)])
def test_plaquette_matches_oracle(dims, kind, eps):
    U, lat, g = _gauge(dims, kind, 3, eps=eps)
    assert abs(g.plaquette() - ogauge.plaquette(U)) < 1e-13


# ---------------------------------------------------------------- matvecs
CASES = [((4, 4, 4, 4), "haar", (1, 1, 1, 1)),
         ((6, 4, 6, 8), "haar", (1, 1, 1, -1)),       # V = 1152: ragged last block
         ((8, 8, 6, 4), "near_identity", (-1, 1, 1, -1))]


@pytest.mark.parametrize("dims,kind,bc", CASES)
@pytest.mark.parametrize("formulation,g55", [(synth.WILSON, 0),
                                             (synth.STAGGERED_WILSON, lq.G55_CORNERS),
                                             (synth.STAGGERED_WILSON, lq.G55_ONTHEFLY)])
@pytest.mark.parametrize("op", [lq.OP_M, lq.OP_MDAG, lq.OP_MDAGM])
@pytest.mark.parametrize("links", [0, 18])
def test_fp64_matvec_matches_oracle(dims, kind, bc, formulation, g55, op, links):
    """links 0 = the FP64 default (12-real reads on these SU(3) fields), 18 = all rows."""
    U, lat, g = _gauge(dims, kind, 11, bc=bc, eps=0.436 if kind != "haar" else None)
    psi = synth.gaussian_field(dims, formulation, 5)
    m = 0.137
    out = lq.apply(g, formulation, m, psi, op=op, g55=g55, links=links).cpu().numpy()
    ref = _oracle_apply(formulation, U, psi, m, op, 1.0, bc)
    assert _relerr(out, ref) <= 1e-13


@pytest.mark.parametrize("r", [0.7, 1.3])
def test_fp64_matvec_general_r(r):
    dims = (4, 6, 4, 4)
    U, lat, g = _gauge(dims, "haar", 12)
    for formulation in FORMS:
        psi = synth.gaussian_field(dims, formulation, 6)
        out = lq.apply(g, formulation, -0.2, psi, op=lq.OP_M, r=r).cpu().numpy()
        ref = _oracle_apply(formulation, U, psi, -0.2, lq.OP_M, r)
        assert _relerr(out, ref) <= 1e-13


@pytest.mark.parametrize("formulation,g55", [(synth.WILSON, 0),
                                             (synth.STAGGERED_WILSON, lq.G55_CORNERS),
                                             (synth.STAGGERED_WILSON, lq.G55_ONTHEFLY)])
@pytest.mark.parametrize("precision,links,bound", [(lq.F32, 18, 2e-6), (lq.F32, 12, 4e-6),
                                                  (lq.Q16, 12, 1e-4), (lq.Q16, 18, 1e-4)])
def test_low_precision_matvec_within_roundoff(formulation, g55, precision, links, bound):
    """FP32: u = 6e-8 per operation over O(30) accumulated terms; Q16 storage:
    each stored component is off by at most 2^-16 of its site's largest
    component (vectors) or of 1 (link and corner entries, all of modulus <= 1),
    about 1.5e-5 relative, accumulated over a few stored inputs per term."""
    dims = (6, 4, 6, 8)
    U, lat, g = _gauge(dims, "near_identity", 21, eps=0.436)
    psi = synth.gaussian_field(dims, formulation, 7)
    out = lq.apply(g, formulation, 0.1, psi, op=lq.OP_M, g55=g55, precision=precision,
                   links=links).cpu().numpy()
    ref = _oracle_apply(formulation, U, psi, 0.1, lq.OP_M)
    assert _relerr(out, ref) <= bound


def test_q16_handles_vanishing_and_denormal_sites():
    """Sites whose largest component is zero, FP32-denormal or tiny (the far
    tail of a point-source solution on a large lattice) must not turn into inf
    or NaN in 16-bit storage: they are stored as zero, far below the
    rounding of the O(1) sites."""
    dims = (6, 4, 6, 8)
    U, lat, g = _gauge(dims, "near_identity", 21, eps=0.436)
    psi = synth.gaussian_field(dims, synth.WILSON, 7).astype(np.complex64)
    flat = psi.reshape(-1, 12)
    flat[0] = 0.0
    flat[1] = 1e-40      # FP32 denormal
    flat[2] = 3e-39
    flat[3] = 1e-33
    out = lq.apply(g, synth.WILSON, 0.1, psi, op=lq.OP_M, precision=lq.Q16, links=12)
    assert torch.isfinite(torch.view_as_real(out)).all()
    ref = _oracle_apply(synth.WILSON, U, psi.astype(np.complex128), 0.1, lq.OP_M)
    assert _relerr(out.cpu().numpy(), ref) <= 1e-4


def test_fp64_matvec_full_size_16x32():
    """16^3 x 32 near-identity field (the workload's field 0): the whole field
    against the oracle, M and M^dag, for Wilson and for staggered Wilson with
    Gamma_55 from the corner matrices and on the fly (the subset recursion's
    level launches and the operator's last level)."""
    dims = (16, 16, 16, 32)
    U, lat, g = _gauge(dims, "near_identity", 2000, eps=0.4359375,
                       features=lq.FEAT_CORNERS)
    for formulation, g55 in [(synth.WILSON, 0), (synth.STAGGERED_WILSON, lq.G55_CORNERS),
                             (synth.STAGGERED_WILSON, lq.G55_ONTHEFLY)]:
        psi = synth.gaussian_field(dims, formulation, 8)
        for op in (lq.OP_M, lq.OP_MDAG):
            out = lq.apply(g, formulation, -0.4, psi, op=op, g55=g55).cpu().numpy()
            ref = _oracle_apply(formulation, U, psi, -0.4, op)
            err = _relerr(out, ref)
            print(f"formulation {formulation} g55 {g55} op {op}: relative error {err:.2e}")
            assert err <= 1e-13


@pytest.mark.timeout(900)
def test_matvecs_at_32x64_match_oracle():
    """32^3 x 64, the largest lattice of the serving workload (the 16^3 x 32
    field repeated twice in every direction): M^dag on a Gaussian field,
    against the oracle over the whole field, in the storages and link forms the
    solvers use -- FP64 (rows 0 and 1 of the links read) within 1e-13, FP32
    and 16-bit within the bounds of test_low_precision_matvec_within_roundoff;
    staggered Wilson with Gamma_55 from corners and on the fly."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "workloads.json")) as f:
        w = json.load(f)
    d16 = tuple(w["dims"])
    dims = tuple(2 * d for d in d16)
    U = np.tile(synth.gauge_field(d16, "near_identity", w["seed"], w["eps"]), (2, 2, 2, 2, 1, 1, 1))
    g = lq.Gauge(lq.Lattice(dims), U, lq.FEAT_CORNERS | lq.FEAT_F32 | lq.FEAT_Q16)
    for formulation, g55s in ((synth.WILSON, (0,)),
                              (synth.STAGGERED_WILSON, (lq.G55_CORNERS, lq.G55_ONTHEFLY))):
        psi = synth.gaussian_field(dims, formulation, 8)
        ref = _oracle_apply(formulation, U, psi, -0.4, lq.OP_MDAG)
        for g55 in g55s:
            for prec, links, bound in ((lq.F64, 12, 1e-13), (lq.F32, 12, 4e-6),
                                       (lq.Q16, 12, 1e-4)):
                out = lq.apply(g, formulation, -0.4, psi, op=lq.OP_MDAG, g55=g55,
                               precision=prec, links=links).cpu().numpy()
                err = _relerr(out, ref)
                print(f"32^3x64 formulation {formulation} g55 {g55} precision {prec}: "
                      f"relative error {err:.2e}")
                assert err <= bound, (formulation, g55, prec, err)


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 6, 8)])
@pytest.mark.parametrize("formulation,g55", [(synth.WILSON, 0),
                                             (synth.STAGGERED_WILSON, lq.G55_CORNERS),
                                             (synth.STAGGERED_WILSON, lq.G55_ONTHEFLY)])
@pytest.mark.parametrize("op", [lq.OP_M, lq.OP_MDAG])
def test_fp64_twelve_real_links_match_oracle(dims, formulation, g55, op):
    """FP64 stencils reading rows 0 and 1 of each link and rebuilding row 2:
    still within 1e-13 of the oracle (which uses all 18 reals) on SU(3) links."""
    U, lat, g = _gauge(dims, "haar", 41)
    psi = synth.gaussian_field(dims, formulation, 4)
    out = lq.apply(g, formulation, 0.2, psi, op=op, g55=g55, links=12).cpu().numpy()
    ref = _oracle_apply(formulation, U, psi, 0.2, op)
    assert _relerr(out, ref) <= 1e-13


def test_twelve_real_links_refused_for_non_su3_field():
    """Links with det != 1 (an SU(3) field times a U(1) phase) break the row-2
    rebuild; 12-real storage is refused while 18-real still matches the oracle."""
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, "haar", 43) * np.exp(0.3j)
    lat = lq.Lattice(dims)
    g = lq.Gauge(lat, U)
    m = U.reshape(-1, 3, 3)
    d = np.conj(np.cross(m[:, 0, :], m[:, 1, :])) - m[:, 2, :]
    expect = max(np.abs(d.real).max(), np.abs(d.imag).max())
    assert abs(g.su3_deviation() - expect) <= 1e-12
    U0, _, g0 = _gauge(dims, "haar", 41)
    assert g0.su3_deviation() <= 1e-14
    psi = synth.gaussian_field(dims, synth.WILSON, 5)
    for prec, links in ((lq.F64, 12), (lq.F32, 12), (lq.Q16, 12)):
        with pytest.raises(lq.LQError):
            lq.apply(g, synth.WILSON, 0.2, psi, op=lq.OP_M, precision=prec, links=links)
    out = lq.apply(g, synth.WILSON, 0.2, psi, op=lq.OP_M).cpu().numpy()
    assert _relerr(out, _oracle_apply(synth.WILSON, U, psi, 0.2, lq.OP_M)) <= 1e-13


# ------------------------------------------------------------------ solves
@pytest.mark.parametrize("formulation", FORMS)
def test_fp64_cg_4x4_matches_oracle(formulation):
    dims = (4, 4, 4, 4)
    U, lat, g = _gauge(dims, "haar", 1000)
    chi = synth.point_source(dims, formulation, 0)
    m, tol = 0.5, 1e-10
    x, info = lq.cg_solve(g, formulation, m, chi, tol)
    assert info["status"] == lq.OK
    xo, oinfo = solvers.cgnr(formulation, U, chi, m, tol, 10000)
    rn, _ = solvers.true_residual(formulation, U, chi, x.cpu().numpy(), m)
    assert rn <= tol
    assert abs(info["iterations"] - oinfo["iterations"]) <= 2
    assert info["true_residual"] <= tol
    assert abs(info["true_residual"] - rn) <= 1e-3 * tol + 1e-15


@pytest.mark.parametrize("formulation", FORMS)
def test_lanczos_4x4_matches_oracle(formulation):
    dims = (4, 4, 4, 4)
    U, lat, g = _gauge(dims, "haar", 1000)
    v0 = synth.gaussian_field(dims, formulation, 7)
    res = lq.condition_number(g, formulation, 0.5, v0, steps=60)
    lo, hi, kap, (a, b) = solvers.condition_number(formulation, U, 0.5, v0, 60)
    np.testing.assert_allclose(res["alpha"][:30], a[:30], rtol=1e-10)
    np.testing.assert_allclose(res["beta"][:30], b[:30], rtol=1e-9)
    assert abs(res["lmin"] - lo) <= 1e-8 * hi
    assert abs(res["lmax"] - hi) <= 1e-10 * hi


def test_fp64_wilson_t_sweep_agrees_with_the_plain_stencil(monkeypatch):
    """16^3 x 32, where the FP64 Wilson stencils sweep t (two slices per block):
    M, M^dag and M^dag M equal the plain one-site-per-thread stencil
    (LQ_TSWEEP=0) to rounding, a plain FP64 CG solve takes the same iterations
    either way, and with the sweep a batch of three systems gives bitwise the
    solutions of the three solves alone (the kernel choice depends on the
    lattice, not on the batch)."""
    dims = (16, 16, 16, 32)
    U, lat, g = _gauge(dims, "near_identity", 2000, eps=0.4359375, features=lq.FEAT_CORNERS)
    psi = synth.gaussian_field(dims, synth.WILSON, 12)
    m = -0.37
    out = {}
    for flag in ("1", "0"):
        monkeypatch.setenv("LQ_TSWEEP", flag)
        out[flag] = [lq.apply(g, synth.WILSON, m, psi, op=op) for op in
                     (lq.OP_M, lq.OP_MDAG, lq.OP_MDAGM)]
    for a, b in zip(out["1"], out["0"]):
        assert (a - b).abs().max().item() <= 1e-14 * b.abs().max().item()
    chis = np.stack([synth.point_source(dims, synth.WILSON, a) for a in (0, 4, 9)])
    its = {}
    for flag in ("0", "1"):
        monkeypatch.setenv("LQ_TSWEEP", flag)
        x, info = lq.cg_solve(g, synth.WILSON, m, chis[0], 1e-8)
        assert info["status"] == lq.OK
        its[flag] = info["iterations"]
    assert abs(its["1"] - its["0"]) <= 1, its
    xb, ib = lq.cg_solve_batch(g, synth.WILSON, [m, m + 0.01, m], chis, [1e-8, 1e-8, 1e-9])
    for k, (mk, tk) in enumerate(((m, 1e-8), (m + 0.01, 1e-8), (m, 1e-9))):
        xa, ia = lq.cg_solve(g, synth.WILSON, mk, chis[k], tk)
        assert ia["iterations"] == ib[k]["iterations"] and torch.equal(xa, xb[k]), k
