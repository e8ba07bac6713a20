"""Pins of the FP64 oracle against mathematics and the paper (CPU only).

Each check is chosen so that a plausible slip in the oracle -- a dropped hop, a
wrong sign, a link taken at the wrong site, a missing dagger, a wrong phase
function -- fails at least one of them:

* free-field plane waves against the closed-form symbols (Sec. 3 free-field
  discussion), on lattices with L = 6 so that a wrong phi(x) is not hidden;
* the closed-form spectra and the paper's 8/sqrt(5) limit (Sec. 3);
* adjoint relations: D_st anti-hermitian, Gamma_55 hermitian, epsilon- and
  gamma_5-hermiticity (Sec. 2);
* gauge covariance M[U^g] = g M[U] g^dag on Haar-random links;
* three independently written forms of Gamma_55;
* CG against dense LU, CG's finite-termination property, Lanczos against dense
  eigenvalues and on a matrix with known spectrum.
"""
import numpy as np
import pytest

import synth
from oracle import dense, freefield, gauge, lattice, solvers
from oracle import staggered_wilson as SW
from oracle import evenodd as EO
from oracle import spectroscopy as SP
from oracle import spectrum as SPEC
from oracle import wilson as W

RNG = np.random.default_rng(12345)
_CACHE = {}


def dense_sw_normal(kind, m):
    """Dense A_SW on 4^4 (free field or the seed-1000 Haar field), cached."""
    key = ("swA", kind, m)
    if key not in _CACHE:
        dims = (4, 4, 4, 4)
        U = synth.gauge_field(dims, kind, 1000)
        M = dense.dense_matrix(lambda v: SW.apply(U, v, m), synth.field_shape(dims, 1))
        _CACHE[key] = (M, M.conj().T @ M)
    return _CACHE[key]


def _inner(a, b):
    return np.vdot(a.ravel(), b.ravel())


def _allowed_momentum(dims, bc, rng):
    p = []
    for mu in range(4):
        th = 0.0 if bc[mu] == 1 else np.pi
        n = rng.integers(0, dims[mu])
        p.append((2 * np.pi * n + th) / dims[mu])
    return np.array(p)


# ---------------------------------------------------------------- gamma basis
def test_gamma_basis_clifford_and_hermitian():
    g = W.GAMMA
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T)
        for nu in range(4):
            ac = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(ac, 2.0 * (mu == nu) * np.eye(4))
    assert np.allclose(W.GAMMA5, np.diag([1, 1, -1, -1]))
    for mu in range(4):
        assert np.linalg.matrix_rank(np.eye(4) - g[mu]) == 2
        assert np.linalg.matrix_rank(np.eye(4) + g[mu]) == 2


# ------------------------------------------------------------- gauge fields
def test_haar_su3_properties():
    rng = np.random.Generator(np.random.PCG64(3))
    u = synth.haar_su3(20000, rng)
    eye = np.eye(3)
    assert np.abs(u @ np.conj(np.swapaxes(u, -1, -2)) - eye).max() < 1e-13
    assert np.abs(np.linalg.det(u) - 1.0).max() < 1e-13
    tr = np.trace(u, axis1=-2, axis2=-1)
    # Haar SU(3): E[tr U] = 0 and E|tr U|^2 = 1 (number of irreducible
    # components of the fundamental representation).
    assert abs(tr.mean()) < 5.0 / np.sqrt(len(tr))
    assert abs(np.mean(np.abs(tr) ** 2) - 1.0) < 0.05


def test_near_identity_is_su3_and_tunes_plaquette():
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, "near_identity", 5, eps=0.44)
    m = U.reshape(-1, 3, 3)
    assert np.abs(m @ np.conj(np.swapaxes(m, -1, -2)) - np.eye(3)).max() < 1e-13
    assert np.abs(np.linalg.det(m) - 1.0).max() < 1e-13
    P = gauge.plaquette(synth.gauge_field((8, 8, 8, 8), "near_identity", 5, eps=0.436))
    assert abs(P - 0.594) < 0.01


def test_plaquette_unit_and_abelian_closed_form():
    dims = (4, 6, 4, 4)
    U = synth.gauge_field(dims, "unit")
    assert abs(gauge.plaquette(U) - 1.0) < 1e-15
    # U_1(x) = exp(i a x2 T), T = diag(1,-1,0), a = 2 pi / L2: every 1-2
    # plaquette equals exp(-i a T), the other five planes are 1.
    a = 2 * np.pi / dims[1]
    x1, x2, x3, x4 = lattice.coords(dims)
    ph = np.exp(1j * a * x2)
    U[..., 0, 0, 0] = ph
    U[..., 0, 1, 1] = np.conj(ph)
    expect = (5.0 + (1.0 + 2.0 * np.cos(a)) / 3.0) / 6.0
    assert abs(gauge.plaquette(U) - expect) < 1e-14


def test_plaquette_gauge_invariant():
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, "haar", 1)
    g = synth.gauge_transform(dims, 2)
    assert abs(gauge.plaquette(U) - gauge.plaquette(gauge.transform_links(U, g))) < 1e-13


# -------------------------------------------------------------------- Wilson
@pytest.mark.parametrize("dims,bc", [((4, 6, 4, 6), (1, 1, 1, 1)),
                                     ((6, 4, 4, 8), (1, 1, 1, -1))])
def test_wilson_free_plane_waves(dims, bc):
    U = synth.gauge_field(dims, "unit")
    for trial in range(6):
        p = _allowed_momentum(dims, bc, RNG)
        u = RNG.standard_normal((4, 3)) + 1j * RNG.standard_normal((4, 3))
        psi = synth.plane_wave(dims, p, u)
        for dagger in (False, True):
            m, r = 0.3, 1.0 if trial % 2 == 0 else 0.7
            Mp = W.momentum_matrix(p, m, r)
            if dagger:
                Mp = Mp.conj().T
            got = W.apply(U, psi, m, r, bc, dagger=dagger)
            want = synth.plane_wave(dims, p, Mp @ u)
            assert np.abs(got - want).max() < 1e-12


def test_wilson_free_all_momenta_give_closed_form_spectrum_and_8_over_sqrt5():
    """Every plane wave on 4^4 is an eigenvector of A_W with the closed-form
    eigenvalue; with the dense staggered Wilson spectrum this fixes both free
    condition numbers, whose square-root ratio tends to 8/sqrt(5) (Sec. 3)."""
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, "unit")
    m = 1e-3
    lam = []
    for p in freefield.momenta(dims):
        u = np.zeros((4, 3), dtype=complex)
        u[:, 0] = RNG.standard_normal(4) + 1j * RNG.standard_normal(4)
        psi = synth.plane_wave(dims, p, u)
        Apsi = W.apply_normal(U, psi, m)
        ratio = _inner(psi, Apsi) / _inner(psi, psi)
        assert np.abs(Apsi - ratio * psi).max() < 1e-12
        lam.append(ratio.real)
    lam = np.sort(np.array(lam))
    closed = np.sort(freefield.wilson_spectrum(dims, m)[::12])
    assert np.abs(lam - closed).max() < 1e-12
    ev = np.linalg.eigvalsh(dense_sw_normal("unit", m)[1])
    ratio = np.sqrt((lam[-1] / lam[0]) / (ev[-1] / ev[0]))
    # lambda_min = m^2 = 1e-6 carries the dense solver's ~1e-14 absolute error
    assert abs(ratio - (8.0 + m) / np.sqrt(4.0 + (1.0 + m) ** 2)) < 1e-6
    assert abs(ratio - 8.0 / np.sqrt(5.0)) < 1e-3


def test_wilson_adjoint_and_gamma5_hermiticity():
    dims = (4, 4, 4, 6)
    bc = (1, 1, 1, -1)
    U = synth.gauge_field(dims, "haar", 11)
    psi = synth.gaussian_field(dims, synth.WILSON, 1)
    chi = synth.gaussian_field(dims, synth.WILSON, 2)
    m = 0.37
    Mpsi = W.apply(U, psi, m, 1.0, bc)
    Mdchi = W.apply(U, chi, m, 1.0, bc, dagger=True)
    assert abs(_inner(chi, Mpsi) - _inner(Mdchi, psi)) < 1e-11
    g5 = W.gamma5(W.apply(U, W.gamma5(psi), m, 1.0, bc))
    assert np.abs(g5 - W.apply(U, psi, m, 1.0, bc, dagger=True)).max() < 1e-13


def test_wilson_gauge_covariance():
    dims = (4, 4, 6, 4)
    U = synth.gauge_field(dims, "haar", 21)
    g = synth.gauge_transform(dims, 22)
    psi = synth.gaussian_field(dims, synth.WILSON, 23)
    Ug = gauge.transform_links(U, g)
    lhs = W.apply(Ug, gauge.transform_fermion(g, psi, synth.WILSON), 0.1)
    rhs = gauge.transform_fermion(g, W.apply(U, psi, 0.1), synth.WILSON)
    assert np.abs(lhs - rhs).max() < 1e-13


# --------------------------------------------------------- staggered Wilson
def test_sw_hermiticity_relations():
    dims = (4, 6, 4, 6)
    bc = (1, 1, 1, -1)
    U = synth.gauge_field(dims, "haar", 31)
    psi = synth.gaussian_field(dims, synth.STAGGERED_WILSON, 1)
    chi = synth.gaussian_field(dims, synth.STAGGERED_WILSON, 2)
    d_psi, d_chi = SW.dst(U, psi, bc), SW.dst(U, chi, bc)
    assert abs(_inner(chi, d_psi) + _inner(d_chi, psi)) < 1e-11
    g_psi, g_chi = SW.gamma55_subsets(U, psi, bc), SW.gamma55_subsets(U, chi, bc)
    assert abs(_inner(chi, g_psi) - _inner(g_chi, psi)) < 1e-11
    m = 0.2
    M = SW.apply(U, psi, m, 1.0, bc)
    eMe = SW.epsilon_mul(SW.apply(U, SW.epsilon_mul(psi), m, 1.0, bc))
    Md = SW.apply(U, psi, m, 1.0, bc, dagger=True)
    assert np.abs(eMe - Md).max() < 1e-13
    assert abs(_inner(chi, M) - _inner(SW.apply(U, chi, m, 1.0, bc, dagger=True), psi)) < 1e-11


def test_sw_gauge_covariance():
    dims = (4, 6, 4, 4)
    U = synth.gauge_field(dims, "haar", 41)
    g = synth.gauge_transform(dims, 42)
    psi = synth.gaussian_field(dims, synth.STAGGERED_WILSON, 43)
    Ug = gauge.transform_links(U, g)
    lhs = SW.apply(Ug, gauge.transform_fermion(g, psi, synth.STAGGERED_WILSON), 0.1)
    rhs = gauge.transform_fermion(g, SW.apply(U, psi, 0.1), synth.STAGGERED_WILSON)
    assert np.abs(lhs - rhs).max() < 1e-13
    # the corner matrices transform as W_s(x) -> g(x) W_s(x) g(x+s)^dag
    Wc, Wg = SW.corners(U), SW.corners(Ug)
    for si, s in enumerate(SW.SIGNS):
        want = g @ Wc[si] @ np.conj(np.swapaxes(SW.gather_field(g, s), -1, -2))
        assert np.abs(Wg[si] - want).max() < 1e-13


@pytest.mark.parametrize("bc", [(1, 1, 1, 1), (1, 1, 1, -1), (-1, 1, -1, 1)])
def test_gamma55_three_forms_agree(bc):
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, "haar", 1000)
    psi = synth.gaussian_field(dims, synth.STAGGERED_WILSON, 3)
    a = SW.gamma55_subsets(U, psi, bc)
    b = SW.gamma55_paths(U, psi, bc)
    c = SW.gamma55_corners(SW.corners(U), psi, bc)
    assert np.abs(a - b).max() < 1e-14
    assert np.abs(a - c).max() < 1e-14


def test_corner_reflection_identity():
    """W_{-s}(x + s)^dag = W_s(x): the reversed path set is the same set."""
    dims = (4, 4, 6, 4)
    U = synth.gauge_field(dims, "haar", 51)
    Wc = SW.corners(U)
    for si, s in enumerate(SW.SIGNS):
        ms = tuple(-v for v in s)
        other = SW.gather_field(Wc[SW.SIGNS.index(ms)], s)
        assert np.abs(np.conj(np.swapaxes(other, -1, -2)) - Wc[si]).max() < 1e-14


@pytest.mark.parametrize("dims,bc", [((6, 6, 6, 6), (1, 1, 1, 1)),
                                     ((4, 6, 8, 6), (1, 1, 1, -1))])
def test_sw_free_plane_waves(dims, bc):
    U = synth.gauge_field(dims, "unit")
    shift = np.array([0.0, np.pi, 0.0, np.pi])
    for trial in range(4):
        p = _allowed_momentum(dims, bc, RNG)
        u = RNG.standard_normal(3) + 1j * RNG.standard_normal(3)
        psi = synth.plane_wave(dims, p, u)
        m, r = 0.25, 1.0 if trial % 2 == 0 else 0.6
        a, b = freefield.sw_normal_on_plane_wave(p, m, r)
        want = a * psi + b * synth.plane_wave(dims, p + shift, u)
        assert np.abs(SW.apply_normal(U, psi, m, r, bc) - want).max() < 1e-12
        # Gamma_55 alone moves p by pi(0,1,0,1) with weight prod cos p
        c = np.prod(np.cos(p))
        g = SW.gamma55_subsets(U, psi, bc)
        assert np.abs(g - c * synth.plane_wave(dims, p + shift, u)).max() < 1e-12


def test_sw_free_dense_spectrum_and_norm_bound():
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, "unit")
    for m in (1e-3,):
        ev = np.linalg.eigvalsh(dense_sw_normal("unit", m)[1])
        assert np.abs(ev - freefield.sw_spectrum(dims, m)).max() < 1e-12
        lo, hi = freefield.extreme_eigenvalues(False, m)
        assert abs(ev[0] - lo) < 1e-12 and abs(ev[-1] - hi) < 1e-12
    Uh = synth.gauge_field(dims, "haar", 61)
    G = dense.dense_matrix(lambda v: SW.gamma55_subsets(Uh, v), synth.field_shape(dims, 1))
    assert np.abs(G - G.conj().T).max() < 1e-15
    assert np.abs(np.linalg.eigvalsh(G)).max() <= 1.0 + 1e-12


def test_sw_free_dst_commutes_with_gamma55_only_with_right_phase():
    """At U = 1 on 6^4, [D_st, Gamma_55] = 0 for phi = (-1)^(x2+x4); a wrong
    phase such as (-1)^(x1+x3) does not commute there."""
    dims = (6, 6, 6, 6)
    U = synth.gauge_field(dims, "unit")
    psi = synth.gaussian_field(dims, synth.STAGGERED_WILSON, 71)
    lhs = SW.dst(U, SW.gamma55_subsets(U, psi))
    rhs = SW.gamma55_subsets(U, SW.dst(U, psi))
    assert np.abs(lhs - rhs).max() < 1e-13
    x = lattice.coords(dims)
    wrong = np.where((x[0] + x[2]) % 2 == 0, 1.0, -1.0) * SW.phi(dims)
    g_wrong = lambda v: lattice.site_mul(wrong, SW.gamma55_subsets(U, v))
    diff = SW.dst(U, g_wrong(psi)) - g_wrong(SW.dst(U, psi))
    assert np.abs(diff).max() > 1e-2


# ---------------------------------------------------------------- solvers
def test_cg_terminates_in_number_of_distinct_eigenvalues():
    """Textbook CG property: with k distinct eigenvalues CG converges in k steps."""
    rng = np.random.default_rng(5)
    n, k = 60, 5
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    d = np.repeat(np.array([1.0, 2.0, 3.5, 7.0, 11.0]), n // k)
    A = (Q * d) @ Q.conj().T
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, info = solvers.cg(lambda v: A @ v, b, 1e-10, 100)
    assert info["iterations"] == k
    assert np.abs(x - np.linalg.solve(A, b)).max() < 1e-10


@pytest.mark.parametrize("formulation", [synth.WILSON, synth.STAGGERED_WILSON])
def test_cgnr_matches_dense_lu_4x4(formulation):
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, "haar", 1000)
    chi = synth.point_source(dims, formulation, 0)
    m = 0.5
    x, info = solvers.cgnr(formulation, U, chi, m, 1e-10, 5000)
    assert info["status"] == solvers.CONVERGED
    assert info["true_residual"] <= 1e-10
    if formulation == synth.WILSON:
        M = dense.dense_matrix(lambda v: W.apply(U, v, m), synth.field_shape(dims, formulation))
    else:
        M = dense_sw_normal("haar", m)[0]
    x_lu = np.linalg.solve(M, chi.ravel())
    # kappa(A) on this field is O(10) (Lanczos below), so the error is ~1e-9
    assert np.linalg.norm(x.ravel() - x_lu) / np.linalg.norm(x_lu) <= 1e-8


def test_cg_detects_breakdown_and_maxiter():
    A = lambda v: v * 2.0
    b = np.ones(8, dtype=complex)
    b[3] = np.nan
    _, info = solvers.cg(A, b, 1e-10, 10)
    assert info["status"] == solvers.BREAKDOWN
    Aop = lambda v: np.arange(1, 9) * v
    _, info = solvers.cg(Aop, np.ones(8, dtype=complex), 1e-14, 3)
    assert info["status"] == solvers.NOT_CONVERGED and info["iterations"] == 3


def test_lanczos_known_spectrum_and_dense_sw():
    rng = np.random.default_rng(9)
    n = 40
    d = np.linspace(0.5, 9.0, n)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    A = (Q * d) @ Q.conj().T
    a, b = solvers.lanczos(lambda v: A @ v, rng.standard_normal(n) + 0j, n)
    assert np.abs(np.sort(solvers.ritz_values(a, b)) - d).max() < 1e-10

    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, "haar", 1000)
    m = 0.5
    ev = np.linalg.eigvalsh(dense_sw_normal("haar", m)[1])
    v0 = synth.gaussian_field(dims, synth.STAGGERED_WILSON, 7)
    lmin, lmax, kappa, _ = solvers.condition_number(synth.STAGGERED_WILSON, U, m, v0, 200)
    assert lmin >= ev[0] - 1e-10 and lmax <= ev[-1] + 1e-10   # Cauchy interlacing
    assert abs(lmax - ev[-1]) / ev[-1] < 1e-8
    assert abs(lmin - ev[0]) / ev[0] < 1e-6
    assert kappa <= ev[-1] / ev[0] * (1 + 1e-10)


# ------------------------------------------------------ even-odd (Schur) CG
def test_evenodd_schur_complement_is_block_elimination():
    """With x_o = -M_oe x_e / d, the full operator gives M (x_e + x_o) =
    M^ x_e on the even sites and 0 on the odd ones: the Schur complement is
    what eliminating the odd half leaves (a dropped 1/d, a sign or a swapped
    parity in schur_apply or reconstruct fails this)."""
    dims = (4, 6, 4, 4)
    bc = (1, 1, 1, -1)
    U = synth.gauge_field(dims, "haar", 31)
    m = -0.23
    xe = EO.project(synth.gaussian_field(dims, synth.WILSON, 3), EO.EVEN)
    full = EO.reconstruct(U, xe, np.zeros_like(xe), m, bc)     # x_e + x_o with chi = 0
    Mx = W.apply(U, full, m, 1.0, bc)
    assert np.abs(EO.project(Mx, EO.ODD)).max() < 1e-13
    assert np.abs(EO.project(Mx, EO.EVEN) - EO.schur_apply(U, xe, m, bc)).max() < 1e-12
    # the odd half of the schur image is zero, and the parities split the lattice evenly
    assert np.abs(EO.project(EO.schur_apply(U, xe, m, bc), EO.ODD)).max() == 0.0
    assert (EO.parity(dims) == 0).sum() * 2 == np.prod(dims)


def test_evenodd_adjoint_and_gamma5_hermiticity():
    dims = (4, 4, 4, 6)
    bc = (1, 1, 1, -1)
    U = synth.gauge_field(dims, "haar", 12)
    m = 0.11
    x = EO.project(synth.gaussian_field(dims, synth.WILSON, 4), EO.EVEN)
    y = EO.project(synth.gaussian_field(dims, synth.WILSON, 5), EO.EVEN)
    Mx = EO.schur_apply(U, x, m, bc)
    Mdy = EO.schur_apply(U, y, m, bc, dagger=True)
    assert abs(_inner(y, Mx) - _inner(Mdy, x)) < 1e-11
    g5 = W.gamma5(EO.schur_apply(U, W.gamma5(x), m, bc))
    assert np.abs(g5 - EO.schur_apply(U, x, m, bc, dagger=True)).max() < 1e-13


def test_evenodd_solution_matches_dense_lu_4x4():
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, "haar", 1000)
    chi = synth.point_source(dims, synth.WILSON, 0)
    m = 0.5
    x, info = EO.cgnr(U, chi, m, 1e-11, 5000)
    assert info["status"] == solvers.CONVERGED
    M = dense.dense_matrix(lambda v: W.apply(U, v, m), synth.field_shape(dims, synth.WILSON))
    x_lu = np.linalg.solve(M, chi.ravel())
    assert np.linalg.norm(x.ravel() - x_lu) / np.linalg.norm(x_lu) <= 1e-9
    assert info["full_residual"] <= 1e-10


def test_evenodd_more_than_halves_cg_iterations():
    """The footnote to eq. (2): preconditioning the Wilson inversion gains more
    than a factor 2.  Per iteration the Schur operator costs the same hops as
    M_W (four half-lattice hop terms), so the iteration ratio is the gain."""
    dims = (8, 8, 8, 8)
    U = synth.gauge_field(dims, "near_identity", 2000, 0.4359375)
    chi = synth.point_source(dims, synth.WILSON, 0)
    m = -0.3
    x0, i0 = solvers.cgnr(synth.WILSON, U, chi, m, 1e-8, 20000)
    x1, i1 = EO.cgnr(U, chi, m, 1e-8, 20000)
    assert i0["status"] == solvers.CONVERGED and i1["status"] == solvers.CONVERGED
    assert i1["iterations"] < 0.5 * i0["iterations"]
    assert np.linalg.norm(x1 - x0) / np.linalg.norm(x0) < 1e-5


# --------------------------------------------------------- pion correlator
def test_pion_correlator_free_field_closed_form():
    """Propagators solved by the oracle's CG at U = 1 against the momentum-space
    closed form (antiperiodic time, so p4 != 0 and the spectrum has no zero)."""
    dims = (4, 4, 4, 8)
    bc = (1, 1, 1, -1)
    U = np.zeros(synth.site_shape(dims) + (4, 3, 3), dtype=np.complex128)
    U[...] = np.eye(3)
    m = 0.2
    props = []
    for a in range(12):
        chi = synth.point_source(dims, synth.WILSON, a)
        x, info = solvers.cgnr(synth.WILSON, U, chi, m, 1e-12, 5000, bc=bc)
        assert info["status"] == solvers.CONVERGED
        props.append(x)
    C = SP.pion_correlator(np.stack(props))
    ref = SP.free_pion_correlator(dims, m, bc)
    assert np.abs(C - ref).max() / ref.max() < 1e-9
    # time reflection of the free field: C(t) = C(L4 - t)
    assert np.abs(C[1:] - C[1:][::-1]).max() / C.max() < 1e-9


def test_effective_mass_of_a_cosh_is_its_mass():
    L, mass = 16, 0.37
    t = np.arange(L)
    C = 2.5 * np.cosh(mass * (t - L / 2))
    meff = SP.effective_mass(C)
    # t = 0 is the wrap-around kink of the periodic cosh: no real solution there
    assert np.abs(meff[1:] - mass).max() < 1e-12 and np.isnan(meff[0])
    assert np.isnan(SP.effective_mass(np.array([1.0, 5.0, 1.0, 5.0]))[1])


# ------------------------------------------------------- spectrum of D_SW
def _multiset(z, nd=8):
    return sorted(zip(np.round(np.real(z), nd), np.round(np.imag(z), nd)))


def test_sw_free_spectrum_closed_form():
    dims = (4, 4, 4, 4)
    U = np.zeros(synth.site_shape(dims) + (4, 3, 3), dtype=np.complex128)
    U[...] = np.eye(3)
    ev = SPEC.dense_eigenvalues(synth.STAGGERED_WILSON, U, m=0.1)
    re, im = SPEC.sw_free_real_imag(dims, m=0.1)
    assert _multiset(ev.real + 1j * np.abs(ev.imag)) == _multiset(re + 1j * im)


def test_sw_spectrum_is_closed_under_conjugation():
    """epsilon-hermiticity (D_SW^dag = epsilon D_SW epsilon) makes the
    characteristic polynomial real: eigenvalues come in conjugate pairs."""
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, "haar", 1000)
    ev = SPEC.dense_eigenvalues(synth.STAGGERED_WILSON, U)
    assert _multiset(ev, 7) == _multiset(np.conj(ev), 7)
    near = SPEC.nearest(ev, 0.3, 6)
    assert np.all(np.diff(np.abs(near - 0.3)) >= 0)
    assert np.abs(near - 0.3).max() <= np.sort(np.abs(ev - 0.3))[5] + 1e-15


# ------------------------------------------------------------------- m_c search
@pytest.mark.parametrize("formulation", [synth.WILSON, synth.STAGGERED_WILSON])
def test_critical_mass_search_free_field_is_zero(formulation):
    """On the free field (U = 1, periodic) the lowest eigenvalue of
    (D+m)^dag (D+m) is m^2 for both operators (p = 0: the Wilson term and
    r(1 - Gamma_55) vanish there), so the mass minimising theta_min is
    m_c = 0 and theta_min(m) = m^2.  The bracket is asymmetric so that no
    grid point lands on 0: the search must find it by the golden section.
    A sign slip in the mass, a wrong bracket update or a max instead of a
    min all move the answer away from 0."""
    from oracle import critical
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, "unit", 0)
    v0 = synth.gaussian_field(dims, formulation, 7)
    for m in (-0.21, 0.13):
        th = critical.theta_min(formulation, U, m, v0, 60)
        assert abs(th - m * m) <= 1e-10, (m, th)
    lo, hi, ngrid, ngolden = -0.35, 0.25, 7, 10
    mc, th, trace = critical.critical_mass(formulation, U, v0, lo, hi, steps=60, ngrid=ngrid,
                                           ngolden=ngolden)
    grid = np.linspace(lo, hi, ngrid)
    assert np.min(np.abs(grid)) > 0.04            # no grid point at the answer
    # the golden section shrinks the two-cell bracket by 0.618 per step
    width = 2 * (hi - lo) / (ngrid - 1) * ((np.sqrt(5) - 1) / 2) ** ngolden
    assert abs(mc) <= width, (mc, width)
    assert abs(th - mc * mc) <= 1e-10
    assert all(t >= mm * mm - 1e-12 for mm, t in trace)


# ---------------------------------------------------- staggered overlap (oracle)
from oracle import overlap as OV  # noqa: E402


def _ov_field(kind):
    dims = (4, 4, 4, 4)
    return dims, synth.gauge_field(dims, kind, 1000 if kind == "haar" else 0)


@pytest.mark.parametrize("kind", ["unit", "haar"])
def test_overlap_dense_ginsparg_wilson_and_epsilon_hermiticity(kind):
    """D_ov = rho (1 + epsilon sign(epsilon A)), A = D_SW - rho: epsilon-
    hermitian, V = D_ov / rho - 1 unitary, the Ginsparg-Wilson relation
    epsilon D + D epsilon = D epsilon D / rho, and every eigenvalue on the
    circle |lambda - rho| = rho.  A wrong epsilon, a missing sign or a
    non-hermitian H breaks each of these."""
    dims, U = _ov_field(kind)
    rho = 1.0
    D, A, eps = OV.dense_overlap(U, rho)
    n = D.shape[0]
    scale = np.abs(D).max()
    assert np.abs(eps @ D @ eps - D.conj().T).max() <= 1e-12 * scale
    V = D / rho - np.eye(n)
    assert np.abs(V.conj().T @ V - np.eye(n)).max() <= 1e-12
    gw = eps @ D + D @ eps - D @ eps @ D / rho
    assert np.abs(gw).max() <= 1e-12 * scale
    ev = np.linalg.eigvals(D)
    assert np.abs(np.abs(ev - rho) - rho).max() <= 1e-11
    # with a mass: (1 - m/(2 rho)) D + m, the circle moves accordingly
    Dm, _, _ = OV.dense_overlap(U, rho, m=0.1)
    assert np.abs(Dm - ((1 - 0.1 / (2 * rho)) * D + 0.1 * np.eye(n))).max() <= 1e-13 * scale


def test_overlap_sign_is_the_unitary_polar_factor():
    """epsilon sign(epsilon A) (eigen-decomposition of the hermitian H) equals
    the unitary factor of A's polar decomposition A = V P computed
    independently from the SVD: V = W Z^dag for A = W S Z^dag."""
    dims, U = _ov_field("haar")
    rho = 1.0
    D, A, eps = OV.dense_overlap(U, rho)
    V = D / rho - np.eye(D.shape[0])
    W, _, Zh = np.linalg.svd(A)
    assert np.abs(V - W @ Zh).max() <= 1e-11


def test_overlap_free_field_closed_form():
    """At U = 1 the kernel is normal and the overlap eigenvalues are
    rho (1 + z/|z|) over the closed-form staggered Wilson spectrum z + rho
    (Re and |Im| compared as multisets)."""
    dims, U = _ov_field("unit")
    for rho, m in ((1.0, 0.0), (1.5, 0.2)):
        D, _, _ = OV.dense_overlap(U, rho, m=m)
        ev = np.linalg.eigvals(D)
        got = np.sort_complex(np.round(ev.real + 1j * np.abs(ev.imag), 9))
        want = np.sort_complex(np.round(OV.free_spectrum(dims, rho, m=m), 9))
        assert np.abs(got - want).max() <= 1e-8


def test_overlap_polynomial_converges_to_dense():
    """The Chebyshev approximation of (A^dag A)^{-1/2} on [lo, hi] containing
    the spectrum of A^dag A: the polynomial itself meets its error bound at
    random points, and D_ov psi from it is within rho * bound * |psi| of the
    dense exact D_ov psi, with an error that falls as the degree grows.  On
    the near-identity field of the workload's spread the kernel is well
    conditioned (kappa(A^dag A) ~ 90 at rho = 1); on Haar-random links A is
    nearly singular and a polynomial alone converges too slowly."""
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, "near_identity", 1000, 0.436)
    rho, m = 1.0, 0.05
    D, A, _ = OV.dense_overlap(U, rho, m=m)
    s = np.linalg.svd(A, compute_uv=False)
    lo, hi = 0.9 * s.min() ** 2, 1.1 * s.max() ** 2
    psi = synth.gaussian_field(dims, synth.STAGGERED_WILSON, 3)
    exact = (D @ psi.ravel()).reshape(psi.shape)
    rng = np.random.default_rng(5)
    errs = []
    for deg in (40, 80, 160):
        c = OV.cheb_coeffs_invsqrt(lo, hi, deg)
        bound = OV.poly_sign_error(lo, hi, deg)
        x = rng.uniform(lo, hi, 200)
        assert np.max(np.abs(np.sqrt(x) * OV.cheb_eval(c, lo, hi, x) - 1)) <= bound * (1 + 1e-9)
        got = OV.overlap_apply_poly(U, psi, rho, m, lo, hi, deg)
        err = np.linalg.norm(got - exact) / np.linalg.norm(psi)
        assert err <= (rho - m / 2) * bound * (1 + 1e-6) + 1e-12, (deg, err, bound)
        errs.append(err)
    assert errs[2] < errs[1] < errs[0]
    assert errs[2] <= 1e-11
