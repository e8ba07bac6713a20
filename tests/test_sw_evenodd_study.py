"""Pins of the even-odd block elimination of the staggered Wilson matrix (CPU).

The study module recovers M_SW as a sparse matrix by probing the oracle's
matvec and takes its parity blocks.  These tests hold it to things fixed
independently of it: the oracle's own D_st and Gamma_55 (which parity each
term connects), the free-field closed form of the spectrum (D_st and Gamma_55
commute at U = 1, so the diagonal blocks carry the real parts m + r (1 -+ c)),
and dense LU for the reconstructed solution.
"""
import numpy as np
import pytest

import synth
from oracle import evenodd_sw as E
from oracle import spectrum as SPEC
from oracle import staggered_wilson as SW


def _fields(dims, seed):
    U = synth.gauge_field(dims, "haar", seed)
    v = synth.gaussian_field(dims, synth.STAGGERED_WILSON, seed + 1)
    return U, v


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 6, 8)])
def test_probed_matrix_is_the_oracle_matvec(dims):
    """(6, 4, 6, 8): probe periods 3, 4, 3, 4, so every probe covers many sites."""
    U, v = _fields(dims, 11)
    B = E.Blocks(U, -0.3)
    ref = SW.apply(U, v, -0.3)
    assert np.abs(B.M @ v.ravel() - ref.ravel()).max() <= 1e-13


def test_parity_blocks_are_dst_and_gamma55():
    """Off-diagonal blocks are exactly D_st; diagonal blocks are (m + r) - r Gamma_55."""
    dims = (4, 4, 6, 4)
    U, v = _fields(dims, 21)
    m, r = -0.3, 1.0
    B = E.Blocks(U, m, r)
    flat = v.ravel()
    ve = np.zeros_like(flat)
    vo = np.zeros_like(flat)
    ve[B.e] = flat[B.e]
    vo[B.o] = flat[B.o]
    shape = v.shape
    dst_o = SW.dst(U, vo.reshape(shape)).ravel()
    g55_e = SW.gamma55_paths(U, ve.reshape(shape)).ravel()
    assert np.abs(B.Deo @ flat[B.o] - dst_o[B.e]).max() <= 1e-13
    assert np.abs(dst_o[B.o]).max() == 0.0
    assert np.abs(B.Aee @ flat[B.e] - ((m + r) * flat[B.e] - r * g55_e[B.e])).max() <= 1e-13
    assert np.abs(g55_e[B.o]).max() == 0.0
    assert abs(B.Aee - B.Aee.conj().T).max() <= 1e-15
    assert abs(B.Doe + B.Deo.conj().T).max() == 0.0


@pytest.mark.parametrize("dims,m", [((4, 4, 4, 4), -0.3), ((6, 4, 4, 4), -0.5)])
def test_free_field_diagonal_blocks_carry_the_real_parts(dims, m):
    """At U = 1 the eigenvalues of A_ee and A_oo together are the real parts
    m + r (1 -+ prod cos p) of the closed-form spectrum, and the two parities
    have the same spectrum.  With L1 = 6, prod cos p takes the value 1/2
    (cos(pi/3) = 1/2), so at m + r = 1/2 the block is singular: m + r lies
    inside Gamma_55's spectrum."""
    U = np.zeros(synth.site_shape(dims) + (4, 3, 3), dtype=np.complex128)
    U[...] = np.eye(3)
    B = E.Blocks(U, m)
    ee = np.linalg.eigvalsh(B.Aee.toarray())
    oo = np.linalg.eigvalsh(B.Aoo.toarray())
    re, _ = SPEC.sw_free_real_imag(dims, m)
    assert np.abs(np.sort(np.concatenate([ee, oo])) - np.sort(re)).max() <= 1e-12
    assert np.abs(ee - oo).max() <= 1e-12
    if dims == (6, 4, 4, 4):
        assert np.abs(oo).min() <= 1e-12


@pytest.mark.parametrize("m", [0.2, -0.3])
def test_schur_solve_equals_dense_solution(m):
    """m = 0.2: A_oo positive definite; m = -0.3: indefinite.  The even-odd
    solution equals dense LU, S is hermitian, and eq. (2)'s residual is met."""
    dims = (4, 4, 4, 4)
    U, v = _fields(dims, 31)
    B = E.Blocks(U, m)
    chi = synth.point_source(dims, synth.STAGGERED_WILSON, 1).ravel()
    x, info = E.solve(B, chi, 1e-10, 1e-13)
    ref = np.linalg.solve(B.M.toarray(), chi)
    assert np.linalg.norm(x - ref) <= 1e-7 * np.linalg.norm(ref)
    assert info["eq2_residual"] <= 1e-9
    S = E.Schur(B, 1e-13)
    a = v.ravel()[B.e]
    b = synth.gaussian_field(dims, synth.STAGGERED_WILSON, 5).ravel()[B.e]
    assert abs(np.vdot(a, S(b)) - np.vdot(S(a), b)) <= 1e-10 * np.linalg.norm(a) * np.linalg.norm(b)


def test_cost_accounting():
    """Outer CG with n applications of S^2 sweeps 2n + 1 S's (plus S b^_e); each
    S is one Gamma_55 sweep of the even sites; the inner sweeps come on top."""
    g, d = E.cost_in_half_sweeps(10, 500)
    assert (g, d) == (21 + 500, 2 * 21 + 2)
    assert E.unpreconditioned_cost(99) == (400, 400)
