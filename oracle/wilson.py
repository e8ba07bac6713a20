"""Usual Wilson Dirac matrix for the oracle (Sec. 2, eq. (2) of the paper).

    (M_W psi)(x) = (m + 4r) psi(x)
                   - 1/2 sum_mu [ (r - gamma_mu) U_mu(x) psi(x + mu)
                                + (r + gamma_mu) U_mu(x - mu)^dag psi(x - mu) ]

M_W = D_W + m is gamma_5-hermitian, gamma_5 M_W gamma_5 = M_W^dag (Sec. 2), so the
adjoint swaps r - gamma_mu and r + gamma_mu.  The paper uses r = 1 (its free-field
8/sqrt(5) limit of Sec. 3 requires it); r is kept as a parameter.

Gamma basis (Euclidean, hermitian; the paper does not state one, and every
quantity compared here is basis-independent except per-source iteration
counts): in 2x2 blocks,
    gamma_1 = [[0, i s1], [-i s1, 0]],  gamma_2 = [[0, -i s2], [i s2, 0]],
    gamma_3 = [[0, i s3], [-i s3, 0]],  gamma_4 = [[0, 1], [1, 0]],
with Pauli matrices s1, s2, s3; then gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4 =
diag(1, 1, -1, -1).
"""
from __future__ import annotations

import numpy as np

from . import lattice
from .gauge import dag, link, shift_links

_s1 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_s2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_s3 = np.array([[1, 0], [0, -1]], dtype=np.complex128)
_I2 = np.eye(2, dtype=np.complex128)
_Z2 = np.zeros((2, 2), dtype=np.complex128)


def _block(ur, ll):
    return np.block([[_Z2, ur], [ll, _Z2]])


GAMMA = np.array([
    _block(1j * _s1, -1j * _s1),
    _block(-1j * _s2, 1j * _s2),
    _block(1j * _s3, -1j * _s3),
    _block(_I2, _I2),
])
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]


def spin_mul(g, psi):
    """Apply a 4x4 spin matrix at every site: (g psi)_s = sum_t g_st psi_t."""
    return np.matmul(g, psi)


def colour_mul(A, psi):
    """Apply a site field of 3x3 colour matrices to a Wilson field."""
    return np.matmul(psi, np.swapaxes(A, -1, -2))


def apply(U, psi, m, r=1.0, bc=(1, 1, 1, 1), dagger=False):
    """M_W psi (or M_W^dag psi) with M_W = D_W + m as in the module docstring."""
    sg = -1.0 if dagger else 1.0
    one = np.eye(4, dtype=np.complex128)
    out = (m + 4.0 * r) * psi
    for mu in range(4):
        Umu = link(U, mu)
        fwd = colour_mul(Umu, lattice.shift(psi, mu, +1, bc))
        bwd = colour_mul(dag(shift_links(Umu, mu, -1)), lattice.shift(psi, mu, -1, bc))
        out = out - 0.5 * (spin_mul(r * one - sg * GAMMA[mu], fwd)
                           + spin_mul(r * one + sg * GAMMA[mu], bwd))
    return out


def apply_normal(U, psi, m, r=1.0, bc=(1, 1, 1, 1)):
    """A psi = M_W^dag M_W psi, the matrix of the normal equations, eq. (2)."""
    return apply(U, apply(U, psi, m, r, bc), m, r, bc, dagger=True)


def gamma5(psi):
    return spin_mul(GAMMA5, psi)


def momentum_matrix(p, m, r=1.0):
    """Free-field (U = 1) symbol: M_W(p) = m + r sum(1 - cos p) + i sum gamma_mu sin p_mu.

    Derived from the position-space formula acting on exp(i p.x) u.
    """
    M = (m + r * np.sum(1.0 - np.cos(p))) * np.eye(4, dtype=np.complex128)
    for mu in range(4):
        M = M + 1j * np.sin(p[mu]) * GAMMA[mu]
    return M
