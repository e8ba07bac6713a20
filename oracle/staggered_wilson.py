"""2-flavour staggered Wilson Dirac matrix for the oracle.

The paper omits the operator (Sec. 2) and refers to Adams, PLB 699 (2011) 394.
This module implements the reading stated for the build: the staggered hopping
term plus the Golterman-Smit flavoured mass term r (1 - Gamma_55), where
Gamma_55 is the epsilon*eta_5-signed symmetrised product of the four link
averaging shifts C_1 C_2 C_3 C_4.  It couples each site to 8 + 16 others
(Sec. 3: "8+16 other sites").  With r = 1 it reproduces the paper's free-field
limit kappa_W^{1/2}/kappa_SW^{1/2} -> 8/sqrt(5) (Sec. 3).

    (V_mu psi)(x)     = U_mu(x) psi(x + mu)
    (V_mu^dag psi)(x) = U_mu(x - mu)^dag psi(x - mu)
    C_mu  = (V_mu + V_mu^dag) / 2
    D_st  = sum_mu eta_mu (V_mu - V_mu^dag) / 2             (anti-hermitian)
    Gamma_55 = phi (1/24) sum_{pi in S4} C_pi1 C_pi2 C_pi3 C_pi4,
               phi(x) = epsilon(x) eta_5(x) = (-1)^(x2 + x4)  (hermitian)
    M_SW = D_st + r (1 - Gamma_55) + m
    M_SW^dag = epsilon M_SW epsilon = -D_st + r (1 - Gamma_55) + m   (Sec. 2)

Gamma_55 is given in three equivalent forms, each written independently:
``gamma55_paths`` applies all 24 x 16 = 384 one-link-per-direction paths one
operator at a time; ``gamma55_subsets`` uses the subset recursion
F_S = sum_{mu in S} C_mu F_{S \\ mu}; ``gamma55_corners`` uses per-site
path-averaged corner matrices W_s(x), s in {+-1}^4, built by walking link
paths on explicit site coordinates.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import lattice
from .gauge import dag, link, shift_links

PERMS = list(itertools.permutations(range(4)))
SIGNS = list(itertools.product((1, -1), repeat=4))


def colour_mul(A, psi):
    return np.matmul(A, psi[..., None])[..., 0]


def hop(U, psi, mu, sign, bc=(1, 1, 1, 1)):
    """V_mu psi for sign = +1, V_mu^dag psi for sign = -1."""
    if sign > 0:
        return colour_mul(link(U, mu), lattice.shift(psi, mu, +1, bc))
    return colour_mul(dag(shift_links(link(U, mu), mu, -1)), lattice.shift(psi, mu, -1, bc))


def C(U, psi, mu, bc=(1, 1, 1, 1)):
    return 0.5 * (hop(U, psi, mu, +1, bc) + hop(U, psi, mu, -1, bc))


def dst(U, psi, bc=(1, 1, 1, 1)):
    """Staggered hopping term D_st psi."""
    dims = lattice.dims_of(psi)
    out = np.zeros_like(psi)
    for mu in range(4):
        d = 0.5 * (hop(U, psi, mu, +1, bc) - hop(U, psi, mu, -1, bc))
        out = out + lattice.site_mul(lattice.eta(dims, mu), d)
    return out


def phi(dims):
    """phi(x) = epsilon(x) eta_5(x)."""
    return lattice.epsilon(dims) * lattice.eta5(dims)


def gamma55_paths(U, psi, bc=(1, 1, 1, 1)):
    """Gamma_55 psi by brute force: for every ordering pi and every choice of
    V or V^dag per factor, apply the four one-link shifts right to left."""
    dims = lattice.dims_of(psi)
    acc = np.zeros_like(psi)
    for pi in PERMS:
        for s in SIGNS:
            v = psi
            for k in (3, 2, 1, 0):
                v = hop(U, v, pi[k], s[k], bc)
            acc = acc + v
    return lattice.site_mul(phi(dims), acc / (24.0 * 16.0))


def gamma55_subsets(U, psi, bc=(1, 1, 1, 1)):
    """Gamma_55 psi by the subset recursion F_S = sum_{mu in S} C_mu F_{S\\mu};
    the sum over the 24 orderings equals F_{1234}."""
    dims = lattice.dims_of(psi)
    F = {(): psi}
    for k in range(1, 5):
        for S in itertools.combinations(range(4), k):
            acc = np.zeros_like(psi)
            for mu in S:
                rest = tuple(nu for nu in S if nu != mu)
                acc = acc + C(U, F[rest], mu, bc)
            F[S] = acc
    return lattice.site_mul(phi(dims), F[(0, 1, 2, 3)] / 24.0)


def _gather_links(U, mu, y):
    """U_mu at integer coordinates y = (y1, y2, y3, y4) (taken mod L)."""
    dims = lattice.dims_of(U)
    i = [np.mod(y[k], dims[k]) for k in range(4)]
    return U[i[3], i[2], i[1], i[0], mu]


def corners(U):
    """W_s(x) for all 16 s, shape (16, L4, L3, L2, L1, 3, 3), ordered as SIGNS.

    W_s(x) = (1/24) sum_pi L(y0, s_pi1 pi1) L(y1, s_pi2 pi2) L(y2, ...) L(y3, ...),
    y0 = x, y_k = y_{k-1} + s_{pi_k} pi_k-hat, with L(y, +mu) = U_mu(y) and
    L(y, -mu) = U_mu(y - mu)^dag.  Gauge links are periodic; fermion boundary
    signs are applied where psi(x + s) is read, not here.
    """
    dims = lattice.dims_of(U)
    x = lattice.coords(dims)
    out = np.zeros((16,) + U.shape[:4] + (3, 3), dtype=np.complex128)
    for si, s in enumerate(SIGNS):
        acc = np.zeros(U.shape[:4] + (3, 3), dtype=np.complex128)
        for pi in PERMS:
            y = [x[k].copy() for k in range(4)]
            P = None
            for mu in pi:
                if s[mu] > 0:
                    L = _gather_links(U, mu, y)
                    y[mu] = y[mu] + 1
                else:
                    y[mu] = y[mu] - 1
                    L = dag(_gather_links(U, mu, y))
                P = L if P is None else P @ L
            acc = acc + P
        out[si] = acc / 24.0
    return out


def corner_bc_sign(dims, s, bc):
    """Product of bc[mu] over the directions in which x -> x + s wraps."""
    x = lattice.coords(dims)
    sign = np.ones(x[0].shape)
    for mu in range(4):
        if bc[mu] == 1:
            continue
        wraps = (x[mu] + s[mu] < 0) | (x[mu] + s[mu] >= dims[mu])
        sign = np.where(wraps, sign * bc[mu], sign)
    return sign


def gather_field(psi, s):
    """psi(x + s) for a diagonal offset s (periodic gather on coordinates)."""
    dims = lattice.dims_of(psi)
    x = lattice.coords(dims)
    i = [np.mod(x[k] + s[k], dims[k]) for k in range(4)]
    return psi[i[3], i[2], i[1], i[0]]


def gamma55_corners(W, psi, bc=(1, 1, 1, 1)):
    """Gamma_55 psi(x) = phi(x) (1/16) sum_s W_s(x) psi(x + s)."""
    dims = lattice.dims_of(psi)
    acc = np.zeros_like(psi)
    for si, s in enumerate(SIGNS):
        v = colour_mul(W[si], gather_field(psi, s))
        acc = acc + lattice.site_mul(corner_bc_sign(dims, s, bc), v)
    return lattice.site_mul(phi(dims), acc / 16.0)


def apply(U, psi, m, r=1.0, bc=(1, 1, 1, 1), dagger=False, g55=None):
    """M_SW psi (or M_SW^dag psi).  ``g55`` optionally supplies Gamma_55 psi
    computed by another form; by default the subset recursion is used."""
    if g55 is None:
        g55 = gamma55_subsets(U, psi, bc)
    d = dst(U, psi, bc)
    if dagger:
        d = -d
    return d + (r + m) * psi - r * g55


def apply_normal(U, psi, m, r=1.0, bc=(1, 1, 1, 1)):
    """A psi = M_SW^dag M_SW psi, eq. (2)."""
    return apply(U, apply(U, psi, m, r, bc), m, r, bc, dagger=True)


def epsilon_mul(psi):
    return lattice.site_mul(lattice.epsilon(lattice.dims_of(psi)), psi)
