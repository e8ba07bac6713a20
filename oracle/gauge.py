"""Gauge-field utilities for the oracle: plaquette, gauge transformations, tuning.

The paper's ensemble is quenched beta = 6 on 16^3 x 32 (Sec. 3).  Its synthetic
stand-in is a field of independent near-identity links whose mean plaquette is
tuned to the typical beta = 6 value 0.594 by bisection on the spread epsilon.
"""
from __future__ import annotations

import numpy as np

from . import lattice

import synth


def link(U, mu):
    """U_mu(x) as a site field of 3x3 matrices."""
    return U[..., mu, :, :]


def dag(a):
    return np.conj(np.swapaxes(a, -1, -2))


def shift_links(A, mu, sign):
    """Periodic shift of a matrix-valued site field: B(x) = A(x + sign*mu)."""
    return np.roll(A, -sign, axis=lattice.axis(mu))


def plaquette(U):
    """Mean plaquette (1/6V) sum_x sum_{mu<nu} (1/3) Re tr U_mu(x) U_nu(x+mu)
    U_mu(x+nu)^dag U_nu(x)^dag."""
    tot = 0.0
    V = np.prod(U.shape[:4])
    for mu in range(4):
        for nu in range(mu + 1, 4):
            a = link(U, mu)
            b = shift_links(link(U, nu), mu, +1)
            c = dag(shift_links(link(U, mu), nu, +1))
            d = dag(link(U, nu))
            p = a @ b @ c @ d
            tot += np.trace(p, axis1=-2, axis2=-1).real.sum() / 3.0
    return tot / (6.0 * V)


def transform_links(U, g):
    """U^g_mu(x) = g(x) U_mu(x) g(x + mu)^dag (periodic links)."""
    out = np.empty_like(U)
    for mu in range(4):
        out[..., mu, :, :] = g @ link(U, mu) @ dag(shift_links(g, mu, +1))
    return out


def transform_fermion(g, psi, formulation):
    """psi^g(x) = g(x) psi(x), colour rotation at each site (and each spin)."""
    if formulation == synth.WILSON:
        return np.einsum("...ab,...sb->...sa", g, psi)
    return np.einsum("...ab,...b->...a", g, psi)


def tune_epsilon(dims, seed, target=0.594, lo=0.3, hi=0.6, tol=5e-4, maxit=40):
    """Bisection on epsilon so that the near-identity field's mean plaquette hits
    ``target`` within ``tol``.  The plaquette decreases with epsilon."""
    def plaq(eps):
        return plaquette(synth.gauge_field(dims, "near_identity", seed, eps))

    p_lo, p_hi = plaq(lo), plaq(hi)
    if not (p_lo > target > p_hi):
        raise ValueError(f"target plaquette not bracketed: P({lo})={p_lo}, P({hi})={p_hi}")
    for _ in range(maxit):
        mid = 0.5 * (lo + hi)
        pm = plaq(mid)
        if abs(pm - target) <= tol:
            return mid, pm
        if pm > target:
            lo = mid
        else:
            hi = mid
    return mid, pm
