"""Closed-form free-field (U = 1) spectra of A = M^dag M for both formulations.

These give the paper's free-field comparison (Sec. 3): with the same bare mass
m and r = 1, kappa_W^{1/2} / kappa_SW^{1/2} -> 8/sqrt(5) as m -> 0.

Momenta: p_mu = (2 pi n_mu + theta_mu) / L_mu, theta_mu = 0 (periodic) or pi
(antiperiodic fermion boundary).

Wilson: M_W(p) = a(p) + i sum gamma_mu sin p_mu with a(p) = m + r sum(1 - cos p);
since the gamma_mu anticommute, M_W(p)^dag M_W(p) = a(p)^2 + sum sin^2 p times
the identity (4 spins x 3 colours).

Staggered Wilson: at U = 1, D_st^2 = sum_mu nabla_mu^2 (the eta phases make
the cross terms cancel), and D_st commutes with Gamma_55.  Gamma_55 maps
exp(i p.x) to c(p) exp(i (p + pi(0,1,0,1)).x) with c(p) = prod_mu cos p_mu
(because phi(x) = (-1)^(x2 + x4)), and c is the same at both momenta of the
pair {p, p + pi(0,1,0,1)}.  On that pair Gamma_55 = [[0, c], [c, 0]], so A has
the eigenvalues sum sin^2 p + (m + r (1 -+ c))^2, 3 colours each.
"""
from __future__ import annotations

import itertools

import numpy as np


def momenta(dims, bc=(1, 1, 1, 1)):
    """All lattice momenta as an (V, 4) array."""
    axes = []
    for mu in range(4):
        L = dims[mu]
        th = 0.0 if bc[mu] == 1 else np.pi
        axes.append((2.0 * np.pi * np.arange(L) + th) / L)
    grid = np.meshgrid(*axes, indexing="ij")
    return np.stack([g.ravel() for g in grid], axis=1)


def wilson_spectrum(dims, m, r=1.0, bc=(1, 1, 1, 1)):
    """Sorted eigenvalues of A_W (multiplicity 12 per momentum)."""
    p = momenta(dims, bc)
    a = m + r * np.sum(1.0 - np.cos(p), axis=1)
    lam = a ** 2 + np.sum(np.sin(p) ** 2, axis=1)
    return np.sort(np.repeat(lam, 12))


def sw_pair_representatives(dims, bc=(1, 1, 1, 1)):
    """One momentum from every pair {p, p + pi(0,1,0,1)}: those with n_2 < L_2/2."""
    axes = []
    for mu in range(4):
        L = dims[mu]
        th = 0.0 if bc[mu] == 1 else np.pi
        n = np.arange(L // 2) if mu == 1 else np.arange(L)
        axes.append((2.0 * np.pi * n + th) / L)
    grid = np.meshgrid(*axes, indexing="ij")
    return np.stack([g.ravel() for g in grid], axis=1)


def sw_spectrum(dims, m, r=1.0, bc=(1, 1, 1, 1)):
    """Sorted eigenvalues of A_SW (3 colours per value)."""
    p = sw_pair_representatives(dims, bc)
    c = np.prod(np.cos(p), axis=1)
    s2 = np.sum(np.sin(p) ** 2, axis=1)
    lam = np.concatenate([s2 + (m + r * (1.0 - c)) ** 2, s2 + (m + r * (1.0 + c)) ** 2])
    return np.sort(np.repeat(lam, 3))


def sw_normal_on_plane_wave(p, m, r=1.0):
    """Coefficients (a, b) with A_SW exp(ipx) = a exp(ipx) + b exp(i(p+pi(0,1,0,1))x)
    at U = 1: a = sum sin^2 p + (m+r)^2 + r^2 c^2, b = -2 r (m+r) c."""
    p = np.asarray(p, dtype=float)
    c = np.prod(np.cos(p))
    a = np.sum(np.sin(p) ** 2) + (m + r) ** 2 + r ** 2 * c ** 2
    b = -2.0 * r * (m + r) * c
    return a, b


def kappa_ratio_sqrt(dims, m, r=1.0):
    """kappa_W^{1/2} / kappa_SW^{1/2} from the closed-form spectra."""
    w = wilson_spectrum(dims, m, r)
    s = sw_spectrum(dims, m, r)
    return np.sqrt((w[-1] / w[0]) / (s[-1] / s[0]))


def kappa_ratio_sqrt_limit():
    """The paper's m -> 0 limit (Sec. 3): 8 / sqrt(5)."""
    return 8.0 / np.sqrt(5.0)


def extreme_eigenvalues(formulation_is_wilson, m, r=1.0):
    """lambda_min, lambda_max at U = 1 on a periodic lattice with every L % 4 == 0.

    Wilson: m^2 (p = 0) and (m + 8r)^2 (p = (pi,pi,pi,pi)).
    Staggered Wilson: m^2 (p = 0, lower branch) and
    max(4 + (m + r)^2, (m + 2r)^2) (all p_mu = pi/2, or p = 0 upper branch).
    """
    if formulation_is_wilson:
        return m * m, (m + 8.0 * r) ** 2
    return m * m, max(4.0 + (m + r) ** 2, (m + 2.0 * r) ** 2)
