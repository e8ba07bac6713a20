"""Lattice helpers for the oracle: shifts with fermion boundary signs and phases.

Fields live in the canonical layout (numpy axes (x4, x3, x2, x1, ...)), so the
lattice direction mu = 0, 1, 2, 3 (x, y, z, t) is numpy axis 3 - mu.  Gauge links
are periodic; a fermion hop that crosses the boundary in direction mu is
multiplied by bc[mu] = +1 or -1 (periodic by default, antiperiodic optional).
"""
from __future__ import annotations

import numpy as np


def axis(mu):
    return 3 - mu


def dims_of(field):
    """(L1, L2, L3, L4) of a canonical-layout field."""
    return (field.shape[3], field.shape[2], field.shape[1], field.shape[0])


def coords(dims):
    """Integer coordinate arrays (x1, x2, x3, x4), each of site shape."""
    L1, L2, L3, L4 = dims
    x4, x3, x2, x1 = np.meshgrid(np.arange(L4), np.arange(L3), np.arange(L2),
                                 np.arange(L1), indexing="ij")
    return x1, x2, x3, x4


def _expand(a, ndim):
    return a.reshape(a.shape + (1,) * (ndim - a.ndim))


def shift(f, mu, sign, bc=(1, 1, 1, 1)):
    """g(x) = b * f(x + sign * mu-hat), with b = bc[mu] where the hop wraps."""
    ax = axis(mu)
    g = np.roll(f, -sign, axis=ax)
    if bc[mu] != 1:
        L = f.shape[ax]
        idx = [slice(None)] * f.ndim
        idx[ax] = L - 1 if sign > 0 else 0
        g[tuple(idx)] *= bc[mu]
    return g


def eta(dims, mu):
    """Staggered phase eta_mu(x) = (-1)^(x_1 + ... + x_{mu-1}) (mu 0-based)."""
    x = coords(dims)
    s = np.zeros(x[0].shape, dtype=np.int64)
    for nu in range(mu):
        s = s + x[nu]
    return np.where(s % 2 == 0, 1.0, -1.0)


def epsilon(dims):
    """epsilon(x) = (-1)^(x1 + x2 + x3 + x4): the flavoured gamma_5 of Sec. 2."""
    x = coords(dims)
    return np.where((x[0] + x[1] + x[2] + x[3]) % 2 == 0, 1.0, -1.0)


def eta5(dims):
    """eta_5(x) = eta_1 eta_2 eta_3 eta_4 = (-1)^(x1 + x3)."""
    e = np.ones(coords(dims)[0].shape)
    for mu in range(4):
        e = e * eta(dims, mu)
    return e


def site_mul(phase, f):
    """Multiply a fermion field by a real per-site function."""
    return _expand(phase, f.ndim) * f
