"""Pion correlator and effective mass from Wilson point-source propagators (oracle).

Test infrastructure only: the library never calls this module.

Fig. 1(a) of the paper (Sec. 3) plots m_pi^2 against the bare mass, measured
from the propagators G(x, 0) = M_W^{-1} chi^(alpha) of the point sources at the
origin (the solutions of eq. (2)).  The paper does not write the correlator
down; the reading here is the usual pseudoscalar one: gamma_5-hermiticity gives
G(0, x) = gamma_5 G(x, 0)^dag gamma_5, so the pion two-point function is

    C(t) = sum_{x vec} tr[G(x, 0)^dag G(x, 0)]
         = sum over x vec, the 12 sources alpha and the 12 sink components of |G|^2,

x = (x vec, t); with periodic time its effective mass is
m_eff(t) = arccosh((C(t-1) + C(t+1)) / (2 C(t))).  The staggered Wilson pion
operator is the one of a cited paper that is not available here, so only the
Wilson correlator is defined.
"""
from __future__ import annotations

import numpy as np

from . import freefield, wilson


def pion_correlator(props):
    """C(t) of propagators props[alpha] in the canonical layout, (L4,)."""
    p = np.asarray(props)
    return np.sum(p.real ** 2 + p.imag ** 2, axis=tuple(i for i in range(p.ndim) if i != 1))


def effective_mass(C):
    """arccosh((C(t-1) + C(t+1)) / (2 C(t))), periodic in t; NaN where the
    argument is below 1 (no real solution)."""
    C = np.asarray(C, dtype=float)
    L = len(C)
    out = np.full(L, np.nan)
    for t in range(L):
        q = (C[(t - 1) % L] + C[(t + 1) % L]) / (2.0 * C[t])
        if q >= 1.0:
            out[t] = np.arccosh(q)
    return out


def free_pion_correlator(dims, m, bc=(1, 1, 1, 1)):
    """C(t) at U = 1 from momentum space, independently of the position-space
    operator: M_W e^{ip.x} u = e^{ip.x} M_W(p) u gives the point-source
    propagator G(x) = (1/V) sum_p e^{ip.x} M_W(p)^{-1} (times the colour
    identity), and Parseval over the spatial momenta turns sum_{x vec} |G|^2
    into (1/V_s) sum_{p vec} ||(1/L4) sum_{p4} e^{i p4 t} M_W(p)^{-1}||_F^2;
    the 3 colours of the identity give the factor 3."""
    L1, L2, L3, L4 = dims
    Vs = L1 * L2 * L3
    mom = freefield.momenta(dims, bc).reshape(L1, L2, L3, L4, 4)
    C = np.zeros(L4)
    for i1 in range(L1):
        for i2 in range(L2):
            for i3 in range(L3):
                inv = [np.linalg.inv(wilson.momentum_matrix(mom[i1, i2, i3, i4], m))
                       for i4 in range(L4)]
                p4 = mom[i1, i2, i3, :, 3]
                for t in range(L4):
                    g = sum(np.exp(1j * p4[i4] * t) * inv[i4] for i4 in range(L4)) / L4
                    C[t] += np.sum(np.abs(g) ** 2)
    return 3.0 * C / Vs
