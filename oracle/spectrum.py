"""Eigenvalues of the Dirac matrices nearest a shift (oracle).

Test infrastructure only: the library never calls this module.

Fig. 1(c) of the paper (Sec. 3) shows the low-lying spectrum of the staggered
Wilson operator D_SW (the matrix of eq. (2) at m = 0) on one background and
reads off the separation between its physical and doubler branches.  The paper
does not say how the eigenvalues were computed; they are fixed by the matrix,
so the oracle takes all of them from the dense matrix (small lattices only)
and orders them by distance from a shift sigma.
"""
from __future__ import annotations

import numpy as np

from . import dense, freefield, staggered_wilson, wilson

import synth


def dense_eigenvalues(formulation, U, m=0.0, r=1.0, bc=(1, 1, 1, 1)):
    """All eigenvalues of M (eq. (2)'s matrix at mass m) from its dense form."""
    dims = (U.shape[3], U.shape[2], U.shape[1], U.shape[0])
    mod = wilson if formulation == synth.WILSON else staggered_wilson
    M = dense.dense_matrix(lambda v: mod.apply(U, v, m, r, bc),
                           synth.field_shape(dims, formulation))
    return np.linalg.eigvals(M)


def nearest(eigs, sigma, k):
    """The k eigenvalues closest to sigma, closest first."""
    eigs = np.asarray(eigs)
    return eigs[np.argsort(np.abs(eigs - sigma), kind="stable")[:k]]


def sw_free_real_imag(dims, m=0.0, r=1.0, bc=(1, 1, 1, 1)):
    """(Re, |Im|) of the free (U = 1) staggered Wilson eigenvalues: D_st and
    Gamma_55 commute there, Gamma_55 = +-c(p) on the momentum pair of p and
    D_st = +-i (sum sin^2 p)^{1/2}, so lambda = m + r (1 -+ c) +- i s, 3 colours."""
    p = freefield.sw_pair_representatives(dims, bc)
    c = np.prod(np.cos(p), axis=1)
    s = np.sqrt(np.sum(np.sin(p) ** 2, axis=1))
    re = np.concatenate([m + r * (1.0 - c), m + r * (1.0 + c)])
    im = np.concatenate([s, s])
    return np.repeat(re, 3), np.repeat(im, 3)
