"""CG on the normal equations and Lanczos for the condition number (oracle).

The paper inverts the Dirac matrix on a point source by CG on
    (D + m)^dag (D + m) psi = (D + m)^dag chi        (eq. (2), Sec. 3)
without preconditioning, and counts the iterations needed for a given CG
residual.  It also computes kappa = lambda_max / lambda_min of (D+m)^dag (D+m)
(Sec. 3, after eq. (3)) without naming a method; the reading used here is a
Lanczos run with full reorthogonalisation from a seeded start vector.

Readings of points the paper leaves open:
* "CG residual" is the non-squared ||r_k|| / ||b|| of the normal equations,
  b = M^dag chi; on exit the same quantity is recomputed from b - A x in FP64
  and must also be below tol, otherwise CG restarts from the current x;
* x0 = 0, and the iteration count is the number of A-applications in the loop.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import eigh_tridiagonal

from . import staggered_wilson, wilson

import synth

CONVERGED = 0
NOT_CONVERGED = 1
BREAKDOWN = -4


def _dot(a, b):
    return np.vdot(a.ravel(), b.ravel())


def _norm2(a):
    return float(np.vdot(a.ravel(), a.ravel()).real)


def operator(formulation, U, m, r=1.0, bc=(1, 1, 1, 1), corners=None):
    """(M, M^dag, A) callables for the chosen formulation.

    For staggered Wilson, ``corners`` (from ``staggered_wilson.corners``) selects
    the corner form of Gamma_55; by default the subset recursion is used.
    """
    if formulation == synth.WILSON:
        M = lambda v: wilson.apply(U, v, m, r, bc)
        Md = lambda v: wilson.apply(U, v, m, r, bc, dagger=True)
    elif corners is None:
        M = lambda v: staggered_wilson.apply(U, v, m, r, bc)
        Md = lambda v: staggered_wilson.apply(U, v, m, r, bc, dagger=True)
    else:
        g = lambda v: staggered_wilson.gamma55_corners(corners, v, bc)
        M = lambda v: staggered_wilson.apply(U, v, m, r, bc, g55=g(v))
        Md = lambda v: staggered_wilson.apply(U, v, m, r, bc, dagger=True, g55=g(v))
    A = lambda v: Md(M(v))
    return M, Md, A


def cg(A, b, tol, maxiter, x0=None, max_restarts=20):
    """Hestenes-Stiefel CG on a Hermitian positive definite A.

    Returns (x, info) with info = dict(status, iterations, applications,
    restarts, iterated_residual, true_residual, history) where history holds
    ||r_k|| / ||b|| after every iteration.
    """
    bnorm = np.sqrt(_norm2(b))
    if bnorm == 0.0:
        return np.zeros_like(b), dict(status=CONVERGED, iterations=0, applications=0,
                                      restarts=0, iterated_residual=0.0,
                                      true_residual=0.0, history=[])
    if x0 is None:
        x = np.zeros_like(b)
        r = b.copy()
        apps = 0
    else:
        x = x0.copy()
        r = b - A(x)
        apps = 1
    p = r.copy()
    rho = _norm2(r)
    it = 0
    restarts = 0
    hist = []
    status = NOT_CONVERGED
    while it < maxiter:
        q = A(p)
        apps += 1
        pq = _dot(p, q).real
        if not np.isfinite(pq) or pq <= 0.0:
            status = BREAKDOWN
            break
        alpha = rho / pq
        x = x + alpha * p
        r = r - alpha * q
        rho_new = _norm2(r)
        it += 1
        hist.append(np.sqrt(rho_new) / bnorm)
        if not np.isfinite(rho_new):
            status = BREAKDOWN
            break
        if np.sqrt(rho_new) <= tol * bnorm:
            rt = b - A(x)
            apps += 1
            rt2 = _norm2(rt)
            if np.sqrt(rt2) <= tol * bnorm or restarts >= max_restarts:
                status = CONVERGED if np.sqrt(rt2) <= tol * bnorm else NOT_CONVERGED
                rho = rho_new
                break
            restarts += 1
            r = rt
            p = r.copy()
            rho = rt2
            continue
        p = r + (rho_new / rho) * p
        rho = rho_new
    true_res = np.sqrt(_norm2(b - A(x))) / bnorm
    return x, dict(status=status, iterations=it, applications=apps, restarts=restarts,
                   iterated_residual=np.sqrt(rho) / bnorm, true_residual=true_res,
                   history=hist)


def cgnr(formulation, U, chi, m, tol, maxiter, r=1.0, bc=(1, 1, 1, 1), corners=None):
    """Solve eq. (2): b = M^dag chi, then CG on A = M^dag M."""
    M, Md, A = operator(formulation, U, m, r, bc, corners)
    b = Md(chi)
    x, info = cg(A, b, tol, maxiter)
    info["b_norm"] = np.sqrt(_norm2(b))
    return x, info


def true_residual(formulation, U, chi, x, m, r=1.0, bc=(1, 1, 1, 1), corners=None):
    """(||b - A x|| / ||b||, ||chi - M x|| / ||chi||) in FP64, b = M^dag chi."""
    M, Md, A = operator(formulation, U, m, r, bc, corners)
    b = Md(chi)
    Mx = M(x)
    rn = np.sqrt(_norm2(b - Md(Mx)) / _norm2(b))
    rd = np.sqrt(_norm2(chi - Mx) / _norm2(chi))
    return rn, rd


def lanczos(A, v0, steps, reorth=True):
    """Lanczos on Hermitian A from start vector v0.

    v_1 = v0/||v0||; for j = 1..steps: w = A v_j - beta_{j-1} v_{j-1};
    alpha_j = Re<v_j, w>; w -= alpha_j v_j; (full reorthogonalisation:
    classical Gram-Schmidt against v_1..v_j, applied twice); beta_j = ||w||;
    v_{j+1} = w / beta_j.  Returns (alpha, beta) with len(beta) = len(alpha)-1
    for the tridiagonal T (stops early on an invariant subspace).
    """
    n = v0.size
    shape = v0.shape
    Vb = np.zeros((steps + 1, n), dtype=np.complex128)
    v = v0.ravel() / np.sqrt(_norm2(v0))
    Vb[0] = v
    alpha, beta = [], []
    v_prev = np.zeros(n, dtype=np.complex128)
    b_prev = 0.0
    for j in range(steps):
        w = A(v.reshape(shape)).ravel() - b_prev * v_prev
        a = float(np.vdot(v, w).real)
        w = w - a * v
        if reorth:
            for _ in range(2):
                # h_k = <v_k, w> = conj(v_k . conj(w)), without copying the basis
                h = np.conj(Vb[: j + 1] @ np.conj(w))
                w = w - Vb[: j + 1].T @ h
        alpha.append(a)
        bj = np.sqrt(_norm2(w))
        if j == steps - 1:
            break
        if bj <= 1e-14 * abs(a):
            break
        beta.append(bj)
        v_prev = v
        v = w / bj
        Vb[j + 1] = v
        b_prev = bj
    return np.array(alpha), np.array(beta)


def ritz_values(alpha, beta):
    """Eigenvalues of the Lanczos tridiagonal matrix."""
    if len(alpha) == 1:
        return np.array(alpha)
    return eigh_tridiagonal(alpha, beta, eigvals_only=True)


def condition_number(formulation, U, m, v0, steps=200, r=1.0, bc=(1, 1, 1, 1),
                     corners=None):
    """kappa_est = theta_max / theta_min from a Lanczos run on A = M^dag M."""
    _, _, A = operator(formulation, U, m, r, bc, corners)
    a, b = lanczos(A, v0, steps)
    th = ritz_values(a, b)
    return th[0], th[-1], th[-1] / th[0], (a, b)
