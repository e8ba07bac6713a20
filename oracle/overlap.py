"""Staggered overlap operator with the staggered Wilson kernel (oracle).

Test infrastructure only: the library never calls this module.

The paper (Secs. 1, 2 and 4) presents the 2-flavour staggered Wilson operator as
the kernel of a staggered version of the overlap operator and argues that it
should make overlap fermions cheaper, but it does not write the operator out.
The reading used here is the usual overlap construction with the flavoured
gamma_5 of staggered fermions, epsilon(x) = (-1)^(x1+x2+x3+x4), in the role of
gamma_5 (Sec. 2: with it the staggered Wilson matrix is "gamma_5-hermitian",
epsilon M epsilon = M^dag):

    A     = D_SW - rho         (the staggered Wilson matrix at bare mass -rho)
    H     = epsilon A          (hermitian)
    V     = epsilon sign(H)    = A (A^dag A)^{-1/2}  (the unitary factor of A)
    D_ov  = rho (1 + V),       D_ov(m) = (1 - m / (2 rho)) D_ov + m.

D_ov obeys the Ginsparg-Wilson relation epsilon D + D epsilon = D epsilon D / rho
and its spectrum lies on the circle |lambda - rho| = rho.

Two evaluations:
* dense_overlap: the exact operator from the dense matrix (small lattices);
  sign(H) from the eigen-decomposition of H;
* overlap_apply_poly: the polynomial approximation the GPU path uses,
  V psi ~ A p(A^dag A) psi, with p the Chebyshev interpolant of x^{-1/2} on an
  interval [lo, hi] that contains the spectrum of A^dag A, applied by the
  three-term Chebyshev recurrence (one A^dag A application per degree).
  Its error in V is max over the spectrum of |x^{1/2} p(x) - 1|
  (poly_sign_error bounds it on [lo, hi]).
"""
from __future__ import annotations

import numpy as np

from . import dense, staggered_wilson

import synth


def kernel_apply(U, psi, rho, r=1.0, bc=(1, 1, 1, 1), dagger=False):
    """A psi = (D_SW - rho) psi (or A^dag psi)."""
    return staggered_wilson.apply(U, psi, -rho, r, bc, dagger=dagger)


def dense_overlap(U, rho, m=0.0, r=1.0, bc=(1, 1, 1, 1)):
    """The dense D_ov(m), with sign(epsilon A) from eigh, and the dense A."""
    dims = (U.shape[3], U.shape[2], U.shape[1], U.shape[0])
    shape = synth.field_shape(dims, synth.STAGGERED_WILSON)
    A = dense.dense_matrix(lambda v: kernel_apply(U, v, rho, r, bc), shape)
    eps = np.diag(staggered_wilson.epsilon_mul(np.ones(shape, dtype=np.complex128)).ravel())
    H = eps @ A
    H = 0.5 * (H + H.conj().T)          # hermitian up to rounding
    w, Q = np.linalg.eigh(H)
    S = (Q * np.sign(w)) @ Q.conj().T
    V = eps @ S
    n = A.shape[0]
    D = rho * (np.eye(n) + V)
    return (1.0 - m / (2.0 * rho)) * D + m * np.eye(n), A, eps


def cheb_coeffs_invsqrt(lo, hi, degree):
    """Coefficients c_0..c_degree of the Chebyshev interpolant of x^{-1/2} on
    [lo, hi] at the degree + 1 Chebyshev points of the first kind:
        p(x) = sum_k c_k T_k(t),  t = (2x - (hi + lo)) / (hi - lo)."""
    n = degree + 1
    th = np.pi * (np.arange(n) + 0.5) / n
    x = 0.5 * (hi + lo) + 0.5 * (hi - lo) * np.cos(th)
    f = x ** -0.5
    c = np.array([2.0 / n * np.sum(f * np.cos(k * th)) for k in range(n)])
    c[0] *= 0.5
    return c


def cheb_eval(c, lo, hi, x):
    """p(x) from its Chebyshev coefficients (numpy's Chebyshev series)."""
    t = (2.0 * np.asarray(x) - (hi + lo)) / (hi - lo)
    return np.polynomial.chebyshev.chebval(t, c)


def poly_sign_error(lo, hi, degree, samples=20001):
    """max over [lo, hi] of |x^{1/2} p(x) - 1|: the largest error of the
    approximate V on any singular direction of A with singular value^2 there."""
    c = cheb_coeffs_invsqrt(lo, hi, degree)
    x = np.concatenate([np.linspace(lo, hi, samples), np.geomspace(lo, hi, samples)])
    return float(np.max(np.abs(np.sqrt(x) * cheb_eval(c, lo, hi, x) - 1.0)))


def invsqrt_poly_apply(B, v, lo, hi, c):
    """sum_k c_k T_k(X) v with X = (2 B - (hi + lo)) / (hi - lo), by the
    recurrence T_{k+1}(X) v = 2 X T_k(X) v - T_{k-1}(X) v."""
    a, b = 2.0 / (hi - lo), -(hi + lo) / (hi - lo)
    t_prev = v
    y = c[0] * t_prev
    if len(c) == 1:
        return y
    t = a * B(v) + b * v
    y = y + c[1] * t
    for k in range(2, len(c)):
        t_next = 2.0 * (a * B(t) + b * t) - t_prev
        y = y + c[k] * t_next
        t_prev, t = t, t_next
    return y


def overlap_apply_poly(U, psi, rho, m, lo, hi, degree, r=1.0, bc=(1, 1, 1, 1)):
    """D_ov(m) psi with V psi ~ A p(A^dag A) psi (see the module docstring):
    D_ov(m) psi = (rho - m/2) (psi + A p(A^dag A) psi) + m psi."""
    c = cheb_coeffs_invsqrt(lo, hi, degree)
    A = lambda v: kernel_apply(U, v, rho, r, bc)
    Ad = lambda v: kernel_apply(U, v, rho, r, bc, dagger=True)
    y = invsqrt_poly_apply(lambda v: Ad(A(v)), psi, lo, hi, c)
    return (rho - 0.5 * m) * (psi + A(y)) + m * psi


def free_spectrum(dims, rho, m=0.0, r=1.0, bc=(1, 1, 1, 1)):
    """The eigenvalues of D_ov(m) on the free field (U = 1) as Re + i|Im| (the
    spectrum is closed under conjugation): there A is normal (D_st
    anti-hermitian and Gamma_55 hermitian commute), so V has the eigenvalues
    z / |z| over the eigenvalues z = D_SW eigenvalue - rho of A, taken from
    the closed-form free staggered Wilson spectrum (given as Re, |Im|)."""
    from . import spectrum
    re, im = spectrum.sw_free_real_imag(dims, 0.0, r, bc)
    z = (re - rho) + 1j * im
    d = (1.0 - m / (2.0 * rho)) * rho * (1.0 + z / np.abs(z)) + m
    return d.real + 1j * np.abs(d.imag)
