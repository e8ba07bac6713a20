"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This module draws random numbers and lays them out in the canonical host layout;
it holds none of the Dirac-operator, solver or eigenvalue arithmetic.  Both the
oracle and the GPU path consume what it returns, and neither imports the other.

Canonical host layout (all arrays C-contiguous numpy):

* lattice dims are given as ``(L1, L2, L3, L4) = (x, y, z, t)``; the site index is
  ``i = x1 + L1*(x2 + L2*(x3 + L3*x4))``, i.e. numpy shape ``(L4, L3, L2, L1, ...)``;
* gauge field ``U``: ``(L4, L3, L2, L1, 4, 3, 3)`` complex128, ``U[..., mu, a, b]``
  is the colour matrix of the link from x to x + mu-hat, mu = 0..3 for x, y, z, t;
* Wilson fermion field: ``(L4, L3, L2, L1, 4, 3)`` complex128 (spin, colour);
* staggered Wilson fermion field: ``(L4, L3, L2, L1, 3)`` complex128 (colour).

The paper's workload is 200 quenched beta=6 configurations on 16^3 x 32 (Sec. 3);
those are not available, so near-identity SU(3) fields with a comparable mean
plaquette stand in for them, and Haar-random fields serve the small checks.
"""
from __future__ import annotations

import numpy as np

WILSON = 0
STAGGERED_WILSON = 1

NSPIN = {WILSON: 4, STAGGERED_WILSON: 1}


def site_shape(dims):
    """numpy shape of the site axes for dims = (L1, L2, L3, L4)."""
    L1, L2, L3, L4 = (int(d) for d in dims)
    return (L4, L3, L2, L1)


def volume(dims):
    return int(np.prod([int(d) for d in dims]))


def field_shape(dims, formulation):
    """Shape of a fermion field in the canonical layout."""
    if formulation == WILSON:
        return site_shape(dims) + (4, 3)
    if formulation == STAGGERED_WILSON:
        return site_shape(dims) + (3,)
    raise ValueError(f"unknown formulation {formulation}")


def _rng(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def complex_normal(rng, shape):
    """Complex Gaussian with E|z|^2 = 1 (real and imaginary parts N(0, 1/2))."""
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * np.sqrt(0.5)


def haar_su3(n, rng):
    """n Haar-distributed SU(3) matrices.

    QR of a complex Ginibre matrix with the diagonal-phase fix gives Haar U(3)
    (Mezzadri, Notices AMS 54 (2007) 592); dividing by a cube root of the
    determinant maps Haar U(3) onto Haar SU(3), since the map commutes with left
    multiplication by SU(3).
    """
    z = complex_normal(rng, (n, 3, 3))
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    q = q * np.exp(-1j * np.angle(det) / 3.0)[:, None, None]
    return q


def near_identity_su3(n, eps, rng):
    """n matrices U = exp(i eps H), H traceless Hermitian, H = (A + A^dag)/2 - tr/3.

    A has i.i.d. complex normal entries with E|A_ij|^2 = 1.  The exponential is
    taken through the eigendecomposition of H, so U is unitary with det U = 1 to
    rounding.
    """
    a = complex_normal(rng, (n, 3, 3))
    h = 0.5 * (a + np.conj(np.swapaxes(a, -1, -2)))
    tr = np.trace(h, axis1=-2, axis2=-1).real / 3.0
    h = h - tr[:, None, None] * np.eye(3)[None]
    w, v = np.linalg.eigh(h)
    ph = np.exp(1j * eps * w)
    return np.einsum("nab,nb,ncb->nac", v, ph, np.conj(v))


def gauge_field(dims, kind="haar", seed=0, eps=None):
    """Seeded gauge field in the canonical layout.

    kind: ``"unit"`` (free field U = 1), ``"haar"`` (independent Haar links) or
    ``"near_identity"`` (independent exp(i eps H) links; ``eps`` required).
    """
    shp = site_shape(dims) + (4, 3, 3)
    n = volume(dims) * 4
    if kind == "unit":
        u = np.zeros(shp, dtype=np.complex128)
        u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1.0
        return u
    rng = _rng(seed)
    if kind == "haar":
        u = haar_su3(n, rng)
    elif kind == "near_identity":
        if eps is None:
            raise ValueError("near_identity needs eps")
        u = near_identity_su3(n, float(eps), rng)
    else:
        raise ValueError(f"unknown gauge kind {kind!r}")
    return np.ascontiguousarray(u.reshape(shp))


def gauge_transform(dims, seed):
    """Seeded site field of Haar SU(3) matrices g(x), shape (L4, L3, L2, L1, 3, 3)."""
    rng = _rng(seed)
    g = haar_su3(volume(dims), rng)
    return np.ascontiguousarray(g.reshape(site_shape(dims) + (3, 3)))


def point_source(dims, formulation, alpha, site=(0, 0, 0, 0)):
    """Point source at ``site`` = (x1, x2, x3, x4) with component alpha.

    Wilson: alpha = 3*spin + colour (12 sources); staggered Wilson: alpha =
    colour (3 sources), as in the source averaging of Sec. 3.
    """
    f = np.zeros(field_shape(dims, formulation), dtype=np.complex128)
    x1, x2, x3, x4 = site
    if formulation == WILSON:
        if not 0 <= alpha < 12:
            raise ValueError("Wilson point-source index must be in [0, 12)")
        f[x4, x3, x2, x1, alpha // 3, alpha % 3] = 1.0
    else:
        if not 0 <= alpha < 3:
            raise ValueError("staggered Wilson point-source index must be in [0, 3)")
        f[x4, x3, x2, x1, alpha] = 1.0
    return f


def z2_source(dims, formulation, seed):
    """Real Z2 noise: every complex component independently +1 or -1."""
    rng = _rng(seed)
    shp = field_shape(dims, formulation)
    return (2.0 * rng.integers(0, 2, size=shp) - 1.0).astype(np.complex128)


def gaussian_field(dims, formulation, seed):
    """Complex Gaussian fermion field with E|z|^2 = 1 per component."""
    rng = _rng(seed)
    return complex_normal(rng, field_shape(dims, formulation))


def plane_wave(dims, p, amplitude):
    """exp(i p.x) times a constant per-site amplitude (spin/colour tensor).

    ``p`` = (p1, p2, p3, p4) in radians; ``amplitude`` is broadcast over sites.
    """
    L1, L2, L3, L4 = dims
    x4, x3, x2, x1 = np.meshgrid(np.arange(L4), np.arange(L3), np.arange(L2),
                                 np.arange(L1), indexing="ij")
    ph = np.exp(1j * (p[0] * x1 + p[1] * x2 + p[2] * x3 + p[3] * x4))
    amp = np.asarray(amplitude, dtype=np.complex128)
    return ph.reshape(ph.shape + (1,) * amp.ndim) * amp


def poisson_arrivals(rate, n, seed):
    """n arrival times (seconds) of a Poisson process with the given rate."""
    rng = _rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def serving_requests(n, seed, dims_choices, deltas=(0.02, 0.05, 0.1),
                     tol_range=(1e-10, 1e-6)):
    """Seeded request descriptors for the solve server.

    Each request draws dims uniformly from ``dims_choices``, the formulation
    uniformly, delta uniformly from ``deltas``, a point or Z2 source, and a
    tolerance log-uniform in ``tol_range``.  Only the descriptors are drawn
    here; source arrays are built from them with :func:`point_source` or
    :func:`z2_source` and the recorded source seed.
    """
    rng = _rng(seed)
    out = []
    lo, hi = np.log10(tol_range[0]), np.log10(tol_range[1])
    for k in range(n):
        dims = tuple(dims_choices[int(rng.integers(0, len(dims_choices)))])
        form = int(rng.integers(0, 2))
        delta = float(deltas[int(rng.integers(0, len(deltas)))])
        kind = "point" if rng.integers(0, 2) == 0 else "z2"
        nalpha = 12 if form == WILSON else 3
        alpha = int(rng.integers(0, nalpha))
        tol = float(10.0 ** rng.uniform(lo, hi))
        out.append(dict(id=k, dims=dims, formulation=form, delta=delta, source=kind,
                        alpha=alpha, source_seed=int(rng.integers(0, 2**31)), tol=tol))
    return out
