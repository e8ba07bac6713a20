"""GPU parity of the shift-invert Arnoldi spectrum against the oracle's dense
eigenvalues (needs an MI355X).

Arnoldi from one start vector resolves each distinct eigenvalue once; the
converged ones (relative Ritz estimate below 1e-8) must be eigenvalues of the
dense matrix, and the one nearest the shift must be among them.
"""
import numpy as np
import pytest

import synth
from oracle import spectrum as SPEC

pytestmark = pytest.mark.gpu

lq = pytest.importorskip("paper_1312_3265_amd")
torch = pytest.importorskip("torch")


def _dist(z, ref):
    return np.abs(np.asarray(ref) - z).min()


@pytest.mark.parametrize("formulation,sigma", [(synth.STAGGERED_WILSON, 0.45),
                                               (synth.STAGGERED_WILSON, 1.55),
                                               (synth.WILSON, 0.45)])
def test_spectrum_matches_dense_4x4(formulation, sigma):
    """A smooth (near-identity) field, shifts beside the low ends of the
    physical (0.45) and doubler (1.55) branches, whose eigenvalues lie at
    similar distances from the shift; 150 Arnoldi steps resolve the nearest."""
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, "near_identity", 2000, 0.436)
    g = lq.Gauge(lq.Lattice(dims), U, lq.FEAT_CORNERS)
    v0 = synth.gaussian_field(dims, formulation, 3)
    ev, res = lq.spectrum(g, formulation, 0.0, sigma, v0, steps=150, tol=1e-12)
    dense = SPEC.dense_eigenvalues(formulation, U)
    conv = ev[res < 1e-8]
    assert len(conv) >= 2
    for z in conv:
        assert _dist(z, dense) <= 1e-7 * max(1.0, abs(z))
    assert _dist(SPEC.nearest(dense, sigma, 1)[0], conv) <= 1e-7
    assert np.all(np.diff(np.abs(ev - sigma)) >= 0)


def test_spectrum_free_field_closed_form():
    dims = (4, 4, 4, 4)
    U = np.zeros(synth.site_shape(dims) + (4, 3, 3), dtype=np.complex128)
    U[...] = np.eye(3)
    g = lq.Gauge(lq.Lattice(dims), U, lq.FEAT_CORNERS)
    v0 = synth.gaussian_field(dims, synth.STAGGERED_WILSON, 4)
    ev, res = lq.spectrum(g, synth.STAGGERED_WILSON, 0.1, 0.3, v0, steps=30, tol=1e-12)
    re, im = SPEC.sw_free_real_imag(dims, m=0.1)
    ref = np.concatenate([re + 1j * im, re - 1j * im])
    conv = ev[res < 1e-9]
    assert len(conv) >= 2
    for z in conv:
        assert _dist(z, ref) <= 1e-9
    assert _dist(SPEC.nearest(np.unique(np.round(ref, 12)), 0.3, 1)[0], conv) <= 1e-9


@pytest.mark.parametrize("formulation,sigma", [(synth.STAGGERED_WILSON, 0.45),
                                               (synth.WILSON, 0.45)])
def test_krylov_schur_restarts_converge_in_a_small_basis(formulation, sigma):
    """30 basis vectors with restarts reach what plain Arnoldi needed 150 for:
    the nearest eigenvalues converged and equal to the dense ones."""
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, "near_identity", 2000, 0.436)
    g = lq.Gauge(lq.Lattice(dims), U, lq.FEAT_CORNERS)
    v0 = synth.gaussian_field(dims, formulation, 3)
    ev, res = lq.spectrum(g, formulation, 0.0, sigma, v0, steps=30, restarts=40, tol=1e-12)
    dense = SPEC.dense_eigenvalues(formulation, U)
    conv = ev[res < 1e-8]
    assert len(conv) >= 4
    for z in conv:
        assert _dist(z, dense) <= 1e-7 * max(1.0, abs(z))
    for z in SPEC.nearest(dense, sigma, 2):
        assert _dist(z, conv) <= 1e-7
