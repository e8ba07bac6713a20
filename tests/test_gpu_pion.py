"""GPU parity of the Wilson pion correlator against the oracle (needs an MI355X).

The library reduces point-source propagators on the device in FP64 (fixed
order); the oracle sums the same propagators with numpy.  Propagators come
from the library's own solver; the free-field case is also held to the
oracle's momentum-space closed form.
"""
import numpy as np
import pytest

import synth
from oracle import spectroscopy as SP

pytestmark = pytest.mark.gpu

lq = pytest.importorskip("paper_1312_3265_amd")
torch = pytest.importorskip("torch")


def _props(g, dims, m, tol, opts=None, bc=None):
    chis = np.stack([synth.point_source(dims, synth.WILSON, a) for a in range(12)])
    x, infos = lq.cg_solve_batch(g, synth.WILSON, [m] * 12, chis, [tol] * 12, opts=opts)
    assert all(i["status"] == lq.OK for i in infos)
    return x


def _check_meff(meff, ref):
    assert np.array_equal(np.isnan(meff), np.isnan(ref))
    ok = ~np.isnan(ref)
    assert np.abs(meff[ok] - ref[ok]).max() <= 1e-10


@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (6, 4, 6, 8)])
def test_pion_correlator_matches_oracle(dims):
    """(6, 4, 6, 8): 144 sites per time slice, so most of the 256 blocks of a
    slice get a short or empty stretch."""
    U = synth.gauge_field(dims, "near_identity", 2000, 0.4359375)
    lat = lq.Lattice(dims)
    g = lq.Gauge(lat, U, lq.FEAT_F32 | lq.FEAT_Q16)
    x = _props(g, dims, -0.25, 1e-8, lq.solve_opts(precision=lq.Q16))
    C, meff = lq.pion_correlator(lat, x)
    ref = SP.pion_correlator(x.cpu().numpy())
    assert np.abs(C - ref).max() / ref.max() <= 1e-13
    _check_meff(meff, SP.effective_mass(ref))


def test_pion_correlator_free_field_closed_form():
    dims = (4, 4, 4, 8)
    bc = (1, 1, 1, -1)
    U = np.zeros(synth.site_shape(dims) + (4, 3, 3), dtype=np.complex128)
    U[...] = np.eye(3)
    lat = lq.Lattice(dims, bc)
    g = lq.Gauge(lat, U, 0)
    x = _props(g, dims, 0.2, 1e-12)
    C, _ = lq.pion_correlator(lat, x)
    ref = SP.free_pion_correlator(dims, 0.2, bc)
    assert np.abs(C - ref).max() / ref.max() <= 1e-9


def test_pion_correlator_full_size_16x32():
    """The 12 propagators of one mass of the 16^3 x 32 workload (16-bit batched
    solve): the device reduction against numpy on the same fields."""
    dims = (16, 16, 16, 32)
    U = synth.gauge_field(dims, "near_identity", 2000, 0.4359375)
    lat = lq.Lattice(dims)
    g = lq.Gauge(lat, U, lq.FEAT_F32 | lq.FEAT_Q16)
    x = _props(g, dims, -0.4721359549995794 + 0.1, 1e-8, lq.solve_opts(precision=lq.Q16))
    C, meff = lq.pion_correlator(lat, x)
    ref = SP.pion_correlator(x.cpu().numpy())
    assert np.abs(C - ref).max() / ref.max() <= 1e-13
    _check_meff(meff, SP.effective_mass(ref))
    assert np.all(C > 0)
