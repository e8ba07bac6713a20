"""GPU parity of the even-odd (Schur complement) Wilson path against the oracle
(needs an MI355X).

The oracle's Schur operator is built from its full Wilson matrix by parity
projection (``oracle/evenodd.py``); the library's from half-lattice hop
kernels over checkerboarded links.  Bars as for the full matvecs: FP64
relative error <= 1e-13 (max-norm), FP32 and 16-bit within their roundoff
bounds, and the odd half of the result exactly zero.
"""
import numpy as np
import pytest

import synth
from oracle import evenodd as EO

pytestmark = pytest.mark.gpu

lq = pytest.importorskip("paper_1312_3265_amd")
torch = pytest.importorskip("torch")

FEATURES = lq.FEAT_EO | lq.FEAT_F32 | lq.FEAT_Q16
_GAUGE = {}


def _gauge(dims, kind, seed, bc=(1, 1, 1, 1), eps=None):
    key = (dims, kind, seed, bc, eps)
    if key not in _GAUGE:
        U = synth.gauge_field(dims, kind, seed, eps)
        _GAUGE[key] = (U, lq.Gauge(lq.Lattice(dims, bc), U, FEATURES))
    return _GAUGE[key]


def _relerr(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


CASES = [((4, 4, 4, 4), "haar", (1, 1, 1, 1)),
         ((6, 4, 6, 8), "haar", (1, 1, 1, -1)),          # V/2 = 576: ragged last block
         ((8, 8, 6, 4), "near_identity", (-1, 1, 1, -1))]


@pytest.mark.parametrize("dims,kind,bc", CASES)
@pytest.mark.parametrize("dagger", [False, True])
@pytest.mark.parametrize("links", [0, 18])
def test_fp64_schur_matches_oracle(dims, kind, bc, dagger, links):
    U, g = _gauge(dims, kind, 11, bc, 0.436 if kind != "haar" else None)
    psi = synth.gaussian_field(dims, synth.WILSON, 5)
    m = -0.21
    out = lq.schur_apply(g, m, psi, dagger=dagger, links=links).cpu().numpy()
    ref = EO.schur_apply(U, EO.project(psi, EO.EVEN), m, bc, dagger)
    assert _relerr(out, ref) <= 1e-13
    assert np.abs(EO.project(out, EO.ODD)).max() == 0.0


@pytest.mark.parametrize("precision,links,bound", [(lq.F32, 18, 2e-6), (lq.F32, 12, 4e-6),
                                                  (lq.Q16, 12, 1e-4), (lq.Q16, 18, 1e-4)])
def test_low_precision_schur_within_roundoff(precision, links, bound):
    """Two hop stencils in sequence, the intermediate stored in the working
    precision: the bounds of the single matvec hold with room to spare."""
    dims = (6, 4, 6, 8)
    U, g = _gauge(dims, "near_identity", 21, eps=0.436)
    psi = synth.gaussian_field(dims, synth.WILSON, 7)
    out = lq.schur_apply(g, 0.1, psi, precision=precision, links=links).cpu().numpy()
    ref = EO.schur_apply(U, EO.project(psi, EO.EVEN), 0.1)
    assert _relerr(out, ref) <= bound


def test_schur_needs_the_even_odd_links():
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, "haar", 3)
    g = lq.Gauge(lq.Lattice(dims), U, lq.FEAT_F32)
    with pytest.raises(lq.LQError):
        lq.schur_apply(g, 0.1, synth.gaussian_field(dims, synth.WILSON, 1))
