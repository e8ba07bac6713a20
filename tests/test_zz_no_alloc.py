"""The allocation-free apply (lq_apply_noalloc): the same results as lq_apply,
from the library's fixed per-GPU scratch, on two calls in a row (the second
smaller, so stale contents of the first would show), with no device memory
allocated by the calls; a lattice above the scratch limit is refused."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

lq = pytest.importorskip("paper_1312_3265_amd")
torch = pytest.importorskip("torch")


def _case(dims, kind, seed, formulation, g55, op, precision):
    U = synth.gauge_field(dims, kind, seed, 0.436 if kind == "near_identity" else None)
    g = lq.Gauge(lq.Lattice(dims), U)
    dt = torch.complex128 if precision == lq.F64 else torch.complex64
    psi = torch.from_numpy(synth.gaussian_field(dims, formulation, seed + 1)).to("cuda", dt)
    return g, psi


def test_noalloc_apply_equals_apply_twice():
    """The first call on a device looks up the scratch's device address (the
    runtime backs the array then); the two calls after it are compared with
    lq_apply and must leave the device's free memory unchanged."""
    g, psi = _case((4, 4, 4, 4), "haar", 3, synth.WILSON, lq.G55_CORNERS, lq.OP_M, lq.F64)
    out = torch.empty_like(psi)
    lq.apply_noalloc(g, synth.WILSON, -0.3, psi, out)
    assert torch.equal(out, lq.apply(g, synth.WILSON, -0.3, psi))
    calls = [
        # the workload's size, FP64 Wilson M^dag M: the largest use of the scratch
        ((16, 16, 16, 32), "near_identity", 2000, synth.WILSON, lq.G55_CORNERS, lq.OP_MDAGM, lq.F64),
        # then a smaller ragged lattice, staggered Wilson on the fly, FP32 M^dag
        ((6, 4, 6, 8), "haar", 7, synth.STAGGERED_WILSON, lq.G55_ONTHEFLY, lq.OP_MDAG, lq.F32),
    ]
    for dims, kind, seed, form, g55, op, prec in calls:
        g, psi = _case(dims, kind, seed, form, g55, op, prec)
        ref = lq.apply(g, form, -0.3, psi, op=op, g55=g55, precision=prec)
        out = torch.empty_like(psi)
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info()
        lq.apply_noalloc(g, form, -0.3, psi, out, op=op, g55=g55, precision=prec)
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        assert free1 == free0, (free0, free1)
        assert torch.equal(out, ref), (dims, form, op)
        assert torch.isfinite(torch.view_as_real(out)).all()


def test_noalloc_apply_refuses_above_its_limit():
    dims = (24, 24, 24, 48)    # FP64 Wilson needs about 380 MB of scratch
    U = synth.gauge_field(dims, "unit", 0)
    g = lq.Gauge(lq.Lattice(dims), U, 0)
    psi = torch.zeros(synth.field_shape(dims, synth.WILSON), dtype=torch.complex128,
                      device="cuda")
    out = torch.empty_like(psi)
    assert lq.lib().lq_apply_noalloc_max_bytes() == 80 << 20
    with pytest.raises(lq.LQError) as e:
        lq.apply_noalloc(g, synth.WILSON, 0.1, psi, out, op=lq.OP_M)
    assert e.value.code == lq.ERR_WORKSPACE
