"""Host-side checks of the C-ABI library (no GPU calls)."""
import ctypes
import os

import pytest

import paper_1312_3265_amd as lq


def test_header_declares_the_boundary():
    names = lq.header_symbols()
    for n in ("lq_lattice_create", "lq_gauge_create", "lq_apply", "lq_cg_solve",
              "lq_cg_solve_batch", "lq_condition_number", "lq_batch_step", "lq_last_error"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(lq.LIB_PATH), reason="liblq.so not built")
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(lq.LIB_PATH)
    missing = [n for n in lq.header_symbols() if not hasattr(L, n)]
    assert not missing, missing
    lq.lib()  # signatures bind


@pytest.mark.skipif(not os.path.exists(lq.LIB_PATH), reason="liblq.so not built")
def test_lattice_validation_without_gpu():
    """Lattice creation is host-only: bad extents and boundary signs are rejected."""
    L = lq.lib()
    h = ctypes.c_void_p()
    bad = (ctypes.c_int32 * 4)(4, 5, 4, 4)
    assert L.lq_lattice_create(bad, None, ctypes.byref(h)) == lq.ERR_ARG
    assert b"even" in L.lq_last_error()
    good = (ctypes.c_int32 * 4)(4, 6, 8, 4)
    badbc = (ctypes.c_int32 * 4)(1, 1, 2, 1)
    assert L.lq_lattice_create(good, badbc, ctypes.byref(h)) == lq.ERR_ARG
    huge = (ctypes.c_int32 * 4)(1024, 1024, 16, 16)       # 2^28 sites: above the limit
    assert L.lq_lattice_create(huge, None, ctypes.byref(h)) == lq.ERR_ARG
    assert b"2^28" in L.lq_last_error()
    small = (ctypes.c_int32 * 4)(4, 2, 4, 4)              # extents below 4
    assert L.lq_lattice_create(small, None, ctypes.byref(h)) == lq.ERR_ARG
    assert L.lq_lattice_create(good, None, ctypes.byref(h)) == lq.OK
    assert L.lq_lattice_volume(h) == 4 * 6 * 8 * 4
    # gauge storage query: 36 FP64 planes of padded length plus scratch
    nb = L.lq_gauge_bytes(h, 0)
    Vp = ((768 + 63) // 64) * 64 + 64
    assert nb >= 36 * Vp * 16
    L.lq_lattice_destroy(h)
