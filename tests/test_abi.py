"""The C ABI library loads on a machine without a GPU, exports every entry
point include/agp.h declares, and its host-only logic behaves as documented
(argument checks run before any device work; weight sequences of Table 1)."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

from paper_2106_03058_amd import agp, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"\b(agp_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(agp.LIB_PATH):
        import __graft_entry__

        __graft_entry__.build()
    return agp.lib()


def test_exports_every_declared_symbol(lib):
    declared = _declared()
    assert "agp_propagate" in declared and "agp_graph_create" in declared
    for name in declared:
        assert hasattr(lib, name), f"{name} declared in include/ but not exported"
    assert set(agp.EXPORTED) <= set(declared)


def test_weight_sequences_match_table1(lib):
    assert np.allclose(agp.weights_ppr(0.2, 20), inputs.weights_ppr(0.2, 20), rtol=1e-15, atol=0)
    assert np.allclose(agp.weights_hkpr(5.0, 10), inputs.weights_hkpr(5.0, 10), rtol=1e-15, atol=0)
    assert np.allclose(agp.weights_katz(0.01, 30), inputs.weights_katz(0.01, 30), rtol=1e-15, atol=0)
    assert np.array_equal(agp.weights_tp(10), inputs.weights_tp(10))
    with pytest.raises(agp.AGPError) as e:
        agp.weights_ppr(0.0, 5)
    assert e.value.code == agp.AGP_EINVAL
    with pytest.raises(agp.AGPError):
        agp.weights_tp(300)


def test_argument_checks_before_device_work(lib):
    w = np.ones(4)
    vp = ct.c_void_p
    # NULL graph
    rc = lib.agp_propagate(None, 0.0, 1.0, w.ctypes.data_as(ct.POINTER(ct.c_double)), 3, vp(8), 1, 0.1,
                           1, None, vp(8), None, None)
    assert rc == agp.AGP_EINVAL
    assert b"graph" in lib.agp_last_error()
    # graph_create rejects bad sizes and NULL out without touching the device
    h = vp()
    rp = np.array([0, 1], dtype=np.int64)
    assert lib.agp_graph_create(-1, 0, rp.ctypes.data, None, agp.AGP_HOST_PTRS, None, ct.byref(h)) == agp.AGP_EINVAL
    assert lib.agp_graph_create(1, 1, rp.ctypes.data, None, agp.AGP_HOST_PTRS, None, None) == agp.AGP_EINVAL
    bad = np.array([0, 2], dtype=np.int64)  # row_ptr[n] != nnz
    col = np.array([0], dtype=np.int32)
    assert lib.agp_graph_create(1, 1, bad.ctypes.data, col.ctypes.data, agp.AGP_HOST_PTRS, None,
                                ct.byref(h)) == agp.AGP_EINVAL
    assert lib.agp_graph_create(1, 1, rp.ctypes.data, col.ctypes.data, 1 << 7, None,
                                ct.byref(h)) == agp.AGP_EINVAL
    assert lib.agp_graph_destroy(None) == agp.AGP_OK
