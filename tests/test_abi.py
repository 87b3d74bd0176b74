"""Host-only checks of the C ABI: the library loads, exports every entry point that
include/hytm.h declares, carries the paper's default constants, and rejects malformed
input before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2208_14935_amd as hy

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "hytm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hytm_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = hy.load()
    names = declared_functions()
    assert "hytm_run" in names and "hytm_graph_create" in names
    for name in names:
        assert hasattr(lib, name), name
    # the binding wraps exactly the declared entry points
    assert sorted(hy._SIGNATURES) == names


def test_default_params_are_the_papers_constants():
    p = hy.default_params()
    assert p.struct_size == ctypes.sizeof(hy.Params)
    assert (p.line_bytes, p.max_outstanding) == (128, 256)             # m, MR (Eq. 1)
    assert (p.alpha_num, p.alpha_den, p.beta_num, p.beta_den) == (4, 5, 2, 5)
    assert (p.gamma_num, p.gamma_den) == (5, 8)                        # 0.625
    assert p.combine_k == 4 and p.index_bytes == 4
    assert p.partition_edges == 32768 and p.pr_iterations == 20 and p.pr_damping == 0.85
    assert p.mode == hy.MODES["hybrid"]


def create(n, m, off, ob, col, w=None, flags=0):
    lib = hy.load()
    h = ctypes.c_void_p()
    st = lib.hytm_graph_create(n, m, off, ob, col, w, flags, 0, ctypes.byref(h))
    return st, lib.hytm_last_error().decode()


def arr(a, dt):
    a = np.ascontiguousarray(a, dtype=dt)
    return a, ctypes.c_void_p(a.ctypes.data)


def test_malformed_inputs_are_rejected_on_the_host():
    off, po = arr([0, 1, 2], np.uint64)
    col, pc = arr([1, 0], np.uint32)
    assert create(2, 2, None, 8, pc)[0] == hy.E_INVAL
    assert create(2, 2, po, 8, None)[0] == hy.E_INVAL
    assert create(2, 2, po, 3, pc)[0] == hy.E_INVAL
    assert create(0, 0, po, 8, pc)[0] == hy.E_INVAL
    st, msg = create(2, 3, po, 8, pc)
    assert st == hy.E_INVAL and "m =" in msg
    bad, pb = arr([0, 2, 1], np.uint64)
    st, msg = create(2, 1, pb, 8, pc)
    assert st == hy.E_INVAL and "decrease" in msg
    badcol, pbc = arr([1, 5], np.uint32)
    st, msg = create(2, 2, po, 8, pbc)
    assert st == hy.E_INVAL and "col[1]" in msg
    assert create(2**32 - 1, 2, po, 8, pc)[0] == hy.E_RANGE
    assert create(2, 2, po, 8, pc, flags=1 << 7)[0] == hy.E_INVAL
    off32, p32 = arr([0, 1, 2], np.uint32)
    # well-formed input reaches the device step: OK with a GPU, E_DEVICE without one
    st, msg = create(2, 2, p32, 4, pc)
    try:
        import torch
        gpu = torch.cuda.is_available()
    except Exception:
        gpu = False
    if not gpu:
        assert st == hy.E_DEVICE and "device" in msg.lower()


def test_binding_validates_before_calling():
    with pytest.raises(ValueError):
        hy.Graph(np.array([0, 1], np.uint64), np.array([0], np.uint32), weights=np.array([1, 2], np.uint32))
    lib = hy.load()
    assert lib.hytm_graph_destroy(None) == hy.OK
    assert lib.hytm_set_device_budget(None, 0) == hy.E_INVAL
    assert lib.hytm_run(None, 0, 0, None, None, None, None) == hy.E_INVAL
    assert lib.hytm_set_params(None, None) == hy.E_INVAL


def test_library_hub_order_matches_the_oracle():
    """The library's host hub sorting (no device needed) against the oracle's."""
    import gen
    import oracle
    for off, col in (gen.rmat(12, 16, seed=3), gen.er(3000, 20000, seed=4),
                     gen.from_pairs(5, np.array([0, 1, 2], np.uint32), np.array([1, 2, 0], np.uint32))):
        order, k = hy.hub_order(off, col)
        want, wk = oracle.hub_order(off, col)
        assert k == wk
        np.testing.assert_array_equal(order, want)
    with pytest.raises(hy.HytmError):
        hy.hub_order(np.array([0, 1], np.uint64), np.array([5], np.uint32))  # col >= n
