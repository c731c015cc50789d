"""CPU-side checks of the C ABI library: it loads, exports every function that
include/fsi.h declares, and its host-only entry points behave as documented.
No compute call is made here."""
import ctypes
import os
import re

import pytest

from paper_2601_01903_amd import fsi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"\b(fsi_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = fsi.load()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(fsi.EXPORTS) == names


def test_num_outputs_host_only():
    for d, l, M in [(8, 2, 37), (14, 3, 470), (20, 2, 211), (20, 4, 6196), (30, 30, 1 << 30)]:
        assert fsi.num_outputs(d, l) == M
    for d, l in [(0, 1), (5, 0), (5, 6), (31, 2), (-1, -1)]:
        assert fsi.num_outputs(d, l) == -1


def test_default_opts_and_last_error():
    lib = fsi.load()
    o = fsi.Opts()
    assert lib.fsi_default_opts(ctypes.byref(o)) == 0
    assert (o.dtype, o.precision, o.algo, o.tile_bits) == (0, 5, 0, 0)
    assert lib.fsi_default_opts(None) == 1
    assert b"NULL" in lib.fsi_last_error()


def test_invalid_arguments_rejected_before_device_use():
    lib = fsi.load()
    h = ctypes.c_void_p()
    for d, l in [(0, 1), (4, 0), (4, 5), (31, 3)]:
        assert lib.fsi_plan(d, l, ctypes.byref(h)) == 1
        assert h.value is None
    assert lib.fsi_plan(4, 2, None) == 1
    darr = (ctypes.c_int * 2)(4, 3)
    larr = (ctypes.c_int * 2)(2, 4)
    assert lib.fsi_plan_batched(2, darr, larr, None, ctypes.byref(h)) == 1
    assert lib.fsi_plan_batched(0, darr, larr, None, ctypes.byref(h)) == 1
    assert lib.fsi_apply(None, None, None, None) == 1
    o = fsi.make_opts(algo="two_pass")
    o.allow_input_overwrite = 2
    assert lib.fsi_plan_ex(10, 2, ctypes.byref(o), ctypes.byref(h)) == 1
    assert b"allow_input_overwrite" in lib.fsi_last_error()
    assert lib.fsi_plan_destroy(None) == 0
    assert lib.fsi_batch_plan_destroy(None) == 0


def test_plan_without_gfx950_is_unsupported():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = fsi.load()
    h = ctypes.c_void_p()
    assert lib.fsi_plan(8, 2, ctypes.byref(h)) == 2
    assert lib.fsi_last_error()


def _forest_call(d, roots, feature, threshold, left, right, value, max_bg=1):
    import numpy as np
    lib = fsi.load()
    P = ctypes.POINTER
    arrs = [np.ascontiguousarray(a, dtype=t) for a, t in (
        (roots, np.int32), (feature, np.int32), (threshold, np.float64),
        (left, np.int32), (right, np.int32), (value, np.float64))]
    r, f, th, lf, rt, val = arrs
    h = ctypes.c_void_p()
    st = lib.fsi_forest_create(d, r.size, r.ctypes.data_as(P(ctypes.c_int32)), f.size,
                               f.ctypes.data_as(P(ctypes.c_int32)),
                               th.ctypes.data_as(P(ctypes.c_double)),
                               lf.ctypes.data_as(P(ctypes.c_int32)),
                               rt.ctypes.data_as(P(ctypes.c_int32)),
                               val.ctypes.data_as(P(ctypes.c_double)), max_bg, ctypes.byref(h))
    return st, h


def test_forest_validation_before_device_use():
    """Malformed forests are rejected on the host (they could otherwise send
    a walk out of bounds or around a cycle)."""
    ok = dict(roots=[0], feature=[0, -1, -1], threshold=[0.5, 0, 0], left=[1, 0, 0],
              right=[2, 0, 0], value=[0, 1, 2])
    bad = [
        dict(ok, d=0), dict(ok, d=31),
        dict(ok, roots=[3]),                                   # root out of range
        dict(ok, left=[7, 0, 0]),                              # child out of range
        dict(ok, right=[-1, 0, 0]),
        dict(ok, feature=[4, -1, -1]),                         # feature >= d
        dict(ok, threshold=[float("nan"), 0, 0]),
        dict(ok, feature=[0, 1, -1], left=[1, 0, 0], right=[2, 1, 0]),   # 1 -> 1 cycle
        dict(ok, max_bg=0), dict(ok, max_bg=5000),
    ]
    # a chain of 65 splits is deeper than the walk allows
    n = 66
    chain = dict(roots=[0], feature=[0] * 65 + [-1], threshold=[0.5] * 65 + [0],
                 left=list(range(1, 66)) + [0], right=list(range(1, 66)) + [0],
                 value=[0.0] * n)
    bad.append(chain)
    for case in bad:
        kw = dict(ok)
        kw.update(case)
        d = kw.pop("d", 4)
        max_bg = kw.pop("max_bg", 1)
        st, h = _forest_call(d, max_bg=max_bg, **kw)
        assert st == 1, case
        assert h.value is None
    lib = fsi.load()
    assert lib.fsi_forest_destroy(None) == 0
    assert lib.fsi_forest_values(None, None, 1, None, 0, None, None) == 1


def test_host_allocation_failure_returns_status(monkeypatch):
    """A std::bad_alloc while a plan is built comes back as
    FSI_ERR_OUT_OF_MEMORY with a message, through every plan entry point; no
    exception crosses the ABI (the process would abort)."""
    lib = fsi.load()
    monkeypatch.setenv("FSI_TEST_FAIL_ALLOC", "host")
    h = ctypes.c_void_p()
    assert lib.fsi_plan(12, 3, ctypes.byref(h)) == 3
    assert h.value is None
    assert b"host allocation failed" in lib.fsi_last_error()
    darr = (ctypes.c_int * 3)(20, 12, 9)
    larr = (ctypes.c_int * 3)(4, 3, 2)
    assert lib.fsi_plan_batched(3, darr, larr, None, ctypes.byref(h)) == 3
    assert h.value is None
    o = fsi.Opts()
    lib.fsi_default_opts(ctypes.byref(o))
    o.dtype, o.autotune = 1, 1
    assert lib.fsi_plan_ex(20, 4, ctypes.byref(o), ctypes.byref(h)) == 3
    assert h.value is None
    # argument errors still win over the hook
    assert lib.fsi_plan(4, 0, ctypes.byref(h)) == 1
    monkeypatch.delenv("FSI_TEST_FAIL_ALLOC")
    # without the hook this host has no gfx950 device
    if not fsi.torch.cuda.is_available():
        assert lib.fsi_plan(12, 3, ctypes.byref(h)) == 2


def test_block_threads_is_reserved():
    lib = fsi.load()
    o = fsi.Opts()
    lib.fsi_default_opts(ctypes.byref(o))
    h = ctypes.c_void_p()
    for bt in (256, 512, -1):
        o.block_threads = bt
        assert lib.fsi_plan_ex(12, 3, ctypes.byref(o), ctypes.byref(h)) == 1
        assert b"block_threads" in lib.fsi_last_error()
