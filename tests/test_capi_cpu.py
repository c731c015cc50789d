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
