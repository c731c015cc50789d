"""FSI oracle package (test infrastructure only; see fsi_oracle.py).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may import
this package. The product library never does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .fsi_oracle import (  # noqa: F401
    fsi,
    fsi_batch,
    mobius,
    mobius_direct,
    num_outputs,
    output_masks,
    superset_masks,
    weight_exact,
    weight_table_f64,
)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fsi_oracle_c.c")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None


def build_c(force: bool = True) -> str:
    """Compile the C twin with gcc into oracle/_build/liboracle.so."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_c(force=False)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_fsi.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp, ip,
                                   ctypes.c_int64, dp, ctypes.c_int]
        lib.oracle_fsi.restype = ctypes.c_int
        lib.oracle_mobius.argtypes = [dp, ctypes.c_int]
        lib.oracle_mobius.restype = None
        _lib = lib
    return _lib


def fsi_c(v, d: int, l: int, nthreads: int = 1) -> np.ndarray:
    """Same result as ``fsi`` (same algorithm), computed by the C twin."""
    if not (1 <= l <= d):
        raise ValueError("need 1 <= l <= d")
    lib = _load()
    v = np.ascontiguousarray(np.asarray(v, dtype=np.float64))
    if v.size != 1 << d:
        raise ValueError("v must have 2^d entries")
    W = np.ascontiguousarray(weight_table_f64(d, l))
    masks = np.ascontiguousarray(output_masks(d, l).astype(np.int64))
    E = np.empty(masks.size, dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int64)
    rc = lib.oracle_fsi(v.ctypes.data_as(dp), d, l, W.ctypes.data_as(dp),
                        masks.ctypes.data_as(ip), masks.size,
                        E.ctypes.data_as(dp), int(nthreads))
    if rc != 0:
        raise MemoryError("oracle_fsi: allocation failed")
    return E


def mobius_c(v) -> np.ndarray:
    lib = _load()
    a = np.array(v, dtype=np.float64, copy=True)
    d = a.size.bit_length() - 1
    lib.oracle_mobius(a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), d)
    return a
