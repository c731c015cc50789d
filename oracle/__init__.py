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
    INDICES,
    bernoulli_exact,
    index_weight_exact,
    index_weight_table_f64,
    interaction,
    interaction_from_mobius,
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

from .forest import forest_value_at, forest_values  # noqa: F401

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
        lib.oracle_superset_sums.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp, ip,
                                             ctypes.c_int64, dp, ctypes.c_int]
        lib.oracle_superset_sums.restype = None
        lib.oracle_mobius.argtypes = [dp, ctypes.c_int]
        lib.oracle_mobius.restype = None
        lib.oracle_ranked_sums_int.argtypes = [ip, ctypes.c_int, ip, ctypes.c_int64,
                                               ip, ip, ctypes.c_int]
        lib.oracle_ranked_sums_int.restype = ctypes.c_int
        _lib = lib
    return _lib


def fsi_c(v, d: int, l: int, nthreads: int = 1, index: str = "fsi") -> np.ndarray:
    """Same result as ``fsi`` (or ``interaction`` for another index; same
    algorithm), computed by the C twin."""
    if not (1 <= l <= d):
        raise ValueError("need 1 <= l <= d")
    lib = _load()
    v = np.ascontiguousarray(np.asarray(v, dtype=np.float64))
    if v.size != 1 << d:
        raise ValueError("v must have 2^d entries")
    W = np.ascontiguousarray(weight_table_f64(d, l) if index == "fsi"
                             else index_weight_table_f64(index, d, l))
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


def interaction_from_mobius_c(a, d: int, l: int, index: str = "fsi", nthreads: int = 1) -> np.ndarray:
    """Same result as ``interaction_from_mobius`` (same algorithm: superset
    sums of the given Moebius coefficients), computed by the C twin."""
    if not (1 <= l <= d):
        raise ValueError("need 1 <= l <= d")
    lib = _load()
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if a.size != 1 << d:
        raise ValueError("a must have 2^d entries")
    W = np.ascontiguousarray(weight_table_f64(d, l) if index == "fsi"
                             else index_weight_table_f64(index, d, l))
    masks = np.ascontiguousarray(output_masks(d, l).astype(np.int64))
    E = np.empty(masks.size, dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int64)
    lib.oracle_superset_sums(a.ctypes.data_as(dp), d, l, W.ctypes.data_as(dp),
                             masks.ctypes.data_as(ip), masks.size, E.ctypes.data_as(dp),
                             int(nthreads))
    return E


def mobius_c(v) -> np.ndarray:
    lib = _load()
    a = np.array(v, dtype=np.float64, copy=True)
    d = a.size.bit_length() - 1
    lib.oracle_mobius(a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), d)
    return a


def fsi_exact_int(v, d: int, l: int, nthreads: int = 1) -> np.ndarray:
    """FSI of an integer-valued v without rounding until the end: the Moebius
    transform and the ranked superset sums A_t(S) are exact int64 (C twin),
    E_S = a(S) + sum_{t > l} w(|S|, t) A_t(S) is summed in exact rationals
    (weights of Eq. 7 as Fractions) and rounded once to FP64."""
    if not (1 <= l <= d):
        raise ValueError("need 1 <= l <= d")
    vi = np.ascontiguousarray(np.asarray(v), dtype=np.int64)
    if vi.size != 1 << d or not np.array_equal(vi, np.asarray(v)):
        raise ValueError("v must hold 2^d integers")
    if np.max(np.abs(vi)) * (1 << d) >= 2 ** 62:
        raise ValueError("values too large for exact int64 accumulation")
    lib = _load()
    masks = np.ascontiguousarray(output_masks(d, l).astype(np.int64))
    A = np.zeros((masks.size, d + 1), dtype=np.int64)
    aS = np.zeros(masks.size, dtype=np.int64)
    ip = ctypes.POINTER(ctypes.c_int64)
    rc = lib.oracle_ranked_sums_int(vi.ctypes.data_as(ip), d, masks.ctypes.data_as(ip),
                                    masks.size, A.ctypes.data_as(ip), aS.ctypes.data_as(ip),
                                    int(nthreads))
    if rc != 0:
        raise MemoryError("oracle_ranked_sums_int: allocation failed")
    from fractions import Fraction
    wq = {(s, t): weight_exact(s, t, l) for s in range(1, l + 1) for t in range(l + 1, d + 1)}
    out = np.empty(masks.size, dtype=np.float64)
    for k, S in enumerate(masks):
        s = bin(int(S)).count("1")
        val = Fraction(int(aS[k]))
        if s >= 1:
            for t in range(l + 1, d + 1):
                if A[k, t]:
                    val += wq[(s, t)] * int(A[k, t])
        out[k] = float(val)
    return out
