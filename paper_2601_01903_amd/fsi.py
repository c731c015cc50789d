"""Python binding of the FSI C ABI (include/fsi.h): argument marshalling only.

Every step of the operator runs in the HIP library ``_lib/libfsi_mi355x.so``;
PyTorch is used for device memory and streams. There is no CPU fallback: if
the library is missing or the device is not gfx950, calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libfsi_mi355x.so")

FSI_OK = 0
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "UNSUPPORTED", 3: "OUT_OF_MEMORY",
                4: "HIP_ERROR", 5: "INTERNAL"}
DTYPES = {"f64": 0, "f32": 1}
PRECISIONS = {"f64": 0, "f32": 1, "f32_compensated": 2, "f32_fp64mob": 3,
              "f32_fp64reg": 4, "auto": 5}
ALGOS = {"auto": 0, "fused": 1, "two_pass": 2}
KERNELS = {"auto": 0, "generic": 1, "register": 2}
INDICES = {"fsi": 0, "stii": 1, "sii": 2, "ksii": 3, "bii": 4}
INPUTS = {"values": 0, "mobius": 1}

# names of every function include/fsi.h declares
EXPORTS = ["fsi_default_opts", "fsi_num_outputs", "fsi_plan", "fsi_plan_ex",
           "fsi_plan_destroy", "fsi_output_masks", "fsi_plan_info", "fsi_apply",
           "fsi_mobius", "fsi_plan_batched", "fsi_batch_plan_destroy",
           "fsi_batch_offsets", "fsi_apply_batched", "fsi_apply_batched_nograph",
           "fsi_apply_batched_noalloc",
           "fsi_batch_num_stages", "fsi_apply_batched_stage", "fsi_plan_schedule",
           "fsi_batch_schedule", "fsi_last_error",
           "fsi_forest_create", "fsi_forest_destroy", "fsi_forest_values",
           "fsi_forest_mobius", "fsi_forest_values_mobius"]


class FsiError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("algo", ctypes.c_int32), ("tile_bits", ctypes.c_int32),
                ("block_threads", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("kernel", ctypes.c_int32), ("index", ctypes.c_int32),
                ("input", ctypes.c_int32), ("allow_input_overwrite", ctypes.c_int32)]


class Schedule(ctypes.Structure):
    _fields_ = [("autotuned", ctypes.c_int32), ("fast_instances", ctypes.c_int32),
                ("tiles_per_item", ctypes.c_int32), ("tile_shift", ctypes.c_int32),
                ("mob_group", ctypes.c_int32), ("tuned_ms", ctypes.c_float)]


def _sched_dict(s: Schedule) -> dict:
    return {k: getattr(s, k) for k, _ in Schedule._fields_}


_lib = None


def load() -> ctypes.CDLL:
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FileNotFoundError(
            f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
            "(hipcc --offload-arch=gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    P = ctypes.POINTER
    lib.fsi_default_opts.argtypes = [P(Opts)]
    lib.fsi_num_outputs.argtypes = [i32, i32]
    lib.fsi_num_outputs.restype = i64
    lib.fsi_plan.argtypes = [i32, i32, P(vp)]
    lib.fsi_plan_ex.argtypes = [i32, i32, P(Opts), P(vp)]
    lib.fsi_plan_destroy.argtypes = [vp]
    lib.fsi_output_masks.argtypes = [vp, P(ctypes.c_uint32)]
    lib.fsi_plan_info.argtypes = [vp, P(i32), P(i32), P(i32), P(i32)]
    lib.fsi_apply.argtypes = [vp, vp, vp, vp]
    lib.fsi_mobius.argtypes = [vp, vp, vp]
    lib.fsi_plan_batched.argtypes = [i32, P(i32), P(i32), P(Opts), P(vp)]
    lib.fsi_batch_plan_destroy.argtypes = [vp]
    lib.fsi_batch_offsets.argtypes = [vp, P(i64), P(i64)]
    lib.fsi_apply_batched.argtypes = [vp, vp, vp, vp]
    lib.fsi_apply_batched_nograph.argtypes = [vp, vp, vp, vp]
    lib.fsi_apply_batched_noalloc.argtypes = [vp, vp, vp, vp]
    lib.fsi_batch_num_stages.argtypes = [vp]
    lib.fsi_apply_batched_stage.argtypes = [vp, vp, vp, i32, vp]
    lib.fsi_plan_schedule.argtypes = [vp, P(Schedule)]
    lib.fsi_batch_schedule.argtypes = [vp, P(Schedule)]
    lib.fsi_forest_create.argtypes = [i32, i32, P(ctypes.c_int32), i32, P(ctypes.c_int32),
                                      P(ctypes.c_double), P(ctypes.c_int32), P(ctypes.c_int32),
                                      P(ctypes.c_double), i32, P(vp)]
    lib.fsi_forest_destroy.argtypes = [vp]
    lib.fsi_forest_values.argtypes = [vp, vp, i32, vp, i32, vp, vp]
    lib.fsi_forest_mobius.argtypes = [vp, vp, i32, vp, vp, vp]
    lib.fsi_forest_values_mobius.argtypes = [vp, vp, i32, vp, vp, i32, vp, vp]
    lib.fsi_last_error.argtypes = []
    lib.fsi_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        fn = getattr(lib, name)
        if name not in ("fsi_num_outputs", "fsi_last_error", "fsi_batch_num_stages"):
            fn.restype = i32
    _lib = lib
    return lib


def _check(status: int, where: str):
    if status != FSI_OK:
        msg = load().fsi_last_error().decode(errors="replace")
        raise FsiError(status, where, msg)


def num_outputs(d: int, l: int) -> int:
    return int(load().fsi_num_outputs(d, l))


def make_opts(dtype="f64", precision="auto", algo="auto", tile_bits=0,
              block_threads=0, kernel="auto", autotune=False, index="fsi",
              input="values", allow_input_overwrite=False) -> Opts:
    o = Opts()
    _check(load().fsi_default_opts(ctypes.byref(o)), "fsi_default_opts")
    o.dtype = DTYPES[dtype]
    o.precision = PRECISIONS[precision]
    o.algo = ALGOS[algo]
    o.tile_bits = int(tile_bits)
    o.block_threads = int(block_threads)
    o.kernel = KERNELS[kernel]
    o.autotune = 1 if autotune else 0
    o.index = INDICES[index]
    o.input = INPUTS[input]
    o.allow_input_overwrite = 1 if allow_input_overwrite else 0
    return o


def _stream_handle(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


_TORCH_DTYPE = {"f64": torch.float64, "f32": torch.float32}


def _check_tensor(t: torch.Tensor, n: int, dtype, what: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{what} must be a HIP device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{what} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{what} must be contiguous with {n} elements")


class Plan:
    """fsi_plan_ex / fsi_apply for one (d, l)."""

    def __init__(self, d: int, l: int, dtype: str = "f64", precision: str = "auto",
                 algo: str = "auto", tile_bits: int = 0, block_threads: int = 0,
                 kernel: str = "auto", autotune: bool = False, index: str = "fsi",
                 input: str = "values", allow_input_overwrite: bool = False):
        lib = load()
        self.d, self.l, self.dtype, self.index = d, l, dtype, index
        self._h = ctypes.c_void_p()
        opts = make_opts(dtype, precision, algo, tile_bits, block_threads, kernel, autotune,
                         index, input, allow_input_overwrite)
        _check(lib.fsi_plan_ex(d, l, ctypes.byref(opts), ctypes.byref(self._h)), "fsi_plan_ex")
        self.M = num_outputs(d, l)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().fsi_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        tb, bt, al, pr = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(load().fsi_plan_info(self._h, ctypes.byref(tb), ctypes.byref(bt),
                                    ctypes.byref(al), ctypes.byref(pr)), "fsi_plan_info")
        return {"tile_bits": tb.value, "block_threads": bt.value, "algo": al.value,
                "precision": pr.value}

    def schedule(self) -> dict:
        sc = Schedule()
        _check(load().fsi_plan_schedule(self._h, ctypes.byref(sc)), "fsi_plan_schedule")
        return _sched_dict(sc)

    def output_masks(self):
        import numpy as np
        m = np.zeros(self.M, dtype=np.uint32)
        _check(load().fsi_output_masks(self._h, m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))),
               "fsi_output_masks")
        return m

    def apply(self, v: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None):
        dt = _TORCH_DTYPE[self.dtype]
        _check_tensor(v, 1 << self.d, dt, "v")
        if out is None:
            out = torch.empty(self.M, dtype=dt, device=v.device)
        _check_tensor(out, self.M, dt, "out")
        _check(load().fsi_apply(self._h, ctypes.c_void_p(v.data_ptr()),
                                ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)),
               "fsi_apply")
        return out

    def mobius(self, a: torch.Tensor, stream=None) -> torch.Tensor:
        """In-place Moebius transform of a (2^d elements, storage dtype)."""
        _check_tensor(a, 1 << self.d, _TORCH_DTYPE[self.dtype], "a")
        _check(load().fsi_mobius(self._h, ctypes.c_void_p(a.data_ptr()), _stream_handle(stream)),
               "fsi_mobius")
        return a


class BatchPlan:
    """fsi_plan_batched / fsi_apply_batched for instances of uneven (d_i, l_i)."""

    def __init__(self, ds: Sequence[int], ls: Sequence[int], dtype: str = "f32",
                 precision: str = "auto", algo: str = "auto", tile_bits: int = 0,
                 block_threads: int = 0, kernel: str = "auto", autotune: bool = False,
                 index: str = "fsi", input: str = "values",
                 allow_input_overwrite: bool = False):
        lib = load()
        n = len(ds)
        if len(ls) != n:
            raise ValueError("ds and ls differ in length")
        self.n, self.dtype = n, dtype
        self.ds, self.ls = list(ds), list(ls)
        darr = (ctypes.c_int * n)(*ds)
        larr = (ctypes.c_int * n)(*ls)
        opts = make_opts(dtype, precision, algo, tile_bits, block_threads, kernel, autotune,
                         index, input, allow_input_overwrite)
        self._h = ctypes.c_void_p()
        _check(lib.fsi_plan_batched(n, darr, larr, ctypes.byref(opts), ctypes.byref(self._h)),
               "fsi_plan_batched")
        vo = (ctypes.c_int64 * (n + 1))()
        oo = (ctypes.c_int64 * (n + 1))()
        _check(lib.fsi_batch_offsets(self._h, vo, oo), "fsi_batch_offsets")
        self.value_offset = list(vo)
        self.out_offset = list(oo)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().fsi_batch_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def apply(self, values: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None,
              graph: bool = True) -> torch.Tensor:
        dt = _TORCH_DTYPE[self.dtype]
        _check_tensor(values, self.value_offset[-1], dt, "values")
        if out is None:
            out = torch.empty(self.out_offset[-1], dtype=dt, device=values.device)
        _check_tensor(out, self.out_offset[-1], dt, "out")
        fn = load().fsi_apply_batched if graph else load().fsi_apply_batched_nograph
        _check(fn(self._h, ctypes.c_void_p(values.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                  _stream_handle(stream)), "fsi_apply_batched")
        return out

    def apply_noalloc(self, values: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
        """fsi_apply_batched_noalloc: the workspaces come from the library's
        static per-GPU scratch array; the caller passes both buffers."""
        dt = _TORCH_DTYPE[self.dtype]
        _check_tensor(values, self.value_offset[-1], dt, "values")
        _check_tensor(out, self.out_offset[-1], dt, "out")
        _check(load().fsi_apply_batched_noalloc(self._h, ctypes.c_void_p(values.data_ptr()),
                                                ctypes.c_void_p(out.data_ptr()),
                                                _stream_handle(stream)),
               "fsi_apply_batched_noalloc")
        return out

    def schedule(self) -> dict:
        sc = Schedule()
        _check(load().fsi_batch_schedule(self._h, ctypes.byref(sc)), "fsi_batch_schedule")
        return _sched_dict(sc)

    def num_stages(self) -> int:
        return int(load().fsi_batch_num_stages(self._h))

    def apply_stage(self, values: torch.Tensor, out: torch.Tensor, stage: int, stream=None):
        """Launch one kernel of the apply sequence (for per-kernel timing)."""
        dt = _TORCH_DTYPE[self.dtype]
        _check_tensor(values, self.value_offset[-1], dt, "values")
        _check_tensor(out, self.out_offset[-1], dt, "out")
        _check(load().fsi_apply_batched_stage(self._h, ctypes.c_void_p(values.data_ptr()),
                                              ctypes.c_void_p(out.data_ptr()), int(stage),
                                              _stream_handle(stream)), "fsi_apply_batched_stage")


class Forest:
    """fsi_forest_create / fsi_forest_values: the interventional value function
    of a tree ensemble over all 2^d coalitions (include/fsi_forest.h).

    Node arrays (host, any integer/float dtype convertible): feature (< 0 marks
    a leaf), threshold, left, right, value; roots holds each tree's root."""

    def __init__(self, d: int, roots, feature, threshold, left, right, value, max_bg: int = 1):
        import numpy as np
        lib = load()
        self.d, self.max_bg = d, max_bg
        self._arrs = [np.ascontiguousarray(a, dtype=t) for a, t in (
            (roots, np.int32), (feature, np.int32), (threshold, np.float64),
            (left, np.int32), (right, np.int32), (value, np.float64))]
        r, f, th, lf, rt, val = self._arrs
        n_nodes = f.size
        if not (th.size == lf.size == rt.size == val.size == n_nodes):
            raise ValueError("node arrays differ in length")
        P = ctypes.POINTER
        self._h = ctypes.c_void_p()
        _check(lib.fsi_forest_create(
            d, r.size, r.ctypes.data_as(P(ctypes.c_int32)), n_nodes,
            f.ctypes.data_as(P(ctypes.c_int32)), th.ctypes.data_as(P(ctypes.c_double)),
            lf.ctypes.data_as(P(ctypes.c_int32)), rt.ctypes.data_as(P(ctypes.c_int32)),
            val.ctypes.data_as(P(ctypes.c_double)), max_bg, ctypes.byref(self._h)),
            "fsi_forest_create")

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().fsi_forest_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check_points(self, x, bg):
        _check_tensor(x, self.d, torch.float64, "x")
        if bg.dim() != 2 or bg.shape[1] != self.d:
            raise ValueError("bg must have shape (n_bg, d)")
        _check_tensor(bg, bg.numel(), torch.float64, "bg")

    def values(self, x: torch.Tensor, bg: torch.Tensor, dtype: str = "f64",
               out: Optional[torch.Tensor] = None, stream=None, method: str = "walk",
               work: Optional[torch.Tensor] = None) -> torch.Tensor:
        """v over all 2^d coalitions for the explained point x (d FP64 values)
        and background rows bg (n_bg x d FP64), both device tensors.
        method "walk": every tree walked per coalition (fsi_forest_values);
        "mobius": path-product Moebius coefficients, then subset sums
        (fsi_forest_values_mobius; work is a 2^d FP64 scratch tensor)."""
        self._check_points(x, bg)
        dt = _TORCH_DTYPE[dtype]
        if out is None:
            out = torch.empty(1 << self.d, dtype=dt, device=x.device)
        _check_tensor(out, 1 << self.d, dt, "out")
        lib = load()
        xp, bp = ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(bg.data_ptr())
        if method == "walk":
            _check(lib.fsi_forest_values(self._h, xp, int(bg.shape[0]), bp, DTYPES[dtype],
                                         ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)),
                   "fsi_forest_values")
        elif method == "mobius":
            if work is None:
                work = out if dtype == "f64" else torch.empty(1 << self.d, dtype=torch.float64,
                                                              device=x.device)
            _check_tensor(work, 1 << self.d, torch.float64, "work")
            _check(lib.fsi_forest_values_mobius(self._h, xp, int(bg.shape[0]), bp,
                                                ctypes.c_void_p(work.data_ptr()), DTYPES[dtype],
                                                ctypes.c_void_p(out.data_ptr()),
                                                _stream_handle(stream)),
                   "fsi_forest_values_mobius")
        else:
            raise ValueError("method must be 'walk' or 'mobius'")
        return out

    def mobius(self, x: torch.Tensor, bg: torch.Tensor, out: Optional[torch.Tensor] = None,
               stream=None) -> torch.Tensor:
        """The Moebius transform of v (2^d FP64) from leaf path products."""
        self._check_points(x, bg)
        if out is None:
            out = torch.empty(1 << self.d, dtype=torch.float64, device=x.device)
        _check_tensor(out, 1 << self.d, torch.float64, "out")
        _check(load().fsi_forest_mobius(self._h, ctypes.c_void_p(x.data_ptr()), int(bg.shape[0]),
                                        ctypes.c_void_p(bg.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)),
               "fsi_forest_mobius")
        return out
