"""Shared test helpers (error metrics, device access)."""
from __future__ import annotations

import sys

import numpy as np


def normwise(x, ref) -> float:
    """max_S |x_S - ref_S| / max_S |ref_S| (per instance)."""
    ref = np.asarray(ref, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    den = float(np.max(np.abs(ref))) if ref.size else 0.0
    if den == 0.0:
        return float(np.max(np.abs(x))) if x.size else 0.0
    return float(np.max(np.abs(x - ref)) / den)


def elementwise(x, ref, floor_frac=1e-3) -> float:
    """max |x_S - ref_S| / |ref_S| over |ref_S| >= floor_frac * max |ref|."""
    ref = np.asarray(ref, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    keep = np.abs(ref) >= floor_frac * np.max(np.abs(ref))
    return float(np.max(np.abs(x[keep] - ref[keep]) / np.abs(ref[keep])))


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()
