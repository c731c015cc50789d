"""GPU test of fsi_apply_batched_noalloc (the entry point for callers that
cannot allocate device memory at apply time): through the C ABI it must give
the outputs of fsi_apply_batched_nograph on the same plan and input, on two
calls in a row (the second plan smaller, so the static scratch array still
holds the first call's words), for fused plans (register-phase kernel with
one-block, small-d and blocked instances, generic kernel) and a two-pass
plan, and it must refuse a plan whose workspaces exceed the scratch array."""
import ctypes

import numpy as np
import pytest
import torch

import games
from paper_2601_01903_amd import BatchPlan, FsiError, fsi

pytestmark = pytest.mark.gpu


def _values(ds, seed, dtype):
    parts = []
    for i, d in enumerate(ds):
        g = games.tree_game(d, 30, 5, games.rng_for(seed, i))
        parts.append(games.tree_values(g))
    return torch.from_numpy(np.concatenate(parts).astype(dtype)).cuda()


def _check_pair(bp, x, tag):
    ref = bp.apply(x, graph=False)
    out = torch.full_like(ref, float("nan"))
    bp.apply_noalloc(x, out)
    torch.cuda.synchronize()
    assert torch.equal(out, ref), tag
    print(f"{tag}: bitwise equal ({out.numel()} outputs)", flush=True)


def test_noalloc_matches_nograph_two_calls():
    # call 1: a larger ragged FP32 batch (register-phase kernel, d = 9 run as
    # d = 11; generic kernel at l = 5), call 2: a smaller one
    ds1, ls1 = [20, 20, 16, 13, 9, 12], [4, 2, 3, 4, 2, 5]
    bp1 = BatchPlan(ds1, ls1, dtype="f32")
    _check_pair(bp1, _values(ds1, 501, np.float32), "fp32 ragged, call 1")
    ds2, ls2 = [12, 8], [3, 2]
    bp2 = BatchPlan(ds2, ls2, dtype="f32")
    _check_pair(bp2, _values(ds2, 502, np.float32), "fp32 small, call 2")
    # FP64 two-pass plan: its Moebius workspace comes from the scratch too
    ds3, ls3 = [14, 10], [3, 2]
    bp3 = BatchPlan(ds3, ls3, dtype="f64", algo="two_pass")
    _check_pair(bp3, _values(ds3, 503, np.float64), "fp64 two-pass, call 3")
    # a register-phase instance of several blocks (d = 21, l = 4: partial
    # sums per block of 2^6 tiles, then the wide gather's partials)
    ds4, ls4 = [21, 11], [4, 4]
    bp4 = BatchPlan(ds4, ls4, dtype="f32")
    _check_pair(bp4, _values(ds4, 505, np.float32), "fp32 blocked, call 4")
    # and the first plan again after the others
    _check_pair(bp1, _values(ds1, 504, np.float32), "fp32 ragged, call 5")
    for bp in (bp1, bp2, bp3, bp4):
        bp.close()


def test_noalloc_refuses_plans_beyond_scratch():
    # generic kernel at d = 25, l = 4: per-tile results alone exceed 64 MiB
    bp = BatchPlan([25], [4], dtype="f32", kernel="generic")
    x = torch.zeros(bp.value_offset[-1], dtype=torch.float32, device="cuda")
    out = torch.zeros(bp.out_offset[-1], dtype=torch.float32, device="cuda")
    with pytest.raises(FsiError) as ei:
        bp.apply_noalloc(x, out)
    assert ei.value.status == 1
    assert b"scratch" in fsi.load().fsi_last_error()
    bp.close()
