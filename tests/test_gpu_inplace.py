"""GPU parity of two-pass plans that run their Moebius butterfly in place on
the input buffer (fsi_plan_opts.allow_input_overwrite = 1): the scores
against the oracle, the input buffer afterwards against the oracle's Moebius
transform (Sec. 2.2), and the cases that must leave the input untouched (a
butterfly wider than the storage type; the fused algorithm)."""
import numpy as np
import pytest

import games
import oracle
from helpers import normwise, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def fsi_mod():
    from paper_2601_01903_amd import fsi
    return fsi


def apply_on(v, d, l, dtype, **kw):
    """One apply on a fresh device copy of v; returns (scores, input buffer after)."""
    fsi = fsi_mod()
    tdt = torch.float64 if dtype == "f64" else torch.float32
    plan = fsi.Plan(d, l, dtype=dtype, allow_input_overwrite=True, **kw)
    x = torch.as_tensor(np.asarray(v), dtype=tdt).to(DEV)
    out = plan.apply(x)
    torch.cuda.synchronize()
    res = out.double().cpu().numpy(), x.double().cpu().numpy()
    plan.close()
    return res


@pytest.mark.parametrize("d,l", [(9, 2), (14, 3), (20, 4)])
def test_two_pass_fp64_in_place(d, l):
    say(f"[case] in-place two-pass FP64 d={d} l={l}")
    v = games.tree_values(games.tree_game(d, 60, 5, games.rng_for(950, d)))
    got, after = apply_on(v, d, l, "f64", algo="two_pass")
    assert normwise(got, oracle.fsi_c(v, d, l, nthreads=16)) < 1e-12
    assert normwise(after, oracle.mobius(v)) < 1e-12


def test_two_pass_fp32_in_place():
    d, l = 16, 3
    say(f"[case] in-place two-pass FP32 (FP32 butterfly) d={d} l={l}")
    v32 = games.tree_values(games.tree_game(d, 60, 5, games.rng_for(951, d))).astype(np.float32)
    v = v32.astype(np.float64)
    got, after = apply_on(v32, d, l, "f32", algo="two_pass", precision="f32")
    assert normwise(got, oracle.fsi_c(v, d, l, nthreads=16)) < 1e-6
    assert normwise(after, oracle.mobius(v)) < 1e-5


@pytest.mark.parametrize("algo,prec", [("two_pass", "f32_compensated"),
                                       ("two_pass", "f32_fp64mob"),
                                       ("fused", "f32"), ("fused", "auto")])
def test_input_kept_where_not_in_place(algo, prec):
    d, l = 14, 3
    say(f"[case] overwrite allowed but not used: algo={algo} prec={prec}")
    v32 = games.tree_values(games.tree_game(d, 60, 5, games.rng_for(952, d))).astype(np.float32)
    got, after = apply_on(v32, d, l, "f32", algo=algo, precision=prec)
    assert np.array_equal(after.astype(np.float32), v32)
    assert normwise(got, oracle.fsi_c(v32.astype(np.float64), d, l, nthreads=16)) < 1e-6


def test_batched_two_pass_in_place():
    fsi = fsi_mod()
    ds, ls = [9, 13, 16, 11], [2, 3, 4, 1]
    say("[case] in-place two-pass batched FP64 (graph replay)")
    vals = [np.random.default_rng(953 + i).standard_normal(1 << d) for i, d in enumerate(ds)]
    bp = fsi.BatchPlan(ds, ls, dtype="f64", algo="two_pass", allow_input_overwrite=True)
    x = torch.from_numpy(np.concatenate(vals)).to(DEV)
    out = bp.apply(x, graph=True)
    torch.cuda.synchronize()
    o, a = out.cpu().numpy(), x.cpu().numpy()
    for i, (v, d, l) in enumerate(zip(vals, ds, ls)):
        assert normwise(o[bp.out_offset[i]:bp.out_offset[i + 1]],
                        oracle.fsi_c(v, d, l, nthreads=16)) < 1e-12, (i, d, l)
        vo = bp.value_offset[i]
        assert normwise(a[vo:vo + (1 << d)], oracle.mobius(v)) < 1e-12, (i, d, l)
    bp.close()
