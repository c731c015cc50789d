"""GPU parity of plans whose input is already the Moebius transform a
(fsi_plan_opts.input = FSI_INPUT_MOBIUS) against the oracle's scores from
given Moebius coefficients, on both tile kernels, FP64 and FP32 storage, the
other indices, the batched form, and the tree-ensemble chain (Moebius
coefficients scattered on the GPU, then the correction)."""
import ctypes

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


def run(a, d, l, **kw):
    fsi = fsi_mod()
    tdt = torch.float64 if kw.get("dtype", "f64") == "f64" else torch.float32
    plan = fsi.Plan(d, l, input="mobius", **kw)
    sched = plan.schedule()
    out = plan.apply(torch.as_tensor(np.asarray(a), dtype=tdt).to(DEV))
    torch.cuda.synchronize()
    res = out.double().cpu().numpy()
    plan.close()
    return res, sched


@pytest.mark.parametrize("kernel", ["register", "generic"])
@pytest.mark.parametrize("d,l", [(12, 2), (16, 3), (20, 4)])
def test_mobius_input_fp64(kernel, d, l):
    say(f"[case] Moebius input d={d} l={l} FP64 kernel={kernel}")
    g = games.tree_game(d, 60, 5, games.rng_for(940, d))
    a = oracle.mobius(games.tree_values(g))
    got, sched = run(a, d, l, kernel=kernel)
    assert sched["fast_instances"] == (1 if kernel == "register" else 0)
    assert normwise(got, oracle.interaction_from_mobius_c(a, d, l, nthreads=16)) < 1e-12


@pytest.mark.parametrize("prec", ["f32_fp64mob", "f32_compensated", "f32"])
def test_mobius_input_fp32_and_blocks(prec):
    for d, l in ((20, 4), (22, 4)):
        say(f"[case] Moebius input d={d} l={l} FP32 {prec}")
        g = games.tree_game(d, 60, 5, games.rng_for(941, d))
        a32 = oracle.mobius(games.tree_values(g)).astype(np.float32)
        got, sched = run(a32, d, l, dtype="f32", precision=prec)
        assert sched["fast_instances"] == 1
        ref = oracle.interaction_from_mobius_c(a32.astype(np.float64), d, l, nthreads=16)
        assert normwise(got, ref) < 1e-6


@pytest.mark.parametrize("index", ["ksii", "bii"])
def test_mobius_input_indices(index):
    d, l = 14, 3
    say(f"[case] Moebius input index={index} d={d} l={l}")
    a = np.random.default_rng(942).standard_normal(1 << d)
    got, _ = run(a, d, l, index=index)
    assert normwise(got, oracle.interaction_from_mobius_c(a, d, l, index, nthreads=16)) < 1e-12


def test_mobius_input_batched():
    fsi = fsi_mod()
    ds, ls = [9, 13, 20, 11], [2, 3, 4, 1]
    say("[case] Moebius input batched")
    vals = [np.random.default_rng(943 + i).standard_normal(1 << d) for i, d in enumerate(ds)]
    bp = fsi.BatchPlan(ds, ls, dtype="f64", input="mobius")
    out = bp.apply(torch.from_numpy(np.concatenate(vals)).to(DEV), graph=True)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    for i, (a, d, l) in enumerate(zip(vals, ds, ls)):
        ref = oracle.interaction_from_mobius_c(a, d, l, nthreads=16)
        assert normwise(o[bp.out_offset[i]:bp.out_offset[i + 1]], ref) < 1e-12, (i, d, l)
    bp.close()


def test_forest_mobius_then_fsi():
    """Tree ensemble -> Moebius coefficients (GPU scatter) -> FSI from them:
    equal to the oracle's FSI of the oracle's value function."""
    fsi = fsi_mod()
    d, l = 14, 3
    g = games.tree_game(d, 50, 4, games.rng_for(944, 0))
    from test_gpu_forest import heap_forest
    forest = heap_forest(g)
    bgs = np.random.default_rng(944).uniform(size=(3, d))
    say("[case] forest -> Moebius -> FSI (Moebius input) d=14 l=3")
    F = fsi.Forest(d, *forest, max_bg=3)
    a = F.mobius(torch.as_tensor(g.x).to(DEV), torch.as_tensor(bgs).to(DEV))
    plan = fsi.Plan(d, l, input="mobius")
    E = plan.apply(a)
    torch.cuda.synchronize()
    ref = oracle.fsi(oracle.forest_values(d, *forest, g.x, bgs), d, l)
    assert normwise(E.cpu().numpy(), ref) < 1e-12
    F.close()
    plan.close()


def test_mobius_input_rejects_two_pass():
    fsi = fsi_mod()
    o = fsi.make_opts(algo="two_pass", input="mobius")
    h = ctypes.c_void_p()
    assert fsi.load().fsi_plan_ex(10, 2, ctypes.byref(o), ctypes.byref(h)) == 1
    assert h.value is None
    o = fsi.make_opts()
    o.input = 5
    assert fsi.load().fsi_plan_ex(10, 2, ctypes.byref(o), ctypes.byref(h)) == 1
