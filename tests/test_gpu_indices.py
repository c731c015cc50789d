"""GPU parity of the other interaction indices (SII, k-SII, STII, BII;
Appendix A) through the C ABI against the CPU oracle. The kernels are the
FSI kernels with the index's weight table; the tolerances are those of the
FSI tests (FP64 1e-12 normwise, FP32 storage 1e-6 on tree and planted games
against the oracle on the same FP32 values widened to FP64)."""
import numpy as np
import pytest

import games
import oracle
from helpers import normwise, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
OTHER = ["stii", "sii", "ksii", "bii"]


def fsi_mod():
    from paper_2601_01903_amd import fsi
    return fsi


def gpu_apply(v, d, l, **kw):
    fsi = fsi_mod()
    tdt = torch.float64 if kw.get("dtype", "f64") == "f64" else torch.float32
    plan = fsi.Plan(d, l, **kw)
    out = plan.apply(torch.as_tensor(np.asarray(v), dtype=tdt).to(DEV))
    torch.cuda.synchronize()
    res = out.double().cpu().numpy()
    plan.close()
    return res


@pytest.mark.parametrize("index", OTHER)
@pytest.mark.parametrize("algo", ["fused", "two_pass"])
def test_index_small_fp64(index, algo):
    say(f"[case] index={index} d=8 l=2 and d=9 l=3 FP64 algo={algo}")
    _, v = games.small_planted(0)
    assert normwise(gpu_apply(v, 8, 2, algo=algo, index=index),
                    oracle.interaction(v, 8, 2, index)) < 1e-12
    vn = games.normal_values(9, games.rng_for(501, 0))
    assert normwise(gpu_apply(vn, 9, 3, algo=algo, index=index),
                    oracle.interaction(vn, 9, 3, index)) < 1e-12


@pytest.mark.parametrize("index", OTHER)
@pytest.mark.parametrize("kernel", ["generic", "register"])
@pytest.mark.parametrize("d,l", [(11, 4), (14, 3), (20, 2), (20, 4)])
def test_index_fp64_kernels(index, kernel, d, l):
    say(f"[case] index={index} d={d} l={l} FP64 kernel={kernel}")
    g = games.tree_game(d, 60, 5, games.rng_for(502, d * 10 + l))
    v = games.tree_values(g)
    got = gpu_apply(v, d, l, kernel=kernel, index=index)
    err = normwise(got, oracle.fsi_c(v, d, l, nthreads=8, index=index))
    say(f"  err {err:.3e}")
    assert err < 1e-12


@pytest.mark.parametrize("index", OTHER)
@pytest.mark.parametrize("prec", ["f32_compensated", "f32", "f32_fp64reg"])
def test_index_d20_fp32(index, prec):
    say(f"[case] index={index} d=20 l=4 FP32 storage prec={prec}")
    for name, v in (("tree", games.d20_tree(0)[1]),
                    ("planted", games.d20_batch_instance(1)[1])):
        v32 = v.astype(np.float32)
        ref = oracle.fsi_c(v32.astype(np.float64), 20, 4, nthreads=8, index=index)
        got = gpu_apply(v32, 20, 4, dtype="f32", precision=prec, index=index)
        err = normwise(got, ref)
        say(f"  {name} err {err:.3e}")
        assert err < 1e-6, name


@pytest.mark.parametrize("index", ["stii", "ksii", "fsi"])
def test_efficiency_at_full_size(index):
    """STII, k-SII and FSI are efficient: the outputs (empty set included)
    sum to v(full set), at d = 20 on both kernels."""
    say(f"[case] efficiency index={index} d=20 l=4")
    _, v = games.d20_tree(0)
    for kernel in ("register", "generic"):
        out = gpu_apply(v, 20, 4, kernel=kernel, index=index)
        assert abs(out.sum() - v[-1]) < 1e-9 * max(1.0, np.abs(out).max()), kernel


@pytest.mark.parametrize("index", OTHER)
def test_index_batched_ragged_fp32(index):
    fsi = fsi_mod()
    rng = np.random.default_rng(503)
    ds = [int(x) for x in rng.integers(8, 21, size=20)]
    ls = [int(rng.integers(1, 5)) for _ in ds]
    say(f"[case] index={index} batched ragged FP32 n={len(ds)}")
    vals = [games.tree_values(games.tree_game(d, 40, 5, games.rng_for(504, i))).astype(np.float32)
            for i, d in enumerate(ds)]
    bp = fsi.BatchPlan(ds, ls, dtype="f32", index=index)
    out = bp.apply(torch.from_numpy(np.concatenate(vals)).to(DEV), graph=True)
    torch.cuda.synchronize()
    o = out.double().cpu().numpy()
    for i, (v, d, l) in enumerate(zip(vals, ds, ls)):
        ref = oracle.fsi_c(v.astype(np.float64), d, l, nthreads=8, index=index)
        assert normwise(o[bp.out_offset[i]:bp.out_offset[i + 1]], ref) < 1e-6, (i, d, l)
    bp.close()


def test_unknown_index_rejected():
    fsi = fsi_mod()
    o = fsi.make_opts()
    o.index = 9
    import ctypes
    h = ctypes.c_void_p()
    st = fsi.load().fsi_plan_ex(8, 2, ctypes.byref(o), ctypes.byref(h))
    assert st == 1  # FSI_ERR_INVALID_ARG
    assert h.value is None


@pytest.mark.parametrize("index", ["ksii", "sii"])
def test_index_blocked_register_kernel(index):
    """d = 22, l = 4 runs the register-phase kernel in blocks of 2^6 tiles."""
    fsi = fsi_mod()
    d, l = 22, 4
    say(f"[case] index={index} d={d} l={l} FP32, blocks")
    g = games.tree_game(d, 60, 5, games.rng_for(505, 0))
    v32 = games.tree_values(g).astype(np.float32)
    plan = fsi.Plan(d, l, dtype="f32", index=index)
    assert plan.schedule()["fast_instances"] == 1
    out = plan.apply(torch.from_numpy(v32).to(DEV))
    torch.cuda.synchronize()
    got = out.double().cpu().numpy()
    plan.close()
    ref = oracle.fsi_c(v32.astype(np.float64), d, l, nthreads=16, index=index)
    assert normwise(got, ref) < 1e-6
