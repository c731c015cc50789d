"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Tolerances: 1e-12 normwise for the FP64 path (the oracle's own FP64
summation differs from the GPU's order by far less). FP32-storage modes are
checked against the oracle evaluated on the same FP32 values widened to FP64,
so only computation error is measured; tree and planted games must be within
1e-6 normwise.
"""
import numpy as np
import pytest

import games
import oracle
from helpers import normwise, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"

# Tolerance for cancellation-heavy integer inputs (random small integers,
# +/-1) against the exact-integer oracle. Both FP64 paths hold 1e-12: the
# fused one weights in-tile Moebius values (|a| <= 2^11), the two-pass one
# (full-range Moebius values, |a(T)| up to 2^|T|, before the cross-tile sum)
# keeps its per-tile results as double-doubles from a compensated dot product
# and adds them with compensated summation (see test_d20_fp64).
INT_TOL = {"fused": 1e-12, "two_pass": 1e-12}


def fsi_mod():
    from paper_2601_01903_amd import fsi
    return fsi


def gpu_apply(v, d, l, **kw):
    fsi = fsi_mod()
    dtype = kw.get("dtype", "f64")
    tdt = torch.float64 if dtype == "f64" else torch.float32
    plan = fsi.Plan(d, l, **kw)
    vt = torch.as_tensor(np.asarray(v), dtype=tdt).to(DEV)
    out = plan.apply(vt)
    torch.cuda.synchronize()
    res = out.double().cpu().numpy()
    info = plan.info()
    plan.close()
    return res, info


@pytest.mark.parametrize("algo", ["fused", "two_pass"])
def test_small_config_fp64(algo):
    say(f"[case] d=8 l=2 planted+normal FP64 algo={algo}")
    g, v = games.small_planted(0)
    got, _ = gpu_apply(v, 8, 2, algo=algo)
    assert normwise(got, oracle.fsi(v, 8, 2)) < 1e-12
    vn = games.small_normal(0)
    got, _ = gpu_apply(vn, 8, 2, algo=algo)
    assert normwise(got, oracle.fsi(vn, 8, 2)) < 1e-12


@pytest.mark.parametrize("algo", ["fused", "two_pass"])
def test_d14_tree_fp64(algo):
    say(f"[case] d=14 l=3 tree FP64 algo={algo}")
    g, v = games.d14_tree(0)
    got, info = gpu_apply(v, 14, 3, algo=algo)
    ref = oracle.fsi_c(v, 14, 3, nthreads=8)
    err = normwise(got, ref)
    say(f"  tile_bits={info['tile_bits']} err={err:.3e}")
    assert err < 1e-12


@pytest.mark.parametrize("l", [2, 4])
@pytest.mark.parametrize("algo", ["fused", "two_pass"])
def test_d20_fp64(l, algo):
    say(f"[case] d=20 l={l} tree and +/-1 FP64 algo={algo}")
    g, v = games.d20_tree(0)
    got, _ = gpu_apply(v, 20, l, algo=algo)
    assert normwise(got, oracle.fsi_c(v, 20, l, nthreads=8)) < 1e-12
    # +/-1: the FP64 oracle's own summation error reaches ~4e-11 here, so the
    # reference is the exact-integer evaluation (rounded once)
    vp = games.d20_pm1(0)
    got, _ = gpu_apply(vp, 20, l, algo=algo)
    err = normwise(got, oracle.fsi_exact_int(vp, 20, l, nthreads=8))
    say(f"  +/-1 err vs exact {err:.3e}")
    # The two-pass path multiplies full-range Moebius values (|a(T)| up to
    # 2^|T|) by the weights before the cross-tile sum, a cancellation-heavy
    # sum (the plain FP64 oracle itself is off by 4.2e-11 here): its per-tile
    # results are double-doubles and the cross-tile sum is compensated, so it
    # holds 1e-12 like the fused path, which weights in-tile Moebius values
    # (|a| <= 2^11).
    assert err < INT_TOL[algo]


_D20_REFS = {}


def _d20_refs(l):
    """Oracle references of the d = 20 inputs on their FP32 values: the tree
    game (FP64 oracle) and the +/-1 vector (exact-integer oracle)."""
    if l not in _D20_REFS:
        g, v = games.d20_tree(0)
        v32 = v.astype(np.float32)
        vp = games.d20_pm1(0).astype(np.float32)
        _D20_REFS[l] = (v32, oracle.fsi_c(v32.astype(np.float64), 20, l, nthreads=16),
                        vp, oracle.fsi_exact_int(vp.astype(np.float64), 20, l, nthreads=16))
    return _D20_REFS[l]


@pytest.mark.parametrize("l", [2, 4])
@pytest.mark.parametrize("prec", ["f32", "f32_compensated", "f32_fp64mob", "auto", "f32_fp64reg"])
@pytest.mark.parametrize("algo", ["fused", "two_pass"])
def test_d20_fp32_modes(prec, algo, l):
    """d = 20, l in {2, 4}, FP32 storage, every precision form: the tree game
    within 1e-6 of the oracle on the same FP32 values. On the +/-1 vector the
    fused algorithm is exact through the FP32 tile (in-tile Moebius values
    are integers below 2^11, in-tile sums below 2^22, the high-site Moebius
    is folded into FP64 weights), so its only error is the final rounding of
    each output to FP32 storage: every output within one FP32 ulp of the
    exact-integer oracle (relative 2^-23), normwise at most 2^-24. The
    two-pass algorithm with the FP64 sweep is held to the same normwise
    bound (its FP64 products of full-range Moebius values with the weights
    leave an absolute error near 1e-11 of the largest output, above one ulp
    of the smallest outputs). The two-pass FP32 sweep adds full-range
    Moebius values (up to 2^20) in FP32: held to the FP32 tolerance."""
    say(f"[case] d=20 l={l} FP32 storage prec={prec} algo={algo}")
    v32, ref, vp, refp = _d20_refs(l)
    got, _ = gpu_apply(v32, 20, l, dtype="f32", precision=prec, algo=algo)
    err = normwise(got, ref)
    say(f"  tree normwise err {err:.3e}")
    assert err < 1e-6
    gotp, _ = gpu_apply(vp, 20, l, dtype="f32", precision=prec, algo=algo)
    errp = normwise(gotp, refp)
    assert np.all(np.isfinite(gotp))
    if algo == "fused":
        ulp = np.max(np.abs(gotp - refp) / np.maximum(np.abs(refp), 1e-300))
        say(f"  +/-1 normwise err {errp:.3e}, max elementwise {ulp:.3e} "
            f"(gated: normwise <= 2^-24, elementwise <= 2^-23, the FP32 output rounding)")
        assert errp <= 2.0 ** -24 * (1 + 1e-6)
        assert np.all(np.abs(gotp - refp) <= 2.0 ** -23 * np.abs(refp) + 1e-13 * np.max(np.abs(refp)))
    elif prec == "f32_fp64reg":
        say(f"  +/-1 normwise err {errp:.3e} (gated: normwise <= 2^-24 + 1e-11)")
        assert errp <= 2.0 ** -24 + 1e-11
    else:
        say(f"  +/-1 normwise err {errp:.3e} (two-pass FP32 sweep: gated at 1e-6)")
        assert errp < 1e-6


@pytest.mark.parametrize("kernel", ["generic", "register"])
@pytest.mark.parametrize("prec", ["f32", "f32_compensated", "f32_fp64mob"])
@pytest.mark.parametrize("d,l", [(12, 4), (13, 2), (16, 3), (20, 4), (20, 1)])
def test_register_kernel_fp32(d, l, prec, kernel):
    say(f"[case] register-phase check d={d} l={l} {prec} kernel={kernel}")
    if d == 20:
        g, v = games.d20_tree(0)
        if l == 1:
            v = games.d20_batch_instance(1)[1]
    else:
        g = games.tree_game(d, 60, 5, games.rng_for(95, d * 10 + l))
        v = games.tree_values(g)
    v32 = v.astype(np.float32)
    ref = oracle.fsi_c(v32.astype(np.float64), d, l, nthreads=8)
    got, info = gpu_apply(v32, d, l, dtype="f32", precision=prec, kernel=kernel)
    err = normwise(got, ref)
    say(f"  tile_bits={info['tile_bits']} err={err:.3e}")
    assert err < 1e-6


@pytest.mark.parametrize("kernel", ["generic", "register"])
@pytest.mark.parametrize("d,l", [(11, 4), (12, 3), (17, 2), (20, 4)])
def test_register_kernel_fp64_exact(d, l, kernel):
    say(f"[case] register-phase FP64 d={d} l={l} kernel={kernel}")
    v = np.random.default_rng(3000 + d * 7 + l).integers(-4, 5, size=1 << d).astype(np.float64)
    got, _ = gpu_apply(v, d, l, kernel=kernel)
    assert normwise(got, oracle.fsi_exact_int(v, d, l, nthreads=8)) < 1e-12


@pytest.mark.parametrize("d,l", [(21, 3), (22, 2), (23, 1), (22, 3), (21, 4), (22, 4)])
def test_register_kernel_wide_high_part(d, l):
    """Up to 12 high bits (2^12 tiles per instance); at l = 4 past d = 20 the
    outputs need more slots than a workgroup holds: work items cover blocks
    of 2^6 tiles and the wide gather adds the blocks' partial sums."""
    say(f"[case] wide high part d={d} l={l}")
    v = np.random.default_rng(5000 + d * 7 + l).integers(-3, 4, size=1 << d).astype(np.float64)
    got, info = gpu_apply(v, d, l)
    say(f"  tile_bits={info['tile_bits']}")
    assert normwise(got, oracle.fsi_exact_int(v, d, l, nthreads=16)) < 1e-12


def test_register_kernel_small_d():
    """d < 11 on the register-phase kernel: the instance runs as d = 11 with
    the value of U taken as v(U & (2^d - 1)) (players past d ignored, so the
    Moebius coefficients vanish on every set holding one and the weights do
    not depend on d). Every (d, l) with d <= 10, l <= min(4, d): FP64 integer
    input against the exact oracle; Moebius input (zero past bit d - 1)
    against the oracle from the coefficients; FP32 storage of a tree game
    against the FP64 oracle."""
    fsi = fsi_mod()
    for d in range(1, 11):
        for l in range(1, min(4, d) + 1):
            say(f"[case] register kernel small d={d} l={l}")
            v = np.random.default_rng(5200 + 16 * d + l).integers(-4, 5, size=1 << d).astype(np.float64)
            plan = fsi.Plan(d, l, kernel="register")
            assert plan.schedule()["fast_instances"] == 1
            got = plan.apply(torch.as_tensor(v).to(DEV)).cpu().numpy()
            plan.close()
            assert normwise(got, oracle.fsi_exact_int(v, d, l, nthreads=4)) < 1e-12, (d, l)
            a = np.random.default_rng(5300 + 16 * d + l).standard_normal(1 << d)
            plan = fsi.Plan(d, l, kernel="register", input="mobius")
            got = plan.apply(torch.as_tensor(a).to(DEV)).cpu().numpy()
            plan.close()
            assert normwise(got, oracle.interaction_from_mobius_c(a, d, l, nthreads=4)) < 1e-12, (d, l)
            g = games.tree_game(d, 30, 4, games.rng_for(5400, d))
            v32 = games.tree_values(g).astype(np.float32)
            plan = fsi.Plan(d, l, dtype="f32", kernel="register")
            got = plan.apply(torch.from_numpy(v32).to(DEV)).double().cpu().numpy()
            plan.close()
            assert normwise(got, oracle.fsi(v32.astype(np.float64), d, l)) < 1e-6, (d, l)


@pytest.mark.parametrize("d,l", [(24, 2), (25, 1)])
def test_register_kernel_beyond_twelve_high_bits(d, l):
    """The register-phase kernel at l <= 3 holds up to 19 high bits (the
    output metadata word packs the Y offset into the bits the order needs)."""
    fsi = fsi_mod()
    say(f"[case] register kernel d={d} l={l} ({d - 11} high bits)")
    v = np.random.default_rng(5100 + d).integers(-3, 4, size=1 << d).astype(np.float64)
    plan = fsi.Plan(d, l, kernel="register")
    assert plan.schedule()["fast_instances"] == 1
    out = plan.apply(torch.as_tensor(v).to(DEV))
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    plan.close()
    assert normwise(got, oracle.fsi_exact_int(v, d, l, nthreads=16)) < 1e-12


def _ragged_batch():
    ds, ls = games.ragged_specs(512)
    built = games.build_many(lambda i: games.ragged_instance(i, ds[i]), range(len(ds)), threads=16)
    return ds, ls, [v for _, v in built]


_RAGGED_REFS = {}


def _ragged_refs(ds, ls, v32):
    """Oracle of every ragged instance on its FP32 values (computed once)."""
    if "r" not in _RAGGED_REFS:
        _RAGGED_REFS["r"] = [oracle.fsi_c(v.astype(np.float64), d, l, nthreads=16)
                             for v, d, l in zip(v32, ds, ls)]
    return _RAGGED_REFS["r"]


@pytest.mark.parametrize("prec,autotune", [("auto", True), ("f32_fp64mob", False),
                                           ("f32_compensated", False), ("f32", False)])
def test_ragged_batch_512_fp32(prec, autotune):
    """The 512-instance ragged batch (d ~ U{8..20}, l ~ U{1..4}, tree games),
    FP32 storage, one launch (graph replay), every instance against the oracle
    on the same FP32 values: <= 1e-6 normwise; the default form both
    autotuned (the launch the benchmark times) and with the default schedule."""
    fsi = fsi_mod()
    ds, ls, vals = _ragged_batch()
    say(f"[case] ragged batch n={len(ds)} {prec} autotune={autotune}, "
        f"{sum(1 << d for d in ds)} values")
    v32 = [v.astype(np.float32) for v in vals]
    refs = _ragged_refs(ds, ls, v32)
    bp = fsi.BatchPlan(ds, ls, dtype="f32", precision=prec, autotune=autotune)
    # every instance on the register-phase kernel: one tile kernel and one
    # reduction
    assert bp.schedule()["fast_instances"] == len(ds) and bp.num_stages() == 2
    flat = torch.from_numpy(np.concatenate(v32)).to(DEV)
    out = bp.apply(flat, graph=True)
    torch.cuda.synchronize()
    o = out.double().cpu().numpy()
    # the stages launched one by one and further replays give the same bits
    o2 = torch.empty_like(out)
    bp.apply_stage(flat, o2, 0)
    bp.apply_stage(flat, o2, 1)
    out3 = bp.apply(flat, graph=True)
    torch.cuda.synchronize()
    assert torch.equal(o2, out) and torch.equal(out3, out)
    errs = []
    for i, (d, l) in enumerate(zip(ds, ls)):
        err = normwise(o[bp.out_offset[i]:bp.out_offset[i + 1]], refs[i])
        errs.append(err)
        assert err < 1e-6, (i, d, l, err)
    say(f"  normwise max {max(errs):.3e} median {float(np.median(errs)):.3e}")
    bp.close()


def test_ragged_batch_512_fp64():
    fsi = fsi_mod()
    ds, ls, vals = _ragged_batch()
    say(f"[case] ragged batch n={len(ds)} FP64")
    bp = fsi.BatchPlan(ds, ls, dtype="f64")
    out = bp.apply(torch.from_numpy(np.concatenate(vals)).to(DEV), graph=True)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    for i, (v, d, l) in enumerate(zip(vals, ds, ls)):
        ref = oracle.fsi_c(v, d, l, nthreads=16)
        assert normwise(o[bp.out_offset[i]:bp.out_offset[i + 1]], ref) < 1e-12, (i, d, l)
    bp.close()


@pytest.mark.parametrize("d,l,tb", [(1, 1, 0), (2, 2, 0), (5, 5, 0), (9, 9, 0), (12, 4, 0),
                                    (13, 4, 0), (10, 3, 3), (11, 1, 4), (16, 2, 0),
                                    (15, 4, 7), (17, 3, 0)])
@pytest.mark.parametrize("algo", ["fused", "two_pass"])
def test_edge_shapes_fp64(d, l, tb, algo):
    say(f"[case] edge d={d} l={l} tile_bits={tb} algo={algo}")
    # small integers: the exact-integer oracle is the reference
    v = np.random.default_rng(1000 + 31 * d + l).integers(-4, 5, size=1 << d).astype(np.float64)
    got, _ = gpu_apply(v, d, l, algo=algo, tile_bits=tb)
    assert normwise(got, oracle.fsi_exact_int(v, d, l, nthreads=8)) < INT_TOL[algo]


def test_output_masks_match_oracle():
    fsi = fsi_mod()
    for d, l in [(8, 2), (14, 3), (20, 4), (6, 6)]:
        p = fsi.Plan(d, l)
        assert np.array_equal(p.output_masks().astype(np.int64), oracle.output_masks(d, l))
        p.close()


@pytest.mark.parametrize("d", [1, 7, 12, 13, 20])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_mobius_standalone(d, dtype):
    say(f"[case] mobius d={d} {dtype}")
    fsi = fsi_mod()
    v = np.random.default_rng(d).integers(-3, 4, size=1 << d).astype(np.float64)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    p = fsi.Plan(d, 1, dtype=dtype)
    a = torch.as_tensor(v, dtype=tdt).to(DEV)
    p.mobius(a)
    torch.cuda.synchronize()
    ref = oracle.mobius(v)  # small integers: exact in both dtypes
    assert np.array_equal(a.double().cpu().numpy(), ref)
    p.close()


def _batch_inputs(ds, seed):
    """Small-integer vectors, so the exact-integer oracle is the reference."""
    return [np.random.default_rng(seed + i).integers(-4, 5, size=1 << d).astype(np.float64)
            for i, d in enumerate(ds)]


@pytest.mark.parametrize("algo", ["fused", "two_pass"])
def test_batched_ragged_fp64(algo):
    fsi = fsi_mod()
    rng = np.random.default_rng(77)
    ds = [int(x) for x in rng.integers(1, 17, size=24)] + [8, 20, 1]
    ls = [int(rng.integers(1, d + 1)) for d in ds]
    say(f"[case] batched ragged FP64 algo={algo} n={len(ds)}")
    bp = fsi.BatchPlan(ds, ls, dtype="f64", algo=algo)
    vals = _batch_inputs(ds, 5000)
    flat = torch.from_numpy(np.concatenate(vals)).to(DEV)
    assert bp.value_offset[-1] == flat.numel()
    for graph in (False, True):
        out = bp.apply(flat, graph=graph)
        torch.cuda.synchronize()
        o = out.cpu().numpy()
        for i, (v, d, l) in enumerate(zip(vals, ds, ls)):
            got = o[bp.out_offset[i]:bp.out_offset[i + 1]]
            assert normwise(got, oracle.fsi_exact_int(v, d, l, nthreads=8)) < INT_TOL[algo], (i, d, l)
    bp.close()


def test_batched_matches_single_and_order():
    """Batched results equal per-instance fsi_apply, independent of order."""
    fsi = fsi_mod()
    ds, ls = [9, 13, 6, 13, 11], [2, 3, 6, 1, 4]
    vals = _batch_inputs(ds, 6000)
    bp = fsi.BatchPlan(ds, ls, dtype="f64")
    out = bp.apply(torch.from_numpy(np.concatenate(vals)).to(DEV)).cpu().numpy()
    perm = [3, 0, 4, 2, 1]
    bp2 = fsi.BatchPlan([ds[i] for i in perm], [ls[i] for i in perm], dtype="f64")
    out2 = bp2.apply(torch.from_numpy(np.concatenate([vals[i] for i in perm])).to(DEV)).cpu().numpy()
    for j, i in enumerate(perm):
        a = out[bp.out_offset[i]:bp.out_offset[i + 1]]
        b = out2[bp2.out_offset[j]:bp2.out_offset[j + 1]]
        single, _ = gpu_apply(vals[i], ds[i], ls[i])
        assert np.array_equal(a, b)
        assert np.array_equal(a, single)
    bp.close()
    bp2.close()


def test_graph_replays_with_eager_work_between():
    fsi = fsi_mod()
    ds, ls = [10, 12, 14, 8], [3, 2, 4, 1]
    say("[case] graph replays")
    vals = _batch_inputs(ds, 7000)
    bp = fsi.BatchPlan(ds, ls, dtype="f32", precision="f32")
    flat = torch.from_numpy(np.concatenate(vals).astype(np.float32)).to(DEV)
    out = torch.empty(bp.out_offset[-1], dtype=torch.float32, device=DEV)
    eager = bp.apply(flat, graph=False).cpu().numpy()
    for rep in range(4):
        out.fill_(float("nan"))
        junk = torch.randn(1 << 16, device=DEV).sum()  # eager work between replays
        bp.apply(flat, out=out, graph=True)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), eager), rep
        del junk
    bp.close()


def test_repeatable_bitwise():
    fsi = fsi_mod()
    g, v = games.d14_tree(0)
    p = fsi.Plan(14, 3)
    vt = torch.from_numpy(v).to(DEV)
    a = p.apply(vt).cpu().numpy()
    for _ in range(3):
        assert np.array_equal(p.apply(vt).cpu().numpy(), a)
    p.close()


def test_error_paths_on_device():
    fsi = fsi_mod()
    with pytest.raises(fsi.FsiError) as e:
        fsi.Plan(0, 1)
    assert e.value.status == 1
    with pytest.raises(fsi.FsiError):
        fsi.Plan(5, 6)
    with pytest.raises(fsi.FsiError):
        fsi.Plan(31, 2)
    with pytest.raises(fsi.FsiError):
        fsi.Plan(10, 2, dtype="f64", precision="f32")
    with pytest.raises(fsi.FsiError):
        fsi.Plan(10, 2, tile_bits=11 + 2)
    p = fsi.Plan(6, 2)
    lib = fsi.load()
    import ctypes
    v = torch.zeros(64, dtype=torch.float64, device=DEV)
    out = torch.zeros(p.M + 1, dtype=torch.float64, device=DEV)
    # misaligned output pointer is rejected before any launch
    st = lib.fsi_apply(p._h, ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(out.data_ptr() + 8), None)
    assert st == 1 and b"aligned" in lib.fsi_last_error()
    st = lib.fsi_apply(p._h, None, ctypes.c_void_p(out.data_ptr()), None)
    assert st == 1
    with pytest.raises(ValueError):
        p.apply(torch.zeros(63, dtype=torch.float64, device=DEV))
    p.close()
    with pytest.raises(fsi.FsiError):
        fsi.BatchPlan([4, 3], [5, 1])


def test_autotuned_plans_match_oracle():
    """fsi_plan_opts.autotune: candidates are timed at plan time, the chosen
    schedule is reported, cached per shape, and the results stay exact."""
    fsi = fsi_mod()
    say("[case] autotune single d=16 l=3 f32")
    g = games.tree_game(16, 60, 5, games.rng_for(96, 1))
    v32 = games.tree_values(g).astype(np.float32)
    p = fsi.Plan(16, 3, dtype="f32", precision="f32_compensated", autotune=True)
    sc = p.schedule()
    say(f"  schedule {sc}")
    assert sc["autotuned"] == 1 and sc["tuned_ms"] > 0
    got = p.apply(torch.from_numpy(v32).to(DEV)).double().cpu().numpy()
    assert normwise(got, oracle.fsi_c(v32.astype(np.float64), 16, 3, nthreads=8)) < 1e-6
    p2 = fsi.Plan(16, 3, dtype="f32", precision="f32_compensated", autotune=True)
    assert p2.schedule()["autotuned"] == 1          # from the cache
    p.close()
    p2.close()
    say("[case] autotune batched ragged FP64, fused and two-pass")
    ds, ls = [9, 12, 14, 11, 13], [2, 4, 3, 1, 4]
    vals = _batch_inputs(ds, 8000)
    flat = torch.from_numpy(np.concatenate(vals)).to(DEV)
    for algo in ("fused", "two_pass"):
        bp = fsi.BatchPlan(ds, ls, dtype="f64", algo=algo, autotune=True)
        sc = bp.schedule()
        say(f"  {algo}: {sc}")
        assert sc["autotuned"] == 1
        if algo == "two_pass":
            assert sc["mob_group"] in (4, 5, 6)
        o = bp.apply(flat, graph=True).cpu().numpy()
        for i, (v, d, l) in enumerate(zip(vals, ds, ls)):
            assert normwise(o[bp.out_offset[i]:bp.out_offset[i + 1]],
                            oracle.fsi_exact_int(v, d, l, nthreads=8)) < INT_TOL[algo], (algo, i)
        bp.close()


def test_auto_algorithm_for_high_orders():
    """FSI_ALGO_AUTO runs the two-pass algorithm when every instance has
    l >= 7, the fused one otherwise (the schedule reports mob_group > 0 for
    two-pass); with the autotuner and every l > 4 it times both. Every
    result is within 1e-12 of the exact-integer oracle."""
    fsi = fsi_mod()
    cases = [([12, 10, 11], [7, 9, 8], True), ([12, 10, 11], [7, 5, 8], False),
             ([12, 13], [4, 7], False)]
    for ds, ls, two_pass in cases:
        say(f"[case] auto algorithm ds={ds} ls={ls}")
        vals = _batch_inputs(ds, 9100)
        bp = fsi.BatchPlan(ds, ls, dtype="f64")
        assert (bp.schedule()["mob_group"] > 0) == two_pass, bp.schedule()
        o = bp.apply(torch.from_numpy(np.concatenate(vals)).to(DEV)).cpu().numpy()
        for i, (v, d, l) in enumerate(zip(vals, ds, ls)):
            assert normwise(o[bp.out_offset[i]:bp.out_offset[i + 1]],
                            oracle.fsi_exact_int(v, d, l, nthreads=8)) < 1e-12, (ds, ls, i)
        bp.close()
    ds, ls = [12, 11], [6, 8]
    say(f"[case] auto algorithm, autotuned, ds={ds} ls={ls}")
    vals = _batch_inputs(ds, 9200)
    bp = fsi.BatchPlan(ds, ls, dtype="f64", autotune=True)
    sc = bp.schedule()
    say(f"  schedule {sc}")
    assert sc["autotuned"] == 1
    o = bp.apply(torch.from_numpy(np.concatenate(vals)).to(DEV)).cpu().numpy()
    for i, (v, d, l) in enumerate(zip(vals, ds, ls)):
        assert normwise(o[bp.out_offset[i]:bp.out_offset[i + 1]],
                        oracle.fsi_exact_int(v, d, l, nthreads=8)) < 1e-12, (i, d, l)
    bp.close()
