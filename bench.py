#!/usr/bin/env python3
"""Benchmark of the FSI operator on one MI355X.

Workload (the configuration the headline metric is quoted on): 256 instances
at d = 20, l = 4 (268,435,456 coalition values, 1 GiB in FP32): even
instances are tree-ensemble games (200 depth-6 trees on 20 features), odd
instances planted sparse games (200 terms, |A| ~ U{1..6}); synthetic, seeded.

Timed: the batched FP32 apply as the library runs it (a replay of the plan's
captured graph; inputs resident in HBM). Reported beside it: per-kernel times
from the same apply launched stage by stage with HIP events between the
stages, the roofline of the dominant kernel, the plain FP64 GPU path on the
same instances (one fsi_apply per instance), the batched FP64 path, the error
of the FP32 path per instance, and the CPU oracle timed on a sample of the
same instances.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FSI coalition-values/s at d=20,l=4: batched FP32 vs plain FP64, % HBM peak"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Files of the dominant kernel's translation unit: the HBM counters stored in
# profiles/ stay valid while these are unchanged.
KERNEL_TU = ("fsi_tile11.hip", "fsi_tile11.h", "fsi_kernels.h", "fsi_internal.h")


def kernel_source_hash() -> str:
    """SHA-256 over the sources the register-phase tile kernel is compiled from."""
    import hashlib
    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_2601_01903_amd", "csrc")
    for f in KERNEL_TU:
        h.update(f.encode())
        with open(os.path.join(src, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload_key: str):
    """HBM bytes per launch of the tile kernel from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration), or None when
    that summary was taken on other kernel sources or another workload."""
    path = os.path.join(ROOT, "profiles", "tile11_kernel_d20_l4_x256_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith((" ", "#")):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != kernel_source_hash() or kv.get("workload") != workload_key:
        return None
    try:
        return {"fetch": float(kv["fetch_bytes_per_launch"]),
                "write": float(kv["write_bytes_per_launch"])}
    except (KeyError, ValueError):
        return None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def elementwise(x, ref, floor_frac=1e-3):
    """Secondary error: max |x_S - ref_S| / |ref_S| over |ref_S| >= floor_frac max |ref|."""
    keep = np.abs(ref) >= floor_frac * np.max(np.abs(ref))
    return float(np.max(np.abs(x[keep] - ref[keep]) / np.abs(ref[keep])))


def normwise(x, ref):
    den = float(np.max(np.abs(ref)))
    return float(np.max(np.abs(x - ref)) / den) if den else float(np.max(np.abs(x)))


def heap_forest(g):
    """Node arrays of a games.TreeGame (full binary trees in heap order)."""
    n_int = (1 << g.depth) - 1
    n_tree = n_int + (1 << g.depth)
    K = g.feat.shape[0]
    feature = np.full(K * n_tree, -1, dtype=np.int32)
    threshold = np.zeros(K * n_tree)
    left = np.zeros(K * n_tree, dtype=np.int32)
    right = np.zeros(K * n_tree, dtype=np.int32)
    value = np.zeros(K * n_tree)
    idx = np.arange(n_int)
    for k in range(K):
        o = k * n_tree
        feature[o:o + n_int] = g.feat[k]
        threshold[o:o + n_int] = g.thr[k]
        left[o:o + n_int] = o + 2 * idx + 1
        right[o:o + n_int] = o + 2 * idx + 2
        value[o + n_int:o + n_tree] = g.leaf[k]
    return np.arange(K, dtype=np.int32) * n_tree, feature, threshold, left, right, value


def bench_forest(args, n, d, N, vals32, x32, stream, bp32, out32, threads):
    """Generate the value functions of the even (tree-game) instances on the
    GPU straight into the FSI input buffer, time that step and the chain
    (generation + batched FSI), check it against the seeded generator, and
    time one forest with 100 background points. Returns the record and the
    sampled GPU values the CPU oracle leg checks."""
    import torch
    import games
    from paper_2601_01903_amd import Forest
    dev = x32.device
    tree_ids = list(range(0, n, 2))
    forests, xs, bgs = [], [], []
    for i in tree_ids:
        g = games.tree_game(d, 200, 6, games.rng_for(games.CFG_D20_BATCH, i))
        forests.append(Forest(d, *heap_forest(g), max_bg=100))
        xs.append(torch.as_tensor(g.x).to(dev))
        bgs.append(torch.as_tensor(g.b[None, :].copy()).to(dev))
        if i == 0:
            g0 = g
    xv = x32.clone()

    def gen():
        for k, i in enumerate(tree_ids):
            forests[k].values(xs[k], bgs[k], dtype="f32", out=xv[i * N:(i + 1) * N])

    work = torch.empty(N, dtype=torch.float64, device=dev)

    def gen_mobius():
        for k, i in enumerate(tree_ids):
            forests[k].values(xs[k], bgs[k], dtype="f32", out=xv[i * N:(i + 1) * N],
                              method="mobius", work=work)

    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    reps = max(1, args.steps // 4)

    def timed(fn, with_fsi=False):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            fn()
            if with_fsi:
                bp32.apply(xv, out32)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    mob_ms = timed(gen_mobius)
    chain_mob_ms = timed(gen_mobius, with_fsi=True)

    # FSI of the 128 tree games straight from their Moebius coefficients
    # (Moebius input: no subset sums, no in-tile butterfly) against the chain
    # through v, both on a 128-instance plan
    from paper_2601_01903_amd import BatchPlan
    nt = len(tree_ids)
    bp_v = BatchPlan([d] * nt, [4] * nt, dtype="f32", autotune=not args.no_autotune)
    bp_a = BatchPlan([d] * nt, [4] * nt, dtype="f32", autotune=not args.no_autotune,
                     input="mobius")
    x128 = torch.empty(nt * N, dtype=torch.float32, device=dev)
    o_v = torch.empty(bp_v.out_offset[-1], dtype=torch.float32, device=dev)
    o_a = torch.empty_like(o_v)

    def chain_v():
        for k in range(nt):
            forests[k].values(xs[k], bgs[k], dtype="f32", out=x128[k * N:(k + 1) * N],
                              method="mobius", work=work)
        bp_v.apply(x128, o_v)

    def chain_a():
        for k in range(nt):
            forests[k].mobius(xs[k], bgs[k], out=work)
            x128[k * N:(k + 1) * N].copy_(work)
        bp_a.apply(x128, o_a)

    chain_v128_ms = timed(chain_v)
    chain_a128_ms = timed(chain_a)
    ov, oa = o_v.double().cpu().numpy(), o_a.double().cpu().numpy()
    M4 = bp_v.out_offset[1]
    chain_diff = max(normwise(oa[k * M4:(k + 1) * M4], ov[k * M4:(k + 1) * M4]) for k in range(nt))
    bp_v.close()
    bp_a.close()
    del x128, o_v, o_a
    got_m = xv.cpu().numpy()
    mob_err = max(float(np.max(np.abs(got_m[i * N:(i + 1) * N] - vals32[i * N:(i + 1) * N]))
                        / np.max(np.abs(vals32[i * N:(i + 1) * N]))) for i in tree_ids)
    gen_ms = timed(gen)
    chain_ms = timed(gen, with_fsi=True)
    got = xv.cpu().numpy()
    # the walked tree games equal the seeded inputs (same order of sums)
    same = all(np.array_equal(got[i * N:(i + 1) * N], vals32[i * N:(i + 1) * N]) for i in tree_ids)
    forest0 = heap_forest(g0)
    rng = np.random.default_rng(5)
    samp = [int(S) for S in rng.integers(0, N, size=200)]
    # interventional game over 100 background points (one forest)
    rbg = torch.as_tensor(np.random.default_rng(6).uniform(size=(100, d))).to(dev)
    vb = torch.empty(N, dtype=torch.float32, device=dev)
    forests[0].values(xs[0], rbg, dtype="f32", out=vb)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        forests[0].values(xs[0], rbg, dtype="f32", out=vb)
    e1.record(stream)
    torch.cuda.synchronize()
    bg_ms = e0.elapsed_time(e1) / reps
    vb_walk = vb.cpu().numpy()
    rb = rbg.cpu().numpy()
    bg_mob_ms = timed(lambda: forests[0].values(xs[0], rbg, dtype="f32", out=vb, method="mobius",
                                                work=work))
    vb_mob = vb.cpu().numpy()
    bg_mob_diff = float(np.max(np.abs(vb_mob.astype(np.float64) - vb_walk)) /
                        max(1.0, float(np.max(np.abs(vb_walk)))))
    for F in forests:
        F.close()
    visits = 200 * 6   # internal nodes on each (tree) walk of a depth-6 forest
    rec = {"instances": len(tree_ids), "trees": 200, "depth": 6, "d": d,
           "ms_per_step": gen_ms,
           "coalitions_per_s": len(tree_ids) * N / (gen_ms * 1e-3),
           "node_visits_per_s": len(tree_ids) * N * visits / (gen_ms * 1e-3),
           "chain_ms_per_step": chain_ms,
           "chain_note": "generate the 128 tree games, then the batched FSI of all 256 instances",
           "equals_seeded_inputs": bool(same),
           "mobius_route": {"ms_per_step": mob_ms,
                            "coalitions_per_s": len(tree_ids) * N / (mob_ms * 1e-3),
                            "chain_ms_per_step": chain_mob_ms,
                            "max_rel_diff_vs_seeded_inputs": mob_err},
           "fsi_of_128_tree_games": {
               "via_values_ms": chain_v128_ms,
               "via_moebius_input_ms": chain_a128_ms,
               "max_normwise_diff": chain_diff,
               "note": "Moebius route to v then FSI, against scattered Moebius coefficients "
                       "then FSI with Moebius input"},
           "multi_background": {"n_bg": 100, "ms": bg_ms,
                                "coalition_values_per_s": N / (bg_ms * 1e-3),
                                "mobius_route_ms": bg_mob_ms,
                                "mobius_route_rel_diff_vs_walk": bg_mob_diff}}
    log(f"value functions (Moebius route): {mob_ms:.3f} ms, chain {chain_mob_ms:.3f} ms, "
        f"max rel diff {mob_err:.2e}")
    log(f"FSI of the 128 tree games: via v {chain_v128_ms:.3f} ms, via Moebius input "
        f"{chain_a128_ms:.3f} ms, diff {chain_diff:.2e}")
    log(f"value functions: {gen_ms:.3f} ms for {len(tree_ids)} forests "
        f"({rec['coalitions_per_s']:.3e} coalitions/s), chain {chain_ms:.3f} ms, "
        f"100 backgrounds {bg_ms:.3f} ms (Moebius route {bg_mob_ms:.3f} ms), "
        f"equal to the seeded inputs {same}")
    ctx = {"forest0": forest0, "x": g0.x, "b": g0.b[None, :], "samp": samp,
           "got": [float(got[S]) for S in samp], "rb": rb,
           "got_bg": [float(vb_walk[S]) for S in samp[:8]]}
    return rec, ctx


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n-inst", type=int, default=256)
    ap.add_argument("--precision", default="f32_fp64mob",
                    help="FP32-storage precision form of the timed region (the library's AUTO "
                         "choice by default); the other forms are timed beside it")
    ap.add_argument("--algo", default="auto")
    ap.add_argument("--tile-bits", type=int, default=0)
    ap.add_argument("--cpu-sample", type=int, default=128)
    ap.add_argument("--check-sample", type=int, default=4)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the single-instance d = 28 and d = 30 timings")
    ap.add_argument("--no-forest", action="store_true",
                    help="skip generating the tree games' value functions on the GPU")
    ap.add_argument("--no-indices", action="store_true",
                    help="skip the other interaction indices (SII, k-SII, STII, BII) on the workload")
    ap.add_argument("--no-ragged", action="store_true",
                    help="skip the 512-instance ragged batch")
    ap.add_argument("--no-c3", action="store_true",
                    help="skip the d = 20 single instances at l = 2 and 4")
    ap.add_argument("--no-closed-form", dest="closed_form", action="store_false",
                    help="skip checking every headline instance against its closed form")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the heuristic schedule instead of timing candidates at plan time")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU (asked for --gpus {args.gpus}); "
              "sharding the batched operator by instance across GPUs is not implemented.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import games
    from paper_2601_01903_amd import BatchPlan, Plan

    dev = torch.device("cuda:0")
    n, d, l = args.n_inst, 20, 4
    N = 1 << d
    threads = min(16, os.cpu_count() or 1)

    t0 = time.time()
    built = games.build_many(games.d20_batch_instance, range(n), threads=threads)
    vals64 = np.concatenate([v for _, v in built])
    del built
    vals32 = vals64.astype(np.float32)
    log(f"generated {n} instances in {time.time() - t0:.1f}s")

    x32 = torch.from_numpy(vals32).to(dev)
    t0 = time.time()
    bp32 = BatchPlan([d] * n, [l] * n, dtype="f32", precision=args.precision, algo=args.algo,
                     tile_bits=args.tile_bits, autotune=not args.no_autotune)
    sched = bp32.schedule()
    log(f"plan in {time.time() - t0:.2f}s, schedule {sched}")
    M = bp32.out_offset[1]
    out32 = torch.empty(bp32.out_offset[-1], dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    # ---- per-kernel durations: the plan's stages launched back to back on
    # one stream with HIP events between them ----
    ns = bp32.num_stages()
    for _ in range(args.warmup):
        for s in range(ns):
            bp32.apply_stage(x32, out32, s)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(ns + 1)] for _ in range(args.steps)]
    for k in range(args.steps):
        evs[k][0].record(stream)
        for s in range(ns):
            bp32.apply_stage(x32, out32, s)
            evs[k][s + 1].record(stream)
    torch.cuda.synchronize()
    eager_ms = evs[0][0].elapsed_time(evs[-1][ns]) / args.steps
    stage_ms = [float(np.mean([evs[k][s].elapsed_time(evs[k][s + 1]) for k in range(args.steps)]))
                for s in range(ns)]
    dom = int(np.argmax(stage_ms))
    log(f"FP32 batched, stages launched one by one with events between them: {eager_ms:.3f} "
        f"ms/step; stage times (ms): {['%.4f' % x for x in stage_ms]}")
    alg_bytes = n * N * 4  # each FP32 coalition value read once by the tile kernel
    achieved = alg_bytes / (stage_ms[dom] * 1e-3) / 1e9

    # ---- timed region: the batched apply as the library runs it (fsi_apply_batched,
    # a replay of the plan's captured graph), K steps between two events ----
    for _ in range(max(2, args.warmup)):
        bp32.apply(x32, out32, graph=True)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        bp32.apply(x32, out32, graph=True)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t_wall) * 1e3 / args.steps
    graph_ms = ev0.elapsed_time(ev1) / args.steps
    ms_per_step = graph_ms
    value = n * N / (ms_per_step * 1e-3)
    log(f"FP32 batched: {ms_per_step:.3f} ms/step (wall {wall_ms:.3f}), {value:.3e} values/s")

    # ---- copy-kernel calibration for the HBM byte counters: a plain
    # device-to-device copy of the FP32 input (known size); also timed, as the
    # bandwidth a plain streaming kernel reaches on this device ----
    cal = torch.empty_like(x32)
    cev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    cev[0].record(stream)
    for i in range(3):
        cal.copy_(x32)
        cev[i + 1].record(stream)
    torch.cuda.synchronize()
    del cal
    copy_ms = float(np.median([cev[i].elapsed_time(cev[i + 1]) for i in range(3)]))
    copy_gbs = 2 * alg_bytes / (copy_ms * 1e-3) / 1e9   # read + write
    log(f"device-to-device copy of the input: {copy_ms:.3f} ms = {copy_gbs:.0f} GB/s (read + write)")
    res32 = out32.double().cpu().numpy()

    # ---- the other interaction indices through the same kernels: same
    # workload, precision and schedule, graph replays timed with events ----
    indices = None
    index_samples = {}
    if not args.no_indices:
        indices = {}
        for index in ("stii", "sii", "ksii", "bii"):
            bpi = BatchPlan([d] * n, [l] * n, dtype="f32", precision=args.precision,
                            algo=args.algo, tile_bits=args.tile_bits,
                            autotune=not args.no_autotune, index=index)
            oi = torch.empty_like(out32)
            for _ in range(args.warmup):
                bpi.apply(x32, oi)
            torch.cuda.synchronize()
            ev0.record(stream)
            for _ in range(args.steps):
                bpi.apply(x32, oi)
            ev1.record(stream)
            torch.cuda.synchronize()
            ims = ev0.elapsed_time(ev1) / args.steps
            index_samples[index] = oi[:min(2, n) * M].double().cpu().numpy()
            indices[index] = {"ms_per_step": ims, "values_per_s": n * N / (ims * 1e-3)}
            bpi.close()
            log(f"index {index}: {ims:.3f} ms/step")

    # ---- the other FP32-storage precision forms on the same workload ----
    forms = {}
    for form in ("f32_compensated", "f32", "f32_fp64mob"):
        if form == args.precision:
            continue
        bpf = BatchPlan([d] * n, [l] * n, dtype="f32", precision=form, algo=args.algo,
                        tile_bits=args.tile_bits, autotune=not args.no_autotune)
        of = torch.empty_like(out32)
        for _ in range(args.warmup):
            bpf.apply(x32, of)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(args.steps):
            bpf.apply(x32, of)
        ev1.record(stream)
        torch.cuda.synchronize()
        fms = ev0.elapsed_time(ev1) / args.steps
        forms[form] = {"ms_per_step": fms, "values_per_s": n * N / (fms * 1e-3),
                       # whole step (tile kernel and reduction) against the
                       # HBM peak, the same algorithmic bytes as the headline
                       "hbm_frac_whole_step": n * N * 4 / (fms * 1e-3) / (HBM_PEAK_GBS * 1e9),
                       "out": of.double().cpu().numpy()}
        bpf.close()
        log(f"precision form {form}: {fms:.3f} ms/step")

    # ---- value functions of the tree-game half generated on the GPU ----
    vfun, forest_ctx = None, None
    if not args.no_forest:
        vfun, forest_ctx = bench_forest(args, n, d, N, vals32, x32, stream, bp32, out32, threads)

    # ---- single instances beyond the register-phase kernel (d = 28, 30) ----
    large = None
    if not args.no_large:
        large = {}
        for dl, ll in ((28, 4), (30, 2)):
            xl = torch.randn(1 << dl, dtype=torch.float32, device=dev)
            pl = Plan(dl, ll, dtype="f32", precision=args.precision)
            ol = pl.apply(xl)
            torch.cuda.synchronize()
            reps = max(1, args.steps // 4)
            ev0.record(stream)
            for _ in range(reps):
                pl.apply(xl, ol)
            ev1.record(stream)
            torch.cuda.synchronize()
            lms = ev0.elapsed_time(ev1) / reps
            large[f"d{dl}_l{ll}"] = {"ms": lms, "values_per_s": (1 << dl) / (lms * 1e-3),
                                     "hbm_frac": (1 << dl) * 4 / (lms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                     "tile_bits": pl.info()["tile_bits"]}
            log(f"single instance d={dl} l={ll}: {lms:.2f} ms ({(1 << dl) / (lms * 1e-3):.3e} values/s)")
            pl.close()
            del xl, ol

    # ---- the 512-instance ragged batch (d ~ U{8..20}, l ~ U{1..4}, tree
    # games, FP32 storage, the default precision form, autotuned): one graph
    # replay per step, the per-kernel stage times beside it ----
    ragged, ragged_ctx = None, None
    if not args.no_ragged:
        rds, rls = games.ragged_specs(512)
        rbuilt = games.build_many(lambda i: games.ragged_instance(i, rds[i]), range(len(rds)),
                                  threads=threads)
        rv32 = np.concatenate([v for _, v in rbuilt]).astype(np.float32)
        del rbuilt
        rx = torch.from_numpy(rv32).to(dev)
        rbp = BatchPlan(rds, rls, dtype="f32", precision=args.precision,
                        autotune=not args.no_autotune)
        rout = rbp.apply(rx, graph=True)
        rns = rbp.num_stages()
        for _ in range(args.warmup):
            rbp.apply(rx, rout, graph=True)
            for s_ in range(rns):
                rbp.apply_stage(rx, rout, s_)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(args.steps):
            rbp.apply(rx, rout, graph=True)
        ev1.record(stream)
        torch.cuda.synchronize()
        rms = ev0.elapsed_time(ev1) / args.steps
        revs = [[torch.cuda.Event(enable_timing=True) for _ in range(rns + 1)]
                for _ in range(args.steps)]
        for k in range(args.steps):
            revs[k][0].record(stream)
            for s_ in range(rns):
                rbp.apply_stage(rx, rout, s_)
                revs[k][s_ + 1].record(stream)
        torch.cuda.synchronize()
        rstage = [float(np.mean([revs[k][s_].elapsed_time(revs[k][s_ + 1])
                                 for k in range(args.steps)])) for s_ in range(rns)]
        rvals = rbp.value_offset[-1]
        rbytes = rvals * 4 + rbp.out_offset[-1] * 4
        ragged = {"n_instances": len(rds), "values": rvals, "outputs": rbp.out_offset[-1],
                  "ms_per_step": rms, "values_per_s": rvals / (rms * 1e-3),
                  "algorithmic_bytes": rbytes,
                  "hbm_frac": rbytes / (rms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                  "stage_ms": rstage, "sum_stage_ms": float(sum(rstage)),
                  "schedule": rbp.schedule(), "precision": args.precision,
                  "what": "512 instances, d ~ U{8..20}, l ~ U{1..4}, each its own tree game "
                          "(100 depth-5 trees), FP32 storage, graph replay"}
        ragged_ctx = {"ds": rds, "ls": rls, "v32": rv32, "out": rout.double().cpu().numpy(),
                      "ooff": list(rbp.out_offset), "voff": list(rbp.value_offset)}
        rbp.close()
        del rx, rout
        log(f"ragged batch: {rms:.3f} ms/step, {ragged['values_per_s']:.3e} values/s, "
            f"{ragged['hbm_frac']:.3f} of HBM peak; stages {['%.4f' % x for x in rstage]}")

    # ---- d = 20 single instances at l = 2 and 4: the FP64 path and the FP32
    # forms on a tree game (200 depth-6 trees) and an i.i.d. +/-1 vector ----
    c3, c3_ctx = None, None
    if not args.no_c3:
        g3, v3 = games.d20_tree(0)
        vp3 = games.d20_pm1(0)
        c3_ctx = {"tree": v3, "pm1": vp3, "got": {}}
        c3 = {}
        for l3 in (2, 4):
            for vname, vv in (("tree", v3), ("pm1", vp3)):
                for form in ("f64", "f32_fp64mob", "f32_compensated", "f32"):
                    dt = "f64" if form == "f64" else "f32"
                    pl3 = Plan(20, l3, dtype=dt, precision="f64" if form == "f64" else form)
                    xv = torch.from_numpy(vv.astype(np.float64 if dt == "f64" else np.float32)).to(dev)
                    o3 = pl3.apply(xv)
                    torch.cuda.synchronize()
                    c3_ctx["got"][(l3, vname, form)] = o3.double().cpu().numpy()
                    pl3.close()
        log("d=20 single instances at l = 2, 4 computed")

    # ---- latency of one instance (fsi_apply: direct launches, default
    # schedule), FP32 storage, the headline's first instance ----
    single = None
    if not args.no_c3:
        single = {}
        xs = x32[:N]
        for l1 in (2, 4):
            p1 = Plan(d, l1, dtype="f32", precision=args.precision)
            o1 = p1.apply(xs)
            for _ in range(5):
                p1.apply(xs, o1)
            torch.cuda.synchronize()
            reps = 50
            ev0.record(stream)
            for _ in range(reps):
                p1.apply(xs, o1)
            ev1.record(stream)
            torch.cuda.synchronize()
            us = ev0.elapsed_time(ev1) / reps * 1e3
            single[f"d{d}_l{l1}"] = {"us_per_apply": us, "values_per_s": N / (us * 1e-6),
                                     "schedule": p1.schedule()}
            p1.close()
        log(f"single-instance latency: {single}")

    # ---- FP64 paths on the same instances ----
    fp64 = None
    errs = None
    if not args.no_fp64:
        del x32
        x64 = torch.from_numpy(vals64).to(dev)
        plan64 = Plan(d, l, dtype="f64")
        o64 = torch.empty(n * M, dtype=torch.float64, device=dev)

        def plain_pass():
            for i in range(n):
                plan64.apply(x64[i * N:(i + 1) * N], o64[i * M:(i + 1) * M])

        plain_pass()
        torch.cuda.synchronize()
        reps = max(1, args.steps // 4)
        ev0.record(stream)
        for _ in range(reps):
            plain_pass()
        ev1.record(stream)
        torch.cuda.synchronize()
        plain_ms = ev0.elapsed_time(ev1) / reps
        res64 = o64.cpu().numpy()
        plan64.close()

        bp64 = BatchPlan([d] * n, [l] * n, dtype="f64")
        ob64 = torch.empty(n * M, dtype=torch.float64, device=dev)
        for _ in range(args.warmup):
            bp64.apply(x64, ob64)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(args.steps):
            bp64.apply(x64, ob64)
        ev1.record(stream)
        torch.cuda.synchronize()
        b64_ms = ev0.elapsed_time(ev1) / args.steps
        # The batched plan splits instances into a different number of work
        # items than the single-instance plan, so the partial sums are added in
        # another order: equal to rounding, not bit for bit.
        rb = ob64.cpu().numpy()
        bdiff = max(normwise(rb[i * M:(i + 1) * M], res64[i * M:(i + 1) * M]) for i in range(n))
        assert bdiff < 1e-12, f"batched FP64 differs from per-instance FP64 by {bdiff:.3e}"
        bp64.close()
        del x64
        fp64 = {"plain_ms_per_pass": plain_ms, "plain_values_per_s": n * N / (plain_ms * 1e-3),
                "batched_ms_per_step": b64_ms, "batched_values_per_s": n * N / (b64_ms * 1e-3)}
        per = [normwise(res32[i * M:(i + 1) * M], res64[i * M:(i + 1) * M]) for i in range(n)]
        errs = {"vs_fp64_gpu_max": float(np.max(per)), "vs_fp64_gpu_median": float(np.median(per)),
                "vs_fp64_gpu_max_tree": float(np.max(per[0::2])),
                "vs_fp64_gpu_max_planted": float(np.max(per[1::2]))}
        log(f"FP64 plain {plain_ms:.2f} ms/pass, batched {b64_ms:.3f} ms; FP32 err {errs}")
        for form, rec_f in forms.items():
            pf = [normwise(rec_f["out"][i * M:(i + 1) * M], res64[i * M:(i + 1) * M])
                  for i in range(n)]
            rec_f["vs_fp64_gpu_max"] = float(np.max(pf))
            rec_f["vs_fp64_gpu_median"] = float(np.median(pf))

    # ---- the CPU oracle leg, the only part of the bench that runs the
    # oracle: its baseline timing, and the oracle values sampled GPU results
    # are compared with (headline, other indices, value functions) ----
    import oracle
    sample_err = []
    for i in range(min(args.check_sample, n)):
        v = vals32[i * N:(i + 1) * N].astype(np.float64)
        ref = oracle.fsi_c(v, d, l, nthreads=threads)
        sample_err.append(normwise(res32[i * M:(i + 1) * M], ref))
    if errs is not None:
        errs["vs_oracle_sample_max"] = float(np.max(sample_err)) if sample_err else None
        errs["oracle_sample"] = len(sample_err)
    if args.check_sample > 0:
        for index, ri in index_samples.items():
            ierr = [normwise(ri[i * M:(i + 1) * M],
                             oracle.fsi_c(vals32[i * N:(i + 1) * N].astype(np.float64), d, l,
                                          nthreads=threads, index=index))
                    for i in range(ri.size // M)]
            indices[index]["vs_oracle_err_max"] = float(max(ierr))
            indices[index]["oracle_sample"] = len(ierr)
            log(f"index {index}: oracle sample err {max(ierr):.2e}")
        if forest_ctx is not None:
            fc = forest_ctx
            t0 = time.perf_counter()
            ref = [oracle.forest_value_at(S, d, *fc["forest0"], fc["x"], fc["b"]) for S in fc["samp"]]
            cpu_el = time.perf_counter() - t0
            vf = vfun
            vf["oracle_sample_exact"] = all(np.float32(g) == np.float32(r)
                                            for g, r in zip(fc["got"], ref))
            ref_bg = [oracle.forest_value_at(S, d, *fc["forest0"], fc["x"], fc["rb"])
                      for S in fc["samp"][:8]]
            vf["multi_background"]["oracle_sample_exact"] = all(
                np.float32(g) == np.float32(r) for g, r in zip(fc["got_bg"], ref_bg))
            vf["cpu_oracle"] = {"coalitions_per_s": len(fc["samp"]) / cpu_el, "cores": 1,
                                "kind": "oracle",
                                "sample": f"{len(fc['samp'])} coalitions of instance 0, "
                                          "single-coalition walk"}
            log(f"value functions: oracle samples exact {vf['oracle_sample_exact']} / "
                f"{vf['multi_background']['oracle_sample_exact']}")
    # every headline instance against the closed form of its game (path
    # products / unanimity terms): FP32 result, and the secondary elementwise
    # error over the outputs with |E| >= 1e-3 max |E|
    if errs is not None and args.closed_form:
        from concurrent.futures import ThreadPoolExecutor
        from oracle import closed_forms as CF

        def cf_ref(i):
            g = games.d20_batch_instance(i)[0]
            m_, c_ = CF.tree_mobius_sparse(g) if i % 2 == 0 else CF.planted_mobius_sparse(g)
            return CF.fsi_from_sparse_mobius(m_, c_, d, l)

        t0 = time.perf_counter()
        with ThreadPoolExecutor(max_workers=threads) as ex:
            cfr = list(ex.map(cf_ref, range(n)))
        nw = np.array([normwise(res32[i * M:(i + 1) * M], cfr[i]) for i in range(n)])
        ew = np.array([elementwise(res32[i * M:(i + 1) * M], cfr[i]) for i in range(n)])
        errs.update({"vs_closed_form_max": float(nw.max()),
                     "vs_closed_form_median": float(np.median(nw)),
                     "vs_closed_form_max_tree": float(nw[0::2].max()),
                     "vs_closed_form_max_planted": float(nw[1::2].max()),
                     "vs_closed_form_instances": n,
                     "elementwise_vs_closed_form_max": float(ew.max()),
                     "elementwise_vs_closed_form_median": float(np.median(ew)),
                     "closed_form_note": "FP64 closed form of each game; the FP32 error "
                                         "includes the rounding of the inputs to FP32"})
        log(f"closed forms of all {n} instances in {time.perf_counter() - t0:.1f}s: "
            f"normwise max {nw.max():.3e} median {np.median(nw):.3e}, elementwise max {ew.max():.3e}")
    if ragged is not None:
        rc = ragged_ctx
        t0 = time.perf_counter()

        def rag_err(i):
            v = rc["v32"][rc["voff"][i]:rc["voff"][i + 1]].astype(np.float64)
            ref = oracle.fsi_c(v, rc["ds"][i], rc["ls"][i], nthreads=1)
            return normwise(rc["out"][rc["ooff"][i]:rc["ooff"][i + 1]], ref)

        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=threads) as ex:
            rerr = np.array(list(ex.map(rag_err, range(len(rc["ds"])))))
        ragged["vs_oracle_max"] = float(rerr.max())
        ragged["vs_oracle_median"] = float(np.median(rerr))
        ragged["vs_oracle_instances"] = int(rerr.size)
        log(f"ragged batch vs oracle (all {rerr.size}): max {rerr.max():.3e} "
            f"({time.perf_counter() - t0:.1f}s)")
    if c3 is not None:
        for l3 in (2, 4):
            refs = {"tree64": oracle.fsi_c(c3_ctx["tree"], 20, l3, nthreads=threads),
                    "tree32": oracle.fsi_c(c3_ctx["tree"].astype(np.float32).astype(np.float64),
                                           20, l3, nthreads=threads),
                    "pm1": oracle.fsi_exact_int(c3_ctx["pm1"], 20, l3, nthreads=threads)}
            for vname in ("tree", "pm1"):
                for form in ("f64", "f32_fp64mob", "f32_compensated", "f32"):
                    ref = refs["pm1"] if vname == "pm1" else (
                        refs["tree64"] if form == "f64" else refs["tree32"])
                    c3[f"l{l3}_{vname}_{form}"] = normwise(c3_ctx["got"][(l3, vname, form)], ref)
        log(f"d=20 errors vs oracle: {c3}")
    cpu = None
    if args.cpu_sample > 0:
        k = min(args.cpu_sample, n)
        t0 = time.perf_counter()
        for i in range(k):
            oracle.fsi_c(vals64[i * N:(i + 1) * N], d, l, nthreads=threads)
        el = time.perf_counter() - t0
        # one instance on one core, split into the Moebius butterfly and the
        # brute-force superset sums
        v0 = vals64[:N]
        t1 = time.perf_counter()
        oracle.mobius_c(v0)
        mob_s = time.perf_counter() - t1
        t1 = time.perf_counter()
        oracle.fsi_c(v0, d, l, nthreads=1)
        one_s = time.perf_counter() - t1
        cpu = {"value": k * N / el, "unit": "coalition-values/s", "cores": threads,
               "kind": "oracle",
               "sample": f"{k} of the {n} instances (d=20, l=4, FP64 C oracle: Moebius "
                         f"butterfly + brute-force superset sums), {el:.1f} s",
               "cpu_model": cpu_model(),
               "one_core": {"instance_s": one_s, "mobius_s": mob_s,
                            "superset_sums_s": max(0.0, one_s - mob_s),
                            "values_per_s": N / one_s,
                            "what": "instance 0 on one thread: the whole oracle, its Moebius "
                                    "butterfly alone, and the difference (superset sums)"}}
        log(f"cpu oracle: {cpu['value']:.3e} values/s on {threads} threads; one core "
            f"{one_s:.2f} s per instance (Moebius {mob_s:.3f} s)")

    wkey = f"{n}x(d={d},l={l}) {args.precision} algo={args.algo} tile_bits={args.tile_bits}"
    traffic = measured_traffic(wkey)
    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "coalition-values/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batched FSI, {n} instances d={d} l={l}, FP32 storage "
                               "(even: tree-ensemble games, 200 depth-6 trees; odd: planted "
                               "games, 200 terms |A|<=6)",
                   "n_instances": n, "d": d, "l": l, "precision": args.precision,
                   "algo": args.algo, "tile_bits": args.tile_bits, "parallelism": "none"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": (traffic["fetch"] + traffic["write"]) if traffic else None,
                     "traffic_fetch": traffic["fetch"] if traffic else None,
                     "traffic_write": traffic["write"] if traffic else None,
                     "traffic_unit": "HBM bytes per launch",
                     "algorithmic_bytes": alg_bytes,
                     "kernel": f"stage {dom} of {ns}", "kernel_ms": stage_ms[dom]},
        "copy_bandwidth": {"gbs": copy_gbs, "ms": copy_ms, "bytes": 2 * alg_bytes,
                           "what": "torch copy_ of the 1 GiB FP32 input, device to device (read + write)",
                           "tile_kernel_frac_of_copy": achieved / copy_gbs},
        "stage_ms": stage_ms,
        "eager_stages_ms_per_step": eager_ms,
        "schedule": sched,
        "hbm_frac_whole_step": (alg_bytes + n * M * 4) / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "fp64": fp64,
        "speedup_vs_plain_fp64": (fp64["plain_ms_per_pass"] / ms_per_step) if fp64 else None,
        "speedup_vs_batched_fp64": (fp64["batched_ms_per_step"] / ms_per_step) if fp64 else None,
        "errors": errs,
        "precision_forms": {k: {kk: vv for kk, vv in v.items() if kk != "out"}
                            for k, v in forms.items()},
        "indices": indices,
        "value_function": vfun,
        "large_instances": large,
        "single_instance": single,
        "ragged": ragged,
        "single_d20": c3,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)
    bp32.close()


if __name__ == "__main__":
    main()
