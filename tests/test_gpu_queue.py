"""The register-phase kernel's work queue. Past the first round of work items
the workgroups claim items from a counter in the plan's tables, and the last
workgroup of a launch resets it for the next launch. Two batches with more
work items than workgroups run through each entry point in turn: graph
replays, direct launches, stage by stage, and the no-allocation scratch.
Their inputs alternate between x and 2x. Scaling by 2 is exact in FP32 and
FP64, so every output for 2x is bitwise twice the one for x. A launch that
skipped items would keep stale partial sums from the other input and miss
that. The first results are also checked against the oracle on the same FP32
values widened to FP64, at 1e-6 normwise."""
import numpy as np
import pytest

import games
import oracle
from helpers import normwise, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"

# one order (l = 3, d from 9 to 20) and four orders on the same shapes:
# 8624 tiles, cut by the default schedule into more work items than the
# workgroups of the grid (asserted below)
_DS = [20] * 16 + [12, 19, 11, 16, 14, 9, 18, 13]
CASES = {
    "one_order": (_DS, [3] * len(_DS)),
    "four_orders": (_DS, [(i % 4) + 1 for i in range(len(_DS))]),
}


def fsi_mod():
    from paper_2601_01903_amd import fsi
    return fsi


def _inputs(ds, seed):
    vals = [games.tree_values(games.tree_game(d, 40, 5, games.rng_for(seed, i))).astype(np.float32)
            for i, d in enumerate(ds)]
    return vals, torch.from_numpy(np.concatenate(vals)).to(DEV)


def _runs(bp, x, n_stages):
    """The entry points in turn, alternating x and 2x; returns (scale, out)."""
    res = []
    for k, how in enumerate(["graph", "direct", "stages", "noalloc", "graph", "direct", "graph"]):
        s = 2.0 if k % 2 else 1.0
        xi = x * s
        if how == "graph":
            o = bp.apply(xi, graph=True)
        elif how == "direct":
            o = bp.apply(xi, graph=False)
        elif how == "stages":
            o = torch.empty(bp.out_offset[-1], dtype=torch.float32, device=DEV)
            for st in range(n_stages):
                bp.apply_stage(xi, o, st)
        else:
            o = torch.empty(bp.out_offset[-1], dtype=torch.float32, device=DEV)
            bp.apply_noalloc(xi, o)
        torch.cuda.synchronize()
        res.append((s, o.clone()))
    return res


def test_work_queue_across_launches():
    fsi = fsi_mod()
    plans, base = {}, {}
    for name, (ds, ls) in CASES.items():
        vals, x = _inputs(ds, 960 + len(plans))
        bp = fsi.BatchPlan(ds, ls, dtype="f32")
        sch = bp.schedule()
        tpi = sch["tiles_per_item"]
        tiles = [1 << max(d - 11, 0) for d in ds]
        items = sum(-(-t // tpi) for t in tiles)
        say(f"[case] work queue {name}: {len(ds)} instances, {sum(tiles)} tiles, "
            f"{tpi} tile(s) per item, {items} items, {bp.num_stages()} stages")
        assert sch["fast_instances"] == len(ds)
        # more work items than the grid's workgroups (two per CU): the queue
        # is used
        assert items > 2 * torch.cuda.get_device_properties(0).multi_processor_count
        plans[name] = (bp, vals, x, ds, ls)
    # interleave the two plans' launch sequences
    runs = {name: [] for name in plans}
    for rep in range(2):
        for name, (bp, vals, x, ds, ls) in plans.items():
            runs[name] += _runs(bp, x, bp.num_stages())
    for name, (bp, vals, x, ds, ls) in plans.items():
        first = runs[name][0][1]
        for s, o in runs[name]:
            assert torch.equal(o, first * s), (name, s)
        o = first.double().cpu().numpy()
        for i, (v, d, l) in enumerate(zip(vals, ds, ls)):
            ref = oracle.fsi_c(v.astype(np.float64), d, l, nthreads=16)
            assert normwise(o[bp.out_offset[i]:bp.out_offset[i + 1]], ref) < 1e-6, (name, i, d, l)
        say(f"  {name}: {len(runs[name])} launches bitwise consistent, oracle ok")
        bp.close()
