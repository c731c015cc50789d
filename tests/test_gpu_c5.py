"""The headline workload at full size, every instance against a closed form.

256 instances at d = 20, l = 4 (1 GiB of FP32 values), built exactly as
bench.py builds them: even instances tree-ensemble games (200 depth-6 trees),
odd instances planted games (200 terms, |A| <= 6). The reference of each
instance is the closed form of its FP64 game (oracle/closed_forms.py: path
products for trees, unanimity games and linearity for planted games), so the
FP32 error below includes the rounding of the inputs to FP32 (1e-8 to 1e-7
normwise on its own). Tolerances: FP32-storage forms <= 1e-6 normwise per
instance, the FP64 path <= 1e-12.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import games
from helpers import elementwise, normwise, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N, D, L = 256, 20, 4
_CACHE = {}


def _workload():
    if "w" not in _CACHE:
        from oracle import closed_forms as CF
        built = games.build_many(games.d20_batch_instance, range(N), threads=16)

        def ref(i):
            g = built[i][0]
            m, c = CF.tree_mobius_sparse(g) if i % 2 == 0 else CF.planted_mobius_sparse(g)
            return CF.fsi_from_sparse_mobius(m, c, D, L)

        with ThreadPoolExecutor(max_workers=16) as ex:
            refs = list(ex.map(ref, range(N)))
        vals = np.concatenate([v for _, v in built])
        _CACHE["w"] = (vals, refs)
    return _CACHE["w"]


def _errors(out, refs, M):
    o = out.double().cpu().numpy().reshape(N, M)
    nw = np.array([normwise(o[i], refs[i]) for i in range(N)])
    ew = np.array([elementwise(o[i], refs[i]) for i in range(N)])
    return nw, ew


@pytest.mark.parametrize("prec,autotune", [("auto", True), ("f32_compensated", False),
                                           ("f32", False)])
def test_c5_fp32_every_instance_vs_closed_form(prec, autotune):
    from paper_2601_01903_amd import BatchPlan
    vals, refs = _workload()
    say(f"[case] 256 x (d=20, l=4) FP32 prec={prec} autotune={autotune}")
    bp = BatchPlan([D] * N, [L] * N, dtype="f32", precision=prec, autotune=autotune)
    x = torch.from_numpy(vals.astype(np.float32)).cuda()
    out = bp.apply(x, graph=True)
    torch.cuda.synchronize()
    M = bp.out_offset[1]
    nw, ew = _errors(out, refs, M)
    say(f"  normwise max {nw.max():.3e} median {np.median(nw):.3e} "
        f"(tree max {nw[0::2].max():.3e}, planted max {nw[1::2].max():.3e}); "
        f"elementwise max {ew.max():.3e} (reported)")
    bp.close()
    assert np.all(nw <= 1e-6), int(np.argmax(nw))


def test_c5_fp64_every_instance_vs_closed_form():
    from paper_2601_01903_amd import BatchPlan
    vals, refs = _workload()
    say("[case] 256 x (d=20, l=4) FP64")
    bp = BatchPlan([D] * N, [L] * N, dtype="f64")
    x = torch.from_numpy(vals).cuda()
    out = bp.apply(x, graph=True)
    torch.cuda.synchronize()
    nw, _ = _errors(out, refs, bp.out_offset[1])
    say(f"  normwise max {nw.max():.3e} median {np.median(nw):.3e}")
    bp.close()
    del x, out
    assert np.all(nw <= 1e-12), int(np.argmax(nw))
