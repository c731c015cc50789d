"""GPU parity of the tree-ensemble value function (include/fsi_forest.h)
against the CPU oracle (oracle/forest.py).

Leaf selection is decided by exact FP64 comparisons on both sides and the
leaf outputs are summed in the same order (backgrounds outer, trees inner,
ascending), so the FP64 output of the walk must equal the oracle bit for bit and the FP32
output must equal the oracle's value rounded once to FP32. The Moebius route
sums +-leaf terms with FP64 atomics and then subset sums, so it is checked to
1e-12 of max |v| (FP64) and 2e-7 (FP32 output)."""
import ctypes

import numpy as np
import pytest

import games
import oracle
from helpers import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def fsi_mod():
    from paper_2601_01903_amd import fsi
    return fsi


def heap_forest(g):
    n_int = (1 << g.depth) - 1
    n_tree = n_int + (1 << g.depth)
    K = g.feat.shape[0]
    feature = np.full(K * n_tree, -1, dtype=np.int32)
    threshold = np.zeros(K * n_tree)
    left = np.zeros(K * n_tree, dtype=np.int32)
    right = np.zeros(K * n_tree, dtype=np.int32)
    value = np.zeros(K * n_tree)
    for k in range(K):
        o = k * n_tree
        idx = np.arange(n_int)
        feature[o:o + n_int] = g.feat[k]
        threshold[o:o + n_int] = g.thr[k]
        left[o:o + n_int] = o + 2 * idx + 1
        right[o:o + n_int] = o + 2 * idx + 2
        value[o + n_int:o + n_tree] = g.leaf[k]
    return np.arange(K, dtype=np.int32) * n_tree, feature, threshold, left, right, value


def random_forest(d, n_trees, max_depth, rng, x=None, bgs=None):
    """Irregular trees: a node splits with probability 0.8 while above
    max_depth; some thresholds equal an x or background value (ties)."""
    feature, threshold, left, right, value = [], [], [], [], []

    def node(depth):
        i = len(feature)
        feature.append(-1); threshold.append(0.0); left.append(0); right.append(0)
        value.append(float(rng.standard_normal()))
        if depth < max_depth and rng.uniform() < 0.8:
            f = int(rng.integers(0, d))
            th = float(rng.uniform())
            u = rng.uniform()
            if x is not None and u < 0.1:
                th = float(x[f])
            elif bgs is not None and u < 0.2:
                th = float(bgs[int(rng.integers(0, len(bgs)))][f])
            feature[i], threshold[i] = f, th
            li = node(depth + 1)
            ri = node(depth + 1)
            left[i], right[i] = li, ri
        return i

    roots = [node(0) for _ in range(n_trees)]
    return (np.array(roots, np.int32), np.array(feature, np.int32), np.array(threshold),
            np.array(left, np.int32), np.array(right, np.int32), np.array(value))


def gpu_values(d, forest, x, bgs, dtype="f64", max_bg=None):
    fsi = fsi_mod()
    bgs = np.atleast_2d(bgs)
    F = fsi.Forest(d, *forest, max_bg=max_bg or bgs.shape[0])
    out = F.values(torch.as_tensor(np.asarray(x, dtype=np.float64)).to(DEV),
                   torch.as_tensor(np.ascontiguousarray(bgs, dtype=np.float64)).to(DEV),
                   dtype=dtype)
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    F.close()
    return res


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("d,K,depth", [(8, 10, 4), (14, 50, 4), (12, 30, 6)])
def test_heap_forest_bitwise(d, K, depth, dtype):
    say(f"[case] forest heap d={d} K={K} depth={depth} {dtype}")
    g = games.tree_game(d, K, depth, games.rng_for(910, d))
    forest = heap_forest(g)
    want = oracle.forest_values(d, *forest, g.x, g.b[None, :])
    got = gpu_values(d, forest, g.x, g.b, dtype)
    if dtype == "f64":
        assert np.array_equal(got, want)
    else:
        assert np.array_equal(got, want.astype(np.float32))


@pytest.mark.parametrize("n_bg", [1, 5, 32, 40, 77])
def test_irregular_trees_many_backgrounds(n_bg):
    d = 11
    rng = np.random.default_rng(911 + n_bg)
    x = rng.uniform(size=d)
    bgs = rng.uniform(size=(n_bg, d))
    forest = random_forest(d, 25, 9, rng, x, bgs)
    say(f"[case] forest irregular d={d} nodes={forest[1].size} n_bg={n_bg}")
    want = oracle.forest_values(d, *forest, x, bgs)
    got = gpu_values(d, forest, x, bgs, "f64", max_bg=n_bg + 3)
    assert np.array_equal(got, want)


def test_d20_full_size_sampled():
    """200 depth-6 trees on 20 features (the d = 20 tree game): sampled
    coalitions against the oracle's single-coalition walk, and every
    coalition against the seeded C generator."""
    say("[case] forest d=20 200 depth-6 trees")
    g, vgen = games.d20_tree(0)
    forest = heap_forest(g)
    got = gpu_values(20, forest, g.x, g.b, "f64")
    rng = np.random.default_rng(912)
    for S in list(rng.integers(0, 1 << 20, size=64)) + [0, (1 << 20) - 1]:
        assert got[S] == oracle.forest_value_at(int(S), 20, *forest, g.x, g.b[None, :]), S
    assert np.max(np.abs(got - vgen)) < 1e-12


def test_edge_forests():
    say("[case] forest edges: d=1, leaf-only tree, shared nodes, d=24")
    # d = 1, a root that is a leaf plus a stump
    forest = (np.array([0, 1], np.int32), np.array([-1, 0, -1, -1], np.int32),
              np.array([0, 0.5, 0, 0]), np.array([0, 2, 0, 0], np.int32),
              np.array([0, 3, 0, 0], np.int32), np.array([1.5, 0, -1.0, 2.0]))
    got = gpu_values(1, forest, [0.9], [[0.1]])
    assert got.tolist() == [1.5 - 1.0, 1.5 + 2.0]
    # two trees sharing a subtree
    d = 6
    rng = np.random.default_rng(913)
    x, bg = rng.uniform(size=d), rng.uniform(size=(2, d))
    feature = np.array([0, 1, -1, -1, 2], np.int32)
    threshold = np.array([0.5, 0.5, 0, 0, 0.3])
    left = np.array([1, 2, 0, 0, 1], np.int32)
    right = np.array([4, 3, 0, 0, 3], np.int32)
    value = np.array([0, 0, 1.0, 2.0, 0])
    forest = (np.array([0, 4], np.int32), feature, threshold, left, right, value)
    assert np.array_equal(gpu_values(d, forest, x, bg), oracle.forest_values(d, *forest, x, bg))
    # d = 24: 16M coalitions, sampled
    d = 24
    x, bg = rng.uniform(size=d), rng.uniform(size=(3, d))
    forest = random_forest(d, 6, 7, rng, x, bg)
    got = gpu_values(d, forest, x, bg, "f32")
    for S in rng.integers(0, 1 << d, size=48):
        assert got[S] == np.float32(oracle.forest_value_at(int(S), d, *forest, x, bg)), S


def test_forest_then_fsi_matches_oracle_chain():
    """The value function generated on the GPU feeds the FSI operator; the
    chain equals the oracle's chain (oracle value function, oracle FSI)."""
    fsi = fsi_mod()
    d, l = 14, 3
    g = games.tree_game(d, 50, 4, games.rng_for(914, 0))
    forest = heap_forest(g)
    rng = np.random.default_rng(914)
    bgs = rng.uniform(size=(4, d))
    say("[case] forest -> FSI chain d=14 l=3, 4 backgrounds")
    F = fsi.Forest(d, *forest, max_bg=4)
    v = F.values(torch.as_tensor(g.x).to(DEV), torch.as_tensor(bgs).to(DEV), dtype="f32")
    plan = fsi.Plan(d, l, dtype="f32")
    E = plan.apply(v)
    torch.cuda.synchronize()
    want_v = oracle.forest_values(d, *forest, g.x, bgs)
    ref = oracle.fsi(want_v.astype(np.float32).astype(np.float64), d, l)
    err = np.max(np.abs(E.double().cpu().numpy() - ref)) / np.max(np.abs(ref))
    assert err < 1e-6
    F.close()
    plan.close()


def test_forest_errors_on_device():
    fsi = fsi_mod()
    g = games.tree_game(6, 3, 3, games.rng_for(915, 0))
    F = fsi.Forest(6, *heap_forest(g), max_bg=2)
    x = torch.zeros(6, dtype=torch.float64, device=DEV)
    bg3 = torch.zeros(3, 6, dtype=torch.float64, device=DEV)
    with pytest.raises(fsi.FsiError):
        F.values(x, bg3)                        # more backgrounds than max_bg
    v = torch.empty(65, dtype=torch.float64, device=DEV)
    lib = fsi.load()
    st = lib.fsi_forest_values(F._h, ctypes.c_void_p(x.data_ptr()), 1,
                               ctypes.c_void_p(bg3.data_ptr()), 0,
                               ctypes.c_void_p(v.data_ptr() + 8), None)
    assert st == 1                              # misaligned output
    st = lib.fsi_forest_values(F._h, ctypes.c_void_p(x.data_ptr()), 1,
                               ctypes.c_void_p(bg3.data_ptr()), 7,
                               ctypes.c_void_p(v.data_ptr()), None)
    assert st == 1                              # unknown dtype
    F.close()


def gpu_mobius_route(d, forest, x, bgs, dtype="f64"):
    fsi = fsi_mod()
    bgs = np.atleast_2d(bgs)
    F = fsi.Forest(d, *forest, max_bg=bgs.shape[0])
    xt = torch.as_tensor(np.asarray(x, dtype=np.float64)).to(DEV)
    bt = torch.as_tensor(np.ascontiguousarray(bgs, dtype=np.float64)).to(DEV)
    a = F.mobius(xt, bt)
    v = F.values(xt, bt, dtype=dtype, method="mobius")
    torch.cuda.synchronize()
    res = a.cpu().numpy(), v.cpu().numpy()
    F.close()
    return res


@pytest.mark.parametrize("case", ["heap8", "heap14", "irregular11_bg5", "irregular12_bg40"])
def test_mobius_route_matches_oracle(case):
    say(f"[case] forest Moebius route {case}")
    if case.startswith("heap"):
        d = int(case[4:])
        g = games.tree_game(d, 40, 5, games.rng_for(916, d))
        forest, x, bgs = heap_forest(g), g.x, g.b[None, :]
    else:
        d, nb = (11, 5) if case.endswith("bg5") else (12, 40)
        rng = np.random.default_rng(917 + d)
        x, bgs = rng.uniform(size=d), rng.uniform(size=(nb, d))
        forest = random_forest(d, 20, 7, rng, x, bgs)
    v_ref = oracle.forest_values(d, *forest, x, bgs)
    a_ref = oracle.mobius(v_ref)
    scale = max(1.0, np.abs(v_ref).max())
    a, v = gpu_mobius_route(d, forest, x, bgs)
    assert np.max(np.abs(a - a_ref)) < 1e-12 * scale
    assert np.max(np.abs(v - v_ref)) < 1e-12 * scale
    _, v32 = gpu_mobius_route(d, forest, x, bgs, "f32")
    assert np.max(np.abs(v32 - v_ref)) < 2e-7 * scale


def test_mobius_route_d20_full_size():
    say("[case] forest Moebius route d=20 200 depth-6 trees")
    g, vgen = games.d20_tree(0)
    forest = heap_forest(g)
    a, v = gpu_mobius_route(20, forest, g.x, g.b)
    scale = np.abs(vgen).max()
    assert np.max(np.abs(v - vgen)) < 1e-12 * scale
    rng = np.random.default_rng(918)
    for S in rng.integers(0, 1 << 20, size=32):
        assert abs(v[S] - oracle.forest_value_at(int(S), 20, *forest, g.x, g.b[None, :])) < 1e-12 * scale
    # the Moebius coefficients of a tree game sit on sets of at most depth features
    support = np.nonzero(np.abs(a) > 1e-12 * scale)[0]
    assert max(bin(int(m)).count("1") for m in support) <= 6


def test_mobius_route_refuses_long_paths():
    fsi = fsi_mod()
    d, k = 26, 25                               # one chain of 25 splits on 26 features
    feature = np.array(list(range(k)) + [-1, -1], np.int32)
    threshold = np.full(k + 2, 0.5)
    left = np.array([k + 1] * k + [0, 0], np.int32)
    right = np.array(list(range(1, k)) + [k, 0, 0], np.int32)
    value = np.zeros(k + 2)
    F = fsi.Forest(d, np.array([0], np.int32), feature, threshold, left, right, value)
    x = torch.zeros(d, dtype=torch.float64, device=DEV)
    bg = torch.zeros(1, d, dtype=torch.float64, device=DEV)
    a = torch.zeros(16, dtype=torch.float64, device=DEV)
    st = fsi.load().fsi_forest_mobius(F._h, ctypes.c_void_p(x.data_ptr()), 1,
                                      ctypes.c_void_p(bg.data_ptr()),
                                      ctypes.c_void_p(a.data_ptr()), None)
    assert st == 2                              # FSI_ERR_UNSUPPORTED, nothing launched
    F.close()
