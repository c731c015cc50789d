"""The operator at the largest sizes one MI355X holds in core (d = 26 to 30;
the paper's own method stops near d = 25 for memory). FP32 storage, and FP64
at d = 26 and 28, on the register-phase kernel (at l = 4 past d = 20 in blocks
of 2^6 tiles whose partial sums the wide gather combines).


d = 26 and 28: sampled outputs against the C oracle, which evaluates only the
requested outputs (its Moebius transform still covers all 2^d values).
d = 29 and 30 (the largest sizes of each kernel and order): the oracle's
FP64 Moebius at 4-8 GiB is too slow for a test, so the check is a property
that holds at any size: for a planted game (integer coefficients, so the
FP32 input is exact) the result equals the unanimity closed form of Eq. 3 +
Eq. 4 summed over the terms, and efficiency holds."""
import numpy as np
import pytest

import games
import oracle
import pins_lib as P
from helpers import normwise, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def integer_planted(d, n_terms, kmax, seed):
    rng = games.rng_for(930, seed)
    g = games.planted_game(d, n_terms, kmax, rng)
    g.coefs = rng.integers(-4, 5, size=n_terms).astype(np.float64)
    return g


def run(d, l, v32, precision="f32_compensated"):
    from paper_2601_01903_amd import fsi
    plan = fsi.Plan(d, l, dtype="f32", precision=precision)
    # the register-phase kernel takes every d <= 30 at l <= 4
    assert plan.schedule()["fast_instances"] == 1
    out = plan.apply(torch.from_numpy(v32).to(DEV))
    torch.cuda.synchronize()
    res = out.double().cpu().numpy()
    plan.close()
    return res


@pytest.mark.parametrize("d,l,n_sample", [(26, 3, 20), (28, 2, 10), (28, 4, 12)])
def test_large_d_sampled_outputs(d, l, n_sample):
    say(f"[case] large d={d} l={l} FP32 planted (integer coefficients)")
    g = integer_planted(d, 30, 5, d)
    v = games.planted_values(g)
    v32 = v.astype(np.float32)
    assert np.array_equal(v32.astype(np.float64), v)
    got = run(d, l, v32)
    masks = oracle.output_masks(d, l)
    rng = np.random.default_rng(d)
    pick = np.unique(np.concatenate([[0, 1, 2], rng.integers(0, masks.size, size=n_sample)]))
    W = oracle.weight_table_f64(d, l)
    # the C oracle on the picked outputs only
    ref = _oracle_subset(v, d, l, W, masks[pick])
    assert normwise(got[pick], ref) < 1e-6
    assert abs(got.sum() - v[-1]) < 1e-4 * max(1.0, np.abs(got).max())


def _oracle_subset(v, d, l, W, masks):
    import ctypes
    lib = oracle._load()
    vv = np.ascontiguousarray(v, dtype=np.float64)
    m = np.ascontiguousarray(masks, dtype=np.int64)
    E = np.empty(m.size)
    dp, ip = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)
    Wc = np.ascontiguousarray(W)
    rc = lib.oracle_fsi(vv.ctypes.data_as(dp), d, l, Wc.ctypes.data_as(dp),
                        m.ctypes.data_as(ip), m.size, E.ctypes.data_as(dp), 16)
    assert rc == 0
    return E


_PLANTED32 = {}


def _planted32(d):
    """FP32 values of the integer planted game at d (exact in FP32), kept
    for the orders tested at the same d."""
    if d not in _PLANTED32:
        _PLANTED32.clear()
        g = integer_planted(d, 16, 6, d)
        _PLANTED32[d] = (g, games.planted_values(g).astype(np.float32))
    return _PLANTED32[d]


@pytest.mark.parametrize("d,l", [(29, 4), (30, 2), (30, 3), (30, 4)])
def test_max_d_planted_closed_form(d, l):
    """The largest instances: d = 29 and 30 at l = 4 (register-phase kernel,
    2^12 and 2^13 blocks of 2^6 tiles), d = 30 at l = 2, 3 (register-phase
    kernel, the whole instance one block)."""
    say(f"[case] large d={d} l={l} FP32 planted, closed form")
    g, v32 = _planted32(d)
    got = run(d, l, v32)
    want = P.fsi_sparse_mobius(zip(g.masks, g.coefs), d, l)
    assert normwise(got, want) < 1e-6
    assert abs(got[0]) == 0.0                          # v(empty) = 0 for a planted game
    assert abs(got.sum() - g.coefs.sum()) < 1e-4 * max(1.0, np.abs(got).max())


@pytest.mark.parametrize("d,l,tb,dtype,prec", [(18, 3, 8, "f64", "f64"),
                                               (16, 4, 6, "f32", "f32_compensated"),
                                               (22, 4, 0, "f32", "f32_compensated")])
def test_wide_gather_matches_oracle(d, l, tb, dtype, prec):
    """Generic instances with at least 2^10 tiles sum their per-tile results
    with the wide gather (tile ranges x output groups); every output against
    the oracle, and two applies bitwise equal."""
    from paper_2601_01903_amd import fsi
    say(f"[case] wide gather d={d} l={l} tile_bits={tb} {prec}")
    g = games.tree_game(d, 60, 5, games.rng_for(931, d))
    v = games.tree_values(g)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    vin = v if dtype == "f64" else v.astype(np.float32).astype(np.float64)
    plan = fsi.Plan(d, l, dtype=dtype, precision=prec, kernel="generic", tile_bits=tb)
    assert d - plan.info()["tile_bits"] >= 10
    x = torch.as_tensor(vin, dtype=tdt).to(DEV)
    o1 = plan.apply(x).double().cpu().numpy()
    o2 = plan.apply(x).double().cpu().numpy()
    torch.cuda.synchronize()
    plan.close()
    assert np.array_equal(o1, o2)
    ref = oracle.fsi_c(vin, d, l, nthreads=16)
    assert normwise(o1, ref) < (1e-12 if dtype == "f64" else 1e-6)


def test_wide_gather_in_a_mixed_batch():
    from paper_2601_01903_amd import fsi
    ds, ls = [20, 22, 12, 19], [4, 4, 2, 1]
    say(f"[case] mixed batch with a wide instance {list(zip(ds, ls))}")
    vals = [games.tree_values(games.tree_game(d, 40, 5, games.rng_for(932, i))).astype(np.float32)
            for i, d in enumerate(ds)]
    bp = fsi.BatchPlan(ds, ls, dtype="f32", kernel="generic")
    out = bp.apply(torch.from_numpy(np.concatenate(vals)).to(DEV), graph=True)
    torch.cuda.synchronize()
    o = out.double().cpu().numpy()
    for i, (v, d, l) in enumerate(zip(vals, ds, ls)):
        ref = oracle.fsi_c(v.astype(np.float64), d, l, nthreads=16)
        assert normwise(o[bp.out_offset[i]:bp.out_offset[i + 1]], ref) < 1e-6, (i, d, l)
    bp.close()


def test_blocked_register_kernel_in_a_batch():
    """A batch that mixes register-phase instances of several blocks (d = 21,
    22 at l = 4: blocks of 2^6 tiles, reduced by the wide gather), a one-block
    instance (d = 20, l = 4), register-phase instances at d = 9 (run as
    d = 11) and d = 13, and a generic one (l = 5): FP64 integer input against
    the exact oracle at 1e-12, two graph replays with eager work between them
    bitwise equal to the eager apply."""
    from paper_2601_01903_amd import fsi
    ds, ls = [21, 20, 22, 9, 13, 12], [4, 4, 4, 3, 2, 5]
    say(f"[case] blocked register kernel in a batch {list(zip(ds, ls))}")
    vals = [np.random.default_rng(933 + i).integers(-3, 4, size=1 << d).astype(np.float64)
            for i, d in enumerate(ds)]
    x = torch.from_numpy(np.concatenate(vals)).to(DEV)
    bp = fsi.BatchPlan(ds, ls, dtype="f64", precision="f64")
    assert bp.schedule()["fast_instances"] == 5
    eager = bp.apply(x, graph=False).cpu().numpy()
    reps = []
    for _ in range(2):
        reps.append(bp.apply(x, graph=True).cpu().numpy())
        torch.cuda.synchronize()
        (x * 2.0).sum().item()      # eager work between the replays
    for r in reps:
        assert np.array_equal(r, eager)
    for i, (v, d, l) in enumerate(zip(vals, ds, ls)):
        ref = oracle.fsi_exact_int(v, d, l, nthreads=16)
        assert normwise(eager[bp.out_offset[i]:bp.out_offset[i + 1]], ref) < 1e-12, (i, d, l)
    bp.close()


@pytest.mark.parametrize("d,l", [(26, 4), (28, 3)])
def test_large_d_fp64_planted_closed_form(d, l):
    """FP64 storage at large d on the register-phase kernel (d = 26, l = 4 in
    blocks of 2^6 tiles; d = 28, l = 3 one block) on a planted game with
    N(0, 1) coefficients: the unanimity closed form of Eq. 3 + Eq. 4 summed
    over the terms, 1e-12 normwise, and efficiency."""
    from paper_2601_01903_amd import fsi
    say(f"[case] large d={d} l={l} FP64 planted, closed form")
    g = games.planted_game(d, 24, 6, games.rng_for(931, d))
    v = games.planted_values(g)
    plan = fsi.Plan(d, l, dtype="f64")
    assert plan.schedule()["fast_instances"] == 1
    out = plan.apply(torch.from_numpy(v).to(DEV))
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    plan.close()
    del out
    want = P.fsi_sparse_mobius(zip(g.masks, g.coefs), d, l)
    assert normwise(got, want) < 1e-12
    assert abs(got.sum() - v[-1]) < 1e-12 * max(1.0, np.abs(got).sum())
