"""The operator at the largest sizes one MI355X holds in core (d = 26, 28, 30;
the paper's own method stops near d = 25 for memory). FP32 storage, generic
tile kernel (the register-phase kernel stops at d = 23).

d = 26 and 28: sampled outputs against the C oracle, which evaluates only the
requested outputs (its Moebius transform still covers all 2^d values).
d = 30: the oracle's 8 GiB FP64 Moebius is too slow for a test, so the check
is a property that holds at any size: for a planted game (integer
coefficients, so the FP32 input is exact) the result equals the unanimity
closed form of Eq. 3 + Eq. 4 summed over the terms, and efficiency holds."""
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
    out = plan.apply(torch.from_numpy(v32).to(DEV))
    torch.cuda.synchronize()
    res = out.double().cpu().numpy()
    plan.close()
    return res


@pytest.mark.parametrize("d,l,n_sample", [(26, 3, 20), (28, 2, 10)])
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


def test_d30_planted_closed_form():
    d, l = 30, 2
    say(f"[case] large d={d} l={l} FP32 planted, closed form")
    g = integer_planted(d, 16, 6, 30)
    v32 = games.planted_values(g).astype(np.float32)
    got = run(d, l, v32)
    want = P.fsi_sparse_mobius(zip(g.masks, g.coefs), d, l)
    assert normwise(got, want) < 1e-6
    assert abs(got[0]) == 0.0                          # v(empty) = 0 for a planted game
    assert abs(got.sum() - g.coefs.sum()) < 1e-4 * max(1.0, np.abs(got).max())
