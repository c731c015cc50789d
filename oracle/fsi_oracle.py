"""Plain FP64 CPU oracle for the Faithful Shapley Interaction (FSI) operator.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import this module:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it. It shares no code with the HIP implementation.

What it computes (paper, Sec. 2.2 "Closed-Form Solution", Eq. 3 and Eq. 4;
weight function of Sec. 4.3, Eq. 7):

    E_S = a(S) + sum_{T superset of S, |T| > l} w(|S|, |T|) * a(T),   |S| <= l,

where a is the Moebius transform of the value vector v
(a(S) = sum_{T subset of S} (-1)^{|S|-|T|} v(T)), and

    w(s, t) = (-1)^{l-s} * s/(l+s) * C(l, s) * C(t-1, l) / C(t+l-1, l+s).

The method here is the paper's "Baseline" (Sec. 4.6, time complexity
paragraph): a direct Moebius butterfly followed by brute-force superset sums
over every (S, T) pair with T a superset of S and |S| <= l. Weights are exact
rationals (``fractions.Fraction``) rounded once to FP64; the paper's log-gamma
route (Sec. 4.3, "Numerical Stability") is replaced by exact evaluation.

Conventions:
  * v has 2^d entries indexed by a d-bit mask; bit i set <=> feature i in S.
  * Outputs are in canonical order: ascending |S|, then ascending mask value.
  * v(empty) need not be 0: the formula is applied as written, so
    E_empty = v(empty) (w(0, t) = 0 because of its factor s).

Every function here is parity-pinned by ``tests/test_oracle_pins.py`` against
definitions that do not reuse this module's arithmetic (the weighted least
squares definition of Eq. 2, Eq. 1 Shapley values, unanimity games, tree-game
path products, exact integer evaluation, and a worked example).
"""
from __future__ import annotations

from fractions import Fraction
from math import comb

import numpy as np

__all__ = [
    "weight_exact",
    "weight_table_f64",
    "mobius",
    "mobius_direct",
    "output_masks",
    "num_outputs",
    "superset_masks",
    "fsi",
    "fsi_batch",
    "INDICES",
    "bernoulli_exact",
    "index_weight_exact",
    "index_weight_table_f64",
    "interaction",
    "interaction_from_mobius",
]


def weight_exact(s: int, t: int, l: int) -> Fraction:
    """Exact correction weight w(s, t) of Eq. 7 (equivalently the coefficient
    of a(v, T) in Eq. 4 with |S| = s and |T| = t)."""
    if not (0 <= s <= l) or t < 1:
        raise ValueError("weight_exact needs 0 <= s <= l and t >= 1")
    sign = -1 if (l - s) % 2 else 1
    return (sign * Fraction(s, l + s) * comb(l, s)
            * Fraction(comb(t - 1, l), comb(t + l - 1, l + s)))


def weight_table_f64(d: int, l: int) -> np.ndarray:
    """Table W[s, t] (shape (l+1, d+1)) of the weight that multiplies a(T) in
    E_S, for |S| = s and |T| = t with T a superset of S:
      * 1 when t == s (the Moebius term a(S) itself, Eq. 3),
      * w(s, t) of Eq. 7 when t > l and s >= 1 (Eq. 4 sums only |T| > l),
      * 0 otherwise.
    Each entry is an exact rational rounded once to FP64."""
    W = np.zeros((l + 1, d + 1), dtype=np.float64)
    for s in range(0, l + 1):
        if s <= d:
            W[s, s] = 1.0
        if s == 0:
            continue
        for t in range(l + 1, d + 1):
            W[s, t] = float(weight_exact(s, t, l))
    return W


def mobius(v: np.ndarray) -> np.ndarray:
    """Moebius transform a = mu_down v (Sec. 4.2 and Appendix B: mu_down is the
    Kronecker product of the 2x2 factors [[1, 0], [-1, 1]]), applied one bit
    axis at a time: for every mask m with bit i set, a[m] -= a[m without i]."""
    a = np.array(v, dtype=np.float64, copy=True)
    n = a.size
    d = n.bit_length() - 1
    if n != 1 << d:
        raise ValueError("length of v must be a power of two")
    for i in range(d):
        view = a.reshape(-1, 2, 1 << i)
        view[:, 1, :] -= view[:, 0, :]
    return a


def mobius_direct(v: np.ndarray) -> np.ndarray:
    """The definition of a(v, S) (Sec. 2.2, below Eq. 3) summed term by term:
    a(S) = sum over T subset of S of (-1)^{|S|-|T|} v(T). O(3^d); small d only."""
    v = np.asarray(v, dtype=np.float64)
    n = v.size
    a = np.zeros(n, dtype=np.float64)
    for S in range(n):
        acc = 0.0
        T = S
        while True:
            sign = -1.0 if (bin(S).count("1") - bin(T).count("1")) % 2 else 1.0
            acc += sign * v[T]
            if T == 0:
                break
            T = (T - 1) & S
        a[S] = acc
    return a


def num_outputs(d: int, l: int) -> int:
    """M(d, l) = number of subsets S of [d] with |S| <= l (S = empty included)."""
    return sum(comb(d, s) for s in range(0, min(l, d) + 1))


def output_masks(d: int, l: int) -> np.ndarray:
    """All masks S with popcount(S) <= l in canonical order: ascending
    popcount, then ascending mask value."""
    masks = np.arange(1 << d, dtype=np.int64)
    pc = np.array([bin(int(m)).count("1") for m in masks]) if d <= 12 else _popcount(masks)
    keep = pc <= l
    m = masks[keep]
    p = pc[keep]
    order = np.lexsort((m, p))
    return m[order]


def _popcount(x: np.ndarray) -> np.ndarray:
    x = x.astype(np.int64)
    c = np.zeros_like(x)
    while np.any(x):
        c += x & 1
        x = x >> 1
    return c


def superset_masks(S: int, d: int) -> np.ndarray:
    """All T with S subset of T subset of [d], in ascending mask order."""
    free = [i for i in range(d) if not (S >> i) & 1]
    idx = np.arange(1 << len(free), dtype=np.int64)
    T = np.full(idx.shape, S, dtype=np.int64)
    for j, bit in enumerate(free):
        T |= ((idx >> j) & 1) << bit
    return T


def fsi(v: np.ndarray, d: int, l: int) -> np.ndarray:
    """FSI scores E_S for all |S| <= l (canonical order), FP64.

    Step 1: a = Moebius(v) (Eq. 5, first term).
    Step 2: for every output S, brute-force sum over all supersets T of
            W[|S|, |T|] * a(T) (Eq. 3 + Eq. 4), the paper's Baseline.
    """
    if not (1 <= l <= d):
        raise ValueError("need 1 <= l <= d")
    return _superset_weighted(v, d, l, weight_table_f64(d, l))


def _superset_weighted(v, d: int, l: int, W: np.ndarray, transform: bool = True) -> np.ndarray:
    """E_S = sum over supersets T of S of W[|S|, |T|] * a(T), a = Moebius(v)
    (or a = v when transform is False), for every |S| <= l in canonical order
    (brute force over (S, T) pairs)."""
    v = np.asarray(v, dtype=np.float64)
    if v.size != 1 << d:
        raise ValueError("v must have 2^d entries")
    a = mobius(v) if transform else v
    out_masks = output_masks(d, l)
    out = np.empty(out_masks.size, dtype=np.float64)
    pc_cache = _popcount(np.arange(1 << d, dtype=np.int64))
    for k, S in enumerate(out_masks):
        S = int(S)
        s = int(pc_cache[S])
        T = superset_masks(S, d)
        wt = W[s, pc_cache[T]]
        out[k] = float(np.dot(wt, a[T]))
    return out


def fsi_batch(values, ds, ls):
    """Per-instance ``fsi`` over a list of value vectors."""
    return [fsi(v, d, l) for v, d, l in zip(values, ds, ls)]


# ---------------------------------------------------------------------------
# Other cardinal interaction indices (Appendix A: SII, k-SII, STII, BII).
#
# Each is linear in v and, written on the Moebius transform, gives every
# superset T of S a weight that depends only on s = |S| and t = |T|:
#     I_S = sum_{T superset of S} W_index(s, t) * a(T),   |S| <= l,
# which is the same shape as FSI's closed form, so the same superset sums
# compute them. The Moebius-side weights used here:
#   sii   1 / (t - s + 1)                (SII's discrete-derivative weights
#                                         of Appendix A, summed over supersets)
#   bii   2^-(t - s)                      (uniform weights over the complement)
#   stii  [t == s] for s < l;  1 / C(t, l) for s == l
#         (top order receives every higher Moebius coefficient split evenly
#          over its l-subsets; lower orders are the Moebius coefficients)
#   ksii  [t == 0] for s == 0; for s >= 1
#         sum_{j=0}^{min(l-s, t-s)} B_j C(t-s, j) / (t-s-j+1)
#         with the Bernoulli numbers B_j (B_1 = -1/2): the SII of S plus the
#         Bernoulli-weighted SII of its supersets up to order l
#   fsi   the weights of Eq. 3, 4 and 7 (``weight_table_f64``)
# For S = empty, FSI, STII and k-SII give v(empty) (a Moebius coefficient);
# SII and BII follow their own definitions (Delta_empty v(T) = v(T)).
# ---------------------------------------------------------------------------

INDICES = ("fsi", "stii", "sii", "ksii", "bii")


def bernoulli_exact(n: int):
    """Bernoulli numbers B_0 .. B_n as Fractions from the recurrence
    sum_{j=0}^{m} C(m+1, j) B_j = 0 for m >= 1, B_0 = 1 (so B_1 = -1/2)."""
    B = [Fraction(0)] * (n + 1)
    B[0] = Fraction(1)
    for m in range(1, n + 1):
        B[m] = -sum(comb(m + 1, j) * B[j] for j in range(m)) / (m + 1)
    return B


def index_weight_exact(index: str, s: int, t: int, l: int) -> Fraction:
    """Exact Moebius-side weight W_index(s, t) for |S| = s <= l, |T| = t >= s."""
    if not (0 <= s <= l) or t < s:
        raise ValueError("need 0 <= s <= l and t >= s")
    if index == "fsi":
        if t == s:
            return Fraction(1)
        return weight_exact(s, t, l) if (t > l and s >= 1) else Fraction(0)
    if index == "sii":
        return Fraction(1, t - s + 1)
    if index == "bii":
        return Fraction(1, 1 << (t - s))
    if index == "stii":
        if s < l:
            return Fraction(1 if t == s else 0)
        return Fraction(1, comb(t, l))
    if index == "ksii":
        if s == 0:
            return Fraction(1 if t == 0 else 0)
        B = bernoulli_exact(l)
        n = t - s
        return sum((B[j] * comb(n, j) / (n - j + 1) for j in range(0, min(l - s, n) + 1)),
                   Fraction(0))
    raise ValueError("unknown index %r (one of %s)" % (index, ", ".join(INDICES)))


def index_weight_table_f64(index: str, d: int, l: int) -> np.ndarray:
    """W[s, t] (shape (l+1, d+1)) of ``index_weight_exact``, each entry an
    exact rational rounded once to FP64; zero for t < s."""
    W = np.zeros((l + 1, d + 1), dtype=np.float64)
    for s in range(0, l + 1):
        for t in range(s, d + 1):
            W[s, t] = float(index_weight_exact(index, s, t, l))
    return W


def interaction(v: np.ndarray, d: int, l: int, index: str = "fsi") -> np.ndarray:
    """Scores I_S of the given index for all |S| <= l (canonical order), FP64:
    the Moebius transform, then brute-force superset sums with that index's
    exact weights. ``interaction(v, d, l, "fsi")`` equals ``fsi(v, d, l)``."""
    if not (1 <= l <= d):
        raise ValueError("need 1 <= l <= d")
    return _superset_weighted(v, d, l, index_weight_table_f64(index, d, l))



def interaction_from_mobius(a: np.ndarray, d: int, l: int, index: str = "fsi") -> np.ndarray:
    """The same scores from the Moebius transform a itself (the correction of
    Eq. 3 - 4 applied to given Moebius coefficients, no butterfly):
    I_S = sum over supersets T of S of W_index(|S|, |T|) a(T)."""
    if not (1 <= l <= d):
        raise ValueError("need 1 <= l <= d")
    W = weight_table_f64(d, l) if index == "fsi" else index_weight_table_f64(index, d, l)
    return _superset_weighted(a, d, l, W, transform=False)
