"""Closed forms of the FSI operator for games whose Moebius transform is
sparse and known (TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``).

Two facts of the paper give E = FSI(v) without touching the 2^d values:

* Unanimity games and linearity (Sec. 2.2, Eq. 3 and Eq. 4): the Moebius
  transform of u_A(S) = [A subset of S] is the indicator of A, so Eq. 3 - 4
  give E_S = [S = A] when |A| <= l, and E_S = w(|S|, |A|) for every S
  strictly inside A with 1 <= |S| <= l when |A| > l (w of Sec. 4.3, Eq. 7;
  w(0, t) = 0). FSI is linear in v (Eq. 3 - 4 are linear in a), so a game
  v = sum_k c_k u_{A_k} has E = sum_k c_k FSI(u_{A_k}).
* Tree games through path products (Sec. 2.1's value function of a tree
  model with the features outside S taken from a baseline point b): the leaf
  of a root-to-leaf path is reached at z(S) iff every split on the path
  passes, so with F the path's distinct features,
  alpha_f = [x passes every split on f] and beta_f = [b passes them],
  the leaf contributes value * prod_{f in F} (beta_f + [f in S](alpha_f - beta_f)).
  Expanding the product, its Moebius coefficients sit on R = B0 union Q with
  B0 = {f : beta_f = 0}, Q any subset of {f : beta_f = 1, alpha_f = 0}, and
  equal value * (-1)^|Q| (a path with alpha_f = beta_f = 0 for some f is
  reached by no coalition and contributes nothing).

Weights are exact rationals (``weight_exact``) rounded once to FP64; sums
are FP64 in the order the terms come. These functions are pinned in
``tests/test_oracle_pins.py`` against the brute-force oracle and against an
independent term-by-term derivation of the same facts.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np

from .fsi_oracle import output_masks, weight_exact

__all__ = ["tree_mobius_sparse", "planted_mobius_sparse", "fsi_from_sparse_mobius"]


def _popcount64(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.int64)
    c = np.zeros(x.shape, dtype=np.int64)
    for i in range(62):
        c += (x >> i) & 1
    return c


def tree_mobius_sparse(g):
    """Moebius coefficients of a tree game (games.TreeGame: full binary trees
    in heap order, go right iff z_f >= threshold) by the path-product rule
    above. Returns (masks, coefs): int64 masks, FP64 coefficients, one entry
    per distinct mask with a nonzero coefficient."""
    depth = int(g.depth)
    n_trees = g.feat.shape[0]
    n_int = (1 << depth) - 1
    n_leaf = 1 << depth
    leaf_ids = np.arange(n_leaf)
    # per (tree, leaf): the masks of features whose splits x (resp. b) fails
    fail_x = np.zeros((n_trees, n_leaf), dtype=np.int64)
    fail_b = np.zeros((n_trees, n_leaf), dtype=np.int64)
    node = np.full(n_leaf, n_int, dtype=np.int64) + leaf_ids
    for _ in range(depth):
        parent = (node - 1) // 2
        right = node == 2 * parent + 2
        f = g.feat[:, parent].astype(np.int64)            # (n_trees, n_leaf)
        th = g.thr[:, parent]
        xf = g.x[f]
        bf = g.b[f]
        pass_x = np.where(right[None, :], xf >= th, xf < th)
        pass_b = np.where(right[None, :], bf >= th, bf < th)
        bit = np.int64(1) << f
        fail_x |= np.where(pass_x, 0, bit)
        fail_b |= np.where(pass_b, 0, bit)
        node = parent
    value = g.leaf.astype(np.float64)
    live = (fail_x & fail_b) == 0                          # no f with alpha = beta = 0
    B0 = fail_b[live]
    Z = (fail_x & ~fail_b)[live]
    val = value[live]
    # every subset Q of Z: walk the submasks Q = Z, (Z - 1) & Z, ..., 0
    masks, coefs = [], []
    Q = Z.copy()
    active = np.ones(Q.shape, dtype=bool)
    while np.any(active):
        sign = np.where(_popcount64(Q[active]) % 2 == 1, -1.0, 1.0)
        masks.append(B0[active] | Q[active])
        coefs.append(val[active] * sign)
        done = Q == 0
        Q = np.where(done, 0, (Q - 1) & Z)
        active &= ~done
    m = np.concatenate(masks)
    c = np.concatenate(coefs)
    uniq, inv = np.unique(m, return_inverse=True)
    tot = np.zeros(uniq.size, dtype=np.float64)
    np.add.at(tot, inv, c)
    keep = tot != 0.0
    return uniq[keep], tot[keep]


def planted_mobius_sparse(g):
    """Moebius coefficients of a planted game v = sum_k c_k u_{A_k}
    (games.PlantedGame): c_k on A_k, repeated masks added."""
    uniq, inv = np.unique(np.asarray(g.masks, dtype=np.int64), return_inverse=True)
    tot = np.zeros(uniq.size, dtype=np.float64)
    np.add.at(tot, inv, np.asarray(g.coefs, dtype=np.float64))
    return uniq, tot


def fsi_from_sparse_mobius(masks, coefs, d: int, l: int) -> np.ndarray:
    """FSI in canonical order of the game whose Moebius transform is
    sum_k coefs[k] * [T = masks[k]], by the unanimity closed form and
    linearity (module docstring)."""
    masks = np.asarray(masks, dtype=np.int64)
    coefs = np.asarray(coefs, dtype=np.float64)
    index = _index_table(d, l)                        # mask -> canonical position
    E = np.zeros(int(np.count_nonzero(index >= 0)), dtype=np.float64)
    sizes = _popcount64(masks)
    # |A| <= l: the Moebius term itself (Eq. 3), no correction
    small = sizes <= l
    if np.any(small):
        np.add.at(E, index[masks[small]], coefs[small])
    # |A| > l: w(|S|, |A|) on every S strictly inside A, 1 <= |S| <= l (Eq. 4)
    for t in np.unique(sizes[~small]):
        t = int(t)
        sel = sizes == t
        A = masks[sel]
        c = coefs[sel]
        # the set bits of each A, in ascending order: (n_terms, t)
        bits = np.zeros((A.size, t), dtype=np.int64)
        rem = A.copy()
        for j in range(t):
            low = rem & -rem
            bits[:, j] = low
            rem ^= low
        for s in range(1, l + 1):
            w = _weight_f64(s, t, l)
            # every s-subset of the t positions
            for combo in _combinations(t, s):
                sub = np.zeros(A.size, dtype=np.int64)
                for j in combo:
                    sub |= bits[:, j]
                np.add.at(E, index[sub], c * w)
    return E


@lru_cache(maxsize=None)
def _weight_f64(s: int, t: int, l: int) -> float:
    return float(weight_exact(s, t, l))


@lru_cache(maxsize=None)
def _combinations(n: int, k: int):
    from itertools import combinations
    return list(combinations(range(n), k))


@lru_cache(maxsize=8)
def _index_table(d: int, l: int) -> np.ndarray:
    outs = output_masks(d, l).astype(np.int64)
    index = np.full(1 << d, -1, dtype=np.int64)
    index[outs] = np.arange(outs.size)
    index.setflags(write=False)
    return index
