"""Seeded synthetic cooperative games (inputs for tests and the benchmark).

This module only builds value vectors v over all 2^d coalitions from a game's
own definition. It holds none of the FSI operator's arithmetic, and it is the
only code shared by the oracle side and the GPU side.

Games (stand-ins for the paper's datasets and trained models, which are not
available; shapes follow the paper's experiments: d in [8, 20], tree models of
depth <= 6, the value function of one background point):
  * planted sparse game: v(S) = sum_k c_k [A_k subset of S], |A_k| ~ U{1..kmax}
    distinct features, c_k ~ N(0, 1); v(empty) = 0.
  * tree-ensemble game: full binary regression trees of a given depth, split
    features i.i.d. U{0..d-1}, thresholds U(0, 1), leaves N(0, 1), go right
    iff z_f >= threshold; instance x and baseline b ~ U(0, 1)^d;
    v(S) = sum_trees tree(z(S)) with z(S)_f = x_f if f in S else b_f.
  * i.i.d. +/-1 vector (maximal Moebius cancellation), i.i.d. N(0, 1) vector.

Seeding: numpy.random.default_rng(SeedSequence([config_id, instance])).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "games.c")
_LIB = os.path.join(_HERE, "_build", "libgames.so")
_lib = None


def build_c(force: bool = True) -> str:
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_c(force=False)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip64 = ctypes.POINTER(ctypes.c_int64)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.games_planted.argtypes = [dp, ctypes.c_int, ctypes.c_int, ip64, dp]
        lib.games_planted.restype = None
        lib.games_tree.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ip, dp, dp, dp, dp]
        lib.games_tree.restype = None
        _lib = lib
    return _lib


def rng_for(config_id: int, instance: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(config_id), int(instance)]))


# --------------------------------------------------------------------------
# planted sparse games
# --------------------------------------------------------------------------
@dataclass
class PlantedGame:
    d: int
    masks: np.ndarray   # int64, one mask per term
    coefs: np.ndarray   # float64


def planted_game(d: int, n_terms: int, kmax: int, rng) -> PlantedGame:
    masks = np.zeros(n_terms, dtype=np.int64)
    coefs = np.zeros(n_terms, dtype=np.float64)
    for k in range(n_terms):
        size = int(rng.integers(1, kmax + 1))
        feats = rng.choice(d, size=size, replace=False)
        masks[k] = int(np.sum(np.int64(1) << feats.astype(np.int64)))
        coefs[k] = rng.standard_normal()
    return PlantedGame(d, masks, coefs)


def planted_values(g: PlantedGame) -> np.ndarray:
    lib = _load()
    v = np.zeros(1 << g.d, dtype=np.float64)
    m = np.ascontiguousarray(g.masks, dtype=np.int64)
    c = np.ascontiguousarray(g.coefs, dtype=np.float64)
    lib.games_planted(v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), g.d,
                      m.size, m.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                      c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return v


def planted_values_direct(g: PlantedGame) -> np.ndarray:
    """Same as planted_values by direct evaluation of [A subset of S] over
    all masks (numpy; for cross-checking the C builder at small d)."""
    S = np.arange(1 << g.d, dtype=np.int64)
    v = np.zeros(S.size, dtype=np.float64)
    for A, c in zip(g.masks, g.coefs):
        v += np.where((S & A) == A, c, 0.0)
    return v


# --------------------------------------------------------------------------
# tree-ensemble games
# --------------------------------------------------------------------------
@dataclass
class TreeGame:
    d: int
    depth: int
    feat: np.ndarray    # int32 (n_trees, 2^depth - 1)
    thr: np.ndarray     # float64 (n_trees, 2^depth - 1)
    leaf: np.ndarray    # float64 (n_trees, 2^depth)
    x: np.ndarray       # float64 (d,)
    b: np.ndarray       # float64 (d,)


def tree_game(d: int, n_trees: int, depth: int, rng) -> TreeGame:
    n_int = (1 << depth) - 1
    feat = rng.integers(0, d, size=(n_trees, n_int)).astype(np.int32)
    thr = rng.uniform(0.0, 1.0, size=(n_trees, n_int))
    leaf = rng.standard_normal(size=(n_trees, 1 << depth))
    x = rng.uniform(0.0, 1.0, size=d)
    b = rng.uniform(0.0, 1.0, size=d)
    return TreeGame(d, depth, feat, thr, leaf, x, b)


def tree_values(g: TreeGame) -> np.ndarray:
    lib = _load()
    v = np.zeros(1 << g.d, dtype=np.float64)
    feat = np.ascontiguousarray(g.feat, dtype=np.int32)
    thr = np.ascontiguousarray(g.thr, dtype=np.float64)
    leaf = np.ascontiguousarray(g.leaf, dtype=np.float64)
    x = np.ascontiguousarray(g.x, dtype=np.float64)
    b = np.ascontiguousarray(g.b, dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.games_tree(v.ctypes.data_as(dp), g.d, feat.shape[0], g.depth,
                   feat.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                   thr.ctypes.data_as(dp), leaf.ctypes.data_as(dp),
                   x.ctypes.data_as(dp), b.ctypes.data_as(dp))
    return v


def tree_values_direct(g: TreeGame) -> np.ndarray:
    """Evaluate every tree at every z(S) (numpy; small d cross-check)."""
    S = np.arange(1 << g.d, dtype=np.int64)
    member = ((S[:, None] >> np.arange(g.d)) & 1).astype(bool)   # (2^d, d)
    z = np.where(member, g.x[None, :], g.b[None, :])
    v = np.zeros(S.size, dtype=np.float64)
    n_int = (1 << g.depth) - 1
    for tr in range(g.feat.shape[0]):
        node = np.zeros(S.size, dtype=np.int64)
        for _ in range(g.depth):
            f = g.feat[tr][node]
            t = g.thr[tr][node]
            right = z[np.arange(S.size), f] >= t
            node = 2 * node + np.where(right, 2, 1)
        v += g.leaf[tr][node - n_int]
    return v


# --------------------------------------------------------------------------
# unstructured vectors
# --------------------------------------------------------------------------
def pm1_values(d: int, rng) -> np.ndarray:
    return rng.choice(np.array([-1.0, 1.0]), size=1 << d)


def normal_values(d: int, rng) -> np.ndarray:
    return rng.standard_normal(1 << d)


# --------------------------------------------------------------------------
# workload recipes
# --------------------------------------------------------------------------
CFG_SMALL, CFG_D14, CFG_D20, CFG_RAGGED, CFG_D20_BATCH = 1, 2, 3, 4, 5


def small_planted(instance: int = 0):
    """d=8: planted game, 40 terms, |A| ~ U{1..4}."""
    g = planted_game(8, 40, 4, rng_for(CFG_SMALL, 2 * instance))
    return g, planted_values(g)


def small_normal(instance: int = 0):
    """d=8: i.i.d. N(0, 1) vector (v(empty) != 0)."""
    return normal_values(8, rng_for(CFG_SMALL, 2 * instance + 1))


def d14_tree(instance: int = 0):
    """d=14: 50 depth-4 trees on 14 features."""
    g = tree_game(14, 50, 4, rng_for(CFG_D14, instance))
    return g, tree_values(g)


def d20_tree(instance: int = 0):
    """d=20: 200 depth-6 trees on 20 features."""
    g = tree_game(20, 200, 6, rng_for(CFG_D20, 2 * instance))
    return g, tree_values(g)


def d20_pm1(instance: int = 0):
    return pm1_values(20, rng_for(CFG_D20, 2 * instance + 1))


def ragged_specs(n: int = 512):
    """(d_i, l_i) for the ragged batch: d ~ U{8..20}, l ~ U{1..4}."""
    rng = rng_for(CFG_RAGGED, 1_000_000)
    ds = rng.integers(8, 21, size=n)
    ls = rng.integers(1, 5, size=n)
    return [int(x) for x in ds], [int(x) for x in ls]


def ragged_instance(i: int, d: int):
    """Instance i of the ragged batch: 100 depth-5 trees on d features."""
    g = tree_game(d, 100, 5, rng_for(CFG_RAGGED, i))
    return g, tree_values(g)


def d20_batch_instance(i: int):
    """Instance i of the d=20 batch: even i -> tree game (200 depth-6 trees),
    odd i -> planted game (200 terms, |A| ~ U{1..6})."""
    if i % 2 == 0:
        g = tree_game(20, 200, 6, rng_for(CFG_D20_BATCH, i))
        return g, tree_values(g)
    g = planted_game(20, 200, 6, rng_for(CFG_D20_BATCH, i))
    return g, planted_values(g)


def build_many(fn, indices, threads: int = 8):
    """Run an instance builder over indices with a thread pool (the C builders
    release the GIL)."""
    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        return list(ex.map(fn, indices))
