"""Pins of the tree-ensemble value-function oracle (oracle/forest.py) against
references that do not walk trees the way it does: hand-evaluated small
trees, the Moebius coefficients of tree games from leaf path products summed
back over subsets, the seeded C generator's heap-order evaluation, and
identities of the interventional value function."""
from __future__ import annotations

import numpy as np
import pytest

import games
import oracle
import pins_lib as P


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
    for k in range(K):
        o = k * n_tree
        for i in range(n_int):
            feature[o + i] = g.feat[k, i]
            threshold[o + i] = g.thr[k, i]
            left[o + i] = o + 2 * i + 1
            right[o + i] = o + 2 * i + 2
        value[o + n_int:o + n_tree] = g.leaf[k]
    roots = np.arange(K, dtype=np.int32) * n_tree
    return roots, feature, threshold, left, right, value


def test_hand_evaluated_irregular_tree():
    # root: feature 0 at 0.5; left -> leaf 1.0; right -> feature 1 at 0.3 -> (2.0, 3.0)
    feature = [0, -1, 1, -1, -1]
    threshold = [0.5, 0, 0.3, 0, 0]
    left = [1, 0, 3, 0, 0]
    right = [2, 0, 4, 0, 0]
    value = [0, 1.0, 0, 2.0, 3.0]
    x, bg = [0.7, 0.1], [[0.2, 0.9]]
    v = oracle.forest_values(2, [0], feature, threshold, left, right, value, x, bg)
    # S = {}: z = (0.2, 0.9) -> left leaf; {0}: (0.7, 0.9) -> 3; {1}: (0.2, 0.1) -> 1;
    # {0, 1}: (0.7, 0.1) -> 2
    assert v.tolist() == [1.0, 3.0, 1.0, 2.0]


def test_stump_closed_form():
    d = 5
    rng = np.random.default_rng(1)
    x = rng.uniform(size=d)
    bgs = rng.uniform(size=(7, d))
    f, th = 3, 0.5
    x[f] = 0.8
    v = oracle.forest_values(d, [0], [f, -1, -1], [th, 0, 0], [1, 0, 0], [2, 0, 0],
                             [0.0, -1.5, 4.0], x, bgs)
    frac_right = np.mean(bgs[:, f] >= th)
    for S in range(1 << d):
        want = 4.0 if (S >> f) & 1 else 4.0 * frac_right - 1.5 * (1 - frac_right)
        assert abs(v[S] - want) < 1e-15


@pytest.mark.parametrize("d,K,depth,seed", [(6, 3, 3, 0), (8, 10, 4, 1), (9, 6, 5, 2)])
def test_tree_games_via_moebius_path_products(d, K, depth, seed):
    g = games.tree_game(d, K, depth, games.rng_for(900, seed))
    v = oracle.forest_values(d, *heap_forest(g), g.x, g.b[None, :])
    want = np.zeros(1 << d)
    for R, c in P.tree_mobius_terms(g).items():
        for S in range(1 << d):
            if S & R == R:
                want[S] += c
    assert np.max(np.abs(v - want)) < 1e-12 * max(1.0, np.abs(want).max())


def test_matches_seeded_c_generator_d14():
    g, vg = games.d14_tree(0)
    v = oracle.forest_values(14, *heap_forest(g), g.x, g.b[None, :])
    assert np.max(np.abs(v - vg)) < 1e-12


def test_single_coalition_walk_and_background_linearity():
    d = 7
    g = games.tree_game(d, 12, 4, games.rng_for(901, 0))
    forest = heap_forest(g)
    rng = np.random.default_rng(3)
    bgs = rng.uniform(size=(5, d))
    v = oracle.forest_values(d, *forest, g.x, bgs)
    per = [oracle.forest_values(d, *forest, g.x, bgs[b:b + 1]) for b in range(5)]
    assert np.max(np.abs(v - np.mean(per, axis=0))) < 1e-13
    for S in (0, 5, 77, (1 << d) - 1):
        assert abs(oracle.forest_value_at(S, d, *forest, g.x, bgs) - v[S]) < 1e-13


def test_complement_symmetry():
    # swapping the explained point and a single background complements S
    d = 8
    g = games.tree_game(d, 9, 4, games.rng_for(902, 0))
    forest = heap_forest(g)
    v = oracle.forest_values(d, *forest, g.x, g.b[None, :])
    w = oracle.forest_values(d, *forest, g.b, g.x[None, :])
    full = (1 << d) - 1
    assert all(v[S] == w[full ^ S] for S in range(1 << d))


def test_threshold_tie_goes_right():
    # z == threshold takes the right branch (the convention of the format)
    v = oracle.forest_values(1, [0], [0, -1, -1], [0.25, 0, 0], [1, 0, 0], [2, 0, 0],
                             [0.0, 1.0, 2.0], [0.25], [[0.0]])
    assert v.tolist() == [1.0, 2.0]


def test_pins_catch_planted_walk_mistakes(monkeypatch):
    from oracle import forest as F
    real = F.forest_values

    def strict(d, roots, feature, threshold, left, right, value, x, bg):
        # '>' instead of '>=': a tie now goes left
        return real(d, roots, feature, np.nextafter(np.asarray(threshold, float), np.inf),
                    left, right, value, x, bg)

    def swapped(d, roots, feature, threshold, left, right, value, x, bg):
        # explained point and background exchanged
        bg = np.atleast_2d(bg)
        return real(d, roots, feature, threshold, left, right, value, bg[0], np.asarray(x)[None, :])

    for mutant in (strict, swapped):
        monkeypatch.setattr(oracle, "forest_values", mutant)
        failed = False
        for test in (test_threshold_tie_goes_right, test_hand_evaluated_irregular_tree,
                     lambda: test_tree_games_via_moebius_path_products(6, 3, 3, 0)):
            try:
                test()
            except AssertionError:
                failed = True
        assert failed, mutant.__name__
        monkeypatch.setattr(oracle, "forest_values", real)
