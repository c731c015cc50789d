"""Plain FP64 CPU oracle for the value function of a tree ensemble.

TEST INFRASTRUCTURE ONLY (same rules as fsi_oracle.py): only tests/,
__graft_entry__.smoke() and bench.py's cpu_baseline leg may use it, and it
shares no code with the HIP implementation.

What it computes: the value function the FSI operator consumes (Sec. 2.1:
v(S) is the model's output when only the features in S are taken from the
explained point), in its interventional form over background points. For an
explained point x, background points bg_1 .. bg_B and regression trees
f_1 .. f_K:

    v(S) = (1/B) sum_b sum_k f_k(z_b(S)),   z_b(S)_i = x_i if i in S else bg_b,i

for every coalition S (bit i of the index <=> feature i in S). The paper
obtains v by one model prediction per coalition (its bottleneck analysis in
the appendix times exactly this step); here every tree is walked for every
coalition and background, vectorised over coalitions.

Tree format: arrays over nodes. Node i is a leaf if feature[i] < 0 (its
output is value[i]); otherwise it sends z to right[i] if
z[feature[i]] >= threshold[i], else to left[i]. roots[k] is tree k's root.
"""
from __future__ import annotations

import numpy as np

__all__ = ["forest_values", "forest_value_at"]


def forest_values(d, roots, feature, threshold, left, right, value, x, bg):
    """v over all 2^d coalitions, FP64 (see the module docstring)."""
    feature = np.asarray(feature, dtype=np.int64)
    threshold = np.asarray(threshold, dtype=np.float64)
    left = np.asarray(left, dtype=np.int64)
    right = np.asarray(right, dtype=np.int64)
    value = np.asarray(value, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    bg = np.atleast_2d(np.asarray(bg, dtype=np.float64))
    if x.shape != (d,) or bg.shape[1] != d:
        raise ValueError("x must have d entries and bg d columns")
    S = np.arange(1 << d, dtype=np.int64)
    member = ((S[:, None] >> np.arange(d)) & 1).astype(bool)   # (2^d, d)
    rows = np.arange(S.size)
    total = np.zeros(S.size, dtype=np.float64)
    for b in range(bg.shape[0]):
        z = np.where(member, x[None, :], bg[b][None, :])         # z_b(S)
        for r in roots:
            node = np.full(S.size, int(r), dtype=np.int64)
            while True:
                inner = feature[node] >= 0
                if not inner.any():
                    break
                f = np.where(inner, feature[node], 0)
                go_right = z[rows, f] >= threshold[node]
                nxt = np.where(go_right, right[node], left[node])
                node = np.where(inner, nxt, node)
            total += value[node]
    return total / bg.shape[0]


def forest_value_at(S, d, roots, feature, threshold, left, right, value, x, bg):
    """v(S) for one coalition by walking each tree with a plain loop."""
    bg = np.atleast_2d(np.asarray(bg, dtype=np.float64))
    acc = 0.0
    for b in range(bg.shape[0]):
        z = [x[i] if (S >> i) & 1 else bg[b][i] for i in range(d)]
        for r in roots:
            n = int(r)
            while feature[n] >= 0:
                n = int(right[n]) if z[int(feature[n])] >= threshold[n] else int(left[n])
            acc += float(value[n])
    return acc / bg.shape[0]
