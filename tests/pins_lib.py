"""Independent references that pin the oracle (test helpers, CPU only).

None of these reuse the oracle's Moebius butterfly or superset-sum loop; each
follows a different definition or closed form from the paper or from the
mathematics:

  * ``fsi_wls``: the weighted least-squares definition of FSI (Sec. 2.2, Eq. 2)
    with the Shapley kernel weights and equality constraints at the empty and
    the full coalition, solved through its KKT system (float or exact).
  * ``shapley_eq1``: Shapley values from Eq. 1 (Sec. 2.1), term by term.
  * ``fsi_unanimity``: FSI of a unanimity game u_A (Moebius coefficients
    delta_A) read off Eq. 3 + Eq. 4 directly.
  * ``tree_mobius_terms``: the exact Moebius coefficients of a single-baseline
    tree-ensemble game from leaf path products.
  * ``fsi_exact_int``: for integer-valued v, the Moebius transform and the
    ranked superset sums in exact integers, the weights as exact rationals,
    one rounding at the end.
  * ``mpo_dense``: the MPO of Sec. 4.3 (bond states (s, t), 0/1 internal cores,
    weighted final core) built as dense cores and contracted site by site
    (Sec. 4.4), optionally precontracted with the Moebius cores (Sec. 4.5).
"""
from __future__ import annotations

from fractions import Fraction
from itertools import combinations
from math import comb, factorial

import numpy as np


# ---------------------------------------------------------------------------
# P1: weighted least squares definition (Eq. 2)
# ---------------------------------------------------------------------------
def _subsets_upto(d, l):
    out = []
    for s in range(l + 1):
        for c in combinations(range(d), s):
            out.append(sum(1 << i for i in c))
    return out


def _pc(x):
    return bin(x).count("1")


def shapley_kernel(d, t):
    """Shapley kernel weight for a coalition of size t, 0 < t < d."""
    return Fraction(d - 1, comb(d, t) * t * (d - t))


def fsi_wls(v, d, l, exact=False):
    """Solve min sum_T mu(T) (v(T) - sum_{S subset T, |S|<=l} I_S)^2 subject to
    equality at T = empty and T = [d]. Returns I in canonical order
    (ascending |S|, then ascending mask) as floats (or Fractions)."""
    S_list = sorted(_subsets_upto(d, l), key=lambda m: (_pc(m), m))
    M = len(S_list)
    full = (1 << d) - 1
    rows_fit = [T for T in range(1 << d) if 0 < _pc(T) < d]
    rows_eq = [0, full] if d >= 1 else [0]
    if exact:
        F = Fraction
        vv = [F(x) if not isinstance(x, Fraction) else x for x in v]
        n = M + len(rows_eq)
        A = [[F(0)] * n for _ in range(n)]
        rhs = [F(0)] * n
        for T in rows_fit:
            mu = shapley_kernel(d, _pc(T))
            xs = [j for j, S in enumerate(S_list) if (S & T) == S]
            for j in xs:
                rhs[j] += mu * vv[T]
                for k in xs:
                    A[j][k] += mu
        for r, T in enumerate(rows_eq):
            xs = [j for j, S in enumerate(S_list) if (S & T) == S]
            for j in xs:
                A[M + r][j] = F(1)
                A[j][M + r] = F(1)
            rhs[M + r] = vv[T]
        sol = _solve_exact(A, rhs)
        return sol[:M]
    v = np.asarray(v, dtype=np.float64)
    X = np.array([[1.0 if (S & T) == S else 0.0 for S in S_list] for T in range(1 << d)])
    mu = np.zeros(1 << d)
    for T in rows_fit:
        mu[T] = float(shapley_kernel(d, _pc(T)))
    Xf = X[rows_fit]
    H = Xf.T @ (mu[rows_fit][:, None] * Xf)
    g = Xf.T @ (mu[rows_fit] * v[rows_fit])
    C = X[rows_eq]
    K = np.block([[H, C.T], [C, np.zeros((len(rows_eq), len(rows_eq)))]])
    rhs = np.concatenate([g, v[rows_eq]])
    sol = np.linalg.solve(K, rhs)
    return sol[:M]


def _solve_exact(A, b):
    n = len(b)
    A = [row[:] + [b[i]] for i, row in enumerate(A)]
    for c in range(n):
        p = next(r for r in range(c, n) if A[r][c] != 0)
        A[c], A[p] = A[p], A[c]
        piv = A[c][c]
        A[c] = [x / piv for x in A[c]]
        for r in range(n):
            if r != c and A[r][c] != 0:
                f = A[r][c]
                A[r] = [x - f * y for x, y in zip(A[r], A[c])]
    return [A[i][n] for i in range(n)]


# ---------------------------------------------------------------------------
# Eq. 1 Shapley values
# ---------------------------------------------------------------------------
def shapley_eq1(v, d):
    v = np.asarray(v, dtype=np.float64)
    phi = np.zeros(d)
    for i in range(d):
        bit = 1 << i
        acc = 0.0
        for S in range(1 << d):
            if S & bit:
                continue
            s = _pc(S)
            wgt = factorial(s) * factorial(d - s - 1) / factorial(d)
            acc += wgt * (v[S | bit] - v[S])
        phi[i] = acc
    return phi


# ---------------------------------------------------------------------------
# P2: unanimity games, read off Eq. 3 + Eq. 4
# ---------------------------------------------------------------------------
def _w_eq7(s, t, l):
    """Eq. 7 typed from the paper (used only where the sum structure, not the
    weight value, is under test; the weights are pinned by P1 and by the
    efficiency identity)."""
    return (Fraction((-1) ** (l - s)) * Fraction(s, l + s) * comb(l, s)
            * Fraction(comb(t - 1, l), comb(t + l - 1, l + s)))


def fsi_unanimity(A, d, l, exact=False):
    """FSI (canonical order) of u_A: v(S) = [A subset of S], whose Moebius
    transform is the indicator of A. Eq. 3: E_S = a(S) + C_S; for S = A the
    Moebius term is 1; Eq. 4 adds w(|S|, |A|) for every S strictly inside A
    with |A| > l."""
    S_list = sorted(_subsets_upto(d, l), key=lambda m: (_pc(m), m))
    a_sz = _pc(A)
    out = []
    for S in S_list:
        val = Fraction(0)
        if S == A:
            val += 1
        if a_sz > l and (S & A) == S and S != A:
            val += _w_eq7(_pc(S), a_sz, l)
        out.append(val)
    return out if exact else np.array([float(x) for x in out])


def fsi_sparse_mobius(terms, d, l):
    """Linearity: FSI of v = sum_k c_k u_{A_k} is sum_k c_k FSI(u_{A_k})."""
    S_list = sorted(_subsets_upto(d, l), key=lambda m: (_pc(m), m))
    index = {S: j for j, S in enumerate(S_list)}
    E = np.zeros(len(S_list))
    for A, c in terms:
        A = int(A)
        a_sz = _pc(A)
        if a_sz <= l:
            E[index[A]] += c
            continue
        sub = A
        while True:
            if sub != A and _pc(sub) <= l:
                E[index[sub]] += c * float(_w_eq7(_pc(sub), a_sz, l))
            if sub == 0:
                break
            sub = (sub - 1) & A
    return E


# ---------------------------------------------------------------------------
# P3: tree games via leaf path products
# ---------------------------------------------------------------------------
def tree_mobius_terms(g):
    """Moebius coefficients of v(S) = sum_trees tree(z(S)). For one leaf with
    distinct path features F, alpha_f = [x passes every test on f],
    beta_f = [b passes every test on f]; the leaf is reached iff every f in F
    passes at z_f, so the leaf contributes
        leaf * prod_{f in F} (beta_f + [f in S] (alpha_f - beta_f)),
    whose Moebius coefficient on R subset of F is
        leaf * prod_{f in R} (alpha_f - beta_f) * prod_{f in F \\ R} beta_f.
    Returns a dict mask -> coefficient."""
    terms = {}
    n_int = (1 << g.depth) - 1
    for tr in range(g.feat.shape[0]):
        for lf in range(1 << g.depth):
            alpha, beta = {}, {}
            node = n_int + lf
            while node > 0:
                parent = (node - 1) // 2
                right = node == 2 * parent + 2
                f = int(g.feat[tr, parent])
                th = g.thr[tr, parent]
                px = (g.x[f] >= th) if right else (g.x[f] < th)
                pb = (g.b[f] >= th) if right else (g.b[f] < th)
                alpha[f] = alpha.get(f, True) and bool(px)
                beta[f] = beta.get(f, True) and bool(pb)
                node = parent
            F = sorted(alpha)
            val = g.leaf[tr, lf]
            for r in range(len(F) + 1):
                for R in combinations(F, r):
                    coef = val
                    for f in F:
                        if f in R:
                            coef *= float(alpha[f]) - float(beta[f])
                        else:
                            coef *= float(beta[f])
                    if coef != 0.0:
                        m = sum(1 << f for f in R)
                        terms[m] = terms.get(m, 0.0) + coef
    return terms


# ---------------------------------------------------------------------------
# P6: exact integer evaluation
# ---------------------------------------------------------------------------
def fsi_exact_int(v_int, d, l):
    """E_S for integer-valued v: the Moebius transform in int64 (exact; the
    values stay below 2^(d+1) in magnitude), ranked superset sums
    A_t(S) = sum_{T superset S, |T| = t} a(T) in int64, and
    E_S = a(S) + sum_{t > l} w(s, t) A_t(S) in exact rationals (weights from
    Eq. 7), rounded once to float."""
    a = np.array(v_int, dtype=np.int64)
    n = 1 << d
    for i in range(d):  # inclusion-exclusion over one bit at a time, integers
        bit = 1 << i
        idx = np.arange(n)
        hi = idx[(idx & bit) != 0]
        a[hi] = a[hi] - a[hi ^ bit]
    pc = np.array([_pc(x) for x in range(n)], dtype=np.int64)
    S_list = sorted(_subsets_upto(d, l), key=lambda m: (_pc(m), m))
    out = []
    for S in S_list:
        s = _pc(S)
        free = [i for i in range(d) if not (S >> i) & 1]
        idx = np.arange(1 << len(free), dtype=np.int64)
        T = np.full(idx.shape, S, dtype=np.int64)
        for j, b in enumerate(free):
            T |= ((idx >> j) & 1) << b
        At = np.bincount(pc[T], weights=None, minlength=d + 1)  # counts only
        sums = np.zeros(d + 1, dtype=np.int64)
        np.add.at(sums, pc[T], a[T])
        val = Fraction(int(a[S]))
        if s >= 1:
            for t in range(l + 1, d + 1):
                if sums[t] != 0:
                    val += _w_eq7(s, t, l) * int(sums[t])
        del At
        out.append(float(val))
    return np.array(out)


# ---------------------------------------------------------------------------
# P8: dense MPO cores and site-by-site contraction (Sec. 4.3 - 4.5)
# ---------------------------------------------------------------------------
def mpo_states(k, l):
    """Bond states after k sites: (s, t) with 0 <= s <= min(k, l), s <= t <= k."""
    return [(s, t) for s in range(min(k, l) + 1) for t in range(s, k + 1)]


def mpo_cores(d, l, precontract=False):
    """Dense cores G[k] of shape (D_{k-1}, 2, 2, D_k) indexed
    [alpha_prev, sigma, tau, alpha_next]. Internal sites carry 1 on valid
    transitions (tau >= sigma, counters advance, s stays <= l); the last site
    carries the weight w(s, t) on valid transitions that end with s <= l and
    t > l, into a single closing state. With precontract=True each core is
    composed with the 2x2 Moebius factor on its input index (Sec. 4.5)."""
    cores = []
    for k in range(1, d + 1):
        prev = mpo_states(k - 1, l)
        last = k == d
        nxt = [(0, 0)] if last else mpo_states(k, l)
        pos = {st: j for j, st in enumerate(nxt)}
        G = np.zeros((len(prev), 2, 2, len(nxt)))
        for ia, (s, t) in enumerate(prev):
            for sg in (0, 1):
                for tau in (0, 1):
                    if tau < sg:
                        continue
                    s2, t2 = s + sg, t + tau
                    if s2 > min(k, l):
                        continue
                    if last:
                        if s2 <= l and t2 > l and s2 >= 1:
                            G[ia, sg, tau, 0] = float(_w_eq7(s2, t2, l))
                    else:
                        G[ia, sg, tau, pos[(s2, t2)]] = 1.0
        if precontract:
            B = np.empty_like(G)
            B[:, :, 0, :] = G[:, :, 0, :] - G[:, :, 1, :]
            B[:, :, 1, :] = G[:, :, 1, :]
            G = B
        cores.append(G)
    return cores


def mpo_apply(cores, x, d, l):
    """Outputs u[S], |S| <= l, of the operator the MPO represents, applied to
    x (length 2^d). By definition of an MPO, its matrix entry for output S and
    input T is the product of the core slices along the sites,
        M[S, T] = G1[., s_1(S), t_1(T), .] G2[., s_2(S), t_2(T), .] ... Gd[...],
    a 1 x 1 matrix (the first and last bond dimensions are 1); site k reads
    bit d - k of the masks (the first site is the most significant bit). So
    u[S] = sum_T M[S, T] x[T], evaluated here pair by pair (all T at once for
    one S, the slice product carried as a row vector per T)."""
    x = np.asarray(x, dtype=np.float64)
    T = np.arange(1 << d)
    out = {}
    for S in _subsets_upto(d, l):
        row = np.ones((T.size, 1))
        for k, G in enumerate(cores, start=1):
            bit = d - k
            sig = (S >> bit) & 1
            tau = (T >> bit) & 1                       # per input T
            slices = G[:, sig, :, :].transpose(1, 0, 2)[tau]   # (n_T, D_prev, D_next)
            row = np.einsum("nd,nde->ne", row, slices)
        out[S] = float(row[:, 0] @ x)
    return out


def fsi_via_mpo(v, d, l, precontract=False):
    """FSI = mu v + A_trunc(mu v) (Eq. 5), or mu v + B_corr v (Sec. 4.5),
    restricted to |S| <= l, in canonical order. The Moebius term uses the
    direct definition so that this path shares nothing with the oracle."""
    v = np.asarray(v, dtype=np.float64)
    from_oracle_free_mobius = _mobius_by_definition(v, d)
    if precontract:
        corr = mpo_apply(mpo_cores(d, l, precontract=True), v, d, l)
    else:
        corr = mpo_apply(mpo_cores(d, l), from_oracle_free_mobius, d, l)
    S_list = sorted(_subsets_upto(d, l), key=lambda m: (_pc(m), m))
    return np.array([from_oracle_free_mobius[S] + corr[S] for S in S_list])


def _mobius_by_definition(v, d):
    n = 1 << d
    a = np.zeros(n)
    for S in range(n):
        T = S
        acc = 0.0
        while True:
            acc += (-1.0) ** (_pc(S) - _pc(T)) * v[T]
            if T == 0:
                break
            T = (T - 1) & S
        a[S] = acc
    return a
