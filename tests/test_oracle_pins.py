"""Pins of the CPU oracle against definitions that do not reuse its arithmetic.

Every test here runs on the CPU (no GPU marker). See tests/pins_lib.py for the
independent references (paper Sec. 2.1-2.2, Sec. 4.3-4.5 and closed forms).
"""
from fractions import Fraction
from math import comb
import os

import numpy as np
import pytest

import games
import oracle
import pins_lib as P

HERE = os.path.dirname(os.path.abspath(__file__))


def normwise(x, ref):
    ref = np.asarray(ref, dtype=np.float64)
    den = max(np.max(np.abs(ref)), 1e-300)
    return float(np.max(np.abs(np.asarray(x) - ref)) / den)


# ---------------------------------------------------------------- P7 golden
def load_golden(name):
    meta, rows = {}, []
    with open(os.path.join(HERE, "golden", name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if parts[0] in ("d", "l"):
                meta[parts[0]] = int(parts[1])
            elif parts[0] == "game":
                meta["game"] = (parts[1], int(parts[2]))
            else:
                rows.append((int(parts[0]), Fraction(parts[1])))
    return meta, rows


def test_worked_example_golden():
    meta, rows = load_golden("worked_d3_l2_unanimity.txt")
    d, l = meta["d"], meta["l"]
    A = meta["game"][1]
    v = np.array([1.0 if (S & A) == A else 0.0 for S in range(1 << d)])
    masks = oracle.output_masks(d, l)
    assert [int(m) for m in masks] == [m for m, _ in rows]
    E = oracle.fsi(v, d, l)
    for e, (_, val) in zip(E, rows):
        assert abs(e - float(val)) < 1e-15
    # the same values from the exact WLS definition
    ex = P.fsi_wls([Fraction(int(x)) for x in v], d, l, exact=True)
    assert ex == [val for _, val in rows]


# ---------------------------------------------------------------- P1 WLS
@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_wls_exact_rationals(d):
    rng = np.random.default_rng(100 + d)
    v = [Fraction(int(x)) for x in rng.integers(-9, 10, size=1 << d)]
    v[0] = Fraction(3)  # v(empty) != 0 on purpose
    for l in range(1, d + 1):
        ex = P.fsi_wls(v, d, l, exact=True)
        E = oracle.fsi(np.array([float(x) for x in v]), d, l)
        ref = np.array([float(x) for x in ex])
        assert normwise(E, ref) < 1e-14, (d, l)


@pytest.mark.parametrize("d", [5, 6, 7, 8])
def test_wls_float_normal(d):
    rng = np.random.default_rng(200 + d)
    v = rng.standard_normal(1 << d)
    for l in range(1, d + 1):
        ref = P.fsi_wls(v, d, l)
        assert normwise(oracle.fsi(v, d, l), ref) < 1e-9, (d, l)


def test_wls_small_config_planted_and_normal():
    g, v = games.small_planted(0)
    assert normwise(oracle.fsi(v, 8, 2), P.fsi_wls(v, 8, 2)) < 1e-9
    vn = games.small_normal(0)
    assert vn[0] != 0.0
    assert normwise(oracle.fsi(vn, 8, 2), P.fsi_wls(vn, 8, 2)) < 1e-9


# ---------------------------------------------------------------- weights
def test_efficiency_identity_exact():
    # sum_{s=1..l} C(t, s) w(s, t) = 1 for every t > l: this is what makes
    # the scores of an l-order surrogate add up to v([d]) (faithfulness).
    for l in range(1, 31):
        for t in range(l + 1, 41):
            tot = sum(comb(t, s) * oracle.weight_exact(s, t, l) for s in range(1, l + 1))
            assert tot == 1, (l, t)


def test_weight_table_structure():
    W = oracle.weight_table_f64(20, 4)
    for s in range(5):
        assert W[s, s] == 1.0
        for t in range(s + 1, 5):
            assert W[s, t] == 0.0
    assert np.all(W[0, 1:] == 0.0)
    assert W[1, 5] == float(oracle.weight_exact(1, 5, 4))


# ---------------------------------------------------------------- Moebius
@pytest.mark.parametrize("d", [1, 3, 6, 9])
def test_mobius_vs_definition(d):
    rng = np.random.default_rng(d)
    v = rng.standard_normal(1 << d)
    a = oracle.mobius(v)
    assert np.max(np.abs(a - oracle.mobius_direct(v))) < 1e-12
    # inversion: v(S) = sum_{T subset S} a(T)
    for S in range(1 << d):
        T, acc = S, 0.0
        while True:
            acc += a[T]
            if T == 0:
                break
            T = (T - 1) & S
        assert abs(acc - v[S]) < 1e-12


# ---------------------------------------------------------------- P2 unanimity
@pytest.mark.parametrize("d,l", [(4, 2), (6, 3), (8, 2), (10, 4), (12, 1)])
def test_unanimity_closed_form(d, l):
    rng = np.random.default_rng(d * 31 + l)
    for _ in range(4):
        A = int(rng.integers(0, 1 << d))
        v = np.array([1.0 if (S & A) == A else 0.0 for S in range(1 << d)])
        assert normwise(oracle.fsi(v, d, l), P.fsi_unanimity(A, d, l)) < 1e-14


def test_planted_small_config_linearity():
    g, v = games.small_planted(0)
    ref = P.fsi_sparse_mobius(zip(g.masks, g.coefs), 8, 2)
    assert normwise(oracle.fsi(v, 8, 2), ref) < 1e-14


# ---------------------------------------------------------------- P3 trees
def test_tree_game_path_products_small():
    g = games.tree_game(10, 12, 4, games.rng_for(90, 0))
    v = games.tree_values(g)
    terms = P.tree_mobius_terms(g)
    a = oracle.mobius(v)
    # the Moebius support of a depth-4 single-baseline tree game is |T| <= 4
    pc = np.array([bin(i).count("1") for i in range(1 << 10)])
    assert np.max(np.abs(a[pc > 4])) < 1e-12
    for l in (2, 3):
        ref = P.fsi_sparse_mobius(terms.items(), 10, l)
        assert normwise(oracle.fsi(v, 10, l), ref) < 1e-12


def test_tree_game_d14_config():
    g, v = games.d14_tree(0)
    ref = P.fsi_sparse_mobius(P.tree_mobius_terms(g).items(), 14, 3)
    assert normwise(oracle.fsi(v, 14, 3), ref) < 1e-12


# ---------------------------------------------------------------- P4 special cases
@pytest.mark.parametrize("d", [3, 6, 9])
def test_l_equals_d_is_mobius(d):
    v = np.random.default_rng(d).standard_normal(1 << d)
    masks = oracle.output_masks(d, d)
    assert masks.size == 1 << d
    assert np.max(np.abs(oracle.fsi(v, d, d) - oracle.mobius_direct(v)[masks])) < 1e-12


def test_l_additive_recovered_exactly():
    for l in (2, 3, 4):
        g = games.planted_game(10, 30, l, games.rng_for(91, l))
        v = games.planted_values(g)
        E = oracle.fsi(v, 10, l)
        a = oracle.mobius_direct(v)
        assert np.max(np.abs(E - a[oracle.output_masks(10, l)])) < 1e-12


@pytest.mark.parametrize("d", [2, 5, 8])
def test_l1_is_shapley_eq1(d):
    v = np.random.default_rng(7 + d).standard_normal(1 << d)
    E = oracle.fsi(v, d, 1)
    assert abs(E[0] - v[0]) < 1e-15
    assert np.max(np.abs(E[1:] - P.shapley_eq1(v, d))) < 1e-12


# ---------------------------------------------------------------- P5 invariants
def test_invariants():
    rng = np.random.default_rng(5)
    d = 9
    v = rng.standard_normal(1 << d)
    w = rng.standard_normal(1 << d)
    for l in (1, 2, 4, 9):
        E = oracle.fsi(v, d, l)
        assert E[0] == v[0]                                   # E_empty = v(empty)
        assert abs(E.sum() - v[-1]) < 1e-11                    # efficiency
        Ew = oracle.fsi(w, d, l)
        assert np.max(np.abs(oracle.fsi(2 * v - 3 * w, d, l) - (2 * E - 3 * Ew))) < 1e-11
    # permutation equivariance
    perm = rng.permutation(d)
    S = np.arange(1 << d)
    Sp = np.zeros_like(S)
    for i in range(d):
        Sp |= ((S >> i) & 1) << perm[i]
    vp = np.empty_like(v)
    vp[Sp] = v                                                # feature i -> perm[i]
    l = 3
    E = oracle.fsi(v, d, l)
    Ep = oracle.fsi(vp, d, l)
    masks = oracle.output_masks(d, l)
    pos = {int(m): k for k, m in enumerate(masks)}
    for k, m in enumerate(masks):
        mp = 0
        for i in range(d):
            if (int(m) >> i) & 1:
                mp |= 1 << int(perm[i])
        assert abs(Ep[pos[mp]] - E[k]) < 1e-11
    # symmetric game: v depends only on |S| -> equal scores within each size
    f = rng.standard_normal(d + 1)
    pc = np.array([bin(int(x)).count("1") for x in S])
    Es = oracle.fsi(f[pc], d, l)
    sizes = np.array([bin(int(m)).count("1") for m in masks])
    for s in range(l + 1):
        grp = Es[sizes == s]
        assert np.max(grp) - np.min(grp) < 1e-11


# ---------------------------------------------------------------- P6 exact integers
@pytest.mark.parametrize("d,l", [(10, 2), (12, 4), (14, 3)])
def test_pm1_exact_integer(d, l):
    v = games.pm1_values(d, games.rng_for(92, d))
    ref = P.fsi_exact_int(v.astype(np.int64), d, l)
    E = oracle.fsi(v, d, l)
    # The only error left is the oracle's FP64 summation: per output, at most
    # n*u*sum_T |W a(T)| with n = 2^(d-|S|) terms (recursive summation bound).
    a = oracle.mobius_direct(v) if d <= 10 else oracle.mobius(v)
    W = oracle.weight_table_f64(d, l)
    pc = np.array([bin(i).count("1") for i in range(1 << d)])
    u = np.finfo(np.float64).eps / 2
    for k, S in enumerate(oracle.output_masks(d, l)):
        S = int(S)
        s = bin(S).count("1")
        T = oracle.superset_masks(S, d)
        bound = (T.size + 1) * u * np.sum(np.abs(W[s, pc[T]] * a[T]))
        assert abs(E[k] - ref[k]) <= bound + 1e-300, (S, E[k] - ref[k], bound)
    assert normwise(E, ref) < 1e-11


# ---------------------------------------------------------------- P8 structure
def test_fig1_state_counts():
    assert [len(P.mpo_states(k, 2)) for k in range(4)] == [1, 3, 6, 9]


@pytest.mark.parametrize("d,l,dmax", [(8, 2, 24), (14, 3, 54), (20, 4, 95)])
def test_bond_dimension(d, l, dmax):
    D = [len(P.mpo_states(k, l)) for k in range(d + 1)]
    assert max(D) == dmax
    for k, Dk in enumerate(D):
        assert Dk <= (min(k, l) + 1) * (k + 1)


def test_core_nnz():
    cores = P.mpo_cores(8, 3)
    for k, G in enumerate(cores, start=1):
        assert np.count_nonzero(G) <= 3 * G.shape[0]


@pytest.mark.parametrize("d,l", [(3, 2), (5, 2), (6, 3), (8, 2), (8, 5)])
def test_mpo_sweep_matches_closed_form(d, l):
    v = np.random.default_rng(d + 10 * l).standard_normal(1 << d)
    E = oracle.fsi(v, d, l)
    assert normwise(P.fsi_via_mpo(v, d, l), E) < 1e-12
    assert normwise(P.fsi_via_mpo(v, d, l, precontract=True), E) < 1e-12


# ---------------------------------------------------------------- bookkeeping
@pytest.mark.parametrize("d,l,M", [(8, 2, 37), (14, 3, 470), (20, 2, 211), (20, 4, 6196)])
def test_num_outputs(d, l, M):
    assert oracle.num_outputs(d, l) == M


def test_output_order():
    m = oracle.output_masks(6, 3)
    pc = [bin(int(x)).count("1") for x in m]
    assert pc == sorted(pc)
    for s in range(4):
        grp = [int(x) for x, p in zip(m, pc) if p == s]
        assert grp == sorted(grp) and len(grp) == comb(6, s)


@pytest.mark.parametrize("d,l", [(8, 2), (11, 4), (14, 3)])
def test_c_twin_matches_python(d, l):
    v = np.random.default_rng(d).standard_normal(1 << d)
    assert normwise(oracle.fsi_c(v, d, l), oracle.fsi(v, d, l)) < 1e-13
    assert normwise(oracle.fsi_c(v, d, l, nthreads=4), oracle.fsi(v, d, l)) < 1e-13


def test_generators_match_direct_definition():
    g = games.tree_game(9, 7, 5, games.rng_for(93, 0))
    assert np.array_equal(games.tree_values(g), games.tree_values_direct(g))
    p = games.planted_game(9, 25, 6, games.rng_for(93, 1))
    assert np.array_equal(games.planted_values(p), games.planted_values_direct(p))
    # seeded reproducibility
    assert np.array_equal(games.d14_tree(0)[1], games.d14_tree(0)[1])


# ---------------------------------------------------------------- mutation check
def _pins_pass(fsi_fn):
    """Run a representative subset of the pins against a candidate oracle."""
    ok = True
    meta, rows = load_golden("worked_d3_l2_unanimity.txt")
    v = np.array([1.0 if (S & 7) == 7 else 0.0 for S in range(8)])
    ok &= normwise(fsi_fn(v, 3, 2), [float(x) for _, x in rows]) < 1e-12
    for d in (5, 7):
        vn = np.random.default_rng(d).standard_normal(1 << d)
        for l in (1, 2, 3):
            ok &= normwise(fsi_fn(vn, d, l), P.fsi_wls(vn, d, l)) < 1e-9
    g, vt = games.d14_tree(0)
    ok &= normwise(fsi_fn(vt, 14, 3),
                   P.fsi_sparse_mobius(P.tree_mobius_terms(g).items(), 14, 3)) < 1e-12
    return bool(ok)


def test_pins_catch_planted_oracle_mistakes(monkeypatch):
    from oracle import fsi_oracle as F
    assert _pins_pass(F.fsi)
    real_w = F.weight_exact
    real_mob = F.mobius
    mutants = {
        "weight sign": lambda s, t, l: -real_w(s, t, l),
        "weight t-1 -> t": lambda s, t, l: real_w(s, t + 1, l),
        "drop s/(l+s)": lambda s, t, l: real_w(s, t, l) * Fraction(l + s, s) if s else real_w(s, t, l),
    }
    for name, fn in mutants.items():
        monkeypatch.setattr(F, "weight_exact", fn)
        assert not _pins_pass(F.fsi), name
        monkeypatch.setattr(F, "weight_exact", real_w)

    def mob_plus(v):  # butterfly with + instead of - (a zeta transform)
        a = np.array(v, dtype=np.float64, copy=True)
        d = a.size.bit_length() - 1
        for i in range(d):
            view = a.reshape(-1, 2, 1 << i)
            view[:, 1, :] += view[:, 0, :]
        return a

    def mob_skip_bit(v):  # one bit axis forgotten
        a = np.array(v, dtype=np.float64, copy=True)
        d = a.size.bit_length() - 1
        for i in range(1, d):
            view = a.reshape(-1, 2, 1 << i)
            view[:, 1, :] -= view[:, 0, :]
        return a

    for name, fn in {"mobius sign": mob_plus, "mobius bit": mob_skip_bit}.items():
        monkeypatch.setattr(F, "mobius", fn)
        assert not _pins_pass(F.fsi), name
        monkeypatch.setattr(F, "mobius", real_mob)

    real_sup = F.superset_masks

    def subsets_instead(S, d):  # transposed operand: subsets instead of supersets
        out, T = [], S
        while True:
            out.append(T)
            if T == 0:
                break
            T = (T - 1) & S
        return np.array(sorted(out), dtype=np.int64)

    monkeypatch.setattr(F, "superset_masks", subsets_instead)
    assert not _pins_pass(F.fsi)
    monkeypatch.setattr(F, "superset_masks", real_sup)


@pytest.mark.parametrize("d,l", [(6, 6), (10, 2), (12, 4), (14, 3)])
def test_exact_int_oracle_matches_pin(d, l):
    v = np.random.default_rng(d + l).integers(-5, 6, size=1 << d)
    ref = P.fsi_exact_int(v.astype(np.int64), d, l)
    assert np.array_equal(oracle.fsi_exact_int(v, d, l), ref)
    assert np.array_equal(oracle.fsi_exact_int(v, d, l, nthreads=4), ref)


# ---------------------------------------------------------------------------
# oracle/closed_forms.py: the sparse-Moebius closed forms used for the
# 256-instance d = 20 check, pinned against the brute-force oracle on the
# game's values and against the term-by-term derivation in pins_lib
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("d,l,depth", [(8, 2, 4), (10, 3, 5), (12, 4, 6), (11, 1, 6)])
def test_closed_form_tree_games(d, l, depth):
    from oracle import closed_forms as CF
    g = games.tree_game(d, 25, depth, games.rng_for(77, 10 * d + l))
    v = games.tree_values(g)
    masks, coefs = CF.tree_mobius_sparse(g)
    dense = np.zeros(1 << d)
    dense[masks] = coefs
    # the path-product Moebius coefficients are the Moebius transform of v
    assert np.max(np.abs(dense - oracle.mobius(v))) < 1e-12 * max(1.0, np.max(np.abs(v)))
    # the closed form equals the brute-force oracle on v
    E = CF.fsi_from_sparse_mobius(masks, coefs, d, l)
    ref = oracle.fsi(v, d, l)
    assert np.max(np.abs(E - ref)) <= 1e-13 * np.max(np.abs(ref))
    # and the independent derivation of the same facts
    E2 = P.fsi_sparse_mobius(list(P.tree_mobius_terms(g).items()), d, l)
    assert np.max(np.abs(E - E2)) <= 1e-13 * np.max(np.abs(ref))
    # efficiency: sum of E over |S| <= l equals v(full set)
    assert abs(E.sum() - v[-1]) <= 1e-12 * max(1.0, abs(v[-1]))


@pytest.mark.parametrize("d,l,kmax", [(8, 2, 4), (12, 3, 6), (14, 4, 6)])
def test_closed_form_planted_games(d, l, kmax):
    from oracle import closed_forms as CF
    g = games.planted_game(d, 60, kmax, games.rng_for(78, 10 * d + l))
    v = games.planted_values(g)
    masks, coefs = CF.planted_mobius_sparse(g)
    E = CF.fsi_from_sparse_mobius(masks, coefs, d, l)
    ref = oracle.fsi(v, d, l)
    assert np.max(np.abs(E - ref)) <= 1e-13 * np.max(np.abs(ref))
    E2 = P.fsi_sparse_mobius(list(zip(g.masks, g.coefs)), d, l)
    assert np.max(np.abs(E - E2)) <= 1e-13 * np.max(np.abs(ref))


def test_closed_form_catches_a_wrong_weight(monkeypatch):
    """A plausible slip in the closed form (a weight of the wrong order, a
    dropped Moebius term) fails the brute-force comparison."""
    from oracle import closed_forms as CF
    d, l = 10, 3
    g = games.tree_game(d, 25, 5, games.rng_for(79, 0))
    v = games.tree_values(g)
    masks, coefs = CF.tree_mobius_sparse(g)
    ref = oracle.fsi(v, d, l)
    real = CF._weight_f64
    CF._weight_f64.cache_clear()
    monkeypatch.setattr(CF, "_weight_f64", lambda s, t, ll: real(s, t, ll + 1) if t > ll + 1 else 0.0)
    bad = CF.fsi_from_sparse_mobius(masks, coefs, d, l)
    assert np.max(np.abs(bad - ref)) > 1e-6 * np.max(np.abs(ref))
    monkeypatch.undo()
    keep = CF._popcount64(masks) > l
    bad2 = CF.fsi_from_sparse_mobius(masks[keep], coefs[keep], d, l)
    assert np.max(np.abs(bad2 - ref)) > 1e-6 * np.max(np.abs(ref))
