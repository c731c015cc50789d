"""Pins of the oracle's other cardinal interaction indices (Appendix A: SII,
k-SII, STII, BII) against their discrete-derivative definitions, evaluated
term by term in exact rationals. None of these references use the Moebius
transform or the superset-weight tables of the oracle.

  * SII   (Appendix A): sum over T in the complement of S of
          |T|! (d-|S|-|T|)! / (d-|S|+1)! * Delta_S v(T).
  * BII   (Appendix A, "uniform weighting"): the plain mean of Delta_S v(T)
          over the 2^(d-|S|) coalitions T of the complement.
  * STII  (Sundararajan et al., the definition Appendix A cites): below the
          top order Delta_S v(empty); at |S| = l,
          (l/d) * sum over T in the complement of Delta_S v(T) / C(d-1, |T|).
  * k-SII (the aggregation Appendix A describes): the SII of S plus the SII
          of every superset S u W (W in the complement, |W| = j <= l - |S|)
          weighted by the Bernoulli number B_j.

with Delta_S v(T) = sum over R subset of S of (-1)^{|S|-|R|} v(T u R).
"""
from __future__ import annotations

from fractions import Fraction
from math import comb, factorial

import numpy as np
import pytest

import oracle
from helpers import normwise
import pins_lib as P

pytestmark = pytest.mark.filterwarnings("ignore")

# Textbook Bernoulli numbers (B_1 = -1/2 convention).
TEXTBOOK_B = {0: Fraction(1), 1: Fraction(-1, 2), 2: Fraction(1, 6), 3: Fraction(0),
              4: Fraction(-1, 30), 5: Fraction(0), 6: Fraction(1, 42), 7: Fraction(0),
              8: Fraction(-1, 30), 10: Fraction(5, 66), 12: Fraction(-691, 2730),
              14: Fraction(7, 6)}


def _pc(x):
    return bin(x).count("1")


def _delta(v, S, T):
    acc = 0
    R = S
    while True:
        sgn = -1 if (_pc(S) - _pc(R)) % 2 else 1
        acc += sgn * v[T | R]
        if R == 0:
            return acc
        R = (R - 1) & S


def _complement_sets(S, d):
    return [T for T in range(1 << d) if T & S == 0]


def sii_def(v, S, d):
    s = _pc(S)
    return sum(Fraction(factorial(_pc(T)) * factorial(d - s - _pc(T)), factorial(d - s + 1))
               * _delta(v, S, T) for T in _complement_sets(S, d))


def bii_def(v, S, d):
    s = _pc(S)
    return Fraction(sum(_delta(v, S, T) for T in _complement_sets(S, d)), 1 << (d - s))


def stii_def(v, S, d, l):
    if _pc(S) < l:
        return Fraction(_delta(v, S, 0))
    return Fraction(l, d) * sum(Fraction(_delta(v, S, T), comb(d - 1, _pc(T)))
                                for T in _complement_sets(S, d))


def ksii_def(v, S, d, l):
    if S == 0:
        return Fraction(v[0])
    s = _pc(S)
    acc = Fraction(0)
    for W in _complement_sets(S, d):
        j = _pc(W)
        if j <= l - s and TEXTBOOK_B[j] != 0:
            acc += TEXTBOOK_B[j] * sii_def(v, S | W, d)
    return acc


DEFS = {
    "sii": lambda v, S, d, l: sii_def(v, S, d),
    "bii": lambda v, S, d, l: bii_def(v, S, d),
    "stii": stii_def,
    "ksii": ksii_def,
}


def _int_game(d, seed):
    return [int(x) for x in np.random.default_rng(seed).integers(-9, 10, size=1 << d)]


def test_bernoulli_numbers_textbook():
    B = oracle.bernoulli_exact(14)
    for j, b in TEXTBOOK_B.items():
        assert B[j] == b, j


@pytest.mark.parametrize("index", ["sii", "bii", "stii", "ksii"])
@pytest.mark.parametrize("d,l", [(4, 2), (5, 3), (6, 2), (6, 4)])
def test_index_matches_discrete_derivative_definition(index, d, l):
    v = _int_game(d, 100 * d + l)
    masks = [int(m) for m in oracle.output_masks(d, l)]
    want = np.array([float(DEFS[index](v, S, d, l)) for S in masks])
    got = oracle.interaction(np.array(v, dtype=np.float64), d, l, index)
    assert normwise(got, want) < 1e-13


@pytest.mark.parametrize("index", ["sii", "bii", "stii", "ksii"])
def test_index_exact_weights_match_definition_exactly(index):
    """Exact rationals end to end: sum_T W(s,|T|) a(T) with the oracle's exact
    weights and a exact Moebius by definition equals the definition."""
    d, l = 5, 3
    v = _int_game(d, 7)
    a = P._mobius_by_definition(np.array(v, dtype=np.float64), d)
    for S in [int(m) for m in oracle.output_masks(d, l)]:
        s = _pc(S)
        val = sum(oracle.index_weight_exact(index, s, _pc(T), l) * int(round(a[T]))
                  for T in range(1 << d) if T & S == S)
        assert val == DEFS[index](v, S, d, l), (index, S)


@pytest.mark.parametrize("d", [5, 7])
def test_order_one_reduces_to_shapley(d):
    v = np.random.default_rng(d).standard_normal(1 << d)
    phi = P.shapley_eq1(v, d)
    for index in ("stii", "ksii", "fsi"):
        out = oracle.interaction(v, d, 1, index)
        assert abs(out[0] - v[0]) < 1e-14
        assert normwise(out[1:], phi) < 1e-13, index
    # SII singletons are Shapley values at every order
    for l in (2, 3):
        out = oracle.interaction(v, d, l, "sii")
        assert normwise(out[1:1 + d], phi) < 1e-13


@pytest.mark.parametrize("d,l", [(6, 2), (8, 3), (9, 4)])
def test_efficiency_of_stii_and_ksii(d, l):
    v = np.random.default_rng(d * l).standard_normal(1 << d)
    for index in ("stii", "ksii"):
        out = oracle.interaction(v, d, l, index)
        assert abs(out.sum() - v[-1]) < 1e-11 * max(1.0, np.abs(v).max()), index
    # SII is not efficient above order 1 (Appendix A)
    assert abs(oracle.interaction(v, d, l, "sii").sum() - v[-1]) > 1e-6


def test_ksii_top_order_is_sii():
    d, l = 7, 3
    v = np.random.default_rng(3).standard_normal(1 << d)
    k = oracle.interaction(v, d, l, "ksii")
    s = oracle.interaction(v, d, l, "sii")
    top = oracle.num_outputs(d, l - 1)
    assert normwise(k[top:], s[top:]) < 1e-14


def test_stii_below_top_order_is_moebius():
    d, l = 7, 3
    v = np.random.default_rng(4).standard_normal(1 << d)
    a = oracle.mobius(v)
    out = oracle.interaction(v, d, l, "stii")
    masks = oracle.output_masks(d, l)
    below = oracle.num_outputs(d, l - 1)
    assert np.max(np.abs(out[:below] - a[masks[:below]])) < 1e-13


def test_fsi_through_interaction_equals_fsi():
    d, l = 9, 3
    v = np.random.default_rng(5).standard_normal(1 << d)
    assert np.array_equal(oracle.interaction(v, d, l, "fsi"), oracle.fsi(v, d, l))


def test_c_twin_index_tables():
    d, l = 10, 4
    v = np.random.default_rng(6).standard_normal(1 << d)
    for index in oracle.INDICES:
        assert normwise(oracle.fsi_c(v, d, l, index=index),
                        oracle.interaction(v, d, l, index)) < 1e-14


def test_unknown_index_rejected():
    with pytest.raises(ValueError):
        oracle.index_weight_exact("shap", 1, 2, 2)


# ---------------------------------------------------------------- mutation check
def _index_pins_pass(index):
    d, l = 5, 3
    v = _int_game(d, 11)
    masks = [int(m) for m in oracle.output_masks(d, l)]
    want = np.array([float(DEFS[index](v, S, d, l)) for S in masks])
    return normwise(oracle.interaction(np.array(v, dtype=np.float64), d, l, index), want) < 1e-13


def test_index_pins_catch_planted_mistakes(monkeypatch):
    from oracle import fsi_oracle as F
    for index in ("sii", "bii", "stii", "ksii"):
        assert _index_pins_pass(index)
    real_b = F.bernoulli_exact
    real_w = F.index_weight_exact

    def b1_plus(n):  # the other B_1 convention
        B = real_b(n)
        B[1] = -B[1]
        return B

    monkeypatch.setattr(F, "bernoulli_exact", b1_plus)
    assert not _index_pins_pass("ksii")
    monkeypatch.setattr(F, "bernoulli_exact", real_b)

    mutants = {
        "sii": lambda i, s, t, l: Fraction(1, t - s + 2) if i == "sii" else real_w(i, s, t, l),
        "bii": lambda i, s, t, l: Fraction(1, 1 << t) if i == "bii" else real_w(i, s, t, l),
        "stii": lambda i, s, t, l: (Fraction(1, t - s + 1) if (i == "stii" and s == l)
                                    else real_w(i, s, t, l)),
        "ksii": lambda i, s, t, l: (real_w("sii", s, t, l) if (i == "ksii" and s >= 1)
                                    else real_w(i, s, t, l)),
    }
    for index, fn in mutants.items():
        monkeypatch.setattr(F, "index_weight_exact", fn)
        assert not _index_pins_pass(index), index
        monkeypatch.setattr(F, "index_weight_exact", real_w)


@pytest.mark.parametrize("index", ["fsi", "stii", "ksii"])
def test_from_mobius_unanimity_closed_form(index):
    """Given Moebius coefficients a = delta_A, the scores are the index's
    weights on the subsets of A: for FSI the unanimity closed form (Eq. 3 +
    Eq. 4, exact rationals), for all indices the definition-based pins."""
    d, l = 7, 3
    rng = np.random.default_rng(17)
    for A in [0b1011, 0b1110110, 0b101]:
        a = np.zeros(1 << d)
        a[A] = 1.0
        out = oracle.interaction_from_mobius(a, d, l, index)
        if index == "fsi":
            assert np.max(np.abs(out - P.fsi_unanimity(A, d, l))) < 1e-15
        v = np.array([1.0 if (S & A) == A else 0.0 for S in range(1 << d)])
        assert normwise(out, oracle.interaction(v, d, l, index)) < 1e-15
    # linear: a random a gives the value vector's scores when v is its zeta transform
    a = rng.standard_normal(1 << d)
    v = np.array([sum(a[T] for T in range(1 << d) if T & S == T) for S in range(1 << d)])
    assert normwise(oracle.interaction_from_mobius(a, d, l, index),
                    oracle.interaction(v, d, l, index)) < 1e-12


def test_from_mobius_c_twin():
    d, l = 11, 4
    a = np.random.default_rng(18).standard_normal(1 << d)
    for index in ("fsi", "sii"):
        assert normwise(oracle.interaction_from_mobius_c(a, d, l, index),
                        oracle.interaction_from_mobius(a, d, l, index)) < 1e-14
