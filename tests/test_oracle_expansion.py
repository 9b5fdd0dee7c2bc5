"""Pins of the oracle's expansion arithmetic against exact rational results.

The arithmetic follows a written specification (error-free transforms,
renormalisation, merge, long division); what pins it is the mathematics: every
result must match the exact rational value within the precision of the
format, exact cases must come out exact, and the operations must have the
algebraic symmetries of the exact ones.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import workloads as W


def F(x):
    return sum((Fraction(float(v)) for v in np.ravel(x)), Fraction(0))


def _rel_errs(got, exact):
    out = []
    for g, e in zip(got, exact):
        if e != 0:
            out.append(abs(float((F(g) - e) / e)))
    return max(out)


@pytest.mark.parametrize("nc", [2, 3, 4])
def test_accuracy_vs_fractions(nc):
    rng = np.random.default_rng(11 + nc)
    a = W.random_expansions(40, 20, nc, rng, exp_sigma=4).reshape(-1, nc)
    b = W.random_expansions(40, 20, nc, rng, exp_sigma=4).reshape(-1, nc)
    c = W.random_expansions(40, 20, nc, rng, exp_sigma=4).reshape(-1, nc)
    Fa = [F(x) for x in a]
    Fb = [F(x) for x in b]
    Fc = [F(x) for x in c]
    bound = 2.0 ** (-(53 * nc - 4))
    assert _rel_errs(O.exp_add(a, b), [x + y for x, y in zip(Fa, Fb)]) < bound
    assert _rel_errs(O.exp_mul(a, b), [x * y for x, y in zip(Fa, Fb)]) < bound
    assert _rel_errs(O.exp_div(a, b), [x / y for x, y in zip(Fa, Fb)]) < bound
    # fms has two roundings; relative to the larger of |c| and |a b|
    r = O.exp_fms(c, a, b)
    for ri, x, y, z in zip(r, Fa, Fb, Fc):
        scale = max(abs(z), abs(x * y))
        assert abs(F(ri) - (z - x * y)) <= scale * bound


@pytest.mark.parametrize("nc", [2, 3, 4])
def test_cancellation_is_exact(nc):
    rng = np.random.default_rng(5)
    a = W.random_expansions(30, 10, nc, rng, exp_sigma=2).reshape(-1, nc)
    # a + (-a) = 0 exactly; a - (a with a perturbed last component) = that perturbation
    z = O.exp_add(a, -a)
    assert np.all(z == 0.0)
    b = a.copy()
    b[:, -1] = 0.0
    d = O.exp_add(a, -b)
    for di, ai in zip(d, a):
        assert F(di) == Fraction(float(ai[-1]))


@pytest.mark.parametrize("nc", [2, 3, 4])
def test_exact_cases_and_symmetries(nc):
    rng = np.random.default_rng(7)
    a = W.random_expansions(25, 8, nc, rng, exp_sigma=3).reshape(-1, nc)
    b = W.random_expansions(25, 8, nc, rng, exp_sigma=3).reshape(-1, nc)
    # multiplication by a power of two and by one is exact
    two = np.zeros_like(a)
    two[:, 0] = 2.0 ** 7
    assert all(F(x) == F(y) * 128 for x, y in zip(O.exp_mul(a, two), a))
    one = np.zeros_like(a)
    one[:, 0] = 1.0
    assert np.array_equal(O.exp_div(a, one), O.exp_mul(a, one))
    # commutativity of add (the merge network is symmetric), sign symmetry
    assert np.array_equal(O.exp_add(a, b), O.exp_add(b, a))
    assert np.array_equal(O.exp_mul(-a, b), -O.exp_mul(a, b))
    assert np.array_equal(O.exp_add(-a, -b), -O.exp_add(a, b))
    # small integers are exact
    ia = np.zeros_like(a)
    ib = np.zeros_like(a)
    ia[:, 0] = rng.integers(-1000, 1000, size=len(a))
    ib[:, 0] = rng.integers(1, 1000, size=len(a))
    assert all(F(x) == F(y) * F(z) for x, y, z in zip(O.exp_mul(ia, ib), ia, ib))
    assert all(F(x) == F(y) + F(z) for x, y, z in zip(O.exp_add(ia, ib), ia, ib))


def test_division_of_rationals():
    # 1/3, 1/7 ... to QD precision: compare with the exact rational
    nc = 4
    for q in (3, 7, 11, 49, 255):
        one = np.array([[1.0, 0, 0, 0]])
        d = np.array([[float(q), 0, 0, 0]])
        r = O.exp_div(one, d)
        err = abs(F(r[0]) - Fraction(1, q)) * q
        assert err < Fraction(1, 2 ** 209)


def test_pivot_order():
    # lexicographic on sign-normalised components = order of |value| for
    # canonical expansions
    a = np.array([1.0, 2.0 ** -60, 0, 0])
    b = np.array([-1.0, -2.0 ** -61, 0, 0])
    c = np.array([-1.0, 2.0 ** -61, 0, 0])
    assert O.abs_greater(a, b) and not O.abs_greater(b, a)
    assert O.abs_greater(b, c)   # |-1 - 2^-61| > |-1 + 2^-61|
    assert not O.abs_greater(a, a)
