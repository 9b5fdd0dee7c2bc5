"""Pins of the limb-format oracle (oracle/limbs.py) against the mathematics.

* RN_p: at p = 53 it must equal Python's correctly rounded float(Fraction),
  ties to even included.
* RN_p(a - c): at p = 53 it must equal IEEE binary64 subtraction (correctly
  rounded by the standard).
* (S2)+(S3): the slices rebuild the fixed-point value and lie in the
  balanced ranges; the textbook CRT of all residues rebuilds every slice.
* end to end, every digit group kept (g0 = 0): the product equals RN_p of
  the exact dot product of the truncated fixed-point inputs (a plain
  definition, computed here with Fractions and floor).
* end to end, default groups: the error against the exact product stays
  within the bound of Prop. 2 plus the input truncation, also at p = 4096
  (S = 24), and the update mode subtracts the rounded product.
"""
import math
import random
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import oracle.limbs as OL
import workloads as W


def textbook_crt(res, moduli):
    P = math.prod(moduli)
    x = 0
    for r, m in zip(res, moduli):
        Mi = P // m
        x += int(r) * Mi * pow(Mi, -1, m)
    x %= P
    return x - P if x > P // 2 else x


def frac_of(t):
    s, m, e = t
    if m == 0:
        return Fraction(0)
    v = Fraction(m) * Fraction(2) ** (e - 53)
    return -v if s else v


def test_rn_int_matches_correct_rounding_at_53_bits():
    rnd = random.Random(7)
    cases = [(1 << 60) + (1 << 7), (1 << 60) + (3 << 7), (1 << 60) + (1 << 7) + 1,
             (1 << 53) - 1, (1 << 53) + 1, (1 << 54) - 1, 12345]
    cases += [rnd.getrandbits(rnd.randint(1, 200)) for _ in range(300)]
    for v in cases:
        for sgn in (1, -1):
            for eps in (-300, -7, 0, 11):
                got = frac_of(OL.rn_int(sgn * v, eps, 53))
                want = Fraction(float(Fraction(sgn * v) * Fraction(2) ** eps))
                assert got == want, (v, sgn, eps)


def test_sub_rn_matches_binary64_subtraction():
    rnd = random.Random(11)
    for _ in range(2000):
        a = rnd.uniform(-1, 1) * 2.0 ** rnd.randint(-40, 40)
        c = a * (1 + rnd.uniform(-1e-9, 1e-9)) if rnd.random() < 0.3 else \
            rnd.uniform(-1, 1) * 2.0 ** rnd.randint(-60, 60)
        ta = OL.rn_fraction(Fraction(a), 53)
        tc = OL.rn_fraction(Fraction(c), 53)
        assert frac_of(ta) == Fraction(a) and frac_of(tc) == Fraction(c)
        got = frac_of(OL.sub_rn(ta, tc, 53))
        assert got == Fraction(a - c), (a, c)


def test_slices_rebuild_and_are_balanced():
    rnd = random.Random(3)
    for _ in range(200):
        S, w = rnd.randint(1, 6), rnd.randint(8, 80)
        X = rnd.getrandbits(S * w - 1) * rnd.choice((1, -1))
        v = OL.slices(X, S, w)
        assert sum(x << (w * t) for t, x in enumerate(v)) == X
        for x in v[:-1]:
            assert -(1 << (w - 1)) <= x < (1 << (w - 1))
        assert abs(v[-1]) <= (1 << (w - 1)) + 1


@pytest.mark.parametrize("nl,K", [(2, 6), (4, 5)])
def test_residues_rebuild_slices(nl, K):
    rng = np.random.default_rng(5)
    A = W.random_limbs(3, K, nl, rng, exp_sigma=3.0, zero_frac=0.1)
    pl = O.make_plan(64 * nl, K)
    ea = OL.exponents(A, True)
    res = OL.residues(A, True, ea, pl)
    p = 64 * nl
    for i in range(3):
        for h in range(K):
            s, m, e = OL.parts(A, i, h)
            X = OL.fixed_point(s, m, e, pl.Q - 1 - int(ea[i]), p) if m else 0
            v = OL.slices(X, pl.S, pl.w)
            for t in range(pl.S):
                assert textbook_crt(res[t, :, i, h], pl.moduli) == v[t]


def _operands(nl, M, N, K, seed, sigma=3.0):
    rng = np.random.default_rng(seed)
    A = W.random_limbs(M, K, nl, rng, exp_sigma=sigma, zero_frac=0.05)
    B = W.random_limbs(K, N, nl, rng, exp_sigma=sigma, zero_frac=0.05)
    return A, B


def _zeros(nl, M, N):
    return (np.zeros((nl, N, M), np.uint64), np.full((N, M), OL.EXP_ZERO, np.int32),
            np.zeros((N, M), np.uint8))


@pytest.mark.parametrize("nl,S", [(2, 2), (4, 3)])
def test_all_groups_equal_rounded_truncated_dot(nl, S):
    M, N, K = 4, 3, 7
    p = 64 * nl
    base = O.make_plan(p, K, nslice=S)
    pl = O.make_plan(p, K, nslice=S, extra_groups=S - 1)
    assert pl.g0 == 0 and pl.S == base.S
    A, B = _operands(nl, M, N, K, 21)
    C, prods = OL.ozgemm(0, A, B, _zeros(nl, M, N), pl)
    ea, eb = OL.exponents(A, True), OL.exponents(B, False)

    def trunc(x: Fraction, mu: int) -> int:
        q = x * Fraction(2) ** mu
        return math.floor(q) if q >= 0 else -math.floor(-q)

    for i in range(M):
        for j in range(N):
            if ea[i] == OL.EXP_ZERO or eb[j] == OL.EXP_ZERO:
                assert prods[(i, j)][1] == 0
                continue
            mu, nu = pl.Q - 1 - int(ea[i]), pl.Q - 1 - int(eb[j])
            s = sum(trunc(OL.value(A, i, h), mu) * trunc(OL.value(B, h, j), nu) for h in range(K))
            want = OL.rn_fraction(Fraction(s) * Fraction(2) ** (-mu - nu), p)
            assert prods[(i, j)] == want, (i, j)
            assert OL.parts(C, i, j) == (want[0], want[1], want[2]) if want[1] else True


@pytest.mark.parametrize("nl,K,S", [(2, 9, 0), (4, 6, 3), (64, 4, 0)])
def test_error_within_prop2_bound(nl, K, S):
    M, N = 3, 2
    p = 64 * nl
    pl = O.make_plan(p, K, nslice=S)
    if nl == 64:
        assert pl.S == 24 and pl.w == 172
    A, B = _operands(nl, M, N, K, 33 + nl)
    C, prods = OL.ozgemm(0, A, B, _zeros(nl, M, N), pl)
    ea, eb = OL.exponents(A, True), OL.exponents(B, False)
    for i in range(M):
        for j in range(N):
            exact = OL.exact_product(A, B, i, j)
            got = OL.value(C, i, j)
            if ea[i] == OL.EXP_ZERO or eb[j] == OL.EXP_ZERO:
                assert got == 0
                continue
            # inputs truncated by < 1 unit of 2^-mu each; the dropped groups
            # are bounded by (S-1) 2^(Q-1) units of 2^-(mu+nu) (Prop. 2); one
            # final rounding at p bits.
            unit = Fraction(2) ** (int(ea[i]) + int(eb[j]) - 2 * pl.Q + 2)
            trunc_in = 2 * K * 2 ** pl.Q * unit
            dropped = (pl.S - 1) * 2 ** (pl.Q - 1) * unit
            bound = trunc_in + dropped + abs(exact) * Fraction(1, 2 ** (p - 1))
            assert abs(got - exact) <= bound


def test_update_mode_subtracts_rounded_product():
    nl, M, N, K = 2, 3, 3, 5
    p = 64 * nl
    pl = O.make_plan(p, K)
    A, B = _operands(nl, M, N, K, 44)
    rng = np.random.default_rng(45)
    C0 = W.random_limbs(M, N, nl, rng, exp_sigma=2.0, zero_frac=0.1)
    C1, prods = OL.ozgemm(1, A, B, C0, pl)
    for i in range(M):
        for j in range(N):
            s, m, e = prods[(i, j)]
            c = Fraction(0) if m == 0 else Fraction(m) * Fraction(2) ** (e - p) * (-1 if s else 1)
            want = OL.rn_fraction(OL.value(C0, i, j) - c, p)
            got = OL.parts(C1, i, j)
            if want[1] == 0:
                assert got[1] == 0
            else:
                assert got == want


def test_lotkin_entries_are_rounded_reciprocals():
    L = W.lotkin_limbs(5, 4)
    for i in range(5):
        for j in range(5):
            d = 1 if i == 0 else i + j + 1
            assert OL.parts(L, i, j) == OL.rn_fraction(Fraction(1, d), 256)


def test_rn_fraction_matches_correct_rounding_at_53_bits():
    rnd = random.Random(13)
    for _ in range(3000):
        x = Fraction(rnd.getrandbits(rnd.randint(1, 150)) + 1, rnd.getrandbits(rnd.randint(1, 150)) + 1)
        x *= Fraction(2) ** rnd.randint(-50, 50)
        for sgn in (1, -1):
            got = frac_of(OL.rn_fraction(sgn * x, 53))
            assert got == Fraction(float(sgn * x)), x
    # exact halfway cases round to even
    for m in range(1 << 52, (1 << 52) + 64):
        x = Fraction(2 * m + 1, 2)
        assert frac_of(OL.rn_fraction(x, 53)) == Fraction(float(x))


def test_limb_generators_return_the_device_layout():
    """Limb matrices go to the device as flat copies addressed plane by plane
    (limb q of element (i, j) at q rows cols + i + j rows), so the seeded
    generators must hand out C-contiguous (nlimb, cols, rows) arrays."""
    for L in (W.lotkin_limbs(9, 3), W.random_limbs(5, 7, 3, np.random.default_rng(1))):
        limb, ex, sg = L
        assert all(x.flags["C_CONTIGUOUS"] for x in L)
        flat = limb.reshape(-1)
        nl, cols, rows = limb.shape
        for q, j, i in ((0, 0, 0), (nl - 1, cols - 1, rows - 1), (1, 2, 3)):
            assert flat[q * rows * cols + i + j * rows] == limb[q, j, i]
