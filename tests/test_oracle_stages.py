"""Pins of the oracle's Ozaki-II stages (S1)-(S6) against the mathematics.

* (S1) exponents: the frexp exponent of the leading component (library).
* (S2)+(S3): slices rebuilt from ALL residues by the textbook CRT must sum to
  a fixed-point value within nc units of x*2^mu (Eq. direct truncates each
  component), and must lie in the balanced ranges of Sec. 3.2.
* (S4): the modular GEMM equals numpy's exact integer matmul reduced mod m.
* (S5): CRT round trip on random integers; CRT of the t-planes equals the
  group sums obtained by brute force from the slices.
* (S6): greedy rounding equals Python's correctly rounded float(Fraction).
* end to end: S = 1 reduces to the correctly rounded exact dot product of the
  truncated inputs; for S > 1 the error against the exact product stays
  within the bound of Prop. 2 plus the conversion truncation.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import workloads as W


def F(x):
    return sum((Fraction(float(v)) for v in np.ravel(x)), Fraction(0))


def textbook_crt(res, moduli):
    P = math.prod(moduli)
    x = 0
    for r, m in zip(res, moduli):
        Mi = P // m
        x += int(r) * Mi * pow(Mi, -1, m)
    x %= P
    return x - P if x > P // 2 else x


def _operands(nc, M, N, K, seed, sigma=3.0):
    rng = np.random.default_rng(seed)
    A = W.random_expansions(M, K, nc, rng, exp_sigma=sigma)   # (K, M, nc)
    B = W.random_expansions(K, N, nc, rng, exp_sigma=sigma)   # (N, K, nc)
    A[1, 2, :] = 0.0          # scattered zeros
    B[0, 1, :] = 0.0
    return A, B


def test_exponents_match_frexp():
    A, B = _operands(4, 7, 5, 6, 1)
    ea = O.exponents(A, True)
    for i in range(7):
        want = max(math.frexp(float(A[h, i, 0]))[1] for h in range(6) if A[h, i, 0] != 0)
        assert ea[i] == want
    Z = np.zeros((3, 4, 2))
    assert np.all(O.exponents(Z, True) == O.EXP_ZERO)


@pytest.mark.parametrize("nc,S,be", [(2, 1, O.BACKEND_INT8), (3, 2, O.BACKEND_INT8),
                                     (4, 2, O.BACKEND_INT8), (4, 3, O.BACKEND_INT8),
                                     (2, 1, O.BACKEND_F64MOD), (4, 2, O.BACKEND_F64MOD)])
def test_residues_rebuild_fixed_point(nc, S, be):
    K = 16
    pl = O.make_plan(53 * nc, K, backend=be, nslice=S)
    A, _ = _operands(nc, 6, 3, K, 2 + S)
    ea = O.exponents(A, True)
    r = O.residues(A, True, ea, pl)          # [S, nmod, M, K]
    assert r.dtype == np.int32
    for l, m in enumerate(pl.moduli):
        assert r[:, l].min() >= -(m // 2) and r[:, l].max() <= (m + 1) // 2 - 1
    for i in range(6):
        mu = pl.Q - 1 - int(ea[i])
        for h in range(K):
            v = [textbook_crt(r[t, :, i, h], pl.moduli) for t in range(S)]
            for t in range(S - 1):
                assert -(2 ** (pl.w - 1)) <= v[t] < 2 ** (pl.w - 1)
            X = sum(vt << (pl.w * t) for t, vt in enumerate(v))
            exact = F(A[h, i]) * Fraction(2) ** mu
            assert abs(X - exact) < nc
            assert abs(X) <= 2 ** (pl.Q - 1) + nc
            # per-component truncation toward zero never moves away from zero
            assert X == 0 or (X > 0) == (exact > 0)


def test_modgemm_matches_numpy_matmul():
    nc, K = 4, 24
    pl = O.make_plan(212, K)
    A, B = _operands(nc, 9, 7, K, 3)
    ra = O.residues(A, True, O.exponents(A, True), pl)
    rb = O.residues(B, False, O.exponents(B, False), pl)
    tpl = O.modgemm(ra, rb, pl)
    for gi, g in enumerate(pl.groups):
        for l, m in enumerate(pl.moduli):
            C = np.zeros((9, 7), dtype=np.int64)
            for ta, tb in pl.pairs(g):
                C += ra[ta, l].astype(np.int64) @ rb[tb, l].astype(np.int64).T
            y = pow((pl.P // m) % m, -1, m)
            want = ((C % m) * y) % m
            assert np.array_equal(tpl[gi, l].T, want)


def test_crt_round_trip():
    pl = O.make_plan(212, 256)
    rng = np.random.default_rng(4)
    vals = [0, 1, -1, pl.P // 2, -(pl.P // 2) + 1]
    vals += [int.from_bytes(rng.bytes(40), "little") % pl.P - pl.P // 2 for _ in range(40)]
    M = len(vals)
    tpl = np.zeros((1, pl.nmod, 1, M), dtype=np.uint32)
    for i, X in enumerate(vals):
        for l, m in enumerate(pl.moduli):
            tpl[0, l, 0, i] = ((X % m) * pl.y[l]) % m
    out = O.crt(tpl, pl, nw=8)
    for i, X in enumerate(vals):
        assert O.limbs_to_int(out[0, 0, i]) == X


@pytest.mark.parametrize("nc,S,E", [(4, 2, 0), (3, 2, 0), (4, 3, 1)])
def test_crt_equals_bruteforce_group_sums(nc, S, E):
    K = 12
    pl = O.make_plan(53 * nc, K, nslice=S, extra_groups=E)
    A, B = _operands(nc, 5, 4, K, 5)
    ea, eb = O.exponents(A, True), O.exponents(B, False)
    ra = O.residues(A, True, ea, pl)
    rb = O.residues(B, False, eb, pl)
    sb = O.crt(O.modgemm(ra, rb, pl), pl, nw=10)
    _, sb_def = O.ozgemm(0, A, B, np.zeros((4, 5, nc)), pl, want_sbar=True, nw_out=10)
    assert np.array_equal(sb, sb_def)
    # brute force from the slices (rebuilt by the textbook CRT)
    va = [[[textbook_crt(ra[t, :, i, h], pl.moduli) for h in range(K)] for i in range(5)]
          for t in range(S)]
    vb = [[[textbook_crt(rb[t, :, j, h], pl.moduli) for h in range(K)] for j in range(4)]
          for t in range(S)]
    for gi, g in enumerate(pl.groups):
        for i in range(5):
            for j in range(4):
                want = sum(va[ta][i][h] * vb[tb][j][h] for ta, tb in pl.pairs(g) for h in range(K))
                assert O.limbs_to_int(sb[gi, j, i]) == want


def test_round_out_matches_correct_rounding():
    rng = np.random.default_rng(6)
    cases = [0, 1, -1, 2 ** 53 + 1, 2 ** 54 + 2, 2 ** 54 + 6, -(2 ** 53 + 1), 3 << 200,
             (1 << 300) + (1 << 100) + 1, -(1 << 400) + (1 << 340) - 7]
    cases += [int.from_bytes(rng.bytes(50), "little") - (1 << 399) for _ in range(60)]
    for nc in (2, 3, 4):
        for v in cases:
            for eps in (-300, -53, 0, 17):
                got = O.round_out(v, eps, nc)
                want = W.greedy_rn(Fraction(v) * Fraction(2) ** eps, nc)
                assert list(got) == want, (v, eps, nc)
    # flush rule: a component below 2^-1022 ends the expansion
    got = O.round_out((1 << 80) + 1, -1100, 4)
    assert got[0] == 2.0 ** -1020 and got[1] == 0.0


@pytest.mark.parametrize("nc,p", [(2, 106), (3, 120), (4, 150)])
def test_single_slice_is_correctly_rounded_dot(nc, p):
    K = 10
    pl = O.make_plan(p, K)
    assert pl.S == 1
    A, B = _operands(nc, 4, 3, K, 8, sigma=2.0)
    Cz = np.zeros((3, 4, nc))
    C, _ = O.ozgemm(0, A, B, Cz, pl)
    ea, eb = O.exponents(A, True), O.exponents(B, False)

    def trunc(x, mu):
        t = 0
        for c in x:
            q = Fraction(float(c)) * Fraction(2) ** mu
            t += math.floor(q) if q >= 0 else -math.floor(-q)
        return t

    for i in range(4):
        for j in range(3):
            mu = pl.Q - 1 - int(ea[i])
            nu = pl.Q - 1 - int(eb[j])
            s = sum(trunc(A[h, i], mu) * trunc(B[j, h], nu) for h in range(K))
            want = W.greedy_rn(Fraction(s) * Fraction(2) ** (-mu - nu), nc)
            assert list(C[j, i]) == want


@pytest.mark.parametrize("nc,S,E", [(4, 2, 0), (4, 3, 0), (3, 2, 0), (4, 3, 1)])
def test_error_within_prop2_bound(nc, S, E):
    K = 20
    pl = O.make_plan(53 * nc, K, nslice=S, extra_groups=E)
    A, B = _operands(nc, 6, 5, K, 9)
    C, _ = O.ozgemm(0, A, B, np.zeros((5, 6, nc)), pl)
    ea, eb = O.exponents(A, True), O.exponents(B, False)
    for i in range(6):
        for j in range(5):
            exact = sum(F(A[h, i]) * F(B[j, h]) for h in range(K))
            # inputs truncated by < nc units of 2^-mu; dropped groups bounded by
            # (S-1) 2^(Q-1) units of 2^-(mu+nu) (Prop. 2); one final rounding.
            unit = Fraction(2) ** (int(ea[i]) + int(eb[j]) - 2 * pl.Q + 2)
            trunc_in = 2 * K * nc * 2 ** pl.Q * unit
            dropped = (S - 1) * 2 ** (pl.Q - 1) * unit * (2 ** (-pl.w * E))
            bound = trunc_in + dropped + abs(exact) * Fraction(1, 2 ** (53 * nc - 2))
            assert abs(F(C[j, i]) - exact) <= bound


def test_update_mode_subtracts():
    nc, K = 4, 8
    pl = O.make_plan(212, K)
    A, B = _operands(nc, 5, 5, K, 10)
    C0 = W.random_expansions(5, 5, nc, np.random.default_rng(3))
    C1, _ = O.ozgemm(1, A, B, C0, pl)
    P, _ = O.ozgemm(0, A, B, np.zeros_like(C0), pl)
    assert np.array_equal(C1, O.exp_add(C0, -P))


def test_naive_gemm_error():
    nc, K = 4, 16
    A, B = _operands(nc, 4, 4, K, 12)
    C = O.naive_gemm(0, A, B, np.zeros((4, 4, nc)))
    for i in range(4):
        for j in range(4):
            exact = sum(F(A[h, i]) * F(B[j, h]) for h in range(K))
            mag = sum(abs(F(A[h, i]) * F(B[j, h])) for h in range(K))
            assert abs(F(C[j, i]) - exact) <= mag * K * Fraction(1, 2 ** (53 * nc - 4))


def test_crt_round_trip_binary64_moduli():
    # the ~22-bit primes of the binary64 back-end: 12 moduli, P of 262 bits
    pl = O.make_plan(212, 256, backend=O.BACKEND_F64MOD)
    rng = np.random.default_rng(14)
    vals = [0, 1, -1, pl.P // 2, -(pl.P // 2) + 1]
    vals += [int.from_bytes(rng.bytes(40), "little") % pl.P - pl.P // 2 for _ in range(40)]
    tpl = np.zeros((1, pl.nmod, 1, len(vals)), dtype=np.uint32)
    for i, X in enumerate(vals):
        for l, m in enumerate(pl.moduli):
            tpl[0, l, 0, i] = ((X % m) * pl.y[l]) % m
    out = O.crt(tpl, pl, nw=8)
    for i, X in enumerate(vals):
        assert O.limbs_to_int(out[0, 0, i]) == X


def test_modgemm_binary64_moduli_exact_and_bounded():
    nc, K = 4, 40
    pl = O.make_plan(212, K, backend=O.BACKEND_F64MOD)
    A, B = _operands(nc, 6, 5, K, 9)
    ra = O.residues(A, True, O.exponents(A, True), pl)
    rb = O.residues(B, False, O.exponents(B, False), pl)
    assert np.abs(ra).max() > 2 ** 20             # large residues really occur
    tpl, cmax = O.modgemm(ra, rb, pl, want_cmax=True)
    assert cmax < 2 ** 53                         # every group product exact in FP64
    for gi, g in enumerate(pl.groups):
        for l, m in enumerate(pl.moduli):
            C = [[sum(int(ra[ta, l, i, h]) * int(rb[tb, l, j, h])
                      for ta, tb in pl.pairs(g) for h in range(K)) for j in range(5)]
                 for i in range(6)]
            want = np.array([[((c % m) * pl.y[l]) % m for c in row] for row in C])
            assert np.array_equal(tpl[gi, l].T, want)
    # the same digit-group sums as the INT8 back-end would give at this (S, w)
    _, sb = O.ozgemm(0, A, B, np.zeros((5, 6, nc)), pl, want_sbar=True, nw_out=10)
    assert np.array_equal(O.crt(tpl, pl, nw=10), sb)


def test_fp8_digits_exhaustive():
    # Eq. (fp8digits) over every centred residue of the moduli <= 256
    r = np.arange(-128, 128, dtype=np.int32)
    d0, d1 = O.fp8_digits(r)
    assert np.array_equal(17 * d1 + d0, r)
    assert np.abs(d0).max() == 8 and np.abs(d1).max() == 8   # -128 gives d1 = -8
    assert np.abs(d1[1:]).max() == 7          # |r| <= 127 gives |d1| <= 7, as the paper says
    # d1 is the nearest integer to r/17 (never a tie: 17 is odd)
    for v, a in zip(r, d1):
        assert abs(Fraction(int(v), 17) - int(a)) < Fraction(1, 2)


def _decode_e4m3(b):
    """Value of an OCP E4M3 byte from the format definition (no NaN here)."""
    sign = -1 if b & 0x80 else 1
    e, f = (b >> 3) & 15, b & 7
    if e == 0:
        return sign * Fraction(f, 8) * Fraction(2) ** -6
    return sign * (1 + Fraction(f, 8)) * Fraction(2) ** (e - 7)


def test_e4m3_encoding_of_digits():
    for d in range(-16, 17):
        b = O.e4m3_int(d)
        assert _decode_e4m3(b) == d
    assert O.e4m3_int(1) == 0x38 and O.e4m3_int(-8) == 0xD0


def test_fp8_subproducts_rebuild_modgemm():
    # rr' = d0 d0' + 17 (d0 d1' + d1 d0') + 289 d1 d1'; the three partial
    # products stay below 2^24 (exact FP32 accumulation) at the plan's K*S
    nc, K = 3, 64
    pl = O.make_plan(159, K, backend=O.BACKEND_FP8_B17)
    A, B = _operands(nc, 5, 4, K, 10)
    ra = O.residues(A, True, O.exponents(A, True), pl)
    rb = O.residues(B, False, O.exponents(B, False), pl)
    a0, a1 = O.fp8_digits(ra)
    b0, b1 = O.fp8_digits(rb)
    tpl = O.modgemm(ra, rb, pl)
    for gi, g in enumerate(pl.groups):
        for l, m in enumerate(pl.moduli):
            P = [np.zeros((5, 4), dtype=np.int64) for _ in range(3)]
            for ta, tb in pl.pairs(g):
                P[0] += a0[ta, l].astype(np.int64) @ b0[tb, l].astype(np.int64).T
                P[1] += (a0[ta, l].astype(np.int64) @ b1[tb, l].astype(np.int64).T
                         + a1[ta, l].astype(np.int64) @ b0[tb, l].astype(np.int64).T)
                P[2] += a1[ta, l].astype(np.int64) @ b1[tb, l].astype(np.int64).T
            for q in P:
                assert np.abs(q).max() < 2 ** 24
            C = P[0] + 17 * P[1] + 289 * P[2]
            want = ((C % m) * pl.y[l]) % m
            assert np.array_equal(tpl[gi, l].T, want)
