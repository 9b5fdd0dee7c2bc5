"""Pins of the p-bit floating-point oracle (oracle/lfloat.c): every operation
against the correctly rounded exact rational, the LU and solve against exact
rational elimination, and the Lotkin experiment of Sec. 4.3 against the
correct bits that Table lotkin prints."""
import math
import random
from fractions import Fraction

import numpy as np
import pytest

import oracle.lfloat as LF

MASK = (1 << 64) - 1


def rn(x: Fraction, p: int):
    """Round to nearest, ties to even, at p bits, straight from the
    definition: |x| 2^k in [2^(p-1), 2^p), q = floor, compare 2 r with d.
    Returns the exact rounded value as a Fraction."""
    if x == 0:
        return Fraction(0)
    a = abs(x)
    n, d = a.numerator, a.denominator
    k = p - (n.bit_length() - d.bit_length())
    # adjust k so that 2^(p-1) <= n 2^k / d < 2^p
    while True:
        num, den = (n << k, d) if k >= 0 else (n, d << -k)
        q = num // den
        if q >= 1 << p:
            k -= 1
        elif q < 1 << (p - 1):
            k += 1
        else:
            break
    r = num - q * den
    if 2 * r > den or (2 * r == den and q & 1):
        q += 1
    v = Fraction(q) / Fraction(2) ** k if k >= 0 else Fraction(q) * Fraction(2) ** -k
    return v if x > 0 else -v


def test_reference_rounding_is_binary64_at_53_bits():
    rng = random.Random(1)
    for _ in range(3000):
        x = Fraction(rng.randrange(1, 1 << 80), rng.randrange(1, 1 << 70))
        x *= Fraction(2) ** rng.randrange(-60, 60)
        if rng.random() < 0.5:
            x = -x
        assert rn(x, 53) == Fraction(float(x))
    # ties: odd and even neighbours
    for m in range(1 << 52, (1 << 52) + 40):
        x = Fraction(2 * m + 1, 2)
        assert rn(x, 53) == Fraction(float(x))


def _rand_num(rng, nl, e_lo=-40, e_hi=40):
    p = 64 * nl
    m = rng.randrange(1 << (p - 1), 1 << p)
    if rng.random() < 0.2:                     # short mantissas: exact cases
        m = (m >> (p - 3)) << (p - 3)
    return m, rng.randrange(e_lo, e_hi), rng.randrange(2)


def _val(t, nl):
    m, e, s = t
    if m == 0:
        return Fraction(0)
    v = Fraction(m) * Fraction(2) ** (e - 64 * nl)
    return -v if s else v


def _check(op, pairs, nl):
    A = LF.pack([a for a, _ in pairs], nl)
    B = LF.pack([b for _, b in pairs], nl)
    R = LF.vec(op, A, B)
    p = 64 * nl
    for k, (a, b) in enumerate(pairs):
        x, y = _val(a, nl), _val(b, nl)
        exact = {"add": x + y, "sub": x - y, "mul": x * y, "div": x / y if y else None}[op]
        got = LF.value(R, k)
        assert got == rn(exact, p), (op, k)
        if got != 0:          # normalised mantissa
            assert int(R[0][k, nl - 1]) >> 63 == 1


@pytest.mark.parametrize("nl", [1, 2, 3])
@pytest.mark.parametrize("op", ["add", "sub", "mul", "div"])
def test_operations_are_correctly_rounded(nl, op):
    rng = random.Random(100 * nl + len(op))
    p = 64 * nl
    pairs = []
    for _ in range(600):
        a = _rand_num(rng, nl)
        b = _rand_num(rng, nl)
        if op in ("add", "sub"):
            # exponent gaps around the guard limbs of the aligned sum
            gap = rng.choice([0, 1, 2, 3, 63, 64, 65, 127, 128, 129, 191, 192, 193, 194,
                              255, 256, p - 1, p, p + 1, p + 190, p + 193, 3 * p + 7])
            b = (b[0], a[1] - gap, b[2])
        pairs.append((a, b))
    # cancellation: b within a few ulps of -a (or of a for sub)
    for _ in range(100):
        a = _rand_num(rng, nl)
        b = (a[0] + rng.randrange(-3, 4), a[1], a[2] ^ (1 if op == "add" else 0))
        if b[0] >> (p - 1) == 1 and b[0] < 1 << p:
            pairs.append((a, b))
    _check(op, pairs, nl)


@pytest.mark.parametrize("nl", [1, 2])
def test_addition_ties_round_to_even(nl):
    p = 64 * nl
    pairs = []
    for odd in (0, 1):
        m = (1 << (p - 1)) | (2 * 12345 + odd)
        half = (1 << (p - 1), 0 - p, 0)         # 2^(-p-1): half an ulp of a number in [1/2, 1)
        a = (m, 0, 0)
        pairs += [(a, half), (a, (half[0], half[1], 1)), ((m, 0, 1), half)]
        # just above / below the tie: sticky bits decide
        pairs += [(a, (half[0] + 1, half[1], 0)), (a, (half[0] + 1, half[1] - 1, 0))]
    _check("add", pairs, nl)


@pytest.mark.parametrize("op", ["add", "sub"])
def test_far_operand_decides_a_tie_through_its_dropped_bits(op):
    # |a| in [1/2, 1), b about 2^-200 |a|: the aligned sum keeps b only down
    # to a fixed guard position and folds the rest into a sticky bit.  b is
    # built so that the kept part puts the sum exactly on a rounding tie
    # (or one unit either side); whether b's dropped bits are zero then
    # decides the rounding, and a difference must treat them as lowering
    # the value, a sum as raising it.
    nl = 4
    P = 64 * nl
    pairs = []
    for m_a in ((1 << (P - 1)), (1 << (P - 1)) + 1, (1 << P) - 1):
        a = (m_a, 0, 0)
        for d in (193, 200, 260):
            drop = d - 192        # bits of b below the guard position
            for pattern in (-1, 0, 1):
                for low in (0, 1, (1 << drop) - 1 if drop > 1 else 1):
                    # kept part Y of b makes S = X -+ Y sit at the tie
                    # (+ pattern) at the rounding position of S
                    for T in (P + 191, P + 192):
                        r = T - P              # rounding position in S
                        want = (1 << (r - 1)) + pattern
                        X = m_a << 192
                        # S mod 2^r = want, with S = X + Y or X - Y
                        Y = (want - X) % (1 << r) if op == "add" else (X - want) % (1 << r)
                        Y |= 1 << (P - 1 - drop)          # keep b normalised
                        m_b = (Y << drop) | (low & ((1 << drop) - 1))
                        if m_b >> (P - 1) != 1 or m_b >= 1 << P:
                            continue
                        pairs.append((a, (m_b, -d, 0)))
    assert len(pairs) > 50
    _check(op, pairs, nl)


def test_zero_operands():
    nl = 2
    z = (0, LF.EXP_ZERO, 0)
    a = (3 << 126, 5, 1)
    _check("add", [(z, a), (a, z), (z, z)], nl)
    _check("sub", [(a, a), (z, a)], nl)
    _check("mul", [(z, a), (a, z)], nl)
    _check("div", [(z, a)], nl)


@pytest.mark.parametrize("nl", [1, 4, 7])
def test_from_doubles_is_the_rounded_exact_sum(nl):
    rng = np.random.default_rng(5)
    x = rng.normal(size=(300, 4)) * np.ldexp(1.0, rng.integers(-200, 200, size=(300, 4)))
    x[::7, 1] = 0.0
    x[3] = [1.0, -1.0, 0.0, 0.0]                  # exact zero
    x[4] = [5e-324, 1e300, -1e300, 0.0]           # subnormal and cancellation
    R = LF.from_doubles(x, nl)
    for k in range(x.shape[0]):
        exact = sum((Fraction(float(v)) for v in x[k]), Fraction(0))
        assert LF.value(R, k) == rn(exact, 64 * nl)


def _exact_lu(Ad):
    n = len(Ad)
    A = [row[:] for row in Ad]
    ipiv = []
    for j in range(n):
        p = max(range(j, n), key=lambda i: (abs(A[i][j]), -i))
        ipiv.append(p)
        A[j], A[p] = A[p], A[j]
        if A[j][j] == 0:
            continue
        for i in range(j + 1, n):
            A[i][j] /= A[j][j]
            for c in range(j + 1, n):
                A[i][c] -= A[i][j] * A[j][c]
    return A, ipiv


def _random_matrix(n, nl, seed):
    rng = random.Random(seed)
    vals = [_rand_num(rng, nl, -3, 3) for _ in range(n * n)]
    A = LF.pack(vals, nl)
    return tuple(x.reshape((n, n) + x.shape[1:]) for x in A)   # (cols, rows, ...)


@pytest.mark.parametrize("nl", [2, 4])
def test_lu_matches_exact_rational_elimination(nl):
    n = 8
    A = _random_matrix(n, nl, 9 + nl)
    Ad = [[LF.value(A, (j, i)) for j in range(n)] for i in range(n)]
    (LU, ipiv, info) = LF.getrf(A)
    assert info == 0
    ex, eip = _exact_lu(Ad)
    assert list(ipiv) == eip
    p = 64 * nl
    for i in range(n):
        for j in range(n):
            e = ex[i][j]
            assert abs(LF.value(LU, (j, i)) - e) <= max(abs(e), Fraction(1)) * Fraction(1, 2 ** (p - 16))


@pytest.mark.parametrize("nl", [2, 8])
def test_solve_matches_exact_rational_solution(nl):
    n = 8
    A = _random_matrix(n, nl, 30 + nl)
    Ad = [[LF.value(A, (j, i)) for j in range(n)] for i in range(n)]
    rng = random.Random(3)
    b = LF.pack([_rand_num(rng, nl, -2, 2) for _ in range(n)], nl)
    B = tuple(x[None] for x in b)
    LU, ipiv, info = LF.getrf(A)
    X = LF.getrs(LU, ipiv, B)
    # exact solution
    M = [row[:] + [LF.value(b, i)] for i, row in enumerate(Ad)]
    for j in range(n):
        pv = max(range(j, n), key=lambda i: abs(M[i][j]))
        M[j], M[pv] = M[pv], M[j]
        for i in range(j + 1, n):
            f = M[i][j] / M[j][j]
            for c in range(j, n + 1):
                M[i][c] -= f * M[j][c]
    x = [Fraction(0)] * n
    for i in range(n - 1, -1, -1):
        x[i] = (M[i][n] - sum(M[i][c] * x[c] for c in range(i + 1, n))) / M[i][i]
    xmax = max(abs(v) for v in x)
    for i in range(n):
        assert abs(LF.value(X, (0, i)) - x[i]) <= xmax * Fraction(1, 2 ** (64 * nl - 24))


def test_lotkin_small_solution_tracks_precision():
    # Lotkin of order 24 (log2 cond about 5.1 n = 122 bits): the correct bits
    # of the solution grow one for one with the precision
    n = 24
    got = []
    for nl in (3, 4, 6):
        A = LF.lotkin(n, nl)
        b = LF.rhs_times_ones(A)
        LU, ipiv, info = LF.getrf(A)
        assert info == 0
        X = LF.getrs(LU, ipiv, b)
        got.append(LF.correct_bits(X))
    p = [192, 256, 384]
    for bits, pp in zip(got, p):
        assert pp - 5.1 * n - 20 < bits < pp - 5.1 * n + 40, (bits, pp)
    assert got[1] - got[0] > 40 and got[2] - got[1] > 100


@pytest.mark.slow
def test_lotkin_n512_p3136_correct_bits_as_printed():
    # Table lotkin (Sec. 4.3): n = 512 at p = 3136 gives 545 (GPU) and 546
    # (CPU) correct bits; implementations agree within 1-3 bits (Finding
    # lotkin), so the pin is [542, 549].
    n, nl = 512, 49
    A = LF.lotkin(n, nl)
    b = LF.rhs_times_ones(A)
    LU, ipiv, info = LF.getrf(A)
    assert info == 0
    X = LF.getrs(LU, ipiv, b)
    bits = LF.correct_bits(X)
    assert 542 <= bits <= 549, bits


def _qd_vs_2p_bits(A, nc, b_blk=16):
    import oracle as O
    import workloads as W
    n = A.shape[0]
    rhs = W.rhs_ones(A)
    LU, ipiv, info, _ = O.getrf(A, b_blk, O.METHOD_OZAKI)
    x = O.getrs(LU, ipiv, rhs)[0]
    nl = 7
    Ll, ipl, infol = LF.getrf(LF.from_doubles(A, nl))
    X = LF.getrs(Ll, ipl, LF.from_doubles(rhs, nl))
    num = max(abs(sum(Fraction(float(c)) for c in x[i]) - LF.value(X, (0, i))) for i in range(n))
    den = max(abs(LF.value(X, (0, i))) for i in range(n))
    rel = num / den
    return rel.denominator.bit_length() - rel.numerator.bit_length()


def test_qd_lu_against_the_2p_oracle():
    # Sec. 4.2: about 208 correct bits for QD on well-conditioned systems;
    # a graded D R D with condition near 10^20 loses about 66 of them
    import workloads as W
    n = 64
    bits_w = _qd_vs_2p_bits(W.wellcond(n, 4, np.random.default_rng(4)), 4)
    bits_g = _qd_vs_2p_bits(W.graded(n, 4, 20.0, np.random.default_rng(5)), 4)
    assert 200 <= bits_w <= 215, bits_w
    assert 120 <= bits_g <= 200, bits_g


@pytest.mark.parametrize("kind", ["wellcond", "graded40"])
def test_stored_2p_references_solve_their_systems(kind):
    # the reference written by tests/golden/make_ref2p.py must solve the
    # system its generator and seed define: exact residuals of sampled rows
    import os
    import workloads as W
    path = os.path.join(os.path.dirname(__file__), "golden", f"ref2p_qd2048_{kind}.npz")
    ref = np.load(path)
    n, nl = 2048, int(ref["nl"])
    rng = np.random.default_rng(int(ref["seed"]))
    A = W.wellcond(n, 4, rng) if kind == "wellcond" else W.graded(n, 4, 40.0, rng)
    b = W.rhs_ones(A)
    X = (ref["m"], ref["e"], ref["s"])
    x = [LF.value(X, i) for i in range(n)]
    for i in (0, 1, 777, n - 1):
        row = [sum(Fraction(float(c)) for c in A[j, i]) for j in range(n)]
        bi = sum(Fraction(float(c)) for c in b[0, i])
        res = sum(a * v for a, v in zip(row, x)) - bi
        scale = sum(abs(a * v) for a, v in zip(row, x))
        assert abs(res) <= scale * Fraction(1, 2 ** 400), (kind, i)
