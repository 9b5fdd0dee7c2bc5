"""Pins of the blocked limb-format LU oracle (oracle/limb_lu.py and the
panel, unit-lower solve and multiply-subtract routines of oracle/lfloat.c).

* With the native Schur update every element receives the operations of
  the unblocked LU in the same order: the blocked result equals the
  unblocked LU (itself pinned to exact rationals and to Table lotkin) bit
  for bit for every panel width, pivots and info included.
* The rectangular panel equals the first columns of the unblocked LU.
* With the Ozaki-II update: b >= n is the unblocked LU; otherwise the
  factors stay within 2^-(p-24) (normwise, relative) of the unblocked
  ones and of the exact rational LU with the same pivots.
* The solve: x of a small system against exact rational elimination."""
from fractions import Fraction

import numpy as np
import pytest

import oracle.lfloat as LF
import oracle.limb_lu as OLU
import workloads as W


def _random(nl, n, seed, singular=False):
    rng = np.random.default_rng(seed)
    A = W.random_limbs(n, n, nl, rng, exp_sigma=3.0, zero_frac=0.05)
    if singular:
        A[0][:, 2, :] = 0
        A[1][2, :] = OLU.EXP32_ZERO
        A[2][2, :] = 0
        for x in A:
            x[..., :, 4] = x[..., :, 1]
    return A


def _eq(X, Y):
    return all(np.array_equal(x, y) for x, y in zip(X, Y))


@pytest.mark.parametrize("nl,n,b", [(1, 13, 3), (2, 17, 4), (1, 9, 1), (3, 20, 7), (2, 12, 12),
                                    (1, 16, 5)])
@pytest.mark.parametrize("singular", [False, True])
def test_native_blocked_equals_unblocked(nl, n, b, singular):
    A = _random(nl, n, 100 * n + b, singular)
    F, ip, info = OLU.getrf(A, b, "native")
    G, ip2, info2 = LF.getrf(OLU.to_lf(A))
    assert _eq(F, OLU.from_lf(G))
    assert np.array_equal(ip, ip2) and info == info2
    if singular:
        assert info > 0


def test_panel_equals_first_columns_of_unblocked():
    import ctypes
    from oracle import _i32p, _i64p, lib
    nl, m, nc = 2, 15, 6
    A = _random(nl, m, 3)
    X = OLU.to_lf(A)
    Y = tuple(x.copy() for x in X)
    piv = np.zeros(nc, dtype=np.int64)
    inf = np.zeros(1, dtype=np.int32)
    lib().orc_lf_getf2(nl, m, nc, *OLU._ptrs(Y, 0, 0, m), m, piv.ctypes.data_as(_i64p),
                       inf.ctypes.data_as(_i32p))
    G, ip, _ = LF.getrf(X)
    assert np.array_equal(piv, ip[:nc])
    # the unblocked LU's later interchanges move whole rows, these columns too
    for j in range(nc, m):
        r = int(ip[j])
        for y in Y:
            y[:nc, [j, r]] = y[:nc, [r, j]]
    for y, g in zip(Y, G):
        assert np.array_equal(y[:nc], g[:nc])


@pytest.mark.parametrize("nl,n", [(1, 10), (2, 14)])
def test_ozaki_with_one_panel_is_unblocked(nl, n):
    A = _random(nl, n, 7 * n)
    F, ip, _ = OLU.getrf(A, n, "ozaki")
    G, ip2, _ = LF.getrf(OLU.to_lf(A))
    assert _eq(F, OLU.from_lf(G)) and np.array_equal(ip, ip2)


def _vals(L):
    limb, ex, sg = L
    nl, cols, rows = limb.shape
    import oracle.limbs as OL
    return [[OL.value(L, i, j) for j in range(cols)] for i in range(rows)]


@pytest.mark.parametrize("nl,n,b", [(1, 24, 4), (2, 20, 8)])
def test_ozaki_blocked_factors_close_to_unblocked(nl, n, b):
    A = _random(nl, n, 11 * n)
    F, ip, _ = OLU.getrf(A, b, "ozaki")
    G, ip2, _ = LF.getrf(OLU.to_lf(A))
    assert np.array_equal(ip, ip2)
    p = 64 * nl
    fv, gv = _vals(F), _vals(OLU.from_lf(G))
    scale = max(abs(x) for row in gv for x in row)
    worst = max(abs(fv[i][j] - gv[i][j]) for i in range(n) for j in range(n))
    assert worst <= scale * Fraction(1, 2 ** (p - 24))
    assert worst > 0          # the blocked update rounds differently somewhere


def _exact_lu(vals, ipiv):
    """Exact rational elimination with the given row interchanges."""
    n = len(vals)
    a = [row[:] for row in vals]
    for j in range(n):
        r = int(ipiv[j])
        a[j], a[r] = a[r], a[j]
        for i in range(j + 1, n):
            a[i][j] = a[i][j] / a[j][j]
            for c in range(j + 1, n):
                a[i][c] -= a[i][j] * a[j][c]
    return a


@pytest.mark.parametrize("nl,b", [(1, 3), (2, 2)])
def test_factors_and_solution_against_exact_lu(nl, b):
    n = 8
    A = _random(nl, n, 5 + nl)
    F, ip, info = OLU.getrf(A, b, "ozaki")
    assert info == 0
    p = 64 * nl
    exact = _exact_lu(_vals(A), ip)
    fv = _vals(F)
    scale = max(abs(x) for row in exact for x in row)
    for i in range(n):
        for j in range(n):
            assert abs(fv[i][j] - exact[i][j]) <= scale * Fraction(1, 2 ** (p - 24))
    # solve A x = b with b = A 1 formed exactly, rounded to p bits
    av = _vals(A)
    rhs = [sum(av[i], Fraction(0)) for i in range(n)]
    B = OLU.from_lf(tuple(x[None] for x in LF.pack([LF.from_fraction(v, nl) for v in rhs], nl)))
    X = OLU.getrs(F, ip, B)
    xv = [v[0] for v in _vals(X)]
    assert all(abs(v - 1) <= Fraction(1, 2 ** (p - 30)) for v in xv)


@pytest.mark.parametrize("n,nl", [(37, 1), (64, 3)])
def test_lotkin_limb_generators_match_oracle(n, nl):
    """The benchmark's Lotkin matrix and right-hand side (workloads) equal
    the oracle's: RN_p of 1/(i+j+1), and RN_p of the exact row sums."""
    assert _eq(W.lotkin_limbs(n, nl), OLU.from_lf(LF.lotkin(n, nl)))
    assert _eq(W.lotkin_rhs_limbs(n, nl), OLU.from_lf(LF.rhs_times_ones(LF.lotkin(n, nl))))


@pytest.mark.parametrize("nl,n,b,leaf", [(1, 24, 16, 4), (2, 30, 12, 3), (1, 37, 37, 8),
                                         (3, 21, 9, 2)])
@pytest.mark.parametrize("singular", [False, True])
def test_recursive_native_panel_equals_unblocked(nl, n, b, leaf, singular):
    A = _random(nl, n, 31 * n + leaf, singular)
    F, ip, info = OLU.getrf(A, b, "native", leaf=leaf)
    G, ip2, info2 = LF.getrf(OLU.to_lf(A))
    assert _eq(F, OLU.from_lf(G))
    assert np.array_equal(ip, ip2) and info == info2


@pytest.mark.parametrize("nl,n,b", [(1, 20, 8), (2, 26, 12)])
def test_recursive_ozaki_with_leaf_at_least_b_is_plain_blocked(nl, n, b):
    A = _random(nl, n, 13 * n)
    F, ip, info = OLU.getrf(A, b, "ozaki", leaf=b)
    G, ip2, info2 = OLU.getrf(A, b, "ozaki")
    assert _eq(F, G) and np.array_equal(ip, ip2)


@pytest.mark.parametrize("nl,n,b,leaf", [(1, 32, 16, 4), (2, 24, 24, 6)])
def test_recursive_ozaki_factors_close_to_unblocked(nl, n, b, leaf):
    A = _random(nl, n, 17 * n)
    F, ip, _ = OLU.getrf(A, b, "ozaki", leaf=leaf)
    G, ip2, _ = LF.getrf(OLU.to_lf(A))
    assert np.array_equal(ip, ip2)
    p = 64 * nl
    fv, gv = _vals(F), _vals(OLU.from_lf(G))
    scale = max(abs(x) for row in gv for x in row)
    worst = max(abs(fv[i][j] - gv[i][j]) for i in range(n) for j in range(n))
    assert 0 < worst <= scale * Fraction(1, 2 ** (p - 24))
    H, ip3, _ = OLU.getrf(A, b, "ozaki")
    assert not _eq(F, H)          # the panel's updates did go through Ozaki-II


def test_split_halves_leaf_blocks():
    assert [OLU.split(w, 32) for w in (256, 96, 40, 64, 33)] == [128, 64, 32, 32, 32]
    assert OLU.split(7, 2) == 4
