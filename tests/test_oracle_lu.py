"""Pins of the oracle LU (Sec. 3.4) against exact rational elimination and
the properties that hold at any size."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import workloads as W


def F(x):
    return sum((Fraction(float(v)) for v in np.ravel(x)), Fraction(0))


def exact_lu(Ad):
    """Gaussian elimination with partial pivoting on exact rationals; ties go
    to the lowest row.  Returns (L, U, ipiv)."""
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


def backward_error(A0, LU, ipiv):
    n = LU.shape[0]
    Ad = W.to_dense_fraction(A0)
    for j, p in enumerate(ipiv):
        Ad[j], Ad[p] = Ad[p], Ad[j]
    LUd = W.to_dense_fraction(LU)
    worst = Fraction(0)
    amax = max(abs(x) for row in Ad for x in row)
    for i in range(n):
        for j in range(n):
            s = sum(LUd[i][k] * LUd[k][j] for k in range(min(i, j))) + \
                (LUd[i][j] if i <= j else LUd[i][j] * LUd[j][j])
            worst = max(worst, abs(s - Ad[i][j]))
    return worst / amax


@pytest.mark.parametrize("nc", [2, 4])
@pytest.mark.parametrize("method", [O.METHOD_NAIVE, O.METHOD_OZAKI])
def test_small_lu_matches_exact(nc, method):
    rng = np.random.default_rng(21)
    n = 8
    A = W.random_expansions(n, n, nc, rng)
    LU, ipiv, info, _ = O.getrf(A, 3, method)
    assert info == 0
    ex, eip = exact_lu(W.to_dense_fraction(A))
    assert list(ipiv) == eip
    for i in range(n):
        for j in range(n):
            e = ex[i][j]
            assert abs(F(LU[j, i]) - e) <= max(abs(e), Fraction(1)) * Fraction(1, 2 ** (53 * nc - 12))


@pytest.mark.parametrize("nc", [2, 3, 4])
def test_blocked_naive_equals_unblocked(nc):
    rng = np.random.default_rng(22)
    n = 37
    A = W.graded(n, nc, 20.0, rng)
    ref = O.getrf(A, 1, O.METHOD_NAIVE)
    for b in (4, 8, 16, 37):
        got = O.getrf(A, b, O.METHOD_NAIVE)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


def test_lotkin_backward_error_and_ozaki_agreement():
    n, nc = 24, 4
    A = W.lotkin(n, nc)
    LUn, ipn, _, _ = O.getrf(A, 8, O.METHOD_NAIVE)
    LUo, ipo, _, _ = O.getrf(A, 8, O.METHOD_OZAKI)
    assert backward_error(A, LUn, ipn) < Fraction(1, 2 ** 200)
    assert backward_error(A, LUo, ipo) < Fraction(1, 2 ** 200)


def test_wellconditioned_correct_bits():
    # Sec. 4.2: QD LU on well-conditioned matrices gives about 208 correct bits
    n, nc = 48, 4
    A = W.wellcond(n, nc, np.random.default_rng(23))
    b = W.rhs_ones(A)
    for method in (O.METHOD_OZAKI, O.METHOD_NAIVE):
        LU, ipiv, info, _ = O.getrf(A, 16, method)
        x = O.getrs(LU, ipiv, b)
        err = max(abs(F(x[0, i]) - 1) for i in range(n))
        bits = -math.log2(err) if err else 999
        assert bits > 200


def _int_triangular_system(n, nc, diag):
    """Unit-lower L and upper U with small integer entries (U's diagonal
    given), the integer solution 1..n and b = P^T L U x with the interchanges
    ipiv: every product, difference and quotient of the solve is an integer
    below 2^53, so an exact substitution returns x exactly."""
    L = np.eye(n)
    U = np.triu(np.arange(1, n * n + 1).reshape(n, n) % 5 + 1.0)
    U[np.diag_indices(n)] = diag
    L[np.tril_indices(n, -1)] = [(k % 3) - 1 for k in range(n * (n - 1) // 2)]
    LU = np.zeros((n, n, nc))
    LU[..., 0] = (np.tril(L, -1) + U).T
    x_true = np.arange(1, n + 1, dtype=float)
    y = L @ U @ x_true
    ipiv = np.array([min(j + (j % 3), n - 1) for j in range(n)], dtype=np.int64)
    # b with the interchanges undone: applying ipiv in order must give y
    b = y.copy()
    for j in range(n - 1, -1, -1):
        b[j], b[ipiv[j]] = b[ipiv[j]], b[j]
    B = np.zeros((1, n, nc))
    B[0, :, 0] = b
    return LU, ipiv, B, x_true


@pytest.mark.parametrize("nc", [2, 3, 4])
def test_getrs_divides_by_non_dyadic_pivots_exactly(nc):
    # Sec. 4.3 solves by forward and backward substitution: x_k is the
    # quotient of its updated right-hand side by u_kk.  With integer data,
    # interchanges and pivots 3, 5, 7, ... every quotient is an exact
    # integer, which the expansion division returns exactly.
    n = 7
    LU, ipiv, B, x_true = _int_triangular_system(n, nc, [3.0, 5.0, 7.0, 6.0, 9.0, 11.0, 12.0])
    x = O.getrs(LU, ipiv, B)
    assert np.array_equal(x[0, :, 0], x_true) and np.all(x[0, :, 1:] == 0)


@pytest.mark.parametrize("nc", [2, 3, 4])
def test_getrs_one_by_one_is_the_division(nc):
    # a 1 x 1 system is solved by one division of the right-hand side by the
    # pivot; random expansions, pivots 3, 7 and a random one
    rng = np.random.default_rng(40 + nc)
    b = W.random_expansions(1, 5, nc, rng)
    for u0 in (3.0, 7.0, None):
        U = W.random_expansions(1, 1, nc, rng) if u0 is None else np.zeros((1, 1, nc))
        if u0 is not None:
            U[0, 0, 0] = u0
        x = O.getrs(U, np.zeros(1, dtype=np.int64), b)
        for r in range(5):
            assert np.array_equal(x[r, 0], O.exp_div(b[r, 0], U[0, 0]))


def exact_solve(Ad, bd):
    """x = A^{-1} b in rationals (Gaussian elimination, partial pivoting)."""
    n = len(Ad)
    M = [row[:] + [bd[i]] for i, row in enumerate(Ad)]
    for j in range(n):
        p = max(range(j, n), key=lambda i: abs(M[i][j]))
        M[j], M[p] = M[p], M[j]
        for i in range(j + 1, n):
            f = M[i][j] / M[j][j]
            for c in range(j, n + 1):
                M[i][c] -= f * M[j][c]
    x = [Fraction(0)] * n
    for i in range(n - 1, -1, -1):
        s = M[i][n] - sum(M[i][c] * x[c] for c in range(i + 1, n))
        x[i] = s / M[i][i]
    return x


@pytest.mark.parametrize("nc", [2, 3, 4])
@pytest.mark.parametrize("method", [O.METHOD_NAIVE, O.METHOD_OZAKI])
def test_lu_solve_matches_exact_rational_solution(nc, method):
    # the n = 8 exact rational LU extended through the solve: random
    # expansions (general, non-dyadic pivots), the oracle's getrf + getrs
    # against the exact A^{-1} b within the expansion precision times a
    # small condition factor
    rng = np.random.default_rng(31 + nc)
    n = 8
    A = W.random_expansions(n, n, nc, rng)
    B = W.random_expansions(n, 2, nc, rng)
    LU, ipiv, info, _ = O.getrf(A, 3, method)
    assert info == 0
    X = O.getrs(LU, ipiv, B)
    Ad = W.to_dense_fraction(A)
    for r in range(2):
        bd = [F(B[r, i]) for i in range(n)]
        xe = exact_solve(Ad, bd)
        xmax = max(abs(v) for v in xe)
        for i in range(n):
            assert abs(F(X[r, i]) - xe[i]) <= xmax * Fraction(1, 2 ** (53 * nc - 24))


def test_singular_sets_info():
    n, nc = 10, 2
    A = W.random_expansions(n, n, nc, np.random.default_rng(24))
    A[:, 3, :] = A[:, 7, :]           # two equal rows: U has an exact zero pivot
    A[:, 5, :] = 0.0
    for method in (O.METHOD_NAIVE, O.METHOD_OZAKI):
        LU, ipiv, info, _ = O.getrf(A, 4, method)
        assert info > 0
        assert np.all(LU[info - 1, info - 1] == 0.0)
