"""p-bit floating-point LU of the CPU oracle (``lfloat.c``).

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no
code with the GPU path.

Numbers are p = 64 nl bit binary floating point, every operation correctly
rounded (to nearest, ties to even: MPFR's RNDN, which the paper's GPU type
reproduces; Sec. 2), x = (-1)^s m 2^(e - p) with 2^(p-1) <= m < 2^p; zero
has m = 0, e = EXP_ZERO.  A vector or matrix is a tuple ``(m, e, s)`` of
numpy arrays, element-major: m has shape (..., nl) uint64 (least
significant limb first), e (...) int64, s (...) uint8; a matrix is stored
column-major as (cols, rows, ...), element (i, j) at ``[j, i]``.

Used as
  * the 2p-bit reference: the LU and solve of a DD/TD/QD system repeated at
    p' >= 2p bits, against which a p-bit result's error is measured;
  * the Lotkin experiment of Sec. 4.3 / Table lotkin (correct bits of the
    solution of A x = A 1), whose printed values pin it.
"""
from __future__ import annotations

from fractions import Fraction
from typing import Tuple

import numpy as np

from . import _p, _i32p, _i64p, _u8p, _u64p, lib

EXP_ZERO = -(2 ** 63)


def zeros(shape, nl: int):
    shape = tuple(shape)
    return (np.zeros(shape + (nl,), dtype=np.uint64), np.full(shape, EXP_ZERO, dtype=np.int64),
            np.zeros(shape, dtype=np.uint8))


def _c(X):
    m, e, s = X
    return (np.ascontiguousarray(m, dtype=np.uint64), np.ascontiguousarray(e, dtype=np.int64),
            np.ascontiguousarray(s, dtype=np.uint8))


def from_fraction(x: Fraction, nl: int) -> Tuple[int, int, int]:
    """(mantissa, exponent, sign) of RN_p(x), p = 64 nl, ties to even."""
    p = 64 * nl
    if x == 0:
        return 0, EXP_ZERO, 0
    s = 1 if x < 0 else 0
    a = -x if s else x
    k = p - (a.numerator.bit_length() - a.denominator.bit_length())
    while a * Fraction(2) ** k >= 2 ** p:
        k -= 1
    while a * Fraction(2) ** k < 2 ** (p - 1):
        k += 1
    t = a * Fraction(2) ** k
    m = t.numerator // t.denominator
    r = t - m
    if r > Fraction(1, 2) or (r == Fraction(1, 2) and m & 1):
        m += 1
    if m == 1 << p:
        m >>= 1
        k -= 1
    return m, p - k, s


def pack(values, nl: int):
    """Vector of (mantissa, exponent, sign) triples -> (m, e, s) arrays."""
    n = len(values)
    X = zeros((n,), nl)
    for k, (m, e, s) in enumerate(values):
        for q in range(nl):
            X[0][k, q] = (m >> (64 * q)) & ((1 << 64) - 1)
        X[1][k] = e
        X[2][k] = s
    return X


def value(X, idx) -> Fraction:
    """Exact value of element idx (a tuple index into the leading dims)."""
    m, e, s = X
    nl = m.shape[-1]
    mm = 0
    for q in range(nl - 1, -1, -1):
        mm = (mm << 64) | int(m[idx + (q,)] if isinstance(idx, tuple) else m[idx][q])
    if mm == 0:
        return Fraction(0)
    ee = int(e[idx])
    v = Fraction(mm) * Fraction(2) ** (ee - 64 * nl)
    return -v if int(s[idx]) else v


def vec(op: str, A, B):
    """Elementwise a+b, a-b, a*b or a/b, each correctly rounded."""
    A, B = _c(A), _c(B)
    nl = A[0].shape[-1]
    cnt = A[1].size
    R = zeros(A[1].shape, nl)
    code = {"add": 0, "sub": 1, "mul": 2, "div": 3}[op]
    lib().orc_lf_vec(code, nl, cnt, _p(A[0], _u64p), _p(A[1], _i64p), _p(A[2], _u8p),
                     _p(B[0], _u64p), _p(B[1], _i64p), _p(B[2], _u8p), _p(R[0], _u64p),
                     _p(R[1], _i64p), _p(R[2], _u8p))
    return R


def from_doubles(x, nl: int):
    """RN_p of the exact sum of the last axis (expansion components) of x."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    nc = x.shape[-1]
    shape = x.shape[:-1]
    R = zeros(shape, nl)
    lib().orc_lf_from_doubles(nl, int(np.prod(shape)), nc, _p(x, C_dp()), _p(R[0], _u64p),
                              _p(R[1], _i64p), _p(R[2], _u8p))
    return R


def C_dp():
    import ctypes
    return ctypes.POINTER(ctypes.c_double)


def getrf(A):
    """LU with partial pivoting (Sec. 3.4) of the n x n matrix A (m of shape
    (n, n, nl), column-major): every division, product and difference
    rounded once to p bits.  Returns (LU, ipiv, info)."""
    m, e, s = (x.copy() for x in _c(A))
    n = e.shape[0]
    nl = m.shape[-1]
    ipiv = np.zeros(n, dtype=np.int64)
    info = np.zeros(1, dtype=np.int32)
    lib().orc_lf_getrf(nl, n, _p(m, _u64p), _p(e, _i64p), _p(s, _u8p), n, _p(ipiv, _i64p),
                       _p(info, _i32p))
    return (m, e, s), ipiv, int(info[0])


def getrs(LU, ipiv, B):
    """Solve from getrf's factors (Sec. 4.3: forward and backward
    substitution); B of shape (nrhs, n, ...)."""
    LU = _c(LU)
    bm, be, bs = (x.copy() for x in _c(B))
    nrhs, n = be.shape
    nl = bm.shape[-1]
    ipiv = np.ascontiguousarray(ipiv, dtype=np.int64)
    lib().orc_lf_getrs(nl, n, _p(LU[0], _u64p), _p(LU[1], _i64p), _p(LU[2], _u8p), n,
                       _p(ipiv, _i64p), nrhs, _p(bm, _u64p), _p(be, _i64p), _p(bs, _u8p), n)
    return bm, be, bs


def lotkin(n: int, nl: int):
    """The Lotkin matrix of Sec. 4.3 (row 0 all ones, a_ij = 1/(i+j+1)
    below, 0-indexed), every entry RN_p of the exact rational; column-major
    (cols, rows) arrays."""
    A = zeros((n, n), nl)
    cache = {}
    for j in range(n):
        for i in range(n):
            x = Fraction(1) if i == 0 else Fraction(1, i + j + 1)
            if x not in cache:
                cache[x] = from_fraction(x, nl)
            mm, ee, ss = cache[x]
            for q in range(nl):
                A[0][j, i, q] = (mm >> (64 * q)) & ((1 << 64) - 1)
            A[1][j, i] = ee
            A[2][j, i] = ss
    return A


def rhs_times_ones(A, nl_out: int = None):
    """b = A 1 formed exactly from the stored entries, rounded to p bits
    (Sec. 4.3: b generated at high precision, rounded to the target)."""
    m, e, s = A
    n = e.shape[0]
    nl = m.shape[-1] if nl_out is None else nl_out
    vals = []
    for i in range(n):
        tot = sum((value(A, (j, i)) for j in range(n)), Fraction(0))
        vals.append(from_fraction(tot, nl))
    X = pack(vals, nl)
    return tuple(x[None] for x in X)


def correct_bits(X, exact=1) -> int:
    """min_i -log2 |x_i - exact|, computed exactly (the binary64 underflow
    that the paper's remark on its first Lotkin numbers warns about cannot
    occur: no double is formed).  X has shape (n,) or (1, n)."""
    m, e, s = X
    if e.ndim == 2:
        m, e, s = m[0], e[0], s[0]
    worst = None
    for i in range(e.shape[0]):
        d = abs(value((m, e, s), i) - exact)
        if d == 0:
            continue
        bits = d.denominator.bit_length() - d.numerator.bit_length()
        # floor(-log2 d) exactly
        if Fraction(2) ** (-bits) < d:
            bits -= 1
        worst = bits if worst is None else min(worst, bits)
    return worst if worst is not None else 1 << 30
