"""Seeded synthetic inputs shared by the tests, the oracle runs and bench.py.

This module holds input recipes only -- none of the method's arithmetic.  It
rounds exact rationals to expansions (greedy round-to-nearest, which defines
the stored matrix) and nothing else.

Matrices are numpy float64 arrays of shape (cols, rows, nc): column-major,
each element an nc-component non-overlapping expansion (DD nc=2, TD nc=3,
QD nc=4).

Recipes (seed = 20260929 + config number unless a test says otherwise):
  * lotkin(n, nc): row 0 all ones, a_ij = 1/(i+j+1) for i >= 1 (0-indexed,
    Sec. 4.3 of the paper), each entry the greedy round-to-nearest expansion of
    the exact rational; rhs b = A*ones formed exactly from the stored entries
    and rounded the same way.
  * graded(n, nc, c, rng): A = D R D with R a random expansion matrix
    (leading components N(0,1)) and D = diag(2^round(log2 10^(c/2 * i/(n-1))));
    D is rounded to powers of two so the scaled entries stay exact expansions.
  * wellcond(n, nc, rng): R + n I with R random expansions (a stand-in for the
    paper's unspecified "diagonally dominant random" matrices).
  * random_expansions(rows, cols, nc, rng, exp_sigma): mantissa magnitude
    uniform in [0.5, 1), random sign, exponent round(N(0, exp_sigma^2)), then
    nc - 1 further components each at most half an ulp of the previous one
    (a canonical expansion), as in the standalone TD product workload.

Limb matrices (p = 64 nlimb bits; value (-1)^sign * mantissa * 2^(exp - p),
mantissa normalised to [2^(p-1), 2^p); zero = all limbs 0, exp INT32_MIN):
tuples (limb (nlimb, cols, rows) uint64, exp (cols, rows) int32, sign
(cols, rows) uint8).
  * random_limbs(rows, cols, nlimb, rng, exp_sigma, zero_frac): uniformly
    random normalised mantissas, random signs, exp round(N(0, exp_sigma^2)),
    a fraction of exact zeros.
  * lotkin_limbs(n, nlimb): the Lotkin matrix with every entry rounded to
    nearest (ties to even) at p bits.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

SEED_BASE = 20260929


def greedy_rn(x: Fraction, nc: int):
    """x_0 = RN(x), x_c = RN(x - x_0 - ... - x_{c-1}) (Python's float(Fraction)
    is correctly rounded, ties to even)."""
    out = []
    r = Fraction(x)
    for _ in range(nc):
        f = float(r)
        out.append(f)
        r -= Fraction(f)
    return out


def greedy_rn_sum(terms, nc: int):
    """Greedy RN expansion of the exact sum of a list of doubles (math.fsum is
    correctly rounded)."""
    terms = [float(t) for t in terms]
    out = []
    for _ in range(nc):
        f = math.fsum(terms + [-x for x in out])
        out.append(f)
    return out


def lotkin(n: int, nc: int):
    vals = {}
    A = np.empty((n, n, nc), dtype=np.float64)
    for s in range(1, 2 * n - 1):
        vals[s] = greedy_rn(Fraction(1, s + 1), nc)
    ii = np.arange(n)
    for j in range(n):
        col = np.array([vals[i + j] if i >= 1 else [1.0] + [0.0] * (nc - 1) for i in ii])
        A[j] = col
    A[:, 0, :] = 0.0
    A[:, 0, 0] = 1.0
    return A


def rhs_ones(A) -> np.ndarray:
    """b = A * ones, exactly from the stored entries, rounded greedily."""
    n_cols, n_rows, nc = A.shape
    b = np.empty((1, n_rows, nc), dtype=np.float64)
    for i in range(n_rows):
        b[0, i] = greedy_rn_sum(A[:, i, :].ravel().tolist(), nc)
    return b


def random_expansions(rows: int, cols: int, nc: int, rng: np.random.Generator,
                      exp_sigma: float = 0.0) -> np.ndarray:
    X = np.empty((cols, rows, nc), dtype=np.float64)
    mag = rng.uniform(0.5, 1.0, size=(cols, rows))
    sign = np.where(rng.random(size=(cols, rows)) < 0.5, -1.0, 1.0)
    e = np.rint(rng.normal(0.0, exp_sigma, size=(cols, rows))).astype(np.int64) if exp_sigma else \
        np.zeros((cols, rows), dtype=np.int64)
    x0 = np.ldexp(sign * mag, e)
    X[..., 0] = x0
    prev = x0
    for c in range(1, nc):
        # |x_c| < ulp(x_{c-1}) / 2: spacing of x_{c-1} is 2^(exponent-52)
        _, pe = np.frexp(prev)
        frac = rng.uniform(-0.5, 0.5, size=(cols, rows)) * (1 - 2.0 ** -20)
        xc = np.ldexp(frac, pe - 53)
        xc = np.where(prev == 0.0, 0.0, xc)
        X[..., c] = xc
        prev = xc
    return X


def graded(n: int, nc: int, c: float, rng: np.random.Generator) -> np.ndarray:
    R = random_expansions(n, n, nc, rng)
    R[..., 0] = rng.normal(size=(n, n))
    # re-derive the tails for the new leading components
    prev = R[..., 0]
    for k in range(1, nc):
        _, pe = np.frexp(prev)
        frac = rng.uniform(-0.5, 0.5, size=(n, n)) * (1 - 2.0 ** -20)
        R[..., k] = np.where(prev == 0.0, 0.0, np.ldexp(frac, pe - 53))
        prev = R[..., k]
    idx = np.arange(n)
    d = np.rint(np.log2(10.0) * (c / 2.0) * idx / max(n - 1, 1)).astype(np.int64)
    # A[j, i] = d_i r_ij d_j  (exact: powers of two)
    return np.ldexp(R, (d[None, :] + d[:, None])[..., None])


def wellcond(n: int, nc: int, rng: np.random.Generator) -> np.ndarray:
    R = random_expansions(n, n, nc, rng)
    for i in range(n):
        R[i, i, 0] += n
        # keep the element canonical: rebuild the tail below the new head
        R[i, i, 1:] = 0.0
    return R


def to_dense_fraction(X):
    """Exact rational matrix (list of rows) from an expansion matrix."""
    cols, rows, nc = X.shape
    return [[sum((Fraction(float(X[j, i, c])) for c in range(nc)), Fraction(0))
             for j in range(cols)] for i in range(rows)]


def batch_systems(count: int, rng: np.random.Generator, n_lo: int = 64, n_hi: int = 512):
    """The batched configuration: `count` independent systems, orders uniform
    in [n_lo, n_hi], even items double-double and odd items quad-double,
    A = D R D with R ~ N(0, 1) and D = diag(10^(c/2 * i/(n-1))), c uniform in
    [20, 60] -- D rounded to powers of two so the scaled entries stay exact
    expansions (the same grading as `graded`) -- and b = A * ones.  Returns a
    list of (nc, A, b) with A of shape (n, n, nc) and b of shape (1, n, nc)."""
    out = []
    for k in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        nc = 2 if k % 2 == 0 else 4
        c = float(rng.uniform(20.0, 60.0))
        A = graded(n, nc, c, rng)
        out.append((nc, A, rhs_ones(A)))
    return out


LIMB_EXP_ZERO = -(2 ** 31)


def random_limbs(rows: int, cols: int, nlimb: int, rng: np.random.Generator,
                 exp_sigma: float = 0.0, zero_frac: float = 0.0):
    limb = rng.integers(0, 2 ** 63, size=(nlimb, cols, rows), dtype=np.uint64) * np.uint64(2) \
        + rng.integers(0, 2, size=(nlimb, cols, rows), dtype=np.uint64)
    limb[nlimb - 1] |= np.uint64(1 << 63)
    e = np.rint(rng.normal(0.0, exp_sigma, size=(cols, rows))).astype(np.int32) if exp_sigma else \
        np.zeros((cols, rows), dtype=np.int32)
    sign = rng.integers(0, 2, size=(cols, rows), dtype=np.uint8)
    if zero_frac > 0:
        z = rng.random(size=(cols, rows)) < zero_frac
        limb[:, z] = 0
        e[z] = LIMB_EXP_ZERO
        sign[z] = 0
    return limb, e, sign


def _limb_of_fraction(x: Fraction, p: int):
    """(sign, mantissa, exp) of the p-bit round-to-nearest-even of x > 0."""
    k = p - (x.numerator.bit_length() - x.denominator.bit_length())
    while x * Fraction(2) ** k >= 2 ** p:
        k -= 1
    while x * Fraction(2) ** k < 2 ** (p - 1):
        k += 1
    t = x * Fraction(2) ** k
    m = t.numerator // t.denominator
    r = t - m
    if r > Fraction(1, 2) or (r == Fraction(1, 2) and m % 2 == 1):
        m += 1
    if m == 2 ** p:
        m //= 2
        k -= 1
    return 0, m, p - k


def lotkin_limbs(n: int, nlimb: int):
    p = 64 * nlimb
    # one rounded reciprocal per denominator 1 .. 2n-1, then gathered
    table = np.zeros((nlimb, 2 * n), dtype=np.uint64)
    texp = np.zeros(2 * n, dtype=np.int32)
    for d in range(1, 2 * n):
        _, m, ex = _limb_of_fraction(Fraction(1, d), p)
        for q in range(nlimb):
            table[q, d] = (m >> (64 * q)) & ((1 << 64) - 1)
        texp[d] = ex
    ii = np.arange(n)[None, :]
    jj = np.arange(n)[:, None]
    dd = np.where(ii == 0, 1, ii + jj + 1)          # (cols, rows)
    # plane-major and C-contiguous, as the device layout (fancy indexing alone
    # would leave the limb index fastest in memory)
    limb = np.ascontiguousarray(table[:, dd])
    e = texp[dd]
    sign = np.zeros((n, n), dtype=np.uint8)
    return limb, e, sign


def lotkin_rhs_limbs(n: int, nlimb: int):
    """b = A 1 for the Lotkin limb matrix: every row of the stored (rounded)
    entries summed exactly, then rounded to nearest-even at p bits (Sec. 4.3:
    b formed at high precision and rounded to the target precision).
    Layout of a one-column limb matrix: (nlimb, 1, n), (1, n), (1, n)."""
    p = 64 * nlimb
    # the stored entry 1/d (d = 1 for row 0) as an integer on the grid 2^(emin - p)
    vals = {}
    for d in range(1, 2 * n):
        _, m, ex = _limb_of_fraction(Fraction(1, d), p)
        vals[d] = (m, ex)
    emin = min(ex for _, ex in vals.values())
    grid = {d: m << (ex - emin) for d, (m, ex) in vals.items()}
    limb_out = np.zeros((nlimb, 1, n), dtype=np.uint64)
    e_out = np.zeros((1, n), dtype=np.int32)
    s_out = np.zeros((1, n), dtype=np.uint8)
    for i in range(n):
        tot = n * grid[1] if i == 0 else sum(grid[i + j + 1] for j in range(n))
        _, m, ex = _limb_of_fraction(Fraction(tot, 1 << (p - emin)), p)
        for q in range(nlimb):
            limb_out[q, 0, i] = (m >> (64 * q)) & ((1 << 64) - 1)
        e_out[0, i] = ex
    return limb_out, e_out, s_out
