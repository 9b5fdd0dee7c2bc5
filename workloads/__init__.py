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
