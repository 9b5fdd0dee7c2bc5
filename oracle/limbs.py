"""CPU oracle for the Ozaki-II product on arbitrary-precision limb numbers.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no
code with the GPU path.

Number format (the MPFR-like arbitrary-precision input of Sec. 3.3 and the
p-bit outputs of (S6)), p = 64 nlimb bits:

    x = (-1)^sign * (sum_q limb_q 2^(64 q)) * 2^(exp - p),

the mantissa normalised (bit 63 of the top limb set), i.e. x = 0.m * 2^exp
as MPFR's mpfr_get_exp reports it; zero has every limb 0 (its exp and sign
are not read; the oracle writes EXP_ZERO and 0).

A matrix is a tuple ``(limb, exp, sign)`` of numpy arrays with shapes
``(nlimb, cols, rows)`` uint64, ``(cols, rows)`` int32 and ``(cols, rows)``
uint8: column-major, element (i, j) at ``[.., j, i]``.

Steps, in the paper's order (Sec. 3.1 (S1)-(S6), Sec. 3.2 slices):
  (S1) e_i = max_h exp(a_ih) over non-zero entries, mu_i = Q - 1 - e_i;
  (S2) X = sgn(x) * trunc(|x| 2^mu)  (the MPFR route mpfr_mul_2si then
       mpfr_get_z, read as truncation like Eq. (direct));
  (S3) balanced w-bit slices of X, centred residues per modulus;
  (S4) modular products per (digit group, modulus) with the t_l epilogue
       of Eq. (crt) -- the oracle's C routine;
  (S5) CRT per digit group -- the oracle's C routine;
  (S6) cbar = sum_g Sbar_g 2^(w (g - g0)), rounded once to p bits,
       c = RN_p(cbar 2^(w g0 - mu_i - nu_j)), ties to even (MPFR's RNDN);
  update mode: C <- RN_p(C - c), one more correctly rounded subtraction
       (mpfr_sub with RNDN).
"""
from __future__ import annotations

from fractions import Fraction
from typing import List, Optional, Tuple

import numpy as np

from . import crt, modgemm, limbs_to_int
from .plan import Plan

EXP_ZERO = -(2 ** 31)
MASK64 = (1 << 64) - 1


# ---------------------------------------------------------------------------
# elements
# ---------------------------------------------------------------------------
def parts(L, i: int, j: int) -> Tuple[int, int, int]:
    """(sign, mantissa, exp) of element (i, j); mantissa 0 for zero."""
    limb, ex, sg = L
    m = 0
    for q in range(limb.shape[0] - 1, -1, -1):
        m = (m << 64) | int(limb[q, j, i])
    return int(sg[j, i]), m, int(ex[j, i])


def set_parts(L, i: int, j: int, sign: int, m: int, e: int) -> None:
    limb, ex, sg = L
    for q in range(limb.shape[0]):
        limb[q, j, i] = (m >> (64 * q)) & MASK64
    if m == 0:
        ex[j, i] = EXP_ZERO
        sg[j, i] = 0
    else:
        ex[j, i] = e
        sg[j, i] = sign


def value(L, i: int, j: int) -> Fraction:
    """The exact value of element (i, j)."""
    s, m, e = parts(L, i, j)
    if m == 0:
        return Fraction(0)
    p = 64 * L[0].shape[0]
    v = Fraction(m) * Fraction(2) ** (e - p)
    return -v if s else v


def rn_int(v: int, eps: int, p: int) -> Tuple[int, int, int]:
    """RN_p(v 2^eps), ties to even, for an integer v: (sign, mantissa, exp)
    with mantissa in [2^(p-1), 2^p) and value mantissa 2^(exp - p)."""
    if v == 0:
        return 0, 0, EXP_ZERO
    s = 1 if v < 0 else 0
    a = -v if v < 0 else v
    L = a.bit_length()
    if L <= p:
        return s, a << (p - L), L + eps
    sh = L - p
    m = a >> sh
    rem = a - (m << sh)
    half = 1 << (sh - 1)
    if rem > half or (rem == half and (m & 1)):
        m += 1
    if m == 1 << p:  # carried out of the p bits
        m >>= 1
        L += 1
    return s, m, L + eps


def rn_fraction(x: Fraction, p: int) -> Tuple[int, int, int]:
    """RN_p of a rational (test helper: inputs rounded to p bits)."""
    if x == 0:
        return 0, 0, EXP_ZERO
    s = 1 if x < 0 else 0
    a = -x if x < 0 else x
    # a = n/d; pick k with 2^(p-1) <= a 2^k < 2^p, then round a 2^k
    k = p - (a.numerator.bit_length() - a.denominator.bit_length())
    while a * Fraction(2) ** k >= 2 ** p:
        k -= 1
    while a * Fraction(2) ** k < 2 ** (p - 1):
        k += 1
    t = a * Fraction(2) ** k
    m = t.numerator // t.denominator
    r = t - m
    if r > Fraction(1, 2) or (r == Fraction(1, 2) and (m & 1)):
        m += 1
    if m == 1 << p:
        m >>= 1
        k -= 1
    return s, m, p - k


def sub_rn(a: Tuple[int, int, int], c: Tuple[int, int, int], p: int) -> Tuple[int, int, int]:
    """RN_p(a - c) of two p-bit numbers given as (sign, mantissa, exp):
    the exact difference as an integer on the finer grid, rounded once."""
    sa, ma, ea = a
    sc, mc, ec = c
    if mc == 0:
        return a if ma else (0, 0, EXP_ZERO)
    if ma == 0:
        return (1 - sc, mc, ec)
    lo = min(ea, ec) - p  # both values are integers times 2^lo
    va = (ma << (ea - p - lo)) * (-1 if sa else 1)
    vc = (mc << (ec - p - lo)) * (-1 if sc else 1)
    return rn_int(va - vc, lo, p)


# ---------------------------------------------------------------------------
# (S1) + (S2) + (S3)
# ---------------------------------------------------------------------------
def exponents(L, rowwise: bool) -> np.ndarray:
    """(S1): e per row (rowwise, operand A) or per column (operand B): the
    largest exp over the non-zero entries, EXP_ZERO for an all-zero line."""
    limb, ex, _ = L
    nz = np.any(limb != 0, axis=0)                    # (cols, rows)
    e = np.where(nz, ex.astype(np.int64), np.int64(EXP_ZERO))
    r = e.max(axis=0) if rowwise else e.max(axis=1)
    return r.astype(np.int64)


def fixed_point(sign: int, m: int, e: int, mu: int, p: int) -> int:
    """(S2): sgn(x) trunc(|x| 2^mu), |x| = m 2^(e - p)."""
    if m == 0:
        return 0
    s = e - p + mu
    t = m << s if s >= 0 else m >> (-s)
    return -t if sign else t


def slices(X: int, S: int, w: int) -> List[int]:
    """Balanced slices (Sec. 3.2): X = sum_t v_t 2^(w t); for t < S-1 the low
    w bits u of the remainder, centred to u - 2^w when u >= 2^(w-1); the top
    slice takes what remains."""
    out = []
    for _ in range(S - 1):
        u = X & ((1 << w) - 1)
        if u >= 1 << (w - 1):
            u -= 1 << w
        out.append(u)
        X = (X - u) >> w
    out.append(X)
    return out


def residues(L, rowwise: bool, exps, plan: Plan) -> np.ndarray:
    """Centred residue planes int32 [S, nmod, nout, K] (layout of the
    expansion oracle's ``residues``)."""
    limb = L[0]
    p = 64 * limb.shape[0]
    cols, rows = L[1].shape
    K, nout = (cols, rows) if rowwise else (rows, cols)
    S, w, Q = plan.S, plan.w, plan.Q
    mods = plan.moduli
    out = np.zeros((S, len(mods), nout, K), dtype=np.int32)
    for o in range(nout):
        e = int(exps[o])
        if e == EXP_ZERO:
            continue
        mu = Q - 1 - e
        for h in range(K):
            i, j = (o, h) if rowwise else (h, o)
            sg, m, ex = parts(L, i, j)
            if m == 0:
                continue
            for t, v in enumerate(slices(fixed_point(sg, m, ex, mu, p), S, w)):
                for li, md in enumerate(mods):
                    r = v % md
                    out[t, li, o, h] = r - md if r >= (md + 1) // 2 else r
    return out


# ---------------------------------------------------------------------------
# the product
# ---------------------------------------------------------------------------
def group_sums(A, B, plan: Plan):
    """(S1)-(S5): exponents and the exact digit-group sums Sbar_g as Python
    ints, list over groups of [N][M] nested lists."""
    ea, eb = exponents(A, True), exponents(B, False)
    pa = residues(A, True, ea, plan)
    pb = residues(B, False, eb, plan)
    tpl = modgemm(pa, pb, plan)
    nw = (plan.P.bit_length() + 64) // 64 + 1
    sb = crt(tpl, plan, nw)                               # [ng, N, M, nw]
    ng, N, M = sb.shape[0], sb.shape[1], sb.shape[2]
    sums = [[[limbs_to_int(sb[g, j, i]) for i in range(M)] for j in range(N)] for g in range(ng)]
    return ea, eb, sums


def ozgemm(mode: int, A, B, C, plan: Plan):
    """C = A B (mode 0) or C = C - A B (mode 1) on limb matrices; returns the
    new C (a copy) and the rounded products c as (sign, mantissa, exp)."""
    p = 64 * A[0].shape[0]
    ea, eb, sums = group_sums(A, B, plan)
    w, g0, Q = plan.w, plan.g0, plan.Q
    ng = len(sums)
    N, M = C[1].shape
    out = tuple(np.array(x, copy=True) for x in C)
    prods = {}
    for j in range(N):
        for i in range(M):
            if ea[i] == EXP_ZERO or eb[j] == EXP_ZERO:
                c = (0, 0, EXP_ZERO)
            else:
                cbar = 0
                for gi in range(ng - 1, -1, -1):
                    cbar = (cbar << w) + sums[gi][j][i]
                eps = w * g0 - (Q - 1 - int(ea[i])) - (Q - 1 - int(eb[j]))
                c = rn_int(cbar, eps, p)
            prods[(i, j)] = c
            r = c if mode == 0 else sub_rn(parts(C, i, j), c, p)
            set_parts(out, i, j, *r)
    return out, prods


def exact_product(A, B, i: int, j: int) -> Fraction:
    """sum_h a_ih b_hj exactly (test helper)."""
    K = A[1].shape[0]
    return sum((value(A, i, h) * value(B, h, j) for h in range(K)), Fraction(0))
