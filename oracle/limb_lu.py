"""Blocked LU with partial pivoting on limb matrices: the CPU oracle of the
limb-format getrf / getrs.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no
code with the GPU path.

Matrices use the limb layout of ``limbs.py``: a tuple ``(limb, exp, sign)``
of shapes ``(nl, cols, rows)`` uint64, ``(cols, rows)`` int32 and
``(cols, rows)`` uint8, x = (-1)^sign m 2^(exp - p), p = 64 nl, zero with
every limb 0.  Every scalar operation is the correctly rounded p-bit one of
``lfloat.c`` (MPFR's RNDN, the number type of Sec. 2).

The blocked right-looking LU of Sec. 3.4, for each panel of b columns:
  1. the unblocked panel (``orc_lf_getf2``): pivot = largest exact magnitude,
     ties to the lowest row, interchange inside the panel, l = RN(a / pivot),
     rank-1 multiply-subtracts RN(a - RN(l u)) on the panel's columns;
  2. the interchanges on the columns left and right of the panel;
  3. U12 <- L11^-1 U12 by the same multiply-subtracts (unit lower solve);
  4. the Schur update A22 <- A22 - L21 U12, either
       "ozaki":  RN_p(a - RN_p(L21 U12)) with the Ozaki-II product of
                 ``limbs.ozgemm`` (plan ``make_plan(p, b)``), or
       "native": RN(a - RN(l_ik u_kj)) for k ascending.
With the native update every element receives the operations of the
unblocked LU in the same order, so the result equals ``orc_lf_getrf`` bit
for bit for any b; with b >= n the Ozaki variant is the unblocked LU too.

With leaf > 0 the panel and the U12 solve recurse (the acceleration of the
panel by Ozaki-II that Sec. 5.2 proposes): a panel of w > leaf columns
factors its left part (w1 = half its leaf-wide blocks), solves the rows
above for its right part, updates the rows below it with the left part's
L (K = w1) and factors the rest; a solve of h > leaf rows solves the top
h1 rows, updates the rest, and solves them.  Leaves are the unblocked
panel (interchanges across the whole panel) and the multiply-subtract
solve.  With multiply-subtract updates the result is still the unblocked
LU bit for bit.
The solve is ``orc_lf_getrs`` (Sec. 4.3: forward and backward substitution,
x_k divided by u_kk).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _i32p, _i64p, _u8p, _u64p, lib, make_plan
from . import limbs as OL
from . import lfloat as LF

EXP32_ZERO = -(2 ** 31)


def to_lf(L):
    """limbs.py layout -> lfloat arrays (m (cols, rows, nl), e int64, s)."""
    limb, ex, sg = L
    m = np.array(np.moveaxis(np.asarray(limb, dtype=np.uint64), 0, 2), order="C", copy=True)
    zero = ~np.any(m != 0, axis=2)
    e = np.where(zero, np.int64(LF.EXP_ZERO), np.asarray(ex).astype(np.int64))
    s = np.where(zero, np.uint8(0), np.asarray(sg).astype(np.uint8))
    return m, np.ascontiguousarray(e), np.ascontiguousarray(s)


def from_lf(X):
    """lfloat arrays -> limbs.py layout (zero: exp INT32_MIN, sign 0)."""
    m, e, s = X
    limb = np.array(np.moveaxis(m, 2, 0), order="C", copy=True)
    ex = np.where(e == LF.EXP_ZERO, np.int64(EXP32_ZERO), e).astype(np.int32)
    return limb, np.ascontiguousarray(ex), np.ascontiguousarray(s.astype(np.uint8))


def _at(arr, off, t):
    """Pointer to element `off` (flat, in elements of the leading layout)."""
    step = arr.strides[1] if arr.ndim == 3 else arr.itemsize
    return ctypes.cast(ctypes.c_void_p(arr.ctypes.data + off * step), t)


def _ptrs(X, i, j, ld):
    m, e, s = X
    off = i + j * ld
    return _at(m, off, _u64p), _at(e, off, _i64p), _at(s, off, _u8p)


def _swap_rows(X, r1, r2, cols):
    m, e, s = X
    for a in (m, e, s):
        t = a[cols, r1].copy()
        a[cols, r1] = a[cols, r2]
        a[cols, r2] = t


def split(w: int, leaf: int) -> int:
    """Left part of a recursive split of w > leaf columns: half of the
    leaf-wide blocks, rounded up."""
    blocks = -(-w // leaf)
    return -(-blocks // 2) * leaf


class _LU:
    """The blocked LU's steps on the lfloat arrays X of an n x n matrix."""

    def __init__(self, X, method, leaf, extra_groups, nslice=0):
        self.X = X
        self.m, self.e, self.s = X
        self.n = self.e.shape[0]
        self.nl = self.m.shape[2]
        self.method = method
        self.leaf = leaf
        self.extra_groups = extra_groups
        self.nslice = nslice
        self.ipiv = np.zeros(self.n, dtype=np.int64)
        self.info = 0

    def update(self, i0, i1, c0, c1, k0, K):
        """A[i0:i1, c0:c1] -= A[i0:i1, k0:k0+K] A[k0:k0+K, c0:c1]."""
        n, nl, X = self.n, self.nl, self.X
        if i1 <= i0 or c1 <= c0 or K == 0:
            return
        if self.method == "native":
            lib().orc_lf_gemm_sub(nl, i1 - i0, c1 - c0, K, *_ptrs(X, i0, k0, n), n,
                                  *_ptrs(X, k0, c0, n), n, *_ptrs(X, i0, c0, n), n)
            return
        m, e, s = self.m, self.e, self.s

        def sub(r0, r1, cc0, cc1):
            return from_lf((m[cc0:cc1, r0:r1], e[cc0:cc1, r0:r1], s[cc0:cc1, r0:r1]))
        plan = make_plan(64 * nl, K, nslice=self.nslice, extra_groups=self.extra_groups)
        out, _ = OL.ozgemm(1, sub(i0, i1, k0, k0 + K), sub(k0, k0 + K, c0, c1),
                           sub(i0, i1, c0, c1), plan)
        om, oe, os_ = to_lf(out)
        m[c0:c1, i0:i1] = om
        e[c0:c1, i0:i1] = oe
        s[c0:c1, i0:i1] = os_

    def trsm(self, r0, h, b0, b1):
        """B = A[r0:r0+h, b0:b1] <- L^-1 B, L the unit lower triangle at
        (r0, r0): multiply-subtracts in leaves, the rest by updates."""
        if b1 <= b0 or h <= 1:
            return
        n, nl, X = self.n, self.nl, self.X
        if not self.leaf or h <= self.leaf:
            lib().orc_lf_trsm_lunit(nl, h, b1 - b0, *_ptrs(X, r0, r0, n), n,
                                    *_ptrs(X, r0, b0, n), n)
            return
        h1 = split(h, self.leaf)
        self.trsm(r0, h1, b0, b1)
        self.update(r0 + h1, r0 + h, b0, b1, r0, h1)
        self.trsm(r0 + h1, h - h1, b0, b1)

    def panel(self, c0, w, P0, P1):
        """Columns [c0, c0+w) over rows [c0, n); interchanges across the
        whole panel [P0, P1)."""
        n, nl, X = self.n, self.nl, self.X
        if not self.leaf or w <= self.leaf:
            piv = np.zeros(w, dtype=np.int64)
            inf = np.zeros(1, dtype=np.int32)
            lib().orc_lf_getf2(nl, n - c0, w, *_ptrs(X, c0, c0, n), n,
                               piv.ctypes.data_as(_i64p), inf.ctypes.data_as(_i32p))
            self.ipiv[c0:c0 + w] = piv + c0
            if inf[0] and not self.info:
                self.info = c0 + int(inf[0])
            others = np.r_[P0:c0, c0 + w:P1]
            for jj in range(c0, c0 + w):
                r = int(self.ipiv[jj])
                if r != jj and others.size:
                    _swap_rows(X, jj, r, others)
            return
        w1 = split(w, self.leaf)
        self.panel(c0, w1, P0, P1)
        self.trsm(c0, w1, c0 + w1, c0 + w)
        self.update(c0 + w1, n, c0 + w1, c0 + w, c0, w1)
        self.panel(c0 + w1, w - w1, P0, P1)


def getrf(A, b: int, method: str = "ozaki", extra_groups: int = 0, leaf: int = 0,
          nslice: int = 0):
    """Blocked LU of the n x n limb matrix A with panel width b.  leaf > 0:
    the panel and the U12 solve recurse on halves down to leaf columns or
    rows, the inner updates made like the Schur update (Ozaki-II or
    multiply-subtracts).  Returns (LU in the limbs.py layout, ipiv (0-based
    rows, LAPACK semantics), info)."""
    if method not in ("ozaki", "native"):
        raise ValueError(method)
    L = _LU(to_lf(A), method, leaf, extra_groups, nslice)
    n = L.n
    b = max(1, int(b))
    for k0 in range(0, n, b):
        kb = min(b, n - k0)
        L.panel(k0, kb, k0, k0 + kb)
        others = np.r_[0:k0, k0 + kb:n]
        for jj in range(k0, k0 + kb):
            r = int(L.ipiv[jj])
            if r != jj and others.size:
                _swap_rows(L.X, jj, r, others)
        if n - k0 - kb == 0:
            continue
        L.trsm(k0, kb, k0 + kb, n)
        L.update(k0 + kb, n, k0 + kb, n, k0, kb)
    return from_lf(L.X), L.ipiv, L.info


def getrs(LU, ipiv, B):
    """Solve from getrf's factors; B in the limbs.py layout with shape
    (nl, nrhs, n); returns X in the same layout."""
    F = to_lf(LU)
    Xb = to_lf(B)
    R = LF.getrs(F, ipiv, Xb)
    return from_lf(R)
