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


def getrf(A, b: int, method: str = "ozaki", extra_groups: int = 0):
    """Blocked LU of the n x n limb matrix A with panel width b.  Returns
    (LU in the limbs.py layout, ipiv (0-based rows, LAPACK semantics), info)."""
    X = to_lf(A)
    m, e, s = X
    n = e.shape[0]
    nl = m.shape[2]
    ld = n
    ipiv = np.zeros(n, dtype=np.int64)
    info = 0
    b = max(1, int(b))
    for k0 in range(0, n, b):
        kb = min(b, n - k0)
        piv = np.zeros(kb, dtype=np.int64)
        inf = np.zeros(1, dtype=np.int32)
        lib().orc_lf_getf2(nl, n - k0, kb, *_ptrs(X, k0, k0, ld), ld, piv.ctypes.data_as(_i64p),
                           inf.ctypes.data_as(_i32p))
        ipiv[k0:k0 + kb] = piv + k0
        if inf[0] and not info:
            info = k0 + int(inf[0])
        others = np.r_[0:k0, k0 + kb:n]
        for jj in range(k0, k0 + kb):
            r = int(ipiv[jj])
            if r != jj and others.size:
                _swap_rows(X, jj, r, others)
        rest = n - k0 - kb
        if rest == 0:
            continue
        lib().orc_lf_trsm_lunit(nl, kb, rest, *_ptrs(X, k0, k0, ld), ld,
                                *_ptrs(X, k0, k0 + kb, ld), ld)
        if method == "native":
            lib().orc_lf_gemm_sub(nl, rest, rest, kb, *_ptrs(X, k0 + kb, k0, ld), ld,
                                  *_ptrs(X, k0, k0 + kb, ld), ld, *_ptrs(X, k0 + kb, k0 + kb, ld),
                                  ld)
        elif method == "ozaki":
            def sub(r0, r1, c0, c1):
                return from_lf((m[c0:c1, r0:r1], e[c0:c1, r0:r1], s[c0:c1, r0:r1]))
            L21 = sub(k0 + kb, n, k0, k0 + kb)
            U12 = sub(k0, k0 + kb, k0 + kb, n)
            A22 = sub(k0 + kb, n, k0 + kb, n)
            plan = make_plan(64 * nl, kb, extra_groups=extra_groups)
            out, _ = OL.ozgemm(1, L21, U12, A22, plan)
            om, oe, os_ = to_lf(out)
            m[k0 + kb:, k0 + kb:] = om
            e[k0 + kb:, k0 + kb:] = oe
            s[k0 + kb:, k0 + kb:] = os_
        else:
            raise ValueError(method)
    return from_lf(X), ipiv, info


def getrs(LU, ipiv, B):
    """Solve from getrf's factors; B in the limbs.py layout with shape
    (nl, nrhs, n); returns X in the same layout."""
    F = to_lf(LU)
    Xb = to_lf(B)
    R = LF.getrs(F, ipiv, Xb)
    return from_lf(R)
