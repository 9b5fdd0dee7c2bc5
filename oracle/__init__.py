"""CPU oracle for the Ozaki-scheme-II multiple-precision LU.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(``paper_2609_29554_amd``) never imports it, and the two share no code.

Matrices are numpy float64 arrays of shape ``(cols, rows, nc)``: column-major,
each element an array of ``nc`` doubles (a DD/TD/QD non-overlapping
expansion, Sec. 2 of the paper).  Element (i, j) component c is ``X[j, i, c]``,
i.e. flat index ``(i + j*rows)*nc + c``.

The heavy lifting is in ``oracle.c`` (plain C, its own big integers, built
with ``-ffp-contract=off``) and ``lfloat.c`` (p-bit floating point with
correct rounding and the LU on it, used at twice the working precision);
``plan.py`` holds the plan rule, ``limbs.py`` the limb-format product and
``lfloat.py`` the p-bit LU.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Tuple

import numpy as np

from .plan import (BACKEND_F64MOD, BACKEND_FP16, BACKEND_FP8_B17, BACKEND_INT8, Plan,  # noqa: F401
                   make_plan, int8_moduli, f64_moduli, lhint)

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
EXP_ZERO = -(2 ** 31)
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (plain gcc, no GPU code)."""
    import subprocess
    srcs = [os.path.join(_HERE, f) for f in ("oracle.c", "lfloat.c")]
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-fopenmp", "-shared", "-fPIC", "-o", tmp] + srcs)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = C.CDLL(_LIB_PATH)
        _declare(_lib)
    return _lib


_dp = C.POINTER(C.c_double)
_i8p = C.POINTER(C.c_int8)
_u8p = C.POINTER(C.c_uint8)
_u32p = C.POINTER(C.c_uint32)
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_u64p = C.POINTER(C.c_uint64)
_i64 = C.c_int64
_int = C.c_int


def _declare(L):
    L.orc_exp_vec.argtypes = [_int, _int, _i64, _dp, _dp, _dp, _dp]
    L.orc_abs_greater.argtypes = [_int, _dp, _dp]
    L.orc_abs_greater.restype = _int
    L.orc_exponents.argtypes = [_int, _i64, _i64, _dp, _i64, _int, _i32p]
    L.orc_residues.argtypes = [_int, _i64, _i64, _dp, _i64, _int, _i32p, _int, _int, _int,
                               _i32p, _i32p]
    L.orc_modgemm.argtypes = [_i64, _i64, _i64, _i32p, _i32p, _int, _int, _i32p, _i32p, _int,
                              _u32p, _i64p]
    L.orc_crt.argtypes = [_i64, _i64, _u32p, _int, _int, _i32p, _int, _u64p]
    L.orc_fp8_digits.argtypes = [_i64, _i32p, _i32p, _i32p]
    L.orc_e4m3_int.argtypes = [C.c_int32]
    L.orc_e4m3_int.restype = C.c_uint8
    L.orc_round_out.argtypes = [_int, _u64p, _int, _int, _dp]
    L.orc_ozgemm.argtypes = [_int, _int, _i64, _i64, _i64, _dp, _i64, _dp, _i64, _dp, _i64,
                             _int, _int, _int, _int, _u64p]
    L.orc_naive_gemm.argtypes = [_int, _int, _i64, _i64, _i64, _dp, _i64, _dp, _i64, _dp, _i64]
    L.orc_getrf.argtypes = [_int, _i64, _dp, _i64, _i64, _int, _int, _int, _int, _i64p, _i32p,
                            _dp]
    L.orc_getrs.argtypes = [_int, _i64, _dp, _i64, _i64p, _i64, _dp, _i64]
    L.orc_lf_vec.argtypes = [_int, _int, _i64, _u64p, _i64p, _u8p, _u64p, _i64p, _u8p, _u64p,
                             _i64p, _u8p]
    L.orc_lf_from_doubles.argtypes = [_int, _i64, _int, _dp, _u64p, _i64p, _u8p]
    L.orc_lf_getrf.argtypes = [_int, _i64, _u64p, _i64p, _u8p, _i64, _i64p, _i32p]
    L.orc_lf_getrs.argtypes = [_int, _i64, _u64p, _i64p, _u8p, _i64, _i64p, _i64, _u64p, _i64p,
                               _u8p, _i64]
    L.orc_lf_getf2.argtypes = [_int, _i64, _i64, _u64p, _i64p, _u8p, _i64, _i64p, _i32p]
    L.orc_lf_trsm_lunit.argtypes = [_int, _i64, _i64, _u64p, _i64p, _u8p, _i64, _u64p, _i64p,
                                    _u8p, _i64]
    L.orc_lf_gemm_sub.argtypes = [_int, _i64, _i64, _i64, _u64p, _i64p, _u8p, _i64, _u64p,
                                  _i64p, _u8p, _i64, _u64p, _i64p, _u8p, _i64]


def _p(a, t):
    return a.ctypes.data_as(t)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# expansion arithmetic (written spec; see oracle.c)
# --------------------------------------------------------------------------
def _vec(op, a, b, c=None):
    a = _f64(a)
    b = _f64(b)
    nc = a.shape[-1]
    cnt = a.size // nc
    r = np.empty_like(a)
    cc = _f64(c) if c is not None else a
    lib().orc_exp_vec(op, nc, cnt, _p(a, _dp), _p(b, _dp), _p(cc, _dp), _p(r, _dp))
    return r


def exp_add(a, b):
    return _vec(0, a, b)


def exp_mul(a, b):
    return _vec(1, a, b)


def exp_fms(c, a, b):
    """c - a*b"""
    return _vec(2, a, b, c)


def exp_div(a, b):
    return _vec(3, a, b)


def abs_greater(a, b) -> bool:
    a = _f64(a)
    b = _f64(b)
    return bool(lib().orc_abs_greater(a.shape[-1], _p(a, _dp), _p(b, _dp)))


# --------------------------------------------------------------------------
# Ozaki-II stages
# --------------------------------------------------------------------------
def exponents(X, rowwise: bool) -> np.ndarray:
    """(S1): max frexp exponent per row (rowwise) or per column."""
    X = _f64(X)
    cols, rows, nc = X.shape
    out = np.empty(rows if rowwise else cols, dtype=np.int32)
    lib().orc_exponents(nc, rows, cols, _p(X, _dp), rows, int(rowwise), _p(out, _i32p))
    return out


def residues(X, rowwise: bool, exps, plan: Plan) -> np.ndarray:
    """(S2)+(S3): centred residues of the balanced slices.

    rowwise (A operand, rows x K): returns int32 [S, nmod, rows, K];
    otherwise (B operand, K x cols): int32 [S, nmod, cols, K]."""
    X = _f64(X)
    cols, rows, nc = X.shape
    exps = np.ascontiguousarray(exps, dtype=np.int32)
    mods = np.array(plan.moduli, dtype=np.int32)
    nout, K = (rows, cols) if rowwise else (cols, rows)
    out = np.empty((plan.S, plan.nmod, nout, K), dtype=np.int32)
    lib().orc_residues(nc, rows, cols, _p(X, _dp), rows, int(rowwise), _p(exps, _i32p),
                       plan.S, plan.w, plan.nmod, _p(mods, _i32p), _p(out, _i32p))
    return out


def modgemm(pa, pb, plan: Plan, want_cmax: bool = False):
    """(S4) + t_l of Eq. (crt): uint32 t-planes [ngroups, nmod, N, M] (values
    below the modulus).  With want_cmax, also max |C| over every product."""
    S, nmod, M, K = pa.shape
    N = pb.shape[2]
    pa = np.ascontiguousarray(pa, dtype=np.int32)
    pb = np.ascontiguousarray(pb, dtype=np.int32)
    mods = np.array(plan.moduli, dtype=np.int32)
    y = np.array(plan.y, dtype=np.int32)
    ng = len(plan.groups)
    out = np.empty((ng, nmod, N, M), dtype=np.uint32)
    cmax = np.zeros(1, dtype=np.int64)
    lib().orc_modgemm(M, N, K, _p(pa, _i32p), _p(pb, _i32p), S, nmod, _p(mods, _i32p),
                      _p(y, _i32p), plan.g0, _p(out, _u32p), _p(cmax, _i64p))
    return (out, int(cmax[0])) if want_cmax else out


def fp8_digits(r):
    """Balanced base-17 digits (d0, d1) of residues r (Eq. fp8digits)."""
    r = np.ascontiguousarray(r, dtype=np.int32)
    d0 = np.empty_like(r)
    d1 = np.empty_like(r)
    lib().orc_fp8_digits(r.size, _p(r, _i32p), _p(d0, _i32p), _p(d1, _i32p))
    return d0, d1


def e4m3_int(d: int) -> int:
    """OCP FP8 E4M3 byte of a small integer (|d| <= 16)."""
    return int(lib().orc_e4m3_int(int(d)))


def crt(tpl, plan: Plan, nw: int = 8) -> np.ndarray:
    """(S5), CPU encoding: signed group sums as nw-limb two's complement,
    uint64 [ngroups, N, M, nw]."""
    ng, nmod, N, M = tpl.shape
    tpl = np.ascontiguousarray(tpl, dtype=np.uint32)
    mods = np.array(plan.moduli, dtype=np.int32)
    out = np.empty((ng, N, M, nw), dtype=np.uint64)
    lib().orc_crt(M, N, _p(tpl, _u32p), ng, nmod, _p(mods, _i32p), nw, _p(out, _u64p))
    return out


def limbs_to_int(a) -> int:
    """Two's-complement little-endian uint64 limbs -> Python int."""
    a = [int(x) for x in np.asarray(a, dtype=np.uint64).ravel()]
    v = 0
    for i, x in enumerate(a):
        v |= x << (64 * i)
    if a and a[-1] >> 63:
        v -= 1 << (64 * len(a))
    return v


def int_to_limbs(v: int, nw: int) -> np.ndarray:
    v &= (1 << (64 * nw)) - 1
    return np.array([(v >> (64 * i)) & ((1 << 64) - 1) for i in range(nw)], dtype=np.uint64)


def round_out(value: int, eps: int, nc: int, nw: int = 16) -> np.ndarray:
    """(S6): greedy round-to-nearest nc-component expansion of value*2^eps."""
    limbs = int_to_limbs(value, nw)
    out = np.zeros(nc, dtype=np.float64)
    lib().orc_round_out(nw, _p(limbs, _u64p), eps, nc, _p(out, _dp))
    return out


def ozgemm(mode: int, A, B, Cm, plan: Plan, want_sbar: bool = False, nw_out: int = 8):
    """Ozaki-II product from its definition.  A: (K, M, nc), B: (N, K, nc),
    C: (N, M, nc).  mode 0: C = A*B; mode 1: C = C - A*B.
    Returns (C, sbar or None); sbar is uint64 [ngroups, N, M, nw_out]."""
    A = _f64(A)
    B = _f64(B)
    Cm = _f64(Cm).copy()
    K, M, nc = A.shape
    N = B.shape[0]
    assert B.shape[1] == K and Cm.shape[:2] == (N, M)
    sb = None
    sbp = None
    if want_sbar:
        sb = np.empty((len(plan.groups), N, M, nw_out), dtype=np.uint64)
        sbp = _p(sb, _u64p)
    lib().orc_ozgemm(mode, nc, M, N, K, _p(A, _dp), M, _p(B, _dp), K, _p(Cm, _dp), M,
                     plan.S, plan.w, plan.g0, nw_out, sbp)
    return Cm, sb


def naive_gemm(mode: int, A, B, Cm):
    A = _f64(A)
    B = _f64(B)
    Cm = _f64(Cm).copy()
    K, M, nc = A.shape
    N = B.shape[0]
    lib().orc_naive_gemm(mode, nc, M, N, K, _p(A, _dp), M, _p(B, _dp), K, _p(Cm, _dp), M)
    return Cm


METHOD_OZAKI = 0
METHOD_NAIVE = 1


def getrf(A, b: int, method: int = METHOD_OZAKI, plan: Optional[Plan] = None):
    """Blocked right-looking LU with partial pivoting (Sec. 3.4).

    A: (n, n, nc).  Returns (LU, ipiv (0-based, LAPACK semantics), info,
    (panel_seconds, update_seconds))."""
    A = _f64(A).copy()
    n = A.shape[0]
    nc = A.shape[2]
    if method == METHOD_OZAKI:
        if plan is None:
            plan = make_plan(53 * nc, b)
        S, w, g0 = plan.S, plan.w, plan.g0
    else:
        S, w, g0 = 1, 1, 0
    ipiv = np.zeros(n, dtype=np.int64)
    info = np.zeros(1, dtype=np.int32)
    tm = np.zeros(2, dtype=np.float64)
    lib().orc_getrf(nc, n, _p(A, _dp), n, b, method, S, w, g0, _p(ipiv, _i64p),
                    _p(info, _i32p), _p(tm, _dp))
    return A, ipiv, int(info[0]), (float(tm[0]), float(tm[1]))


def getrs(LU, ipiv, B):
    """Solve from getrf's factors; B: (nrhs, n, nc)."""
    LU = _f64(LU)
    B = _f64(B).copy()
    n = LU.shape[0]
    nc = LU.shape[2]
    nrhs = B.shape[0]
    ipiv = np.ascontiguousarray(ipiv, dtype=np.int64)
    lib().orc_getrs(nc, n, _p(LU, _dp), n, _p(ipiv, _i64p), nrhs, _p(B, _dp), n)
    return B
