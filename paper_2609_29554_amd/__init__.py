"""Python binding of libozii (Ozaki-scheme-II multiple-precision LU on gfx950).

Argument marshalling only: every step runs in the HIP kernels of libozii.so.
PyTorch supplies device memory and the stream.  There is no CPU fallback: if
the library is not built, importing works but every call raises.

Matrices are float64 CUDA tensors of shape (cols, rows, nc), contiguous: the
column-major array of nc-component expansions that the C ABI expects
(element (i, j) component c at flat index (i + j*rows)*nc + c).
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import sys
import weakref
from typing import Optional, Tuple

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libozii.so")

OK, EINVAL, ECAPACITY, EOVERFLOW, ENOMEM, EHIP, EUNSUPPORTED, EDEVICE = range(8)
BE_AUTO, BE_INT8, BE_FP8_B17, BE_F64MOD, BE_FP16 = range(5)
METHOD_OZAKI, METHOD_NAIVE = 0, 1
TILE_AUTO, TILE_128x128, TILE_256x128, TILE_256x256 = range(4)
F_NO_LOOKAHEAD = 1
F_FUSED = 2


class OziiError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ozii status {status}: {msg}")
        self.status = status


class Opts(C.Structure):
    _fields_ = [("backend", C.c_int32), ("nslice", C.c_int32), ("extra_groups", C.c_int32),
                ("guard_ex", C.c_int32), ("block", C.c_int32), ("method", C.c_int32),
                ("flags", C.c_int32), ("gemm_tile", C.c_int32), ("qbits", C.c_int32),
                ("panel_leaf", C.c_int32)]


_lib = None
_p = C.c_void_p
_i64 = C.c_int64
_i32 = C.c_int32

EXPORTED = ["ozII_create", "ozII_destroy", "ozII_set_stream", "ozII_plan_query", "ozII_reserve",
            "ozII_gemm", "ozII_gemm_noalloc", "ozII_gemm_noalloc_capacity",
            "ozII_gemm_limbs", "ozII_gemm_limbs_stages", "ozII_gemm_stages",
            "ozII_gemm_stage_dims",
            "ozII_getrf", "ozII_getrs", "ozII_getrf_limbs", "ozII_getrs_limbs",
            "ozII_limbs_arith",
            "ozII_batch_prepare", "ozII_batch_prepare_ex", "ozII_batch_run", "ozII_tune",
            "ozII_tune_limbs",
            "ozII_stream_of",
            "ozII_sync_check", "ozII_set_profiling",
            "ozII_profile_read", "ozII_status_string", "ozII_last_error"]

class Limbs(C.Structure):
    """ozII_limbs: limb planes, exponents, signs, ld, plane (device pointers)."""
    _fields_ = [("limb", C.c_void_p), ("exp", C.c_void_p), ("sign", C.c_void_p),
                ("ld", C.c_int64), ("plane", C.c_int64)]


class BatchItem(C.Structure):
    _fields_ = [("nc", C.c_int32), ("reserved", C.c_int32), ("n", C.c_int64), ("A", C.c_void_p),
                ("b", C.c_void_p), ("ipiv", C.c_void_p), ("info", C.c_void_p)]


TUNE_RETUNE = 1
TUNE_MAXCAND = 40


class TuneReport(C.Structure):
    _fields_ = [("ncand", C.c_int32), ("best", C.c_int32), ("from_cache", C.c_int32),
                ("reserved", C.c_int32), ("cand", Opts * TUNE_MAXCAND),
                ("ms", C.c_double * TUNE_MAXCAND), ("model_ms", C.c_double * TUNE_MAXCAND)]

STAGES = ["exponents", "producer", "gemm", "consumer", "panel", "laswp", "trsm", "naive_update",
          "getrs", "round", "fused"]


def lib():
    """Load libozii.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        # torch first: PyTorch ships its own HIP runtime under the same soname,
        # and the library must bind to that one.  Loaded first, the library
        # would pull in the system runtime and torch its own, and two HIP
        # runtimes in one process do not share devices, memory or streams.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        OP = C.POINTER(Opts)
        L.ozII_create.argtypes = [C.POINTER(_p), C.c_int, _p]
        L.ozII_destroy.argtypes = [_p]
        L.ozII_set_stream.argtypes = [_p, _p]
        L.ozII_plan_query.argtypes = [_i32, _i64, OP, C.POINTER(_i32), C.POINTER(_i32),
                                      C.POINTER(_i32), C.POINTER(_i32), C.POINTER(_i32)]
        L.ozII_reserve.argtypes = [_p, _i32, _i64, _i64, _i64, _i64, OP]
        L.ozII_gemm.argtypes = [_p, _i32, _i32, _i64, _i64, _i64, _p, _i64, _p, _i64, _p, _i64, OP]
        L.ozII_gemm_noalloc.argtypes = L.ozII_gemm.argtypes
        L.ozII_gemm_noalloc_capacity.argtypes = [C.POINTER(_i64)]
        LP = C.POINTER(Limbs)
        L.ozII_gemm_limbs.argtypes = [_p, _i32, _i32, _i64, _i64, _i64, LP, LP, LP, OP]
        L.ozII_gemm_limbs_stages.argtypes = [_p, _i32, _i32, _i64, _i64, _i64, LP, LP, LP, OP,
                                             _p, _i32]
        L.ozII_gemm_stages.argtypes = [_p, _i32, _i32, _i64, _i64, _i64, _p, _i64, _p, _i64, _p,
                                       _i64, OP, _p, _p, _p, _p, _p, _p, _i32]
        L.ozII_gemm_stage_dims.argtypes = [_i32, _i64, _i64, _i64, OP, C.POINTER(_i64),
                                           C.POINTER(_i64), C.POINTER(_i64), C.POINTER(_i32),
                                           C.POINTER(_i32), C.POINTER(_i32)]
        L.ozII_getrf.argtypes = [_p, _i32, _i64, _p, _i64, _p, _p, OP]
        L.ozII_getrs.argtypes = [_p, _i32, _i64, _i64, _p, _i64, _p, _p, _i64]
        L.ozII_getrf_limbs.argtypes = [_p, _i32, _i64, LP, _p, _p, OP]
        L.ozII_getrs_limbs.argtypes = [_p, _i32, _i64, _i64, LP, _p, LP]
        L.ozII_limbs_arith.argtypes = [_p, _i32, _i32, _i64, LP, LP, LP]
        L.ozII_tune.argtypes = [_p, _i32, _i64, C.c_char_p, _i32, OP, C.POINTER(TuneReport)]
        L.ozII_tune_limbs.argtypes = [_p, _i32, _i64, C.c_char_p, _i32, OP,
                                      C.POINTER(TuneReport)]
        L.ozII_batch_prepare.argtypes = [_p, _i32, C.POINTER(BatchItem)]
        L.ozII_batch_prepare_ex.argtypes = [_p, _i32, C.POINTER(BatchItem), OP]
        L.ozII_batch_run.argtypes = [_p, _p]
        L.ozII_stream_of.argtypes = [_p, C.POINTER(_p)]
        L.ozII_sync_check.argtypes = [_p]
        L.ozII_set_profiling.argtypes = [_p, _i32]
        L.ozII_profile_read.argtypes = [_p, _i32, _p, _p, _p, _p]
        L.ozII_status_string.argtypes = [C.c_int]
        L.ozII_status_string.restype = C.c_char_p
        L.ozII_last_error.argtypes = [_p]
        L.ozII_last_error.restype = C.c_char_p
        for name in EXPORTED:
            if name not in ("ozII_status_string", "ozII_last_error"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def noalloc_capacity() -> int:
    """Workspace bytes of ozII_gemm_noalloc's static scratch."""
    v = _i64()
    st = lib().ozII_gemm_noalloc_capacity(C.byref(v))
    if st != OK:
        raise OziiError(st, "capacity")
    return v.value


def make_opts(backend: int = 0, nslice: int = 0, extra_groups: int = 0, guard_ex: int = 0,
              block: int = 0, method: int = 0, gemm_tile: int = 0, flags: int = 0,
              qbits: int = 0, panel_leaf: int = 0) -> Opts:
    return Opts(backend, nslice, extra_groups, guard_ex, block, method, flags, gemm_tile, qbits,
                panel_leaf)


def plan_query(p: int, K: int, opts: Optional[Opts] = None):
    """Plan of Sec. 3.2 as the library computes it: (S, w, Q, nmod, moduli)."""
    S, w, Q, n = _i32(), _i32(), _i32(), _i32()
    mods = (_i32 * 64)()
    st = lib().ozII_plan_query(p, K, C.byref(opts) if opts else None, C.byref(S), C.byref(w),
                               C.byref(Q), C.byref(n), mods)
    if st != OK:
        raise OziiError(st, lib().ozII_status_string(st).decode())
    return S.value, w.value, Q.value, n.value, list(mods[: n.value])


def _ptr(t) -> int:
    return t.data_ptr()


def _check_mat(t, nc: Optional[int] = None):
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.dim() == 3):
        raise ValueError("expected a contiguous float64 CUDA tensor of shape (cols, rows, nc)")
    if t.shape[2] not in (2, 3, 4):
        raise ValueError("expansions have 2, 3 or 4 components")
    if nc is not None and t.shape[2] != nc:
        raise ValueError("component count mismatch")


def _check_vec(t, dtype, length: int, name: str):
    """A contiguous CUDA vector of `dtype` with at least `length` entries."""
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous() and t.dim() == 1):
        raise ValueError(f"{name}: expected a contiguous 1-D {dtype} CUDA tensor")
    if t.numel() < length:
        raise ValueError(f"{name}: needs at least {length} entries, has {t.numel()}")


def check_limb_mat(X, nl=None, device=None):
    """(nlimb, cols, rows) of a limb matrix (limb, exp, sign): contiguous
    CUDA tensors of shapes (nlimb, cols, rows) int64, (cols, rows) int32 and
    (cols, rows) uint8, nlimb in 1..64 (a mismatch would be read out of
    bounds on the device)."""
    import torch
    if not (isinstance(X, (tuple, list)) and len(X) == 3):
        raise ValueError("limb matrix: tuple (limb, exp, sign)")
    lb, ex, sg = X
    for t in (lb, ex, sg):
        if not (getattr(t, "is_cuda", False) and t.is_contiguous()):
            raise ValueError("limb matrix: contiguous CUDA tensors")
        if device is not None and t.device != device:
            raise ValueError("limb operands must be on one device")
    if lb.dtype != torch.int64 or lb.dim() != 3 or not 1 <= lb.shape[0] <= 64:
        raise ValueError("limbs: int64 tensor (nlimb, cols, rows), nlimb 1..64")
    if nl is not None and lb.shape[0] != nl:
        raise ValueError("limb count mismatch")
    if ex.dtype != torch.int32 or sg.dtype != torch.uint8 or \
            tuple(ex.shape) != tuple(lb.shape[1:]) or tuple(sg.shape) != tuple(lb.shape[1:]):
        raise ValueError("exp int32 / sign uint8 of shape (cols, rows)")
    return lb.shape[0], lb.shape[1], lb.shape[2]


def check_getrs_limbs_args(LU, ipiv, B):
    """Validate a limb solve's operands; returns (nlimb, n, nrhs)."""
    import torch
    nl, cols, n = check_limb_mat(LU)
    if cols != n:
        raise ValueError("LU must be square")
    _, nrhs, rows = check_limb_mat(B, nl, LU[0].device)
    if rows != n:
        raise ValueError("B must have shape (nlimb, nrhs, n)")
    _check_vec(ipiv, torch.int64, n, "ipiv")
    if ipiv.device != LU[0].device:
        raise ValueError("ipiv must be on the device of LU")
    return nl, n, nrhs


def _check_square(A, name: str):
    _check_mat(A)
    if A.shape[0] != A.shape[1]:
        raise ValueError(f"{name} must be square: shape (n, n, nc)")


def check_getrs_args(LU, ipiv, B):
    """Validate the operands of a solve before they reach the C ABI (a
    mismatched pivot vector or right-hand side would be read out of
    bounds on the device)."""
    import torch
    _check_square(LU, "LU")
    n, nc = LU.shape[0], LU.shape[2]
    _check_mat(B, nc)
    if B.shape[1] != n:
        raise ValueError("B must have shape (nrhs, n, nc)")
    _check_vec(ipiv, torch.int64, n, "ipiv")
    if not (LU.device == B.device == ipiv.device):
        raise ValueError("LU, ipiv and B must be on the same device")


def check_batch_item(A, b, ipiv, info):
    """Validate one system of a batch: A (n, n, nc) float64, b None or
    (1, n, nc) float64, ipiv int64[n], info int32[1], all contiguous CUDA
    tensors on one device."""
    import torch
    _check_square(A, "A")
    n, nc = A.shape[0], A.shape[2]
    if n < 1 or n > 4096:
        raise ValueError("batched systems have 1 <= n <= 4096")
    if b is not None:
        _check_mat(b, nc)
        if tuple(b.shape) != (1, n, nc):
            raise ValueError("b must have shape (1, n, nc)")
    _check_vec(ipiv, torch.int64, n, "ipiv")
    _check_vec(info, torch.int32, 1, "info")
    devs = {A.device, ipiv.device, info.device} | ({b.device} if b is not None else set())
    if len(devs) != 1:
        raise ValueError("the tensors of a system must be on one device")


_LIVE = weakref.WeakSet()


def close_all():
    """Destroy every open handle (registered with atexit, so the library's
    device memory is released while the HIP runtime is still fully up)."""
    for c in list(_LIVE):
        c.close()


atexit.register(close_all)


class Context:
    """A libozii handle bound to one device and (by default) torch's current
    stream on it.  Close it explicitly (or use it as a context manager); an
    open handle is closed at interpreter exit by close_all()."""

    def __init__(self, device: int = 0):
        import torch
        self.device = device
        torch.cuda.set_device(device)
        self._h = _p()
        st = lib().ozII_create(C.byref(self._h), device, self._stream())
        if st != OK:
            raise OziiError(st, "ozII_create failed")
        _LIVE.add(self)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    @staticmethod
    def _stream():
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)

    def _call(self, st: int):
        if st != OK:
            msg = lib().ozII_last_error(self._h).decode()
            raise OziiError(st, f"{lib().ozII_status_string(st).decode()}: {msg}")

    def _bind(self):
        lib().ozII_set_stream(self._h, self._stream())

    def close(self):
        if self._h:
            lib().ozII_destroy(self._h)
            self._h = _p()
        _LIVE.discard(self)

    def __del__(self, _finalizing=sys.is_finalizing):
        # no HIP calls while the interpreter shuts down: the runtime (and a
        # profiler attached to it) may already be gone; close_all() has run
        # by then for every handle that was still open.  The check is bound
        # at definition time: module globals such as sys may already be None.
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def reserve(self, nc: int, M: int, N: int, K: int, n: int = 0, opts: Optional[Opts] = None):
        self._call(lib().ozII_reserve(self._h, nc, M, N, K, n, C.byref(opts) if opts else None))

    def gemm(self, mode: int, A, B, Cm, opts: Optional[Opts] = None):
        """mode 0: C = A B; mode 1: C = C - A B.  A: (K, M, nc), B: (N, K, nc),
        C: (N, M, nc)."""
        nc = A.shape[2]
        for t in (A, B, Cm):
            _check_mat(t, nc)
        K, M = A.shape[0], A.shape[1]
        N = B.shape[0]
        if B.shape[1] != K or Cm.shape[0] != N or Cm.shape[1] != M:
            raise ValueError("shape mismatch")
        self._bind()
        self._call(lib().ozII_gemm(self._h, mode, nc, M, N, K, _ptr(A), max(M, 1), _ptr(B),
                                   max(K, 1), _ptr(Cm), max(M, 1), C.byref(opts) if opts else None))
        return Cm

    @staticmethod
    def _limb_shapes(A, B, Cm):
        import torch
        nl = A[0].shape[0]
        for X in (A, B, Cm):
            lb, ex, sg = X
            if not (lb.is_cuda and lb.dtype == torch.int64 and lb.is_contiguous() and lb.dim() == 3
                    and lb.shape[0] == nl):
                raise ValueError("limbs: contiguous int64 CUDA tensor (nlimb, cols, rows)")
            if ex.dtype != torch.int32 or sg.dtype != torch.uint8 or \
                    tuple(ex.shape) != tuple(lb.shape[1:]) or tuple(sg.shape) != tuple(lb.shape[1:]) \
                    or not (ex.is_contiguous() and sg.is_contiguous()):
                raise ValueError("exp int32 / sign uint8 of shape (cols, rows)")
        K, M = A[0].shape[1], A[0].shape[2]
        N = B[0].shape[1]
        if B[0].shape[2] != K or Cm[0].shape[1] != N or Cm[0].shape[2] != M:
            raise ValueError("shape mismatch")
        return nl, M, N, K

    @staticmethod
    def _limb_desc(X):
        lb, ex, sg = X
        rows, cols = lb.shape[2], lb.shape[1]
        return Limbs(_ptr(lb), _ptr(ex), _ptr(sg), max(rows, 1), max(rows, 1) * cols)

    def gemm_limbs(self, mode: int, A, B, Cm, opts: Optional[Opts] = None):
        """Limb-format product, mode 0: C = RN_p(A B); mode 1: C = RN_p(C - RN_p(A B)).
        Each matrix is a tuple (limb, exp, sign) of contiguous CUDA tensors of
        shapes (nlimb, cols, rows) int64 (the uint64 limbs), (cols, rows) int32
        and (cols, rows) uint8."""
        nl, M, N, K = self._limb_shapes(A, B, Cm)
        dA, dB, dC = (self._limb_desc(X) for X in (A, B, Cm))
        self._bind()
        self._call(lib().ozII_gemm_limbs(self._h, mode, nl, M, N, K, C.byref(dA), C.byref(dB),
                                         C.byref(dC), C.byref(opts) if opts else None))
        return Cm

    def gemm_noalloc(self, mode: int, A, B, Cm, opts: Optional[Opts] = None):
        """gemm() through ozII_gemm_noalloc: plan tables and workspace in the
        library's static per-GPU scratch, no device allocation."""
        nc = A.shape[2]
        for t in (A, B, Cm):
            _check_mat(t, nc)
        K, M = A.shape[0], A.shape[1]
        N = B.shape[0]
        if B.shape[1] != K or Cm.shape[0] != N or Cm.shape[1] != M:
            raise ValueError("shape mismatch")
        self._bind()
        self._call(lib().ozII_gemm_noalloc(self._h, mode, nc, M, N, K, _ptr(A), max(M, 1),
                                           _ptr(B), max(K, 1), _ptr(Cm), max(M, 1),
                                           C.byref(opts) if opts else None))
        return Cm

    def gemm_limbs_stages(self, mode: int, A, B, Cm, opts: Optional[Opts] = None,
                          nlimb_out: int = 6):
        """gemm_limbs with the (S5) group sums returned: int64 CUDA tensor of
        shape (ng, N, M, nlimb_out), two's-complement 64-bit limbs."""
        import torch
        sh = self._limb_shapes(A, B, Cm)
        nl, M, N, K = sh
        S, w, Q, nmod, _ = plan_query(64 * nl, max(K, 1), opts)
        ng = 2 * S - 1 - max(0, S - 1 - (opts.extra_groups if opts is not None else 0))
        sbar = torch.zeros(ng * N * M * nlimb_out, dtype=torch.int64, device=A[0].device)
        dA, dB, dC = (self._limb_desc(X) for X in (A, B, Cm))
        self._bind()
        self._call(lib().ozII_gemm_limbs_stages(self._h, mode, nl, M, N, K, C.byref(dA),
                                                C.byref(dB), C.byref(dC),
                                                C.byref(opts) if opts else None, _ptr(sbar),
                                                nlimb_out))
        return sbar.view(ng, N, M, nlimb_out)

    def gemm_stages(self, mode: int, A, B, Cm, opts: Optional[Opts] = None, nlimb: int = 6):
        """Product with every intermediate stage returned (parity hooks):
        dict(ea, eb, planesA, planesB, tpl, sbar, dims)."""
        import torch
        nc = A.shape[2]
        K, M = A.shape[0], A.shape[1]
        N = B.shape[0]
        Mp, Np, Kp = _i64(), _i64(), _i64()
        S, nmod, ng = _i32(), _i32(), _i32()
        st = lib().ozII_gemm_stage_dims(nc, M, N, K, C.byref(opts) if opts else None,
                                        C.byref(Mp), C.byref(Np), C.byref(Kp), C.byref(S),
                                        C.byref(nmod), C.byref(ng))
        if st != OK:
            raise OziiError(st, "stage dims")
        dev = A.device
        backend = opts.backend if opts is not None and opts.backend else BE_INT8
        # plane element type and planes per (slice, modulus); t-value type
        pdt, per, tdt = {BE_INT8: (torch.int8, 1, torch.uint8),
                         BE_FP8_B17: (torch.uint8, 2, torch.uint8),
                         BE_F64MOD: (torch.float64, 1, torch.int32),
                         BE_FP16: (torch.int8, 1, torch.uint8)}[backend]
        npl = S.value * nmod.value * per
        ea = torch.empty(M, dtype=torch.int32, device=dev)
        eb = torch.empty(N, dtype=torch.int32, device=dev)
        pa = torch.empty(npl * Mp.value * Kp.value, dtype=pdt, device=dev)
        pb = torch.empty(npl * Np.value * Kp.value, dtype=pdt, device=dev)
        tpl = torch.empty(ng.value * nmod.value * Np.value * Mp.value, dtype=tdt, device=dev)
        sbar = torch.empty(ng.value * N * M * nlimb, dtype=torch.int64, device=dev)
        self._bind()
        self._call(lib().ozII_gemm_stages(self._h, mode, nc, M, N, K, _ptr(A), M, _ptr(B), K,
                                          _ptr(Cm), M, C.byref(opts) if opts else None, _ptr(ea),
                                          _ptr(eb), _ptr(pa), _ptr(pb), _ptr(tpl), _ptr(sbar),
                                          nlimb))
        dims = dict(Mp=Mp.value, Np=Np.value, Kp=Kp.value, S=S.value, nmod=nmod.value,
                    ng=ng.value, M=M, N=N, K=K, backend=backend, nplanes=npl)
        return dict(ea=ea, eb=eb, planesA=pa, planesB=pb, tpl=tpl, sbar=sbar, dims=dims)

    def getrf(self, A, block: int = 256, method: int = METHOD_OZAKI, opts: Optional[Opts] = None):
        """In-place LU of the n x n matrix A (shape (n, n, nc)); returns
        (ipiv int64[n] 0-based LAPACK semantics, info int32[1]) on the device."""
        import torch
        _check_mat(A)
        n, nc = A.shape[0], A.shape[2]
        if A.shape[1] != n:
            raise ValueError("A must be square")
        o = opts if opts is not None else Opts()
        o.block = block
        o.method = method
        ipiv = torch.empty(max(n, 1), dtype=torch.int64, device=A.device)
        info = torch.zeros(1, dtype=torch.int32, device=A.device)
        self._bind()
        self._call(lib().ozII_getrf(self._h, nc, n, _ptr(A), max(n, 1), _ptr(ipiv), _ptr(info),
                                    C.byref(o)))
        return ipiv, info

    def getrs(self, LU, ipiv, B):
        """Solve in place: B (shape (nrhs, n, nc)) <- A^{-1} B."""
        check_getrs_args(LU, ipiv, B)
        n, nc = LU.shape[0], LU.shape[2]
        nrhs = B.shape[0]
        self._bind()
        self._call(lib().ozII_getrs(self._h, nc, n, nrhs, _ptr(LU), max(n, 1), _ptr(ipiv),
                                    _ptr(B), max(n, 1)))
        return B

    def getrf_limbs(self, A, block: int = 256, method: int = METHOD_OZAKI,
                    opts: Optional[Opts] = None, leaf: Optional[int] = None):
        """In-place LU of the n x n limb matrix A = (limb, exp, sign);
        returns (ipiv int64[n] 0-based, info int32[1]) on the device.
        leaf > 0: recursive panel and U12 solve down to leaf columns."""
        import torch
        nl, cols, rows = check_limb_mat(A)
        if cols != rows:
            raise ValueError("A must be square")
        n = rows
        o = opts if opts is not None else Opts()
        o.block = block
        o.method = method
        if leaf is not None:
            o.panel_leaf = leaf
        ipiv = torch.empty(max(n, 1), dtype=torch.int64, device=A[0].device)
        info = torch.zeros(1, dtype=torch.int32, device=A[0].device)
        d = self._limb_desc(A)
        self._bind()
        self._call(lib().ozII_getrf_limbs(self._h, nl, n, C.byref(d), _ptr(ipiv), _ptr(info),
                                          C.byref(o)))
        return ipiv, info

    def getrs_limbs(self, LU, ipiv, B):
        """Solve in place: B = (limb (nl, nrhs, n), exp, sign) <- A^{-1} B."""
        nl, n, nrhs = check_getrs_limbs_args(LU, ipiv, B)
        dL, dB = self._limb_desc(LU), self._limb_desc(B)
        self._bind()
        self._call(lib().ozII_getrs_limbs(self._h, nl, n, nrhs, C.byref(dL), _ptr(ipiv),
                                          C.byref(dB)))
        return B

    def limbs_arith(self, op: str, A, B, Cm):
        """Elementwise C = RN_p(A op B) on limb vectors (shape (nl, 1, count))."""
        nl, c1, cnt = check_limb_mat(A)
        dev = A[0].device
        for X in (B, Cm):
            if check_limb_mat(X, nl, dev)[1:] != (c1, cnt):
                raise ValueError("shape mismatch")
        if c1 != 1:
            raise ValueError("vectors: shape (nlimb, 1, count)")
        code = {"add": 0, "sub": 1, "mul": 2, "div": 3}[op]
        dA, dB, dC = (self._limb_desc(X) for X in (A, B, Cm))
        self._bind()
        self._call(lib().ozII_limbs_arith(self._h, code, nl, cnt, C.byref(dA), C.byref(dB),
                                          C.byref(dC)))
        return Cm

    def batch_prepare(self, systems, opts: Optional[Opts] = None):
        """Upload a batch: systems = [(A, b or None, ipiv, info), ...] of CUDA
        tensors, A (n, n, nc) float64, b (1, n, nc) float64, ipiv int64[n],
        info int32[1]; the tensors must stay alive while the batch is used.
        opts None: unblocked LU with the native update; opts with method
        Ozaki-II: blocked LU (opts.block, default 32, at most 256) with the
        Ozaki-II update on the INT8 back-end."""
        arr = (BatchItem * max(len(systems), 1))()
        for i, (A, b, ipiv, info) in enumerate(systems):
            check_batch_item(A, b, ipiv, info)
            arr[i] = BatchItem(A.shape[2], 0, A.shape[0], _ptr(A), _ptr(b) if b is not None else None,
                               _ptr(ipiv), _ptr(info))
        self._batch_refs = list(systems)
        self._bind()
        if opts is None:
            self._call(lib().ozII_batch_prepare(self._h, len(systems), arr))
        else:
            self._call(lib().ozII_batch_prepare_ex(self._h, len(systems), arr, C.byref(opts)))

    def batch_run(self, times=None):
        """Factor and solve the prepared batch (graph-capturable); times: CUDA
        int64 tensor of 2 * count, start/end stamps of the 100 MHz counter."""
        self._bind()
        self._call(lib().ozII_batch_run(self._h, _ptr(times) if times is not None else None))

    def tune(self, nc: int, n: int, cache_path: Optional[str] = None, retune: bool = False):
        """Autotune (block, back-end or native update) for order n; returns
        (Opts, report dict with the timed candidates)."""
        best = Opts()
        rep = TuneReport()
        self._bind()
        self._call(lib().ozII_tune(self._h, nc, n, cache_path.encode() if cache_path else None,
                                   TUNE_RETUNE if retune else 0, C.byref(best), C.byref(rep)))
        names = {BE_INT8: "int8", BE_FP8_B17: "fp8", BE_F64MOD: "f64", BE_FP16: "fp16"}
        cands = []
        for i in range(rep.ncand):
            o = rep.cand[i]
            cands.append({"block": o.block,
                          "update": "native" if o.method == METHOD_NAIVE else names.get(o.backend, "?"),
                          "lookahead": not (o.flags & F_NO_LOOKAHEAD), "nslice": o.nslice,
                          "gemm_tile": o.gemm_tile, "fused": bool(o.flags & F_FUSED),
                          "ms": rep.ms[i], "model_ms": rep.model_ms[i]})
        return best, {"from_cache": bool(rep.from_cache), "best": rep.best, "candidates": cands}

    def tune_limbs(self, nlimb: int, n: int, cache_path: Optional[str] = None,
                   retune: bool = False):
        """Autotune the limb LU (block, panel leaf, native or Ozaki-II, then
        S and the GEMM tile) for order n; returns (Opts, report dict)."""
        best = Opts()
        rep = TuneReport()
        self._bind()
        self._call(lib().ozII_tune_limbs(self._h, nlimb, n,
                                         cache_path.encode() if cache_path else None,
                                         TUNE_RETUNE if retune else 0, C.byref(best),
                                         C.byref(rep)))
        cands = []
        for i in range(rep.ncand):
            o = rep.cand[i]
            cands.append({"block": o.block,
                          "update": "native" if o.method == METHOD_NAIVE else "int8",
                          "panel_leaf": o.panel_leaf, "nslice": o.nslice,
                          "gemm_tile": o.gemm_tile, "ms": rep.ms[i]})
        return best, {"from_cache": bool(rep.from_cache), "best": rep.best, "candidates": cands}

    def sync_check(self):
        self._call(lib().ozII_sync_check(self._h))

    def set_profiling(self, on: bool):
        self._call(lib().ozII_set_profiling(self._h, 1 if on else 0))

    def profile_read(self):
        """Per-stage {name: (ms, launches, algorithmic bytes, algorithmic ops)}
        since the last read (waits for the stream)."""
        n = len(STAGES)
        ms = (C.c_double * n)()
        la = (C.c_int64 * n)()
        by = (C.c_double * n)()
        op = (C.c_double * n)()
        self._call(lib().ozII_profile_read(self._h, n, ms, la, by, op))
        return {STAGES[i]: (ms[i], la[i], by[i], op[i]) for i in range(n)}


def unfragment(planes, n_planes: int, noutp: int, Kp: int, backend: int = BE_INT8):
    """Residue planes from fragment order to [plane][row][k] (numpy, for
    tests).  A block (ob, kb) is 1 KiB; lane l holds row l%16 and
      INT8 / FP8: bytes for k = 16*(l/16) .. +15 of a 64-k block;
      F64: doubles for k = l/16 and 4 + l/16 of an 8-k block."""
    import numpy as np
    if backend == BE_F64MOD:
        a = np.asarray(planes).reshape(n_planes, noutp // 16, Kp // 8, 4, 16, 2)
        # axes: plane, ob, kb, kgroup, row, slot -> plane, ob, row, kb, slot, kgroup
        return a.transpose(0, 1, 4, 2, 5, 3).reshape(n_planes, noutp, Kp)
    a = np.asarray(planes).reshape(n_planes, noutp // 16, Kp // 64, 4, 16, 16)
    # axes: plane, ob, kb, kgroup, row, byte -> plane, ob, row, kb, kgroup, byte
    return a.transpose(0, 1, 4, 2, 3, 5).reshape(n_planes, noutp, Kp)
