"""ozII_gemm_noalloc (the product for callers that cannot allocate device
memory) against ozII_gemm, bit for bit, through the C ABI: two calls in a
row on the static scratch, the second with a smaller input and another
plan, then a product beyond the scratch, which must be refused before
anything runs."""
import ctypes as C

import numpy as np
import pytest

import workloads as W
from gpu_util import ctx, note, to_dev, to_host

pytestmark = pytest.mark.gpu


def _call(fn, c, mode, A, B, Cm, opts):
    import paper_2609_29554_amd as Z
    nc = A.shape[2]
    K, M = A.shape[0], A.shape[1]
    N = B.shape[0]
    c._bind()
    return fn(c._h, mode, nc, M, N, K, A.data_ptr(), max(M, 1), B.data_ptr(), max(K, 1),
              Cm.data_ptr(), max(M, 1), C.byref(opts) if opts is not None else None)


@pytest.mark.parametrize("backend", [1, 2, 3], ids=["int8", "fp8", "f64"])
def test_gemm_noalloc_matches_gemm(backend):
    import paper_2609_29554_amd as Z
    L = Z.lib()
    c = ctx()
    rng = np.random.default_rng(77 + backend)
    cases = [(4, 300, 200, 256, 1), (2, 70, 45, 33, 0)]   # second: smaller, other plan
    for nc, M, N, K, mode in cases:
        note(f"gemm_noalloc backend={backend} nc={nc} {M}x{N}x{K} mode={mode}")
        A = W.random_expansions(M, K, nc, rng, exp_sigma=3)
        B = W.random_expansions(K, N, nc, rng, exp_sigma=3)
        C0 = W.random_expansions(M, N, nc, rng, exp_sigma=3)
        dA, dB = to_dev(A), to_dev(B)
        ref, got = to_dev(C0), to_dev(C0)
        opts = Z.make_opts(backend=backend)
        assert _call(L.ozII_gemm, c, mode, dA, dB, ref, opts) == Z.OK
        assert _call(L.ozII_gemm_noalloc, c, mode, dA, dB, got, opts) == Z.OK
        c.sync_check()
        assert np.array_equal(to_host(got), to_host(ref))


def test_gemm_noalloc_refuses_products_beyond_the_scratch():
    import torch
    import paper_2609_29554_amd as Z
    L = Z.lib()
    c = ctx()
    cap = Z.noalloc_capacity()
    assert cap >= 32 << 20
    n, nc = 2048, 4                      # QD 2048 x 2048 x 2048: far beyond the scratch
    note(f"gemm_noalloc refusal n={n}")
    A = torch.zeros((n, n, nc), dtype=torch.float64, device="cuda")
    Cm = torch.zeros_like(A)
    st = _call(L.ozII_gemm_noalloc, c, 0, A, A, Cm, Z.make_opts())
    assert st == Z.EINVAL
    assert b"static scratch" in L.ozII_last_error(c._h)
