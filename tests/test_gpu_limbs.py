"""GPU parity of the limb-format Ozaki-II product (ozII_gemm_limbs) against
the limb oracle: every limb, exponent and sign of the result bit for bit, at
p = 64 .. 4096 (S = 1 .. 24 slices), ragged sizes spanning several residue
blocks and GEMM tiles, both modes, zero rows/columns and zero entries."""
import numpy as np
import pytest

import oracle as O
import oracle.limbs as OL
import workloads as W
from tests.gpu_util import ctx, note, to_dev, to_host

pytestmark = pytest.mark.gpu


def _dev(L):
    import torch
    limb, ex, sg = L
    return (to_dev(limb.view(np.int64)), to_dev(ex), to_dev(sg))


def _host(L):
    limb, ex, sg = L
    return (to_host(limb).view(np.uint64), to_host(ex), to_host(sg))


def _case(nl, M, N, K, mode, seed, sigma=4.0, zero_frac=0.05, opts=None, plan_kw=None):
    rng = np.random.default_rng(seed)
    A = W.random_limbs(M, K, nl, rng, exp_sigma=sigma, zero_frac=zero_frac)
    B = W.random_limbs(K, N, nl, rng, exp_sigma=sigma, zero_frac=zero_frac)
    C0 = W.random_limbs(M, N, nl, rng, exp_sigma=sigma, zero_frac=0.1)
    if M > 2:
        A[0][:, :, 2] = 0          # a zero row of A
        A[1][:, 2] = OL.EXP_ZERO
        A[2][:, 2] = 0
    return A, B, C0


@pytest.mark.parametrize("nl,M,N,K,mode,seed", [
    (1, 16, 16, 16, 0, 1),
    (2, 37, 29, 40, 0, 2),
    (2, 130, 3, 70, 1, 3),
    (4, 20, 17, 130, 1, 4),
    (8, 5, 9, 64, 0, 5),
    (64, 9, 7, 20, 0, 6),
    (64, 33, 5, 65, 1, 7),
])
def test_gemm_limbs_bit_exact(nl, M, N, K, mode, seed):
    note(f"gemm_limbs nl={nl} {M}x{N}x{K} mode={mode}")
    A, B, C0 = _case(nl, M, N, K, mode, seed)
    pl = O.make_plan(64 * nl, K)
    want, _ = OL.ozgemm(mode, A, B, C0, pl)
    dA, dB, dC = _dev(A), _dev(B), _dev(C0)
    ctx().gemm_limbs(mode, dA, dB, dC)
    ctx().sync_check()
    got = _host(dC)
    for g, w_, name in zip(got, want, ("limbs", "exp", "sign")):
        assert np.array_equal(g, w_), name


def test_gemm_limbs_extra_group_and_wide_exponents():
    import paper_2609_29554_amd as Z
    nl, M, N, K = 4, 12, 11, 33
    note("gemm_limbs extra group, sigma 40")
    A, B, C0 = _case(nl, M, N, K, 0, 9, sigma=40.0)
    pl = O.make_plan(64 * nl, K, extra_groups=1)
    want, _ = OL.ozgemm(0, A, B, C0, pl)
    dA, dB, dC = _dev(A), _dev(B), _dev(C0)
    ctx().gemm_limbs(0, dA, dB, dC, Z.make_opts(extra_groups=1))
    ctx().sync_check()
    got = _host(dC)
    for g, w_ in zip(got, want):
        assert np.array_equal(g, w_)


def test_gemm_limbs_lotkin_blocks_p4096():
    """The Schur-update shape of the Lotkin LU at p = 4096: L21-like and
    U12-like blocks of the Lotkin matrix, C -= L21 U12."""
    nl, n, b = 64, 24, 8
    note("gemm_limbs lotkin p=4096")
    L = W.lotkin_limbs(n, nl)

    def block(r0, r1, c0, c1):
        return tuple(np.ascontiguousarray(x[..., c0:c1, r0:r1]) for x in L)

    A = block(b, n, 0, b)
    B = block(0, b, b, n)
    C0 = block(b, n, b, n)
    pl = O.make_plan(64 * nl, b)
    want, _ = OL.ozgemm(1, A, B, C0, pl)
    dA, dB, dC = _dev(A), _dev(B), _dev(C0)
    ctx().gemm_limbs(1, dA, dB, dC)
    ctx().sync_check()
    got = _host(dC)
    for g, w_ in zip(got, want):
        assert np.array_equal(g, w_)


def test_gemm_limbs_k_zero_and_errors():
    import paper_2609_29554_amd as Z
    nl = 2
    A, B, C0 = _case(nl, 4, 3, 1, 0, 11)
    A0 = tuple(np.ascontiguousarray(x[..., :0, :]) for x in A)
    B0 = tuple(np.ascontiguousarray(x[..., :, :0]) for x in B)
    dC = _dev(C0)
    ctx().gemm_limbs(0, _dev(A0), _dev(B0), dC)
    ctx().sync_check()
    got = _host(dC)
    assert not got[0].any() and (got[1] == OL.EXP_ZERO).all() and not got[2].any()
    with pytest.raises(Z.OziiError):
        ctx().gemm_limbs(0, _dev(A), _dev(B), _dev(C0), Z.make_opts(backend=Z.BE_FP8_B17))


def test_limb_schur_first_update_p4096_full_size_sampled():
    """The first Schur update of the limb benchmark in its launch
    configuration -- the Lotkin matrix n = 2048 at p = 4096 (64 limbs),
    C = RN_p(C - RN_p(A B)) with M = N = 1792, K = 256, on sub-block
    descriptors of the whole matrix in device memory -- with 16 outputs
    checked against the limb oracle, which needs only their rows of A and
    columns of B (exponents are per row of A and per column of B)."""
    import ctypes
    import torch
    import paper_2609_29554_amd as Z
    n, b, nl = 2048, 256, 64
    note("limb Schur update p=4096, 1792 x 1792 x 256, sampled")
    limb, ex, sg = W.lotkin_limbs(n, nl)
    dl = torch.from_numpy(limb.view(np.int64)).cuda()
    de = torch.from_numpy(ex).cuda()
    ds = torch.from_numpy(sg).cuda()

    def desc(r0, c0):
        off = r0 + c0 * n
        return Z.Limbs(dl.data_ptr() + 8 * off, de.data_ptr() + 4 * off, ds.data_ptr() + off, n,
                       n * n)

    c = ctx()
    c._bind()
    A, B, Cd = desc(b, 0), desc(0, b), desc(b, b)
    c._call(Z.lib().ozII_gemm_limbs(c._h, 1, nl, n - b, n - b, b, ctypes.byref(A), ctypes.byref(B),
                                    ctypes.byref(Cd), None))
    c.sync_check()
    rows = np.array([0, 1, 900, n - b - 1])
    cols = np.array([0, 2, 1000, n - b - 1])

    def sub(r, cc):
        return tuple(np.ascontiguousarray(x[..., cc, :][..., r]) for x in (limb, ex, sg))

    want, _ = OL.ozgemm(1, sub(b + rows, np.arange(b)), sub(np.arange(b), b + cols),
                        sub(b + rows, b + cols), O.make_plan(64 * nl, b))
    ci, ri = torch.from_numpy(b + cols).cuda(), torch.from_numpy(b + rows).cuda()
    got = (dl[:, ci][:, :, ri].cpu().numpy().view(np.uint64), de[ci][:, ri].cpu().numpy(),
           ds[ci][:, ri].cpu().numpy())
    for g, w_, name in zip(got, want, ("limbs", "exp", "sign")):
        assert np.array_equal(g, w_), name


@pytest.mark.parametrize("nl,M,N,K,E,seed", [
    (4, 20, 17, 40, 0, 21),
    (64, 9, 7, 20, 0, 22),      # p = 4096: 54 moduli, the 48-byte-column CRT
    (64, 33, 5, 65, 1, 23),     # an extra digit group
    (16, 40, 3, 130, 0, 24),
])
def test_gemm_limbs_group_sums_bit_exact(nl, M, N, K, E, seed):
    """(S5) of the limb product: the group sums that the limb consumer's CRT
    routine forms, exported by it, against the oracle's exact digit-group
    sums (below the final rounding, which hides their low bits)."""
    import paper_2609_29554_amd as Z
    note(f"gemm_limbs group sums nl={nl} {M}x{N}x{K} E={E}")
    A, B, C0 = _case(nl, M, N, K, 1, seed)
    pl = O.make_plan(64 * nl, K, extra_groups=E)
    _, _, sums = OL.group_sums(A, B, pl)
    want, _ = OL.ozgemm(1, A, B, C0, pl)
    dA, dB, dC = _dev(A), _dev(B), _dev(C0)
    sb = ctx().gemm_limbs_stages(1, dA, dB, dC, Z.make_opts(extra_groups=E), nlimb_out=6)
    ctx().sync_check()
    got = to_host(sb).view(np.uint64)
    assert got.shape == (len(pl.groups), N, M, 6)
    for g in range(len(pl.groups)):
        for j in range(N):
            for i in range(M):
                assert O.limbs_to_int(got[g, j, i]) == sums[g][j][i], (g, i, j)
    for g_, w_ in zip(_host(dC), want):
        assert np.array_equal(g_, w_)


@pytest.mark.parametrize("nl,M,N,K,mode,seed", [
    (1, 16, 16, 16, 0, 31),
    (2, 37, 29, 40, 1, 32),
    (2, 130, 3, 130, 0, 33),    # two 128-row GEMM tiles, a ragged tail
    (8, 5, 9, 64, 1, 34),
    (64, 9, 7, 20, 0, 35),      # p = 4096: 20 slices, 20 moduli
    (64, 33, 5, 65, 1, 36),
])
def test_gemm_limbs_f64_bit_exact(nl, M, N, K, mode, seed):
    """The limb product on the binary64 moduli (the back-end comparison of
    Sec. 4.1.6): residues as doubles, FP64 MFMA, 32-bit t-values, the CRT of
    the binary64 consumer, then the same group sums and RN_p as on INT8."""
    import paper_2609_29554_amd as Z
    note(f"gemm_limbs binary64 nl={nl} {M}x{N}x{K} mode={mode}")
    A, B, C0 = _case(nl, M, N, K, mode, seed)
    pl = O.make_plan(64 * nl, K, backend=O.BACKEND_F64MOD)
    want, _ = OL.ozgemm(mode, A, B, C0, pl)
    dA, dB, dC = _dev(A), _dev(B), _dev(C0)
    ctx().gemm_limbs(mode, dA, dB, dC, Z.make_opts(backend=Z.BE_F64MOD))
    ctx().sync_check()
    got = _host(dC)
    for g, w_, name in zip(got, want, ("limbs", "exp", "sign")):
        assert np.array_equal(g, w_), name


@pytest.mark.parametrize("nl,M,N,K,mode,backend,seed", [
    (128, 5, 4, 9, 0, "int8", 41),      # p = 8192: 48 slices, 53 moduli
    (128, 6, 3, 9, 1, "f64", 42),
    (256, 4, 5, 9, 1, "int8", 43),      # p = 16384: 95 slices, 54 moduli
    (256, 3, 4, 20, 0, "f64", 44),
])
def test_gemm_limbs_wide_precision_bit_exact(nl, M, N, K, mode, backend, seed):
    """p = 8192 and 16384 (the top of Sec. 4.1.6's sweep) on both back-ends."""
    import paper_2609_29554_amd as Z
    note(f"gemm_limbs nl={nl} {M}x{N}x{K} mode={mode} {backend}")
    A, B, C0 = _case(nl, M, N, K, mode, seed)
    obe, zbe = (O.BACKEND_INT8, Z.BE_INT8) if backend == "int8" else (O.BACKEND_F64MOD, Z.BE_F64MOD)
    pl = O.make_plan(64 * nl, K, backend=obe)
    want, _ = OL.ozgemm(mode, A, B, C0, pl)
    dA, dB, dC = _dev(A), _dev(B), _dev(C0)
    ctx().gemm_limbs(mode, dA, dB, dC, Z.make_opts(backend=zbe))
    ctx().sync_check()
    got = _host(dC)
    for g, w_, name in zip(got, want, ("limbs", "exp", "sign")):
        assert np.array_equal(g, w_), name


@pytest.mark.parametrize("nl,M,N,K,seed", [(4, 20, 17, 40, 51), (2, 130, 3, 70, 52)])
def test_gemm_limbs_f64_group_sums_bit_exact(nl, M, N, K, seed):
    """(S5) on the binary64 moduli: the group sums the limb consumer's CRT
    forms from 32-bit t-values, exported, against the oracle's."""
    import paper_2609_29554_amd as Z
    note(f"gemm_limbs binary64 group sums nl={nl} {M}x{N}x{K}")
    A, B, C0 = _case(nl, M, N, K, 1, seed)
    pl = O.make_plan(64 * nl, K, backend=O.BACKEND_F64MOD)
    assert pl.P.bit_length() < 6 * 64   # the exported limbs hold every sum
    _, _, sums = OL.group_sums(A, B, pl)
    dA, dB, dC = _dev(A), _dev(B), _dev(C0)
    sb = ctx().gemm_limbs_stages(1, dA, dB, dC, Z.make_opts(backend=Z.BE_F64MOD), nlimb_out=6)
    ctx().sync_check()
    got = to_host(sb).view(np.uint64)
    for g in range(len(pl.groups)):
        for j in range(N):
            for i in range(M):
                assert O.limbs_to_int(got[g, j, i]) == sums[g][j][i], (g, i, j)


def test_gemm_limbs_rejects_limb_counts_beyond_the_product_range():
    import paper_2609_29554_amd as Z
    A, B, C0 = _case(257, 2, 2, 2, 0, 61)
    with pytest.raises(Z.OziiError):
        ctx().gemm_limbs(0, _dev(A), _dev(B), _dev(C0))
