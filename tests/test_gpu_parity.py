"""GPU parity of the Ozaki-II product and the LU against the CPU oracle.

Bar: bit-exact for every integer stage (exponents, residue planes, t-planes,
group sums) and, since the HIP path and the oracle follow the same rounding
specification, bit-exact for the rounded outputs and the factors as well.
"""
import functools

import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import ctx, note, to_dev, to_host

pytestmark = pytest.mark.gpu

STAGE_CASES = [
    # nc, M, N, K, nslice, extra_groups
    (4, 37, 29, 40, 0, 0),
    (2, 20, 17, 33, 0, 0),
    (3, 25, 19, 64, 0, 0),
    (4, 16, 16, 130, 3, 1),
    (4, 200, 150, 256, 0, 0),
    (4, 1, 1, 1, 0, 0),
    (2, 130, 3, 7, 0, 0),
    (4, 129, 257, 65, 2, 1),
    (2, 260, 140, 192, 1, 0),   # 3 inner steps per product (odd, below the stage count)
    (2, 300, 130, 448, 1, 0),   # 7 inner steps: loads issued inside the loop
]


def _operands(nc, M, N, K, seed):
    rng = np.random.default_rng(seed)
    A = W.random_expansions(M, K, nc, rng, exp_sigma=3)
    B = W.random_expansions(K, N, nc, rng, exp_sigma=3)
    if M > 3 and K > 2:
        A[2, 3, :] = 0.0
        A[:, min(5, M - 1), :] = 0.0      # a zero row of A
    if N > 4 and K > 1:
        B[min(4, N - 1), :, :] = 0.0      # a zero column of B
    C0 = W.random_expansions(M, N, nc, rng, exp_sigma=3)
    return A, B, C0


@functools.lru_cache(maxsize=16)
def _stage_reference(case):
    """Oracle stages of one case (cached across the tile parametrisation)."""
    nc, M, N, K, S_f, E = case
    A, B, C0 = _operands(nc, M, N, K, 100 + M + N + K)
    pl = O.make_plan(53 * nc, K, nslice=S_f, extra_groups=E)
    ea, eb = O.exponents(A, True), O.exponents(B, False)
    ra, rb = O.residues(A, True, ea, pl), O.residues(B, False, eb, pl)
    tpl = O.modgemm(ra, rb, pl)
    Cref, sb = O.ozgemm(0, A, B, np.zeros((N, M, nc)), pl, want_sbar=True, nw_out=6)
    C1ref, _ = O.ozgemm(1, A, B, C0, pl)
    return A, B, C0, pl, ea, eb, ra, rb, tpl, Cref, sb, C1ref


# every (S4) workgroup tile: 0 = automatic, 1 = 128x128, 2 = 256x128, 3 = 256x256
@pytest.mark.parametrize("tile", [0, 1, 2, 3], ids=["auto", "t128x128", "t256x128", "t256x256"])
@pytest.mark.parametrize("case", STAGE_CASES, ids=lambda c: "nc{}-{}x{}x{}-S{}-E{}".format(*c))
def test_gemm_stages_bit_exact(case, tile):
    import paper_2609_29554_amd as Z
    nc, M, N, K, S_f, E = case
    note(f"gemm stages {case} tile {tile}")
    A, B, C0, pl, ea, eb, ra, rb, tpl, Cref, sb, C1ref = _stage_reference(case)
    opts = Z.make_opts(nslice=S_f, extra_groups=E, gemm_tile=tile)

    dA, dB = to_dev(A), to_dev(B)
    dC = to_dev(np.zeros((N, M, nc)))
    st = ctx().gemm_stages(0, dA, dB, dC, opts, nlimb=6)
    d = st["dims"]
    assert (d["S"], d["nmod"], d["ng"]) == (pl.S, pl.nmod, len(pl.groups))
    assert np.array_equal(to_host(st["ea"]), ea)
    assert np.array_equal(to_host(st["eb"]), eb)
    P = pl.S * pl.nmod
    ga = Z.unfragment(to_host(st["planesA"]), P, d["Mp"], d["Kp"])
    gb = Z.unfragment(to_host(st["planesB"]), P, d["Np"], d["Kp"])
    assert np.array_equal(ga[:, :M, :K], ra.reshape(P, M, K))
    assert np.array_equal(gb[:, :N, :K], rb.reshape(P, N, K))
    assert not ga[:, M:, :].any() and not ga[:, :, K:].any()
    assert not gb[:, N:, :].any() and not gb[:, :, K:].any()
    gt = to_host(st["tpl"]).reshape(len(pl.groups), pl.nmod, d["Np"], d["Mp"])
    assert np.array_equal(gt[:, :, :N, :M], tpl)
    gs = to_host(st["sbar"]).view(np.uint64).reshape(len(pl.groups), N, M, 6)
    assert np.array_equal(gs, sb)
    assert np.array_equal(to_host(dC), Cref)
    dC1 = to_dev(C0)
    ctx().gemm(1, dA, dB, dC1, opts)
    assert np.array_equal(to_host(dC1), C1ref)


LU_CASES = [
    # nc, n, b, kind
    (4, 100, 32, "lotkin"),
    (2, 70, 16, "random"),
    (3, 64, 32, "graded"),
    (4, 129, 64, "graded"),
    (2, 128, 32, "lotkin"),          # the DD Lotkin configuration, n = 128, b = 32
    (4, 520, 256, "lotkin"),         # wide panel, 174 workgroups, ragged last panel
]


def _matrix(nc, n, kind, seed):
    rng = np.random.default_rng(seed)
    if kind == "lotkin":
        return W.lotkin(n, nc)
    if kind == "graded":
        return W.graded(n, nc, 30.0, rng)
    return W.random_expansions(n, n, nc, rng, exp_sigma=2)


@pytest.mark.parametrize("method", [O.METHOD_OZAKI, O.METHOD_NAIVE], ids=["ozaki", "naive"])
@pytest.mark.parametrize("case", LU_CASES, ids=lambda c: "nc{}-n{}-b{}-{}".format(*c))
def test_getrf_getrs_bit_exact(case, method):
    nc, n, b, kind = case
    note(f"getrf/getrs {case} method={method}")
    A = _matrix(nc, n, kind, 7 + n)
    LU, ipiv, info, _ = O.getrf(A, b, method)
    rhs = W.rhs_ones(A)
    X = O.getrs(LU, ipiv, rhs)
    dA = to_dev(A)
    dip, dinfo = ctx().getrf(dA, block=b, method=method)
    ctx().sync_check()
    assert int(to_host(dinfo)[0]) == info
    assert np.array_equal(to_host(dip), ipiv)
    assert np.array_equal(to_host(dA), LU)
    dX = to_dev(rhs)
    ctx().getrs(dA, dip, dX)
    ctx().sync_check()
    assert np.array_equal(to_host(dX), X)


def test_unblocked_equals_blocked_naive_on_gpu():
    nc, n = 4, 80
    note("unblocked vs blocked naive")
    A = W.graded(n, nc, 25.0, np.random.default_rng(3))
    d1, d2 = to_dev(A), to_dev(A)
    p1, _ = ctx().getrf(d1, block=1, method=O.METHOD_NAIVE)
    p2, _ = ctx().getrf(d2, block=32, method=O.METHOD_NAIVE)
    ctx().sync_check()
    assert np.array_equal(to_host(d1), to_host(d2))
    assert np.array_equal(to_host(p1), to_host(p2))


def test_singular_info():
    nc, n = 2, 40
    note("singular matrix")
    A = W.random_expansions(n, n, nc, np.random.default_rng(9))
    A[:, 3, :] = A[:, 17, :]
    A[:, 30, :] = 0.0
    for method in (O.METHOD_OZAKI, O.METHOD_NAIVE):
        LU, ipiv, info, _ = O.getrf(A, 16, method)
        dA = to_dev(A)
        dip, dinfo = ctx().getrf(dA, block=16, method=method)
        ctx().sync_check()
        assert info > 0 and int(to_host(dinfo)[0]) == info
        assert np.array_equal(to_host(dA), LU)
