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
    (2, 40, 30, 1100, 1, 0),    # 39 moduli, 20 CRT digits: the 48-byte-column CRT
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


@pytest.mark.parametrize("case", [(3, 40, 33, 300, 159), (2, 130, 129, 64, 106),
                                  (4, 17, 5, 520, 170)],
                         ids=lambda c: "nc{}-{}x{}x{}-q{}".format(*c))
def test_gemm_literal_scaling_bit_exact(case):
    """The unsliced product at a stated scaling (ozII_opts.qbits): one slice,
    |a_bar| < 2^qbits, N_mod covering 2 K 2^(2 qbits); residues, t-planes,
    group sums and both product modes against the oracle with that plan."""
    import paper_2609_29554_amd as Z
    nc, M, N, K, qb = case
    note(f"gemm literal scaling {case}")
    A, B, C0 = _operands(nc, M, N, K, 300 + M + N + K)
    pl = O.make_plan(53 * nc, K, qbits=qb)
    opts = Z.make_opts(qbits=qb)
    ea, eb = O.exponents(A, True), O.exponents(B, False)
    ra, rb = O.residues(A, True, ea, pl), O.residues(B, False, eb, pl)
    tpl = O.modgemm(ra, rb, pl)
    Cref, sb = O.ozgemm(0, A, B, np.zeros((N, M, nc)), pl, want_sbar=True, nw_out=6)
    C1ref, _ = O.ozgemm(1, A, B, C0, pl)
    dA, dB = to_dev(A), to_dev(B)
    dC = to_dev(np.zeros((N, M, nc)))
    st = ctx().gemm_stages(0, dA, dB, dC, opts, nlimb=6)
    d = st["dims"]
    assert (d["S"], d["nmod"], d["ng"]) == (1, pl.nmod, 1)
    P = pl.nmod
    ga = Z.unfragment(to_host(st["planesA"]), P, d["Mp"], d["Kp"])
    assert np.array_equal(ga[:, :M, :K], ra.reshape(P, M, K))
    gt = to_host(st["tpl"]).reshape(1, pl.nmod, d["Np"], d["Mp"])
    assert np.array_equal(gt[:, :, :N, :M], tpl)
    gs = to_host(st["sbar"]).view(np.uint64).reshape(1, N, M, 6)
    assert np.array_equal(gs, sb)
    assert np.array_equal(to_host(dC), Cref)
    dC1 = to_dev(C0)
    ctx().gemm(1, dA, dB, dC1, opts)
    assert np.array_equal(to_host(dC1), C1ref)


def _e4m3_table():
    """Integer value of every E4M3 byte that encodes an integer in [-16, 16],
    from the OCP format definition (bias 7, 3 fraction bits)."""
    from fractions import Fraction
    tab = {}
    for b in range(256):
        e, f = (b >> 3) & 15, b & 7
        if e == 15 and f == 7:
            continue  # NaN
        v = (Fraction(f, 8) * Fraction(2) ** -6) if e == 0 else (1 + Fraction(f, 8)) * Fraction(2) ** (e - 7)
        v = -v if b & 0x80 else v
        if v.denominator == 1 and abs(v) <= 16:
            tab[b] = int(v)
    return tab


BACKEND_CASES = [c for c in STAGE_CASES if c[1] * c[2] > 1][:6] + [(2, 300, 130, 448, 1, 0)]


@pytest.mark.parametrize("backend", [O.BACKEND_FP8_B17, O.BACKEND_F64MOD, O.BACKEND_FP16],
                         ids=["fp8", "f64", "fp16"])
@pytest.mark.parametrize("case", BACKEND_CASES + [(2, 40, 33, 1500, 2, 0)],
                         ids=lambda c: "nc{}-{}x{}x{}-S{}-E{}".format(*c))
def test_gemm_stages_backends(case, backend):
    """Residue (or digit) planes, t-planes, group sums and products of the
    FP8 base-17, binary64-moduli and FP16 back-ends against the oracle (the
    K = 1500 case spans more than 1024 inner terms per FP16 partial sum, so
    the FP32 partial sums are folded into int32 mid-way)."""
    import paper_2609_29554_amd as Z
    nc, M, N, K, S_f, E = case
    note(f"gemm stages {case} backend {backend}")
    A, B, C0 = _operands(nc, M, N, K, 100 + M + N + K)
    pl = O.make_plan(53 * nc, K, backend=backend, nslice=S_f, extra_groups=E)
    opts = Z.make_opts(backend=backend, nslice=S_f, extra_groups=E)
    ea, eb = O.exponents(A, True), O.exponents(B, False)
    ra, rb = O.residues(A, True, ea, pl), O.residues(B, False, eb, pl)
    tpl = O.modgemm(ra, rb, pl)
    Cref, sb = O.ozgemm(0, A, B, np.zeros((N, M, nc)), pl, want_sbar=True, nw_out=6)
    C1ref, _ = O.ozgemm(1, A, B, C0, pl)

    dA, dB = to_dev(A), to_dev(B)
    dC = to_dev(np.zeros((N, M, nc)))
    st = ctx().gemm_stages(0, dA, dB, dC, opts, nlimb=6)
    d = st["dims"]
    assert (d["S"], d["nmod"], d["ng"]) == (pl.S, pl.nmod, len(pl.groups))
    P = pl.S * pl.nmod
    ga = Z.unfragment(to_host(st["planesA"]), d["nplanes"], d["Mp"], d["Kp"], backend)
    gb = Z.unfragment(to_host(st["planesB"]), d["nplanes"], d["Np"], d["Kp"], backend)
    if backend == O.BACKEND_FP8_B17:
        tab = _e4m3_table()
        dec = np.vectorize(lambda b: tab[int(b)])
        for g_, r_, n_ in ((ga, ra, M), (gb, rb, N)):
            vals = dec(g_.reshape(P, 2, -1, d["Kp"]))
            d0, d1 = O.fp8_digits(r_.reshape(P, n_, K))
            assert np.array_equal(vals[:, 0, :n_, :K], d0)
            assert np.array_equal(vals[:, 1, :n_, :K], d1)
            assert not vals[:, :, n_:, :].any() and not vals[:, :, :, K:].any()
    else:
        assert np.array_equal(ga[:, :M, :K], ra.reshape(P, M, K))
        assert np.array_equal(gb[:, :N, :K], rb.reshape(P, N, K))
        assert not ga[:, M:, :].any() and not ga[:, :, K:].any()
    gt = to_host(st["tpl"]).view(np.uint32 if backend == O.BACKEND_F64MOD else np.uint8)
    gt = gt.reshape(len(pl.groups), pl.nmod, d["Np"], d["Mp"])
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


@pytest.mark.parametrize("backend", [O.BACKEND_FP8_B17, O.BACKEND_F64MOD, O.BACKEND_FP16],
                         ids=["fp8", "f64", "fp16"])
@pytest.mark.parametrize("case", [(4, 100, 32, "lotkin"), (3, 129, 64, "graded"),
                                  (2, 300, 128, "lotkin")],
                         ids=lambda c: "nc{}-n{}-b{}-{}".format(*c))
def test_getrf_getrs_backends(case, backend):
    """The LU with its Schur updates on the FP8 / binary64 back-ends, against
    the oracle LU with that back-end's plan."""
    import paper_2609_29554_amd as Z
    nc, n, b, kind = case
    note(f"getrf/getrs {case} backend={backend}")
    A = _matrix(nc, n, kind, 7 + n)
    plan = O.make_plan(53 * nc, b, backend=backend)
    LU, ipiv, info, _ = O.getrf(A, b, O.METHOD_OZAKI, plan=plan)
    rhs = W.rhs_ones(A)
    X = O.getrs(LU, ipiv, rhs)
    dA = to_dev(A)
    dip, dinfo = ctx().getrf(dA, block=b, opts=Z.make_opts(backend=backend))
    ctx().sync_check()
    assert int(to_host(dinfo)[0]) == info
    assert np.array_equal(to_host(dip), ipiv)
    assert np.array_equal(to_host(dA), LU)
    dX = to_dev(rhs)
    ctx().getrs(dA, dip, dX)
    ctx().sync_check()
    assert np.array_equal(to_host(dX), X)


@pytest.mark.parametrize("method", [O.METHOD_OZAKI, O.METHOD_NAIVE], ids=["ozaki", "naive"])
@pytest.mark.parametrize("case", [(4, 520, 256, "lotkin"), (2, 300, 64, "random"),
                                  (3, 200, 96, "graded")],
                         ids=lambda c: "nc{}-n{}-b{}-{}".format(*c))
def test_getrf_with_and_without_lookahead(case, method):
    """The default schedule updates the next panel's columns first and the
    rest of each Schur update on a side stream while the next panel runs;
    OZII_F_NO_LOOKAHEAD runs each update as one product.  Both equal the
    oracle bit for bit."""
    import paper_2609_29554_amd as Z
    nc, n, b, kind = case
    note(f"getrf lookahead on/off {case} method={method}")
    A = _matrix(nc, n, kind, 11 + n)
    LU, ipiv, info, _ = O.getrf(A, b, method)
    for flags in (0, Z.F_NO_LOOKAHEAD):
        dA = to_dev(A)
        dip, dinfo = ctx().getrf(dA, block=b, method=method, opts=Z.make_opts(flags=flags))
        ctx().sync_check()
        assert int(to_host(dinfo)[0]) == info
        assert np.array_equal(to_host(dip), ipiv)
        assert np.array_equal(to_host(dA), LU)


def test_getrs_several_rhs():
    """Three right-hand sides take the blocked solve (one takes the pipelined
    one); both against the oracle."""
    nc, n, b = 4, 300, 64
    note("getrs nrhs=3")
    A = _matrix(nc, n, "graded", 17)
    LU, ipiv, info, _ = O.getrf(A, b, O.METHOD_NAIVE)
    rng = np.random.default_rng(5)
    R = W.random_expansions(n, 3, nc, rng, exp_sigma=2)          # (3, n, nc)
    X = O.getrs(LU, ipiv, R)
    dLU, dX = to_dev(LU), to_dev(R)
    import torch
    ctx().getrs(dLU, torch.from_numpy(ipiv).cuda(), dX)
    ctx().sync_check()
    assert np.array_equal(to_host(dX), X)
    dX1 = to_dev(np.ascontiguousarray(R[1:2]))
    ctx().getrs(dLU, torch.from_numpy(ipiv).cuda(), dX1)
    ctx().sync_check()
    assert np.array_equal(to_host(dX1), X[1:2])


@pytest.mark.parametrize("nc,n", [(4, 200), (3, 356), (2, 65), (4, 129)],
                         ids=lambda v: str(v))
def test_getrs_blocked_ragged(nc, n):
    """The blocked solve's unit-lower blocks of up to 256 rows run on one,
    two or four chained wavefronts per column; orders whose last block
    leaves a wavefront partly filled (200: 8 rows in the fourth, 356: a
    100-row block, 65: one row in the second, 129: one row in the third,
    none in the fourth) against the oracle."""
    note(f"getrs nrhs=2 nc={nc} n={n}")
    A = _matrix(nc, n, "graded", 23)
    LU, ipiv, info, _ = O.getrf(A, 32, O.METHOD_NAIVE)
    rng = np.random.default_rng(n)
    R = W.random_expansions(n, 2, nc, rng, exp_sigma=2)          # (2, n, nc)
    X = O.getrs(LU, ipiv, R)
    dLU, dX = to_dev(LU), to_dev(R)
    import torch
    ctx().getrs(dLU, torch.from_numpy(ipiv).cuda(), dX)
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


FUSED_CASES = [
    # nc, M, N, K, forced S, extra groups
    (4, 37, 29, 40, 0, 0),
    (2, 70, 33, 130, 0, 1),
    (3, 64, 64, 256, 2, 0),
    (4, 130, 97, 128, 0, 0),
    (2, 1, 1, 1, 0, 0),
    (4, 300, 130, 448, 0, 0),
    (3, 97, 150, 256, 3, 0),
    (4, 64, 33, 64, 2, 1),      # 102 products
    (4, 70, 40, 128, 3, 2),     # 115 products, near the LDS limit
    (4, 50, 45, 128, 4, 3),     # 126 products: the three-kernel path
]
# (group, modulus) products whose t-bytes the fused kernel keeps in LDS
FUSED_MAX_PRODUCTS = 120


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("case", FUSED_CASES, ids=lambda c: "nc{}-{}x{}x{}-S{}-E{}".format(*c))
def test_gemm_fused_bit_exact(case, mode):
    """The fused (S4)-(S6) kernel (t-values of a 32 x 32 tile kept in LDS)
    against the oracle's product, ragged tiles included."""
    import paper_2609_29554_amd as Z
    nc, M, N, K, S_f, E = case
    note(f"fused gemm {case} mode {mode}")
    A, B, C0 = _operands(nc, M, N, K, 300 + M + N + K)
    pl = O.make_plan(53 * nc, K, nslice=S_f, extra_groups=E)
    start = C0 if mode else np.zeros((N, M, nc))
    want, _ = O.ozgemm(mode, A, B, start, pl)
    dA, dB, dC = to_dev(A), to_dev(B), to_dev(start)
    c = ctx()
    c.set_profiling(True)
    try:
        c.gemm(mode, dA, dB, dC, Z.make_opts(nslice=S_f, extra_groups=E, flags=Z.F_FUSED))
        c.sync_check()
        launches = c.profile_read()["fused"][1]
    finally:
        c.set_profiling(False)
    assert np.array_equal(to_host(dC), want)
    # the fused kernel runs whenever the plan's t-bytes fit its LDS tile,
    # the three-kernel path otherwise
    assert (launches > 0) == (len(pl.groups) * pl.nmod <= FUSED_MAX_PRODUCTS)


@pytest.mark.parametrize("lookahead", [True, False])
@pytest.mark.parametrize("case", [(4, 100, 32, "lotkin"), (2, 130, 64, "random"),
                                  (4, 260, 128, "graded")],
                         ids=lambda c: "nc{}-n{}-b{}-{}".format(*c))
def test_getrf_fused_bit_exact(case, lookahead):
    import paper_2609_29554_amd as Z
    nc, n, b, kind = case
    note(f"getrf fused {case} lookahead={lookahead}")
    A = _matrix(nc, n, kind, 11 + n)
    LU, ipiv, info, _ = O.getrf(A, b, O.METHOD_OZAKI)
    flags = Z.F_FUSED | (0 if lookahead else Z.F_NO_LOOKAHEAD)
    dA = to_dev(A)
    dip, dinfo = ctx().getrf(dA, block=b, opts=Z.make_opts(flags=flags))
    ctx().sync_check()
    assert int(to_host(dinfo)[0]) == info
    assert np.array_equal(to_host(dip), ipiv)
    assert np.array_equal(to_host(dA), LU)
