"""GPU parity of the LU on limb matrices (ozII_getrf_limbs / ozII_getrs_limbs)
and of its p-bit arithmetic (ozII_limbs_arith) against the CPU oracle:
every limb, exponent and sign bit for bit.

* arithmetic: add / sub / mul / div at p = 64 .. 4096 on random operands,
  exponent gaps around p, near-cancellation, ties and carries out of the
  mantissa, against ``oracle/lfloat.c`` (itself pinned to exact rationals);
* the LU with the native update equals the oracle's unblocked LU for every
  panel width (a property of the specification), pivots and info included;
* the LU with the Ozaki-II update equals the oracle's blocked LU
  (``oracle/limb_lu.py``: the same panel, U12 solve and the limb Ozaki-II
  product of ``oracle/limbs.py``);
* the solve equals the oracle's substitution;
* Lotkin n = 512 at p = 3136 (Table lotkin): the solution's correct bits."""
import random

import numpy as np
import pytest

import oracle.lfloat as LF
import oracle.limb_lu as OLU
import workloads as W
from tests.gpu_util import ctx, note, to_dev, to_host

pytestmark = pytest.mark.gpu


def _dev(L):
    limb, ex, sg = L
    return (to_dev(np.ascontiguousarray(limb).view(np.int64)), to_dev(np.ascontiguousarray(ex)),
            to_dev(np.ascontiguousarray(sg)))


def _host(L):
    limb, ex, sg = L
    return (to_host(limb).view(np.uint64), to_host(ex), to_host(sg))


def _same(got, want):
    for g, w, name in zip(got, want, ("limbs", "exp", "sign")):
        assert np.array_equal(g, w), name


# ---------------------------------------------------------------------------
# arithmetic
# ---------------------------------------------------------------------------
def _num(rng, nl):
    p = 64 * nl
    m = rng.randrange(1 << (p - 1), 1 << p)
    r = rng.random()
    if r < 0.15:
        m = (m >> (p - 3)) << (p - 3)            # short mantissa: exact results
    elif r < 0.22:
        m = (1 << p) - 1 - rng.randrange(4)      # all ones: carries out on rounding
    elif r < 0.3:
        m = (1 << (p - 1)) + rng.randrange(4)    # at a power of two
    return m, rng.randrange(-40, 40), rng.randrange(2)


def _arith_cases(op, nl, count, seed):
    rng = random.Random(seed)
    p = 64 * nl
    out = []
    for _ in range(count):
        a, b = _num(rng, nl), _num(rng, nl)
        if op in ("add", "sub"):
            gap = rng.choice([0, 1, 2, 3, 63, 64, 65, 127, 128, 129, p - 2, p - 1, p, p + 1,
                              p + 2, p + 3, 3 * p + 7, rng.randrange(p + 3)])
            b = (b[0], a[1] - gap if rng.random() < 0.5 else a[1] + gap, b[2])
        out.append((a, b))
    for _ in range(count // 5):                   # near-cancellation
        a = _num(rng, nl)
        b = (a[0] + rng.randrange(-3, 4), a[1] + rng.choice([0, 0, 1, -1]),
             a[2] ^ (1 if op == "add" else 0))
        if b[0] >> (p - 1) == 1 and b[0] < 1 << p:
            out.append((a, b))
    for odd in (0, 1):                           # exact ties and their neighbours
        m = (1 << (p - 1)) | (2 * 12345 + odd)
        for sg in (0, 1):
            out += [((m, 0, 0), (1 << (p - 1), -p, sg)), ((m, 0, 0), (1 << (p - 1), -p - 1, sg)),
                    ((1 << (p - 1), 0, 0), (1 << (p - 1), -p - 1, sg)),
                    ((1 << (p - 1), 0, 0), ((1 << p) - 1, -p - 1, sg))]
    z = (0, LF.EXP_ZERO, 0)
    out += [(z, _num(rng, nl))]
    if op != "div":
        out += [(_num(rng, nl), z), (z, z)]
    else:
        for _ in range(8):
            a = _num(rng, nl)
            out += [(a, a), (a, (1 << (p - 1), 3, 0)), (a, (3 << (p - 2), 2, 1))]
    return out


def _pack_vec(vals, nl):
    X = LF.pack([(m, e if m else LF.EXP_ZERO, s if m else 0) for m, e, s in vals], nl)
    return OLU.from_lf(tuple(x[None] for x in X))      # (nl, 1, count)


@pytest.mark.parametrize("nl", [1, 2, 3, 8, 49, 64])
@pytest.mark.parametrize("op", ["add", "sub", "mul", "div"])
def test_limbs_arith_bit_exact(nl, op):
    note(f"limbs_arith nl={nl} op={op}")
    cs = _arith_cases(op, nl, 150 if nl <= 8 else 60, 1000 * nl + len(op))
    A = _pack_vec([a for a, _ in cs], nl)
    B = _pack_vec([b for _, b in cs], nl)
    want = OLU.from_lf(LF.vec(op, OLU.to_lf(A), OLU.to_lf(B)))
    dA, dB = _dev(A), _dev(B)
    dC = _dev(tuple(np.zeros_like(x) for x in A))
    ctx().limbs_arith(op, dA, dB, dC)
    ctx().sync_check()
    _same(_host(dC), want)


# ---------------------------------------------------------------------------
# LU and solve
# ---------------------------------------------------------------------------
def _matrix(nl, n, seed, kind="random"):
    rng = np.random.default_rng(seed)
    A = W.random_limbs(n, n, nl, rng, exp_sigma=3.0, zero_frac=0.05)
    if kind == "singular" and n > 3:
        for x in A:                               # column 2 = 0, row 4 = row 1
            x[..., 2, :] = 0 if x is not A[1] else OLU.EXP32_ZERO
        for x in A:
            x[..., :, 4] = x[..., :, 1]
    return A


def _lu(A, b, method, leaf=0):
    import paper_2609_29554_amd as Z
    dA = _dev(A)
    ipiv, info = ctx().getrf_limbs(dA, block=b,
                                   method=Z.METHOD_NAIVE if method == "native" else Z.METHOD_OZAKI,
                                   leaf=leaf)
    ctx().sync_check()
    return _host(dA), to_host(ipiv), int(to_host(info)[0])


@pytest.mark.parametrize("nl,n,b", [(1, 1, 8), (1, 5, 2), (2, 37, 8), (1, 70, 16), (4, 40, 256),
                                    (2, 33, 1), (64, 9, 4)])
def test_getrf_limbs_native_equals_unblocked(nl, n, b):
    note(f"getrf_limbs native nl={nl} n={n} b={b}")
    A = _matrix(nl, n, 10 * n + nl)
    got, ipiv, info = _lu(A, b, "native")
    F, ip, inf = LF.getrf(OLU.to_lf(A))
    _same(got, OLU.from_lf(F))
    assert np.array_equal(ipiv[:n], ip) and info == inf


@pytest.mark.parametrize("nl,n,b", [(1, 12, 4), (2, 40, 8), (1, 70, 16), (4, 33, 8), (2, 48, 16),
                                    (8, 20, 8)])
def test_getrf_limbs_ozaki_bit_exact(nl, n, b):
    note(f"getrf_limbs ozaki nl={nl} n={n} b={b}")
    A = _matrix(nl, n, 7 * n + nl)
    got, ipiv, info = _lu(A, b, "ozaki")
    want, ip, inf = OLU.getrf(A, b, "ozaki")
    _same(got, want)
    assert np.array_equal(ipiv[:n], ip) and info == inf


@pytest.mark.parametrize("nl,n,b,leaf", [(1, 40, 16, 4), (2, 70, 32, 8), (1, 33, 33, 5),
                                         (4, 48, 24, 6)])
def test_getrf_limbs_recursive_panel_bit_exact(nl, n, b, leaf):
    """The recursive panel and U12 solve with Ozaki-II inner updates against
    the oracle's same recursion; with multiply-subtract updates the result
    is the unblocked LU."""
    note(f"getrf_limbs recursive nl={nl} n={n} b={b} leaf={leaf}")
    A = _matrix(nl, n, 19 * n + leaf)
    got, ipiv, info = _lu(A, b, "ozaki", leaf)
    want, ip, inf = OLU.getrf(A, b, "ozaki", leaf=leaf)
    _same(got, want)
    assert np.array_equal(ipiv[:n], ip) and info == inf
    got, ipiv, info = _lu(A, b, "native", leaf)
    F, ip, inf = LF.getrf(OLU.to_lf(A))
    _same(got, OLU.from_lf(F))
    assert np.array_equal(ipiv[:n], ip) and info == inf


@pytest.mark.parametrize("method", ["native", "ozaki"])
def test_getrf_limbs_singular(method):
    nl, n, b = 2, 20, 8
    note(f"getrf_limbs singular {method}")
    A = _matrix(nl, n, 5, "singular")
    got, ipiv, info = _lu(A, b, method)
    want, ip, inf = OLU.getrf(A, b, method)
    assert inf > 0
    _same(got, want)
    assert np.array_equal(ipiv[:n], ip) and info == inf


@pytest.mark.parametrize("nl,n,b,nrhs", [(1, 37, 8, 1), (2, 40, 16, 3), (3, 17, 4, 2)])
def test_getrs_limbs_bit_exact(nl, n, b, nrhs):
    note(f"getrs_limbs nl={nl} n={n} nrhs={nrhs}")
    A = _matrix(nl, n, 3 * n + nl)
    F, ip, _ = OLU.getrf(A, b, "ozaki")
    rng = np.random.default_rng(n)
    B = W.random_limbs(n, nrhs, nl, rng, exp_sigma=2.0, zero_frac=0.05)
    want = OLU.getrs(F, ip, B)
    import torch
    dF, dB = _dev(F), _dev(B)
    dip = torch.from_numpy(ip.copy()).cuda()
    ctx().getrs_limbs(dF, dip, dB)
    ctx().sync_check()
    _same(_host(dB), want)


@pytest.mark.parametrize("leaf", [0, 32])
def test_lotkin_limb_lu_p3136_correct_bits(leaf):
    """Table lotkin, n = 512 at p = 3136, b = 256: 545 correct bits on the
    GPU (546 on the CPU); the bound p - log2 cond is 525."""
    n, nl, b = 512, 49, 256
    note(f"lotkin limb LU n=512 p=3136 leaf={leaf}")
    A = OLU.from_lf(LF.lotkin(n, nl))
    rhs = OLU.from_lf(LF.rhs_times_ones(LF.lotkin(n, nl)))
    import paper_2609_29554_amd as Z
    dA, dX = _dev(A), _dev(rhs)
    ipiv, info = ctx().getrf_limbs(dA, block=b, method=Z.METHOD_OZAKI, leaf=leaf)
    ctx().getrs_limbs(dA, ipiv, dX)
    ctx().sync_check()
    assert int(to_host(info)[0]) == 0
    bits = LF.correct_bits(OLU.to_lf(_host(dX)))
    assert 542 <= bits <= 549, bits


def test_tune_limbs_report_and_choice(tmp_path):
    """The limb autotuner times its candidates, returns the fastest, caches
    it, and its choice factors a matrix exactly like an explicit call."""
    import paper_2609_29554_amd as Z
    nl, n = 2, 160
    note(f"tune_limbs nl={nl} n={n}")
    cache = str(tmp_path / "tune.json")
    best, rep = ctx().tune_limbs(nl, n, cache)
    assert not rep["from_cache"] and len(rep["candidates"]) >= 4
    ms = [c["ms"] for c in rep["candidates"]]
    assert all(m > 0 for m in ms) and ms[rep["best"]] == min(ms)
    chosen = rep["candidates"][rep["best"]]
    assert best.block == chosen["block"] and best.panel_leaf == chosen["panel_leaf"]
    assert {c["update"] for c in rep["candidates"]} == {"int8", "native"}
    assert any(c["panel_leaf"] > 0 for c in rep["candidates"])
    best2, rep2 = ctx().tune_limbs(nl, n, cache)
    assert rep2["from_cache"] and (best2.block, best2.panel_leaf, best2.method, best2.gemm_tile,
                                   best2.nslice) == (best.block, best.panel_leaf, best.method,
                                                     best.gemm_tile, best.nslice)
    A = _matrix(nl, 70, 3)
    dA = _dev(A)
    o = Z.make_opts(block=best.block, method=best.method, panel_leaf=best.panel_leaf,
                    gemm_tile=best.gemm_tile)
    ipiv, info = ctx().getrf_limbs(dA, block=best.block, method=best.method, opts=o)
    ctx().sync_check()
    meth = "native" if best.method == Z.METHOD_NAIVE else "ozaki"
    want, ip, _ = OLU.getrf(A, best.block, meth, leaf=best.panel_leaf, nslice=best.nslice)
    _same(_host(dA), want)
