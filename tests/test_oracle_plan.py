"""Pins of the oracle plan rule against counts printed in the paper."""
import math
import os

import pytest

from oracle import plan as P

GOLD = os.path.join(os.path.dirname(__file__), "golden", "plan_counts.txt")


def _rows():
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        src, p, K, cnt, nmod = line.split()
        yield src, int(p), int(K), (None if cnt == "-" else int(cnt)), (None if nmod == "-" else int(nmod))


@pytest.mark.parametrize("row", list(_rows()), ids=lambda r: f"{r[0]}-p{r[1]}-K{r[2]}")
def test_printed_counts(row):
    src, p, K, cnt, nmod = row
    backend = P.BACKEND_F64MOD if src.endswith(":f64") else P.BACKEND_INT8
    pl = P.make_plan(p, K, backend=backend)
    if cnt is not None:
        assert pl.gemm_count == cnt
        assert pl.S * (pl.S + 1) // 2 * pl.nmod == cnt  # Eq. (gemmcount)
    if nmod is not None:
        assert pl.nmod == nmod


def test_modulus_set_capacity():
    mods = P.int8_moduli()
    assert len(mods) == 54                      # Sec. 3.2: 54 moduli
    cap = sum(math.log2(m) for m in mods)
    assert abs(cap - 362.8) < 0.05              # Sec. 3.2: about 362.8 bits
    for i, a in enumerate(mods):                # pairwise coprime
        for b in mods[i + 1:]:
            assert math.gcd(a, b) == 1
    assert max(mods) == 256 and min(mods) == 17


def test_constants_and_bounds():
    pl = P.make_plan(212, 256)
    assert (pl.S, pl.w, pl.nmod) == (2, 119, 35)
    assert pl.P == math.prod(pl.moduli)
    for m, Mi, y in zip(pl.moduli, pl.M, pl.y):
        assert (Mi * y) % m == 1
    # uniqueness: |S_g| <= S*K*2^(2w) stays well inside P/2
    assert pl.S * pl.K * 2 ** (2 * pl.w) < pl.P // 2
    # INT32 accumulator bound of Sec. 3.2 (residues in [-128,127])
    assert pl.K * pl.S * 128 * 128 < 2 ** 31
    assert pl.groups == [1, 2]
    assert pl.pairs(1) == [(0, 1), (1, 0)] and pl.pairs(2) == [(1, 1)]
    assert pl.gemm_count == 105


def test_forced_and_rejected():
    with pytest.raises(ValueError):
        P.make_plan(212, 256, nslice=1)       # need exceeds the 362.8-bit capacity
    pl = P.make_plan(212, 256, nslice=3)
    assert pl.S == 3 and pl.w == 79
    pl = P.make_plan(212, 256, extra_groups=1)
    assert pl.groups == [0, 1, 2]


def test_fp8_and_f64_plans():
    p8 = P.make_plan(212, 256, backend=P.BACKEND_FP8_B17)
    p1 = P.make_plan(212, 256)
    assert (p8.S, p8.w, p8.nmod) == (p1.S, p1.w, p1.nmod)   # same capacity as INT8
    # FP8: the three FP32 accumulators (weights 1, 17, 289) stay exact
    assert 2 * p8.K * p8.S * 64 < 2 ** 24
    pf = P.make_plan(212, 256, backend=P.BACKEND_F64MOD)
    for m in pf.moduli:
        assert pf.K * pf.S * m * m < 2 ** 53                   # Eq. (fp64mod), no factor 4
        assert all(m % q for q in range(2, math.isqrt(m) + 1))  # prime
    assert pf.moduli == sorted(pf.moduli, reverse=True) and pf.nmod <= P.F64_MAXMOD
    # "a third or less" of the INT8 GEMM count (Sec. binary64 back-end)
    assert pf.gemm_count * 2.9 <= p1.gemm_count
    # uniqueness of the CRT with the binary64 set, as for INT8
    assert pf.S * pf.K * 2 ** (2 * pf.w) < pf.P // 2


def test_lhint_table_phase():
    # Table "phase" (n = 512, INT8, r = 30): S* = 3/4/5/8/11 for
    # p = 1024..16384, with t = p + slack (slack = 26 at K = 512) and the
    # hint rounded to nearest.
    slack = math.ceil(math.log2(2 * 512)) + 16
    got = [P.lhint(30.0, p + slack, 512, 512) for p in (1024, 2048, 4096, 8192, 16384)]
    assert got == [3, 4, 5, 8, 11]
