"""Parity at the benchmark sizes.

* QD Lotkin LU, n = 2048, b = 256 and b = 128 (the bench workload; the
  autotuner picks one of the two): pivots, info and a SHA-256 of the whole
  factor array and of the solution must equal the values the oracle wrote
  into tests/golden/ (bit-exact for every element).
* QD Lotkin LU, n = 1024, b = 128, on each Schur-update back-end (INT8,
  FP8 base-17, binary64 moduli) and the native update: the whole factor
  array, pivots, info and solution against the oracle LU with that
  back-end's plan, bit for bit.
* Standalone TD product, m = n = k = 4096 (the MFMA-bound workload): every
  output element depends only on its row of A and column of B (the shared
  exponents are per row / per column), so the oracle evaluates sampled rows
  and columns exactly at full inner dimension.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import ctx, note, to_dev, to_host

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden", "lu_lotkin_qd2048_b{}.json")


def _sha(x):
    return hashlib.sha256(np.ascontiguousarray(x, dtype="<f8").tobytes()).hexdigest()


@pytest.mark.parametrize("block", [256, 128])
def test_lu_lotkin_qd2048_matches_oracle_golden(block):
    g = json.load(open(GOLD.format(block)))
    n, b, nc = g["n"], g["b"], g["nc"]
    note(f"full-size LU Lotkin n={n} b={b} nc={nc}")
    A = W.lotkin(n, nc)
    rhs = W.rhs_ones(A)
    dA = to_dev(A)
    dip, dinfo = ctx().getrf(dA, block=b)
    dx = to_dev(rhs)
    ctx().getrs(dA, dip, dx)
    ctx().sync_check()
    assert int(to_host(dinfo)[0]) == g["info"]
    assert [int(v) for v in to_host(dip)] == g["ipiv"]
    LU = to_host(dA)
    for i, j, v in g["samples"]:
        assert list(LU[j, i]) == v
    assert _sha(LU) == g["lu_sha256"]
    assert _sha(to_host(dx)) == g["x_sha256"]


def td_operands(n, seed=20260932):
    rng = np.random.default_rng(seed)
    A = W.random_expansions(n, n, 3, rng, exp_sigma=4.0)
    B = W.random_expansions(n, n, 3, rng, exp_sigma=4.0)
    return A, B


@pytest.mark.parametrize("mode,plan", [(0, "rule"), (1, "rule"), (0, "literal"), (1, "literal")])
def test_gemm_td4096_sampled(mode, plan):
    """plan "rule": the plan rule of Sec. 3.2 (S = 2, 28 moduli); "literal":
    the product at 159-bit scaling as the TD workload states it (one slice,
    48 moduli covering 2 k 2^318)."""
    import paper_2609_29554_amd as Z
    n = 4096
    qb = 159 if plan == "literal" else 0
    note(f"full-size TD product {n}^3 mode={mode} plan={plan}")
    A, B = td_operands(n)
    C0 = W.random_expansions(n, n, 3, np.random.default_rng(5), exp_sigma=4.0) if mode else \
        np.zeros((n, n, 3))
    dC = to_dev(C0)
    ctx().gemm(mode, to_dev(A), to_dev(B), dC, Z.make_opts(qbits=qb))
    ctx().sync_check()
    C = to_host(dC)
    rng = np.random.default_rng(11)
    rows = np.sort(rng.choice(n, 12, replace=False))
    cols = np.sort(rng.choice(n, 12, replace=False))
    rows[0], cols[-1] = 0, n - 1
    pl = O.make_plan(159, n, qbits=qb)
    Asub = np.ascontiguousarray(A[:, rows, :])      # (K, 12, nc): rows of A
    Bsub = np.ascontiguousarray(B[cols, :, :])      # (12, K, nc): columns of B
    Csub0 = np.ascontiguousarray(C0[cols][:, rows, :])
    want, _ = O.ozgemm(mode, Asub, Bsub, Csub0, pl)
    got = C[cols][:, rows, :]
    assert np.array_equal(got, want)


@pytest.mark.parametrize("backend", ["int8", "fp8", "f64", "fp16", "native"])
def test_lu_lotkin_qd1024_backends_match_oracle(backend):
    import paper_2609_29554_amd as Z
    n, b, nc = 1024, 128, 4
    note(f"full-size LU Lotkin n={n} b={b} nc={nc} update={backend}")
    A = W.lotkin(n, nc)
    rhs = W.rhs_ones(A)
    if backend == "native":
        LU, ipiv, info, _ = O.getrf(A, b, O.METHOD_NAIVE)
        method, opts = Z.METHOD_NAIVE, None
    else:
        be = {"int8": O.BACKEND_INT8, "fp8": O.BACKEND_FP8_B17, "f64": O.BACKEND_F64MOD,
              "fp16": O.BACKEND_FP16}[backend]
        LU, ipiv, info, _ = O.getrf(A, b, O.METHOD_OZAKI, plan=O.make_plan(53 * nc, b, backend=be))
        method, opts = Z.METHOD_OZAKI, Z.make_opts(backend=be)
    X = O.getrs(LU, ipiv, rhs)
    dA = to_dev(A)
    dip, dinfo = ctx().getrf(dA, block=b, method=method, opts=opts)
    dx = to_dev(rhs)
    ctx().getrs(dA, dip, dx)
    ctx().sync_check()
    assert int(to_host(dinfo)[0]) == info
    assert np.array_equal(to_host(dip), ipiv)
    assert np.array_equal(to_host(dA), LU)
    assert np.array_equal(to_host(dx), X)
