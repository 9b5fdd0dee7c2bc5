"""GPU tests of the autotuner: every candidate timed, the fastest chosen,
the choice cached, and the LU with the tuned configuration still bit-exact
with the oracle."""
import json

import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import ctx, note, to_dev, to_host

pytestmark = pytest.mark.gpu


def test_tune_times_candidates_and_caches(tmp_path):
    import paper_2609_29554_amd as Z
    nc, n = 3, 300
    note(f"tune nc={nc} n={n}")
    cache = str(tmp_path / "tune.json")
    opts, rep = ctx().tune(nc, n, cache)
    cands = rep["candidates"]
    assert not rep["from_cache"] and len(cands) >= 8
    assert all(c["ms"] > 0 for c in cands)
    best = cands[rep["best"]]
    assert best["ms"] == min(c["ms"] for c in cands)
    assert opts.block == best["block"] and opts.block < n
    data = json.load(open(cache))
    assert len(data) == 1 and data[0]["block"] == opts.block
    opts2, rep2 = ctx().tune(nc, n, cache)
    assert rep2["from_cache"]
    fields = ("block", "backend", "method", "nslice", "gemm_tile", "flags")
    assert all(getattr(opts2, f) == getattr(opts, f) for f in fields)
    # stage 1 covers both schedules; stage 2 refines an Ozaki-II winner
    assert {c["lookahead"] for c in cands} == {True, False}

    # the LU with the tuned configuration against the oracle with that plan
    A = W.graded(n, nc, 20.0, np.random.default_rng(31))
    if opts.method == Z.METHOD_NAIVE:
        LU, ipiv, info, _ = O.getrf(A, opts.block, O.METHOD_NAIVE)
    else:
        plan = O.make_plan(53 * nc, opts.block, backend=opts.backend, nslice=opts.nslice)
        LU, ipiv, info, _ = O.getrf(A, opts.block, O.METHOD_OZAKI, plan=plan)
    dA = to_dev(A)
    dip, dinfo = ctx().getrf(dA, block=opts.block, method=opts.method, opts=opts2)
    ctx().sync_check()
    assert int(to_host(dinfo)[0]) == info
    assert np.array_equal(to_host(dip), ipiv)
    assert np.array_equal(to_host(dA), LU)


def test_tune_rejects_bad_arguments():
    import paper_2609_29554_amd as Z
    with pytest.raises(Z.OziiError):
        ctx().tune(5, 100)
    with pytest.raises(Z.OziiError):
        ctx().tune(2, 1)
