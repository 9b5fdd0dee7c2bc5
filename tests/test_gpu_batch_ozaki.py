"""GPU parity of the batched persistent LU with the in-workgroup Ozaki-II
Schur update (ozII_batch_prepare_ex, method Ozaki-II) against the oracle's
blocked LU with the Ozaki-II update at the same block (INT8 plan at K = b)
and its solve: factors, pivots, info and solutions bit for bit, for DD / TD
/ QD systems whose trailing blocks span several 64-wide tiles with ragged
edges, systems no larger than one block, a singular system, b = 16 / 32 /
64 / 96 / 128 (one to two 64-wide inner blocks), eagerly and replayed from a captured hipGraph."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import ctx, note, to_dev, to_host

pytestmark = pytest.mark.gpu


def _systems(seed=20260951):
    rng = np.random.default_rng(seed)
    out = []
    for nc, n, kind in [(4, 130, "graded"), (2, 1, "graded"), (3, 17, "lotkin"),
                        (2, 64, "graded"), (4, 65, "graded"), (2, 100, "lotkin"),
                        (3, 90, "graded"), (4, 40, "singular"), (2, 257, "graded"),
                        (4, 33, "lotkin"), (4, 200, "graded"), (2, 5, "graded")]:
        A = W.lotkin(n, nc) if kind == "lotkin" else W.graded(n, nc, float(rng.uniform(20, 60)), rng)
        if kind == "singular":
            A[7, :, :] = 0.0          # a zero column: info = 8
        out.append((nc, A, W.rhs_ones(A)))
    return out


def _expected(systems, b):
    exp = []
    for nc, A, rhs in systems:
        LU, ipiv, info, _ = O.getrf(A, b, O.METHOD_OZAKI, O.make_plan(53 * nc, b))
        X = O.getrs(LU, ipiv, rhs) if info == 0 else None
        exp.append((LU, ipiv, info, X))
    return exp


def _device(systems):
    import torch
    return [(to_dev(A), to_dev(rhs), torch.zeros(A.shape[0], dtype=torch.int64, device="cuda"),
             torch.zeros(1, dtype=torch.int32, device="cuda")) for _, A, rhs in systems]


def _check(dev, exp, systems):
    for (dA, db, dip, dinfo), (LU, ipiv, info, X), (nc, A, _) in zip(dev, exp, systems):
        tag = f"nc={nc} n={A.shape[0]}"
        assert int(to_host(dinfo)[0]) == info, tag
        assert np.array_equal(to_host(dip), ipiv), tag
        assert np.array_equal(to_host(dA), LU), tag
        if X is not None:
            assert np.array_equal(to_host(db), X), tag


@pytest.mark.parametrize("b", [32, 16, 64, 128, 96])
def test_batch_ozaki_matches_oracle(b):
    import torch
    import paper_2609_29554_amd as Z
    note(f"batched Ozaki-II LU b={b}")
    systems = _systems()
    exp = _expected(systems, b)
    dev = _device(systems)
    ctx().batch_prepare(dev, Z.make_opts(block=b, method=Z.METHOD_OZAKI))
    times = torch.zeros(2 * len(dev), dtype=torch.int64, device="cuda")
    ctx().batch_run(times)
    ctx().sync_check()
    _check(dev, exp, systems)
    t = to_host(times).reshape(-1, 2)
    assert np.all(t[:, 1] >= t[:, 0]) and np.all(t[:, 0] > 0)


def test_batch_ozaki_graph_replays():
    import torch
    import paper_2609_29554_amd as Z
    note("batched Ozaki-II LU in a captured graph")
    systems = _systems(20260952)[:6]
    exp = _expected(systems, 32)
    src = _device(systems)
    work = _device(systems)
    ctx().batch_prepare(work, Z.make_opts(block=32, method=Z.METHOD_OZAKI))
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            for (a0, b0, _, _), (a, b, _, _) in zip(src, work):
                a.copy_(a0)
                b.copy_(b0)
            ctx().batch_run()
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        for (_, _, ip, inf) in work:
            ip.zero_()
            inf.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ctx().sync_check()
        _check(work, exp, systems)


def test_batch_ozaki_rejects_unsupported():
    import torch
    import paper_2609_29554_amd as Z
    note("batched Ozaki-II LU errors")
    systems = _systems()[:2]
    dev = _device(systems)
    with pytest.raises(Z.OziiError):
        ctx().batch_prepare(dev, Z.make_opts(block=320, method=Z.METHOD_OZAKI))
    with pytest.raises(Z.OziiError):
        ctx().batch_prepare(dev, Z.make_opts(block=32, method=Z.METHOD_OZAKI, backend=Z.BE_FP8_B17))
    # the native path still works after a rejected call
    ctx().batch_prepare(dev)
    ctx().batch_run()
    ctx().sync_check()


def test_batch_ozaki_full_workload_sampled():
    """The benchmarked workload itself -- 256 systems, n uniform in [64, 512],
    half DD half QD, b = 64, one persistent launch -- with the largest QD and
    DD systems and four others checked against the oracle bit for bit."""
    import torch
    import paper_2609_29554_amd as Z
    note("batched Ozaki-II LU, 256 systems, sampled against the oracle")
    rng = np.random.default_rng(20260934)
    systems = W.batch_systems(256, rng)
    dev = _device(systems)
    ctx().batch_prepare(dev, Z.make_opts(block=64, method=Z.METHOD_OZAKI))
    ctx().batch_run()
    ctx().sync_check()
    ns = [(i, nc, A.shape[0]) for i, (nc, A, _) in enumerate(systems)]
    pick = {max((x for x in ns if x[1] == 4), key=lambda x: x[2])[0],
            max((x for x in ns if x[1] == 2), key=lambda x: x[2])[0]}
    pick |= set(np.random.default_rng(5).choice(len(systems), 4, replace=False).tolist())
    sub = [systems[i] for i in sorted(pick)]
    _check([dev[i] for i in sorted(pick)], _expected(sub, 64), sub)
    assert all(int(to_host(d[3])[0]) == 0 for d in dev)
