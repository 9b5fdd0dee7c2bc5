"""GPU parity of the batched persistent LU + solve against the oracle's
unblocked LU (b = 1, native update) and solve, eagerly and replayed from a
captured hipGraph."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import ctx, note, to_dev, to_host

pytestmark = pytest.mark.gpu


def _systems():
    rng = np.random.default_rng(20260933)
    out = []
    for k, (nc, n, kind) in enumerate([(2, 1, "graded"), (4, 2, "graded"), (3, 17, "lotkin"),
                                       (2, 64, "graded"), (4, 65, "graded"), (2, 100, "lotkin"),
                                       (4, 130, "graded"), (3, 90, "graded"), (4, 40, "singular"),
                                       (2, 257, "graded"), (4, 33, "lotkin"), (2, 5, "graded")]):
        if kind == "lotkin":
            A = W.lotkin(n, nc)
        else:
            A = W.graded(n, nc, float(rng.uniform(20, 60)), rng)
        if kind == "singular":
            A[7, :, :] = 0.0          # a zero column: info = 8
        out.append((nc, A, W.rhs_ones(A)))
    return out


def _expected(systems):
    exp = []
    for nc, A, b in systems:
        LU, ipiv, info, _ = O.getrf(A, 1, O.METHOD_NAIVE)
        X = O.getrs(LU, ipiv, b) if info == 0 else None
        exp.append((LU, ipiv, info, X))
    return exp


def _device(systems):
    import torch
    dev = []
    for nc, A, b in systems:
        n = A.shape[0]
        dev.append((to_dev(A), to_dev(b), torch.zeros(n, dtype=torch.int64, device="cuda"),
                    torch.zeros(1, dtype=torch.int32, device="cuda")))
    return dev


def _check(dev, exp):
    for (dA, db, dip, dinfo), (LU, ipiv, info, X) in zip(dev, exp):
        assert int(to_host(dinfo)[0]) == info
        assert np.array_equal(to_host(dip), ipiv)
        assert np.array_equal(to_host(dA), LU)
        if X is not None:
            assert np.array_equal(to_host(db), X)


def test_batch_matches_oracle():
    import torch
    note("batched LU eager")
    systems = _systems()
    exp = _expected(systems)
    dev = _device(systems)
    ctx().batch_prepare(dev)
    times = torch.zeros(2 * len(dev), dtype=torch.int64, device="cuda")
    ctx().batch_run(times)
    ctx().sync_check()
    _check(dev, exp)
    t = to_host(times).reshape(-1, 2)
    assert np.all(t[:, 1] >= t[:, 0]) and np.all(t[:, 0] > 0)


def test_batch_graph_replays():
    import torch
    note("batched LU in a captured graph")
    systems = _systems()[:8]
    exp = _expected(systems)
    src = _device(systems)        # pristine inputs
    work = _device(systems)       # what the batch factors in place
    ctx().batch_prepare(work)
    times = torch.zeros(2 * len(work), dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            for (a0, b0, _, _), (a, b, _, _) in zip(src, work):
                a.copy_(a0)
                b.copy_(b0)
            ctx().batch_run(times)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        # eager work between replays, then the replay, checked every time
        for (_, _, ip, inf) in work:
            ip.zero_()
            inf.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ctx().sync_check()
        _check(work, exp)
