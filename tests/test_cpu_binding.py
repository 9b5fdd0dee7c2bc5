"""Host-only checks of the C-ABI library: it loads, exports every symbol the
header declares, and its host-side plan rule agrees with the oracle's."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "ozii.h")


def _lib():
    import paper_2609_29554_amd as Z
    if not os.path.exists(Z.LIB_PATH):
        pytest.skip("libozii.so not built")
    return Z


def test_exports_match_header():
    Z = _lib()
    text = open(HDR).read()
    declared = set(re.findall(r"\b(ozII_[a-z_]+)\s*\(", text))
    assert declared, "no declarations found"
    L = Z.lib()
    for name in declared:
        assert hasattr(L, name), name
    assert declared == set(Z.EXPORTED)


@pytest.mark.parametrize("p,K", [(106, 32), (212, 128), (212, 256), (159, 512), (1024, 1024),
                                 (8192, 512), (212, 256), (4096, 256), (256, 64)])
def test_plan_matches_oracle(p, K):
    Z = _lib()
    import oracle as O
    got = Z.plan_query(p, K)
    pl = O.make_plan(p, K)
    assert got == (pl.S, pl.w, pl.Q, pl.nmod, pl.moduli)


def test_plan_options_and_errors():
    Z = _lib()
    import oracle as O
    got = Z.plan_query(212, 256, Z.make_opts(nslice=3, guard_ex=5))
    pl = O.make_plan(212, 256, nslice=3, guard_ex=5)
    assert got[:4] == (pl.S, pl.w, pl.Q, pl.nmod)
    with pytest.raises(Z.OziiError) as e:
        Z.plan_query(212, 256, Z.make_opts(nslice=1))
    assert e.value.status == Z.ECAPACITY
    with pytest.raises(Z.OziiError) as e:
        Z.plan_query(0, 256)
    assert e.value.status == Z.EINVAL
    Z.plan_query(212, 256, Z.make_opts(gemm_tile=Z.TILE_256x256))  # a valid tile is accepted
    for bad in (-1, 4):
        with pytest.raises(Z.OziiError) as e:
            Z.plan_query(212, 256, Z.make_opts(gemm_tile=bad))
        assert e.value.status == Z.EINVAL
    with pytest.raises(Z.OziiError) as e:
        Z.plan_query(212, 256, Z.make_opts(backend=7))
    assert e.value.status == Z.EINVAL


@pytest.mark.parametrize("be", [2, 3, 4], ids=["fp8", "f64", "fp16"])
@pytest.mark.parametrize("p,K", [(106, 32), (159, 512), (212, 256), (212, 512), (212, 4096)])
def test_backend_plans_match_oracle(be, p, K):
    Z = _lib()
    import oracle as O
    got = Z.plan_query(p, K, Z.make_opts(backend=be))
    pl = O.make_plan(p, K, backend=be)
    assert got == (pl.S, pl.w, pl.Q, pl.nmod, pl.moduli)


def test_status_strings():
    Z = _lib()
    for s in range(8):
        assert Z.lib().ozII_status_string(s)


class _FakeCuda:
    """Stands in for a CUDA tensor: the binding's checks read only shape,
    dtype, device and layout, so they can be exercised without a GPU."""

    def __init__(self, shape, dtype, contiguous=True, device="cuda:0"):
        self.shape = tuple(shape)
        self.dtype = dtype
        self.is_cuda = True
        self.device = device
        self._c = contiguous

    def is_contiguous(self):
        return self._c

    def dim(self):
        return len(self.shape)

    def numel(self):
        n = 1
        for s in self.shape:
            n *= s
        return n


def test_getrs_arguments_are_validated():
    Z = _lib()
    import torch
    f64, i64, i32 = torch.float64, torch.int64, torch.int32
    n, nc = 6, 4
    LU = _FakeCuda((n, n, nc), f64)
    ok = dict(LU=LU, ipiv=_FakeCuda((n,), i64), B=_FakeCuda((2, n, nc), f64))
    Z.check_getrs_args(**ok)
    bad = [
        dict(ok, LU=_FakeCuda((n, n + 1, nc), f64)),            # not square
        dict(ok, ipiv=_FakeCuda((n,), i32)),                    # wrong pivot type
        dict(ok, ipiv=_FakeCuda((n - 1,), i64)),                # too short
        dict(ok, ipiv=_FakeCuda((n,), i64, device="cuda:1")),   # other device
        dict(ok, B=_FakeCuda((2, n + 1, nc), f64)),             # wrong order
        dict(ok, B=_FakeCuda((2, n, 2), f64)),                  # other format
        dict(ok, B=_FakeCuda((2, n, nc), f64, contiguous=False)),
        dict(ok, LU=_FakeCuda((n, n, 5), f64)),                 # 5 components
    ]
    for kw in bad:
        with pytest.raises(ValueError):
            Z.check_getrs_args(**kw)


def test_limb_solve_arguments_are_validated():
    Z = _lib()
    import torch
    i64, i32, u8 = torch.int64, torch.int32, torch.uint8
    n, nl = 6, 3

    def mat(cols, rows, nlimb=nl, **kw):
        return (_FakeCuda((nlimb, cols, rows), i64, **kw), _FakeCuda((cols, rows), i32),
                _FakeCuda((cols, rows), u8))

    ok = dict(LU=mat(n, n), ipiv=_FakeCuda((n,), i64), B=mat(2, n))
    assert Z.check_getrs_limbs_args(**ok) == (nl, n, 2)
    bad = [
        dict(ok, LU=mat(n + 1, n)),                              # not square
        dict(ok, LU=mat(n, n, nlimb=65)),                        # too many limbs
        dict(ok, B=mat(2, n, nlimb=2)),                          # other precision
        dict(ok, B=mat(2, n + 1)),                               # wrong order
        dict(ok, B=mat(2, n, contiguous=False)),
        dict(ok, B=(ok["B"][0], _FakeCuda((2, n), i64), ok["B"][2])),   # exp dtype
        dict(ok, B=(ok["B"][0], ok["B"][1], _FakeCuda((2, n - 1), u8))),  # sign shape
        dict(ok, ipiv=_FakeCuda((n,), i32)),
        dict(ok, ipiv=_FakeCuda((n - 1,), i64)),
        dict(ok, ipiv=_FakeCuda((n,), i64, device="cuda:1")),
        dict(ok, LU=ok["LU"][:2]),                               # not a triple
    ]
    for kw in bad:
        with pytest.raises(ValueError):
            Z.check_getrs_limbs_args(**kw)


def test_batch_items_are_validated():
    Z = _lib()
    import torch
    f64, i64, i32 = torch.float64, torch.int64, torch.int32
    n, nc = 5, 2
    ok = dict(A=_FakeCuda((n, n, nc), f64), b=_FakeCuda((1, n, nc), f64),
              ipiv=_FakeCuda((n,), i64), info=_FakeCuda((1,), i32))
    Z.check_batch_item(**ok)
    Z.check_batch_item(**dict(ok, b=None))
    bad = [
        dict(ok, A=_FakeCuda((n, n - 1, nc), f64)),
        dict(ok, b=_FakeCuda((2, n, nc), f64)),
        dict(ok, b=_FakeCuda((1, n, 4), f64)),
        dict(ok, ipiv=_FakeCuda((n,), i32)),
        dict(ok, ipiv=_FakeCuda((n - 2,), i64)),
        dict(ok, info=_FakeCuda((1,), i64)),
        dict(ok, info=_FakeCuda((0,), i32)),
        dict(ok, A=_FakeCuda((5000, 5000, nc), f64)),
        dict(ok, info=_FakeCuda((1,), i32, device="cuda:1")),
    ]
    for kw in bad:
        with pytest.raises(ValueError):
            Z.check_batch_item(**kw)


def test_literal_scaling_plan_matches_oracle():
    # the standalone TD product "at 159-bit scaling": one slice, Q = 160,
    # N_mod the fewest moduli with log2 P > 1 + log2 K + 2*159 = 331
    Z = _lib()
    import math
    import oracle as O
    for p, K, qb, be in ((159, 4096, 159, 1), (106, 512, 106, 1), (159, 4096, 159, 2),
                         (212, 256, 160, 1), (159, 4096, 159, 3)):
        got = Z.plan_query(p, K, Z.make_opts(backend=be, qbits=qb))
        pl = O.make_plan(p, K, backend=be, qbits=qb)
        assert got == (pl.S, pl.w, pl.Q, pl.nmod, pl.moduli)
        assert pl.S == 1 and pl.Q == qb + 1
        need = 1 + math.log2(K) + 2 * qb
        assert math.log2(pl.P) > need
        assert sum(math.log2(m) for m in pl.moduli[:-1]) <= need
    assert O.make_plan(159, 4096, qbits=159).nmod == 48
    with pytest.raises(Z.OziiError):
        Z.plan_query(159, 4096, Z.make_opts(qbits=159, nslice=2))
