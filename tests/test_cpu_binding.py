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


@pytest.mark.parametrize("be", [2, 3], ids=["fp8", "f64"])
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
