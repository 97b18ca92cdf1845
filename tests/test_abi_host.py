"""The C-ABI library loads on a machine without a GPU, exports every symbol
include/discover.h declares, and its host-only space queries (candidate
count and ID decoding) agree with the oracle's enumeration."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def dsc():
    import paper_2602_06986_amd as D
    if not os.path.exists(D.LIB_PATH):
        from paper_2602_06986_amd import build
        build.build()
    D.lib()
    return D


def header_functions():
    src = open(os.path.join(ROOT, "include", "discover.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(discover_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol(dsc):
    names = header_functions()
    assert len(names) >= 10
    L = C.CDLL(dsc.LIB_PATH)
    for nm in names:
        assert hasattr(L, nm), nm
    assert sorted(dsc.SYMBOLS) == names


def test_error_paths_without_gpu(dsc):
    h = C.c_void_p()
    rc = dsc.lib().discover_create(0, C.byref(h))
    if rc == 0:                     # a GPU is visible after all
        dsc.lib().discover_destroy(h)
        pytest.skip("GPU present")
    assert rc in (-1, -3)
    assert dsc.lib().discover_last_error()
    assert dsc.lib().discover_create(0, None) == -1


@pytest.mark.parametrize("p,R,limited", [(6, 1, None), (6, 2, None), (16, 2, None), (3, 3, None),
                                         (24, 3, 0), (5, 2, 0)])
def test_count_matches_oracle(dsc, oracle_mod, p, R, limited):
    O = oracle_mod
    rung_ops = [None] * 4
    rung_pool = [None] * 4
    if limited is not None:
        rung_ops[R] = ("add", "sub", "mul", "div", "rdiv")
        rung_pool[R] = limited
    sp = O.Space(p, R, O.OPS, rung_ops, rung_pool)
    prm = dsc.params(rung=R, rung_ops=rung_ops, rung_pool=rung_pool)
    assert dsc.count(p, prm) == sp.N


def test_decode_matches_oracle(dsc, oracle_mod):
    O = oracle_mod
    for p, R, ops in [(4, 2, O.OPS), (3, 2, ("mul", "rdiv", "log", "sq")), (16, 2, O.OPS)]:
        sp = O.Space(p, R, ops)
        prm = dsc.params(ops=ops, rung=R)
        ids = range(sp.N) if sp.N < 5000 else np.random.default_rng(0).choice(sp.N, 3000, replace=False)
        for cid in ids:
            assert dsc.decode(p, prm, int(cid)) == sp.expr(int(cid))
    with pytest.raises(dsc.DiscoverError):
        dsc.decode(4, dsc.params(rung=1), 10 ** 9)
