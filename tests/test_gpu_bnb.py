"""GPU parity of the branch-and-bound exact L0 (discover_l0_bnb) with the
plain definition of Eq. (1): the oracle's direct Householder QR of every
D-subset (oracle.l0, mode "direct"), and, for D <= 3 at sizes the oracle
would take long on, the GPU's exhaustive L0.  Same bar as the exhaustive
L0 tests (tests/checks.py): identical subsets (by candidate ID), RMSE and
coefficients within 1e-10.
"""
import json
import math
import os

import numpy as np
import pytest

import synth
from tests.checks import check_model

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


@pytest.fixture(scope="module")
def ctx(torch):
    import paper_2602_06986_amd as D
    c = D.Context(0)
    yield c
    c.close()


def dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def _families(rng, S, n):
    """Rows in correlated families (a base row, scaled noisy copies), as
    generated features are."""
    base = rng.lognormal(0, 0.5, size=(max(2, S // 3), n))
    F = np.empty((S, n))
    for i in range(S):
        b = base[i % len(base)]
        F[i] = b * rng.uniform(0.5, 2.0) + rng.normal(scale=rng.uniform(0.05, 0.6), size=n) + rng.normal()
    return F


def _compare(ref, sub, rmse, coef, res, ids, y, what):
    for q, mo in enumerate(ref):
        s = sub[q].cpu().numpy()
        check_model([int(ids[i]) for i in s], float(rmse[q]), coef[q].cpu().numpy(), mo, y, "%s q%d" % (what, q))
        if res is not None:
            np.testing.assert_allclose(res[q].cpu().numpy(), mo["resid"], rtol=0,
                                       atol=1e-10 * np.max(np.abs(mo["resid"])))


# (seed, S, n, D, m, noise): every D; weak signals (large noise) make the
# search visit more of the tree
CASES = [(0, 12, 50, 1, 1, 0.1), (1, 16, 64, 2, 3, 0.3), (2, 20, 97, 3, 4, 0.5), (3, 24, 130, 4, 2, 0.2),
         (4, 28, 200, 5, 1, 0.05), (5, 22, 150, 6, 2, 0.3), (6, 18, 120, 7, 1, 0.1), (7, 16, 100, 8, 1, 0.2),
         (8, 26, 61, 4, 5, 2.0), (9, 30, 250, 3, 64, 1.0)]


@pytest.mark.parametrize("seed,S,n,D,m,noise", CASES)
def test_bnb_against_direct_qr(torch, ctx, oracle_mod, seed, S, n, D, m, noise):
    O = oracle_mod
    rng = np.random.default_rng(900 + seed)
    F = _families(rng, S, n)
    rows = rng.choice(S, size=D, replace=False)
    yc = sum(rng.uniform(0.5, 2.0) * rng.choice([-1, 1]) * (F[r] - F[r].mean()) / F[r].std() for r in rows)
    y = 0.5 + yc + noise * rng.normal(size=n)
    ids = rng.permutation(10 ** 7)[:S].astype(np.int64)
    ref = O.l0(F, ids, y, D, m=m, mode="direct")
    sub, rmse, coef, res, st = ctx.l0_bnb(dev(torch, F), dev(torch, ids), dev(torch, y), D, m)
    _compare(ref, sub, rmse, coef, res, ids, y, "seed %d" % seed)
    assert st["n_subsets"] == math.comb(S, D)
    assert st["status"] == 0
    assert st["n_leaves"] <= st["n_subsets"]
    for q in range(len(ref), m):
        assert int(sub[q][0]) == -1


def test_bnb_singular_and_duplicates(torch, ctx, oracle_mod):
    """An exact linear dependency (f5 = f2 + f3), an exact duplicate (f9 =
    f4) and a constant row: no returned model is singular or uses the
    constant row, and the models are the oracle's."""
    rng = np.random.default_rng(950)
    S, n = 24, 80
    F = _families(rng, S, n)
    F[5] = F[2] + F[3]
    F[9] = F[4]
    F[13] = 3.0
    y = F[2] + F[3] - 0.5 * F[5] + 0.4 * F[20] + 0.3 * F[7] + 0.05 * rng.normal(size=n)
    ids = np.arange(S, dtype=np.int64) * 11 + 3
    for D, m in ((3, 6), (4, 4)):
        ref = oracle_mod.l0(F, ids, y, D, m=m, mode="direct")
        sub, rmse, coef, res, st = ctx.l0_bnb(dev(torch, F), dev(torch, ids), dev(torch, y), D, m)
        for q in range(len(ref)):
            s = set(sub[q].cpu().numpy().tolist())
            assert not {2, 3, 5} <= s and not {4, 9} <= s and 13 not in s
        _compare(ref, sub, rmse, coef, res, ids, y, "singular D=%d" % D)


@pytest.mark.parametrize("D,per", [(4, 15), (5, 8)])
def test_bnb_generated_subspace(torch, ctx, oracle_mod, D, per):
    """Rows of a real SISSO subspace (the first `per` features each dimension
    of the units16 reference selected): nearly collinear generated features,
    the hard case for the bound."""
    O = oracle_mod
    w = synth.make("units16")
    with open(os.path.join(GOLDEN, "units16.json")) as f:
        g = json.load(f)
    S_ids = np.array(g["S_ids"], np.int64)
    k = w["k"]
    ids = np.concatenate([S_ids[d * k:d * k + per] for d in range(3)])
    F, _ = O.values(O.Space.of(w), w["X"], w["units"], ids)
    y = w["Y"][0]
    ref = O.l0(F, ids, y, D, m=2, mode="direct")
    sub, rmse, coef, res, st = ctx.l0_bnb(dev(torch, F), dev(torch, ids), dev(torch, y), D, 2)
    _compare(ref, sub, rmse, coef, res, ids, y, "units16 rows D=%d" % D)


def test_bnb_equals_exhaustive_gpu(torch, ctx):
    """D <= 3 on a subspace of 400 rows: the same models as the exhaustive
    GPU L0 (discover_l0_fit)."""
    rng = np.random.default_rng(960)
    S, n = 400, 700
    F = _families(rng, S, n)
    y = 1.0 + F[10] - 0.6 * F[200] + 0.3 * F[377] + 0.2 * rng.normal(size=n)
    ids = rng.permutation(10 ** 8)[:S].astype(np.int64)
    Fd, idd, yd = dev(torch, F), dev(torch, ids), dev(torch, y)
    for D, m in ((1, 5), (2, 8), (3, 8)):
        s1, r1, c1, _, _ = ctx.l0_fit(Fd, idd, yd, D, m)
        s2, r2, c2, _, st = ctx.l0_bnb(Fd, idd, yd, D, m)
        for q in range(m):
            assert sorted(ids[s1[q].cpu().numpy()].tolist()) == sorted(ids[s2[q].cpu().numpy()].tolist()), (D, q)
            assert abs(float(r1[q]) - float(r2[q])) <= 1e-10 * float(r1[q]) + 1e-13 * np.std(y)
        if D == 3:
            assert st["n_leaves"] < st["n_subsets"]


def test_bnb_planted_prunes(torch, ctx, oracle_mod):
    """A strongly planted 5-row model among 120 rows: the search evaluates a
    small fraction of the 1.9e8 subsets and finds the planted rows."""
    rng = np.random.default_rng(970)
    S, n, D = 120, 1000, 5
    F = rng.lognormal(0, 0.5, size=(S, n))
    rows = sorted(rng.choice(S, size=D, replace=False).tolist())
    y = 0.5 + sum((F[r] - F[r].mean()) / F[r].std() for r in rows) + 0.01 * rng.normal(size=n)
    ids = np.arange(S, dtype=np.int64)
    sub, rmse, coef, _, st = ctx.l0_bnb(dev(torch, F), dev(torch, ids), dev(torch, y), D, 1)
    assert sorted(sub[0].cpu().numpy().tolist()) == rows
    print("planted search:", st)
    assert st["n_leaves"] < 1e-2 * st["n_subsets"], st
    ref = oracle_mod.lsq([F[r] for r in rows], y)
    assert abs(float(rmse[0]) - math.sqrt(ref[1] / n)) <= 1e-10 * math.sqrt(ref[1] / n)


def test_bnb_node_limit_and_errors(torch, ctx):
    import paper_2602_06986_amd as Dm
    rng = np.random.default_rng(980)
    S, n = 60, 100
    F = _families(rng, S, n)
    y = rng.normal(size=n)
    ids = np.arange(S, dtype=np.int64)
    Fd, idd, yd = dev(torch, F), dev(torch, ids), dev(torch, y)
    with pytest.raises(Dm.DiscoverError) as e:
        ctx.l0_bnb(Fd, idd, yd, 5, 1, max_nodes=3)
    assert e.value.code == -6
    with pytest.raises(Dm.DiscoverError):
        ctx.l0_bnb(Fd, idd, yd, 9, 1)
    with pytest.raises(Dm.DiscoverError):
        ctx.l0_bnb(Fd, idd, yd, 3, 65)
    with pytest.raises(Dm.DiscoverError):
        ctx.l0_bnb(Fd, idd, dev(torch, np.ones(n)), 2, 1)
    # the context still works afterwards
    sub, _, _, _, st = ctx.l0_bnb(Fd, idd, yd, 2, 1)
    assert st["status"] == 0 and int(sub[0][0]) >= 0
