"""Simulated annealing over D-subsets (discover_l0_anneal) against the
oracle's annealing: the same seeded trajectory, so every chain's best
subset and its energy must be identical, bit for bit (both sides compute
every decision with one IEEE rounding per operation in the same order, and
draw the same counter-based SplitMix64 numbers).  The winner's QR refit is
compared with the oracle's least squares to the parity bar, and on small
problems the annealing must find the exhaustive L0 winner (the GPU's own
exhaustive kernel and brute force agree with it)."""
import itertools
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


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


def dev(torch, a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _problem(seed, S, n, D, collinear=False):
    rng = np.random.default_rng(seed)
    F = rng.lognormal(0, 0.4, size=(S, n)) * rng.uniform(0.5, 5, size=(S, 1))
    if collinear:
        F[5] = 2.0 * F[1] - F[3]
        F[9] = F[2].copy()
    rows = rng.choice(S, size=D, replace=False)
    y = 0.7 + sum(rng.uniform(0.5, 2) * rng.choice([-1, 1]) * F[r] / F[r].std() for r in rows)
    y = y + 0.2 * rng.normal(size=n)
    ids = rng.permutation(20 * S)[:S].astype(np.int64)
    return F, ids, y


@pytest.mark.parametrize("S,n,D,Q,K,T0,alpha,seed,init,collinear", [
    (60, 150, 4, 32, 2000, 0.02, 0.999, 1, None, False),
    (200, 301, 5, 96, 3000, 0.01, 0.9995, 2, (0, 7, 11, 50, 199), False),
    (40, 90, 1, 8, 500, 0.05, 0.99, 3, None, False),
    (31, 77, 8, 16, 1500, 0.02, 0.998, 4, None, True),
    (12, 40, 3, 5, 0, 0.01, 1.0, 5, (2, 0, 9), True),
    (9, 30, 9 - 1, 4, 300, 0.0, 1.0, 6, None, False),
    # singular starts: rows 2 and 9 are equal, rows 1, 3, 5 collinear
    (14, 50, 4, 8, 800, 0.02, 0.999, 7, (0, 2, 9, 4), True),
    (14, 50, 6, 8, 800, 0.02, 0.999, 8, (1, 3, 5, 2, 9, 7), True),
    (120, 200, 6, 64, 1500, 0.01, 0.998, 9, None, True),
    (60, 100, 7, 32, 1000, 0.02, 0.998, 10, (2, 9, 1, 3, 5, 11, 40), True)])
def test_anneal_trajectory_equals_oracle(torch, ctx, oracle_mod, S, n, D, Q, K, T0, alpha, seed, init,
                                         collinear):
    O = oracle_mod
    F, ids, y = _problem(seed, S, n, D, collinear)
    w, B, E = O.anneal(F, ids, y, D, Q, K, T0, alpha, seed, init=init)
    rows, rmse, coef, en, crow, cen, res = ctx.anneal(dev(torch, F), dev(torch, ids), dev(torch, y), D,
                                                      chains=Q, steps=K, T0=T0, alpha=alpha, seed=seed,
                                                      init=init, chain_results=True, resid=True)
    assert np.array_equal(crow.cpu().numpy(), B), "chain best subsets"
    assert np.array_equal(cen.cpu().numpy().view(np.int64), E.view(np.int64)), "chain energies (bits)"
    assert rows.cpu().numpy().tolist() == B[w].tolist()
    assert float(en) == E[w] or (math.isinf(E[w]) and math.isinf(float(en)))
    if math.isinf(E[w]):
        return
    # the winner's QR refit against the oracle's least squares
    oc, rss = O.lsq([F[r] for r in B[w]], y)
    o_rmse = math.sqrt(rss / n)
    assert abs(float(rmse) - o_rmse) <= 1e-10 * o_rmse + 1e-13 * np.std(y)
    scale = np.max(np.abs(oc))
    assert np.max(np.abs(coef.cpu().numpy() - oc)) <= 1e-10 * scale
    A = np.column_stack([np.ones(n)] + [F[r] for r in B[w]])
    np.testing.assert_allclose(res.cpu().numpy(), y - A @ oc, rtol=0, atol=1e-9 * np.abs(y).max())


def test_anneal_finds_exhaustive_winner(torch, ctx, oracle_mod):
    """D = 3 on 40 rows: the annealing's winner is the exhaustive L0 winner
    (the GPU's exhaustive kernel and brute force over the oracle's energy)."""
    O = oracle_mod
    F, ids, y = _problem(11, 40, 120, 3)
    Cm, c = O.sa_corr(F, y)
    brute = min(itertools.combinations(range(40), 3), key=lambda a: O.sa_energy(Cm, c, a))
    rows, rmse, coef, en, *_ = ctx.anneal(dev(torch, F), dev(torch, ids), dev(torch, y), 3, chains=256,
                                          steps=4000, T0=0.02, alpha=0.999, seed=9)
    sub, l0_rmse, l0_coef, _, _ = ctx.l0_fit(dev(torch, F), dev(torch, ids), dev(torch, y), 3)
    assert tuple(rows.cpu().numpy()) == tuple(brute) == tuple(sub[0].cpu().numpy())
    assert abs(float(rmse) - float(l0_rmse[0])) <= 1e-12 * float(l0_rmse[0])


def test_anneal_batch_and_init_rules(torch, ctx):
    """Two subspaces in one call equal two calls; a warm start whose rows
    repeat or leave 0..S-1 is replaced by the random start."""
    Fa, ia, ya = _problem(21, 50, 100, 4)
    Fb, ib, yb = _problem(22, 70, 160, 4)
    kw = dict(chains=64, steps=1500, T0=0.02, alpha=0.998, seed=5, chain_results=True)
    both = ctx.anneal_batch([dev(torch, Fa), dev(torch, Fb)], [dev(torch, ia), dev(torch, ib)],
                            [dev(torch, ya), dev(torch, yb)], 4, **kw)
    for (F, i, y), got in zip(((Fa, ia, ya), (Fb, ib, yb)), both):
        one = ctx.anneal(dev(torch, F), dev(torch, i), dev(torch, y), 4, **kw)
        assert np.array_equal(one[4].cpu().numpy(), got[4].cpu().numpy())
        assert np.array_equal(one[5].cpu().numpy(), got[5].cpu().numpy())
    rnd = ctx.anneal(dev(torch, Fa), dev(torch, ia), dev(torch, ya), 4, **kw)
    for bad in ((1, 1, 2, 3), (0, 1, 2, 50), (-1, 1, 2, 3)):
        got = ctx.anneal(dev(torch, Fa), dev(torch, ia), dev(torch, ya), 4, init=bad, **kw)
        assert np.array_equal(got[4].cpu().numpy(), rnd[4].cpu().numpy()), bad


def test_anneal_argument_errors(torch, ctx):
    import paper_2602_06986_amd as D
    F, ids, y = _problem(31, 20, 40, 3)
    args = (dev(torch, F), dev(torch, ids), dev(torch, y))
    for bad in (dict(D=9), dict(D=3, chains=0), dict(D=3, alpha=1.5), dict(D=3, alpha=0.0),
                dict(D=3, T0=-1.0), dict(D=21)):
        Dd = bad.pop("D")
        with pytest.raises(D.DiscoverError):
            ctx.anneal(*args, Dd, **bad)
