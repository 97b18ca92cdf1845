"""Pins of the oracle's simulated annealing over D-subsets (the stochastic
search the paper names for the sparsifying step, Software Description; its
energy is the least-squares fit of Eq. (1)), each chosen so that a plausible
mistake in it fails one:

* the random stream against SplitMix64's published first output for state
  0 (the same value as Java's SplittableRandom(0).nextLong());
* the exp(-x) used in the acceptance test against libm's exp;
* the correlation matrix against numpy.corrcoef, and the energy
  1 - R^2 against an independent least-squares fit (numpy.linalg.lstsq);
  a collinear subset is singular;
* on small problems enough chains find the exhaustive optimum;
* with T0 = 0 every chain only accepts improvements, so its best is its
  start or better; results do not depend on the number of threads, and the
  seed changes the trajectory.
"""
import itertools
import math

import numpy as np
import pytest


def test_splitmix_published_value(oracle_mod):
    O = oracle_mod
    assert O.lib().or_splitmix_at(0, 1) == 0xE220A8397B1DCDAF
    # the stream is x0 + i * gamma through the finaliser: output i of state x0
    # is output 1 of state x0 + (i - 1) * gamma
    g = 0x9E3779B97F4A7C15
    for i in (2, 3, 1000):
        assert O.lib().or_splitmix_at(0, i) == O.lib().or_splitmix_at(((i - 1) * g) & (2 ** 64 - 1), 1)


def test_exp_neg_matches_libm(oracle_mod):
    O = oracle_mod
    f = O.lib().or_sa_exp_neg
    assert f(0.0) == 1.0 and f(-3.0) == 1.0 and f(800.0) == 0.0 and f(math.inf) == 0.0
    for x in np.concatenate([np.linspace(0, 2, 101), np.linspace(2, 60, 117), [0.6931471805599453, 1e-12]]):
        ref = math.exp(-x)
        # range reduction with a rounded ln 2 costs about k ulps for x = k ln 2 + r
        assert abs(f(float(x)) - ref) <= (4 + x) * 2.3e-16 * ref, x


def test_sa_corr_and_energy(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(5)
    S, n = 9, 80
    F = rng.lognormal(0, 0.5, size=(S, n)) * rng.uniform(0.5, 20, size=(S, 1))
    F[4] = 3.0 * F[1] - 2.0 * F[6]                        # collinear with rows 1 and 6
    y = F[0] - 0.5 * F[2] + 0.3 * F[7] + rng.normal(size=n)
    Cm, c = O.sa_corr(F, y)
    ref = np.corrcoef(np.vstack([F, y]))
    np.testing.assert_allclose(Cm, ref[:S, :S], rtol=0, atol=3e-15)
    np.testing.assert_allclose(c, ref[:S, S], rtol=0, atol=3e-15)
    assert np.array_equal(Cm, Cm.T)
    yc = y - y.mean()
    for rows in ((0,), (0, 2), (2, 0, 7), (3, 8, 5, 0)):
        A = np.column_stack([np.ones(n)] + [F[r] for r in rows])
        res = y - A @ np.linalg.lstsq(A, y, rcond=None)[0]
        e = float(res @ res) / float(yc @ yc)
        assert abs(O.sa_energy(Cm, c, rows) - e) <= 1e-12, rows
    assert O.sa_energy(Cm, c, (1, 4, 6)) == math.inf
    assert O.sa_energy(Cm, c, (4, 6, 1)) == math.inf


@pytest.mark.parametrize("S,D", [(12, 3), (14, 4)])
def test_anneal_finds_exhaustive_optimum(oracle_mod, S, D):
    O = oracle_mod
    rng = np.random.default_rng(S + D)
    n = 60
    F = rng.normal(size=(S, n))
    coef = rng.uniform(0.5, 1.5, size=D) * rng.choice([-1, 1], size=D)
    rows = rng.choice(S, size=D, replace=False)
    y = 1.0 + sum(c_ * F[r] for c_, r in zip(coef, rows)) + 0.3 * rng.normal(size=n)
    ids = np.arange(100, 100 + S)
    Cm, c = O.sa_corr(F, y)
    best = min(itertools.combinations(range(S), D), key=lambda a: O.sa_energy(Cm, c, a))
    w, B, E = O.anneal(F, ids, y, D, chains=16, steps=3000, T0=0.05, alpha=0.998, seed=7)
    assert tuple(B[w]) == tuple(sorted(best))
    # (the chain's energy is formed in its own array order)
    assert abs(E[w] - O.sa_energy(Cm, c, tuple(sorted(best)))) <= 1e-13
    assert np.all(np.diff(B, axis=1) > 0)


def test_anneal_greedy_threads_and_seed(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(3)
    S, n, D = 30, 50, 5
    F = rng.normal(size=(S, n))
    y = F[1] + F[5] - F[9] + 0.5 * F[20] + rng.normal(size=n)
    ids = rng.permutation(1000)[:S]
    Cm, c = O.sa_corr(F, y)
    init = np.array([0, 2, 3, 4, 6])
    e0 = O.sa_energy(Cm, c, init)
    w, B, E = O.anneal(F, ids, y, D, chains=4, steps=500, T0=0.0, alpha=1.0, seed=1, init=init)
    assert np.all(E <= e0)
    runs = []
    for threads in (1, 3):
        O.lib().or_set_threads(threads)
        runs.append(O.anneal(F, ids, y, D, chains=6, steps=800, T0=0.02, alpha=0.995, seed=11))
    O.lib().or_set_threads(O.lib().or_max_threads())
    assert runs[0][0] == runs[1][0]
    assert np.array_equal(runs[0][1], runs[1][1]) and np.array_equal(runs[0][2], runs[1][2])
    other = O.anneal(F, ids, y, D, chains=6, steps=800, T0=0.02, alpha=0.995, seed=12)
    assert not (np.array_equal(other[1], runs[0][1]) and np.array_equal(other[2], runs[0][2]))
