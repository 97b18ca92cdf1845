"""Pins of the oracle's L0 search (Eq. (1), Core Optimization Objective),
OMP (Software Description) and the SISSO loop.

Eq. (1) is least squares under a support-size bound; with an intercept the
per-support solution is ordinary least squares, so numpy.linalg.lstsq and
the closed forms of one- and two-feature regression pin it."""
import itertools
import math

import numpy as np
import pytest


def _design(rng, S=7, n=40, corr=0.3):
    base = rng.normal(size=(3, n))
    F = rng.normal(size=(S, n)) + corr * base[rng.integers(0, 3, size=S)]
    F = F * rng.uniform(0.5, 3.0, size=(S, 1)) + rng.normal(size=(S, 1))
    return F


@pytest.mark.parametrize("D", [1, 2, 3])
def test_direct_rss_matches_lstsq(oracle_mod, D):
    O = oracle_mod
    rng = np.random.default_rng(D)
    F = _design(rng)
    y = rng.normal(size=F.shape[1]) + F[0] - 0.5 * F[3]
    S, n = F.shape
    rss = np.empty(math.comb(S, D))
    O.lib().or_l0_direct(n, S, O._p(np.ascontiguousarray(F)), O._p(y), D, O.PIV_TOL, O._p(rss))
    for t, sub in enumerate(itertools.combinations(range(S), D)):
        A = np.column_stack([np.ones(n)] + [F[i] for i in sub])
        beta, res, *_ = np.linalg.lstsq(A, y, rcond=None)
        ref = float(np.sum((y - A @ beta) ** 2))
        assert abs(rss[t] - ref) <= 1e-12 * float(np.sum((y - y.mean()) ** 2))


def test_closed_forms(oracle_mod):
    """D=1: RSS = yy (1 - r^2).  D=2: R^2 = (r1^2 + r2^2 - 2 r1 r2 c12) / (1 - c12^2)."""
    O = oracle_mod
    rng = np.random.default_rng(10)
    F = _design(rng, S=5, n=60)
    y = rng.normal(size=60) + F[1]
    yy = float(np.sum((y - y.mean()) ** 2))
    for a in range(5):
        r = np.corrcoef(F[a], y)[0, 1]
        _, rss = O.lsq([F[a]], y)
        assert abs(rss - yy * (1 - r * r)) <= 1e-12 * yy
    for a, b in itertools.combinations(range(5), 2):
        r1, r2 = np.corrcoef(F[a], y)[0, 1], np.corrcoef(F[b], y)[0, 1]
        c = np.corrcoef(F[a], F[b])[0, 1]
        R2 = (r1 * r1 + r2 * r2 - 2 * r1 * r2 * c) / (1 - c * c)
        _, rss = O.lsq([F[a], F[b]], y)
        assert abs(rss - yy * (1 - R2)) <= 1e-12 * yy


def test_pivots_are_cholesky_of_correlation(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(11)
    F = _design(rng, S=4, n=50)
    Cm = np.corrcoef(F)
    L = np.linalg.cholesky(Cm)
    np.testing.assert_allclose(O.pivots(list(F)), np.diag(L) ** 2, rtol=1e-12)


def test_singular_subset_rejected(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(12)
    F = _design(rng, S=5, n=30)
    F[4] = 3.0 * F[1] - 2.0                 # affine copy of row 1
    y = rng.normal(size=30)
    models = O.l0(F, np.arange(5), y, 2, m=10, mode="direct")
    assert all(set(mo["positions"]) != {1, 4} for mo in models)
    models_g = O.l0(F, np.arange(5), y, 2, m=10, mode="gram")
    assert all(set(mo["positions"]) != {1, 4} for mo in models_g)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_gram_mode_equals_direct_mode(oracle_mod, seed):
    O = oracle_mod
    rng = np.random.default_rng(seed)
    F = _design(rng, S=12, n=80, corr=0.8)
    y = rng.normal(size=80) + 0.7 * F[2] - F[5] + 0.3 * F[9]
    ids = rng.permutation(1000)[:12]
    for D in (1, 2, 3):
        a = O.l0(F, ids, y, D, m=3, mode="direct")
        b = O.l0(F, ids, y, D, m=3, mode="gram")
        assert [x["ids"] for x in a] == [x["ids"] for x in b]
        for x, z in zip(a, b):
            assert abs(x["rss"] - z["rss"]) <= 1e-12 * x["rss"]


def test_planted_recovery_noise_free(oracle_mod):
    """y = c0 + c1 f_a + c2 f_b exactly: the D=2 winner is {a, b} with RMSE
    near zero and the planted coefficients."""
    O = oracle_mod
    rng = np.random.default_rng(13)
    F = _design(rng, S=15, n=100, corr=0.5)
    y = 0.7 + 1.3 * F[4] - 2.1 * F[11]
    for mode in ("direct", "gram"):
        mo = O.l0(F, np.arange(15), y, 2, mode=mode)[0]
        assert mo["positions"] == (4, 11)
        assert mo["rmse"] <= 1e-12 * np.std(y)
        np.testing.assert_allclose(mo["coef"], [0.7, 1.3, -2.1], rtol=1e-10)


def test_noisy_rmse_expectation(oracle_mod):
    """With Gaussian noise sigma the winning RMSE is close to
    sigma * sqrt((n - D - 1) / n)."""
    O = oracle_mod
    rng = np.random.default_rng(14)
    n, sig = 4000, 0.05
    F = _design(rng, S=6, n=n)
    y = 1.0 + F[0] - F[2] + sig * rng.normal(size=n)
    mo = O.l0(F, np.arange(6), y, 2, mode="direct")[0]
    assert mo["positions"] == (0, 2)
    assert abs(mo["rmse"] / (sig * math.sqrt((n - 3) / n)) - 1) < 0.05


def test_d1_winner_is_sis_top1(oracle_mod):
    import synth
    O = oracle_mod
    w = synth.tiny()
    sp = O.Space.of(w)
    (sel,), _, _ = O.sis(sp, w["X"], None, w["Y"], 20)
    V, _ = O.values(sp, w["X"], None, sel[0])
    mo = O.l0(V, sel[0], w["Y"][0], 1)[0]
    assert mo["ids"] == (sel[0][0],)


# ------------------------------------------------------------------ OMP
def test_omp_first_pick_is_top_correlation(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(15)
    F = _design(rng, S=20, n=70)
    y = rng.normal(size=70) + F[7]
    act, coef, rmse, resid = O.omp(F, np.arange(20), y, 1)
    r = [abs(np.corrcoef(f, y)[0, 1]) for f in F]
    assert act == [int(np.argmax(r))]


def test_omp_orthonormal_design(oracle_mod):
    """Centered orthonormal columns: OMP adds features in descending |r|
    and matches the exhaustive L0 optimum at every size."""
    O = oracle_mod
    rng = np.random.default_rng(16)
    n, S = 64, 10
    Q, _ = np.linalg.qr(rng.normal(size=(n, S + 1)))
    Q = Q[:, 1:] - Q[:, 1:].mean(axis=0)
    Q, _ = np.linalg.qr(np.column_stack([np.ones(n), Q]))
    F = Q[:, 1:S + 1].T.copy()
    y = F.T @ rng.normal(size=S) * 3 + 0.1 * rng.normal(size=n)
    act, _, _, _ = O.omp(F, np.arange(S), y, 5)
    r = np.abs([np.corrcoef(f, y)[0, 1] for f in F])
    assert act == list(np.argsort(-r)[:5])
    for D in range(1, 5):
        mo = O.l0(F, np.arange(S), y, D, mode="direct")[0]
        assert set(mo["positions"]) == set(act[:D])


def test_omp_matches_sklearn(oracle_mod):
    from sklearn.linear_model import OrthogonalMatchingPursuit
    O = oracle_mod
    rng = np.random.default_rng(17)
    F = _design(rng, S=25, n=120, corr=0.6)
    y = 2 * F[3] - F[17] + 0.5 * F[8] + 0.2 * rng.normal(size=120)
    act, coef, rmse, _ = O.omp(F, np.arange(25), y, 4)
    Fc = F - F.mean(axis=1, keepdims=True)
    Z = (Fc / np.linalg.norm(Fc, axis=1, keepdims=True)).T
    sk = OrthogonalMatchingPursuit(n_nonzero_coefs=4, fit_intercept=False).fit(Z, y - y.mean())
    assert set(act) == set(np.nonzero(sk.coef_)[0])
    # refit coefficients agree with plain least squares on the active set
    A = np.column_stack([np.ones(120)] + [F[i] for i in act])
    beta = np.linalg.lstsq(A, y, rcond=None)[0]
    np.testing.assert_allclose(coef, beta, rtol=1e-9, atol=1e-12)


def test_omp_warm_start(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(18)
    F = _design(rng, S=15, n=90)
    y = F[1] + F[2] + F[3] + 0.5 * F[10] + 0.05 * rng.normal(size=90)
    act, coef, rmse, resid = O.omp(F, np.arange(15), y, 5, init=(1, 2, 3))
    assert act[:3] == [1, 2, 3] and act[3] == 10 and len(act) == 5
    assert abs(np.dot(resid, F[1] - F[1].mean())) < 1e-9 * np.linalg.norm(F[1])


# ---------------------------------------------------------------- SISSO
def test_sisso_tiny_recovers_planted(oracle_mod):
    """y = 1.5 x0 x1 - 0.7 exp(-x2) + N(0, 1e-3): with rung 2 the D=2 model
    is x0*x1 and 1/exp(x2) with the planted coefficients."""
    import synth
    O = oracle_mod
    w = synth.tiny(rung=2)
    res = O.sisso(w)
    sp = res["space"]
    mo = res["dims"][1]["models"][0]
    names = sorted(sp.expr(i) for i in mo["ids"])
    assert names == ["(x0 * x1)", "inv(exp(x2))"]
    np.testing.assert_allclose(sorted(mo["coef"][1:]), [-0.7, 1.5], atol=3e-3)
    assert mo["rmse"] < 2e-3


@pytest.mark.slow
def test_sisso_units16_recovers_planted(oracle_mod):
    import synth
    O = oracle_mod
    w = synth.units16()
    res = O.sisso(w)
    mo = res["dims"][2]["models"][0]
    V, _ = O.values(res["space"], w["X"], w["units"], list(mo["ids"]))
    for term in w["planted"]:
        tv = synth.workloads._ev(term, w["X"])
        assert max(abs(np.corrcoef(v, tv)[0, 1]) for v in V) > 1 - 1e-9
    assert len(res["dims"][0]["sel_ids"]) == 500
    assert res["dims"][0]["nvalid"] <= 336214
