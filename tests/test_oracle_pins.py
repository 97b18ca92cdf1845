"""Further pins of the oracle, each chosen so that a plausible mistake in the
pinned routine fails it:

* the zero-score rule of the selection (a candidate with no linear
  association with the target is never selected);
* the L0 tie rule (models whose RSS differ by less than TAU_TIE of the
  target's centred sum of squares are tied, and the smaller sorted ID tuple
  wins), on a constructed near-tie;
* the correlation matrix of the Gram route against numpy.corrcoef;
* Gram mode on a near-collinear winner (a pivot near 1e-9, where the
  Gram route's explained fraction carries an error near eps / pivot): it
  must return the QR winner and its RSS;
* streamed screening (rung R-1 never stored) against the full screen, and
  direct mode's ranking by threshold against a plain sort of every subset.

The paper (Core Optimization Objective, Eq. (1)) defines the per-support
least-squares problem; the selection and tie rules are readings of it where
it is silent (top-k screening of the cited SISSO method, Summary)."""
import itertools
import math

import numpy as np
import pytest

import synth


def test_zero_score_never_selected(oracle_mod):
    """k exceeds the number of positive scores; the orthogonal candidates
    (score exactly 0) are valid but not selected."""
    O = oracle_mod
    score = np.array([np.nan, 0.5, 0.0, 0.25, 0.0, np.nan, 0.75])
    ids, sc, rec = O.select(score, 5)
    assert ids.tolist() == [6, 1, 3]
    assert sc.tolist() == [0.75, 0.5, 0.25]


def test_zero_score_constructed_orthogonal(oracle_mod):
    """A feature exactly orthogonal to the centred target has Pearson r = 0
    in exact arithmetic: y and f are built from orthogonal +-1 patterns, so
    every product and sum below is exact in IEEE double."""
    O = oracle_mod
    n = 8
    h1 = np.array([1, -1, 1, -1, 1, -1, 1, -1], float)
    h2 = np.array([1, 1, -1, -1, 1, 1, -1, -1], float)
    h3 = np.array([1, 1, 1, 1, -1, -1, -1, -1], float)
    F = np.vstack([3.0 + h2, 5.0 + 2.0 * h3, 1.0 + h1 + 0.5 * h2])
    y = 2.0 + h1
    r = O.pearson(F, y)[0]
    assert r[0] == 0.0 and r[1] == 0.0 and r[2] > 0
    ids, sc, _ = O.select(np.abs(r), 3)
    assert ids.tolist() == [2]


def _near_tie_design(rng, n=60):
    """Rows f0, f1, f2 with f2 = f1 + eps*z: the models {0, 1} and {0, 2}
    fit y = 1 + f0 + f1 + noise almost equally well."""
    f0 = rng.normal(size=n)
    f1 = rng.normal(size=n)
    y = 1.0 + f0 + f1 + 0.1 * rng.normal(size=n)
    # z orthogonal to 1, f0, f1 and the residual of {0, 1}: the RSS gap of
    # {0, 2} over {0, 1} then grows as eps^2
    A = np.column_stack([np.ones(n), f0, f1])
    r = y - A @ np.linalg.lstsq(A, y, rcond=None)[0]
    Q, _ = np.linalg.qr(np.column_stack([A, r]))
    z = rng.normal(size=n)
    z = z - Q @ (Q.T @ z)
    return f0, f1, z, y


def _gap(O, f0, f1, z, y, eps):
    _, r01 = O.lsq([f0, f1], y)
    _, r02 = O.lsq([f0, f1 + eps * z], y)
    return r02 - r01


@pytest.mark.parametrize("ratio,expect_tie", [(0.4, True), (4.0, False)])
def test_l0_tie_rule(oracle_mod, ratio, expect_tie):
    """Row 2 (the perturbed copy) carries the smaller candidate ID.  With an
    RSS gap of 0.4 TAU_TIE * yy the two models are tied and the smaller ID
    tuple wins although its RSS is larger; with 4 TAU_TIE * yy the smaller
    RSS wins."""
    O = oracle_mod
    rng = np.random.default_rng(21)
    f0, f1, z, y = _near_tie_design(rng)
    yc = y - y.mean()
    yy = float(yc @ yc)
    target = ratio * O.TAU_TIE * yy
    eps = 1e-3
    g = _gap(O, f0, f1, z, y, eps)
    assert g > 0
    for _ in range(3):                      # the gap grows as eps^2
        eps *= math.sqrt(target / g)
        g = _gap(O, f0, f1, z, y, eps)
    assert 0.8 * target < g < 1.25 * target, (g, target)
    F = np.vstack([f0, f1, f1 + eps * z])
    ids = np.array([10, 30, 20])            # row 2 has the smaller ID
    for mode in ("direct", "gram"):
        mo = O.l0(F, ids, y, 2, m=2, mode=mode)
        first = tuple(sorted(mo[0]["ids"]))
        if expect_tie:
            assert first == (10, 20), (mode, mo[0]["ids"])
            assert mo[0]["rss"] > mo[1]["rss"]
        else:
            assert first == (10, 30), (mode, mo[0]["ids"])
            assert mo[0]["rss"] < mo[1]["rss"]


def test_corr_matrix_matches_numpy(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(22)
    F = rng.lognormal(0, 0.5, size=(9, 70)) * rng.uniform(0.1, 10, size=(9, 1))
    y = F[2] - F[5] + rng.normal(size=70)
    Cm, c, yy = O.corr_matrix(F, y)
    ref = np.corrcoef(np.vstack([F, y]))
    np.testing.assert_allclose(Cm, ref[:9, :9], rtol=0, atol=2e-15)
    np.testing.assert_allclose(c, ref[:9, 9], rtol=0, atol=2e-15)
    assert abs(yy - float(np.sum((y - y.mean()) ** 2))) <= 1e-13 * yy


def test_gram_band_conditioning_allowance(oracle_mod):
    """The winning subset has a tiny pivot, so its Gram-route explained
    fraction carries an error near eps / pivot; Gram mode (whose band
    widens with 1 / pivot) must still return the QR winner and RSS."""
    O = oracle_mod
    rng = np.random.default_rng(23)
    n = 80
    a = rng.normal(size=n)
    b = a + 3e-5 * rng.normal(size=n)       # pivot of {a, b} near 1e-9
    others = rng.normal(size=(6, n))
    y = 50.0 * (b - a) / 3e-5 + a + 0.01 * rng.normal(size=n)
    F = np.vstack([a, b, others])
    ids = np.arange(F.shape[0])
    piv = O.pivots([a, b])
    assert piv.min() < 1e-7
    d = O.l0(F, ids, y, 2, m=1, mode="direct")[0]
    g = O.l0(F, ids, y, 2, m=1, mode="gram")[0]
    assert sorted(d["ids"]) == [0, 1]
    assert sorted(g["ids"]) == sorted(d["ids"])
    assert abs(g["rss"] - d["rss"]) <= 1e-12 * float(np.sum((y - y.mean()) ** 2))


def test_direct_threshold_ranking_equals_full_sort(oracle_mod):
    """Direct mode ranks only the subsets within TAU_TIE * yy of the m-th
    smallest RSS; a plain ranking of every subset gives the same models."""
    O = oracle_mod
    rng = np.random.default_rng(24)
    S, n, D, m = 9, 45, 3, 6
    F = rng.normal(size=(S, n))
    y = F[1] - 2 * F[4] + F[7] + rng.normal(size=n)
    ids = rng.permutation(100)[:S]
    mo = O.l0(F, ids, y, D, m=m, mode="direct")
    yy = float(np.sum((y - y.mean()) ** 2))
    cands = []
    for sub in itertools.combinations(range(S), D):
        _, r = O.lsq([F[i] for i in sub], y)
        cands.append((r, tuple(sorted(int(ids[i]) for i in sub)), sub))
    ref = O._rank_models(cands, m, yy)
    assert [tuple(sorted(x["ids"])) for x in mo] == [c[1] for c in ref]


@pytest.mark.parametrize("mode", ["max", "per_target"])
def test_streamed_screen_equals_full(oracle_mod, mode):
    """Operator-limited rung 3 (binary operators, partners primaries) with
    units, negative values and an exact zero: the streamed screen visits
    candidates grouped by their rung-2 operand and must reproduce the full
    screen's scores, NaN pattern and status counts exactly."""
    O = oracle_mod
    rng = np.random.default_rng(0)
    p, n = 5, 40
    X = rng.lognormal(0, 0.5, size=(p, n))
    X[1, 3] = -0.5
    X[2, 5] = 0.0
    units = rng.integers(-1, 2, size=(p, 2)).astype(np.int32)
    units[0] = 0
    units[3] = units[4]
    Y = np.vstack([X[0] * X[1] + rng.normal(size=n), rng.normal(size=n),
                   X[2] + rng.normal(size=n)])
    sp = O.Space(p, 3, synth.ALL_OPS, rung_ops=(None, None, None, synth.BINARY_OPS),
                 rung_pool=(None, None, None, 0))
    a, nva, sta, ca = O.screen_scores(sp, X, Y, units, mode)
    assert sta is not None
    old = O.STREAM_BYTES
    O.STREAM_BYTES = 0
    try:
        b, nvb, stb, cb = O.screen_scores(sp, X, Y, units, mode)
    finally:
        O.STREAM_BYTES = old
    assert stb is None
    assert nva == nvb and np.array_equal(ca, cb)
    assert np.array_equal(np.isnan(a), np.isnan(b))
    assert np.array_equal(a[~np.isnan(a)], b[~np.isnan(b)])
    assert ca[O.ST_NONFINITE] > 0 and ca[O.ST_UNIT] > 0 and ca[O.ST_CHILD] > 0
