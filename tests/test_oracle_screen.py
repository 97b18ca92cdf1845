"""Pins of the oracle's screening score, validity rules and exact top-k.

The paper screens candidates against the target (Figure 1 caption; SIS of
the cited SISSO method, Summary) without printing a formula or values, so the
score is pinned to numpy's Pearson correlation, to the invariances every
correlation obeys, and to a brute force over expression trees.
"""
import numpy as np
import pytest

from tests import brute


def test_pearson_matches_numpy(oracle_mod):
    rng = np.random.default_rng(0)
    F = rng.normal(size=(20, 57)) * rng.uniform(0.1, 10, size=(20, 1)) + rng.normal(size=(20, 1)) * 5
    Y = rng.normal(size=(3, 57))
    r = oracle_mod.pearson(F, Y)
    for t in range(3):
        for j in range(20):
            assert abs(r[t, j] - np.corrcoef(F[j], Y[t])[0, 1]) < 1e-14


def test_pearson_invariances(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(1)
    f = rng.lognormal(size=200)
    y = rng.normal(size=200) + f
    r0 = O.pearson(f, y)[0, 0]
    assert abs(r0) <= 1.0
    assert abs(O.pearson(y, y)[0, 0] - 1.0) < 1e-15
    for a, b in [(3.5, -2.0), (-0.01, 100.0), (1e6, 1e3)]:
        assert abs(O.pearson(a * f + b, y)[0, 0] - np.sign(a) * r0) < 1e-13
    # a centered vector orthogonal to the centered target
    yc = y - y.mean()
    g = rng.normal(size=200)
    g -= g.mean()
    g -= yc * np.dot(g, yc) / np.dot(yc, yc)
    assert abs(O.pearson(g + 7.0, y)[0, 0]) < 1e-14


def test_validity_rules(oracle_mod):
    """log of a non-positive sample, division by an exact zero, exp
    overflow and a constant feature are invalid, and so is every parent of
    an invalid feature."""
    O = oracle_mod
    n = 40
    rng = np.random.default_rng(2)
    X = rng.uniform(0.5, 2.0, size=(4, n))
    X[1, 3] = -0.5              # log(x1) non-finite
    X[2] = 800.0 + rng.uniform(0, 1, n)   # exp(x2) overflows
    X[3] = 5.0                  # constant primary
    sp = O.Space(4, 2, O.OPS)
    r, status, nv = O.screen_all(sp, X, X[0] * 2 + rng.normal(size=n), None)
    code = lambda *a: [i for i in range(sp.N) if sp.decode(i)[1:] == a][0]
    log1 = code(O.OP_CODE["log"], 1, -1)
    exp2 = code(O.OP_CODE["exp"], 2, -1)
    assert status[3] == O.ST_CONST
    assert status[log1] == O.ST_NONFINITE
    assert status[exp2] == O.ST_NONFINITE
    assert np.isnan(r[0, log1]) and np.isnan(r[0, 3])
    # every rung-2 feature with an invalid operand is ST_CHILD
    rung, op, a, b = sp.enumerate()
    bad = {3, log1, exp2}
    for t in np.nonzero(rung == 2)[0]:
        if a[t] in bad or b[t] in bad:
            assert status[t] in (O.ST_CHILD, O.ST_UNIT)
    # inv(exp(x2)) would be finite (0) but its operand is invalid
    assert status[code(O.OP_CODE["inv"], exp2, -1)] == O.ST_CHILD
    # (x0 / x1) * (x1 / x0) is constant
    d01 = code(O.OP_CODE["div"], 0, 1)
    r01 = code(O.OP_CODE["rdiv"], 0, 1)
    X2 = X.copy(); X2[1] = rng.uniform(0.5, 2.0, n)
    r2, st2, _ = O.screen_all(sp, X2, X[0] + rng.normal(size=n), None)
    assert st2[code(O.OP_CODE["mul"], d01, r01)] == O.ST_CONST


@pytest.mark.parametrize("p,R,seed", [(3, 2, 0), (2, 2, 1), (4, 1, 2)])
def test_scores_against_brute_force(oracle_mod, p, R, seed):
    """Every candidate's |r| equals numpy.corrcoef of an independently
    built and evaluated expression tree with the same canonical form."""
    O = oracle_mod
    rng = np.random.default_rng(seed)
    n = 30
    X = rng.uniform(0.5, 2.0, size=(p, n))
    y = rng.normal(size=n) + X[0] * X[-1]
    sp = O.Space(p, R, O.OPS)
    r, status, nv = O.screen_all(sp, X, y, None)
    ref = {}
    for lv in brute.trees_by_depth(p, R, O.OPS):
        for t in lv:
            v = brute.evaluate(t, X)
            ok = np.all(np.isfinite(v)) and np.std(v) > 1e-8 * np.sqrt(np.mean(v * v))
            if ok and t[0] in ("add", "sub"):
                va, vb = brute.evaluate(t[1], X), brute.evaluate(t[2], X)
                ok = np.sum(v * v) > 1e-20 * np.sum(va * va + vb * vb)
            if ok:
                ref[brute.canon(t)] = abs(np.corrcoef(v, y)[0, 1])
    for cid in range(sp.N):
        key = brute.canon(brute.oracle_tree(sp, cid))
        if status[cid] == O.ST_VALID:
            assert abs(abs(r[0, cid]) - ref[key]) < 1e-12, key
        elif status[cid] in (O.ST_NONFINITE, O.ST_CONST):
            assert key not in ref


def test_materialised_and_recursive_agree(oracle_mod):
    """Scores from the screen (operands kept per rung) equal scores from
    the recursive evaluation of the same IDs, bit for bit."""
    import synth
    O = oracle_mod
    w = synth.tiny(rung=2)
    sp = O.Space.of(w)
    r, status, _ = O.screen_all(sp, w["X"], w["Y"], None)
    ids = np.random.default_rng(3).choice(sp.N, 300, replace=False)
    V, st = O.values(sp, w["X"], None, ids)
    r2 = O.pearson(V, w["Y"])
    for t, cid in enumerate(ids):
        assert st[t] == status[cid]
        if st[t] == O.ST_VALID:
            assert r2[0, t] == r[0, cid]


# ---------------------------------------------------------------- top-k
def test_topk_without_dedup_is_full_sort(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(4)
    s = rng.uniform(size=5000)
    s[rng.choice(5000, 300, replace=False)] = np.nan
    s[100] = s[200] = s[300] = 0.99999          # exact ties: ID decides
    ids, sc, _ = O.select(s, 50, dedup=False)
    valid = np.nonzero(~np.isnan(s))[0]
    ref = sorted(valid, key=lambda i: (-s[i], i))[:50]
    assert list(ids) == ref
    assert list(ids[:3]) == [100, 200, 300]
    # exclusion removes exactly the excluded IDs
    ids2, _, _ = O.select(s, 50, exclude=ref[:5], dedup=False)
    assert list(ids2) == sorted([i for i in valid if i not in ref[:5]], key=lambda i: (-s[i], i))[:50]


def _space_with_dups(O):
    """x0..x2 on [0.5, 2]; rung 2 contains many exact rewrites of
    lower-rung features, e.g. (x0*x1)/x1 == x0 and inv(inv(x0)) == x0."""
    rng = np.random.default_rng(5)
    n = 50
    X = rng.uniform(0.5, 2.0, size=(3, n))
    y = 2.0 * X[0] + 0.01 * rng.normal(size=n)
    sp = O.Space(3, 2, O.OPS)
    return sp, X, y


def test_dedup_groups_collapse_to_min_id(oracle_mod):
    O = oracle_mod
    sp, X, y = _space_with_dups(O)
    (res,), status, _ = O.sis(sp, X, None, y[None, :], 10)
    ids, sc, rec = res
    # x0 is the planted feature; every exact rewrite of x0 is merged into it
    assert ids[0] == 0
    V, _ = O.values(sp, X, None, ids)
    for a in range(len(ids)):
        for b in range(a + 1, len(ids)):
            c = abs(np.corrcoef(V[a], V[b])[0, 1])
            assert c < 1 - 1e-9                   # no two selected are duplicates
    # the group of x0 holds its rewrites: count them by brute force
    r, status, _ = O.screen_all(sp, X, y, None)
    x0 = X[0]
    dup = [i for i in range(sp.N) if status[i] == O.ST_VALID and
           abs(abs(r[0, i]) - abs(r[0, 0])) <= 1e-9 * abs(r[0, 0]) and
           abs(np.corrcoef(O.values(sp, X, None, [i])[0][0], x0)[0, 1]) >= 1 - 1e-9]
    assert len(dup) >= 5 and min(dup) == 0
    # sqrt(sq(x0)), inv(inv(x0)), (x0*x1)/x1 are among them
    names = {sp.expr(i) for i in dup}
    assert "sqrt(sq(x0))" in names and "inv(inv(x0))" in names


def test_dedup_is_order_independent(oracle_mod):
    """Perturbing the scores of duplicates by a few ulps (which reorders
    them) does not change the selection."""
    O = oracle_mod
    sp, X, y = _space_with_dups(O)
    r, status, _ = O.screen_all(sp, X, y, None)
    s = np.abs(r[0])
    vcache = {}

    def vf(c):
        if c not in vcache:
            vcache[c] = O.values(sp, X, None, [c])[0][0]
        return vcache[c]

    base = O.select(s, 15, (), True, vf)[0]
    rng = np.random.default_rng(6)
    for _ in range(5):
        s2 = s * (1 + rng.integers(-4, 5, size=s.shape) * 2.0 ** -52)
        assert list(O.select(s2, 15, (), True, vf)[0]) == list(base)


def test_dedup_blocks_groups_of_excluded(oracle_mod):
    O = oracle_mod
    sp, X, y = _space_with_dups(O)
    (res,), _, _ = O.sis(sp, X, None, y[None, :], 10, exclude=[0])
    ids = res[0]
    V, _ = O.values(sp, X, None, ids)
    for t in range(len(ids)):
        assert ids[t] != 0
        assert abs(np.corrcoef(V[t], X[0])[0, 1]) < 1 - 1e-9


def test_max_mode_scores(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(8)
    r = rng.uniform(-1, 1, size=(4, 100))
    r[:, 5] = np.nan
    m = O.combine_scores(r, "max")
    assert m.shape == (1, 100) and np.isnan(m[0, 5])
    assert np.allclose(np.delete(m[0], 5), np.delete(np.abs(r).max(axis=0), 5))


def test_cancellation_rule(oracle_mod):
    """A sum or difference that cancels to rounding noise (x - exp(log x),
    x - sqrt(sq x)) is constant whatever the math library's last bits; a
    genuinely small difference (relative size 1e-6) is not."""
    O = oracle_mod
    rng = np.random.default_rng(9)
    n = 50
    X = rng.uniform(0.5, 2.0, size=(3, n))
    X[1] = X[0] * (1 + 1e-6 * rng.normal(size=n))
    sp = O.Space(3, 3, O.OPS, [None, None, None, ("sub",)], [None, None, None, 0])
    names = {"(x0 - exp(log(x0)))", "(x0 - sqrt(sq(x0)))", "(x2 - inv(inv(x2)))"}
    ids = [i for i in range(sp.levels[:3].sum(), sp.N) if sp.expr(i) in names]
    assert len(ids) == 3
    _, st = O.values(sp, X, None, ids)
    assert all(v == O.ST_CONST for v in st)
    small = [i for i in range(sp.levels[0], sp.levels[:2].sum()) if sp.expr(i) == "(x0 - x1)"]
    _, st = O.values(sp, X, None, small)
    assert st[0] == O.ST_VALID
