"""Pins of the oracle's constraint rules (Design Philosophy and
Constraints: rules on variable combinations and functional forms,
complexity limits, the target-unit filter), each checked against the
printed expression of every candidate of a small space rather than against
the rule code's own recursion:

* complexity = the number of operator tokens in the printed expression;
* a forbidden pair of primaries never appears together in an allowed
  expression, and every expression without the pair is allowed;
* exp directly over exp or log never appears in an allowed expression;
* the target-unit filter keeps exactly the unit-legal candidates with the
  target's exponents;
* rules are hereditary (an allowed candidate has allowed operands), and a
  selection under rules equals a plain sort of the allowed scores.
"""
import re

import numpy as np
import pytest


def _space(O, p=4, R=2):
    return O.Space(p, R, O.OPS)


def _n_ops(text):
    return len(re.findall(r"\b(exp|log|sqrt|sq|inv)\(", text)) + len(re.findall(r" [-+*/] ", text))


@pytest.mark.parametrize("cmax", [0, 1, 2])
def test_complexity_limit(oracle_mod, cmax):
    O = oracle_mod
    sp = _space(O)
    al = sp.rules_allowed(None, {"max_complexity": cmax})
    for cid in range(sp.N):
        assert al[cid] == (_n_ops(sp.expr(cid)) <= cmax), (cid, sp.expr(cid))


def test_forbidden_pair(oracle_mod):
    O = oracle_mod
    sp = _space(O)
    al = sp.rules_allowed(None, {"forbid_pairs": [[0, 2]]})
    for cid in range(sp.N):
        t = sp.expr(cid)
        both = re.search(r"\bx0\b", t) and re.search(r"\bx2\b", t)
        assert al[cid] == (not both), (cid, t)


def test_forbidden_nesting(oracle_mod):
    O = oracle_mod
    sp = _space(O, p=3, R=2)
    al = sp.rules_allowed(None, {"forbid_nest": {"exp": ["exp", "log"], "sq": ["sqrt"]}})
    for cid in range(sp.N):
        t = sp.expr(cid)
        bad = "exp(exp(" in t or "exp(log(" in t or "sq(sqrt(" in t
        assert al[cid] == (not bad), (cid, t)


def test_target_unit_filter(oracle_mod):
    O = oracle_mod
    sp = _space(O, p=4, R=2)
    units = np.array([[1, 0], [0, 1], [1, -1], [0, 0]], np.int32)
    uo, legal = sp.units(units)
    al = sp.rules_allowed(units, {"target_units": [1, 0]})
    want = legal & np.all(uo == np.array([1, 0]) * (1 << sp.R), axis=1)
    assert np.array_equal(al, want)
    assert al.sum() > 0


def test_hereditary_and_selection(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(4)
    sp = _space(O, p=4, R=2)
    rules = {"max_complexity": 2, "forbid_pairs": [[1, 3]], "forbid_nest": {"log": ["exp"]}}
    al = sp.rules_allowed(None, rules)
    rung, op, a, b = sp.enumerate()
    for t in range(sp.N):
        if al[t] and op[t] != O.OP_NONE:
            assert al[a[t]] and (b[t] < 0 or al[b[t]])
    X = rng.uniform(0.5, 2.0, size=(4, 60))
    y = X[1] * X[3] + X[0] + 0.1 * rng.normal(size=60)
    (lst,), status, nvalid = O.sis(sp, X, None, y[None], 15, (), "per_target", False, allowed=al)
    (full,), status2, nvalid2 = O.sis(sp, X, None, y[None], 15, (), "per_target", False)
    assert nvalid == nvalid2                    # rules do not change the counts
    assert all(al[i] for i in lst[0])
    sc, _, _, _ = O.screen_scores(sp, X, y[None], None, "per_target")
    s = np.where(al & (sc[0] > 0), sc[0], np.nan)
    idx = np.nonzero(~np.isnan(s))[0]
    ref = idx[np.lexsort((idx, -s[idx]))][:15]
    assert list(lst[0]) == list(ref)
