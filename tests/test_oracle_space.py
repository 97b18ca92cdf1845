"""Pins of the oracle's candidate enumeration and unit rules.

The paper generates candidates iteratively from primary features and an
operator library (Software Description) and drops dimensionally invalid
expressions (Physics-Informed Constraints).  It prints no counts, so these
tests pin the oracle with closed forms, an independent brute force over
expression trees, and the physical scaling law that unit exponents encode.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from tests import brute

GOLD = os.path.join(os.path.dirname(__file__), "golden", "space_counts.json")


def closed_form(p, R, n_un=5, n_bin=5, limited=None):
    """|L_r| = n_un |L_{r-1}| + n_bin (C(|P_{r-1}|,2) - C(|P_{r-2}|,2));
    an operator-limited rung (binary only, partner pool P_q) has
    n_bin |L_{r-1}| |P_q|."""
    L = [p]
    P = [p]
    for r in range(1, R + 1):
        if limited and r in limited:
            nb, q = limited[r]
            L.append(nb * L[r - 1] * P[q])
        else:
            P2 = P[r - 2] if r >= 2 else 0
            L.append(n_un * L[r - 1] + n_bin * (math.comb(P[r - 1], 2) - math.comb(P2, 2)))
        P.append(P[r - 1] + L[r])
    return L, P[R]


def test_golden_counts(oracle_mod):
    O = oracle_mod
    with open(GOLD) as f:
        gold = json.load(f)
    for case in gold["cases"]:
        rung_ops = rung_pool = None
        if case.get("limited"):
            rung_ops = [None] * 4
            rung_pool = [None] * 4
            for r, (ops, q) in case["limited"].items():
                rung_ops[int(r)] = ops
                rung_pool[int(r)] = q
        sp = O.Space(case["p"], case["R"], O.OPS, rung_ops, rung_pool)
        assert sp.N == case["total"], case
        assert list(sp.levels) == case["levels"], case


@pytest.mark.parametrize("p,R", [(1, 1), (2, 2), (3, 2), (6, 1), (6, 2), (13, 2), (16, 2), (5, 3)])
def test_closed_form_counts(oracle_mod, p, R):
    sp = oracle_mod.Space(p, R, oracle_mod.OPS)
    L, tot = closed_form(p, R)
    assert list(sp.levels) == L
    assert sp.N == tot


def test_operator_limited_rung(oracle_mod):
    O = oracle_mod
    sp = O.Space(24, 3, O.OPS, [None, None, None, ("add", "sub", "mul", "div", "rdiv")],
                 [None, None, None, 0])
    L, tot = closed_form(24, 3, limited={3: (5, 0)})
    assert list(sp.levels) == L and sp.N == tot == 702860274


def test_masks_change_counts(oracle_mod):
    O = oracle_mod
    sp = O.Space(6, 2, ("mul", "div", "sq"))
    L, tot = closed_form(6, 2, n_un=1, n_bin=2)
    assert sp.N == tot


@pytest.mark.parametrize("p,R", [(2, 2), (3, 2), (4, 1), (1, 3)])
def test_brute_force_tree_set(oracle_mod, p, R):
    """The oracle's candidates, rung by rung, are exactly the expression
    trees of that depth (as canonical strings, no duplicates)."""
    O = oracle_mod
    sp = O.Space(p, R, O.OPS)
    lv = brute.trees_by_depth(p, R, O.OPS)
    rung, op, a, b = sp.enumerate()
    for r in range(R + 1):
        mine = [brute.canon(brute.oracle_tree(sp, int(i))) for i in np.nonzero(rung == r)[0]]
        ref = [brute.canon(t) for t in lv[r]]
        assert len(mine) == len(set(mine))
        assert sorted(mine) == sorted(ref)


def test_decode_roundtrip_and_order(oracle_mod):
    """decode(id) equals the enumerated record, and records follow the
    documented order: rung blocks, unary before binary, operator blocks in
    library order, then j ascending, then i ascending."""
    O = oracle_mod
    sp = O.Space(4, 2, O.OPS)
    rung, op, a, b = sp.enumerate()
    for cid in range(sp.N):
        assert sp.decode(cid) == (int(rung[cid]), int(op[cid]), int(a[cid]), int(b[cid]))
    idx = np.arange(sp.N)
    key = np.stack([rung, np.where(op == O.OP_NONE, -1, op),
                    np.where(op == O.OP_NONE, idx, np.where(b < 0, a, b)),
                    np.where(b < 0, 0, a)], axis=1).astype(np.int64)
    for t in range(1, sp.N):
        assert tuple(key[t - 1]) < tuple(key[t])
    assert np.all(a[b >= 0] < b[b >= 0])


def test_decode_limited_rung(oracle_mod):
    O = oracle_mod
    sp = O.Space(3, 3, O.OPS, [None, None, ("mul",), ("add", "rdiv")], [None, None, None, 0])
    rung, op, a, b = sp.enumerate()
    for cid in range(sp.N):
        assert sp.decode(cid) == (int(rung[cid]), int(op[cid]), int(a[cid]), int(b[cid]))
    r3 = rung == 3
    assert np.all(a[r3] < 3) and np.all(b[r3] >= sp.levels[:2].sum())


# ------------------------------------------------------------------ units
def _frac_units(t, units):
    """Independent unit inference with exact fractions; None = invalid."""
    if t[0] == "x":
        return tuple(Fraction(int(v)) for v in units[t[1]])
    if len(t) == 2:
        u = _frac_units(t[1], units)
        if u is None:
            return None
        if t[0] in ("exp", "log"):
            return u if all(v == 0 for v in u) else None
        f = {"sqrt": Fraction(1, 2), "sq": Fraction(2), "inv": Fraction(-1)}[t[0]]
        return tuple(v * f for v in u)
    ua, ub = _frac_units(t[1], units), _frac_units(t[2], units)
    if ua is None or ub is None:
        return None
    if t[0] in ("add", "sub"):
        return ua if ua == ub else None
    if t[0] == "mul":
        return tuple(x + y for x, y in zip(ua, ub))
    if t[0] == "div":
        return tuple(x - y for x, y in zip(ua, ub))
    return tuple(y - x for x, y in zip(ua, ub))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_units_against_fractions(oracle_mod, seed):
    O = oracle_mod
    rng = np.random.default_rng(seed)
    p, R, B = 4, 2, 2
    units = rng.integers(-1, 2, size=(p, B)).astype(np.int32)
    units[0] = 0                       # keep one dimensionless primary
    sp = O.Space(p, R, O.OPS)
    uo, legal = sp.units(units)
    Q = 1 << R
    for cid in range(sp.N):
        ref = _frac_units(brute.oracle_tree(sp, cid), units)
        assert legal[cid] == (ref is not None)
        if ref is not None:
            assert tuple(Fraction(int(v), Q) for v in uo[cid]) == ref


def test_units16_unit_valid_counts(oracle_mod):
    """Unit-valid counts per rung of the 16-feature, 3-base-unit workload;
    the same numbers follow from the fraction-based rule above."""
    import synth
    O = oracle_mod
    w = synth.units16()
    sp = O.Space.of(w)
    rung, _, _, _ = sp.enumerate()
    _, legal = sp.units(w["units"])
    assert [int(legal[rung == r].sum()) for r in range(3)] == [16, 448, 335750]


def test_distinct_units_forbid_add_sub(oracle_mod):
    O = oracle_mod
    units = np.eye(3, dtype=np.int32)          # three different base units
    sp = O.Space(3, 1, O.OPS)
    rung, op, a, b = sp.enumerate()
    _, legal = sp.units(units)
    addsub = (op == O.OP_CODE["add"]) | (op == O.OP_CODE["sub"])
    assert not legal[addsub].any()
    explog = (op == O.OP_CODE["exp"]) | (op == O.OP_CODE["log"])
    assert not legal[explog].any()
    assert legal[(op == O.OP_CODE["mul"])].all()


def test_units_scaling_law(oracle_mod):
    """Dimensional analysis: rescaling every primary by lambda^(its unit
    exponents) rescales a unit-legal candidate by lambda^(its exponents)."""
    import synth
    O = oracle_mod
    w = synth.units16()
    sp = O.Space.of(w)
    uo, legal = sp.units(w["units"])
    Q = 1 << sp.R
    lam = np.array([1.7, 0.6, 2.3])
    Xs = w["X"] * np.prod(lam[None, :] ** w["units"], axis=1)[:, None]
    rng = np.random.default_rng(7)
    ids = rng.choice(np.nonzero(legal)[0], 400, replace=False)
    V0, st0 = O.values(sp, w["X"], w["units"], ids)
    V1, st1 = O.values(sp, Xs, w["units"], ids)
    for t, cid in enumerate(ids):
        if st0[t] != O.ST_VALID:
            continue
        scale = np.prod(lam ** (uo[cid] / Q))
        np.testing.assert_allclose(V1[t], scale * V0[t], rtol=1e-12)
    # an add of mismatched units does not obey any such law
    bad = [i for i in np.nonzero(~legal)[0][:2000]
           if sp.decode(int(i))[1] == O.OP_CODE["add"] and sp.decode(int(i))[0] == 1][:5]
    assert bad
    V0, _ = O.values(sp, w["X"], w["units"], bad)
    V1, _ = O.values(sp, Xs, w["units"], bad)
    for t in range(len(bad)):
        ratio = V1[t] / V0[t]
        assert np.std(ratio) > 1e-3 * abs(np.mean(ratio))
