"""GPU parity of the constraint rules (Design Philosophy and Constraints:
rules on variable combinations and functional forms, complexity limits, the
target-unit filter): the library's selection under rules against the
oracle's selection over the scores of the candidates its rule mask allows
(Space.rules_allowed, pinned in test_oracle_rules.py).  Same bar as the
other screening tests: identical IDs, scores within 1e-10 relative, and the
generation counts unchanged by the rules.
"""
import numpy as np
import pytest

from tests.checks import check_selection

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


@pytest.fixture(scope="module")
def D():
    import paper_2602_06986_amd as D
    return D


def dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


RULES = {
    "cplx1": {"max_complexity": 1},
    "cplx2": {"max_complexity": 2},
    "pairs": {"forbid_pairs": [[0, 1], [2, 2]]},
    "nest": {"forbid_nest": {"exp": ["exp", "log"], "sq": ["sqrt", "sq"], "mul": ["div", "rdiv"],
                             "add": ["sub"]}},
    "mixed": {"max_complexity": 3, "forbid_pairs": [[1, 3]], "forbid_nest": {"log": ["exp"]}},
    "target": {"target_units": [1, 0]},
    "target_mixed": {"target_units": [0, 0], "forbid_pairs": [[0, 2]], "max_complexity": 2},
}


def _units(rng, p, B):
    if not B:
        return None
    u = rng.integers(-1, 2, size=(p, B)).astype(np.int32)
    u[0] = [1] + [0] * (B - 1)
    u[1] = 0
    return u


# (seed, p, n, B, R, rules, k, mode, T, precision)
CASES = [
    (0, 5, 70, 0, 2, "cplx1", 25, "per_target", 1, "fp64"),
    (1, 6, 129, 0, 2, "cplx2", 40, "per_target", 1, "fp64"),
    (2, 5, 64, 0, 2, "pairs", 60, "per_target", 1, "fp64"),
    (3, 4, 97, 0, 2, "nest", 80, "per_target", 1, "fp64"),
    (4, 6, 150, 2, 2, "mixed", 50, "max", 3, "fp64"),
    (5, 5, 90, 2, 2, "target", 30, "per_target", 1, "fp64"),
    (6, 6, 200, 2, 2, "target_mixed", 40, "max", 2, "fp64"),
    (7, 5, 130, 0, 1, "pairs", 15, "per_target", 1, "fp64"),
    (8, 6, 160, 0, 2, "mixed", 60, "per_target", 1, "bf16"),
    (9, 5, 130, 2, 2, "target", 30, "max", 4, "bf16"),
    # k beyond the number of allowed candidates: every allowed valid one, then -1
    (10, 4, 50, 2, 2, "target", 5000, "per_target", 1, "fp64"),
]


@pytest.mark.parametrize("seed,p,n,B,R,rname,k,mode,T,prec", CASES)
def test_rules_against_oracle(torch, ctx, D, oracle_mod, seed, p, n, B, R, rname, k, mode, T, prec):
    O = oracle_mod
    rules = RULES[rname]
    rng = np.random.default_rng(700 + seed)
    X = rng.lognormal(0, 0.4, size=(p, n))
    units = _units(rng, p, B)
    Y = np.array([X[0] * X[-1] + 0.3 * X[1] + 0.05 * (t + 1) * rng.normal(size=n) for t in range(T)])
    sp = O.Space(p, R, O.OPS)
    allowed = sp.rules_allowed(units, rules)
    lists, status, nvalid = O.sis(sp, X, units, Y, k, (), mode, True, allowed=allowed)
    q = D.params(rung=R, k=k, score_mode=D.SCORE_MAX if mode == "max" else D.SCORE_PER_TARGET,
                 precision=D.BF16_GUARD if prec == "bf16" else D.FP64)
    ctx.set_rules(rules)
    try:
        ids, sc, vals, st = ctx.generate_screen(dev(torch, X), dev(torch, Y), q, units=units)
    finally:
        ctx.set_rules(None)
    for t, (li, ls, _) in enumerate(lists):
        g = ids[t].cpu().numpy()
        check_selection(g, sc[t].cpu().numpy(), li, ls, what="%s list %d" % (rname, t))
        n_sel = int((g >= 0).sum())
        assert n_sel == len(li)
        assert bool((g[n_sel:] == -1).all())
        assert all(allowed[c] for c in g[:n_sel])
    # the rules change what is selected, not what is generated and scored
    assert st["n_raw"] == sp.N
    assert st["n_unit_valid"] == int((status != O.ST_UNIT).sum())
    assert st["n_scored"] == nvalid
    if prec == "bf16":
        assert st["max_lowprec_err"] <= st["guard_band"]
    if seed == 10:
        assert len(lists[0][0]) < k


def test_rules_rung3_limited(torch, ctx, D, oracle_mod):
    """Operator-limited rung 3 (rung-2 operands regenerated on the fly): the
    rules also reach inside the regenerated operand."""
    O = oracle_mod
    rng = np.random.default_rng(790)
    p, n = 5, 140
    X = rng.lognormal(0, 0.4, size=(p, n))
    units = np.array([[1, 0], [0, 0], [0, 1], [1, -1], [0, 0]], np.int32)
    Y = np.array([X[0] * X[1] * X[-1] + 0.2 * X[2] + 0.05 * rng.normal(size=n)])
    rung_ops = [None, None, None, ("add", "sub", "mul", "div", "rdiv")]
    rung_pool = [None, None, None, 0]
    sp = O.Space(p, 3, O.OPS, rung_ops, rung_pool)
    for rules in ({"max_complexity": 2, "forbid_pairs": [[0, 4]]},
                  {"forbid_nest": {"mul": ["div", "rdiv"], "div": ["exp"]}, "target_units": [1, 0]}):
        allowed = sp.rules_allowed(units, rules)
        (lst,), status, nvalid = O.sis(sp, X, units, Y, 40, (), "per_target", True, allowed=allowed)
        q = D.params(rung=3, k=40, rung_ops=rung_ops, rung_pool=rung_pool)
        ctx.set_rules(rules)
        try:
            ids, sc, _, st = ctx.generate_screen(dev(torch, X), dev(torch, Y), q, units=units)
        finally:
            ctx.set_rules(None)
        check_selection(ids[0].cpu().numpy(), sc[0].cpu().numpy(), lst[0], lst[1], what=str(rules))
        assert st["n_scored"] == nvalid


def test_rules_cleared(torch, ctx, D, oracle_mod):
    """After set_rules(None) the selection is the unrestricted one again."""
    O = oracle_mod
    rng = np.random.default_rng(791)
    X = rng.lognormal(0, 0.4, size=(5, 80))
    y = X[0] * X[2] + 0.1 * rng.normal(size=80)
    sp = O.Space(5, 2, O.OPS)
    (lst,), _, _ = O.sis(sp, X, None, y[None], 30)
    q = D.params(rung=2, k=30)
    ctx.set_rules({"max_complexity": 0})
    ids0, _, _, _ = ctx.generate_screen(dev(torch, X), dev(torch, y[None]), q)
    assert set(int(v) for v in ids0[0].cpu().numpy() if v >= 0) <= set(range(5))
    ctx.set_rules(None)
    ids, sc, _, _ = ctx.generate_screen(dev(torch, X), dev(torch, y[None]), q)
    check_selection(ids[0].cpu().numpy(), sc[0].cpu().numpy(), lst[0], lst[1], what="cleared")


def test_rules_errors(ctx, D):
    with pytest.raises(D.DiscoverError):
        ctx.set_rules({"forbid_pairs": [[0, 64]]})
    with pytest.raises(D.DiscoverError):
        ctx.set_rules({"max_complexity": -2})
    ctx.set_rules(None)
