"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle on
the same seeded inputs.

Bar (derived from the FP64 rounding of the two-pass moments and the QR refit):
  * selected candidate IDs, unit-prune counts and L0 winners: identical;
    where the oracle itself has a near-tie (|delta s| <= 1e-12 s at the
    cut, not a duplicate) either member is accepted;
  * scores: |s_gpu - s_oracle| <= 1e-10 s_oracle;
  * RMSE: <= 1e-10 relative (+1e-13 std(y) absolute);
  * coefficients: <= 1e-10 relative to the largest |coef| of the model.
"""
import math

import numpy as np
import pytest

from tests.checks import S_RTOL, TIE, check_model, check_selection  # noqa: F401

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


def dev(torch, a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def prm_of(D, w, k=None, dedup=True, mode=None):
    return D.params(ops=w["ops"], rung=w["rung"], k=k or w["k"],
                    score_mode=D.SCORE_MAX if (mode or w["score_mode"]) == "max" else D.SCORE_PER_TARGET,
                    dedup=dedup, rung_ops=w.get("rung_ops"), rung_pool=w.get("rung_pool"))


def run_both(torch, ctx, D, O, w, l0_mode="auto"):
    ref = O.sisso(w, l0_mode=l0_mode)
    X = dev(torch, w["X"])
    y = dev(torch, w["Y"][0])
    got = ctx.sisso(X, y, prm_of(D, w), w["D"], units=w["units"], n_resid=w["n_resid"],
                    omp_D=w["omp_D"])
    return ref, got


def compare_sisso(ref, got, w, what):
    y = w["Y"][0]
    S_g = got["S_ids"].cpu().numpy()
    for d, (rd, gd) in enumerate(zip(ref["dims"], got["dims"])):
        check_selection(gd["sel_ids"].cpu().numpy(), gd["sel_scores"].cpu().numpy(),
                        rd["sel_ids"], rd["sel_scores"], what="%s dim %d" % (what, d + 1))
        st = gd["screen_stats"]
        assert st["n_raw"] == ref["space"].N
        assert st["n_unit_valid"] == int((rd["status"] != 1).sum()), (st, what)
        assert st["n_scored"] == rd["nvalid"], (st["n_scored"], rd["nvalid"], what)
        subs = gd["subsets"].cpu().numpy()
        for q, mo in enumerate(rd["models"]):
            ids_g = [int(S_g[i]) for i in subs[q]]
            check_model(ids_g, float(gd["rmse"][q]), gd["coef"][q].cpu().numpy(), mo, y,
                        "%s dim %d model %d" % (what, d + 1, q))


# ---------------------------------------------------------------- SISSO loops
@pytest.mark.parametrize("name", ["tiny", "tiny_r2"])
def test_sisso_small(torch, ctx, D, oracle_mod, name):
    import synth
    w = synth.make(name)
    ref, got = run_both(torch, ctx, D, oracle_mod, w)
    compare_sisso(ref, got, w, name)


# ---------------------------------------------------------------- screening
def test_multitarget_per_target(torch, ctx, D, oracle_mod):
    import synth
    O = oracle_mod
    w = synth.multitarget16()
    sp = O.Space.of(w)
    (lists), status, nvalid = O.sis(sp, w["X"], None, w["Y"], w["k"], (), "per_target")
    ids, sc, vals, st = ctx.generate_screen(dev(torch, w["X"]), dev(torch, w["Y"]),
                                            prm_of(D, w, mode="per_target"))
    assert ids.shape == (16, 20)
    for t in range(16):
        check_selection(ids[t].cpu().numpy(), sc[t].cpu().numpy(), lists[t][0], lists[t][1],
                        what="target %d" % t)
    # the returned values are the selected features' values
    V, _ = O.values(sp, w["X"], None, ids[3].cpu().numpy())
    np.testing.assert_allclose(vals[3].cpu().numpy(), V, rtol=1e-12, atol=0)


# seeds 7 and 8: k large enough that the pool exceeds 4096 entries (the
# duplicate groups are then formed in global memory instead of LDS); seed 9:
# more than 1024 representatives from a pool within 4096 entries (the LDS
# group kernel orders them by rank counts instead of its bitonic sort)
@pytest.mark.parametrize("seed,p,n,B,R,dedup,k", [
    (0, 5, 37, 0, 2, True, 7), (1, 7, 129, 2, 2, True, 40), (2, 4, 64, 0, 2, False, 25),
    (3, 6, 65, 3, 2, True, 300), (4, 3, 20, 1, 1, True, 50), (5, 9, 200, 0, 1, True, 10),
    (6, 5, 3, 0, 1, True, 5), (7, 7, 90, 0, 2, True, 2600), (8, 6, 65, 2, 2, True, 2100),
    (9, 7, 90, 0, 2, True, 1200)])
def test_screen_random(torch, ctx, D, oracle_mod, seed, p, n, B, R, dedup, k):
    """Ragged sizes (n and operand counts off the 64 grid), units on/off,
    duplicates on/off, k beyond the number of valid candidates."""
    O = oracle_mod
    rng = np.random.default_rng(100 + seed)
    X = rng.lognormal(0, 0.4, size=(p, n))
    units = rng.integers(-1, 2, size=(p, B)).astype(np.int32) if B else None
    if B:
        units[: max(1, p // 3)] = 0
    y = X[0] * X[-1] + 0.3 * X[1 % p] + 0.05 * rng.normal(size=n)
    sp = O.Space(p, R, O.OPS)
    (lst,), status, nvalid = O.sis(sp, X, units, y[None], k, (), "per_target", dedup)
    ids, sc, vals, st = ctx.generate_screen(dev(torch, X), dev(torch, y[None]),
                                            D.params(rung=R, k=k, dedup=dedup), units=units)
    check_selection(ids[0].cpu().numpy(), sc[0].cpu().numpy(), lst[0], lst[1], what="seed %d" % seed)
    assert st["n_unit_valid"] == int((status != O.ST_UNIT).sum())
    assert st["n_scored"] == nvalid
    n_sel = int((ids[0] >= 0).sum())
    assert n_sel == len(lst[0])
    if n_sel < k:
        assert bool((ids[0][n_sel:] == -1).all())
    # the returned values are the selected features' values (copied from the
    # rescoring's stored rows, or evaluated where none is stored)
    V, _ = O.values(sp, X, units, ids[0][:n_sel].cpu().numpy())
    np.testing.assert_allclose(vals[0][:n_sel].cpu().numpy(), V, rtol=1e-12, atol=0)


def test_screen_duplicates_second_round(torch, ctx, D, oracle_mod):
    """Nine power-of-two multiples of one column and four of another: most
    candidates duplicate a better one, so the first pool holds fewer than k
    representatives and the selection takes a second, wider round; the
    list and the returned values still match."""
    O = oracle_mod
    rng = np.random.default_rng(321)
    n, k = 77, 40
    base = rng.lognormal(0, 0.4, size=(3, n))
    X = np.stack([base[0] * 2.0 ** j for j in range(9)] + [base[1] * 2.0 ** -j for j in range(4)]
                 + [base[2]])
    y = base[0] * base[1] + 0.3 * base[2] + 0.05 * rng.normal(size=n)
    sp = O.Space(X.shape[0], 2, O.OPS)
    (lst,), status, nvalid = O.sis(sp, X, None, y[None], k, (), "per_target", True)
    ids, sc, vals, st = ctx.generate_screen(dev(torch, X), dev(torch, y[None]), D.params(rung=2, k=k))
    check_selection(ids[0].cpu().numpy(), sc[0].cpu().numpy(), lst[0], lst[1], what="duplicates")
    assert st["pool_rounds"] >= 1
    assert st["n_merged"] > 0
    V, _ = O.values(sp, X, None, ids[0].cpu().numpy())
    np.testing.assert_allclose(vals[0].cpu().numpy(), V, rtol=1e-12, atol=0)


@pytest.mark.parametrize("T", [1, 2, 3])
def test_tile_width_invariant(torch, ctx, D, T):
    """The dense pair kernel's tile width (forced 1/2/4, or autotuned) and
    its schedule (one block per tile, or one persistent launch over a device
    work queue, or autotuned) do not change a single bit of the selected
    IDs, scores or values, nor the counts."""
    rng = np.random.default_rng(77 + T)
    p, n = 11, 203
    X = rng.lognormal(0, 0.5, size=(p, n))
    Y = np.stack([X[t] * X[-1 - t] + 0.1 * rng.normal(size=n) for t in range(T)])
    Xd, Yd = dev(torch, X), dev(torch, Y)
    runs = {}
    for tj in (0, 1, 2, 4):
        for sched in (0, -1, 1):
            ids, sc, vals, st = ctx.generate_screen(Xd, Yd, D.params(rung=2, k=60, tile_j=tj, sched=sched))
            runs[tj, sched] = (ids.cpu().numpy(), sc.cpu().numpy(), st["tile_j"], vals.cpu().numpy(),
                               st["n_scored"], st["n_unit_valid"])
    widest = {1: 4, 2: 2}.get(T, 1)
    ref = runs[1, -1]
    for (tj, sched), r in runs.items():
        if tj:
            assert r[2] == min(tj, widest)
        else:
            assert r[2] in (1, 2, 4) and r[2] <= widest
        assert np.array_equal(r[0], ref[0]), (tj, sched)
        assert np.array_equal(r[1].view(np.int64), ref[1].view(np.int64)), (tj, sched)
        assert np.array_equal(r[3].view(np.int64), ref[3].view(np.int64)), (tj, sched)
        assert r[4:] == ref[4:], (tj, sched)
    with pytest.raises(D.DiscoverError):
        ctx.generate_screen(Xd, Yd, D.params(rung=2, k=60, tile_j=5))
    with pytest.raises(D.DiscoverError):
        ctx.generate_screen(Xd, Yd, D.params(rung=2, k=60, sched=2))


def test_screen_exclusion(torch, ctx, D, oracle_mod):
    """IDs already in the subspace and their duplicate groups are not
    selected again."""
    import synth
    O = oracle_mod
    w = synth.tiny(rung=2)
    sp = O.Space.of(w)
    (first,), _, _ = O.sis(sp, w["X"], None, w["Y"], 20)
    excl = first[0][:7]
    (lst,), _, _ = O.sis(sp, w["X"], None, w["Y"], 20, excl)
    ids, sc, _, _ = ctx.generate_screen(dev(torch, w["X"]), dev(torch, w["Y"]), prm_of(D, w),
                                        exclude=dev(torch, excl, torch.int64))
    check_selection(ids[0].cpu().numpy(), sc[0].cpu().numpy(), lst[0], lst[1], what="exclude")
    assert not set(excl) & set(ids[0].cpu().numpy().tolist())


def test_screen_errors(torch, ctx, D):
    X = dev(torch, np.random.default_rng(0).uniform(0.5, 2, size=(4, 30)))
    with pytest.raises(D.DiscoverError) as e:
        ctx.generate_screen(X, dev(torch, np.ones((1, 30))), D.params(rung=1, k=5))
    assert e.value.code == -5
    with pytest.raises(D.DiscoverError) as e:
        ctx.generate_screen(X, dev(torch, np.arange(30.0)[None]), D.params(rung=5, k=5))
    assert e.value.code == -1
    with pytest.raises(D.DiscoverError) as e:
        ctx.generate_screen(X, dev(torch, np.arange(30.0)[None]), D.params(rung=1, k=0))
    assert e.value.code == -1


# ---------------------------------------------------------------- L0 / OMP
def _design(rng, S, n, corr=0.5):
    base = rng.normal(size=(3, n))
    F = rng.normal(size=(S, n)) + corr * base[rng.integers(0, 3, size=S)]
    return F * rng.uniform(0.5, 3.0, size=(S, 1)) + rng.normal(size=(S, 1))


# D = 3 with m <= 16 runs the bounded sweep (a lower bound from m rows);
# m = 17, 20 the unbounded one; S = 4, m = 3 has fewer rows holding a triple
# than m (the bound is switched off inside the bounded sweep).
@pytest.mark.parametrize("Dd,S,n,m", [(1, 70, 97, 3), (2, 70, 97, 3), (3, 70, 97, 3), (3, 131, 50, 1),
                                      (2, 5, 7, 4), (3, 3, 6, 1), (3, 200, 301, 8), (3, 90, 80, 16),
                                      (3, 90, 80, 17), (3, 70, 97, 20), (3, 4, 9, 3), (3, 5, 9, 10)])
def test_l0_against_oracle(torch, ctx, D, oracle_mod, Dd, S, n, m):
    O = oracle_mod
    rng = np.random.default_rng(S * 10 + Dd)
    F = _design(rng, S, n)
    y = 0.3 + F[S // 2] - 0.7 * F[S - 1] + 0.2 * F[0] + 0.1 * rng.normal(size=n)
    ids = rng.permutation(10 ** 6)[:S].astype(np.int64)
    ref = O.l0(F, ids, y, Dd, m=m, mode="direct")
    sub, rmse, coef, res, st = ctx.l0_fit(dev(torch, F), dev(torch, ids), dev(torch, y), Dd, m)
    assert st["n_subsets"] == math.comb(S, Dd)
    for q, mo in enumerate(ref):
        s = sub[q].cpu().numpy()
        check_model([int(ids[i]) for i in s], float(rmse[q]), coef[q].cpu().numpy(), mo, y, "q%d" % q)
        np.testing.assert_allclose(res[q].cpu().numpy(), mo["resid"], rtol=0,
                                   atol=1e-10 * np.max(np.abs(mo["resid"])))
    for q in range(len(ref), m):
        assert int(sub[q][0]) == -1


def test_l0_noise_free_planted(torch, ctx, D, oracle_mod):
    """y = c0 + c1 f_a + c2 f_b exactly: winner {a, b}, RMSE ~ 0, planted
    coefficients; at D = 3 every superset fits exactly and the smallest ID
    tuple wins."""
    rng = np.random.default_rng(42)
    F = _design(rng, 60, 120)
    y = 0.7 + 1.3 * F[17] - 2.1 * F[44]
    ids = np.arange(60, dtype=np.int64) * 3 + 5
    sub, rmse, coef, _, _ = ctx.l0_fit(dev(torch, F), dev(torch, ids), dev(torch, y), 2, 1)
    assert sorted(sub[0].cpu().numpy().tolist()) == [17, 44]
    assert float(rmse[0]) <= 1e-12 * np.std(y)
    np.testing.assert_allclose(coef[0].cpu().numpy(), [0.7, 1.3, -2.1], rtol=1e-10)
    ref = oracle_mod.l0(F, ids, y, 3, mode="direct")[0]
    sub3, _, _, _, _ = ctx.l0_fit(dev(torch, F), dev(torch, ids), dev(torch, y), 3, 1)
    assert sorted(ids[sub3[0].cpu().numpy()].tolist()) == sorted(ref["ids"])


def test_l0_singular_rejected(torch, ctx, D):
    rng = np.random.default_rng(3)
    F = _design(rng, 8, 40)
    F[5] = 2.0 * F[2] + 1.0
    y = F[2] + F[6] + 0.01 * rng.normal(size=40)
    ids = np.arange(8, dtype=np.int64)
    sub, _, _, _, _ = ctx.l0_fit(dev(torch, F), dev(torch, ids), dev(torch, y), 2, 20)
    for q in range(20):
        s = set(sub[q].cpu().numpy().tolist())
        assert s != {2, 5}


@pytest.mark.parametrize("m", [1, 6, 30])
def test_l0_d3_singular_and_duplicates(torch, ctx, D, oracle_mod, m):
    """D = 3 with an exact linear dependency (f5 = f2 + f3, so {2, 3, 5} is
    singular but fits y perfectly) and an exact duplicate row (f9 = f4):
    every returned model matches the oracle's, none is singular."""
    rng = np.random.default_rng(11)
    F = _design(rng, 40, 60)
    F[5] = F[2] + F[3]
    F[9] = F[4]
    y = F[2] + F[3] - 0.5 * F[5] + 0.4 * F[30] + 0.05 * rng.normal(size=60)
    ids = np.arange(40, dtype=np.int64) * 7 + 1
    ref = oracle_mod.l0(F, ids, y, 3, m=m, mode="direct")
    sub, rmse, coef, _, _ = ctx.l0_fit(dev(torch, F), dev(torch, ids), dev(torch, y), 3, m)
    for q, mo in enumerate(ref):
        s = sub[q].cpu().numpy()
        assert set(s.tolist()) != {2, 3, 5} and not {4, 9} <= set(s.tolist())
        check_model([int(ids[i]) for i in s], float(rmse[q]), coef[q].cpu().numpy(), mo, y, "q%d" % q)


@pytest.mark.parametrize("init", [None, (3, 9)])
def test_omp_against_oracle(torch, ctx, D, oracle_mod, init):
    O = oracle_mod
    rng = np.random.default_rng(7)
    F = _design(rng, 90, 150, corr=0.6)
    y = 2 * F[3] - F[17] + 0.5 * F[8] + 0.3 * F[60] + 0.2 * rng.normal(size=150)
    ids = np.arange(90, dtype=np.int64) + 1000
    act_o, coef_o, rmse_o, res_o = O.omp(F, ids, y, 6, init or ())
    it = None if init is None else dev(torch, np.array(init, np.int32), torch.int32)
    act, coef, rmse, res = ctx.omp(dev(torch, F), dev(torch, ids), dev(torch, y), 6, it)
    assert act.cpu().numpy().tolist() == act_o
    np.testing.assert_allclose(coef.cpu().numpy(), coef_o, rtol=1e-10, atol=1e-10 * np.max(np.abs(coef_o)))
    assert abs(float(rmse[0]) - rmse_o) <= 1e-10 * rmse_o


# ------------------------------------------------------------ precision forms
@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_precision_multitarget(torch, ctx, D, oracle_mod, prec):
    """16 targets at once through the MFMA form: every per-target top-20
    equals the FP64 oracle's, and the measured low-precision error stays
    inside the guard half-width."""
    import synth
    O = oracle_mod
    w = synth.multitarget16()
    sp = O.Space.of(w)
    lists, status, nvalid = O.sis(sp, w["X"], None, w["Y"], w["k"], (), "per_target")
    q = prm_of(D, w, mode="per_target")
    q.precision = D.BF16_GUARD if prec == "bf16" else D.FP16_GUARD
    q.lp_pairs = 1                                  # the MFMA form, whatever the autotuner prefers
    ids, sc, _, st = ctx.generate_screen(dev(torch, w["X"]), dev(torch, w["Y"]), q)
    for t in range(16):
        check_selection(ids[t].cpu().numpy(), sc[t].cpu().numpy(), lists[t][0], lists[t][1],
                        what="%s target %d" % (prec, t))
    # FP16: delta of standardised values; BF16: 1.1 delta (shifted values,
    # scores stored for kappa <= 1.21, error delta * sqrt(kappa))
    assert 0 < st["guard_band"] < (0.01 if prec == "fp16" else 0.02)
    assert st["max_lowprec_err"] <= st["guard_band"]


@pytest.mark.parametrize("prec,T,B,rung", [("bf16", 8, 0, 2), ("fp16", 8, 0, 2), ("bf16", 16, 2, 2),
                                           ("fp16", 3, 3, 2), ("bf16", 1, 0, 2)])
def test_precision_max_mode(torch, ctx, D, oracle_mod, prec, T, B, rung):
    """Several residual-like targets scored by their maximum |r| (one list)."""
    O = oracle_mod
    rng = np.random.default_rng(T * 7 + B)
    p, n = 6, 203
    X = rng.lognormal(0, 0.4, size=(p, n))
    units = rng.integers(-1, 2, size=(p, B)).astype(np.int32) if B else None
    if B:
        units[:2] = 0
    Y = np.array([X[t % p] * X[(t + 1) % p] + rng.normal(size=n) * (0.2 + 0.1 * t) for t in range(T)])
    sp = O.Space(p, rung, O.OPS)
    (lst,), status, nvalid = O.sis(sp, X, units, Y, 60, (), "max")
    q = D.params(rung=rung, k=60, score_mode=D.SCORE_MAX,
                 precision=D.BF16_GUARD if prec == "bf16" else D.FP16_GUARD, lp_pairs=1)
    ids, sc, _, st = ctx.generate_screen(dev(torch, X), dev(torch, Y), q, units=units)
    check_selection(ids[0].cpu().numpy(), sc[0].cpu().numpy(), lst[0], lst[1], what="max %s" % prec)
    assert st["n_scored"] == nvalid
    assert st["max_lowprec_err"] <= st["guard_band"]


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_precision_choice_invariant(torch, ctx, D, prec):
    """The precision form of the pair tiles, the FP64 tiles and the
    autotuner's choice between them select the same features with the same
    exact scores and values."""
    rng = np.random.default_rng(91)
    p, n, T = 7, 311, 8
    X = rng.lognormal(0, 0.4, size=(p, n))
    Y = np.array([X[t % p] / X[(t + 2) % p] + rng.normal(size=n) * 0.3 for t in range(T)])
    out = []
    for lp in (1, -1, 0):
        q = D.params(rung=2, k=40, score_mode=D.SCORE_MAX, lp_pairs=lp,
                     precision=D.BF16_GUARD if prec == "bf16" else D.FP16_GUARD)
        out.append(ctx.generate_screen(dev(torch, X), dev(torch, Y), q))
    for ids, sc, vals, st in out[1:]:
        assert np.array_equal(ids.cpu().numpy(), out[0][0].cpu().numpy())
        assert np.array_equal(sc.cpu().numpy(), out[0][1].cpu().numpy())
        assert np.array_equal(vals.cpu().numpy(), out[0][2].cpu().numpy())


# ------------------------------------------------------- operator-limited rung 3
@pytest.mark.parametrize("seed,p,n,B,T,mode,prec", [
    (0, 4, 61, 0, 1, "per_target", "fp64"), (1, 5, 130, 2, 1, "per_target", "fp64"),
    (2, 4, 97, 0, 3, "max", "fp64"), (3, 5, 64, 3, 2, "max", "fp64"),
    (4, 5, 130, 2, 1, "per_target", "bf16"), (5, 4, 97, 0, 3, "max", "bf16"),
    (6, 6, 200, 3, 8, "max", "bf16"), (7, 4, 33, 0, 5, "per_target", "bf16")])
def test_screen_rung3_limited(torch, ctx, D, oracle_mod, seed, p, n, B, T, mode, prec):
    """Rung 3 restricted to binary operators with a primary partner: the
    rung-2 operand of every rung-3 candidate is regenerated on the fly (FP64
    matrix products, or the BF16 precision form with its exact rescoring of
    the guard band)."""
    O = oracle_mod
    rng = np.random.default_rng(300 + seed)
    X = rng.lognormal(0, 0.4, size=(p, n))
    units = rng.integers(-1, 2, size=(p, B)).astype(np.int32) if B else None
    if B:
        units[:2] = 0
    Y = np.array([X[0] * X[1] * X[-1] + 0.2 * X[2] + 0.05 * (t + 1) * rng.normal(size=n) for t in range(T)])
    rung_ops = [None, None, None, ("add", "sub", "mul", "div", "rdiv")]
    rung_pool = [None, None, None, 0]
    sp = O.Space(p, 3, O.OPS, rung_ops, rung_pool)
    lists, status, nvalid = O.sis(sp, X, units, Y, 30, (), mode)
    q = D.params(rung=3, k=30, rung_ops=rung_ops, rung_pool=rung_pool,
                 score_mode=D.SCORE_MAX if mode == "max" else D.SCORE_PER_TARGET,
                 precision=D.BF16_GUARD if prec == "bf16" else D.FP64)
    ids, sc, vals, st = ctx.generate_screen(dev(torch, X), dev(torch, Y), q, units=units)
    if prec == "bf16":
        assert st["max_lowprec_err"] <= st["guard_band"]
    for t, (li, ls, _) in enumerate(lists):
        check_selection(ids[t].cpu().numpy(), sc[t].cpu().numpy(), li, ls, what="r3 list %d" % t)
    assert st["n_raw"] == sp.N
    assert st["n_unit_valid"] == int((status != O.ST_UNIT).sum())
    assert st["n_scored"] == nvalid
    V, _ = O.values(sp, X, units, ids[0].cpu().numpy())
    np.testing.assert_allclose(vals[0].cpu().numpy(), V, rtol=1e-12, atol=0)


# ------------------------------------------------ degenerate inputs
def _degenerate_X(rng, p, n):
    """Primaries that exercise every validity path: negatives (log and sqrt
    of values <= 0), exact zeros (division by zero, log 0), magnitudes whose
    exp overflows, a constant offset far above the spread (large
    mean-to-spread ratio: the one-pass moments are not trusted and the exact
    fix-up decides), a NaN (every candidate built on that column is
    invalid) and an affine copy of another column (duplicate groups)."""
    X = rng.lognormal(0, 0.5, size=(p, n))
    X[1] -= 1.0
    X[2, ::7] = 0.0
    X[3] *= 400.0
    X[4] = 1000.0 + rng.uniform(0.0, 1.0, size=n)
    X[5, 5] = np.nan
    if p > 6:
        X[6] = 2.0 * X[0] + 1.0
    return X


@pytest.mark.parametrize("seed,p,n,R,fixcap", [(0, 7, 64, 2, 0), (1, 7, 130, 2, 3),
                                              (2, 6, 45, 3, 0), (3, 6, 70, 3, 5)])
def test_screen_degenerate_inputs(torch, ctx, D, oracle_mod, seed, p, n, R, fixcap):
    """Non-finite and degenerate candidates are pruned exactly as the oracle
    prunes them (counts of unit-valid and scored candidates equal), and the
    selection matches.  With a tiny fix-up capacity the screen overflows its
    fix-up list, grows it and runs again with the same result."""
    import synth
    O = oracle_mod
    rng = np.random.default_rng(500 + seed)
    X = _degenerate_X(rng, p, n)
    y = X[0] * np.abs(X[1]) + 0.5 * np.exp(-X[0]) + 0.01 * rng.normal(size=n)
    if R == 3:
        sp = O.Space(p, 3, O.OPS, rung_ops=(None, None, None, synth.BINARY_OPS),
                     rung_pool=(None, None, None, 0))
        prm = D.params(rung=3, k=30, rung_ops=(None, None, None, synth.BINARY_OPS),
                       rung_pool=(None, None, None, 0))
    else:
        sp = O.Space(p, R, O.OPS)
        prm = D.params(rung=R, k=30)
    (lst,), status, nvalid = O.sis(sp, X, None, y[None], 30, (), "per_target", True)
    counts = status if len(status) == 5 else np.bincount(status, minlength=5)
    assert counts[O.ST_NONFINITE] > 0 and counts[O.ST_CONST] >= 0 and counts[O.ST_CHILD] > 0
    if fixcap:
        ctx.set_fixup_capacity(fixcap)
    try:
        ids, sc, vals, st = ctx.generate_screen(dev(torch, X), dev(torch, y[None]), prm)
    finally:
        if fixcap:
            ctx.set_fixup_capacity(1 << 22)
    check_selection(ids[0].cpu().numpy(), sc[0].cpu().numpy(), lst[0], lst[1],
                    what="degenerate seed %d" % seed)
    assert st["n_unit_valid"] == sp.N - int(counts[O.ST_UNIT])
    assert st["n_scored"] == nvalid, (st["n_scored"], nvalid)
    n_sel = int((ids[0] >= 0).sum())
    V, vst = O.values(sp, X, None, ids[0][:n_sel].cpu().numpy())
    assert bool((vst == 0).all())
    np.testing.assert_allclose(vals[0][:n_sel].cpu().numpy(), V, rtol=1e-10,
                               atol=1e-14 * float(np.max(np.abs(V))))


@pytest.mark.parametrize("seed,p,n,R,big", [(4, 7, 96, 3, 400.0), (5, 7, 75, 3, 1e7), (6, 6, 64, 2, 1e7)])
def test_screen_degenerate_inputs_bf16(torch, ctx, D, oracle_mod, seed, p, n, R, big):
    """The same degenerate primaries through the BF16 precision form: the
    rung-3 products on the matrix cores with their range checks (a column of
    magnitude 1e7 puts rung-3 values beyond the FP32 limits, which must go
    to the exact fix-up), the rung-2 BF16 pair tiles, and the exact rescore
    of the guard band reproduce the oracle's counts and selection."""
    import synth
    O = oracle_mod
    rng = np.random.default_rng(700 + seed)
    X = _degenerate_X(rng, p, n)
    X[3] = X[3] / 400.0 * big
    y = X[0] * np.abs(X[1]) + 0.5 * np.exp(-X[0]) + 0.01 * rng.normal(size=n)
    if R == 3:
        sp = O.Space(p, 3, O.OPS, rung_ops=(None, None, None, synth.BINARY_OPS),
                     rung_pool=(None, None, None, 0))
        prm = D.params(rung=3, k=30, rung_ops=(None, None, None, synth.BINARY_OPS),
                       rung_pool=(None, None, None, 0), precision=D.BF16_GUARD)
    else:
        sp = O.Space(p, R, O.OPS)
        prm = D.params(rung=R, k=30, precision=D.BF16_GUARD, lp_pairs=1)
    (lst,), status, nvalid = O.sis(sp, X, None, y[None], 30, (), "per_target", True)
    counts = status if len(status) == 5 else np.bincount(status, minlength=5)
    assert counts[O.ST_NONFINITE] > 0
    ids, sc, vals, st = ctx.generate_screen(dev(torch, X), dev(torch, y[None]), prm)
    check_selection(ids[0].cpu().numpy(), sc[0].cpu().numpy(), lst[0], lst[1],
                    what="degenerate bf16 seed %d" % seed)
    assert st["n_unit_valid"] == sp.N - int(counts[O.ST_UNIT])
    assert st["n_scored"] == nvalid, (st["n_scored"], nvalid)
    assert st["max_lowprec_err"] <= st["guard_band"]


def test_sisso_degenerate_inputs(torch, ctx, D, oracle_mod):
    """The whole loop (screen, L0 D <= 2, residuals) on the degenerate
    primaries, rung 2."""
    O = oracle_mod
    rng = np.random.default_rng(600)
    X = _degenerate_X(rng, 7, 90)
    y = 1.5 * X[0] * X[3] / 400.0 - 0.7 * np.exp(-X[0]) + 1e-3 * rng.normal(size=90)
    w = {"name": "degenerate", "X": X, "Y": y[None], "units": None, "p": 7, "n": 90, "T": 1,
         "B": 0, "ops": O.OPS, "rung": 2, "rung_ops": None, "rung_pool": None, "k": 15, "D": 2,
         "score_mode": "per_target", "n_resid": 1, "omp_D": 0}
    ref, got = run_both(torch, ctx, D, O, w)
    compare_sisso(ref, got, w, "degenerate")
