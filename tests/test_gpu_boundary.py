"""The asynchronous and captured forms of the three calls, through the C ABI.

With stats in device memory a call does not wait for the stream and
reports its outcome (stats.status) on the device.  Made on a stream the
caller is capturing (torch.cuda.graph, relaxed mode) the call is recorded
into the caller's graph; every replay recomputes from the inputs' current
contents.  Each form runs the same kernels on the same data as the eager
call, so the outputs must be bit-identical to it; the eager call itself is
anchored to the oracle in the parity tests, and once more here.

Between replays the program does eager work of its own and synchronises,
and every replay is checked, not only the last.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

E_ARG, E_NUMERIC, E_CAPACITY = -1, -5, -6


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


@pytest.fixture(scope="module")
def D():
    import paper_2602_06986_amd as D
    return D


@pytest.fixture
def fresh(D):
    """A context of its own: a capture pins the workspace of its context."""
    made = []

    def make():
        c = D.Context(0)
        made.append(c)
        return c
    yield make
    for c in made:
        c.close()


def dev(torch, a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def same(a, b, what):
    """Bit-identical tensors (NaN where NaN)."""
    x = a.detach().cpu().numpy()
    z = b.detach().cpu().numpy()
    assert x.shape == z.shape, (what, x.shape, z.shape)
    assert np.array_equal(x, z, equal_nan=x.dtype.kind == "f"), what


def capture(torch, fn):
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, capture_error_mode="relaxed"):
        out = fn()
    return g, out


def units16_inputs(torch, D, k=120, precision=None, seed=None):
    w = synth.units16()
    y = w["Y"][0]
    if seed is not None:                       # the same form, another noise draw
        rng = np.random.default_rng(seed)
        y = y + 0.01 * np.std(y) * rng.normal(size=y.shape)
    prm = D.params(ops=w["ops"], rung=2, k=k, precision=D.FP64 if precision is None else precision)
    return w, dev(torch, w["X"]), dev(torch, y[None]), w["units"], prm


# tile_j is a timed choice of the context, not a result: compared only
# within one context
SCREEN_FIELDS = ("n_raw", "n_unit_valid", "n_scored", "n_merged", "n_selected", "max_lowprec_err",
                 "guard_band")


@pytest.mark.parametrize("prec", ["fp64", "bf16"])
def test_screen_device_stats_equal_host(torch, D, fresh, prec):
    """A first device-stats call (which settles the sizes, waiting once) and
    a second one (which does not wait) both equal the host-stats call."""
    w, X, Y, u, prm = units16_inputs(torch, D, precision=D.FP64 if prec == "fp64" else D.BF16_GUARD)
    ctx = fresh()
    first = ctx.generate_screen(X, Y, prm, units=u, device_stats=True)
    ref = fresh().generate_screen(X, Y, prm, units=u)
    again = ctx.generate_screen(X, Y, prm, units=u, device_stats=True)
    torch.cuda.synchronize()
    for got, what in ((first, "first"), (again, "async")):
        same(got[0], ref[0], what + " ids")
        same(got[1], ref[1], what + " scores")
        same(got[2], ref[2], what + " values")
        s = D.decode_stats(got[3], D.ScreenStats)[0]
        assert s["status"] == 0, (what, s)
        for f in SCREEN_FIELDS:
            assert s[f] == ref[3][f], (what, f, s[f], ref[3][f])
        if ref[3]["pool_rounds"] == 0:
            assert s["pool_size"] == ref[3]["pool_size"], what


def test_screen_device_stats_batch(torch, D, fresh):
    """Several problems of uneven shapes, two targets each (per-target
    lists): every problem's device stats and outputs equal the host call."""
    rng = np.random.default_rng(7)
    Xs, Ys = [], []
    for b, (p, n) in enumerate([(6, 80), (9, 200), (5, 61)]):
        X = rng.uniform(0.5, 2.0, size=(p, n))
        Y = np.vstack([X[0] * X[1] + 0.01 * rng.normal(size=n), np.exp(-X[2]) + 0.01 * rng.normal(size=n)])
        Xs.append(dev(torch, X))
        Ys.append(dev(torch, Y))
    prm = D.params(rung=2, k=25)
    ref = fresh().generate_screen_batch(Xs, Ys, prm)
    ctx = fresh()
    own = ctx.generate_screen_batch(Xs, Ys, prm)            # settles the sizes
    got = ctx.generate_screen_batch(Xs, Ys, prm, device_stats=True)
    torch.cuda.synchronize()
    st = D.decode_stats(got[0][3], D.ScreenStats)
    assert len(st) == 3
    for b in range(3):
        same(got[b][0], ref[b][0], "ids %d" % b)
        same(got[b][1], ref[b][1], "scores %d" % b)
        same(got[b][2], ref[b][2], "values %d" % b)
        assert st[b]["status"] == 0
        for f in SCREEN_FIELDS:
            assert st[b][f] == ref[b][3][f], (b, f)
        assert st[b]["tile_j"] == own[b][3]["tile_j"]


def test_l0_device_stats_equal_host(torch, D, fresh):
    w, X, Y, u, prm = units16_inputs(torch, D)
    ctx = fresh()
    ids, sc, V, _ = ctx.generate_screen(X, Y, prm, units=u)
    F, I, y = V[0], ids[0], Y[0]
    ref = ctx.l0_fit(F, I, y, 2, m=4)
    got = ctx.l0_fit(F, I, y, 2, m=4, device_stats=True)
    torch.cuda.synchronize()
    for i, what in enumerate(("subsets", "rmse", "coef", "resid")):
        same(got[i], ref[i], what)
    s = D.decode_stats(got[4], D.L0Stats)[0]
    assert s["status"] == 0
    assert s["n_subsets"] == ref[4]["n_subsets"] and s["n_band"] == ref[4]["n_band"]


def _chain(torch, D, ctx, X, Y, u, prm, ds):
    """Screen -> L0 (D = 1) -> screen of the residuals (MAX score, first
    selection excluded) -> L0 (D = 2) over both selections -> OMP to 4 rows:
    one SISSO-style sequence with its glue in torch."""
    prm_max = D.params(ops=synth.ALL_OPS, rung=2, k=prm.k, score_mode=D.SCORE_MAX)
    ids1, sc1, V1, st1 = ctx.generate_screen(X, Y, prm, units=u, device_stats=ds)
    sub1, rmse1, coef1, res1, l1 = ctx.l0_fit(V1[0], ids1[0], Y[0], 1, m=2, device_stats=ds)
    ids2, sc2, V2, st2 = ctx.generate_screen(X, res1, prm_max, units=u, exclude=ids1[0], device_stats=ds)
    F = torch.cat([V1[0], V2[0]])
    I = torch.cat([ids1[0], ids2[0]])
    sub2, rmse2, coef2, res2, l2 = ctx.l0_fit(F, I, Y[0], 2, m=2, device_stats=ds)
    act, ocoef, ormse, ores = ctx.omp(F, I, Y[0], 4, init=sub2[0])
    outs = [ids1, sc1, V1, sub1, rmse1, coef1, res1, ids2, sc2, V2, sub2, rmse2, coef2, res2,
            act, ocoef, ormse, ores]
    return outs, [st1, st2], [l1, l2]


def _check_chain(D, got, ref, what):
    names = ["ids1", "sc1", "V1", "sub1", "rmse1", "coef1", "res1", "ids2", "sc2", "V2", "sub2",
             "rmse2", "coef2", "res2", "omp_act", "omp_coef", "omp_rmse", "omp_res"]
    for a, b, nm in zip(got[0], ref[0], names):
        same(a, b, "%s %s" % (what, nm))
    for t in got[1]:
        assert D.decode_stats(t, D.ScreenStats)[0]["status"] == 0, what
    for t in got[2]:
        assert D.decode_stats(t, D.L0Stats)[0]["status"] == 0, what


def test_capture_sisso_chain(torch, D, fresh, oracle_mod):
    """The whole sequence captured into one caller graph, replayed three
    times with eager work between, then once more after the target changed
    in place: each replay equals the eager sequence on the current data."""
    O = oracle_mod
    w, X, Y, u, prm = units16_inputs(torch, D)
    _, _, Y2, _, _ = units16_inputs(torch, D, seed=11)
    ctx = fresh()
    ref = _chain(torch, D, ctx, X, Y, u, prm, False)          # settles every size
    torch.cuda.synchronize()
    # the eager sequence against the oracle's first selection
    sp = O.Space.of(w)
    (lst,), _, _ = O.sis(sp, w["X"], w["units"], w["Y"][:1], prm.k, (), "per_target", True)
    assert [int(v) for v in ref[0][0][0].cpu().numpy()] == [int(v) for v in lst[0]]
    Yc = Y.clone()
    g, got = capture(torch, lambda: _chain(torch, D, ctx, X, Yc, u, prm, True))
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        _check_chain(D, got, ref, "replay %d" % rep)
        junk = torch.randn(1 << 16, device="cuda", dtype=torch.float64)   # eager work between replays
        assert float((junk * junk).sum().item()) > 0
    ref2 = _chain(torch, D, fresh(), X, Y2, u, prm, False)
    Yc.copy_(Y2)
    g.replay()
    torch.cuda.synchronize()
    _check_chain(D, got, ref2, "replay on new target")


def test_reserve_then_capture(torch, D, fresh):
    """discover_reserve alone sizes a context for a captured screen, L0 and
    OMP: no eager call of the shape runs before the capture."""
    w, X, Y, u, prm = units16_inputs(torch, D)

    def seq(ctx, ds):
        ids, sc, V, st = ctx.generate_screen(X, Y, prm, units=u, device_stats=ds)
        sub, rmse, coef, res, l0 = ctx.l0_fit(V[0], ids[0], Y[0], 1, m=2, device_stats=ds)
        act, ocoef, ormse, ores = ctx.omp(V[0], ids[0], Y[0], 4, init=sub[0])
        return [ids, sc, V, sub, rmse, coef, res, act, ocoef, ormse, ores], st, l0

    ref, _, _ = seq(fresh(), False)
    ctx = fresh()
    ctx.reserve([X], [Y], prm, D_max=1, m=2, units=[u])
    g, (got, st, l0) = capture(torch, lambda: seq(ctx, True))
    for rep in range(2):
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(got, ref):
            same(a, b, "reserved replay %d" % rep)
        assert D.decode_stats(st, D.ScreenStats)[0]["status"] == 0
        assert D.decode_stats(l0, D.L0Stats)[0]["status"] == 0


def test_capture_refusals(torch, D, fresh):
    """A captured call needs device stats (E_ARG) and a shape that ran, or
    was reserved, outside capture (E_CAPACITY); after a capture the
    context's referenced workspace cannot grow (E_CAPACITY), and the graph
    still replays correctly."""
    w, X, Y, u, prm = units16_inputs(torch, D, k=60)
    ctx = fresh()
    with pytest.raises(D.DiscoverError) as e:
        capture(torch, lambda: ctx.generate_screen(X, Y, prm, units=u, device_stats=True))
    assert e.value.code == E_CAPACITY
    ref = ctx.generate_screen(X, Y, prm, units=u)
    with pytest.raises(D.DiscoverError) as e:
        capture(torch, lambda: ctx.generate_screen(X, Y, prm, units=u))
    assert e.value.code == E_ARG
    g, got = capture(torch, lambda: ctx.generate_screen(X, Y, prm, units=u, device_stats=True))
    # a larger problem would need a larger screening arena than the graph's
    rng = np.random.default_rng(3)
    Xb = dev(torch, rng.lognormal(0, 0.5, size=(16, 4000)))
    Yb = dev(torch, rng.normal(size=(1, 4000)))
    with pytest.raises(D.DiscoverError) as e:
        ctx.generate_screen(Xb, Yb, prm, units=u)
    assert e.value.code == E_CAPACITY and "captured" in str(e.value)
    g.replay()
    torch.cuda.synchronize()
    for i in range(3):
        same(got[i], ref[i], "replay after refusal")
    assert D.decode_stats(got[3], D.ScreenStats)[0]["status"] == 0


def _offset_inputs(rng, p=7, n=130):
    """Primaries far from zero relative to their spread: the one-pass moments
    of many candidates are not trusted and go to the exact fix-up list."""
    X = rng.lognormal(0, 0.5, size=(p, n))
    X[4] = 1000.0 + rng.uniform(0.0, 1.0, size=n)
    X[5] = 3000.0 + rng.uniform(0.0, 1.0, size=n)
    y = X[0] * X[1] + (X[4] - 1000.5) + 0.01 * rng.normal(size=n)
    return X, y


def test_device_status_capacity(torch, D, fresh):
    """A fix-up list too small for the data: the asynchronous call reports
    E_CAPACITY in its device stats; the host-stats call grows the list and
    returns the same selection as a context that never overflowed."""
    rng = np.random.default_rng(41)
    X, y = _offset_inputs(rng)
    Xd, Yd = dev(torch, X), dev(torch, y[None])
    prm = D.params(rung=2, k=30)
    ref = fresh().generate_screen(Xd, Yd, prm)
    ctx = fresh()
    ctx.generate_screen(Xd, Yd, prm)
    ctx.set_fixup_capacity(1)
    got = ctx.generate_screen(Xd, Yd, prm, device_stats=True)
    torch.cuda.synchronize()
    s = D.decode_stats(got[3], D.ScreenStats)[0]
    assert s["status"] == E_CAPACITY, s
    again = ctx.generate_screen(Xd, Yd, prm)
    same(again[0], ref[0], "ids after regrow")
    same(again[1], ref[1], "scores after regrow")
    assert again[3]["status"] == 0


def test_device_status_numeric(torch, D, fresh):
    """L0 over identical rows (no non-singular pair): the host call fails
    with E_NUMERIC, the asynchronous call reports it in its device stats."""
    rng = np.random.default_rng(42)
    n, S = 40, 12
    row = rng.normal(size=n)
    F = dev(torch, np.tile(row, (S, 1)))
    ids = dev(torch, np.arange(S), torch.int64)
    y = dev(torch, row + rng.normal(size=n))
    ctx = fresh()
    with pytest.raises(D.DiscoverError) as e:
        ctx.l0_fit(F, ids, y, 2)
    assert e.value.code == E_NUMERIC
    got = ctx.l0_fit(F, ids, y, 2, device_stats=True)
    torch.cuda.synchronize()
    assert D.decode_stats(got[4], D.L0Stats)[0]["status"] == E_NUMERIC
