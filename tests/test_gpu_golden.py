"""Full-size parity against stored oracle references.

tests/golden/<workload>.json holds the oracle's whole SISSO run on a
workload (written once by oracle/make_golden.py, which calls nothing but
the oracle and the seeded input generators):

* units16: n = 500, p = 16 with exponent vectors over three base units,
  rung 2, top-500 per dimension, D <= 3, one residual; every L0 dimension
  of the reference was solved by Householder QR of every subset (5.6e8
  subsets at d = 3).
* large24: n = 2000, p = 24 with units, rung 2 plus an operator-limited
  rung 3 (702,860,274 raw candidates per dimension), top-1000 per
  dimension, 8 residual targets with the max score from d = 2, D <= 3, OMP
  to 6; L0 by QR of every subset for d <= 2 and in Gram mode for d = 3,
  checked by QR of the Gram band of the 64 best explained fractions and of
  200,000 random subsets (the check is stored with the reference).

The GPU runs the SISSO loop with the FP64 screening and with the BF16
precision form of the screening (L0 and OMP in FP64 in both); each must
reproduce the reference to the parity bar of tests/checks.py: the same
selected IDs in the same order, scores within 1e-10 relative, the same
models with RMSE and coefficients within 1e-10, the same OMP path.
"""
import hashlib
import json
import math
import os

import numpy as np
import pytest

import synth
from tests.checks import check_model, check_selection

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
CASES = [(name, prec) for name in ("units16", "large24") for prec in ("fp64", "bf16")
         if os.path.exists(os.path.join(GOLDEN, name + ".json"))]


def fingerprint(w):
    """SHA-256 of the generated inputs: the reference belongs to these."""
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(w["X"], np.float64).tobytes())
    h.update(np.ascontiguousarray(w["Y"], np.float64).tobytes())
    if w["units"] is not None:
        h.update(np.ascontiguousarray(w["units"], np.int32).tobytes())
    return h.hexdigest()


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


def test_references_present():
    assert [c[0] for c in CASES].count("units16") == 2, "tests/golden/units16.json is missing"


@pytest.mark.parametrize("name,prec", CASES)
def test_sisso_against_reference(torch, ctx, name, prec):
    import paper_2602_06986_amd as D
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        gold = json.load(f)
    w = synth.make(name)
    assert fingerprint(w) == gold["fingerprint"], "the generator no longer makes the reference's inputs"
    prm = D.params(ops=w["ops"], rung=w["rung"], k=w["k"], rung_ops=w.get("rung_ops"),
                   rung_pool=w.get("rung_pool"),
                   precision=D.FP64 if prec == "fp64" else D.BF16_GUARD)
    y = w["Y"][0]
    got = ctx.sisso(torch.as_tensor(w["X"], device="cuda"), torch.as_tensor(y, device="cuda"), prm,
                    w["D"], units=w["units"], n_resid=w["n_resid"], omp_D=w["omp_D"])
    S_g = got["S_ids"].cpu().numpy()
    assert [int(v) for v in S_g] == gold["S_ids"]
    for d, (gd, rd) in enumerate(zip(got["dims"], gold["dims"])):
        what = "%s %s dim %d" % (name, prec, d + 1)
        check_selection(gd["sel_ids"].cpu().numpy(), gd["sel_scores"].cpu().numpy(),
                        rd["sel_ids"], rd["sel_scores"], what=what)
        st = gd["screen_stats"]
        assert st["n_raw"] == gold["N"], what
        assert st["n_unit_valid"] == rd["n_unit_valid"], (what, st["n_unit_valid"], rd["n_unit_valid"])
        assert st["n_scored"] == rd["n_valid"], (what, st["n_scored"], rd["n_valid"])
        if prec == "bf16":
            assert st["max_lowprec_err"] <= st["guard_band"], what
        subs = gd["subsets"].cpu().numpy()
        assert len(rd["models"]) == w["n_resid"]
        for q, mo in enumerate(rd["models"]):
            check_model([int(S_g[i]) for i in subs[q][:d + 1]], float(gd["rmse"][q]),
                        gd["coef"][q].cpu().numpy(), mo, y, "%s model %d" % (what, q))
        assert gd["l0_stats"]["n_subsets"] == math.comb(len(S_g[:(d + 1) * w["k"]]), d + 1)
        if "gram_check" in rd:                   # how the Gram-mode reference was checked
            gc = rd["gram_check"]
            assert gc["top_models_agree"] and gc["band_min_rss"] >= gc["winner_rss"] * (1 - 1e-9)
    if name == "units16":
        assert got["dims"][0]["screen_stats"]["n_unit_valid"] == 336214
    if "omp" in gold:
        om = gold["omp"]
        act = got["omp"]["active"].cpu().numpy()
        assert [int(S_g[a]) for a in act] == om["ids"], (name, prec, "omp path")
        coef = got["omp"]["coef"].cpu().numpy()
        scale = np.max(np.abs(om["coef"]))
        assert np.max(np.abs(coef - np.array(om["coef"]))) <= 1e-10 * scale
        rmse = float(got["omp"]["rmse"].cpu().numpy().reshape(-1)[0])
        assert abs(rmse - om["rmse"]) <= 1e-10 * om["rmse"] + 1e-13 * np.std(y)


def _compare_dataset(name, gold, sel, models, counts, y):
    """sel[d] = (ids, scores); models[d][q] = (candidate IDs, rmse, coef with
    the intercept first and the rest in the models' row order)."""
    for d, rd in enumerate(gold["dims"]):
        what = "%s dim %d" % (name, d + 1)
        check_selection(sel[d][0], sel[d][1], rd["sel_ids"], rd["sel_scores"], what=what)
        if counts is not None:
            assert counts[d] == (rd["n_valid"], rd["n_unit_valid"]), (what, counts[d])
        for q, mo in enumerate(rd["models"]):
            ids_g, rmse_g, coef_g = models[d][q]
            check_model(ids_g, rmse_g, coef_g, mo, y, "%s model %d" % (what, q))


def test_batch128_against_reference(torch, ctx):
    """All 128 datasets of the batched workload (n ~ U{50..2000}, p ~
    U{6..20}, rung 2, top-200, D <= 3), through the batched per-dimension
    calls and through the captured loop (its first call eager, the second a
    graph replay), against the stored oracle reference of every dataset."""
    import paper_2602_06986_amd as D
    path = os.path.join(GOLDEN, "batch128.json")
    assert os.path.exists(path), "tests/golden/batch128.json is missing"
    with open(path) as f:
        gold = json.load(f)["datasets"]
    ws = synth.batch128()
    assert len(gold) == len(ws) == 128
    for w, g in zip(ws, gold):
        assert fingerprint(w) == g["fingerprint"], w["name"]
    Xs = [torch.as_tensor(w["X"], device="cuda") for w in ws]
    ys = [torch.as_tensor(w["Y"][0], device="cuda").contiguous() for w in ws]
    prm = D.params(ops=ws[0]["ops"], rung=2, k=ws[0]["k"])
    Dd = ws[0]["D"]
    loop = ctx.sisso_batch(Xs, ys, prm, Dd)
    for b, (w, g, r) in enumerate(zip(ws, gold, loop)):
        S = r["S_ids"].cpu().numpy()
        assert [int(v) for v in S] == g["S_ids"], w["name"]
        sel = [(dd["sel_ids"].cpu().numpy(), dd["sel_scores"].cpu().numpy()) for dd in r["dims"]]
        models = [[([int(S[i]) for i in dd["subsets"][q].cpu().numpy()], float(dd["rmse"][q]),
                    dd["coef"][q].cpu().numpy()) for q in range(len(dd["rmse"]))] for dd in r["dims"]]
        counts = [(dd["screen_stats"]["n_scored"], dd["screen_stats"]["n_unit_valid"]) for dd in r["dims"]]
        _compare_dataset(w["name"] + " (batched calls)", g, sel, models, counts, w["Y"][0])
    for call in range(2):
        ids, sc, sub, rmse, coef, rep = ctx.sisso_batch_graph(Xs, ys, prm, Dd, m=1)
        assert rep == (1 if call else 0), (call, rep)
        ids, sc, sub, rmse, coef = (t.cpu().numpy() for t in (ids, sc, sub, rmse, coef))
        for b, (w, g) in enumerate(zip(ws, gold)):
            S = ids[b].reshape(-1)
            sel = [(ids[b, d], sc[b, d]) for d in range(Dd)]
            models = [[([int(S[i]) for i in sub[b, d, 0, :d + 1]], float(rmse[b, d, 0]),
                        coef[b, d, 0, :d + 2])] for d in range(Dd)]
            _compare_dataset("%s (graph call %d)" % (w["name"], call), g, sel, models, None, w["Y"][0])
