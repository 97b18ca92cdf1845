"""run_discover end to end on the GPU: a configuration (data, unit strings,
search settings, rules) in, named expressions out.

* units16 given as a configuration whose features carry unit strings
  ("m^a kg^b s^c") reproduces the stored oracle reference of units16 (the
  same subspace, selections and models) — the configuration layer adds no
  arithmetic;
* rules written with feature names and a target unit string select what the
  oracle selects under the same rules;
* the omp and anneal methods return what the direct calls return on the
  same subspace;
* the command line reads a JSON file and writes the result file.
"""
import json
import os

import numpy as np
import pytest

import synth
from tests.checks import check_selection

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def unit_strings(units):
    return [" ".join("%s^%d" % (b, e) for b, e in zip(("m", "kg", "s"), row) if e) or "1" for row in units]


def test_units16_config_matches_reference(torch):
    from paper_2602_06986_amd.run import run_discover
    w = synth.make("units16")
    with open(os.path.join(GOLDEN, "units16.json")) as f:
        gold = json.load(f)
    names = ["f%d" % i for i in range(w["p"])]
    cfg = {"data": {"X": w["X"], "y": w["Y"][0], "features": names},
           "units": dict(zip(names, unit_strings(w["units"]))),
           "search": {"rung": w["rung"], "ops": list(w["ops"]), "k": w["k"], "D": w["D"],
                      "n_resid": w["n_resid"]}}
    out = run_discover(cfg)
    assert out["base_units"] == ["m", "kg", "s"]
    assert out["candidates_per_dimension"] == gold["N"]
    for d, (od, rd) in enumerate(zip(out["dimensions"], gold["dims"])):
        ids = [s["id"] for s in od["selected"]]
        sc = [s["score"] for s in od["selected"]]
        check_selection(np.array(ids), np.array(sc), rd["sel_ids"], rd["sel_scores"], what="dim %d" % (d + 1))
        assert od["screen"]["n_unit_valid"] == rd["n_unit_valid"]
        best, ref = od["models"][0], rd["models"][0]
        assert sorted(best["ids"]) == sorted(ref["ids"]), (d, best["ids"], ref["ids"])
        assert abs(best["rmse"] - ref["rmse"]) <= 1e-10 * ref["rmse"] + 1e-13 * np.std(w["Y"][0])
        for t in best["terms"]:
            assert "x" not in t.replace("exp", "")      # every primary carries its name
    # the planted three-term model is found at D = 3
    assert out["dimensions"][-1]["models"][0]["r2"] > 0.999


def test_rules_by_name(torch, oracle_mod):
    from paper_2602_06986_amd.run import run_discover
    O = oracle_mod
    rng = np.random.default_rng(810)
    p, n = 5, 120
    X = rng.lognormal(0, 0.4, size=(p, n))
    y = X[0] * X[1] / X[3] + 0.3 * X[2] + 0.02 * rng.normal(size=n)
    names = ["T", "P", "V", "rho", "c"]
    ustr = {"T": "K", "P": "Pa", "V": "m^3", "rho": "kg/m^3", "c": "1"}
    rules_cfg = {"max_complexity": 3, "forbid_pairs": [["T", "rho"]], "forbid_nest": {"exp": ["exp"]},
                 "target_unit": "J"}
    cfg = {"data": {"X": X, "y": y, "features": names}, "units": ustr,
           "search": {"rung": 2, "k": 25, "D": 1}, "rules": rules_cfg}
    out = run_discover(cfg)
    from paper_2602_06986_amd import units as U
    units, bases = U.exponent_matrix([ustr[f] for f in names])
    assert out["base_units"] == bases
    sp = O.Space(p, 2, O.OPS)
    tu = U.parse_unit("J")
    allowed = sp.rules_allowed(units, {"max_complexity": 3, "forbid_pairs": [[0, 3]],
                                       "forbid_nest": {"exp": ["exp"]},
                                       "target_units": [int(tu[U.BASE.index(b)]) for b in bases]})
    (lst,), _, _ = O.sis(sp, X, units, y[None], 25, (), "per_target", True, allowed=allowed)
    sel = out["dimensions"][0]["selected"]
    check_selection(np.array([s["id"] for s in sel]), np.array([s["score"] for s in sel]),
                    lst[0], lst[1], what="rules by name")
    assert len(sel) > 0
    for s in sel:
        assert "T" not in s["expression"] or "rho" not in s["expression"]


def test_methods_omp_and_anneal(torch):
    import paper_2602_06986_amd as D
    from paper_2602_06986_amd.run import run_discover
    rng = np.random.default_rng(811)
    p, n = 6, 300
    X = rng.lognormal(0, 0.4, size=(p, n))
    y = 1.5 * X[0] * X[1] - 0.7 * X[2] / X[4] + 0.4 * np.sqrt(X[5]) + 0.01 * rng.normal(size=n)
    base = {"data": {"X": X, "y": y}, "search": {"rung": 1, "k": 30, "D": 2}}
    omp = run_discover(dict(base, search=dict(base["search"], method="omp", omp_D=4)))
    ann = run_discover(dict(base, search=dict(base["search"], method="anneal",
                                              anneal={"D": 3, "chains": 512, "steps": 400, "seed": 5})))
    # the same subspace from the direct calls
    ctx = D.Context(0)
    try:
        prm = D.params(rung=1, k=30)
        Xd = torch.as_tensor(X, device="cuda")
        yd = torch.as_tensor(y, device="cuda")
        res = ctx.sisso(Xd, yd, prm, 2, omp_D=4)
        S = res["S_ids"].cpu().numpy()
        act = [int(a) for a in res["omp"]["active"].cpu().numpy()]
        assert omp["omp"]["ids"] == [int(S[a]) for a in act]
        assert abs(omp["omp"]["rmse"] - float(res["omp"]["rmse"].cpu()[0])) == 0.0
        rows, rmse, coef, en, *_ = ctx.anneal(res["F"], res["S_ids"], yd, 3, chains=512, steps=400, seed=5,
                                              T0=0.01, alpha=0.999)
        assert ann["anneal"]["ids"] == [int(S[r]) for r in rows.cpu().numpy()]
        assert ann["anneal"]["energy"] == float(en)
        assert ann["anneal"]["rmse"] <= omp["dimensions"][1]["models"][0]["rmse"] * (1 + 1e-12)
    finally:
        ctx.close()


def test_command_line(torch, tmp_path):
    from paper_2602_06986_amd.run import main
    rng = np.random.default_rng(812)
    X = rng.lognormal(0, 0.4, size=(4, 80))
    y = X[0] * X[2] + 0.01 * rng.normal(size=80)
    with open(tmp_path / "d.csv", "w") as f:
        f.write("a,b,c,d,y\n")
        for i in range(80):
            f.write(",".join(repr(float(v)) for v in list(X[:, i]) + [y[i]]) + "\n")
    cfg = {"data": {"file": "d.csv", "target": "y"}, "search": {"rung": 1, "k": 10, "D": 1},
           "output": "result.json"}
    (tmp_path / "c.json").write_text(json.dumps(cfg))
    assert main([str(tmp_path / "c.json")]) == 0
    with open(tmp_path / "result.json") as f:
        res = json.load(f)
    assert res["dimensions"][0]["models"][0]["terms"] == ["(a * c)"]
