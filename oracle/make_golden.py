"""Builds the stored oracle references under tests/golden/.

TEST INFRASTRUCTURE ONLY: this script calls nothing but the oracle (this
folder) and the seeded input generators (synth/); no value in its output
comes from the GPU library.  It runs for hours on a CPU and is run once;
the GPU parity tests and the benchmark's parity gate read its output.

    python oracle/make_golden.py units16|large24|batch128 [--threads N]

What each reference holds, per SISSO dimension d (Summary: SIS then the L0
problem of Eq. (1), Core Optimization Objective, on the union subspace):
the selected IDs and FP64 scores in (-score, ID) order, the number of
valid and of unit-valid candidates, and the best models of dimension d
(candidate IDs, RSS, RMSE, coefficients with the intercept first); then
the OMP extension of the final winner where the workload asks for it.

L0 is solved by Householder QR of every subset ("direct") wherever that is
affordable: every dimension of units16 (5.6e8 subsets at d = 3), and
d <= 2 elsewhere.  Where it is not (d = 3 of large24 and of the batch
datasets), the oracle's Gram mode is used and checked against direct QR
on (a) every subset of the Gram band of the 64 best explained fractions
and (b) a seeded random sample of subsets; the check is stored with the
reference.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
# run as a script, this folder comes first on the path and its oracle.py
# would shadow the package of the same name
sys.path[:] = [q for q in sys.path if os.path.abspath(q or ".") != HERE]
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import oracle as O  # noqa: E402

GOLDEN = os.path.join(ROOT, "tests", "golden")


def fingerprint(w):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(w["X"], np.float64).tobytes())
    h.update(np.ascontiguousarray(w["Y"], np.float64).tobytes())
    if w["units"] is not None:
        h.update(np.ascontiguousarray(w["units"], np.int32).tobytes())
    return h.hexdigest()


def model_rec(mo):
    return {"ids": [int(v) for v in mo["ids"]],
            "positions": [int(v) for v in mo["positions"]],
            "rss": float(mo["rss"]), "rmse": float(mo["rmse"]),
            "coef": [float(v) for v in mo["coef"]]}


def gram_check(F, ids, y, D, models, n_top=64, n_random=200000, seed=0):
    """Direct QR against the Gram-mode result: the band of the n_top best
    explained fractions and a random sample of subsets, each refitted by
    QR.  Returns a record; raises if QR finds a better model than the
    Gram-mode winner."""
    S = F.shape[0]
    yc = y - y.mean()
    yy = float(yc @ yc)
    Cm, c, _ = O.corr_matrix(F, y)
    cap = 1 << 16
    while True:
        band = np.empty((cap, D), np.int32)
        bq = np.empty(cap, np.float64)
        cnt = O.lib().or_l0_gram_band(S, O._p(Cm), O._p(c), D, O.PIV_TOL, n_top, 0.0,
                                      cap, O._p(band), O._p(bq))
        if cnt <= cap:
            break
        cap = int(cnt)
    if cnt <= 0:
        raise AssertionError("no non-singular subset in the Gram band (code %d)" % cnt)
    band = band[:cnt]
    rss_band = O.subset_rss(F, y, band)
    rng = np.random.default_rng(seed)
    R = np.sort(rng.integers(0, S, size=(n_random, D)), axis=1)
    R = R[np.all(np.diff(R, axis=1) > 0, axis=1)] if D > 1 else R
    rss_rand = O.subset_rss(F, y, R)
    best = models[0]["rss"]
    tol = O.TAU_TIE * yy
    fb = rss_band[~np.isnan(rss_band)]
    fr = rss_rand[~np.isnan(rss_rand)]
    # the winner by QR over the checked band, with the tie rule
    cands = [(float(r), tuple(sorted(int(ids[i]) for i in sub)), tuple(int(v) for v in sub))
             for r, sub in zip(rss_band, band) if not np.isnan(r)]
    top = O._rank_models(cands, len(models), yy)
    agree = [list(t[1]) for t in top] == [sorted(m["ids"]) for m in models]
    if len(fb) and fb.min() < best - tol:
        raise AssertionError("direct QR beats the Gram-mode winner in the band")
    if len(fr) and fr.min() < best - tol:
        raise AssertionError("direct QR beats the Gram-mode winner in the sample")
    return {"band_subsets": int(cnt), "band_min_rss": float(fb.min()) if len(fb) else None,
            "random_subsets": int(len(R)), "random_min_rss": float(fr.min()) if len(fr) else None,
            "winner_rss": float(best), "top_models_agree": bool(agree)}


def sisso_record(w, l0_modes, check_gram=None):
    """The oracle's SISSO loop on one workload, dimension by dimension."""
    space = O.Space.of(w)
    X, units = w["X"], w["units"]
    y = w["Y"][0]
    k, D, m = w["k"], w["D"], w["n_resid"]
    S_ids = np.zeros(0, np.int64)
    F = np.zeros((0, w["n"]))
    targets = y[None, :]
    dims = []
    for d in range(1, D + 1):
        t0 = time.time()
        mode = "max" if targets.shape[0] > 1 or w["score_mode"] == "max" else "per_target"
        out, status, nvalid = O.sis(space, X, units, targets, k, S_ids, mode, True)
        counts = status if len(status) == 5 else np.bincount(status, minlength=5)[:5]
        sel_ids, sel_sc, rec = out[0]
        V, _ = O.values(space, X, units, sel_ids)
        S_ids = np.concatenate([S_ids, sel_ids])
        F = np.vstack([F, V])
        t1 = time.time()
        models = O.l0(F, S_ids, y, d, m, l0_modes[d - 1])
        t2 = time.time()
        rec_d = {"d": d, "T": int(targets.shape[0]), "score_mode": mode,
                 "sel_ids": [int(v) for v in sel_ids], "sel_scores": [float(v) for v in sel_sc],
                 "n_valid": int(nvalid), "n_unit_valid": int(space.N - counts[O.ST_UNIT]),
                 "groups": rec["groups"], "merged": rec["merged"],
                 "l0_mode": l0_modes[d - 1], "models": [model_rec(mo) for mo in models],
                 "seconds_screen": round(t1 - t0, 1), "seconds_l0": round(t2 - t1, 1)}
        if l0_modes[d - 1] == "gram" and check_gram:
            rec_d["gram_check"] = gram_check(F, S_ids, y, d, [model_rec(mo) for mo in models],
                                             **check_gram)
        print("  d=%d: screen %.0f s, L0 (%s) %.0f s, winner %s rmse %.6g" %
              (d, t1 - t0, l0_modes[d - 1], t2 - t1, models[0]["ids"], models[0]["rmse"]),
              flush=True)
        dims.append(rec_d)
        targets = np.array([mo["resid"] for mo in models])
    res = {"workload": w["name"], "fingerprint": fingerprint(w), "N": int(space.N),
           "dims": dims, "S_ids": [int(v) for v in S_ids]}
    if w.get("omp_D", 0) > D:
        act, coef, rmse, _ = O.omp(F, S_ids, y, w["omp_D"], dims[-1]["models"][0]["positions"])
        res["omp"] = {"positions": [int(a) for a in act], "ids": [int(S_ids[a]) for a in act],
                      "coef": [float(v) for v in coef], "rmse": float(rmse)}
    return res


def write(name, obj):
    os.makedirs(GOLDEN, exist_ok=True)
    path = os.path.join(GOLDEN, name)
    with open(path + ".tmp", "w") as f:
        json.dump(obj, f, separators=(",", ":"))
    os.replace(path + ".tmp", path)
    print("wrote", path, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["units16", "large24", "batch128"])
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--first", type=int, default=0, help="batch128: first dataset")
    ap.add_argument("--count", type=int, default=128, help="batch128: datasets")
    a = ap.parse_args()
    O.build()
    if a.threads:
        O.lib().or_set_threads(a.threads)
    t0 = time.time()
    if a.which == "units16":
        w = synth.units16()
        res = sisso_record(w, ["direct", "direct", "direct"])
        res["note"] = "every L0 dimension by Householder QR of every subset"
        write("units16.json", res)
    elif a.which == "large24":
        w = synth.large24()
        res = sisso_record(w, ["direct", "direct", "gram"],
                           check_gram={"n_top": 64, "n_random": 200000, "seed": 5})
        res["note"] = ("d <= 2 by QR of every subset; d = 3 in Gram mode, checked by QR of the "
                       "band of the 64 best explained fractions and of 200,000 random subsets")
        write("large24.json", res)
    else:
        ws = synth.batch128()
        out = []
        path = os.path.join(GOLDEN, "batch128.json")
        if os.path.exists(path) and a.first:
            out = json.load(open(path))["datasets"][:a.first]
        for b in range(a.first, min(128, a.first + a.count)):
            w = ws[b]
            print("dataset %d: n=%d p=%d" % (b, w["n"], w["p"]), flush=True)
            out.append(sisso_record(w, ["direct", "direct", "gram"],
                                    check_gram={"n_top": 64, "n_random": 20000, "seed": b}))
            write("batch128.json", {"datasets": out,
                                    "note": "d <= 2 by QR of every subset; d = 3 in Gram mode, "
                                            "checked by QR of the band of the 64 best explained "
                                            "fractions and of 20,000 random subsets"})
    print("total %.0f s" % (time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
