"""run_discover: the method end to end from a configuration (the user-facing
layer the paper describes: a configuration file names the data, the
features' physical units, the operator library and the search settings;
Statement of Need, Physics-Informed Constraints).

    python -m paper_2602_06986_amd.run config.json      (or .yaml)

Configuration keys (JSON or YAML):

    data:      {file: path.csv | path.npz, target: name, features: [names]}
               or {X: [[...] per feature], y: [...], features: [names]}
               CSV: a header row of column names; npz: arrays X [p][n] (or
               [n][p] with transpose: true), y [n], names (optional)
    units:     {feature: "unit string"}      (physical units, optional)
    search:    rung (0..3), ops [names], rung_ops {r: [names]},
               rung_pool {r: partner rung}, k, D, n_resid (residuals carried
               to the next dimension), score_mode (per_target | max),
               precision (fp64 | bf16 | fp16), omp_D (0: no OMP extension),
               method (l0 | omp | anneal), anneal {D, chains, steps, T0,
               alpha, seed}
    rules:     {max_complexity, forbid_nest {op: [ops]}, forbid_pairs
               [[feature, feature], ...], target_unit "unit string"}
    output:    path of a JSON result file (optional)

Every step of the search runs in the GPU library; this module parses, moves
data to the device, calls the C ABI and turns candidate IDs into
expressions with the features' names.
"""
import json
import os
import re
import sys

import numpy as np

from . import units as U

OP_NAMES = ("add", "sub", "mul", "div", "rdiv", "exp", "log", "sqrt", "sq", "inv")


class ConfigError(ValueError):
    pass


def load_config(cfg):
    """A configuration dict, or the path of a JSON or YAML file."""
    if isinstance(cfg, dict):
        return dict(cfg), None
    path = str(cfg)
    with open(path) as f:
        text = f.read()
    if path.endswith((".yaml", ".yml")):
        import yaml
        out = yaml.safe_load(text)
    else:
        out = json.loads(text)
    if not isinstance(out, dict):
        raise ConfigError("the configuration must be a mapping")
    return out, os.path.dirname(os.path.abspath(path))


def load_data(data, base_dir=None):
    """(X [p][n], y [n], feature names)."""
    if data is None:
        raise ConfigError("data: missing")
    if "X" in data:
        X = np.asarray(data["X"], np.float64)
        y = np.asarray(data["y"], np.float64)
        names = list(data.get("features") or ["x%d" % i for i in range(X.shape[0])])
    else:
        path = data.get("file")
        if not path:
            raise ConfigError("data: give X and y, or file")
        if base_dir and not os.path.isabs(path):
            path = os.path.join(base_dir, path)
        if path.endswith(".npz"):
            z = np.load(path, allow_pickle=False)
            X = np.asarray(z["X"], np.float64)
            if data.get("transpose"):
                X = X.T
            y = np.asarray(z["y"], np.float64)
            names = [str(s) for s in z["names"]] if "names" in z else ["x%d" % i for i in range(X.shape[0])]
        else:
            with open(path) as f:
                header = [h.strip() for h in f.readline().strip().split(",")]
            M = np.loadtxt(path, delimiter=",", skiprows=1, ndmin=2)
            target = data.get("target")
            if target not in header:
                raise ConfigError("data: target %r is not a column of %s" % (target, path))
            feats = data.get("features") or [h for h in header if h != target]
            X = np.stack([M[:, header.index(h)] for h in feats])
            y = M[:, header.index(target)]
            names = list(feats)
        if data.get("features") and len(data["features"]) == X.shape[0]:
            names = list(data["features"])
    if X.ndim != 2 or y.ndim != 1 or X.shape[1] != y.shape[0]:
        raise ConfigError("data: X must be [features][samples] and y [samples]")
    if len(names) != X.shape[0]:
        raise ConfigError("data: %d names for %d features" % (len(names), X.shape[0]))
    return X, y, names


def _ops(names, where):
    out = []
    for o in names:
        if o not in OP_NAMES:
            raise ConfigError("%s: unknown operator %r (known: %s)" % (where, o, ", ".join(OP_NAMES)))
        out.append(o)
    return tuple(out)


def resolve_rules(rules, names, unit_names):
    """The configuration's rules in the library's form: feature names of
    forbidden pairs become primary indices, a target unit string becomes
    exponents over the base units the features use (unit_names)."""
    if not rules:
        return None
    known = {"max_complexity", "forbid_nest", "forbid_pairs", "target_unit"}
    extra = set(rules) - known
    if extra:
        raise ConfigError("rules: unknown keys %s (known: %s)" % (sorted(extra), sorted(known)))
    out = {"max_complexity": int(rules.get("max_complexity", -1))}
    if out["max_complexity"] < -1:
        raise ConfigError("rules.max_complexity: -1 (none) or >= 0")
    nest = {}
    for o, cs in (rules.get("forbid_nest") or {}).items():
        _ops([o], "rules.forbid_nest")
        nest[o] = list(_ops(cs, "rules.forbid_nest[%s]" % o))
    out["forbid_nest"] = nest
    pairs = []
    for pr in rules.get("forbid_pairs") or ():
        if len(pr) != 2:
            raise ConfigError("rules.forbid_pairs: pairs of feature names")
        ij = []
        for f in pr:
            if f not in names:
                raise ConfigError("rules.forbid_pairs: %r is not a feature" % (f,))
            i = names.index(f)
            if i >= 64:
                raise ConfigError("rules.forbid_pairs: only the first 64 features can be named")
            ij.append(i)
        pairs.append(ij)
    out["forbid_pairs"] = pairs
    tu = rules.get("target_unit")
    if tu is not None:
        v = U.parse_unit(tu)
        used = [U.BASE.index(b) for b in unit_names]
        if any(v[b] != 0 for b in range(len(U.BASE)) if b not in used):
            raise ConfigError("rules.target_unit %r needs a base unit no feature has" % (tu,))
        # without units every expression is dimensionless and the filter passes
        out["target_units"] = [int(v[b]) for b in used] if used else None
    return out


def expression(text, names):
    """Replace the library's x<i> operand names by the features' names."""
    return re.sub(r"\bx(\d+)\b", lambda m: names[int(m.group(1))], text)


def run_discover(cfg, device=0, verbose=False):
    """Run the configured search; returns a result dict (also written to
    `output` when given)."""
    import torch
    from . import Context, params, decode, count, SCORE_MAX, SCORE_PER_TARGET, FP64, BF16_GUARD, \
        FP16_GUARD
    cfg, base_dir = load_config(cfg)
    X, y, names = load_data(cfg.get("data"), base_dir)
    p, n = X.shape
    search = dict(cfg.get("search") or {})
    rung = int(search.get("rung", 1))
    ops = _ops(search.get("ops", OP_NAMES), "search.ops")
    rung_ops = [None] * 4
    for r, v in (search.get("rung_ops") or {}).items():
        rung_ops[int(r)] = _ops(v, "search.rung_ops[%s]" % r)
    rung_pool = [None] * 4
    for r, v in (search.get("rung_pool") or {}).items():
        rung_pool[int(r)] = int(v)
    k = int(search.get("k", 20))
    D = int(search.get("D", 2))
    n_resid = int(search.get("n_resid", 1))
    omp_D = int(search.get("omp_D", 0))
    method = search.get("method", "l0")
    if method not in ("l0", "omp", "anneal"):
        raise ConfigError("search.method: l0, omp or anneal")
    prec = {"fp64": FP64, "bf16": BF16_GUARD, "fp16": FP16_GUARD}.get(search.get("precision", "fp64"))
    if prec is None:
        raise ConfigError("search.precision: fp64, bf16 or fp16")
    mode = search.get("score_mode", "per_target")
    if mode not in ("per_target", "max"):
        raise ConfigError("search.score_mode: per_target or max")
    units = None
    unit_names = []
    ucfg = cfg.get("units") or {}
    if ucfg:
        missing = [f for f in names if f not in ucfg]
        if missing:
            raise ConfigError("units: no unit for %s" % ", ".join(missing))
        units, unit_names = U.exponent_matrix([ucfg[f] for f in names])
        if units is not None and units.shape[1] > 8:
            raise ConfigError("units: more than 8 base units")
    rules = resolve_rules(cfg.get("rules"), names, unit_names)
    if method == "omp" and omp_D <= D:
        raise ConfigError("search.method omp: omp_D must exceed D")
    prm = params(ops=ops, rung=rung, k=k, rung_ops=rung_ops, rung_pool=rung_pool,
                 score_mode=SCORE_MAX if mode == "max" else SCORE_PER_TARGET, precision=prec)
    ctx = Context(device)
    dev = torch.device("cuda", device)
    Xd = torch.as_tensor(np.ascontiguousarray(X), device=dev)
    yd = torch.as_tensor(np.ascontiguousarray(y), device=dev)
    try:
        ctx.set_rules(rules)
        res = ctx.sisso(Xd, yd, prm, D, units=units, n_resid=n_resid, omp_D=omp_D)
        S_ids = res["S_ids"].cpu().numpy()

        def expr(cid):
            return expression(decode(p, prm, int(cid)), names)
        out = {"n_samples": int(n), "features": names, "base_units": unit_names,
               "candidates_per_dimension": int(count(p, prm)), "dimensions": []}
        yc = y - y.mean()
        yy = float(yc @ yc)
        for d, dim in enumerate(res["dims"]):
            sel = dim["sel_ids"].cpu().numpy()
            sc = dim["sel_scores"].cpu().numpy()
            models = []
            for q in range(len(dim["rmse"])):
                rows = [int(r) for r in dim["subsets"][q].cpu().numpy()[:d + 1]]
                coef = dim["coef"][q].cpu().numpy()
                rmse = float(dim["rmse"][q])
                models.append({"ids": [int(S_ids[r]) for r in rows],
                               "terms": [expr(S_ids[r]) for r in rows],
                               "intercept": float(coef[0]), "coefficients": [float(c) for c in coef[1:d + 2]],
                               "rmse": rmse, "r2": 1.0 - rmse * rmse * n / yy})
            out["dimensions"].append({
                "d": d + 1, "selected": [{"id": int(i), "expression": expr(i), "score": float(s)}
                                         for i, s in zip(sel, sc) if i >= 0],
                "screen": {kk: v for kk, v in dim["screen_stats"].items()},
                "models": models})
        if "omp" in res:
            act = [int(a) for a in res["omp"]["active"].cpu().numpy() if a >= 0]
            coef = res["omp"]["coef"].cpu().numpy()
            out["omp"] = {"terms": [expr(S_ids[a]) for a in act], "ids": [int(S_ids[a]) for a in act],
                          "intercept": float(coef[0]), "coefficients": [float(c) for c in coef[1:len(act) + 1]],
                          "rmse": float(res["omp"]["rmse"].cpu().numpy().reshape(-1)[0])}
        if method == "anneal":
            a = dict(search.get("anneal") or {})
            Da = int(a.get("D", D + 1))
            F = res["F"]
            rows, rmse, coef, en, *_ = ctx.anneal(F, res["S_ids"], yd, Da, chains=int(a.get("chains", 4096)),
                                                  steps=int(a.get("steps", 5000)), T0=float(a.get("T0", 0.01)),
                                                  alpha=float(a.get("alpha", 0.999)),
                                                  seed=int(a.get("seed", 0)))
            rows = [int(r) for r in rows.cpu().numpy()]
            coef = coef.cpu().numpy()
            out["anneal"] = {"D": Da, "terms": [expr(S_ids[r]) for r in rows], "ids": [int(S_ids[r]) for r in rows],
                             "intercept": float(coef[0]), "coefficients": [float(c) for c in coef[1:]],
                             "rmse": float(rmse), "energy": float(en)}
    finally:
        ctx.close()
    if cfg.get("output"):
        path = cfg["output"]
        if base_dir and not os.path.isabs(path):
            path = os.path.join(base_dir, path)
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
    if verbose:
        best = out["dimensions"][-1]["models"][0]
        print("best %d-term model: y = %.6g %s   (rmse %.6g)" % (
            len(best["terms"]), best["intercept"],
            " ".join("%+.6g*%s" % (c, t) for c, t in zip(best["coefficients"], best["terms"])), best["rmse"]))
    return out


def main(argv=None):
    argv = sys.argv[1:] if argv is None else argv
    if len(argv) != 1:
        print("usage: python -m paper_2602_06986_amd.run config.json|config.yaml", file=sys.stderr)
        return 2
    run_discover(argv[0], verbose=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
