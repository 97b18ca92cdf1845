"""Seeded synthetic workloads shaped like the method's use cases.

This module only draws numbers: primary-feature matrices, unit-exponent
tables and planted targets.  It holds none of the screening or fitting
arithmetic (no candidate enumeration, no correlation, no least squares); both
the FP64 oracle and the GPU path read the same arrays from here.

The paper (Software Description; Physics-Informed Constraints) describes
SISSO-style descriptor search over candidate expressions of primary features
with physical units.  It ships no data, so each workload below is a recipe:
distribution, size, unit table and a planted descriptor whose terms are
themselves reachable candidate expressions.

Array conventions (shared by every consumer):
  X      float64 [p, n]   feature-major, X[f, s]
  Y      float64 [T, n]   target-major,  Y[t, s]
  units  int32   [p, B]   integer exponents over B base units, or None
"""
from __future__ import annotations

import numpy as np

# Operator library order.  Unary operators first, then binary ones; the
# enumeration order of candidates follows this list.
UNARY_OPS = ("exp", "log", "sqrt", "sq", "inv")
BINARY_OPS = ("add", "sub", "mul", "div", "rdiv")
ALL_OPS = UNARY_OPS + BINARY_OPS
# {+,-,*,/,exp,log,sqrt,^2,^-1}: "/" is taken in both operand orders.
STANDARD_OPS = ALL_OPS


# ---------------------------------------------------------------------------
# planted-term evaluation (data synthesis only)
# ---------------------------------------------------------------------------
def _ev(term, X):
    """Evaluate a planted term written as a nested tuple, e.g.
    ("mul", ("x", 7), ("sq", ("x", 13))).  Used only to synthesise targets."""
    with np.errstate(all="ignore"):
        return _ev_raw(term, X)


def _ev_raw(term, X):
    tag = term[0]
    if tag == "x":
        return X[term[1]]
    if tag in UNARY_OPS:
        a = _ev_raw(term[1], X)
        return {"exp": np.exp, "log": np.log, "sqrt": np.sqrt,
                "sq": lambda v: v * v, "inv": lambda v: 1.0 / v}[tag](a)
    a = _ev_raw(term[1], X)
    b = _ev_raw(term[2], X)
    return {"add": a + b, "sub": a - b, "mul": a * b, "div": a / b,
            "rdiv": b / a}[tag]


def _noise(rng, y_clean, frac):
    """Additive Gaussian noise with sigma = frac * std(y_clean)."""
    return rng.normal(0.0, frac * np.std(y_clean), size=y_clean.shape)


def _workload(name, X, Y, units, *, rung, k, D, ops=STANDARD_OPS,
              rung_ops=None, rung_pool=None, score_mode="per_target",
              n_resid=1, omp_D=0, planted=None, note=""):
    X = np.ascontiguousarray(X, dtype=np.float64)
    Y = np.ascontiguousarray(np.atleast_2d(Y), dtype=np.float64)
    if units is not None:
        units = np.ascontiguousarray(units, dtype=np.int32)
    return {
        "name": name, "X": X, "Y": Y, "units": units,
        "p": X.shape[0], "n": X.shape[1], "T": Y.shape[0],
        "B": 0 if units is None else units.shape[1],
        "ops": tuple(ops), "rung": rung,
        "rung_ops": rung_ops, "rung_pool": rung_pool,
        "k": k, "D": D, "score_mode": score_mode,
        "n_resid": n_resid, "omp_D": omp_D,
        "planted": planted, "note": note,
    }


# ---------------------------------------------------------------------------
# the workloads
# ---------------------------------------------------------------------------
def tiny(rung=1):
    """n=100, p=6 uniform on [0.5, 2], y = 1.5*x1*x2 - 0.7*exp(-x3) + noise
    (1-based names; columns 0, 1, 2 here).  Noise sigma = 1e-3."""
    rng = np.random.default_rng(1)
    X = rng.uniform(0.5, 2.0, size=(6, 100))
    y = 1.5 * X[0] * X[1] - 0.7 * np.exp(-X[2]) + rng.normal(0.0, 1e-3, 100)
    planted = [("mul", ("x", 0), ("x", 1)), ("inv", ("exp", ("x", 2)))]
    return _workload("tiny_r%d" % rung, X, y, None, rung=rung, k=20, D=2,
                     planted=planted)


C2_UNITS = np.array([[0, 0, 0]] * 4 + [[1, 0, 0]] * 3 + [[0, 1, 0]] * 3 +
                    [[0, 0, 1]] * 3 + [[1, 0, -1]] * 2 + [[2, 1, -2]],
                    dtype=np.int32)


def units16():
    """n=500, p=16 lognormal(0, 0.5) with exponent vectors over [L, M, T];
    planted energy-unit descriptor, 1% noise; rung 2, top-500, D<=3."""
    rng = np.random.default_rng(2)
    X = rng.lognormal(mean=0.0, sigma=0.5, size=(16, 500))
    fa = ("mul", ("x", 7), ("sq", ("x", 13)))
    fb = ("mul", ("x", 15), ("exp", ("x", 0)))
    fc = ("rdiv", ("x", 3), ("mul", ("x", 2), ("x", 15)))
    yc = 0.5 + 2.0 * _ev(fa, X) - 1.3 * _ev(fb, X) + 0.8 * _ev(fc, X)
    y = yc + _noise(rng, yc, 0.01)
    return _workload("units16", X, y, C2_UNITS, rung=2, k=500, D=3,
                     planted=[fa, fb, fc])


def _random_rung1_term(rng, p):
    ops = ALL_OPS
    op = ops[rng.integers(len(ops))]
    if op in UNARY_OPS:
        return (op, ("x", int(rng.integers(p))))
    i, j = sorted(rng.choice(p, size=2, replace=False).tolist())
    return (op, ("x", i), ("x", j))


def multitarget16():
    """The tiny workload's X with 16 targets y_t = c0 + c1*f_a + c2*f_b +
    N(0, 1e-3), (f_a, f_b) random rung<=1 forms, |c| ~ U[0.5, 2] with random
    sign.  Screening only (per-target top-20)."""
    X = tiny()["X"]
    rng = np.random.default_rng(3)
    Y, planted = [], []
    for _ in range(16):
        fa = _random_rung1_term(rng, 6)
        fb = _random_rung1_term(rng, 6)
        while fb == fa:
            fb = _random_rung1_term(rng, 6)
        c = rng.uniform(0.5, 2.0, 3) * rng.choice([-1.0, 1.0], 3)
        Y.append(c[0] + c[1] * _ev(fa, X) + c[2] * _ev(fb, X)
                 + rng.normal(0.0, 1e-3, X.shape[1]))
        planted.append((fa, fb))
    return _workload("multitarget16", X, np.array(Y), None, rung=1, k=20,
                     D=0, planted=planted)


def _random_rung2_term(rng, p):
    """A random expression of depth exactly 2 over p primaries."""
    inner = _random_rung1_term(rng, p)
    op = ALL_OPS[rng.integers(len(ALL_OPS))]
    if op in UNARY_OPS:
        return (op, inner)
    return (op, ("x", int(rng.integers(p))), inner)


def batch128(n_datasets=128):
    """128 independent datasets: n ~ U{50..2000}, p ~ U{6..20},
    X ~ U[0.5, 2] dimensionless, three planted depth-2 terms with
    coefficients +-U[0.5, 2], intercept U[-1, 1], 1% noise."""
    out = []
    for b in range(n_datasets):
        rng = np.random.default_rng(4000 + b)
        n = int(rng.integers(50, 2001))
        p = int(rng.integers(6, 21))
        X = rng.uniform(0.5, 2.0, size=(p, n))
        terms, yc = [], rng.uniform(-1.0, 1.0)
        for _ in range(3):
            t = _random_rung2_term(rng, p)
            v = _ev(t, X)
            tries = 0
            while (not np.all(np.isfinite(v)) or np.std(v) < 1e-6) and tries < 50:
                t = _random_rung2_term(rng, p)
                v = _ev(t, X)
                tries += 1
            c = rng.uniform(0.5, 2.0) * rng.choice([-1.0, 1.0])
            yc = yc + c * v
            terms.append(t)
        y = yc + _noise(rng, yc, 0.01)
        out.append(_workload("batch128[%d]" % b, X, y, None, rung=2, k=200,
                             D=3, planted=terms))
    return out


C5_UNITS = np.array([[0, 0, 0]] * 6 + [[1, 0, 0]] * 4 + [[0, 1, 0]] * 4 +
                    [[0, 0, 1]] * 4 + [[1, 0, -1]] * 3 + [[2, 1, -2]] * 2 +
                    [[-3, 1, 0]], dtype=np.int32)


def large24():
    """n=2000, p=24 lognormal(0, 0.5) with units; rung 2 plus an
    operator-limited rung 3 (binary operators only, partner a primary);
    8 residual targets (max score), top-1000, L0 D<=3, OMP to D=6."""
    rng = np.random.default_rng(5)
    X = rng.lognormal(mean=0.0, sigma=0.5, size=(24, 2000))
    t1 = ("mul", ("x", 0), ("mul", ("x", 10), ("sq", ("x", 18))))
    t2 = ("mul", ("x", 21), ("exp", ("x", 1)))
    t3 = ("rdiv", ("x", 3), ("mul", ("x", 2), ("x", 22)))
    t4 = ("mul", ("x", 11), ("sq", ("x", 19)))
    t5 = ("div", ("x", 21), ("x", 4))
    yc = (0.5 + 2.0 * _ev(t1, X) - 1.3 * _ev(t2, X) + 0.8 * _ev(t3, X)
          + 0.3 * _ev(t4, X) - 0.2 * _ev(t5, X))
    y = yc + _noise(rng, yc, 0.01)
    bin_mask = tuple(BINARY_OPS)
    return _workload("large24", X, y, C5_UNITS, rung=3, k=1000, D=3,
                     rung_ops=(None, None, None, bin_mask),
                     rung_pool=(None, None, None, 0), score_mode="max",
                     n_resid=8, omp_D=6, planted=[t1, t2, t3, t4, t5])


def subspace3000():
    """A subspace shaped like the large workload's dimension-3 union, for
    the annealing search: S = 3000 rows over n = 2000 samples, each the
    product of two or three of 24 lognormal(0, 0.5) latent columns raised
    to powers in {-2, -1, 1, 2} (so rows correlate as generated features
    do); a planted 6-row model with coefficients +-U[0.5, 2] on
    standardised rows, intercept 0.5, 1 % noise; candidate IDs are 3000
    distinct values below 7e8.  D = 6 (exhaustive L0 would visit 1e18
    subsets)."""
    rng = np.random.default_rng(6)
    n, S, p = 2000, 3000, 24
    Z = rng.lognormal(0.0, 0.5, size=(p, n))
    F = np.empty((S, n))
    for i in range(S):
        k = int(rng.integers(2, 4))
        cols = rng.choice(p, size=k, replace=False)
        pw = rng.choice([-2, -1, 1, 2], size=k)
        F[i] = np.prod([Z[c] ** e for c, e in zip(cols, pw)], axis=0)
    rows = rng.choice(S, size=6, replace=False)
    coef = rng.uniform(0.5, 2.0, size=6) * rng.choice([-1.0, 1.0], size=6)
    yc = 0.5 + sum(c * (F[r] - F[r].mean()) / F[r].std() for c, r in zip(coef, rows))
    y = yc + _noise(rng, yc, 0.01)
    ids = np.sort(rng.choice(700_000_000, size=S, replace=False)).astype(np.int64)
    return {"name": "subspace3000", "F": F, "y": y, "ids": ids, "n": n, "S": S, "D": 6,
            "planted_rows": sorted(int(r) for r in rows)}


def subspace512():
    """A subspace for the exact branch-and-bound L0: S = 512 rows over n =
    2000 samples built like subspace3000's (products of two or three of 24
    lognormal(0, 0.5) latent columns raised to powers in {-2, -1, 1, 2}); a
    planted 5-row model with coefficients +-U[0.5, 2] on standardised rows,
    intercept 0.5, 1 % noise; candidate IDs are 512 distinct values below
    7e8.  D = 5 (C(512, 5) = 2.9e11 subsets)."""
    rng = np.random.default_rng(7)
    n, S, p, D = 2000, 512, 24, 5
    Z = rng.lognormal(0.0, 0.5, size=(p, n))
    F = np.empty((S, n))
    for i in range(S):
        k = int(rng.integers(2, 4))
        cols = rng.choice(p, size=k, replace=False)
        pw = rng.choice([-2, -1, 1, 2], size=k)
        F[i] = np.prod([Z[c] ** e for c, e in zip(cols, pw)], axis=0)
    rows = rng.choice(S, size=D, replace=False)
    coef = rng.uniform(0.5, 2.0, size=D) * rng.choice([-1.0, 1.0], size=D)
    yc = 0.5 + sum(c * (F[r] - F[r].mean()) / F[r].std() for c, r in zip(coef, rows))
    y = yc + _noise(rng, yc, 0.01)
    ids = np.sort(rng.choice(700_000_000, size=S, replace=False)).astype(np.int64)
    return {"name": "subspace512", "F": F, "y": y, "ids": ids, "n": n, "S": S, "D": D,
            "planted_rows": sorted(int(r) for r in rows)}


def random_small(seed, p=4, n=30, rung=2, T=1, units_B=0, lo=0.5, hi=2.0):
    """Small random problem for brute-force cross checks."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(lo, hi, size=(p, n))
    Y = rng.normal(size=(T, n)) + X[0] * X[-1]
    units = None
    if units_B:
        units = rng.integers(-1, 2, size=(p, units_B)).astype(np.int32)
    return _workload("random_small[%d]" % seed, X, Y, units, rung=rung,
                     k=5, D=2)


WORKLOADS = {
    "tiny": tiny,
    "tiny_r2": lambda: tiny(rung=2),
    "units16": units16,
    "multitarget16": multitarget16,
    "large24": large24,
}


def make(name):
    return WORKLOADS[name]()
