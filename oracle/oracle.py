"""FP64 CPU oracle of the DISCOVER / SISSO-style hot path (arXiv 2602.06986).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke entry point and the
benchmark's CPU-baseline leg may import this module; the GPU library never
calls it and shares no code with it.

The arithmetic lives in ``discover_oracle.c`` (plain loops, IEEE double, no
FMA contraction, no fast-math); this module marshals arrays and writes the
selection, L0 ranking, OMP and SISSO loop out step by step.

Readings of the paper (which gives only Eq. (1) and the workflow prose):
  * Screening score: |Pearson r| of each candidate against the target
    (the SIS step of the cited SISSO method, Summary; Figure 1 caption).
  * Selection: candidates sorted by (-score, ID); duplicates (candidates
    whose values are affinely identical to an earlier group head,
    |corr| >= 1 - TAU_DUP, and whose scores agree within TAU_NEAR) form one
    group represented by its smallest ID; groups containing a feature that
    is already in the subspace are dropped; the first k groups are taken.
  * L0 (Eq. (1), Core Optimization Objective): every D-subset of the
    subspace is fitted by least squares with an intercept; subsets whose
    normalized Cholesky pivot is <= PIV_TOL are rank-deficient and skipped;
    ranking by RSS, where RSS values within TAU_TIE * ||y - mean||^2 count as
    tied and the smallest sorted ID tuple wins.
  * OMP (Software Description, cited OMP): greedy addition of the feature
    with the largest |centered correlation| with the residual, refit by QR
    with an intercept.
  * SISSO loop: dimension d screens against the residuals of the best
    model(s) of dimension d-1 and fits the original y over the union of all
    selected features.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "discover_oracle.c")

OPS = ("exp", "log", "sqrt", "sq", "inv", "add", "sub", "mul", "div", "rdiv")
OP_CODE = {name: i for i, name in enumerate(OPS)}
OP_NONE = 15
ST_VALID, ST_UNIT, ST_CHILD, ST_NONFINITE, ST_CONST = range(5)

TAU_NEAR = 1e-9     # relative score agreement for a duplicate pair
TAU_DUP = 1e-9      # 1 - |corr| below which two features are duplicates
PIV_TOL = 1e-10     # normalized Cholesky pivot at or below which a subset is singular
GRAM_DELTA = 1e-7   # band (explained fraction) refitted by QR after the Gram scan
TAU_TIE = 1e-11     # RSS tie tolerance relative to ||y - mean||^2
DIRECT_MAX = 4_000_000   # "auto" L0 fits every subset by QR up to this many subsets


def build(force=False):
    """Compile the C oracle with gcc (no GPU code involved)."""
    if not force and os.path.exists(LIB_PATH) and \
            os.path.getmtime(LIB_PATH) >= os.path.getmtime(SRC_PATH):
        return LIB_PATH
    cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
           "-shared", "-fPIC", "-o", LIB_PATH + ".tmp", SRC_PATH, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.or_count.restype = C.c_int64
        L.or_count.argtypes = [C.c_int, C.c_int, P, P, P]
        L.or_enumerate.restype = C.c_int64
        L.or_enumerate.argtypes = [C.c_int, C.c_int, P, P, C.c_int64, P, P, P, P]
        L.or_decode.restype = C.c_int
        L.or_decode.argtypes = [C.c_int, C.c_int, P, P, C.c_int64, P, P, P, P]
        L.or_units.restype = None
        L.or_units.argtypes = [C.c_int, C.c_int, P, C.c_int, C.c_int64, P, P, P, P, P]
        L.or_screen.restype = C.c_int64
        L.or_screen.argtypes = [C.c_int, C.c_int, P, C.c_int, P, C.c_int, P,
                                C.c_int, P, P, C.c_int64, P, P]
        L.or_values.restype = C.c_int
        L.or_values.argtypes = [C.c_int, C.c_int, P, C.c_int, P, C.c_int, P, P,
                                C.c_int64, P, P, P]
        L.or_pearson.restype = C.c_int
        L.or_pearson.argtypes = [C.c_int, C.c_int64, P, C.c_int, P, P]
        L.or_lsq.restype = C.c_double
        L.or_lsq.argtypes = [C.c_int, C.c_int, P, P, P]
        L.or_pivots.restype = None
        L.or_pivots.argtypes = [C.c_int, C.c_int, P, P]
        L.or_l0_direct.restype = C.c_int64
        L.or_l0_direct.argtypes = [C.c_int, C.c_int, P, P, C.c_int, C.c_double, P]
        L.or_l0_subsets.restype = None
        L.or_l0_subsets.argtypes = [C.c_int, P, P, C.c_int, C.c_int64, P, C.c_double, P]
        L.or_screen_stream.restype = C.c_int64
        L.or_screen_stream.argtypes = [C.c_int, C.c_int, P, C.c_int, P, C.c_int, P,
                                       C.c_int, P, P, C.c_int64, C.c_int, C.c_int64,
                                       C.c_int64, P, P]
        L.or_corr_matrix.restype = None
        L.or_corr_matrix.argtypes = [C.c_int, C.c_int, P, P, P, P, P]
        L.or_l0_gram_band.restype = C.c_int64
        L.or_l0_gram_band.argtypes = [C.c_int, P, P, C.c_int, C.c_double, C.c_int,
                                      C.c_double, C.c_int64, P, P]
        L.or_splitmix_at.restype = C.c_uint64
        L.or_splitmix_at.argtypes = [C.c_uint64, C.c_uint64]
        L.or_sa_exp_neg.restype = C.c_double
        L.or_sa_exp_neg.argtypes = [C.c_double]
        L.or_sa_corr.restype = None
        L.or_sa_corr.argtypes = [C.c_int, C.c_int, P, P, P, P]
        L.or_sa_energy.restype = C.c_double
        L.or_sa_energy.argtypes = [C.c_int, P, P, C.c_int, P]
        L.or_sa_run.restype = C.c_int
        L.or_sa_run.argtypes = [C.c_int, P, P, P, C.c_int, C.c_int, C.c_int64, C.c_double,
                                C.c_double, C.c_uint64, P, P, P]
        L.or_rules.restype = None
        L.or_rules.argtypes = [C.c_int64, P, P, P, C.c_int, P, P, C.c_int, C.c_int, P, P, P, P]
        L.or_max_threads.restype = C.c_int
        L.or_set_threads.restype = None
        L.or_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


# ---------------------------------------------------------------------------
# search space
# ---------------------------------------------------------------------------
def op_mask(ops):
    m = 0
    for o in ops:
        m |= 1 << OP_CODE[o]
    return m


class Space:
    """Raw candidate space P_R: primaries (rung 0) and R rungs of operators.

    ``rung_ops[r]`` (r = 1..R) restricts the operators of rung r (None: all
    of ``ops``); ``rung_pool[r]`` restricts the first operand of binary
    operators at rung r to P_pool (None: P_{r-1}, with i < j)."""

    def __init__(self, p, R, ops, rung_ops=None, rung_pool=None):
        self.p, self.R = int(p), int(R)
        base = op_mask(ops)
        self.masks = np.zeros(4, dtype=np.uint32)
        self.pools = np.full(4, -1, dtype=np.int32)
        for r in range(1, self.R + 1):
            ro = rung_ops[r] if rung_ops is not None and rung_ops[r] is not None else None
            self.masks[r] = base if ro is None else op_mask(ro)
            if rung_pool is not None and rung_pool[r] is not None:
                self.pools[r] = int(rung_pool[r])
        self.levels = np.zeros(self.R + 1, dtype=np.int64)
        self.N = int(lib().or_count(self.p, self.R, _p(self.masks), _p(self.pools),
                                    _p(self.levels)))
        if self.N < 0:
            raise ValueError("invalid search space")

    @property
    def streamable(self):
        """True when the top rung is operator-limited with partners from
        P_pool, pool <= R-2 (its rung R-1 operand can be streamed)."""
        return self.R >= 2 and 0 <= int(self.pools[self.R]) <= self.R - 2

    @property
    def rung_start(self):
        """ID of the first candidate of each rung 0..R, and N."""
        return np.concatenate([[0], np.cumsum(self.levels)]).astype(np.int64)

    @classmethod
    def of(cls, w):
        return cls(w["p"], w["rung"], w["ops"], w.get("rung_ops"), w.get("rung_pool"))

    def enumerate(self):
        N = self.N
        rung = np.empty(N, np.int8); op = np.empty(N, np.int8)
        a = np.empty(N, np.int64); b = np.empty(N, np.int64)
        t = lib().or_enumerate(self.p, self.R, _p(self.masks), _p(self.pools), N,
                               _p(rung), _p(op), _p(a), _p(b))
        assert t == N
        return rung, op, a, b

    def decode(self, cid):
        rung = np.zeros(1, np.int8); op = np.zeros(1, np.int8)
        a = np.zeros(1, np.int64); b = np.zeros(1, np.int64)
        rc = lib().or_decode(self.p, self.R, _p(self.masks), _p(self.pools), int(cid),
                             _p(rung), _p(op), _p(a), _p(b))
        if rc:
            raise ValueError("bad id %d" % cid)
        return int(rung[0]), int(op[0]), int(a[0]), int(b[0])

    def units(self, units):
        """(unit vectors scaled by 2^R [N][B], legality [N]) of every record."""
        rung, op, a, b = self.enumerate()
        B = 0 if units is None else units.shape[1]
        uo = np.zeros((self.N, max(B, 1)), np.int32)
        legal = np.zeros(self.N, np.uint8)
        uin = None if units is None else np.ascontiguousarray(units, np.int32)
        lib().or_units(self.p, B, _p(uin), self.R, self.N, _p(op), _p(a), _p(b),
                       _p(uo), _p(legal))
        return uo[:, :B], legal.astype(bool)

    def rules_allowed(self, units, rules):
        """Mask of the candidates the constraint rules allow (or_rules):
        rules = {max_complexity: int, forbid_nest: {op: [ops]}, forbid_pairs:
        [[i, j], ...] (primaries < 64), target_units: [B] exponents or None}."""
        rung, op, a, b = self.enumerate()
        B = 0 if units is None else units.shape[1]
        uo = np.zeros((self.N, max(B, 1)), np.int32)
        legal = np.zeros(self.N, np.uint8)
        uin = None if units is None else np.ascontiguousarray(units, np.int32)
        lib().or_units(self.p, B, _p(uin), self.R, self.N, _p(op), _p(a), _p(b), _p(uo), _p(legal))
        nest = np.zeros(10, np.uint32)
        for o, cs in (rules.get("forbid_nest") or {}).items():
            for c_ in cs:
                nest[OPS.index(o)] |= np.uint32(1 << OPS.index(c_))
        forb = np.zeros(64, np.uint64)
        for u, v in rules.get("forbid_pairs") or ():
            forb[u] |= np.uint64(1 << v)
            forb[v] |= np.uint64(1 << u)
        tu = rules.get("target_units")
        on = tu is not None
        tunit = np.zeros(max(B, 1), np.int32)
        if on:
            tunit[:B] = np.asarray(tu, np.int64) * (1 << self.R)
        allowed = np.zeros(self.N, np.uint8)
        lib().or_rules(self.N, _p(op), _p(a), _p(b), int(rules.get("max_complexity", -1)), _p(nest),
                       _p(forb), 1 if on else 0, B, _p(np.ascontiguousarray(uo[:, :max(B, 1)])),
                       _p(legal), _p(tunit), _p(allowed))
        return allowed.astype(bool)

    def expr(self, cid):
        """Readable expression of an ID (primaries named x0, x1, ...)."""
        r, op, a, b = self.decode(cid)
        if op == OP_NONE:
            return "x%d" % cid
        name = OPS[op]
        if b < 0:
            return "%s(%s)" % (name, self.expr(a))
        sym = {"add": "+", "sub": "-", "mul": "*", "div": "/"}
        if name == "rdiv":
            return "(%s / %s)" % (self.expr(b), self.expr(a))
        return "(%s %s %s)" % (self.expr(a), sym[name], self.expr(b))


# ---------------------------------------------------------------------------
# screening
# ---------------------------------------------------------------------------
def screen_all(space, X, Y, units):
    """Signed Pearson r [T][N] (NaN if invalid) and status [N] of every raw
    candidate, plus the number of valid candidates."""
    X = np.ascontiguousarray(X, np.float64)
    Y = np.ascontiguousarray(np.atleast_2d(Y), np.float64)
    T, n = Y.shape
    B = 0 if units is None else units.shape[1]
    uin = None if units is None else np.ascontiguousarray(units, np.int32)
    scores = np.empty((T, space.N), np.float64)
    status = np.empty(space.N, np.uint8)
    nv = lib().or_screen(n, space.p, _p(X), T, _p(Y), B, _p(uin), space.R,
                         _p(space.masks), _p(space.pools), space.N, _p(scores),
                         _p(status))
    if nv == -5:
        raise ValueError("constant target")
    if nv < 0:
        raise RuntimeError("or_screen failed (%d)" % nv)
    return scores, status, int(nv)


STREAM_BYTES = 2 << 30   # score arrays larger than this are screened by streaming


def screen_scores(space, X, Y, units, mode, j_range=None):
    """Combined screening scores of every raw candidate: [T'][N] with
    T' = 1 (mode "max": max_t |r_t|) or T (|r_t| per target), NaN when
    invalid; the number of valid candidates; the per-candidate status
    (None when streamed); the count of each status code.  Spaces whose top rung is
    operator-limited are screened by streaming their rung R-1 operand
    (same arithmetic, no [T][N] array of signed r); ``j_range`` then
    restricts the streamed rung-(R-1) features (a timing sample; the other
    entries of those rungs stay NaN)."""
    X = np.ascontiguousarray(X, np.float64)
    Y = np.ascontiguousarray(np.atleast_2d(Y), np.float64)
    T, n = Y.shape
    big = space.N * T * 8 > STREAM_BYTES
    if not space.streamable or (not big and j_range is None):
        r, status, nvalid = screen_all(space, X, Y, units)
        counts = np.bincount(status, minlength=5)[:5].astype(np.int64)
        return combine_scores(r, mode), int(nvalid), status, counts
    B = 0 if units is None else units.shape[1]
    uin = None if units is None else np.ascontiguousarray(units, np.int32)
    Tp = 1 if mode == "max" else T
    out = np.full((Tp, space.N), np.nan, np.float64)
    counts = np.zeros(5, np.int64)
    lo, hi = (0, int(space.levels[space.R - 1])) if j_range is None else j_range
    rc = lib().or_screen_stream(n, space.p, _p(X), T, _p(Y), B, _p(uin), space.R,
                                _p(space.masks), _p(space.pools), space.N,
                                1 if mode == "max" else 0, int(lo), int(hi),
                                _p(out), _p(counts))
    if rc == -5:
        raise ValueError("constant target")
    if rc < 0:
        raise RuntimeError("or_screen_stream failed (%d)" % rc)
    return out, int(counts[ST_VALID]), None, counts


def values(space, X, units, ids):
    """Values [m][n] and status [m] of candidate IDs, evaluated recursively
    from the primaries."""
    ids = np.ascontiguousarray(np.asarray(ids, np.int64).reshape(-1))
    X = np.ascontiguousarray(X, np.float64)
    n = X.shape[1]
    B = 0 if units is None else units.shape[1]
    uin = None if units is None else np.ascontiguousarray(units, np.int32)
    V = np.empty((len(ids), n), np.float64)
    st = np.empty(len(ids), np.uint8)
    if len(ids):
        rc = lib().or_values(n, space.p, _p(X), B, _p(uin), space.R, _p(space.masks),
                             _p(space.pools), len(ids), _p(ids), _p(V), _p(st))
        if rc:
            raise ValueError("bad ids")
    return V, st


def pearson(F, Y):
    """Pearson r [T][m] of feature rows F [m][n] against targets Y [T][n]."""
    F = np.ascontiguousarray(np.atleast_2d(F), np.float64)
    Y = np.ascontiguousarray(np.atleast_2d(Y), np.float64)
    r = np.empty((Y.shape[0], F.shape[0]), np.float64)
    if lib().or_pearson(F.shape[1], F.shape[0], _p(F), Y.shape[0], _p(Y), _p(r)):
        raise ValueError("constant target")
    return r


def combine_scores(r, mode):
    """Screening score from signed r [T][N]: |r| per target, or the maximum
    over targets (several residuals screened at once)."""
    a = np.abs(r)
    if mode == "max":       # validity is per candidate: NaN in every row at once
        return np.max(a, axis=0)[None, :]
    return a


def _corr_abs(u, v):
    u = u - u.mean()
    v = v - v.mean()
    return abs(float(np.dot(u, v)) / math.sqrt(float(np.dot(u, u)) * float(np.dot(v, v))))


def select(score, k, exclude=(), dedup=True, value_fn=None):
    """Exact top-k of one score vector (index = candidate ID; NaN = invalid)
    with the duplicate-group rule.  A score of exactly 0 (a candidate with no
    linear association with the target) is never selected.  Returns (ids,
    scores) of the selected group representatives in (-score, ID) order, and
    the scan record (groups formed, duplicates merged)."""
    score = np.asarray(score, np.float64)
    valid = np.nonzero(score > 0)[0]          # NaN and exact zeros drop out
    excl = set(int(e) for e in exclude)
    # The scan visits candidates in (-s, ID) order and stops early.  For a
    # long vector, sort only the candidates above the K-th largest score
    # (strictly, so the kept set does not depend on how ties are split),
    # and accept the scan if it stopped inside them; otherwise keep more.
    keep = 16 * (k + len(excl)) + 4096
    while True:
        if len(valid) > 4 * keep:
            sv = score[valid]
            thr = np.partition(sv, len(sv) - keep)[len(sv) - keep]
            cand = valid[sv > thr]
            complete = False
        else:
            cand = valid
            complete = True
        order = cand[np.lexsort((cand, -score[cand]))]       # (-s, ID)
        res = _scan(score, order, k, excl, dedup, value_fn)
        if complete or res[3]:
            return res[:3]
        keep *= 8


def _scan(score, order, k, excl, dedup, value_fn):
    heads, members, blocked = [], [], []          # per group
    vals = {}

    def val(cid):
        if cid not in vals:
            vals[cid] = value_fn(cid)
        return vals[cid]

    def kth_unblocked_head_score():
        cnt = 0
        for g in range(len(heads)):
            if not blocked[g]:
                cnt += 1
                if cnt == k:
                    return score[heads[g]]
        return None

    n_merged = 0
    stopped = False
    for c in order:
        c = int(c)
        sc = score[c]
        lim = kth_unblocked_head_score()
        if lim is not None and sc < (1.0 - TAU_NEAR) * lim:
            stopped = True
            break
        grp = -1
        if dedup:
            # heads are in descending score order: walk back over the ones
            # whose score is within the near window, keep the earliest match
            g = len(heads) - 1
            while g >= 0 and score[heads[g]] - sc <= TAU_NEAR * score[heads[g]]:
                if _corr_abs(val(c), val(heads[g])) >= 1.0 - TAU_DUP:
                    grp = g
                g -= 1
        if grp < 0:
            heads.append(c); members.append([c]); blocked.append(c in excl)
        else:
            members[grp].append(c)
            n_merged += 1
            if c in excl:
                blocked[grp] = True
    reps = []
    for g in range(len(heads)):
        if blocked[g]:
            continue
        reps.append(min(members[g]))
        if len(reps) == k:
            break
    reps = np.array(reps, np.int64)
    sc = score[reps] if len(reps) else np.zeros(0)
    o = np.lexsort((reps, -sc))
    return reps[o], sc[o], {"groups": len(heads), "merged": n_merged}, stopped


def sis(space, X, units, targets, k, exclude=(), mode="per_target", dedup=True, allowed=None):
    """Screen every candidate against the targets and select the top-k
    (per target, or one list scored by the maximum over targets).  Returns
    (one (ids, scores, record) per list, status, number of valid
    candidates); status is the per-candidate ST_* array, or, when the space
    was streamed, the count of each ST_* code.  allowed: a boolean mask of
    the candidates the rules allow (Space.rules_allowed), or None."""
    sc, nvalid, status, counts = screen_scores(space, X, targets, units, mode)
    if allowed is not None:
        sc = sc.copy()
        sc[:, ~np.asarray(allowed, bool)] = np.nan   # never selected; counts unchanged
    cache = {}

    def value_fn(cid):
        if cid not in cache:
            cache[cid] = values(space, X, units, [cid])[0][0]
        return cache[cid]

    out = [select(sc[t], k, exclude, dedup, value_fn) for t in range(sc.shape[0])]
    if status is None:
        status = counts
    return out, status, nvalid


# ---------------------------------------------------------------------------
# L0 and OMP
# ---------------------------------------------------------------------------
def lsq(F_rows, y):
    """Least squares of y on [1, rows of F] by Householder QR:
    (coef with intercept first, RSS)."""
    F_rows = [np.ascontiguousarray(f, np.float64) for f in F_rows]
    y = np.ascontiguousarray(y, np.float64)
    d = len(F_rows)
    ptrs = (C.c_void_p * max(d, 1))(*[f.ctypes.data for f in F_rows])
    coef = np.zeros(d + 1, np.float64)
    rss = lib().or_lsq(len(y), d, ptrs, _p(y), _p(coef))
    return coef, float(rss)


def pivots(F_rows):
    F_rows = [np.ascontiguousarray(f, np.float64) for f in F_rows]
    d = len(F_rows)
    ptrs = (C.c_void_p * d)(*[f.ctypes.data for f in F_rows])
    piv = np.zeros(d, np.float64)
    lib().or_pivots(len(F_rows[0]), d, ptrs, _p(piv))
    return piv


def corr_matrix(F, y):
    F = np.ascontiguousarray(F, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    S, n = F.shape
    Cm = np.empty((S, S), np.float64)
    c = np.empty(S, np.float64)
    yy = np.zeros(1, np.float64)
    lib().or_corr_matrix(n, S, _p(F), _p(y), _p(Cm), _p(c), _p(yy))
    return Cm, c, float(yy[0])


def sa_corr(F, y):
    """Correlation matrix and target correlations in the fixed order the
    annealing reads (left-to-right sums, one rounding per operation)."""
    F = np.ascontiguousarray(F, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    S, n = F.shape
    Cm = np.empty((S, S), np.float64)
    c = np.empty(S, np.float64)
    lib().or_sa_corr(n, S, _p(F), _p(y), _p(Cm), _p(c))
    return Cm, c


def sa_energy(Cm, c, rows):
    """1 - R^2 of the subset `rows` (array order) from sa_corr's matrices;
    inf when a Cholesky pivot is at or below 1e-10."""
    a = np.ascontiguousarray(rows, np.int32)
    return float(lib().or_sa_energy(Cm.shape[0], _p(Cm), _p(c), len(a), _p(a)))


def anneal(F, ids, y, D, chains, steps, T0, alpha, seed, init=None):
    """Simulated annealing over D-subsets of the rows of F (the
    stochastic search the paper names for the sparsifying step, Software
    Description): `chains` independent Metropolis chains of `steps`
    single-row swaps under geometric cooling T0 * alpha^k, random numbers
    from counter-based SplitMix64 (or_sa_run states every rule).  Returns
    (winning chain, best rows of every chain [chains][D] ascending, their
    energies 1 - R^2 [chains])."""
    Cm, c = sa_corr(F, y)
    S = Cm.shape[0]
    ids = np.ascontiguousarray(ids, np.int64)
    best = np.zeros((chains, D), np.int32)
    be = np.zeros(chains, np.float64)
    ini = None
    if init is not None:
        ini = np.ascontiguousarray(init, np.int32)
        assert len(ini) == D and len(set(ini.tolist())) == D and ini.min() >= 0 and ini.max() < S
    w = lib().or_sa_run(S, _p(Cm), _p(c), _p(ids), D, chains, int(steps), float(T0), float(alpha),
                        int(seed) & 0xFFFFFFFFFFFFFFFF, _p(ini), _p(best), _p(be))
    if w < 0:
        raise ValueError("anneal: D must be in 1..8 and at most S, chains >= 1")
    return int(w), best, be


def _rank_models(cands, m, yy):
    """cands: list of (rss, sorted_id_tuple, positions).  Ties within
    TAU_TIE * yy of the current minimum go to the smallest ID tuple."""
    rem = list(cands)
    out = []
    while rem and len(out) < m:
        rmin = min(c[0] for c in rem)
        tie = [c for c in rem if c[0] <= rmin + TAU_TIE * yy]
        pick = min(tie, key=lambda c: c[1])
        out.append(pick)
        rem.remove(pick)
    return out


def all_subsets(S, D):
    import itertools
    return list(itertools.combinations(range(S), D))


def unrank(t, S, D):
    """The t-th D-subset of range(S) in lexicographic order."""
    out, lo = [], 0
    for k in range(D):
        v = lo
        while True:
            cnt = math.comb(S - 1 - v, D - 1 - k)
            if t < cnt:
                break
            t -= cnt
            v += 1
        out.append(v)
        lo = v + 1
    return tuple(out)


def subset_rss(F, y, subsets):
    """RSS by QR with an intercept of each subset (rows [count][D] of
    positions into F); NaN when a normalized pivot is <= PIV_TOL."""
    F = np.ascontiguousarray(F, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    sub = np.ascontiguousarray(np.atleast_2d(subsets), np.int32)
    rss = np.empty(sub.shape[0], np.float64)
    if sub.shape[0]:
        lib().or_l0_subsets(F.shape[1], _p(F), _p(y), sub.shape[1], sub.shape[0],
                            _p(sub), PIV_TOL, _p(rss))
    return rss


def l0(F, ids, y, D, m=1, mode="auto"):
    """Exhaustive L0 over every D-subset of the rows of F (Eq. (1) with an
    intercept).  mode "direct" fits every subset by QR; "gram" scans the
    explained fraction from the correlation matrix and refits the band
    within GRAM_DELTA of the m-th best by QR (a shortcut for subset counts
    where QR of every subset takes hours; its agreement with direct mode is
    checked by the test suite and by the reference-building script); "auto"
    is direct up to DIRECT_MAX subsets.  Returns a list of m models: dicts
    with positions, ids, rss, rmse, coef, resid."""
    F = np.ascontiguousarray(F, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    S, n = F.shape
    ids = np.asarray(ids, np.int64)
    yc = y - y.mean()
    yy = float(np.dot(yc, yc))
    if mode == "auto":
        mode = "direct" if math.comb(S, D) <= DIRECT_MAX else "gram"
    cands = []
    if mode == "direct":
        tot = math.comb(S, D)
        rss = np.empty(tot, np.float64)
        got = lib().or_l0_direct(n, S, _p(F), _p(y), D, PIV_TOL, _p(rss))
        assert got == tot
        # Every model the ranking below can pick has an RSS within TAU_TIE * yy
        # of the m-th smallest RSS, so only those subsets are ranked.
        fin = rss[~np.isnan(rss)]
        if len(fin):
            mth = np.partition(fin, min(m, len(fin)) - 1)[min(m, len(fin)) - 1]
            for t in np.nonzero(rss <= mth + TAU_TIE * yy)[0]:
                sub = unrank(int(t), S, D)
                cands.append((float(rss[t]), tuple(sorted(int(ids[i]) for i in sub)), sub))
    else:
        Cm, c, _ = corr_matrix(F, y)
        cap = 1 << 16
        while True:
            band = np.empty((cap, D), np.int32)
            bq = np.empty(cap, np.float64)
            cnt = lib().or_l0_gram_band(S, _p(Cm), _p(c), D, PIV_TOL, m, GRAM_DELTA,
                                        cap, _p(band), _p(bq))
            if cnt <= cap:
                break
            cap = int(cnt)
        for t in range(max(cnt, 0)):
            sub = tuple(int(v) for v in band[t])
            _, r = lsq([F[i] for i in sub], y)
            cands.append((r, tuple(sorted(int(ids[i]) for i in sub)), sub))
    out = []
    for rss, idt, sub in _rank_models(cands, m, yy):
        coef, r = lsq([F[i] for i in sub], y)
        pred = coef[0] + sum(coef[1 + q] * F[i] for q, i in enumerate(sub))
        out.append({"positions": tuple(sub), "ids": tuple(int(ids[i]) for i in sub),
                    "rss": r, "rmse": math.sqrt(r / n), "coef": coef,
                    "resid": y - pred})
    return out


def omp(F, ids, y, D_max, init=()):
    """Orthogonal matching pursuit over the rows of F: starting from the
    active set ``init``, repeatedly add the row with the largest
    |sum (f - mean f) r| / ||f - mean f|| (ties: smallest ID) and refit y on
    [1, active rows] by QR.  Returns (active positions, coef, rmse, resid)."""
    F = np.ascontiguousarray(F, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    ids = np.asarray(ids, np.int64)
    S, n = F.shape
    active = [int(a) for a in init]
    Fc = F - F.mean(axis=1, keepdims=True)
    nrm = np.sqrt(np.einsum("ij,ij->i", Fc, Fc))

    def fit(act):
        coef, r = lsq([F[i] for i in act], y)
        pred = coef[0] + sum(coef[1 + q] * F[i] for q, i in enumerate(act))
        return coef, r, y - pred

    coef, rss, resid = fit(active)
    while len(active) < D_max:
        g = np.abs(Fc @ resid) / np.where(nrm > 0, nrm, np.inf)
        g[active] = -1.0
        cand = np.nonzero(g >= 0)[0]
        if len(cand) == 0:
            break
        j = int(cand[np.lexsort((ids[cand], -g[cand]))[0]])
        active.append(j)
        coef, rss, resid = fit(active)
    return active, coef, math.sqrt(rss / n), resid


# ---------------------------------------------------------------------------
# SISSO loop
# ---------------------------------------------------------------------------
def sisso(w, dedup=True, l0_mode="auto"):
    """Run the full loop of one workload dict (see synth.workloads)."""
    space = Space.of(w)
    X, units = w["X"], w["units"]
    y = w["Y"][0]
    k, D, m = w["k"], w["D"], w["n_resid"]
    res = {"space": space, "dims": []}
    if D == 0:      # screening only, one list per target
        out, status, nvalid = sis(space, X, units, w["Y"], k, (), "per_target", dedup)
        res["sis"] = out
        res["status"] = status
        res["nvalid"] = nvalid
        return res
    S_ids = np.zeros(0, np.int64)
    F = np.zeros((0, w["n"]))
    targets = y[None, :]
    for d in range(1, D + 1):
        mode = "max" if targets.shape[0] > 1 or w["score_mode"] == "max" else "per_target"
        out, status, nvalid = sis(space, X, units, targets, k, S_ids, mode, dedup)
        sel_ids, sel_sc, rec = out[0]
        V, _ = values(space, X, units, sel_ids)
        S_ids = np.concatenate([S_ids, sel_ids])
        F = np.vstack([F, V])
        models = l0(F, S_ids, y, d, m, l0_mode)
        res["dims"].append({"sel_ids": sel_ids, "sel_scores": sel_sc, "record": rec,
                            "nvalid": nvalid, "status": status, "models": models,
                            "targets": targets})
        targets = np.array([mo["resid"] for mo in models])
    res["S_ids"] = S_ids
    res["F"] = F
    if w.get("omp_D", 0) > D:
        act, coef, rmse, resid = omp(F, S_ids, y, w["omp_D"], res["dims"][-1]["models"][0]["positions"])
        res["omp"] = {"positions": act, "ids": [int(S_ids[a]) for a in act], "coef": coef,
                      "rmse": rmse, "resid": resid}
    return res
