/*
 * FP64 CPU oracle for the SISSO-style descriptor search of DISCOVER
 * (arXiv 2602.06986).  TEST INFRASTRUCTURE ONLY: the product path never
 * links, loads or calls this file; it exists so that the GPU library can be
 * checked against a plain, slow, obviously correct implementation.
 *
 * What the paper fixes, and where:
 *   - candidate features are generated iteratively from primary features
 *     and an operator library, with pruning by physical constraints
 *     (Software Description; Figure 1 caption);
 *   - dimensional consistency removes invalid expressions early
 *     (Physics-Informed Constraints);
 *   - candidates are screened against the target (Figure 1 caption; SIS as
 *     in the cited SISSO method, Summary);
 *   - the sparse model solves the L0-constrained least squares of Eq. (1)
 *     (Core Optimization Objective), with OMP among the search strategies
 *     (Software Description).
 * Everything finer (enumeration order, unit arithmetic, validity, score,
 * duplicate rule, intercept, tolerances) is a reading of the paper where it
 * is silent; each routine states the reading it implements.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC.
 * Parallel loops only distribute independent candidates or subsets; every
 * reduction runs in a fixed order, so results do not depend on the number
 * of threads.
 *
 * Operator codes (library order): 0 exp, 1 log, 2 sqrt, 3 sq, 4 inv,
 * 5 add, 6 sub, 7 mul, 8 div, 9 rdiv.  A rung operator mask has bit c set
 * when operator c is enabled at that rung.
 *
 * Parity unpinned by the paper: the enumeration order, the unit rules,
 * validity thresholds, the duplicate rule and the L0 tolerances are this
 * implementation's readings; they are pinned only by closed forms, brute
 * force and library cross-checks in the test suite.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXR 4
#define OR_MAXB 8

enum { OP_EXP = 0, OP_LOG, OP_SQRT, OP_SQ, OP_INV,
       OP_ADD, OP_SUB, OP_MUL, OP_DIV, OP_RDIV, OP_NONE = 15 };

enum { ST_VALID = 0, ST_UNIT = 1, ST_CHILD = 2, ST_NONFINITE = 3,
       ST_CONST = 4 };

/* A feature is numerically constant when its population standard deviation
 * is at most this fraction of its root-mean-square value. */
static const double OR_CONST_TOL = 1e-8;
/* A sum or difference whose root-mean-square value is at most this fraction
 * of its operands' combined root-mean-square value is cancellation noise
 * (e.g. x - exp(log(x))) and counts as constant. */
static const double OR_CANCEL_TOL = 1e-10;

/* ------------------------------------------------------------------------ */
/* Search-space description                                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int p, R;
    uint32_t ops[OR_MAXR];   /* ops[r] for r = 1..R */
    int32_t pool[OR_MAXR];   /* partner rung for binary ops at rung r */
    int64_t L[OR_MAXR];      /* raw size of each rung */
    int64_t off[OR_MAXR + 1];/* off[r] = |P_{r-1}|, start of rung r */
} space_t;

static int popc(uint32_t m) { int c = 0; while (m) { c += m & 1u; m >>= 1; } return c; }

static int64_t choose2(int64_t m) { return m * (m - 1) / 2; }

/* Number of partner pairs at rung r: every (i, j) with j in rung r-1 and i
 * either below j inside P_{r-1} (pool = r-1) or anywhere in P_pool. */
static int64_t pairs_at(const space_t* s, int r) {
    if (s->pool[r] == r - 1)
        return choose2(s->off[r]) - choose2(s->off[r - 1]);
    return s->L[r - 1] * s->off[s->pool[r] + 1];
}

static int space_init(space_t* s, int p, int R, const uint32_t* rung_ops,
                      const int32_t* rung_pool) {
    memset(s, 0, sizeof(*s));
    if (p < 1 || R < 0 || R >= OR_MAXR) return -1;
    s->p = p; s->R = R;
    s->L[0] = p; s->off[0] = 0; s->off[1] = p;
    for (int r = 1; r <= R; r++) {
        s->ops[r] = rung_ops ? rung_ops[r] : 0x3FFu;
        int pl = rung_pool ? rung_pool[r] : -1;
        if (pl < 0) pl = r - 1;
        if (pl > r - 1) return -1;
        s->pool[r] = pl;
        int nu = popc(s->ops[r] & 0x1Fu), nb = popc(s->ops[r] & 0x3E0u);
        s->L[r] = (int64_t)nu * s->L[r - 1] + (int64_t)nb * pairs_at(s, r);
        s->off[r + 1] = s->off[r] + s->L[r];
    }
    return 0;
}

/* Raw rung sizes L_0..L_R; returns |P_R|. */
int64_t or_count(int p, int R, const uint32_t* rung_ops, const int32_t* rung_pool,
                 int64_t* level_sizes) {
    space_t s;
    if (space_init(&s, p, R, rung_ops, rung_pool)) return -1;
    for (int r = 0; r <= R; r++) level_sizes[r] = s.L[r];
    return s.off[R + 1];
}

/* Enumerate the raw candidate list P_R in canonical order (the ID of a
 * candidate is its position).  Rung r (r >= 1) holds, in this order: one
 * block per enabled unary operator (operand runs over rung r-1 in index
 * order), then one block per enabled binary operator (j runs over rung r-1
 * in increasing index, i over the partner pool below j).  For each record:
 * rung, op (OP_NONE for primaries), operand a (the unary operand, or i) and
 * operand b (j, or -1). */
int64_t or_enumerate(int p, int R, const uint32_t* rung_ops,
                     const int32_t* rung_pool, int64_t cap, int8_t* rung,
                     int8_t* op, int64_t* a, int64_t* b) {
    space_t s;
    if (space_init(&s, p, R, rung_ops, rung_pool)) return -1;
    if (s.off[R + 1] > cap) return -2;
    int64_t t = 0;
    for (int64_t f = 0; f < p; f++) {
        rung[t] = 0; op[t] = OP_NONE; a[t] = -1; b[t] = -1; t++;
    }
    for (int r = 1; r <= R; r++) {
        for (int u = 0; u < 5; u++) {
            if (!(s.ops[r] >> u & 1u)) continue;
            for (int64_t x = s.off[r - 1]; x < s.off[r]; x++) {
                rung[t] = (int8_t)r; op[t] = (int8_t)u; a[t] = x; b[t] = -1; t++;
            }
        }
        for (int o = 5; o < 10; o++) {
            if (!(s.ops[r] >> o & 1u)) continue;
            for (int64_t j = s.off[r - 1]; j < s.off[r]; j++) {
                int64_t ilim = (s.pool[r] == r - 1) ? j : s.off[s.pool[r] + 1];
                for (int64_t i = 0; i < ilim; i++) {
                    rung[t] = (int8_t)r; op[t] = (int8_t)o; a[t] = i; b[t] = j; t++;
                }
            }
        }
    }
    return t;
}

/* Decode one ID without enumerating: walk the rung blocks, then the
 * operator blocks, then (for pair blocks) scan j upward.  Returns 0 on
 * success. */
int or_decode(int p, int R, const uint32_t* rung_ops, const int32_t* rung_pool,
              int64_t id, int8_t* rung, int8_t* op, int64_t* a, int64_t* b) {
    space_t s;
    if (space_init(&s, p, R, rung_ops, rung_pool)) return -1;
    if (id < 0 || id >= s.off[R + 1]) return -2;
    if (id < p) { *rung = 0; *op = OP_NONE; *a = -1; *b = -1; return 0; }
    int r = 1;
    while (id >= s.off[r + 1]) r++;
    int64_t q = id - s.off[r];
    *rung = (int8_t)r;
    for (int u = 0; u < 5; u++) {
        if (!(s.ops[r] >> u & 1u)) continue;
        if (q < s.L[r - 1]) { *op = (int8_t)u; *a = s.off[r - 1] + q; *b = -1; return 0; }
        q -= s.L[r - 1];
    }
    int64_t np = pairs_at(&s, r);
    for (int o = 5; o < 10; o++) {
        if (!(s.ops[r] >> o & 1u)) continue;
        if (q < np) {
            *op = (int8_t)o;
            if (s.pool[r] == r - 1) {
                int64_t j = s.off[r - 1];
                while (q >= j) { q -= j; j++; }
                *a = q; *b = j;
            } else {
                int64_t w = s.off[s.pool[r] + 1];
                *a = q % w; *b = s.off[r - 1] + q / w;
            }
            return 0;
        }
        q -= np;
    }
    return -3;
}

/* ------------------------------------------------------------------------ */
/* Units: integer exponent vectors over B base units, stored multiplied by  */
/* Q = 2^R so that square roots stay integral.                                */
/* ------------------------------------------------------------------------ */
/* Unit rule for one operator.  Returns 1 (legal) and writes the result, or
 * 0 (dimensionally invalid). */
static int unit_rule(int o, int B, const int32_t* ua, const int32_t* ub, int32_t* out) {
    int k;
    switch (o) {
    case OP_EXP: case OP_LOG:               /* argument must be dimensionless */
        for (k = 0; k < B; k++) if (ua[k] != 0) return 0;
        for (k = 0; k < B; k++) out[k] = 0;
        return 1;
    case OP_SQRT:
        for (k = 0; k < B; k++) if (ua[k] % 2 != 0) return 0;
        for (k = 0; k < B; k++) out[k] = ua[k] / 2;
        return 1;
    case OP_SQ:  for (k = 0; k < B; k++) out[k] = 2 * ua[k]; return 1;
    case OP_INV: for (k = 0; k < B; k++) out[k] = -ua[k]; return 1;
    case OP_ADD: case OP_SUB:               /* operands must agree */
        for (k = 0; k < B; k++) if (ua[k] != ub[k]) return 0;
        for (k = 0; k < B; k++) out[k] = ua[k];
        return 1;
    case OP_MUL:  for (k = 0; k < B; k++) out[k] = ua[k] + ub[k]; return 1;
    case OP_DIV:  for (k = 0; k < B; k++) out[k] = ua[k] - ub[k]; return 1;
    case OP_RDIV: for (k = 0; k < B; k++) out[k] = ub[k] - ua[k]; return 1;
    }
    return 0;
}

/* Unit vector (scaled by 2^R) and legality of every record of an
 * enumeration.  A record is legal when its operands are legal and the
 * operator's rule accepts their units. */
void or_units(int p, int B, const int32_t* units, int R, int64_t N,
              const int8_t* op, const int64_t* a, const int64_t* b,
              int32_t* uout, uint8_t* legal) {
    const int32_t Q = 1 << R;
    for (int64_t t = 0; t < N; t++) {
        int32_t* u = uout + t * B;
        if (op[t] == OP_NONE) {
            for (int k = 0; k < B; k++) u[k] = units ? units[t * B + k] * Q : 0;
            legal[t] = 1;
            continue;
        }
        const int64_t ia = a[t], ib = b[t];
        if (!legal[ia] || (ib >= 0 && !legal[ib])) {
            legal[t] = 0;
            for (int k = 0; k < B; k++) u[k] = 0;
            continue;
        }
        legal[t] = (uint8_t)unit_rule(op[t], B, uout + ia * B,
                                      ib >= 0 ? uout + ib * B : NULL, u);
        if (!legal[t]) for (int k = 0; k < B; k++) u[k] = 0;
    }
}

/* ------------------------------------------------------------------------ */
/* Values, validity and the Pearson score                                    */
/* ------------------------------------------------------------------------ */
static void apply_op(int o, int n, const double* x, const double* y, double* f) {
    int s;
    switch (o) {
    case OP_EXP:  for (s = 0; s < n; s++) f[s] = exp(x[s]); break;
    case OP_LOG:  for (s = 0; s < n; s++) f[s] = log(x[s]); break;
    case OP_SQRT: for (s = 0; s < n; s++) f[s] = sqrt(x[s]); break;
    case OP_SQ:   for (s = 0; s < n; s++) f[s] = x[s] * x[s]; break;
    case OP_INV:  for (s = 0; s < n; s++) f[s] = 1.0 / x[s]; break;
    case OP_ADD:  for (s = 0; s < n; s++) f[s] = x[s] + y[s]; break;
    case OP_SUB:  for (s = 0; s < n; s++) f[s] = x[s] - y[s]; break;
    case OP_MUL:  for (s = 0; s < n; s++) f[s] = x[s] * y[s]; break;
    case OP_DIV:  for (s = 0; s < n; s++) f[s] = x[s] / y[s]; break;
    case OP_RDIV: for (s = 0; s < n; s++) f[s] = y[s] / x[s]; break;
    }
}

/* Neumaier-compensated sum. */
static double nsum(const double* v, int n) {
    double s = 0.0, c = 0.0;
    for (int i = 0; i < n; i++) {
        double t = s + v[i];
        if (fabs(s) >= fabs(v[i])) c += (s - t) + v[i];
        else c += (v[i] - t) + s;
        s = t;
    }
    return s + c;
}

/* Numerical checks of a feature's values: all finite, finite second
 * moment, not constant.  On success writes the mean and the centered sum of
 * squares.  `tmp` has n entries. */
static int feature_checks(int n, const double* f, double* tmp, double* mean, double* sxx) {
    for (int s = 0; s < n; s++) if (!isfinite(f[s])) return ST_NONFINITE;
    double m = nsum(f, n) / n;
    for (int s = 0; s < n; s++) { double d = f[s] - m; tmp[s] = d * d; }
    double ss = nsum(tmp, n);
    if (!isfinite(ss)) return ST_NONFINITE;
    double sd = sqrt(ss / n), rms = sqrt(ss / n + m * m);
    if (!(sd > OR_CONST_TOL * rms)) return ST_CONST;
    *mean = m; *sxx = ss;
    return ST_VALID;
}

/* Cancellation rule for add/sub: sum f^2 <= tol^2 (sum a^2 + sum b^2). */
static int cancelled(int o, int n, const double* f, const double* a, const double* b, double* tmp) {
    if (o != OP_ADD && o != OP_SUB) return 0;
    for (int s = 0; s < n; s++) tmp[s] = f[s] * f[s];
    const double ff = nsum(tmp, n);
    for (int s = 0; s < n; s++) tmp[s] = a[s] * a[s] + b[s] * b[s];
    const double ab = nsum(tmp, n);
    return ff <= OR_CANCEL_TOL * OR_CANCEL_TOL * ab;
}

/* Pearson r of f against a centered target yc (sum of squares syy):
 * two-pass, compensated, r = sum (f-m)(yc) / sqrt(sxx * syy). */
static double pearson(int n, const double* f, double m, double sxx,
                      const double* yc, double syy, double* tmp) {
    for (int s = 0; s < n; s++) tmp[s] = (f[s] - m) * yc[s];
    return nsum(tmp, n) / sqrt(sxx * syy);
}

/* Center every target; returns nonzero when a target is constant. */
static int prep_targets(int n, int T, const double* Y, double* Yc, double* syy, double* tmp) {
    for (int t = 0; t < T; t++) {
        const double* y = Y + (int64_t)t * n;
        double m = nsum(y, n) / n;
        for (int s = 0; s < n; s++) Yc[(int64_t)t * n + s] = y[s] - m;
        for (int s = 0; s < n; s++) tmp[s] = Yc[(int64_t)t * n + s] * Yc[(int64_t)t * n + s];
        syy[t] = nsum(tmp, n);
        double sd = sqrt(syy[t] / n), rms = sqrt(syy[t] / n + m * m);
        if (!(sd > OR_CONST_TOL * rms)) return 1;
    }
    return 0;
}

/* Screen every raw candidate of P_R.  Features of rungs below R are
 * evaluated once and kept (rung R needs them as operands); each rung-R
 * candidate is evaluated on the fly from its two operands.
 *   X       [p][n]; Y [T][n]
 *   scores  [T][N]  Pearson r (signed) for valid candidates, NaN otherwise
 *   status  [N]     ST_* code
 * Returns the number of valid candidates, or <0 on error
 * (-5: a constant target). */
int64_t or_screen(int n, int p, const double* X, int T, const double* Y,
                  int B, const int32_t* units, int R, const uint32_t* rung_ops,
                  const int32_t* rung_pool, int64_t N, double* scores,
                  uint8_t* status) {
    space_t s;
    if (space_init(&s, p, R, rung_ops, rung_pool)) return -1;
    if (N != s.off[R + 1]) return -2;
    int8_t* rg = malloc(N); int8_t* op = malloc(N);
    int64_t* ia = malloc(N * 8); int64_t* ib = malloc(N * 8);
    int32_t* uu = malloc((B ? B : 1) * N * 4); uint8_t* legal = malloc(N);
    const int64_t M = s.off[R];                 /* |P_{R-1}| features kept */
    double* V = malloc((M ? M : 1) * (int64_t)n * 8);
    double* Yc = malloc((int64_t)T * n * 8); double* syy = malloc(T * 8);
    double* tmp0 = malloc((int64_t)n * 8);
    int64_t nvalid = 0;
    or_enumerate(p, R, rung_ops, rung_pool, N, rg, op, ia, ib);
    or_units(p, B, units, R, N, op, ia, ib, uu, legal);
    if (prep_targets(n, T, Y, Yc, syy, tmp0)) { nvalid = -5; goto done; }
    /* Rungs below R, in order (operands always precede their parents). */
    for (int64_t t = 0; t < M; t++) {
        double* f = V + t * n;
        if (op[t] == OP_NONE) memcpy(f, X + t * n, (size_t)n * 8);
        else apply_op(op[t], n, V + ia[t] * n, ib[t] >= 0 ? V + ib[t] * n : NULL, f);
    }
    for (int64_t t = 0; t < M; t++) {
        if (!legal[t]) status[t] = ST_UNIT;
        else if ((op[t] != OP_NONE) &&
                 (status[ia[t]] != ST_VALID || (ib[t] >= 0 && status[ib[t]] != ST_VALID)))
            status[t] = ST_CHILD;
        else {
            double m, sxx;
            status[t] = (uint8_t)feature_checks(n, V + t * n, tmp0, &m, &sxx);
            if (status[t] == ST_VALID && ib[t] >= 0 &&
                cancelled(op[t], n, V + t * n, V + ia[t] * n, V + ib[t] * n, tmp0))
                status[t] = ST_CONST;
        }
    }
    #pragma omp parallel
    {
        double* f = malloc((int64_t)n * 8);
        double* tmp = malloc((int64_t)n * 8);
        #pragma omp for schedule(dynamic, 256)
        for (int64_t t = 0; t < N; t++) {
            const double* fv;
            if (t >= M) {
                if (!legal[t]) { status[t] = ST_UNIT; goto fill; }
                if (status[ia[t]] != ST_VALID || (ib[t] >= 0 && status[ib[t]] != ST_VALID)) {
                    status[t] = ST_CHILD; goto fill;
                }
                apply_op(op[t], n, V + ia[t] * n, ib[t] >= 0 ? V + ib[t] * n : NULL, f);
                double m, sxx;
                status[t] = (uint8_t)feature_checks(n, f, tmp, &m, &sxx);
                if (status[t] == ST_VALID && ib[t] >= 0 &&
                    cancelled(op[t], n, f, V + ia[t] * n, V + ib[t] * n, tmp))
                    status[t] = ST_CONST;
                if (status[t] != ST_VALID) goto fill;
                fv = f;
                for (int q = 0; q < T; q++)
                    scores[(int64_t)q * N + t] = pearson(n, fv, m, sxx, Yc + (int64_t)q * n, syy[q], tmp);
                continue;
            } else {
                if (status[t] != ST_VALID) goto fill;
                double m, sxx;
                feature_checks(n, V + t * n, tmp, &m, &sxx);
                for (int q = 0; q < T; q++)
                    scores[(int64_t)q * N + t] = pearson(n, V + t * n, m, sxx, Yc + (int64_t)q * n, syy[q], tmp);
                continue;
            }
        fill:
            for (int q = 0; q < T; q++) scores[(int64_t)q * N + t] = NAN;
        }
        free(f); free(tmp);
    }
    for (int64_t t = 0; t < N; t++) nvalid += status[t] == ST_VALID;
done:
    free(rg); free(op); free(ia); free(ib); free(uu); free(legal);
    free(V); free(Yc); free(syy); free(tmp0);
    return nvalid;
}

/* Scores of one valid feature against the centered targets, combined as
 * max_t |r_t| (mode 1: out[id]) or |r_t| per target (mode 0: out[t*N+id]). */
static void score_feature(int n, const double* f, int T, const double* Yc, const double* syy,
                          int mode, int64_t N, int64_t id, double* out, double* tmp) {
    double m, sxx;
    feature_checks(n, f, tmp, &m, &sxx);
    double best = 0.0;
    for (int q = 0; q < T; q++) {
        double r = fabs(pearson(n, f, m, sxx, Yc + (int64_t)q * n, syy[q], tmp));
        if (mode == 1) { if (r > best || q == 0) best = r; }
        else out[(int64_t)q * N + id] = r;
    }
    if (mode == 1) out[id] = best;
}

static void mark_invalid(int T, int mode, int64_t N, int64_t id, double* out) {
    if (mode == 1) out[id] = NAN;
    else for (int q = 0; q < T; q++) out[(int64_t)q * N + id] = NAN;
}

/* Status of a feature f = op(a, b) whose operands have statuses sa, sb and
 * which is unit-legal: ST_CHILD, or the numerical checks of or_screen. */
static int derived_status(int o, int n, const double* f, const double* fa, const double* fb,
                          int sa, int sb, double* tmp) {
    if (sa != ST_VALID || (fb && sb != ST_VALID)) return ST_CHILD;
    double m, sxx;
    int st = feature_checks(n, f, tmp, &m, &sxx);
    if (st == ST_VALID && fb && cancelled(o, n, f, fa, fb, tmp)) st = ST_CONST;
    return st;
}

/* Screening of a space whose top rung R is operator-limited (binary
 * partners drawn from P_pool with pool <= R-2), without keeping rung R-1 in
 * memory.  Candidates are taken in a different order than in or_screen but
 * each one is evaluated, checked and scored by the same routines, so every
 * score and status is the one or_screen gives:
 *   - P_{R-2} is evaluated once and kept (values, units, status), and its
 *     members are scored;
 *   - for each feature g of rung R-1 with local index j in [j_lo, j_hi):
 *     g is evaluated from its operands in P_{R-2}, checked and scored; then
 *     every rung-R candidate with g as its rung-(R-1) operand (unary u(g),
 *     and op(f_i, g) for i in P_pool) is evaluated, checked and scored.
 * Candidates of rungs R-1 and R outside the j range are left untouched.
 *   out     mode 1: [N] max_t |r_t|; mode 0: [T][N] |r_t|; NaN when invalid
 *   counts  [5] number of visited candidates per ST_* code
 * Returns 0, or <0 on error (-5: a constant target, -4: the space is not of
 * this shape). */
int64_t or_screen_stream(int n, int p, const double* X, int T, const double* Y,
                         int B, const int32_t* units, int R, const uint32_t* rung_ops,
                         const int32_t* rung_pool, int64_t N, int mode,
                         int64_t j_lo, int64_t j_hi, double* out, int64_t* counts) {
    space_t s;
    if (space_init(&s, p, R, rung_ops, rung_pool)) return -1;
    if (N != s.off[R + 1]) return -2;
    if (R < 2 || s.pool[R] > R - 2) return -4;
    const int64_t M = s.off[R - 1];             /* |P_{R-2}|: kept */
    const int64_t L1 = s.L[R - 1];              /* rung R-1: streamed */
    if (j_lo < 0) j_lo = 0;
    if (j_hi > L1) j_hi = L1;
    const int32_t Q = 1 << R;
    const int Bq = B ? B : 1;
    double* V = malloc(M * (int64_t)n * 8);
    int32_t* U = calloc((size_t)(M * Bq), 4);
    uint8_t* legal = malloc(M); uint8_t* st = malloc(M);
    double* Yc = malloc((int64_t)T * n * 8); double* syy = malloc(T * 8);
    double* tmp0 = malloc((int64_t)n * 8);
    int64_t cnt[5] = {0, 0, 0, 0, 0};
    int64_t rc = 0;
    if (prep_targets(n, T, Y, Yc, syy, tmp0)) { rc = -5; goto done; }
    /* P_{R-2}: values, units, status (operands precede their parents) */
    for (int64_t t = 0; t < M; t++) {
        int8_t rg, o; int64_t a, b;
        or_decode(p, R, s.ops, s.pool, t, &rg, &o, &a, &b);
        double* f = V + t * n;
        int32_t* u = U + t * Bq;
        if (o == OP_NONE) {
            memcpy(f, X + t * n, (size_t)n * 8);
            for (int k = 0; k < B; k++) u[k] = units ? units[t * B + k] * Q : 0;
            legal[t] = 1;
        } else {
            apply_op(o, n, V + a * n, b >= 0 ? V + b * n : NULL, f);
            legal[t] = legal[a] && (b < 0 || legal[b]) &&
                       unit_rule(o, B, U + a * Bq, b >= 0 ? U + b * Bq : NULL, u);
            if (!legal[t]) for (int k = 0; k < B; k++) u[k] = 0;
        }
        if (!legal[t]) st[t] = ST_UNIT;
        else if (o == OP_NONE) { double m, sxx; st[t] = (uint8_t)feature_checks(n, f, tmp0, &m, &sxx); }
        else st[t] = (uint8_t)derived_status(o, n, f, V + a * n, b >= 0 ? V + b * n : NULL,
                                             st[a], b >= 0 ? st[b] : ST_VALID, tmp0);
        cnt[st[t]]++;
        if (st[t] == ST_VALID) score_feature(n, f, T, Yc, syy, mode, N, t, out, tmp0);
        else mark_invalid(T, mode, N, t, out);
    }
    {
        const int nu = popc(s.ops[R] & 0x1Fu);
        const int64_t w = s.off[s.pool[R] + 1];       /* partner pool size */
        #pragma omp parallel
        {
            double* g = malloc((int64_t)n * 8); double* f = malloc((int64_t)n * 8);
            double* tmp = malloc((int64_t)n * 8);
            int32_t ug[OR_MAXB], uc[OR_MAXB];
            int64_t lc[5] = {0, 0, 0, 0, 0};
            #pragma omp for schedule(dynamic, 16)
            for (int64_t j = j_lo; j < j_hi; j++) {
                const int64_t gid = s.off[R - 1] + j;
                int8_t rg, o; int64_t a, b;
                or_decode(p, R, s.ops, s.pool, gid, &rg, &o, &a, &b);
                apply_op(o, n, V + a * n, b >= 0 ? V + b * n : NULL, g);
                int gl = legal[a] && (b < 0 || legal[b]) &&
                         unit_rule(o, B, U + a * Bq, b >= 0 ? U + b * Bq : NULL, ug);
                int gs = !gl ? ST_UNIT
                             : derived_status(o, n, g, V + a * n, b >= 0 ? V + b * n : NULL,
                                              st[a], b >= 0 ? st[b] : ST_VALID, tmp);
                lc[gs]++;
                if (gs == ST_VALID) score_feature(n, g, T, Yc, syy, mode, N, gid, out, tmp);
                else mark_invalid(T, mode, N, gid, out);
                /* rung-R children of g, in the order of their IDs */
                int64_t base = s.off[R];
                int ui = 0;
                for (int uo = 0; uo < 5; uo++) {
                    if (!(s.ops[R] >> uo & 1u)) continue;
                    const int64_t cid = base + (int64_t)ui * L1 + j;
                    ui++;
                    int cs;
                    if (!gl || !unit_rule(uo, B, ug, NULL, uc)) cs = ST_UNIT;
                    else {
                        apply_op(uo, n, g, NULL, f);
                        cs = derived_status(uo, n, f, g, NULL, gs, ST_VALID, tmp);
                    }
                    lc[cs]++;
                    if (cs == ST_VALID) score_feature(n, f, T, Yc, syy, mode, N, cid, out, tmp);
                    else mark_invalid(T, mode, N, cid, out);
                }
                base += (int64_t)nu * L1;
                for (int bo = 5; bo < 10; bo++) {
                    if (!(s.ops[R] >> bo & 1u)) continue;
                    for (int64_t i = 0; i < w; i++) {
                        const int64_t cid = base + j * w + i;
                        int cs;
                        if (!gl || !legal[i] || !unit_rule(bo, B, U + i * Bq, ug, uc)) cs = ST_UNIT;
                        else {
                            apply_op(bo, n, V + i * n, g, f);
                            cs = derived_status(bo, n, f, V + i * n, g, st[i], gs, tmp);
                        }
                        lc[cs]++;
                        if (cs == ST_VALID) score_feature(n, f, T, Yc, syy, mode, N, cid, out, tmp);
                        else mark_invalid(T, mode, N, cid, out);
                    }
                    base += L1 * w;
                }
            }
            #pragma omp critical
            for (int k = 0; k < 5; k++) cnt[k] += lc[k];
            free(g); free(f); free(tmp);
        }
    }
    for (int k = 0; k < 5; k++) counts[k] = cnt[k];
done:
    free(V); free(U); free(legal); free(st); free(Yc); free(syy); free(tmp0);
    return rc;
}

/* Recursive evaluation of one ID from the primaries, with its status (the
 * same rules as or_screen: unit legality, valid operands, finite values,
 * not constant).  `f` receives n values.  Unit vectors of the operands are
 * computed recursively as well.  Returns the ST_* code. */
static int eval_rec(const space_t* s, int n, const double* X, int B,
                    const int32_t* units, int64_t id, double* f, int32_t* u,
                    double* tmp) {
    int8_t rg, o; int64_t a, b;
    or_decode(s->p, s->R, s->ops, s->pool, id, &rg, &o, &a, &b);
    const int32_t Q = 1 << s->R;
    if (o == OP_NONE) {
        memcpy(f, X + id * n, (size_t)n * 8);
        for (int k = 0; k < B; k++) u[k] = units ? units[id * B + k] * Q : 0;
    } else {
        double* fa = malloc((int64_t)n * 8); double* fb = b >= 0 ? malloc((int64_t)n * 8) : NULL;
        int32_t ua[OR_MAXB], ub[OR_MAXB];
        int sa = eval_rec(s, n, X, B, units, a, fa, ua, tmp);
        int sb = b >= 0 ? eval_rec(s, n, X, B, units, b, fb, ub, tmp) : ST_VALID;
        int leg = (sa != ST_UNIT) && (sb != ST_UNIT) && unit_rule(o, B, ua, ub, u);
        apply_op(o, n, fa, fb, f);         /* values are returned in every case */
        int st = ST_VALID;
        if (!leg) { for (int k = 0; k < B; k++) u[k] = 0; st = ST_UNIT; }
        else if (sa != ST_VALID || sb != ST_VALID) st = ST_CHILD;
        else {
            double m, sxx;
            st = feature_checks(n, f, tmp, &m, &sxx);
            if (st == ST_VALID && fb && cancelled(o, n, f, fa, fb, tmp)) st = ST_CONST;
        }
        free(fa); free(fb);
        return st;
    }
    double m, sxx;
    return feature_checks(n, f, tmp, &m, &sxx);
}

/* Values and status of a list of IDs, each evaluated recursively from the
 * primaries.  values [m][n] (filled even when invalid), status [m]. */
int or_values(int n, int p, const double* X, int B, const int32_t* units,
              int R, const uint32_t* rung_ops, const int32_t* rung_pool,
              int64_t m, const int64_t* ids, double* values, uint8_t* status) {
    space_t s;
    if (space_init(&s, p, R, rung_ops, rung_pool)) return -1;
    for (int64_t t = 0; t < m; t++) if (ids[t] < 0 || ids[t] >= s.off[R + 1]) return -2;
    #pragma omp parallel
    {
        double* tmp = malloc((int64_t)n * 8);
        int32_t u[OR_MAXB];
        #pragma omp for schedule(dynamic, 4)
        for (int64_t t = 0; t < m; t++)
            status[t] = (uint8_t)eval_rec(&s, n, X, B, units, ids[t], values + t * n, u, tmp);
        free(tmp);
    }
    return 0;
}

/* Pearson r of given feature values against given targets (same formula as
 * the screen): f [m][n], Y [T][n] -> r [T][m]; NaN for constant or
 * non-finite features. */
int or_pearson(int n, int64_t m, const double* F, int T, const double* Y, double* r) {
    double* Yc = malloc((int64_t)T * n * 8); double* syy = malloc(T * 8);
    double* tmp = malloc((int64_t)n * 8);
    int bad = prep_targets(n, T, Y, Yc, syy, tmp);
    if (!bad) {
        for (int64_t t = 0; t < m; t++) {
            double mm, sxx;
            int st = feature_checks(n, F + t * n, tmp, &mm, &sxx);
            for (int q = 0; q < T; q++)
                r[(int64_t)q * m + t] = st == ST_VALID
                    ? pearson(n, F + t * n, mm, sxx, Yc + (int64_t)q * n, syy[q], tmp) : NAN;
        }
    }
    free(Yc); free(syy); free(tmp);
    return bad ? -5 : 0;
}

/* ------------------------------------------------------------------------ */
/* Least squares (Eq. 1 restricted to one support, with an intercept)       */
/* ------------------------------------------------------------------------ */
/* Householder QR least squares of y on the n x m design A (column-major,
 * overwritten).  Writes the coefficients (m), the residual sum of squares
 * and |R_jj| (m).  Textbook Householder reflections, applied column by
 * column; returns 0. */
static int householder_lsq(int n, int m, double* A, double* y, double* coef,
                           double* rss, double* rdiag) {
    for (int j = 0; j < m; j++) {
        double* aj = A + (int64_t)j * n;
        double nrm = 0.0;
        for (int i = j; i < n; i++) nrm += aj[i] * aj[i];
        nrm = sqrt(nrm);
        double alpha = aj[j] > 0 ? -nrm : nrm;
        double v0 = aj[j] - alpha;
        double vv = v0 * v0;
        for (int i = j + 1; i < n; i++) vv += aj[i] * aj[i];
        aj[j] = v0;                          /* v stored in place */
        if (vv > 0.0) {
            for (int c = j + 1; c < m; c++) {
                double* ac = A + (int64_t)c * n;
                double d = 0.0;
                for (int i = j; i < n; i++) d += aj[i] * ac[i];
                double g = 2.0 * d / vv;
                for (int i = j; i < n; i++) ac[i] -= g * aj[i];
            }
            double d = 0.0;
            for (int i = j; i < n; i++) d += aj[i] * y[i];
            double g = 2.0 * d / vv;
            for (int i = j; i < n; i++) y[i] -= g * aj[i];
        }
        rdiag[j] = alpha;
        aj[j] = alpha;
    }
    /* back substitution with R (upper triangle of A, diagonal = alpha) */
    for (int j = m - 1; j >= 0; j--) {
        double acc = y[j];
        for (int c = j + 1; c < m; c++) acc -= A[(int64_t)c * n + j] * coef[c];
        coef[j] = acc / A[(int64_t)j * n + j];
    }
    double r = 0.0;
    for (int i = m; i < n; i++) r += y[i] * y[i];
    *rss = r;
    for (int j = 0; j < m; j++) rdiag[j] = fabs(rdiag[j]);
    return 0;
}

/* Least-squares fit of y on [1, f_1..f_d] (the columns given as pointers)
 * with caller-provided work space: A n*(d+1), w n.  coef[0] is the
 * intercept.  Returns the RSS. */
static double lsq_buf(int n, int d, const double* const* cols, const double* y,
                      double* coef, double* A, double* w) {
    int m = d + 1;
    double rd[16];
    for (int i = 0; i < n; i++) A[i] = 1.0;
    for (int j = 0; j < d; j++) memcpy(A + (int64_t)(j + 1) * n, cols[j], (size_t)n * 8);
    memcpy(w, y, (size_t)n * 8);
    double rss;
    householder_lsq(n, m, A, w, coef, &rss, rd);
    return rss;
}

/* Squared |R_jj| of the QR of the centered, unit-norm columns (in the given
 * order): the Cholesky pivots of their correlation matrix.  Work space:
 * A n*d, w n. */
static void pivots_buf(int n, int d, const double* const* cols, double* piv,
                       double* A, double* w) {
    double coef[16], rd[16], rss;
    for (int i = 0; i < n; i++) w[i] = 0.0;
    for (int j = 0; j < d; j++) {
        double* c = A + (int64_t)j * n;
        memcpy(c, cols[j], (size_t)n * 8);
        double m = nsum(c, n) / n;
        for (int i = 0; i < n; i++) c[i] -= m;
        double ss = 0.0;
        for (int i = 0; i < n; i++) ss += c[i] * c[i];
        double inv = 1.0 / sqrt(ss);
        for (int i = 0; i < n; i++) c[i] *= inv;
    }
    householder_lsq(n, d, A, w, coef, &rss, rd);
    for (int j = 0; j < d; j++) piv[j] = rd[j] * rd[j];
}

double or_lsq(int n, int d, const double* const* cols, const double* y, double* coef) {
    double* A = malloc((int64_t)n * (d + 1) * 8); double* w = malloc((int64_t)n * 8);
    double rss = lsq_buf(n, d, cols, y, coef, A, w);
    free(A); free(w);
    return rss;
}

void or_pivots(int n, int d, const double* const* cols, double* piv) {
    double* A = malloc((int64_t)n * d * 8); double* w = malloc((int64_t)n * 8);
    pivots_buf(n, d, cols, piv, A, w);
    free(A); free(w);
}

/* Lexicographic successor of a D-subset of {0..S-1}; 0 when exhausted. */
static int next_comb(int* c, int D, int S) {
    int i = D - 1;
    while (i >= 0 && c[i] == S - D + i) i--;
    if (i < 0) return 0;
    c[i]++;
    for (int k = i + 1; k < D; k++) c[k] = c[k - 1] + 1;
    return 1;
}

static int64_t binom(int64_t a, int64_t b) {
    if (b < 0 || a < b) return 0;
    int64_t r = 1;
    for (int64_t z = 0; z < b; z++) r = r * (a - z) / (z + 1);
    return r;
}

/* RSS of one subset by QR with an intercept (Eq. (1)), or NaN when its
 * smallest normalized pivot is <= piv_tol.  Work space A n*(D+1), w n. */
static double subset_rss(int n, const double* F, const double* y, int D, const int* sub,
                         double piv_tol, double* A, double* w) {
    const double* cols[8]; double coef[9], piv[8];
    for (int k = 0; k < D; k++) cols[k] = F + (int64_t)sub[k] * n;
    pivots_buf(n, D, cols, piv, A, w);
    double mn = piv[0];
    for (int k = 1; k < D; k++) if (piv[k] < mn) mn = piv[k];
    return (mn > piv_tol) ? lsq_buf(n, D, cols, y, coef, A, w) : NAN;
}

/* Direct mode: every D-subset of the S rows of F ([S][n]) in lexicographic
 * order is fitted by Householder QR with an intercept.  rss[t] is NaN when
 * the subset's smallest pivot (see or_pivots) is <= piv_tol.  The subsets
 * with first element a occupy the C(S-1-a, D-1) positions after those of
 * a-1; each thread walks the subsets of one a in order.  Returns the number
 * of subsets. */
int64_t or_l0_direct(int n, int S, const double* F, const double* y, int D,
                     double piv_tol, double* rss) {
    if (D < 1 || D > 8 || S < D) return 0;
    const int64_t total = binom(S, D);
    int64_t* start = malloc((size_t)(S + 1) * 8);
    start[0] = 0;
    for (int a = 0; a < S; a++) start[a + 1] = start[a] + binom(S - 1 - a, D - 1);
    #pragma omp parallel
    {
        double* A = malloc((int64_t)n * (D + 1) * 8); double* w = malloc((int64_t)n * 8);
        int cc[8];
        #pragma omp for schedule(dynamic, 1)
        for (int a = 0; a <= S - D; a++) {
            for (int k = 0; k < D; k++) cc[k] = a + k;
            int64_t t = start[a];
            do {
                rss[t++] = subset_rss(n, F, y, D, cc, piv_tol, A, w);
            } while (next_comb(cc, D, S) && cc[0] == a);
        }
        free(A); free(w);
    }
    free(start);
    return total;
}

/* RSS by QR (as in direct mode) of a list of D-subsets: sub [count][D]
 * positions into F ([S][n]); rss [count], NaN for singular subsets. */
void or_l0_subsets(int n, const double* F, const double* y, int D, int64_t count,
                   const int32_t* sub, double piv_tol, double* rss) {
    #pragma omp parallel
    {
        double* A = malloc((int64_t)n * (D + 1) * 8); double* w = malloc((int64_t)n * 8);
        int cc[8];
        #pragma omp for schedule(dynamic, 16)
        for (int64_t t = 0; t < count; t++) {
            for (int k = 0; k < D; k++) cc[k] = sub[t * D + k];
            rss[t] = subset_rss(n, F, y, D, cc, piv_tol, A, w);
        }
        free(A); free(w);
    }
}

/* Correlation matrix of the centered, unit-norm rows of F ([S][n]) and
 * their correlations with the centered, unit-norm y:
 *   C [S][S], c [S]; yy = sum (y - mean)^2.  Plain compensated dot
 * products. */
void or_corr_matrix(int n, int S, const double* F, const double* y, double* C,
                    double* c, double* yy) {
    double* Z = malloc((int64_t)S * n * 8); double* z = malloc((int64_t)n * 8);
    double* tmp = malloc((int64_t)n * 8);
    for (int a = 0; a < S; a++) {
        const double* f = F + (int64_t)a * n; double* q = Z + (int64_t)a * n;
        double m = nsum(f, n) / n;
        for (int s = 0; s < n; s++) q[s] = f[s] - m;
        for (int s = 0; s < n; s++) tmp[s] = q[s] * q[s];
        double inv = 1.0 / sqrt(nsum(tmp, n));
        for (int s = 0; s < n; s++) q[s] *= inv;
    }
    double m = nsum(y, n) / n;
    for (int s = 0; s < n; s++) z[s] = y[s] - m;
    for (int s = 0; s < n; s++) tmp[s] = z[s] * z[s];
    *yy = nsum(tmp, n);
    double inv = 1.0 / sqrt(*yy);
    for (int s = 0; s < n; s++) z[s] *= inv;
    #pragma omp parallel
    {
        double* t2 = malloc((int64_t)n * 8);
        #pragma omp for schedule(dynamic, 4)
        for (int a = 0; a < S; a++) {
            const double* qa = Z + (int64_t)a * n;
            for (int b = a; b < S; b++) {
                const double* qb = Z + (int64_t)b * n;
                for (int s = 0; s < n; s++) t2[s] = qa[s] * qb[s];
                C[(int64_t)a * S + b] = C[(int64_t)b * S + a] = nsum(t2, n);
            }
            for (int s = 0; s < n; s++) t2[s] = qa[s] * z[s];
            c[a] = nsum(t2, n);
        }
        free(t2);
    }
    free(Z); free(z); free(tmp);
}

/* Explained fraction q = c_S^T C_SS^{-1} c_S of one subset by Cholesky of
 * the D x D correlation block in subset order; the pivots are the
 * squared diagonal of the Cholesky factor.  Returns 0 when any pivot is
 * <= piv_tol (rank-deficient), 1 otherwise; *pmin receives the smallest
 * pivot. */
static int gram_subset(int S, const double* C, const double* c, int D, const int* sub,
                       double piv_tol, double* q, double* pmin) {
    double L[8][8], z[8];
    double mn = 1.0;
    for (int i = 0; i < D; i++) {
        for (int j = 0; j <= i; j++) {
            double acc = C[(int64_t)sub[i] * S + sub[j]];
            for (int k = 0; k < j; k++) acc -= L[i][k] * L[j][k];
            if (i == j) {
                if (!(acc > piv_tol)) return 0;
                if (acc < mn) mn = acc;
                L[i][i] = sqrt(acc);
            } else {
                L[i][j] = acc / L[j][j];
            }
        }
    }
    double acc2 = 0.0;
    for (int i = 0; i < D; i++) {
        double acc = c[sub[i]];
        for (int k = 0; k < i; k++) acc -= L[i][k] * z[k];
        z[i] = acc / L[i][i];
        acc2 += z[i] * z[i];
    }
    *q = acc2;
    *pmin = mn;
    return 1;
}

/* Rounding allowance of a Gram-route explained fraction: the correlation
 * entries carry errors of a few ulps, which the solve amplifies by the
 * condition number of the block, about D / (smallest pivot). */
static double gram_slack(int D, double pmin) {
    return 64.0 * D * 2.220446049250313e-16 / pmin;
}

/* Gram mode, used where fitting every subset by QR is too slow: the
 * explained fraction of each D-subset from the correlation matrix
 * (mathematically RSS = yy (1 - q)).  Pass 1 finds the m-th largest q over
 * all non-singular subsets; pass 2 returns every subset with
 * q >= q_(m) - delta - (its rounding allowance, which grows as its smallest
 * pivot shrinks): the band that is then refitted by QR.
 *   band  [cap][D] positions (ascending), bq [cap]
 * Returns the band size (which may exceed cap: then only cap are written),
 * or -1 if fewer than one non-singular subset exists. */
int64_t or_l0_gram_band(int S, const double* C, const double* c, int D,
                        double piv_tol, int m, double delta, int64_t cap,
                        int32_t* band, double* bq) {
    if (D < 1 || D > 8 || S < D || m < 1 || m > 64) return -1;
    double best[64]; int nb = 0;
    #pragma omp parallel
    {
        double lb[64]; int ln = 0;
        int sub[8];
        #pragma omp for schedule(dynamic, 1)
        for (int a = 0; a <= S - D; a++) {
            sub[0] = a;
            for (int k = 1; k < D; k++) sub[k] = a + k;
            do {
                double q, pm;
                if (gram_subset(S, C, c, D, sub, piv_tol, &q, &pm)) {
                    if (ln < m || q > lb[ln - 1]) {   /* keep top-m, descending */
                        int pos = ln < m ? ln++ : m - 1;
                        while (pos > 0 && lb[pos - 1] < q) { lb[pos] = lb[pos - 1]; pos--; }
                        lb[pos] = q;
                    }
                }
                /* advance the tail (positions 1..D-1) keeping sub[0] = a */
                int i = D - 1;
                while (i >= 1 && sub[i] == S - D + i) i--;
                if (i < 1) break;
                sub[i]++;
                for (int k = i + 1; k < D; k++) sub[k] = sub[k - 1] + 1;
            } while (1);
        }
        #pragma omp critical
        {
            for (int t = 0; t < ln; t++) {
                double q = lb[t];
                if (nb < m || q > best[nb - 1]) {
                    int pos = nb < m ? nb++ : m - 1;
                    while (pos > 0 && best[pos - 1] < q) { best[pos] = best[pos - 1]; pos--; }
                    best[pos] = q;
                }
            }
        }
    }
    if (nb == 0) return -1;
    const double thr = best[nb - 1] - delta;
    int64_t count = 0;
    #pragma omp parallel
    {
        int sub[8];
        #pragma omp for schedule(dynamic, 1)
        for (int a = 0; a <= S - D; a++) {
            sub[0] = a;
            for (int k = 1; k < D; k++) sub[k] = a + k;
            do {
                double q, pm;
                if (gram_subset(S, C, c, D, sub, piv_tol, &q, &pm) &&
                    q >= thr - gram_slack(D, pm)) {
                    int64_t slot;
                    #pragma omp atomic capture
                    slot = count++;
                    if (slot < cap) {
                        for (int k = 0; k < D; k++) band[slot * D + k] = sub[k];
                        bq[slot] = q;
                    }
                }
                int i = D - 1;
                while (i >= 1 && sub[i] == S - D + i) i--;
                if (i < 1) break;
                sub[i]++;
                for (int k = i + 1; k < D; k++) sub[k] = sub[k - 1] + 1;
            } while (1);
        }
    }
    return count;
}

int or_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* ------------------------------------------------------------------------ */
/* Simulated annealing over D-subsets                                        */
/* ------------------------------------------------------------------------ */
/* The paper names simulated annealing among the stochastic strategies for
 * the sparsifying step (Software Description) when exhaustive L0 over the
 * subsets of Eq. (1) is out of reach.  The reading implemented here:
 *
 *   state    a D-subset a[0..D-1] of the S rows (an ordered array);
 *   energy   E(a) = 1 - R^2 of the least-squares fit of y on [1, rows a],
 *            from the correlation matrix: E = 1 - c_a^T C_aa^{-1} c_a, by
 *            Cholesky of C_aa in array order; a pivot at or below 1e-10
 *            (R10) makes the subset singular, E = +inf;
 *   move     a uniform position p of the array and a uniform row r; a row
 *            already in the subset leaves the state unchanged;
 *   accept   Metropolis: E' <= E, or u < exp(-(E' - E) / T) for a uniform
 *            u in [0, 1); T starts at T0 and is multiplied by alpha after
 *            every proposal (geometric cooling);
 *   chains   independent, each with its own random stream; each keeps its
 *            best state (smallest E, ties: the smaller sorted candidate-ID
 *            tuple), and the problem's result is the best over chains.
 *
 * Random numbers: the SplitMix64 generator (Steele, Lea and Flood, OOPSLA
 * 2014), used counter-based.  Output i (i >= 1) of the stream with state
 * x0 is mix(x0 + i * 0x9E3779B97F4A7C15).  Chain q's key is output q + 1
 * of the stream with state seed; its draw number c is output c + 1 of the
 * stream with state key.  A row draw is draw mod S, a uniform is
 * (draw >> 11) * 2^-53.
 *
 * Every quantity that decides a move (correlations, Cholesky, exp) is
 * computed in IEEE double with one rounding per operation (no fused
 * multiply-add, built with -ffp-contract=off), in a fixed order, so that
 * an implementation that does the same obtains the same trajectory bit for
 * bit.  exp(-x) is evaluated by the range reduction x = k ln 2 + r and the
 * Taylor series of exp(-r) to degree 18 in Horner form (an approximation
 * of exp accurate to a few ulps; the same function on both sides is what
 * matters for the trajectory).
 */
static const uint64_t SM_GAMMA = 0x9E3779B97F4A7C15ull;

uint64_t or_splitmix_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Output i (i >= 1) of the SplitMix64 stream with state x0. */
uint64_t or_splitmix_at(uint64_t x0, uint64_t i) { return or_splitmix_mix(x0 + i * SM_GAMMA); }

static uint64_t sa_draw(uint64_t key, uint64_t c) { return or_splitmix_at(key, c + 1); }

double or_sa_exp_neg(double x) {
    if (!(x < 700.0)) return 0.0;
    if (x <= 0.0) return 1.0;
    const double LN2 = 0.6931471805599453;
    const double INV_LN2 = 1.4426950408889634;
    const int k = (int)(x * INV_LN2);
    const double t = (double)k * LN2;
    const double r = x - t;
    double p = 1.0;
    for (int i = 18; i >= 1; i--) {
        double q = p * -r;
        q = q / (double)i;
        p = 1.0 + q;
    }
    return ldexp(p, -k);
}

/* Correlation matrix in the fixed order the annealing reads: per row, the
 * mean as a left-to-right sum over samples divided by n, centred values,
 * norm = sqrt of the left-to-right sum of squares; C[i][j] = (left-to-right
 * sum of z_i z_j) / (norm_i * norm_j), c[i] the same with the centred
 * target; a constant row gets norm 0 and C = c = 0 in its row and column. */
void or_sa_corr(int n, int S, const double* F, const double* y, double* C, double* c) {
    double* Z = (double*)malloc(sizeof(double) * (size_t)(S + 1) * n);
    double* nrm = (double*)malloc(sizeof(double) * (size_t)(S + 1));
    for (int i = 0; i <= S; i++) {
        const double* f = i < S ? F + (size_t)i * n : y;
        double s = 0.0;
        for (int t = 0; t < n; t++) s = s + f[t];
        const double m = s / (double)n;
        double q = 0.0;
        for (int t = 0; t < n; t++) {
            const double d = f[t] - m;
            Z[(size_t)i * n + t] = d;
            q = q + d * d;
        }
        nrm[i] = sqrt(q);
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < S; i++) {
        for (int j = 0; j <= S; j++) {
            double v = 0.0;
            if (nrm[i] > 0.0 && nrm[j] > 0.0) {
                double d = 0.0;
                for (int t = 0; t < n; t++) d = d + Z[(size_t)i * n + t] * Z[(size_t)j * n + t];
                v = d / (nrm[i] * nrm[j]);
            }
            if (j < S) C[(size_t)i * S + j] = v;
            else c[i] = v;
        }
    }
    free(Z);
    free(nrm);
}

/* E = 1 - R^2 of the subset a (array order), +inf when singular. */
double or_sa_energy(int S, const double* C, const double* c, int D, const int* a) {
    double L[8][8], w[8];
    for (int j = 0; j < D; j++) {
        double d = C[(size_t)a[j] * S + a[j]];
        for (int k = 0; k < j; k++) d = d - L[j][k] * L[j][k];
        if (!(d > 1e-10)) return INFINITY;
        const double ljj = sqrt(d);
        L[j][j] = ljj;
        for (int i = j + 1; i < D; i++) {
            double v = C[(size_t)a[i] * S + a[j]];
            for (int k = 0; k < j; k++) v = v - L[i][k] * L[j][k];
            L[i][j] = v / ljj;
        }
    }
    double ex = 0.0;
    for (int j = 0; j < D; j++) {
        double v = c[a[j]];
        for (int k = 0; k < j; k++) v = v - L[j][k] * w[k];
        w[j] = v / L[j][j];
        ex = ex + w[j] * w[j];
    }
    return 1.0 - ex;
}

static void sort_rows(int D, int* s) {
    for (int i = 1; i < D; i++)
        for (int j = i; j > 0 && s[j] < s[j - 1]; j--) { int t = s[j]; s[j] = s[j - 1]; s[j - 1] = t; }
}

/* ID tuple of sorted rows a before that of b (rows are sorted by row index;
 * the tuples compare by sorted candidate ID). */
static int ids_before(int D, const int* a, const int* b, const int64_t* ids) {
    int64_t ia[8], ib[8];
    for (int i = 0; i < D; i++) { ia[i] = ids[a[i]]; ib[i] = ids[b[i]]; }
    for (int i = 1; i < D; i++)
        for (int j = i; j > 0; j--) {
            if (ia[j] < ia[j - 1]) { int64_t t = ia[j]; ia[j] = ia[j - 1]; ia[j - 1] = t; }
            if (ib[j] < ib[j - 1]) { int64_t t = ib[j]; ib[j] = ib[j - 1]; ib[j - 1] = t; }
        }
    for (int i = 0; i < D; i++)
        if (ia[i] != ib[i]) return ia[i] < ib[i];
    return 0;
}

/* Annealing of Q chains; chain q's best subset (rows ascending) goes to
 * best + q D and its energy to best_e[q]; init (D rows) or NULL for a
 * random start (rows drawn with draws 0, 1, ... of the chain, repeats
 * skipped).  Proposal k uses draws 2^40 + 3k (position), + 1 (row), + 2
 * (uniform).  Returns the chain holding the overall best. */
int or_sa_run(int S, const double* C, const double* c, const int64_t* ids, int D, int Q,
              int64_t K, double T0, double alpha, uint64_t seed, const int* init, int* best,
              double* best_e) {
    if (D < 1 || D > 8 || D > S || Q < 1) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int q = 0; q < Q; q++) {
        const uint64_t key = or_splitmix_at(seed, (uint64_t)q + 1);
        int a[8], b[8], bs[8];
        if (init) {
            for (int j = 0; j < D; j++) a[j] = init[j];
        } else {
            uint64_t ctr = 0;
            for (int j = 0; j < D; j++) {
                for (;;) {
                    const int r = (int)(sa_draw(key, ctr++) % (uint64_t)S);
                    int dup = 0;
                    for (int i = 0; i < j; i++) dup |= a[i] == r;
                    if (!dup) { a[j] = r; break; }
                }
            }
        }
        double E = or_sa_energy(S, C, c, D, a);
        double bE = E;
        for (int j = 0; j < D; j++) bs[j] = a[j];
        sort_rows(D, bs);
        double T = T0;
        const uint64_t base = (uint64_t)1 << 40;
        for (int64_t k = 0; k < K; k++) {
            const int p = (int)(sa_draw(key, base + 3 * (uint64_t)k) % (uint64_t)D);
            const int r = (int)(sa_draw(key, base + 3 * (uint64_t)k + 1) % (uint64_t)S);
            const double u = (double)(sa_draw(key, base + 3 * (uint64_t)k + 2) >> 11) * 0x1.0p-53;
            int in = 0;
            for (int j = 0; j < D; j++) in |= a[j] == r;
            if (!in) {
                for (int j = 0; j < D; j++) b[j] = a[j];
                b[p] = r;
                const double En = or_sa_energy(S, C, c, D, b);
                int acc = En <= E;
                if (!acc && En < INFINITY) acc = u < or_sa_exp_neg((En - E) / T);
                if (acc) {
                    for (int j = 0; j < D; j++) a[j] = b[j];
                    E = En;
                    int sa[8];
                    for (int j = 0; j < D; j++) sa[j] = a[j];
                    sort_rows(D, sa);
                    if (E < bE || (E == bE && ids_before(D, sa, bs, ids))) {
                        bE = E;
                        for (int j = 0; j < D; j++) bs[j] = sa[j];
                    }
                }
            }
            T = T * alpha;
        }
        for (int j = 0; j < D; j++) best[(size_t)q * D + j] = bs[j];
        best_e[q] = bE;
    }
    int w = 0;
    for (int q = 1; q < Q; q++)
        if (best_e[q] < best_e[w] || (best_e[q] == best_e[w] && ids_before(D, best + (size_t)q * D, best + (size_t)w * D, ids)))
            w = q;
    return w;
}

/* ------------------------------------------------------------------------ */
/* The constraint language (Design Philosophy and Constraints)               */
/* ------------------------------------------------------------------------ */
/* Rules that restrict the expressions allowed as descriptors (a reading of
 * the paper's rules on variable combinations and functional forms, its
 * complexity limits and the target-unit filter):
 *   complexity    the number of operator nodes of the expression (a
 *                 primary has 0, op(f) has 1 + c(f), op(f, g) has
 *                 1 + c(f) + c(g)) is at most max_cplx (-1: no limit);
 *   nesting       nest[o] bit c set: operator c may not be the top operator
 *                 of a direct operand of operator o (e.g. exp of exp);
 *   variables     forb[u] bit v set: primaries u and v (both < 64) may not
 *                 appear together in one expression;
 *   target unit   (target_on) the expression's unit vector equals tunit
 *                 (scaled by 2^R as the unit vectors are).
 * The first three are hereditary: an expression is allowed only if every
 * sub-expression is.  Rules restrict which candidates can be selected; they
 * do not change the search space, its unit-valid counts or the values of
 * any candidate.  allowed[t] = 1 for an allowed record of an enumeration
 * (records list their operands first); uout are or_units' vectors. */
void or_rules(int64_t N, const int8_t* op, const int64_t* a, const int64_t* b, int max_cplx,
              const uint32_t* nest, const uint64_t* forb, int target_on, int B, const int32_t* uout,
              const uint8_t* legal, const int32_t* tunit, uint8_t* allowed) {
    int32_t* cplx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(N > 0 ? N : 1));
    uint64_t* vars = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(N > 0 ? N : 1));
    uint8_t* ok = (uint8_t*)malloc((size_t)(N > 0 ? N : 1));
    for (int64_t t = 0; t < N; t++) {
        if (op[t] == OP_NONE) {
            cplx[t] = 0;
            vars[t] = t < 64 ? (uint64_t)1 << t : 0;
            ok[t] = 1;
        } else {
            const int64_t ia = a[t], ib = b[t];
            cplx[t] = 1 + cplx[ia] + (ib >= 0 ? cplx[ib] : 0);
            vars[t] = vars[ia] | (ib >= 0 ? vars[ib] : 0);
            int good = ok[ia] && (ib < 0 || ok[ib]);
            if (max_cplx >= 0 && cplx[t] > max_cplx) good = 0;
            if (op[ia] != OP_NONE && (nest[op[t]] >> op[ia] & 1u)) good = 0;
            if (ib >= 0 && op[ib] != OP_NONE && (nest[op[t]] >> op[ib] & 1u)) good = 0;
            if (ib >= 0)
                for (int u = 0; u < 64; u++)
                    if ((vars[ia] >> u & 1u) && (forb[u] & vars[ib])) good = 0;
            ok[t] = (uint8_t)good;
        }
        int al = ok[t];
        if (al && target_on) {
            if (!legal[t]) al = 0;
            for (int k = 0; k < B && al; k++) al = uout[t * B + k] == tunit[k];
        }
        allowed[t] = (uint8_t)al;
    }
    free(cplx);
    free(vars);
    free(ok);
}
