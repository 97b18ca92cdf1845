/*
 * discover.h -- C ABI of the MI355X (gfx950) hot path of the DISCOVER /
 * SISSO-style symbolic regression method (arXiv 2602.06986).
 *
 * The method (Software Description; Figure 1 caption) generates candidate
 * expressions from primary features and an operator library, screens them
 * against the target, and selects a sparse linear model solving the
 * L0-constrained least squares of Eq. (1) (Core Optimization Objective).
 * Dimensional consistency prunes candidates during generation
 * (Physics-Informed Constraints).  Three calls cover that path:
 *
 *   discover_generate_screen  enumerate + unit-prune + screen + exact top-k
 *   discover_l0_fit           exhaustive L0 over all D-subsets of a subspace
 *   discover_omp              orthogonal matching pursuit over a subspace
 *
 * Conventions shared by every call
 *   - Pointers documented as "device" are HIP device memory on the
 *     context's device; "host" pointers are ordinary host memory.  The
 *     caller owns every input and output buffer; the library never frees
 *     caller memory.  The context owns only its internal workspace.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is
 *     enqueued on it.  Screening and L0 pool sizes are data dependent, so
 *     how a call waits depends on where its stats go:
 *       * out_stats NULL or host memory: the call waits for the stream,
 *         regrows any pool that overflowed and runs again, and returns with
 *         its results complete;
 *       * out_stats device memory: the call does not wait.  It runs once at
 *         the sizes that an earlier call of the same shape (parameters,
 *         sizes, units; not the data) settled on, and each problem's
 *         stats.status reports, on the device, DISCOVER_OK or why the
 *         outputs are not valid (E_CAPACITY: a pool was too small for this
 *         data, so run the call once with host stats to grow it;
 *         E_NUMERIC).  The first call of a shape sizes its pools as a host
 *         call does, waiting once; discover_reserve does that ahead of time.
 *     discover_omp never waits.  The outputs are valid once the stream has
 *     completed the work.  A context's calls must be ordered (one stream, or
 *     streams the caller orders): they share the context's workspace.
 *   - Graph capture: a screening, L0 or OMP call made on a stream that the
 *     caller is capturing (hipStreamBeginCapture, torch.cuda.graph) is
 *     recorded into the caller's graph.  It must pass out_stats in device
 *     memory, and a call of the same shape must have run outside capture
 *     first (or discover_reserve), else it returns E_CAPACITY.  The library
 *     may allocate workspace and upload argument tables through a private
 *     stream while the capture runs: capture in relaxed mode
 *     (hipStreamCaptureModeRelaxed; torch: capture_error_mode="relaxed").
 *     Every replay recomputes the outputs and stats from the inputs'
 *     current contents.  Workspace that a captured graph references is
 *     never freed while the context lives: a later call that would have to
 *     grow it returns E_CAPACITY (reserve first, or use a separate
 *     context).  Destroy the graph before the context.
 *   - Errors: every argument is validated before any launch; on error the
 *     call returns a negative discover_status, writes no output, and
 *     discover_last_error() describes the failure.  No C++ exception or
 *     abort crosses the ABI.
 *   - A context is not thread-safe; separate contexts are independent.
 *
 * Candidate IDs.  Rung 0 holds the p primary features (ID = column).  Rung
 * r >= 1 holds, in this order: one block per enabled unary operator
 * (exp, log, sqrt, sq, inv) applied to every rung r-1 feature in index
 * order, then one block per enabled binary operator (add, sub, mul, div,
 * rdiv) over every pair (i, j) with j in rung r-1 (increasing) and i in
 * the partner pool (increasing): i < j inside P_{r-1} by default, or all of
 * P_pool for an operator-limited rung.  add = f_i + f_j, sub = f_i - f_j,
 * mul = f_i f_j, div = f_i / f_j, rdiv = f_j / f_i.  The ID of a candidate
 * is its position in this list; IDs never depend on data or pruning.
 */
#ifndef DISCOVER_H
#define DISCOVER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DISCOVER_OK = 0,
    DISCOVER_E_ARG = -1,          /* invalid argument (nothing launched) */
    DISCOVER_E_NOMEM = -2,        /* device workspace allocation failed */
    DISCOVER_E_HIP = -3,          /* a HIP runtime call failed */
    DISCOVER_E_UNSUPPORTED = -4,  /* valid but not implemented combination */
    DISCOVER_E_NUMERIC = -5,      /* e.g. a constant target column */
    DISCOVER_E_CAPACITY = -6      /* an internal pool could not be grown */
} discover_status;

/* Operator bits (library order). */
#define DISCOVER_OP_EXP  (1u << 0)
#define DISCOVER_OP_LOG  (1u << 1)
#define DISCOVER_OP_SQRT (1u << 2)
#define DISCOVER_OP_SQ   (1u << 3)
#define DISCOVER_OP_INV  (1u << 4)
#define DISCOVER_OP_ADD  (1u << 5)
#define DISCOVER_OP_SUB  (1u << 6)
#define DISCOVER_OP_MUL  (1u << 7)
#define DISCOVER_OP_DIV  (1u << 8)
#define DISCOVER_OP_RDIV (1u << 9)
#define DISCOVER_OPS_ALL 0x3FFu

#define DISCOVER_SCORE_PER_TARGET 0   /* one top-k list per target column */
#define DISCOVER_SCORE_MAX        1   /* one list scored by max_t |r_t| */

#define DISCOVER_FP64        0        /* FP64 screening */
#define DISCOVER_BF16_GUARD  1        /* BF16 MFMA screening + FP64 rescore of a guard band */
#define DISCOVER_FP16_GUARD  2        /* FP16 MFMA screening + FP64 rescore of a guard band */

#define DISCOVER_MAX_RUNG    3
#define DISCOVER_MAX_UNITS   8
#define DISCOVER_MAX_TARGETS 16
#define DISCOVER_MAX_D       8

typedef struct discover_ctx discover_ctx;

/* Create a context bound to HIP device `device`.  *out receives the
 * handle.  Errors: E_ARG (bad device or NULL out), E_HIP. */
discover_status discover_create(int device, discover_ctx** out);

/* Release the context and its workspace (NULL is ignored). */
void discover_destroy(discover_ctx* ctx);

/* Text of the last error on the calling thread; valid until the next call
 * on this thread.  Never NULL. */
const char* discover_last_error(void);

/* One dataset.  Arrays of these form a batched call. */
typedef struct {
    int32_t n;                /* samples, >= 3 */
    int32_t p;                /* primary features, 1..4096 */
    int32_t T;                /* target / residual columns, 1..DISCOVER_MAX_TARGETS */
    int32_t B;                /* base units, 0..DISCOVER_MAX_UNITS (0: dimensionless) */
    const double* X;          /* device, feature-major: X[f * ldx + s] */
    int64_t ldx;              /* >= n */
    const double* Y;          /* device, Y[t * ldy + s] */
    int64_t ldy;              /* >= n */
    const int32_t* units;     /* host, units[f * B + b] integer exponents; NULL when B = 0 */
    const int64_t* exclude;   /* device, IDs already in the subspace (their duplicate
                                 groups are not selected again); may be NULL */
    int32_t n_exclude;        /* entries in exclude, >= 0 */
} discover_problem;

/* Screening parameters (shared by every problem of a call). */
typedef struct {
    uint32_t ops;             /* enabled operators (DISCOVER_OP_* bits) */
    int32_t rung;             /* R, 0..DISCOVER_MAX_RUNG */
    uint32_t rung_ops[4];     /* rung_ops[r] (r = 1..R): operators of rung r; 0 = ops */
    int32_t rung_pool[4];     /* rung_pool[r]: binary partners drawn from P_pool; -1 = r-1 */
    int32_t k;                /* selected features per list, >= 1 */
    int32_t score_mode;       /* DISCOVER_SCORE_PER_TARGET or DISCOVER_SCORE_MAX */
    int32_t precision;        /* DISCOVER_FP64, DISCOVER_BF16_GUARD or DISCOVER_FP16_GUARD */
    int32_t dedup;            /* 1: duplicate groups are merged (default); 0: off */
    int32_t tile_j;           /* FP64 dense pair kernel tile width: 0 = autotuned
                                 (default), or 1, 2, 4 operand features per wave
                                 (capped by what the target count allows); the
                                 scores do not depend on it */
    int32_t lp_pairs;         /* precision forms, pair candidates of rungs <= 2: 0 = the
                                 MFMA form or the FP64 tiles, whichever the autotuner
                                 times faster for the shape (default); 1 = always the
                                 MFMA form; -1 = always FP64.  The selection does not
                                 depend on it */
    int32_t sched;            /* FP64 dense pair tiles: 0 = autotuned (default), 1 = one
                                 persistent launch whose blocks take tiles from a device
                                 work queue (heaviest first), -1 = one block per tile.
                                 The scores do not depend on it */
} discover_screen_params;

/* Per-problem counters of one screening call (host memory). */
typedef struct {
    int64_t n_raw;            /* |P_R|: every enumerated candidate */
    int64_t n_unit_valid;     /* candidates passing the unit rules */
    int64_t n_scored;         /* candidates with a finite, non-constant value vector */
    int64_t pool_size;        /* candidates in the selection pools (summed over lists);
                                 exactly rescored are those of them whose screening
                                 score plus the margin reaches a lower bound of the
                                 K-th exact score */
    int64_t pool_rounds;      /* pool enlargements needed (0 normally) */
    int64_t n_merged;         /* duplicates merged into an earlier group */
    int64_t n_selected;       /* selected features (summed over lists) */
    double  max_lowprec_err;  /* precision forms: max |s_lowprec - s_fp64| over the pool */
    double  guard_band;       /* precision forms: the guard half-width used */
    int32_t tile_j;           /* FP64 dense pair kernel: operand features per wave,
                                 chosen by timing 1/2/4 on the first call for a
                                 search space (0 when that kernel did not run) */
    int32_t status;           /* DISCOVER_OK, or (device stats) E_CAPACITY / E_NUMERIC:
                                 this problem's outputs are not valid */
} discover_screen_stats;

/* Enumerate the candidates of P_R (rungs 0..R), drop those failing the unit
 * rules (add/sub need equal exponent vectors, exp/log a dimensionless
 * argument, sqrt halves, sq doubles, inv negates, mul/div add/subtract
 * exponents; a candidate with an invalid operand is invalid), evaluate
 * every remaining candidate on the fly, and screen it by |Pearson r|
 * against each target column (SIS of the cited SISSO method; Summary and
 * Figure 1 caption).  A candidate is scored when all of its n values are
 * finite and its standard deviation exceeds 1e-8 of its root-mean-square
 * value.  Selection is exact: candidates ordered by (-score, ID);
 * duplicates (|corr| >= 1 - 1e-9 with scores within 1e-9 relative) merge
 * into one group represented by its smallest ID; groups containing an
 * excluded ID are dropped; the first k groups are returned.
 *
 *   probs      host array of n_problems problem descriptions
 *   prm        host, screening parameters
 *   out_ids    device int64 [n_problems][T'][k], T' = T (PER_TARGET) or 1 (MAX);
 *              ordered by (-score, ID); unused entries -1
 *   out_scores device double, same shape: FP64 |r| (or max_t |r_t|); unused NaN
 *   out_values device double [n_problems][T'][k][ldv] values of the selected
 *              features, or NULL
 *   ldv        >= max n when out_values is not NULL
 *   out_stats  host or device, n_problems entries, or NULL (see the conventions:
 *              device stats make the call asynchronous and capturable)
 * Errors: E_ARG, E_NUMERIC (constant target), E_NOMEM, E_HIP,
 * E_UNSUPPORTED (rung 3 without an operator-limited partner pool),
 * E_CAPACITY (captured before a call of this shape ran). */
discover_status discover_generate_screen(discover_ctx* ctx, const discover_problem* probs,
                                         int32_t n_problems, const discover_screen_params* prm,
                                         int64_t* out_ids, double* out_scores,
                                         double* out_values, int64_t ldv,
                                         discover_screen_stats* out_stats, void* stream);

/* One subspace for the sparsifying step. */
typedef struct {
    int32_t n;                /* samples */
    int32_t S;                /* subspace rows, >= D */
    const double* F;          /* device, F[row * ldf + s]: values of the subspace features */
    int64_t ldf;              /* >= n */
    const int64_t* ids;       /* device [S] candidate IDs of the rows (tie-breaks) */
    const double* y;          /* device [n] target */
} discover_l0_problem;

typedef struct {
    int64_t n_subsets;        /* C(S, D) */
    int64_t n_band;           /* subsets refitted by Householder QR */
    int64_t n_singular;       /* (informational) 0 when not counted */
    int32_t status;           /* DISCOVER_OK, or (device stats) E_CAPACITY (the band
                                 overflowed) / E_NUMERIC (no non-singular subset) */
    int32_t reserved;
} discover_l0_stats;

/* Exhaustive L0 (Eq. (1), Core Optimization Objective) with an intercept:
 * every D-subset of the S rows is a support; its least-squares residual
 * sum of squares RSS = ||y - beta0 - F_sub^T beta||^2.  Subsets whose
 * normalized Cholesky pivot (centered, unit-norm columns, in row order)
 * is <= 1e-10 are rank-deficient and skipped.  The scan uses the
 * correlation matrix (per-thread Schur / Cholesky solves); every subset
 * within 1e-7 (explained fraction) of the m-th best is refitted by FP64
 * Householder QR on the raw data, and models are ranked by the QR RSS,
 * values within 1e-11 ||y - mean||^2 counting as tied (smallest sorted
 * candidate-ID tuple first).
 *
 *   D            1..3
 *   m            models returned per problem, 1..64
 *   out_subsets  device int32 [n_problems][m][D] row indices, ascending; -1 if absent
 *   out_rmse     device double [n_problems][m] sqrt(RSS / n)
 *   out_coef     device double [n_problems][m][D+1], intercept first, then the rows in
 *                ascending order
 *   out_resid    device double [n_problems][m][ldr] residuals y - prediction, or NULL
 *   out_stats    host or device [n_problems], or NULL (device: asynchronous, capturable;
 *                a call with no earlier call of its shape starts from the default
 *                band size)
 * Errors: E_ARG, E_NUMERIC (constant y, or no non-singular subset), E_NOMEM, E_HIP. */
discover_status discover_l0_fit(discover_ctx* ctx, const discover_l0_problem* probs,
                                int32_t n_problems, int32_t D, int32_t m,
                                int32_t* out_subsets, double* out_rmse, double* out_coef,
                                double* out_resid, int64_t ldr,
                                discover_l0_stats* out_stats, void* stream);

/* Orthogonal matching pursuit (cited OMP, Software Description) over the
 * rows of each problem: starting from init_active, repeatedly add the row
 * with the largest |sum_s (f_s - mean f) r_s| / ||f - mean f|| (ties: the
 * smaller candidate ID) and refit y on [1, active rows] by Householder QR,
 * until D_max rows are active.
 *
 *   init_active  device int32 [n_problems][n_init] warm start (rows), or NULL (n_init = 0);
 *                a row outside 0..S-1 or already listed is dropped, and the model then
 *                ends with fewer than D_max rows
 *   out_active   device int32 [n_problems][D_max] rows in order of addition (-1 past the
 *                model's rows)
 *   out_coef     device double [n_problems][D_max+1], intercept first, then the rows
 *                in order of addition
 *   out_rmse     device double [n_problems]
 *   out_resid    device double [n_problems][ldr] or NULL
 * The call does not wait for the stream (the method has no data-dependent
 * sizes here) and can be captured.
 * Errors: E_ARG (D_max > S or D_max > DISCOVER_MAX_D), E_NOMEM, E_HIP. */
discover_status discover_omp(discover_ctx* ctx, const discover_l0_problem* probs,
                             int32_t n_problems, int32_t D_max,
                             const int32_t* init_active, int32_t n_init,
                             int32_t* out_active, double* out_coef, double* out_rmse,
                             double* out_resid, int64_t ldr, void* stream);

/* Constraint rules on the expressions that may be selected (Design
 * Philosophy and Constraints: rules on variable combinations and functional
 * forms, complexity limits, a target-unit filter).  The first three are
 * hereditary: an expression is allowed only if every sub-expression is.
 *   max_complexity  operator nodes of the expression at most this (a primary
 *                   has 0, op(f) 1 + c(f), op(f, g) 1 + c(f) + c(g)); -1: none
 *   forbid_nest[o]  bit c (DISCOVER_OP_* order): operator c may not be the top
 *                   operator of a direct operand of operator o (e.g. exp(exp(f)))
 *   forbid_pairs    host [n_forbid_pairs][2]: primaries (index < 64) that may
 *                   not appear together in one expression
 *   target_unit     1: the expression's unit vector must equal target_units
 *                   (exponents over each problem's B base units)
 * Rules restrict selection only: candidates are still generated, screened
 * and counted as before (stats are unchanged), and an operand feature stays
 * usable inside larger expressions subject to the hereditary rules. */
typedef struct {
    int32_t max_complexity;
    uint32_t forbid_nest[10];
    int32_t n_forbid_pairs;
    const int32_t* forbid_pairs;
    int32_t target_unit;
    int32_t target_units[8];
} discover_rules;

/* Rules for every later screening call on this context (copied; NULL
 * clears them).  Waits for the device; graphs captured and selection sizes
 * memoised before are discarded.
 * Errors: E_ARG, E_HIP. */
discover_status discover_set_rules(discover_ctx* ctx, const discover_rules* rules);

/* Parameters of the annealing search (discover_l0_anneal). */
typedef struct {
    int32_t chains;           /* independent chains per problem, 1..2^20 (thousands fill the GPU) */
    int32_t reserved;         /* 0 */
    int64_t steps;            /* proposals per chain, >= 0 */
    double T0;                /* initial temperature, in units of the energy 1 - R^2, >= 0 */
    double alpha;             /* cooling factor per proposal, 0 < alpha <= 1 */
    uint64_t seed;            /* random stream (SplitMix64, counter-based) */
} discover_anneal_params;

/* Simulated annealing over D-subsets of each subspace (a stochastic search
 * for the L0 problem of Eq. (1), Core Optimization Objective; named among
 * the search strategies in Software Description), for D up to 8 or
 * subspaces too large for exhaustive L0.  Each of `chains` independent
 * chains starts from init_active (the same rows for every chain) or from
 * random rows, and makes `steps` proposals: replace the row at a uniform
 * position by a uniform row (a row already in the subset: no move), accept
 * when the energy E = 1 - R^2 of the fit of y on [1, rows] does not rise, or
 * with probability exp(-(E' - E) / T), T = T0 alpha^k.  E comes from the
 * correlation matrix by Cholesky; a pivot <= 1e-10 makes the subset
 * singular (E = +inf).  Each chain keeps the best subset it visited (ties:
 * the smaller sorted candidate-ID tuple); the problem's result is the best
 * over chains, refitted by Householder QR.  Every rule, and the random
 * stream (chain q's key = output q + 1 of SplitMix64 with state seed; draw
 * c = output c + 1 with state key; random starts use draws 0, 1, ...,
 * proposal k uses draws 2^40 + 3k, + 1, + 2), is computed with one IEEE
 * rounding per operation, so the same seed gives the same result on every
 * run and on an implementation that follows the same rules.
 *
 *   probs            host [n_problems]; S <= 16384 rows, n >= D + 2
 *   D                1..DISCOVER_MAX_D
 *   init_active      device int32 [n_problems][D] distinct rows 0..S-1, or NULL (random
 *                    starts); a problem whose rows are not distinct and in range starts
 *                    randomly
 *   out_subsets      device int32 [n_problems][D] rows of the best subset, ascending
 *   out_rmse         device double [n_problems] sqrt(RSS / n) of its QR fit
 *   out_coef         device double [n_problems][D+1] intercept first, then the rows
 *   out_energy       device double [n_problems] its energy 1 - R^2 as the chains computed it
 *   out_chain_subsets device int32 [n_problems][chains][D] every chain's best, or NULL
 *   out_chain_energy device double [n_problems][chains], or NULL
 *   out_resid        device double [n_problems][ldr] residuals of the QR fit, or NULL
 * The call does not wait for the stream and can be captured.
 * Errors: E_ARG, E_NOMEM, E_HIP. */
discover_status discover_l0_anneal(discover_ctx* ctx, const discover_l0_problem* probs,
                                   int32_t n_problems, int32_t D, const discover_anneal_params* prm,
                                   const int32_t* init_active, int32_t* out_subsets, double* out_rmse,
                                   double* out_coef, double* out_energy, int32_t* out_chain_subsets,
                                   double* out_chain_energy, double* out_resid, int64_t ldr,
                                   void* stream);

/* Limits of the branch-and-bound search (discover_l0_bnb). */
typedef struct {
    int64_t max_nodes;        /* prefixes expanded before the search stops with E_CAPACITY; 0: no limit */
    int64_t reserved;         /* 0 */
} discover_bnb_params;

/* What one problem's branch-and-bound search did.  The counts depend on the
 * order in which the GPU happened to visit the tree; the result does not. */
typedef struct {
    int64_t n_subsets;        /* C(S, D) */
    int64_t n_nodes;          /* prefixes (partial subsets) expanded */
    int64_t n_bounds;         /* bound evaluations */
    int64_t n_leaves;         /* D-subsets whose explained fraction was computed */
    int64_t n_refit;          /* subsets refitted by Householder QR */
    int32_t m0;               /* trailing rows over which the bound is trusted (see below) */
    int32_t status;           /* DISCOVER_OK, E_CAPACITY (max_nodes reached), E_NUMERIC */
} discover_bnb_stats;

/* Exact L0 (Eq. (1), Core Optimization Objective, with an intercept) by
 * branch and bound on the correlation matrix, the exact alternative to
 * enumeration the paper names beside the stochastic searches (Software
 * Description): the same problem and result as discover_l0_fit (singular
 * subsets skipped, the band within 1e-7 of the m-th best refitted by QR,
 * ties within 1e-11 ||y - mean||^2 to the smallest sorted ID tuple) for D
 * up to 8, without visiting every subset.
 *
 * Subsets are grown row by row in ascending row order.  A prefix P whose
 * next row is j can only be completed from rows >= j, and the explained
 * fraction never falls when rows are added, so R^2(P + rows >= j) bounds
 * every subset below that branch; a branch whose bound is below the m-th
 * best fraction found so far (less a margin of 1e-6 + 1e-7) is cut, and
 * since the bound falls as j grows, so are all later siblings.  The bounds
 * come from one Cholesky factor of the correlation matrix in reverse row
 * order; once that factor meets a pivot <= 1e-6 (rows nearly dependent on
 * the rows after them), branches needing more of it are not cut (m0 in
 * the stats: the number of trailing rows it covers).  The search is exact;
 * how much of the tree it skips depends on the data (strongly planted
 * models: almost all of it; nearly collinear subspaces: less).
 *
 *   D, m           1..DISCOVER_MAX_D, 1..64
 *   S              D..2048
 *   prm            limits, or NULL for none
 *   out_*          as discover_l0_fit
 *   out_stats      host [n_problems], or NULL
 * The call waits for the stream (the host steers the search) and cannot be
 * captured.
 * Errors: E_ARG, E_CAPACITY (max_nodes), E_NUMERIC (constant y, or no
 * non-singular subset), E_NOMEM, E_HIP. */
discover_status discover_l0_bnb(discover_ctx* ctx, const discover_l0_problem* probs,
                                int32_t n_problems, int32_t D, int32_t m,
                                const discover_bnb_params* prm, int32_t* out_subsets,
                                double* out_rmse, double* out_coef, double* out_resid, int64_t ldr,
                                discover_bnb_stats* out_stats, void* stream);

/* discover_omp for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the same arguments, kernels and results, with the work buffers taken
 * from a fixed 64 MiB device array that the library holds on each GPU it
 * runs on (set up by discover_create) until the process ends.  The call
 * allocates nothing and creates no events; it does not wait for the
 * stream.  Work space per problem, in bytes (each term rounded up to 256):
 * 8 (S + 1) ceil16(n) + 2 (8 S) + 8 (D_max + 2) n, + 8 n when out_resid is
 * NULL, + 768; a call whose problems need more than 64 MiB in total fails with
 * E_ARG before any launch.  Every call on a GPU uses that GPU's one array
 * (whatever the context), so calls that overlap in time on one GPU, on
 * different streams or from different threads, race: order them.  Nothing
 * in the array needs to start at zero; it keeps the last call's contents.
 * Errors: as discover_omp. */
discover_status discover_omp_noalloc(discover_ctx* ctx, const discover_l0_problem* probs,
                                     int32_t n_problems, int32_t D_max,
                                     const int32_t* init_active, int32_t n_init,
                                     int32_t* out_active, double* out_coef, double* out_rmse,
                                     double* out_resid, int64_t ldr, void* stream);

/* The SISSO loop (cited SISSO method, Summary; iterative generation ->
 * screening -> sparsifying, Software Description) over a batch of datasets
 * of uneven n and p, as one sequence of batched launches: for d = 1..D
 * every dataset is screened (FP64 or the precision form of prm) against
 * its target (d = 1) or the residuals of its m best (d-1)-models (MAX
 * score when m > 1), the k selected features are appended to its
 * subspace (earlier selections and their duplicate groups excluded), and
 * exhaustive L0 (as discover_l0_fit) fits its target over all d-subsets.
 * With use_graph = 1 the first call with a given set of inputs and outputs
 * runs eagerly and then captures the sequence into a hipGraph; a later
 * call with the same pointers and sizes replays the graph, checks on the
 * device that every capacity held and every selection was complete, and
 * runs eagerly instead if not.  The call returns with results ready.
 *
 *   probs        host [n_problems]; T = 1 (Y = the target), no exclude list
 *   prm          score_mode DISCOVER_SCORE_PER_TARGET (the first dimension has one target)
 *   D, m         1..3 dimensions; models per dimension 1..DISCOVER_MAX_TARGETS
 *   out_ids      device int64 [n_problems][D][k]: the subspace rows in order
 *   out_scores   device double [n_problems][D][k]
 *   out_subsets  device int32 [n_problems][D][m][3] rows of the subspace (first d used, rest -1)
 *   out_rmse     device double [n_problems][D][m]
 *   out_coef     device double [n_problems][D][m][4] intercept first (first d+1 used, rest NaN)
 *   omp_D        0, or D < omp_D <= DISCOVER_MAX_D: the best D-model of each dataset is then
 *                extended by OMP (as discover_omp, warm start = its rows) over the subspace
 *   out_omp_active  device int32 [n_problems][omp_D] subspace rows (NULL when omp_D = 0)
 *   out_omp_coef    device double [n_problems][omp_D+1] intercept first (NULL when omp_D = 0)
 *   out_omp_rmse    device double [n_problems] (NULL when omp_D = 0)
 *   out_replayed host int32, or NULL: 1 when a captured graph was replayed, 0 when
 *                the call ran eagerly, -1 when it ran eagerly and capturing the graph
 *                for later calls failed (discover_last_error says why)
 * Errors: as discover_generate_screen and discover_l0_fit. */
discover_status discover_sisso_batch(discover_ctx* ctx, const discover_problem* probs,
                                     int32_t n_problems, const discover_screen_params* prm,
                                     int32_t D, int32_t m, int32_t use_graph,
                                     int64_t* out_ids, double* out_scores, int32_t* out_subsets,
                                     double* out_rmse, double* out_coef, int32_t omp_D,
                                     int32_t* out_omp_active, double* out_omp_coef,
                                     double* out_omp_rmse, int32_t* out_replayed, void* stream);

/* Sizes the context's workspace for later calls that must not wait or
 * allocate (device stats, graph capture): runs discover_generate_screen on
 * these problems and parameters with host stats (settling plans, tile
 * choices and selection pool sizes for this shape and data), then, for
 * every D in 1..D_max, discover_l0_fit with m models over stand-in
 * subspaces of D * k * T' rows (T' = T per target, 1 in MAX mode) of each
 * problem's n, and discover_omp up to DISCOVER_MAX_D rows over the last of
 * them.  Call it once per call shape to be captured.  Waits for the stream.
 *   D_max  0..3 (0: screening only);  m  1..64 when D_max > 0
 * Errors: as discover_generate_screen and discover_l0_fit; E_ARG while the
 * stream is capturing. */
discover_status discover_reserve(discover_ctx* ctx, const discover_problem* probs, int32_t n_problems,
                                 const discover_screen_params* prm, int32_t D_max, int32_t m,
                                 void* stream);

/* Initial capacity (entries per problem, >= 1) of the screening's exact
 * fix-up lists: candidates whose one-pass moments cannot be trusted (a
 * large mean-to-spread ratio, a sum that may have cancelled) are listed
 * and decided by the exact two-pass formula.  A screen that lists more
 * grows the capacity and runs again (in a captured graph the replay's
 * device-side check fails instead and the call reruns eagerly), so the
 * value only trades memory for reruns.  Default 4,194,304.
 * Errors: E_ARG. */
discover_status discover_set_fixup_capacity(discover_ctx* ctx, int64_t entries);

/* Number of raw candidates |P_R| of a search space (host only). */
int64_t discover_count(int32_t p, const discover_screen_params* prm);

/* Expression text of a candidate ID, e.g. "((x2 * x15) / x3)" (host only).
 * Writes at most len bytes including the terminator.  E_ARG on a bad ID. */
discover_status discover_decode(int32_t p, const discover_screen_params* prm, int64_t id,
                                char* buf, size_t len);

/* Kernel timing: when enabled, the named kernels are bracketed by HIP
 * events on the stream they are launched on.  discover_timing reports the
 * number of launches and the summed event time (ms) since the last reset
 * for one kernel name ("screen_pairs", "l0_sweep", ...). */
discover_status discover_set_timing(discover_ctx* ctx, int32_t enable);
/* Kernel names (comma-separated, e.g. "l0_sweep3"; NULL or "" for none)
 * whose launches are also bracketed by events inside graphs captured by
 * discover_sisso_batch, so that replays report their time while timing is
 * on.  Graphs captured before the change are discarded (recaptured on the
 * next call).  Event-record nodes cost some microseconds each: name only
 * the kernels to be measured. */
discover_status discover_set_graph_timing(discover_ctx* ctx, const char* names);
discover_status discover_timing(discover_ctx* ctx, const char* kernel, int64_t* launches,
                                double* total_ms);
discover_status discover_reset_timing(discover_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* DISCOVER_H */
