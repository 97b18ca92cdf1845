// Simulated annealing over D-subsets of a subspace, the stochastic search
// the paper names for the sparsifying step (Software Description) when the
// exhaustive L0 of Eq. (1) (Core Optimization Objective) is out of reach:
// D > 3, or subspaces too large for every subset.
//
// Chains are independent: one lane runs one chain (thousands of chains keep
// the CUs busy; a chain's steps are a dependent sequence of gathers from
// the correlation matrix and a small Cholesky).  The rules, which an
// implementation elsewhere can follow to reproduce a trajectory bit for bit:
//
//   energy   E(a) = 1 - c_a^T C_aa^{-1} c_a for the subset array a, by a
//            Cholesky of C_aa in array order (pivot <= 1e-10: singular,
//            E = +inf), C and c the correlations of the rows and target;
//   move     position p = draw mod D, row r = draw mod S; a row already in
//            the subset leaves the state unchanged;
//   accept   E' <= E, or u < exp(-(E' - E) / T), u = (draw >> 11) 2^-53;
//            T = T0 alpha^k, formed by one multiplication per proposal;
//   best     per chain the smallest E seen (ties: the smaller sorted
//            candidate-ID tuple); per problem the best over chains.
//
// Random numbers are SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) used
// counter-based: chain q's key is output q + 1 of the stream with state
// seed, its draw c is output c + 1 of the stream with state key.  Random
// starts use draws 0, 1, ... (repeats skipped); proposal k uses draws
// 2^40 + 3k (position), + 1 (row), + 2 (uniform).
//
// Every operation that decides a move is one IEEE double operation with
// one rounding: this file is compiled with -ffp-contract=off, correlations
// are left-to-right sums over samples, and exp(-x) is the range reduction
// x = k ln 2 + r with the degree-18 Taylor series of exp(-r) in Horner form.
#include "dsc_internal.h"

#include <string>

namespace dsc {
namespace {

constexpr uint64_t SM_GAMMA = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint64_t sm_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Output i (i >= 1) of the SplitMix64 stream with state x0.
__device__ __forceinline__ uint64_t sm_at(uint64_t x0, uint64_t i) { return sm_mix(x0 + i * SM_GAMMA); }

__device__ __forceinline__ double exp_neg(double x) {
    if (!(x < 700.0)) return 0.0;
    if (x <= 0.0) return 1.0;
    const double LN2 = 0.6931471805599453;
    const double INV_LN2 = 1.4426950408889634;
    const int k = (int)(x * INV_LN2);
    const double t = (double)k * LN2;
    const double r = x - t;
    double p = 1.0;
#pragma unroll
    for (int i = 18; i >= 1; i--) {
        double q = p * -r;
        q = q / (double)i;
        p = 1.0 + q;
    }
    return ldexp(p, -k);
}

struct SaArgs {
    int n, S, ldz;
    const double* F;
    int64_t ldf;
    const double* y;
    const int64_t* ids;
    double* Zt;               // [n][ldz] centred values, sample-major (S rows + the target)
    double* nrm;              // [S + 1]
    double* C;                // [S][S]
    double* c;                // [S]
    const int32_t* init;      // [D] or NULL
    int32_t* chain_rows;      // [chains][D] best rows per chain, ascending
    double* chain_e;          // [chains]
    int32_t* out_rows;        // [D]
    double* out_e;
};

// Row i of the problem (i = S: the target): mean and centred values as
// left-to-right sums, norm = sqrt(sum of squares).  One thread per row.
__global__ __launch_bounds__(256) void k_sa_prep(ctab<SaArgs> A) {
    const SaArgs& a = tab(A, blockIdx.y);
    DSC_GLOBAL(a.F); DSC_GLOBAL(a.y); DSC_GLOBAL(a.Zt); DSC_GLOBAL(a.nrm);
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i > a.S) return;
    const double* f = i < a.S ? a.F + (int64_t)i * a.ldf : a.y;
    double s = 0.0;
    for (int t = 0; t < a.n; t++) s = s + f[t];
    const double m = s / (double)a.n;
    double q = 0.0;
    for (int t = 0; t < a.n; t++) {
        const double d = f[t] - m;
        a.Zt[(int64_t)t * a.ldz + i] = d;
        q = q + d * d;
    }
    a.nrm[i] = sqrt(q);
}

// C[i][j] = (left-to-right sum of z_i z_j) / (nrm_i nrm_j), and c[i] for
// j = S.  A block takes CI consecutive rows i and 256 columns j; each thread
// keeps CI independent sequential sums, so every entry is summed in sample
// order while the rows' values are read once per block (scalar loads).
constexpr int CI = 16;

__global__ __launch_bounds__(256) void k_sa_corr(ctab<SaArgs> A) {
    const SaArgs& a = tab(A, blockIdx.z);
    DSC_GLOBAL(a.Zt); DSC_GLOBAL(a.nrm); DSC_GLOBAL(a.C); DSC_GLOBAL(a.c);
    const int i0 = blockIdx.y * CI;
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (i0 >= a.S || blockIdx.x * 256 > a.S) return;
    const int jj = min(j, a.S);
    double d[CI];
#pragma unroll
    for (int k = 0; k < CI; k++) d[k] = 0.0;
    for (int t = 0; t < a.n; t++) {
        const double* zt = a.Zt + (int64_t)t * a.ldz;
        const double zj = zt[jj];
#pragma unroll
        for (int k = 0; k < CI; k++) d[k] = d[k] + zt[min(i0 + k, a.S)] * zj;
    }
    if (j > a.S) return;
    const double nj = a.nrm[j];
#pragma unroll
    for (int k = 0; k < CI; k++) {
        const int i = i0 + k;
        if (i >= a.S) break;
        const double ni = a.nrm[i];
        const double v = ni > 0.0 && nj > 0.0 ? d[k] / (ni * nj) : 0.0;
        if (j < a.S) a.C[(int64_t)i * a.S + j] = v;
        else a.c[i] = v;
    }
}

template <int D>
__device__ __forceinline__ double energy(const double* __restrict__ C, const double* __restrict__ c, int S,
                                         const int* a) {
    double L[D][D], w[D];
#pragma unroll
    for (int j = 0; j < D; j++) {
        double d = C[(int64_t)a[j] * S + a[j]];
#pragma unroll
        for (int k = 0; k < j; k++) d = d - L[j][k] * L[j][k];
        if (!(d > 1e-10)) return INFINITY;
        const double ljj = sqrt(d);
        L[j][j] = ljj;
#pragma unroll
        for (int i = j + 1; i < D; i++) {
            double v = C[(int64_t)a[i] * S + a[j]];
#pragma unroll
            for (int k = 0; k < j; k++) v = v - L[i][k] * L[j][k];
            L[i][j] = v / ljj;
        }
    }
    double ex = 0.0;
#pragma unroll
    for (int j = 0; j < D; j++) {
        double v = c[a[j]];
#pragma unroll
        for (int k = 0; k < j; k++) v = v - L[j][k] * w[k];
        w[j] = v / L[j][j];
        ex = ex + w[j] * w[j];
    }
    return 1.0 - ex;
}

// The same energy for a chain that keeps its factor: M holds C[a_i][a_j]
// (i >= j) of the current subset, L its Cholesky factor and w the forward
// solution.  A proposal that replaces a[p] reloads only the D correlations
// of the new row; of the factor only row p (columns before p) and the
// columns from p on change, and each entry is recomputed with exactly the
// operations of the full computation (same values, bit for bit), as are
// the forward solution and the explained fraction from p on.
template <int D>
struct Factor {
    double M[D][D], L[D][D], w[D], ex[D + 1];   // ex[j]: explained fraction of rows < j
    bool ok[D + 1];                             // ok[j]: rows < j non-singular
};

template <int D>
__device__ __forceinline__ void factor_from(Factor<D>& f, int p) {
#pragma unroll
    for (int j = 0; j < D; j++) {
        if (j < p) {
            // columns before p: only row p's entry depends on the new row
            if (!f.ok[j + 1]) continue;
            double v = f.M[p][j];
#pragma unroll
            for (int k = 0; k < j; k++) v = v - f.L[p][k] * f.L[j][k];
            f.L[p][j] = v / f.L[j][j];
            continue;
        }
        f.ok[j + 1] = false;
        if (!f.ok[j]) continue;
        double d = f.M[j][j];
#pragma unroll
        for (int k = 0; k < j; k++) d = d - f.L[j][k] * f.L[j][k];
        if (!(d > 1e-10)) continue;
        const double ljj = sqrt(d);
        f.L[j][j] = ljj;
#pragma unroll
        for (int i = j + 1; i < D; i++) {
            double v = f.M[i][j];
#pragma unroll
            for (int k = 0; k < j; k++) v = v - f.L[i][k] * f.L[j][k];
            f.L[i][j] = v / ljj;
        }
        f.ok[j + 1] = true;
    }
}

// Forward solution and explained fraction from row p on, as far as the
// factor is non-singular (a singular subset keeps them for its leading
// rows, which a later proposal may reuse).
template <int D>
__device__ __forceinline__ double solve_from(Factor<D>& f, const double* __restrict__ c, const int* a, int p) {
#pragma unroll
    for (int j = 0; j < D; j++) {
        if (j < p) continue;
        if (!f.ok[j + 1]) break;
        double v = c[a[j]];
#pragma unroll
        for (int k = 0; k < j; k++) v = v - f.L[j][k] * f.w[k];
        f.w[j] = v / f.L[j][j];
        f.ex[j + 1] = f.ex[j] + f.w[j] * f.w[j];
    }
    return f.ok[D] ? 1.0 - f.ex[D] : INFINITY;
}

template <int D>
__device__ __forceinline__ void sort_rows(int* s) {
#pragma unroll
    for (int i = 1; i < D; i++)
#pragma unroll
        for (int j = i; j > 0; j--)
            if (s[j] < s[j - 1]) { const int t = s[j]; s[j] = s[j - 1]; s[j - 1] = t; }
}

// Sorted candidate-ID tuple of rows a before that of rows b.
template <int D>
__device__ __forceinline__ bool ids_before(const int* a, const int* b, const int64_t* __restrict__ ids) {
    int64_t ia[D], ib[D];
#pragma unroll
    for (int i = 0; i < D; i++) { ia[i] = ids[a[i]]; ib[i] = ids[b[i]]; }
#pragma unroll
    for (int i = 1; i < D; i++)
#pragma unroll
        for (int j = i; j > 0; j--) {
            if (ia[j] < ia[j - 1]) { const int64_t t = ia[j]; ia[j] = ia[j - 1]; ia[j - 1] = t; }
            if (ib[j] < ib[j - 1]) { const int64_t t = ib[j]; ib[j] = ib[j - 1]; ib[j - 1] = t; }
        }
#pragma unroll
    for (int i = 0; i < D; i++)
        if (ia[i] != ib[i]) return ia[i] < ib[i];
    return false;
}

struct SaRun {
    int Q;
    int64_t K;
    double T0, alpha;
    uint64_t seed;
};

// One lane = one chain; grid (chain blocks, problems).
template <int D>
__global__ __launch_bounds__(256) void k_sa_run(ctab<SaArgs> A, SaRun R) {
    const SaArgs& g = tab(A, blockIdx.y);
    DSC_GLOBAL(g.C); DSC_GLOBAL(g.c); DSC_GLOBAL(g.ids); DSC_GLOBAL(g.init); DSC_GLOBAL(g.chain_rows); DSC_GLOBAL(g.chain_e);
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= R.Q) return;
    const int S = g.S;
    const uint64_t key = sm_at(R.seed, (uint64_t)q + 1);
    int a[D], b[D], bs[D];
    bool use_init = g.init != nullptr;
    if (use_init) {                          // distinct rows in 0..S-1, else a random start
#pragma unroll
        for (int j = 0; j < D; j++) {
            a[j] = g.init[j];
            use_init = use_init && a[j] >= 0 && a[j] < S;
#pragma unroll
            for (int i = 0; i < j; i++) use_init = use_init && a[i] != a[j];
        }
    }
    if (!use_init) {
        uint64_t ctr = 0;
#pragma unroll
        for (int j = 0; j < D; j++) {
            for (;;) {
                const int r = (int)(sm_at(key, ++ctr) % (uint64_t)S);
                bool dup = false;
#pragma unroll
                for (int i = 0; i < j; i++) dup |= a[i] == r;
                if (!dup) { a[j] = r; break; }
            }
        }
    }
    // the factor of the current subset
    Factor<D> f;
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; j <= i; j++) f.M[i][j] = g.C[(int64_t)a[i] * S + a[j]];
    f.ok[0] = true;
    f.ex[0] = 0.0;
    factor_from<D>(f, 0);
    double E = solve_from<D>(f, g.c, a, 0);
    double bE = E;
#pragma unroll
    for (int j = 0; j < D; j++) bs[j] = a[j];
    sort_rows<D>(bs);
    double T = R.T0;
    const uint64_t base = (uint64_t)1 << 40;
    for (int64_t k = 0; k < R.K; k++) {
        const uint64_t c0 = base + 3 * (uint64_t)k;
        const int p = (int)(sm_at(key, c0 + 1) % (uint64_t)D);
        const int r = (int)(sm_at(key, c0 + 2) % (uint64_t)S);
        const double u = (double)(sm_at(key, c0 + 3) >> 11) * 0x1.0p-53;
        bool in = false;
#pragma unroll
        for (int j = 0; j < D; j++) in |= a[j] == r;
        if (!in) {
#pragma unroll
            for (int j = 0; j < D; j++) b[j] = j == p ? r : a[j];
            Factor<D> h = f;
#pragma unroll
            for (int j = 0; j < D; j++) {              // row / column p of the new subset
                const double v = g.C[(int64_t)r * S + b[j]];
                if (j <= p) h.M[p][j] = v;
                if (j >= p) h.M[j][p] = v;
            }
            factor_from<D>(h, p);
            const double En = solve_from<D>(h, g.c, b, p);
            bool acc = En <= E;
            if (!acc && En < INFINITY) acc = u < exp_neg((En - E) / T);
            if (acc) {
#pragma unroll
                for (int j = 0; j < D; j++) a[j] = b[j];
                f = h;
                E = En;
                int sa[D];
#pragma unroll
                for (int j = 0; j < D; j++) sa[j] = a[j];
                sort_rows<D>(sa);
                if (E < bE || (E == bE && ids_before<D>(sa, bs, g.ids))) {
                    bE = E;
#pragma unroll
                    for (int j = 0; j < D; j++) bs[j] = sa[j];
                }
            }
        }
        T = T * R.alpha;
    }
#pragma unroll
    for (int j = 0; j < D; j++) g.chain_rows[(int64_t)q * D + j] = bs[j];
    g.chain_e[q] = bE;
}

// The best chain of each problem, in chain order with the same tie rule
// (one thread per problem).
template <int D>
__global__ __launch_bounds__(64) void k_sa_pick(ctab<SaArgs> A, int nb, int Q) {
    const int b = blockIdx.x * 64 + threadIdx.x;
    if (b >= nb) return;
    const SaArgs& g = tab(A, b);
    DSC_GLOBAL(g.chain_rows); DSC_GLOBAL(g.chain_e); DSC_GLOBAL(g.out_rows); DSC_GLOBAL(g.out_e); DSC_GLOBAL(g.ids);
    int w = 0;
    for (int q = 1; q < Q; q++) {
        const double eq = g.chain_e[q], ew = g.chain_e[w];
        if (eq < ew || (eq == ew && ids_before<D>(g.chain_rows + (int64_t)q * D, g.chain_rows + (int64_t)w * D, g.ids)))
            w = q;
    }
    for (int j = 0; j < D; j++) g.out_rows[j] = g.chain_rows[(int64_t)w * D + j];
    *g.out_e = g.chain_e[w];
}

template <int D>
void launch_run(ctab<SaArgs> A, int nb, const SaRun& R, hipStream_t st) {
    k_sa_run<D><<<dim3((unsigned)cdiv(R.Q, 256), nb), 256, 0, st>>>(A, R);
    k_sa_pick<D><<<(unsigned)cdiv(nb, 64), 64, 0, st>>>(A, nb, R.Q);
}

}  // namespace
}  // namespace dsc

extern "C" discover_status discover_l0_anneal(discover_ctx* ctx, const discover_l0_problem* probs,
                                              int32_t n_problems, int32_t D,
                                              const discover_anneal_params* prm,
                                              const int32_t* init_active, int32_t* out_subsets,
                                              double* out_rmse, double* out_coef, double* out_energy,
                                              int32_t* out_chain_subsets, double* out_chain_energy,
                                              double* out_resid, int64_t ldr, void* stream) {
    using namespace dsc;
    return guarded([&] {
        DSC_REQUIRE(ctx && probs && prm && n_problems >= 1 && n_problems <= 65535, "ctx/probs/prm/n_problems");
        DSC_REQUIRE(D >= 1 && D <= DISCOVER_MAX_D, "D = %d outside 1..%d", D, DISCOVER_MAX_D);
        DSC_REQUIRE(prm->chains >= 1 && prm->chains <= (1 << 20), "chains = %d outside 1..2^20", prm->chains);
        DSC_REQUIRE(prm->steps >= 0, "steps < 0");
        DSC_REQUIRE(prm->T0 >= 0.0 && prm->T0 < INFINITY, "T0 must be finite and >= 0");
        DSC_REQUIRE(prm->alpha > 0.0 && prm->alpha <= 1.0, "alpha outside (0, 1]");
        DSC_REQUIRE(out_subsets && out_rmse && out_coef && out_energy, "outputs required");
        for (int b = 0; b < n_problems; b++) {
            const discover_l0_problem& p = probs[b];
            DSC_REQUIRE(p.S >= D && p.S <= 16384, "problem %d: S = %d outside D..16384", b, p.S);
            DSC_REQUIRE(p.n >= D + 2, "problem %d: n = %d < D + 2", b, p.n);
            DSC_REQUIRE(p.F && p.ids && p.y && p.ldf >= p.n, "problem %d: F/ids/y/ldf", b);
            DSC_REQUIRE(!out_resid || ldr >= p.n, "problem %d: ldr < n", b);
        }
        DSC_HIP(hipSetDevice(ctx->device));
        const hipStream_t st = (hipStream_t)stream;
        CallMode mode(ctx, stream_capturing(st), false);
        const int Q = prm->chains;
        std::vector<SaArgs> sa(n_problems);
        int Smax = 0, nmax = 0;
        for (int b = 0; b < n_problems; b++) {
            const discover_l0_problem& p = probs[b];
            const std::string sfx = std::to_string(b) + ctx->tag;
            SaArgs& a = sa[b];
            a = SaArgs{};
            a.n = p.n; a.S = p.S; a.ldz = (int)cdiv(p.S + 1, 64) * 64;
            a.F = p.F; a.ldf = p.ldf; a.y = p.y; a.ids = p.ids;
            a.Zt = ctx->buf<double>("sa_Zt" + sfx, (size_t)p.n * a.ldz);
            a.nrm = ctx->buf<double>("sa_nrm" + sfx, (size_t)p.S + 1);
            a.C = ctx->buf<double>("sa_C" + sfx, (size_t)p.S * p.S);
            a.c = ctx->buf<double>("sa_c" + sfx, (size_t)p.S);
            a.init = init_active ? init_active + (int64_t)b * D : nullptr;
            a.chain_rows = out_chain_subsets ? out_chain_subsets + (int64_t)b * Q * D
                                             : ctx->buf<int32_t>("sa_rows" + sfx, (size_t)Q * D);
            a.chain_e = out_chain_energy ? out_chain_energy + (int64_t)b * Q
                                         : ctx->buf<double>("sa_e" + sfx, (size_t)Q);
            a.out_rows = out_subsets + (int64_t)b * D;
            a.out_e = out_energy + b;
            Smax = std::max(Smax, p.S);
            nmax = std::max(nmax, p.n);
        }
        const ctab<SaArgs> dA = ct(ctx->upload("sa_args", sa, st));
        {
            KTimer kt(ctx, st, "anneal_corr");
            k_sa_prep<<<dim3((unsigned)cdiv(Smax + 1, 256), n_problems), 256, 0, st>>>(dA);
            k_sa_corr<<<dim3((unsigned)cdiv(Smax + 1, 256), (unsigned)cdiv(Smax, CI), n_problems), 256, 0, st>>>(dA);
            check_launch("k_sa_corr");
        }
        const SaRun R{Q, prm->steps, prm->T0, prm->alpha, prm->seed};
        {
            KTimer kt(ctx, st, "anneal");
            switch (D) {
            case 1: launch_run<1>(dA, n_problems, R, st); break;
            case 2: launch_run<2>(dA, n_problems, R, st); break;
            case 3: launch_run<3>(dA, n_problems, R, st); break;
            case 4: launch_run<4>(dA, n_problems, R, st); break;
            case 5: launch_run<5>(dA, n_problems, R, st); break;
            case 6: launch_run<6>(dA, n_problems, R, st); break;
            case 7: launch_run<7>(dA, n_problems, R, st); break;
            default: launch_run<8>(dA, n_problems, R, st); break;
            }
            check_launch("k_sa_run");
        }
        fit_rows(ctx, probs, n_problems, D, out_subsets, D, out_coef, D + 1, out_rmse, out_resid, ldr, st);
    });
}
