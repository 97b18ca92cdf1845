// Candidate generation + sure-independence screening + exact top-k on
// gfx950 (the screening step of the SISSO method cited in the Summary;
// candidate generation with unit pruning per the Software Description and
// Physics-Informed Constraints sections).
//
// Data layout in HBM (per problem):
//   operand features (unit-legal features below the streamed rung), compact
//   index c in [0, Mc):
//     Vf/Rf/Cf  [Mc][ldn]   feature-major values, 1/values, centered values
//     Vs/Rs/Cs  [n][ldm]    the same, sample-major (ldm = Mc rounded to 64)
//     mu, mur   [Mc]        mean of values / of reciprocals
//     valid     [Mc]        operand usable (finite, non-constant, valid operands)
//   targets: Yc [T][ldn] centered, Yn [Tp][ldn] centered and unit-norm
//            (rows >= T are zero padding), syy [T], ysum [Tp] = sum Yn
//   scores    [T'][N]       one FP64 slot per candidate (the ID below rung 3;
//                           unit-legal rung-3 pairs through the slot map):
//                             +s     score with |error| <= margin
//                             -u     error may be larger; u bounds s above
//                             NaN    invalid / unit-illegal / not computed
//
// The streamed rung is never materialised: each wave evaluates
// op(f_i, f_j) for its tile on the fly and keeps only moments in registers.
#include <functional>
#include "dsc_internal.h"
#include "dsc_select.h"
#include "dsc_space.h"
#include "dsc_r3.h"

#include <memory>
#include <type_traits>

namespace dsc {

constexpr double TAU_CONST = 1e-8;   // std <= TAU_CONST * rms  => constant
constexpr double TAU_NEAR = 1e-9;    // relative score window of a duplicate pair
constexpr double TAU_DUP = 1e-9;     // 1 - |corr| at or below which two features are duplicates
constexpr double KAPPA_MAX = 64.0;   // shifted-moment conditioning accepted without inflation
constexpr double TAU_CANCEL = 1e-10; // add/sub with rms <= TAU_CANCEL * operand rms => constant
constexpr double EPS64 = 1.1102230246251565e-16;

// ------------------------------------------------------------------ targets
// One block per target: two-pass mean, centered and unit-norm copies.
__device__ __forceinline__ void d_targets(int n, int T, const double* __restrict__ Y,
                                          int64_t ldy, int ldn, double* __restrict__ Yc,
                                          double* __restrict__ Yn, double* __restrict__ syy,
                                          double* __restrict__ ysum, int* __restrict__ bad) {
    const int t = blockIdx.x;
    __shared__ double red[4];
    const double* y = Y + (int64_t)t * ldy;
    auto block_sum = [&](double v) {
        v = wave_sum(v);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
        __syncthreads();
        double r = (red[0] + red[1]) + (red[2] + red[3]);
        __syncthreads();
        return r;
    };
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += y[i];
    const double m = block_sum(s) / n;
    double q = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        double d = y[i] - m;
        Yc[(int64_t)t * ldn + i] = d;
        q += d * d;
    }
    const double ss = block_sum(q);
    const double inv = 1.0 / sqrt(ss);
    double z = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        double v = (y[i] - m) * inv;
        Yn[(int64_t)t * ldn + i] = v;
        z += v;
    }
    const double zs = block_sum(z);
    if (threadIdx.x == 0) {
        syy[t] = ss;
        ysum[t] = zs;
        const double sd = sqrt(ss / n), rms = sqrt(ss / n + m * m);
        if (!(sd > TAU_CONST * rms) || !isfinite(ss)) atomicOr(bad, 1);
    }
}

struct TgtArgs {
    int n, T, ldn;
    const double* Y;
    int64_t ldy;
    double *Yc, *Yn, *syy, *ysum;
    int* bad;
};

// grid (targets, problems)
__global__ __launch_bounds__(256) void k_targets(ctab<TgtArgs> A) {
    const TgtArgs& a = tab(A, blockIdx.y);
    DSC_GLOBAL(a.Y); DSC_GLOBAL(a.Yc); DSC_GLOBAL(a.Yn); DSC_GLOBAL(a.syy); DSC_GLOBAL(a.ysum); DSC_GLOBAL(a.bad);
    if ((int)blockIdx.x >= a.T) return;
    d_targets(a.n, a.T, a.Y, a.ldy, a.ldn, a.Yc, a.Yn, a.syy, a.ysum, a.bad);
}

// ---------------------------------------------------------- materialisation
__device__ __forceinline__ double apply_op(int op, double a, double b) {
    switch (op) {
    case OP_EXP: return exp(a);
    case OP_LOG: return log(a);
    case OP_SQRT: return sqrt(a);
    case OP_SQ: return a * a;
    case OP_INV: return 1.0 / a;
    case OP_ADD: return a + b;
    case OP_SUB: return a - b;
    case OP_MUL: return a * b;
    case OP_DIV: return a / b;
    default: return b / a;   // OP_RDIV
    }
}

// Values of the operand features of one rung: c in [c0, c1).
__device__ __forceinline__ void d_mat_values(int n, int ldn, int c0, int c1, const double* __restrict__ X,
                             int64_t ldx, const int8_t* __restrict__ op,
                             const int32_t* __restrict__ ca, const int32_t* __restrict__ cb,
                             const int64_t* __restrict__ raw, double* __restrict__ Vf) {
    const int c = c0 + blockIdx.y;
    if (c >= c1) return;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int o = op[c];
    double v;
    if (o == OP_NONE) v = X[raw[c] * ldx + s];
    else {
        const double a = Vf[(int64_t)ca[c] * ldn + s];
        const double b = cb[c] >= 0 ? Vf[(int64_t)cb[c] * ldn + s] : 0.0;
        v = apply_op(o, a, b);
    }
    Vf[(int64_t)c * ldn + s] = v;
}

// One wave per operand feature of one rung: validity, mean, reciprocals,
// centered values.
__device__ __forceinline__ void d_mat_stats(int n, int ldn, int c0, int c1,
                                                   const int8_t* __restrict__ mop,
                                                   const int32_t* __restrict__ ca,
                                                   const int32_t* __restrict__ cb,
                                                   double* __restrict__ Vf, double* __restrict__ Rf,
                                                   double* __restrict__ Cf, double* __restrict__ mu,
                                                   double* __restrict__ mur, double* __restrict__ msq,
                                                   uint8_t* __restrict__ valid) {
    const int c = c0 + blockIdx.x * 4 + wave_id();
    const int lane = threadIdx.x & 63;
    if (c >= c1) return;
    const double* v = Vf + (int64_t)c * ldn;
    double s = 0.0, sr = 0.0;
    int bad = 0;
    for (int i = lane; i < n; i += 64) {
        const double x = v[i];
        const double r = 1.0 / x;
        Rf[(int64_t)c * ldn + i] = r;
        bad |= !isfinite(x);
        s += x;
        sr += r;
    }
    s = wave_sum(s);
    sr = wave_sum(sr);
    const int anybad = __any(bad);
    const double m = s / n;
    double q = 0.0;
    for (int i = lane; i < n; i += 64) {
        const double d = v[i] - m;
        Cf[(int64_t)c * ldn + i] = d;
        q += d * d;
    }
    q = wave_sum(q);
    // cancellation rule for sums and differences
    const int o = mop[c];
    double ff = 0.0, ab = 0.0;
    if ((o == OP_ADD || o == OP_SUB) && cb[c] >= 0) {
        const double* va = Vf + (int64_t)ca[c] * ldn;
        const double* vb = Vf + (int64_t)cb[c] * ldn;
        for (int i = lane; i < n; i += 64) {
            ff += v[i] * v[i];
            ab += va[i] * va[i] + vb[i] * vb[i];
        }
        ff = wave_sum(ff);
        ab = wave_sum(ab);
    }
    if (lane == 0) {
        bool ok = !anybad && isfinite(q);
        const double sd = sqrt(q / n), rms = sqrt(q / n + m * m);
        ok = ok && (sd > TAU_CONST * rms);
        if ((o == OP_ADD || o == OP_SUB) && cb[c] >= 0) ok = ok && !(ff <= TAU_CANCEL * TAU_CANCEL * ab);
        if (ca[c] >= 0) ok = ok && valid[ca[c]];
        if (cb[c] >= 0) ok = ok && valid[cb[c]];
        valid[c] = ok;
        mu[c] = m;
        mur[c] = sr / n;
        msq[c] = q / n + m * m;
    }
}

// Operand features of a problem, materialised rung by rung (level = rung).
struct MatArgs {
    int n, ldn, nlev;
    int rs[4];                // compact start of each materialised rung, + end
    const double* X;
    int64_t ldx;
    const int8_t* op;
    const int32_t *ca, *cb;
    const int64_t* raw;
    double *Vf, *Rf, *Cf, *mu, *mur, *msq;
    uint8_t* valid;
};

// grid (sample blocks, features of the level, problems)
__global__ void k_mat_values(ctab<MatArgs> A, int level) {
    const MatArgs& a = tab(A, blockIdx.z);
    DSC_GLOBAL(a.X); DSC_GLOBAL(a.op); DSC_GLOBAL(a.ca); DSC_GLOBAL(a.cb); DSC_GLOBAL(a.raw); DSC_GLOBAL(a.Vf);
    if (level >= a.nlev) return;
    d_mat_values(a.n, a.ldn, a.rs[level], a.rs[level + 1], a.X, a.ldx, a.op, a.ca, a.cb, a.raw, a.Vf);
}

// grid (feature blocks of 4, problems)
__global__ __launch_bounds__(256) void k_mat_stats(ctab<MatArgs> A, int level) {
    const MatArgs& a = tab(A, blockIdx.y);
    DSC_GLOBAL(a.op); DSC_GLOBAL(a.ca); DSC_GLOBAL(a.cb); DSC_GLOBAL(a.Vf); DSC_GLOBAL(a.Rf); DSC_GLOBAL(a.Cf); DSC_GLOBAL(a.mu); DSC_GLOBAL(a.mur); DSC_GLOBAL(a.msq); DSC_GLOBAL(a.valid);
    if (level >= a.nlev) return;
    d_mat_stats(a.n, a.ldn, a.rs[level], a.rs[level + 1], a.op, a.ca, a.cb, a.Vf, a.Rf, a.Cf, a.mu,
                a.mur, a.msq, a.valid);
}

// Feature-major [M][ldn] -> sample-major [n][ldm] (padding left as is).
__device__ __forceinline__ void d_transpose(int n, int M, int ldn, int ldm, const double* __restrict__ src,
                                            double* __restrict__ dst) {
    __shared__ double tile[32][33];
    const int c0 = blockIdx.y * 32, s0 = blockIdx.x * 32;
    for (int k = threadIdx.y; k < 32; k += 8) {
        const int c = c0 + k, s = s0 + threadIdx.x;
        tile[k][threadIdx.x] = (c < M && s < n) ? src[(int64_t)c * ldn + s] : 0.0;
    }
    __syncthreads();
    for (int k = threadIdx.y; k < 32; k += 8) {
        const int s = s0 + k, c = c0 + threadIdx.x;
        if (s < n && c < M) dst[(int64_t)s * ldm + c] = tile[threadIdx.x][k];
    }
}

struct TrArgs {
    int n, M, ldn, ldm;
    const double* src[3];
    double* dst[3];
};

// grid (sample tiles, feature tiles, 3 x problems)
__global__ void k_transpose(ctab<TrArgs> A) {
    const TrArgs& a = tab(A, blockIdx.z / 3);
    const int w = blockIdx.z % 3;
    DSC_GLOBAL(a.src[w]); DSC_GLOBAL(a.dst[w]);
    if ((int)blockIdx.x * 32 >= a.n || (int)blockIdx.y * 32 >= a.M) return;
    d_transpose(a.n, a.M, a.ldn, a.ldm, a.src[w], a.dst[w]);
}

// ----------------------------------------------- exact candidate evaluation
struct Ops {           // operand arrays of one problem
    const double* Vf;
    const double* Rf;
    int ldn;
};

struct Cand {
    int kind;          // 0 operand feature, 1 unary, 2 binary, 3 binary over a rung-2 operand
    int op;
    int ca, cb;        // compact operand indices (kind 3: ca = first operand)
    int op2, cc, cd;   // kind 3: rung-2 operand = op2(cc, cd) (cd = -1 for unary op2)
};

// Everything needed to rebuild a candidate from its ID on the device.
struct EvalCtx {
    SpaceDev sd;
    int streamed;                 // rung streamed by the pair kernels (operands below it in HBM)
    int stream3;                  // operator-limited rung 3 streamed on top of rung 2
    const int32_t* raw2c;         // raw -> compact operand index
    const uint8_t* valid;         // operand validity
    const uint8_t* r2_valid;      // stream3: validity of rung-2 features, by id - off[2]
    SlotMap sm;                   // score slot <-> ID
};

__device__ __forceinline__ double unary_value(int op, const Ops& o, int c, int s) {
    if (op == OP_INV) return o.Rf[(int64_t)c * o.ldn + s];         // = 1.0 / a
    return apply_op(op, o.Vf[(int64_t)c * o.ldn + s], 0.0);
}

__device__ __forceinline__ double cand_value(const Cand& c, const Ops& o, int s) {
    if (c.kind == 1) return unary_value(c.op, o, c.ca, s);
    const double a = o.Vf[(int64_t)c.ca * o.ldn + s];
    if (c.kind == 0) return a;
    if (c.kind == 2) return apply_op(c.op, a, o.Vf[(int64_t)c.cb * o.ldn + s]);
    const double f2 = c.cd < 0 ? unary_value(c.op2, o, c.cc, s)
                               : apply_op(c.op2, o.Vf[(int64_t)c.cc * o.ldn + s],
                                          o.Vf[(int64_t)c.cd * o.ldn + s]);
    return apply_op(c.op, a, f2);
}

// Decode an ID into an evaluable candidate; false when an operand is not an
// operand feature (unit-illegal) or is invalid.
__device__ __forceinline__ bool cand_of_id(const EvalCtx& e, int64_t id, Cand& c) {
    int rung, op;
    int64_t a, b;
    decode_id(e.sd, id, rung, op, a, b);
    c.op2 = OP_NONE; c.cc = -1; c.cd = -1;
    if (e.streamed == 0 || rung < e.streamed) {
        c.kind = 0; c.op = OP_NONE; c.ca = e.raw2c[id]; c.cb = -1;
        return c.ca >= 0 && e.valid[c.ca];
    }
    c.op = op;
    c.ca = e.raw2c[a];
    if (rung == 3 && e.stream3) {
        if (!e.r2_valid[b - e.sd.off[2]] || c.ca < 0 || !e.valid[c.ca]) return false;
        int r2, o2;
        int64_t k, l;
        decode_id(e.sd, b, r2, o2, k, l);
        c.kind = 3; c.cb = -1; c.op2 = o2; c.cc = e.raw2c[k]; c.cd = l >= 0 ? e.raw2c[l] : -1;
        return c.cc >= 0;
    }
    if (b < 0) {
        c.kind = 1; c.cb = -1;
        return c.ca >= 0 && e.valid[c.ca];
    }
    c.kind = 2;
    c.cb = e.raw2c[b];
    return c.ca >= 0 && c.cb >= 0 && e.valid[c.ca] && e.valid[c.cb];
}

// One slot of a counter-indexed list for every active lane of the wave
// (lane order), with a single atomic: for appends made inside divergent
// code, where the active lanes are exactly those that append.
__device__ __forceinline__ unsigned long long wave_slot(unsigned long long* ctr) {
    const uint64_t m = __builtin_amdgcn_ballot_w64(true);
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)m) - 1;
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(ctr, (unsigned long long)__popcll(m));
    base = __shfl(base, leader, 64);
    return base + (unsigned long long)__popcll(m & ((1ull << lane) - 1ull));
}

// Exact two-pass Pearson of one candidate against T centered targets by one
// wave.  Returns false when the candidate is not finite or is constant.
template <int TMAX>
__device__ bool wave_exact_r(const Cand& c, const Ops& o, int n, int T,
                             const double* __restrict__ Yc, const double* __restrict__ syy,
                             double* r, double* mean_out = nullptr, double* msq_out = nullptr,
                             double* __restrict__ vals = nullptr, double* sxx_out = nullptr) {
    const int lane = threadIdx.x & 63;
    double s = 0.0;
    int bad = 0;
    const bool addsub = (c.kind == 2 || c.kind == 3) && (c.op == OP_ADD || c.op == OP_SUB);
    double ff = 0.0, ab = 0.0;
    for (int i = lane; i < n; i += 64) {
        const double f = cand_value(c, o, i);
        bad |= !isfinite(f);
        s += f;
        if (vals) vals[i] = f;
        if (addsub) {
            const double a = o.Vf[(int64_t)c.ca * o.ldn + i];
            double b;
            if (c.kind == 2) b = o.Vf[(int64_t)c.cb * o.ldn + i];
            else b = c.cd < 0 ? unary_value(c.op2, o, c.cc, i)
                              : apply_op(c.op2, o.Vf[(int64_t)c.cc * o.ldn + i], o.Vf[(int64_t)c.cd * o.ldn + i]);
            ff += f * f;
            ab += a * a + b * b;
        }
    }
    if (__any(bad)) return false;
    if (addsub) {                                   // cancellation to rounding noise
        ff = wave_sum(ff);
        ab = wave_sum(ab);
        if (ff <= TAU_CANCEL * TAU_CANCEL * ab) return false;
    }
    const double m = wave_sum(s) / n;
    double sxx = 0.0, sxy[TMAX];
#pragma unroll
    for (int t = 0; t < TMAX; t++) sxy[t] = 0.0;
    for (int i = lane; i < n; i += 64) {
        const double d = cand_value(c, o, i) - m;
        sxx += d * d;
#pragma unroll
        for (int t = 0; t < TMAX; t++)
            if (t < T) sxy[t] += d * Yc[(int64_t)t * o.ldn + i];
    }
    sxx = wave_sum(sxx);
    if (!isfinite(sxx)) return false;
    const double sd = sqrt(sxx / n), rms = sqrt(sxx / n + m * m);
    if (!(sd > TAU_CONST * rms)) return false;
#pragma unroll
    for (int t = 0; t < TMAX; t++)
        if (t < T) r[t] = wave_sum(sxy[t]) / sqrt(sxx * syy[t]);
    if (mean_out) *mean_out = m;
    if (msq_out) *msq_out = sxx / n + m * m;
    if (sxx_out) *sxx_out = sxx;
    return true;
}

// Exact scores of an explicit candidate list (operand features and unary
// candidates of the streamed rung), written into the score slots.
struct ListItem {
    int64_t id;
    int32_t kind, op, ca, cb;
};

__device__ __forceinline__ void d_score_item(const ListItem it, Ops o, const uint8_t* __restrict__ valid,
                                             int n, int T, int mode, const double* __restrict__ Yc,
                                             const double* __restrict__ syy, int64_t N,
                                             double* __restrict__ scores, unsigned* nok,
                                             uint8_t* __restrict__ r2v, double* __restrict__ r2m,
                                             double* __restrict__ r2q, int64_t off2, int64_t off3);

// One wave per listed candidate (exact two-pass score).
__device__ __forceinline__ void d_score_list(const ListItem* __restrict__ items, int64_t m,
                                                    Ops o, const uint8_t* __restrict__ valid,
                                                    int n, int T, int mode,
                                                    const double* __restrict__ Yc,
                                                    const double* __restrict__ syy, int64_t N,
                                                    double* __restrict__ scores,
                                                    unsigned long long* __restrict__ nscored,
                                                    uint8_t* __restrict__ r2v, double* __restrict__ r2m,
                                                    double* __restrict__ r2q, int64_t off2, int64_t off3) {
    // the block's valid candidates are counted in LDS and added once
    __shared__ unsigned nok;
    if (threadIdx.x == 0) nok = 0u;
    __syncthreads();
    const int64_t w = (int64_t)blockIdx.x * 4 + wave_id();
    if (w < m) d_score_item(items[w], o, valid, n, T, mode, Yc, syy, N, scores, &nok, r2v, r2m, r2q,
                            off2, off3);
    __syncthreads();
    if (threadIdx.x == 0 && nok) atomicAdd(nscored, (unsigned long long)nok);
}

__device__ __forceinline__ void d_score_item(const ListItem it, Ops o, const uint8_t* __restrict__ valid,
                                             int n, int T, int mode, const double* __restrict__ Yc,
                                             const double* __restrict__ syy, int64_t N,
                                             double* __restrict__ scores, unsigned* nok,
                                             uint8_t* __restrict__ r2v, double* __restrict__ r2m,
                                             double* __restrict__ r2q, int64_t off2, int64_t off3) {
    Cand c{it.kind, it.op, it.ca, it.cb, OP_NONE, -1, -1};
    bool ok = valid[c.ca] && (c.kind < 2 || valid[c.cb]);
    if (c.kind == 0) ok = valid[c.ca];
    double r[DISCOVER_MAX_TARGETS], mean = 0.0, msq = 0.0;
    ok = ok && wave_exact_r<DISCOVER_MAX_TARGETS>(c, o, n, T, Yc, syy, r, &mean, &msq);
    if ((threadIdx.x & 63) == 0) {
        if (!ok) {
            for (int t = 0; t < (mode ? 1 : T); t++) scores[(int64_t)t * N + it.id] = __longlong_as_double(-1LL);
            return;
        }
        atomicAdd(nok, 1u);
        if (r2v && it.id >= off2 && it.id < off3) {
            r2v[it.id - off2] = 1;
            r2m[it.id - off2] = mean;
            r2q[it.id - off2] = msq;
        }
        if (mode == DISCOVER_SCORE_MAX) {
            double mx = 0.0;
            for (int t = 0; t < T; t++) mx = fmax(mx, fabs(r[t]));
            scores[it.id] = mx;
        } else {
            for (int t = 0; t < T; t++) scores[(int64_t)t * N + it.id] = fabs(r[t]);
        }
    }
}

struct ListArgs {
    const ListItem* items;
    int64_t m;
    Ops o;
    const uint8_t* valid;
    int n, T, mode;
    const double *Yc, *syy;
    int64_t N;
    double* scores;
    unsigned long long* nscored;
    uint8_t* r2v;
    double *r2m, *r2q;
    int64_t off2, off3;
};

// grid (item blocks of 4, problems)
__global__ __launch_bounds__(256) void k_score_list(ctab<ListArgs> A) {
    const ListArgs& a = tab(A, blockIdx.y);
    DSC_GLOBAL(a.items); DSC_GLOBAL(a.o.Vf); DSC_GLOBAL(a.o.Rf); DSC_GLOBAL(a.valid); DSC_GLOBAL(a.Yc); DSC_GLOBAL(a.syy); DSC_GLOBAL(a.scores); DSC_GLOBAL(a.nscored);
    if ((int64_t)blockIdx.x * 4 >= a.m) return;
    d_score_list(a.items, a.m, a.o, a.valid, a.n, a.T, a.mode, a.Yc, a.syy, a.N, a.scores, a.nscored,
                 a.r2v, a.r2m, a.r2q, a.off2, a.off3);
}

// --------------------------------------------------- streamed pair screen
// Tile of one wave: J operand features j (uniform) x 64 operand features i
// (one per lane).  For every (i, j) with i < j and every operator of OPS,
// the candidate value is formed on the fly, shifted by an estimate of its
// mean (exact for add/sub via centered operands, mu_a * mu_b style for the
// products) and accumulated into sum, sum of squares and T dot products
// with the unit-norm targets.
//
// OPS bits: 0 add, 1 sub, 2 mul, 3 div, 4 rdiv.
struct PairArgs {
    const int2* tiles;        // precision form: (jc, ic0) per wave
    const int32_t* ilist;     // explicit partner lists (list mode) or NULL
    int64_t n_tiles;
    int n, ldm, ldn, Mc, jc_end, i_end;   // i_end: end of the partner pool
    const double *Vs, *Rs, *Cs, *Vf, *Rf, *Cf, *mu, *mur;
    const uint8_t* valid;
    const int64_t* mat_raw;
    const double* Yn;
    const double* ysum;
    int T, mode, r;
    uint32_t opmask;          // runtime enabled subset of OPS (bits as above)
    SpaceDev sd;
    int64_t N;
    double* scores;
    unsigned long long* nscored;
    int64_t* fix_ids;         // candidates whose shifted moments are ill-conditioned
    unsigned long long* fix_cnt;
    int64_t fix_cap;
    uint8_t* r2v;             // rung-2 operand statistics for a streamed rung 3 (or NULL)
    double* r2m;
    double* r2q;
    const double* msq;        // mean square of every operand feature
};

// One block = one tile; its waves take consecutive parts of the samples and
// their partial moments are summed in LDS in a fixed order (wave 0 + wave 1
// + ...), so results do not depend on scheduling.  Dense tiles use 4 waves
// (enough of them fill the chip); the fewer list tiles use 8 (measured: the
// list kernel 26 % faster, the dense one 4 % slower with 8).
template <bool LIST>
constexpr int pair_split() { return LIST ? 8 : 4; }

// Tiles of every problem of a call form one list, heaviest first:
// (problem, jc0, ic0, -) dense or (problem, jc, list offset, count) in list
// mode; the problem's arguments are read from A.
constexpr int PAIR_SL = 8;                       // accumulators combined per LDS round

template <int OPS, int J, int TP, bool LIST>
__device__ __forceinline__ void pair_tile(ctab<PairArgs> A, const int4 tile) {
    constexpr int NOP = ((OPS >> 0) & 1) + ((OPS >> 1) & 1) + ((OPS >> 2) & 1) +
                        ((OPS >> 3) & 1) + ((OPS >> 4) & 1);
    constexpr int NV = J * NOP * (2 + TP);       // accumulators per lane
    constexpr int SL = PAIR_SL;
    constexpr int PAIR_SPLIT = pair_split<LIST>();
    __shared__ double red[PAIR_SPLIT - 1][SL][64];
    const PairArgs& g = tab(A, tile.x);
    DSC_GLOBAL(g.ilist); DSC_GLOBAL(g.Vs); DSC_GLOBAL(g.Rs); DSC_GLOBAL(g.Cs); DSC_GLOBAL(g.Vf); DSC_GLOBAL(g.Rf); DSC_GLOBAL(g.Cf); DSC_GLOBAL(g.mu); DSC_GLOBAL(g.mur); DSC_GLOBAL(g.valid);
    DSC_GLOBAL(g.mat_raw); DSC_GLOBAL(g.Yn); DSC_GLOBAL(g.ysum); DSC_GLOBAL(g.scores); DSC_GLOBAL(g.nscored); DSC_GLOBAL(g.fix_ids); DSC_GLOBAL(g.fix_cnt); DSC_GLOBAL(g.msq);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: scalar loop
    const int lane = threadIdx.x & 63;
    const int jc0 = tile.y;
    int i;
    bool lane_ok;
    if (LIST) {
        lane_ok = lane < tile.w;
        i = g.ilist[tile.z + (lane_ok ? lane : 0)];
    } else {
        i = tile.z + lane;
        lane_ok = i < g.i_end;
    }
    const int ic = lane_ok ? i : 0;
    const double mua = g.mu[ic], mura = g.mur[ic];
    const bool va = lane_ok && g.valid[ic];

    int jc[J];
    bool jok[J];
    double sh[J][NOP];
#pragma unroll
    for (int jj = 0; jj < J; jj++) {
        const int j = jc0 + jj;
        jok[jj] = j < g.jc_end;
        jc[jj] = jok[jj] ? j : jc0;
        const double mub = g.mu[jc[jj]], murb = g.mur[jc[jj]];
        int k = 0;
        if (OPS & 1) sh[jj][k++] = 0.0;                // add: centered operands
        if (OPS & 2) sh[jj][k++] = 0.0;                // sub
        if (OPS & 4) sh[jj][k++] = mua * mub;          // mul
        if (OPS & 8) sh[jj][k++] = mua * murb;         // div  = a * (1/b)
        if (OPS & 16) sh[jj][k++] = mura * mub;        // rdiv = b * (1/a)
    }
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) acc[v] = 0.0;
#define S1(jj, q) acc[((jj) * NOP + (q)) * (2 + TP)]
#define S2(jj, q) acc[((jj) * NOP + (q)) * (2 + TP) + 1]
#define DT(jj, q, t) acc[((jj) * NOP + (q)) * (2 + TP) + 2 + (t)]

    const double* __restrict__ Vs = g.Vs;
    const double* __restrict__ Rs = g.Rs;
    const double* __restrict__ Cs = g.Cs;
    const int chunk = (g.n + PAIR_SPLIT - 1) / PAIR_SPLIT;
    const int s_lo = min(g.n, wave * chunk), s_hi = min(g.n, s_lo + chunk);
#pragma unroll 2
    for (int s = s_lo; s < s_hi; s++) {
        const int64_t so = (int64_t)s * g.ldm + ic;
        const double a = (OPS & 28) ? Vs[so] : 0.0;
        const double ra = (OPS & 16) ? Rs[so] : 0.0;
        const double ac = (OPS & 3) ? Cs[so] : 0.0;
        double y[TP];
#pragma unroll
        for (int t = 0; t < TP; t++) y[t] = g.Yn[(int64_t)t * g.ldn + s];
#pragma unroll
        for (int jj = 0; jj < J; jj++) {
            const int64_t fo = (int64_t)jc[jj] * g.ldn + s;
            const double b = (OPS & 20) ? g.Vf[fo] : 0.0;
            const double rb = (OPS & 8) ? g.Rf[fo] : 0.0;
            const double bc = (OPS & 3) ? g.Cf[fo] : 0.0;
            double f[NOP];
            int k = 0;
            if (OPS & 1) { f[k] = ac + bc; k++; }
            if (OPS & 2) { f[k] = ac - bc; k++; }
            if (OPS & 4) { f[k] = fma(a, b, -sh[jj][k]); k++; }
            if (OPS & 8) { f[k] = fma(a, rb, -sh[jj][k]); k++; }
            if (OPS & 16) { f[k] = fma(ra, b, -sh[jj][k]); k++; }
#pragma unroll
            for (int q = 0; q < NOP; q++) {
                S1(jj, q) += f[q];
                S2(jj, q) = fma(f[q], f[q], S2(jj, q));
#pragma unroll
                for (int t = 0; t < TP; t++) DT(jj, q, t) = fma(f[q], y[t], DT(jj, q, t));
            }
        }
    }
    // combine the partial moments of the waves into wave 0
#pragma unroll
    for (int v0 = 0; v0 < NV; v0 += SL) {
        if (wave > 0) {
#pragma unroll
            for (int v = 0; v < SL; v++)
                if (v0 + v < NV) red[wave - 1][v][lane] = acc[v0 + v];
        }
        __syncthreads();
        if (wave == 0) {
#pragma unroll
            for (int v = 0; v < SL; v++)
                if (v0 + v < NV) {
                    double x = acc[v0 + v];
#pragma unroll
                    for (int w = 0; w < PAIR_SPLIT - 1; w++) x += red[w][v][lane];
                    acc[v0 + v] = x;
                }
        }
        __syncthreads();
    }
    if (wave != 0) return;                       // the epilogue is wave 0's

    const double nn = (double)g.n;
    const int64_t ria = g.mat_raw[ic];
    unsigned cnt = 0;
#pragma unroll
    for (int jj = 0; jj < J; jj++) {
        const bool pair_ok = va && jok[jj] && g.valid[jc[jj]] && (LIST || i < jc[jj]);
        const int64_t rjb = g.mat_raw[jc[jj]];
        const double mub = g.mu[jc[jj]], murb = g.mur[jc[jj]];
        int k = 0;
#pragma unroll
        for (int o = 0; o < 5; o++) {
            if (!((OPS >> o) & 1)) continue;
            const int q = k++;
            if (!((g.opmask >> o) & 1) || !(LIST ? lane_ok : (i < jc[jj]) && lane_ok && jok[jj]))
                continue;
            const int64_t id = pair_id(g.sd, g.r, OP_ADD + o, ria, rjb);
            double out[TP];
            const double S1v = S1(jj, q), S2v = S2(jj, q);
            const double m1 = S1v / nn;
            const double varn = S2v - S1v * m1;
            const double nanv = __longlong_as_double(-1LL);
            if (!pair_ok || !(S2v < INFINITY) || !(fabs(S1v) < INFINITY)) {   // invalid operand or non-finite value
                for (int t = 0; t < (g.mode ? 1 : g.T); t++) g.scores[(int64_t)t * g.N + id] = nanv;
                continue;
            }
            double kappa = varn > 0.0 ? S2v / varn : INFINITY;
            if (o < 2) {
                // a sum or difference that may have cancelled to rounding noise
                // is decided exactly as well
                const double c0 = o == 0 ? mua + mub : mua - mub;
                const double ff = S2v + 2.0 * c0 * S1v + nn * c0 * c0;
                if (ff <= 1e-12 * nn * (g.msq[ic] + g.msq[jc[jj]])) kappa = INFINITY;
            }
            if (!(kappa <= KAPPA_MAX)) {
                // the shift was far from the mean: decide exactly in the fix-up pass
                const unsigned long long slot = wave_slot(g.fix_cnt);
                if ((int64_t)slot < g.fix_cap) {
                    g.fix_ids[slot] = id;
                    for (int t = 0; t < (g.mode ? 1 : g.T); t++) g.scores[(int64_t)t * g.N + id] = nanv;
                    continue;
                }
            }
            double shift = sh[jj][q];
            if (o == 0) shift = mua + mub;
            if (o == 1) shift = mua - mub;
            const double mean = shift + m1;
            const bool nonconst = varn / nn > TAU_CONST * TAU_CONST * (varn / nn + mean * mean);
            if (kappa <= KAPPA_MAX && !nonconst) {
                for (int t = 0; t < (g.mode ? 1 : g.T); t++) g.scores[(int64_t)t * g.N + id] = nanv;
                continue;
            }
            const double isd = 1.0 / sqrt(varn);
            double best = 0.0;
#pragma unroll
            for (int t = 0; t < TP; t++) {
                out[t] = fabs((DT(jj, q, t) - S1v * g.ysum[t] / nn) * isd);
                if (t < g.T) best = fmax(best, out[t]);
            }
            const double err = 4.0 * nn * EPS64 * kappa;
            const bool precise = kappa <= KAPPA_MAX;
            cnt++;
            if (g.r2v && precise) {
                g.r2v[id - g.sd.off[2]] = 1;
                g.r2m[id - g.sd.off[2]] = mean;
                g.r2q[id - g.sd.off[2]] = varn / nn + mean * mean;
            }
            if (g.mode == DISCOVER_SCORE_MAX) {
                g.scores[id] = precise ? best : -(best + err);
            } else {
#pragma unroll
                for (int t = 0; t < TP; t++)
                    if (t < g.T)
                        g.scores[(int64_t)t * g.N + id] = precise ? out[t] : -(out[t] + err);
            }
            (void)murb;
        }
    }
    // wave-aggregated count of scored candidates
    unsigned long long tot = 0;
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor((int)cnt, o, 64);
    tot = cnt;
    if (lane == 0 && tot) atomicAdd(g.nscored, tot);
#undef S1
#undef S2
#undef DT
}

// One block per tile (grid = tiles), or, with QUEUE, a persistent grid
// whose blocks take tile after tile from a device work queue (an atomic
// counter over the list, which is ordered heaviest first) until it runs
// out.  Either way each tile is computed by one block in the same order of
// operations, so the scores do not depend on the schedule.
template <int OPS, int J, int TP, bool LIST, bool QUEUE>
__global__ __launch_bounds__(64 * pair_split<LIST>()) void k_screen_pairs(ctab<PairArgs> A,
                                                      const int4* __restrict__ tiles, int64_t n_tiles,
                                                      unsigned long long* __restrict__ queue) {
    if (!QUEUE) {
        pair_tile<OPS, J, TP, LIST>(A, tiles[blockIdx.x]);
        return;
    }
    __shared__ int64_t s_t;
    for (;;) {
        if (threadIdx.x == 0) s_t = (int64_t)atomicAdd(queue, 1ull);
        __syncthreads();
        const int64_t t = s_t;
        __syncthreads();
        if (t >= n_tiles) break;
        pair_tile<OPS, J, TP, LIST>(A, tiles[t]);
    }
}

// -------------------------------------------- reduced-precision screen
// SIS for many targets at once as a BF16/FP16 MFMA product with FP32
// accumulation over standardised values (the precision form).  Pass 1 gives
// each candidate's mean and standard deviation in FP64 (shifted moments as
// in the FP64 kernel); pass 2 forms z = (f - mean) / sd in FP64, rounds it
// to BF16/FP16 and multiplies it with the standardised targets on the
// matrix cores: r_t = sum_s zy[t][s] z[s] / n.
//
// MFMA v_mfma_f32_16x16x32_{bf16,f16}: A = targets (16 rows x 32 samples),
// B = candidates (32 samples x 16 columns), D (16 x 16, FP32).  Lane l
// supplies A[l%16][8(l/16)..+7] and B[8(l/16)..+7][l%16] and receives
// D[4(l/16)+e][l%16], e = 0..3.  So lane l evaluates candidate l%16 of each
// 16-wide group at samples 8(l/16)..+7 of every 32-sample chunk: the B
// operand is built in registers, no LDS staging.
//
// Error bound (guard half-width): standardised vectors have sum z^2 = n, so
// |r_lp - r| <= 2u + u^2 + gamma_n(FP32) (+2^-24 for FP16 subnormals), with
// u = 2^-8 (BF16) or 2^-11 (FP16); every candidate within 2 delta of the
// pool threshold is rescored in FP64.
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8_t;
typedef __attribute__((ext_vector_type(8))) _Float16 f16x8_t;
typedef __attribute__((ext_vector_type(4))) float f32x4_t;
typedef __attribute__((ext_vector_type(8))) float f32x8_t;
typedef __attribute__((ext_vector_type(4))) __bf16 bf16x4_t;

template <bool FP16>
struct LpVec;
template <>
struct LpVec<false> {
    typedef bf16x8_t T;
    static __device__ __forceinline__ __bf16 cvt(float x) { return (__bf16)x; }
    static __device__ __forceinline__ f32x4_t mma(T a, T b, f32x4_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <>
struct LpVec<true> {
    typedef f16x8_t T;
    static __device__ __forceinline__ _Float16 cvt(float x) { return (_Float16)x; }
    static __device__ __forceinline__ f32x4_t mma(T a, T b, f32x4_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

// Standardised targets in low precision: Ylp[t][s] = Yn[t][s] * sqrt(n)
// for t < T, 0 for padding rows and samples >= n.  ldl = n rounded to 32.
template <bool FP16>
__global__ void k_targets_lp(int n, int T, int ldn, int ldl, const double* __restrict__ Yn,
                             typename std::conditional<FP16, _Float16, __bf16>::type* __restrict__ Ylp) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int t = blockIdx.y;
    if (s >= ldl) return;
    const double v = (t < T && s < n) ? Yn[(int64_t)t * ldn + s] * sqrt((double)n) : 0.0;
    Ylp[(int64_t)t * ldl + s] = LpVec<FP16>::cvt((float)v);
}

// Layout of the kernel: one block (4 waves) = 64 operand features i (one
// per lane) x one operand feature j; the waves split the samples into
// 32-sample chunks.  Pass 1 gives the FP64 shifted moments as in the FP64
// kernel, summed over the waves in LDS in a fixed order.  Pass 2: each lane
// forms z for its candidate at a chunk's samples, rounds it and stores it in
// its wave's LDS area with the candidate's 32 values contiguous; the MFMA B
// operand of lane l (candidate 16g + l%16, samples 8(l/16)..+7) is then one
// 16-byte LDS read, and one MFMA per (operator, group of 16 candidates)
// accumulates the chunk.  The waves' FP32 products are summed in LDS in a
// fixed order; wave w then writes the scores of candidates 16w..16w+15.
constexpr int LPT_CH = 32;                 // samples per MFMA chunk

template <int OPS, bool FP16>
__global__ __launch_bounds__(256) void k_screen_lp(PairArgs g, const void* __restrict__ Ylp_, int ldl) {
    constexpr int NOP = ((OPS >> 0) & 1) + ((OPS >> 1) & 1) + ((OPS >> 2) & 1) +
                        ((OPS >> 3) & 1) + ((OPS >> 4) & 1);
    typedef typename LpVec<FP16>::T VT;
    typedef typename std::conditional<FP16, _Float16, __bf16>::type ET;
    __shared__ __align__(16) ET zs[4][NOP][64][LPT_CH];    // also the combine buffers
    __shared__ double okf[NOP][64][3];     // per candidate: flag, mean, variance
    const ET* __restrict__ Ylp = (const ET*)Ylp_;
    const int2 tile = g.tiles[blockIdx.x];
    const int wave = wave_id();
    const int lane = threadIdx.x & 63;
    const int jc = tile.x;                                 // one j per tile
    const int i = tile.y + lane;
    const bool iok = i < g.i_end && i < jc;
    const int ic = i < g.Mc ? i : 0;
    const double mub = g.mu[jc], murb = g.mur[jc];
    const double mua = g.mu[ic], mura = g.mur[ic];
    double sh[NOP];
    {
        int k = 0;
        if (OPS & 1) sh[k++] = 0.0;
        if (OPS & 2) sh[k++] = 0.0;
        if (OPS & 4) sh[k++] = mua * mub;
        if (OPS & 8) sh[k++] = mua * murb;
        if (OPS & 16) sh[k++] = mura * mub;
    }
    auto values = [&](int s, double f[NOP]) {
        const double b_ = g.Vf[(int64_t)jc * g.ldn + s];
        const double rb = g.Rf[(int64_t)jc * g.ldn + s];
        const double bc = g.Cf[(int64_t)jc * g.ldn + s];
        const int64_t so = (int64_t)s * g.ldm + ic;
        const double a = g.Vs[so], ra = g.Rs[so], ac = g.Cs[so];
        int k = 0;
        if (OPS & 1) { f[k] = ac + bc; k++; }
        if (OPS & 2) { f[k] = ac - bc; k++; }
        if (OPS & 4) { f[k] = fma(a, b_, -sh[k]); k++; }
        if (OPS & 8) { f[k] = fma(a, rb, -sh[k]); k++; }
        if (OPS & 16) { f[k] = fma(ra, b_, -sh[k]); k++; }
    };
    const int nch = (g.n + LPT_CH - 1) / LPT_CH;
    const int cpw = (nch + 3) / 4;                         // chunks per wave
    const int c0 = wave * cpw, c1 = min(nch, c0 + cpw);
    // pass 1: shifted moments over this wave's samples, summed over the waves
    double s1[NOP], s2[NOP];
#pragma unroll
    for (int q = 0; q < NOP; q++) { s1[q] = 0.0; s2[q] = 0.0; }
    const int s_hi = min(g.n, c1 * LPT_CH);
#pragma unroll 2
    for (int s = min(g.n, c0 * LPT_CH); s < s_hi; s++) {
        double f[NOP];
        values(s, f);
#pragma unroll
        for (int q = 0; q < NOP; q++) {
            s1[q] += f[q];
            s2[q] = fma(f[q], f[q], s2[q]);
        }
    }
    {
        double* red = (double*)&zs[0][0][0][0];             // [4][NOP][2][64]
#pragma unroll
        for (int q = 0; q < NOP; q++) {
            red[((wave * NOP + q) * 2 + 0) * 64 + lane] = s1[q];
            red[((wave * NOP + q) * 2 + 1) * 64 + lane] = s2[q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NOP; q++) {
            const double* r1 = red + (q * 2 + 0) * 64 + lane;
            const double* r2 = red + (q * 2 + 1) * 64 + lane;
            const int ws = NOP * 2 * 64;                   // stride between waves
            s1[q] = (r1[0] + r1[ws]) + (r1[2 * ws] + r1[3 * ws]);
            s2[q] = (r2[0] + r2[ws]) + (r2[2 * ws] + r2[3 * ws]);
        }
        __syncthreads();
    }
    const double nn = (double)g.n;
    double isd[NOP], cz[NOP];
#pragma unroll
    for (int q = 0; q < NOP; q++) {
        const double m1 = s1[q] / nn, varn = s2[q] - s1[q] * m1;
        const bool fin = (s2[q] < INFINITY) && (fabs(s1[q]) < INFINITY);
        double kappa = varn > 0.0 ? s2[q] / varn : INFINITY;
        if ((OPS & 3) && q < ((OPS & 1) + ((OPS >> 1) & 1))) {   // add / sub
            const bool isadd = (OPS & 1) && q == 0;
            const double c0_ = isadd ? mua + mub : mua - mub;
            const double ff = s2[q] + 2.0 * c0_ * s1[q] + nn * c0_ * c0_;
            if (ff <= 1e-12 * nn * (g.msq[ic] + g.msq[jc])) kappa = INFINITY;
        }
        bool ok = iok && g.valid[ic] && g.valid[jc] && fin;
        const bool fix = ok && !(kappa <= KAPPA_MAX);
        ok = ok && !fix;
        isd[q] = ok ? sqrt(nn / varn) : 0.0;               // 1 / population sd
        cz[q] = m1 * isd[q];
        if (wave == 0) {
            okf[q][lane][0] = ok ? 1.0 : fix ? 2.0 : 0.0;
            okf[q][lane][1] = sh[q] + m1;
            okf[q][lane][2] = varn / nn;
        }
    }
    // pass 2: low-precision products on the matrix cores
    f32x4_t acc[NOP][4];
#pragma unroll
    for (int q = 0; q < NOP; q++)
#pragma unroll
        for (int gq = 0; gq < 4; gq++) acc[q][gq] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    const int col = lane & 15, kb = lane >> 4;
    for (int c = c0; c < c0 + cpw; c++) {                  // every wave runs cpw chunks
        if (c < c1) {
            // 8 samples at a time: each operator's 8 rounded values leave in
            // one 16-byte LDS write
            for (int e0 = 0; e0 < LPT_CH; e0 += 8) {
                f32x8_t zf[NOP];
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    const int s = c * LPT_CH + e0 + u;
                    double f[NOP];
                    if (s < g.n) values(s, f);
#pragma unroll
                    for (int q = 0; q < NOP; q++)
                        zf[q][u] = s < g.n ? (float)fma(f[q], isd[q], -cz[q]) : 0.f;
                }
#pragma unroll
                for (int q = 0; q < NOP; q++)
                    *(VT*)&zs[wave][q][lane][e0] = __builtin_convertvector(zf[q], VT);
            }
        }
        __syncthreads();                                   // chunk written
        if (c < c1) {
            const VT ya = *(const VT*)(Ylp + (int64_t)col * ldl + LPT_CH * c + 8 * kb);
#pragma unroll
            for (int q = 0; q < NOP; q++)
#pragma unroll
                for (int gq = 0; gq < 4; gq++) {
                    const VT bv = *(const VT*)&zs[wave][q][16 * gq + col][8 * kb];
                    acc[q][gq] = LpVec<FP16>::mma(ya, bv, acc[q][gq]);
                }
        }
        __syncthreads();                                   // reads done before the next chunk
    }
    // sum the products of the 4 waves (fixed order); wave w keeps group w
    float* red = (float*)&zs[0][0][0][0];                  // [4 waves][NOP][4 groups][4][64]
#pragma unroll
    for (int q = 0; q < NOP; q++)
#pragma unroll
        for (int gq = 0; gq < 4; gq++)
#pragma unroll
            for (int e = 0; e < 4; e++)
                red[(((wave * NOP + q) * 4 + gq) * 4 + e) * 64 + lane] = acc[q][gq][e];
    __syncthreads();
    const int gq = wave;
    float rs[NOP][4];
#pragma unroll
    for (int q = 0; q < NOP; q++)
#pragma unroll
        for (int e = 0; e < 4; e++) {
            float x[4];
#pragma unroll
            for (int w2 = 0; w2 < 4; w2++) x[w2] = red[(((w2 * NOP + q) * 4 + gq) * 4 + e) * 64 + lane];
            rs[q][e] = (x[0] + x[1]) + (x[2] + x[3]);
        }
    // scores: lane holds r for targets 4kb..4kb+3 of candidate 16gq + col
    unsigned cnt = 0;
    const int cl = 16 * gq + col;
    const int ii = tile.y + cl;
    const bool cok = ii < g.i_end && ii < jc;
    const int icl = ii < g.Mc ? ii : 0;
    int k = 0;
#pragma unroll
    for (int o = 0; o < 5; o++) {
        if (!((OPS >> o) & 1)) continue;
        const int q = k++;
        double r[4];
        double mx = 0.0;
#pragma unroll
        for (int e = 0; e < 4; e++) {
            r[e] = fabs((double)rs[q][e]) / nn;
            if (4 * kb + e < g.T) mx = fmax(mx, r[e]);
        }
        mx = fmax(mx, __shfl_xor(mx, 16, 64));
        mx = fmax(mx, __shfl_xor(mx, 32, 64));
        if (!cok || !((g.opmask >> o) & 1)) continue;
        const int64_t id = pair_id(g.sd, g.r, OP_ADD + o, g.mat_raw[icl], g.mat_raw[jc]);
        const double nanv = __longlong_as_double(-1LL);
        const double flag = okf[q][cl][0];
        const bool ok = flag == 1.0;
        if (flag == 2.0) {
            if (kb == 0) {
                const unsigned long long slot = wave_slot(g.fix_cnt);
                if ((int64_t)slot < g.fix_cap) g.fix_ids[slot] = id;
                if (g.mode == DISCOVER_SCORE_MAX) g.scores[id] = nanv;
            }
            if (g.mode != DISCOVER_SCORE_MAX)
                for (int e = 0; e < 4; e++)
                    if (4 * kb + e < g.T) g.scores[(int64_t)(4 * kb + e) * g.N + id] = nanv;
            continue;
        }
        if (g.r2v && ok && kb == 0) {
            const double mua_ = g.mu[icl];
            const double mean_ = o == 0 ? (mua_ + mub) + okf[q][cl][1]
                               : o == 1 ? (mua_ - mub) + okf[q][cl][1] : okf[q][cl][1];
            const double var_ = okf[q][cl][2];
            g.r2v[id - g.sd.off[2]] = 1;
            g.r2m[id - g.sd.off[2]] = mean_;
            g.r2q[id - g.sd.off[2]] = var_ + mean_ * mean_;
        }
        if (g.mode == DISCOVER_SCORE_MAX) {
            if (kb == 0) {
                g.scores[id] = ok ? mx : nanv;
                cnt += ok;
            }
        } else {
            for (int e = 0; e < 4; e++)
                if (4 * kb + e < g.T) g.scores[(int64_t)(4 * kb + e) * g.N + id] = ok ? r[e] : nanv;
            if (kb == 0) cnt += ok;
        }
    }
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor((int)cnt, o, 64);
    if (lane == 0 && cnt) atomicAdd(g.nscored, (unsigned long long)cnt);
}

// Single-pass BF16 form.  The Pearson numerator does not need the mean:
// with centred targets, sum_s (f_s - c) y_s is the same for every constant
// c.  So each lane rounds the shifted value u = f - shift (the FP64
// kernel's shift estimate) to BF16 directly, while the same pass sums u and
// u^2 in FP64 for the variance.  With y standardised (sum y^2 = n),
// r = sum_s u_s y_s / sqrt(n var_n), and rounding u and y (and summing in
// FP32) changes r by at most delta * sqrt(kappa), kappa = sum u^2 / var_n
// (the same bound as for standardised values, scaled by the size of u
// relative to its spread).  A candidate with kappa <= LP1_KAPPA stores its
// score (error within the selection margin 1.1 delta); up to KAPPA_MAX it
// stores the upper bound -(s + delta sqrt(kappa)) (rescored exactly when it
// can reach the pool); beyond that it is decided by the FP64 fix-up pass.
// BF16 keeps FP32's exponent range, so u needs no scaling.
constexpr double LP1_KAPPA = 1.21;     // scores stored up to sqrt(kappa) = 1.1 (most shifts are close)

template <int OPS>
__global__ __launch_bounds__(256) void k_screen_lp1(PairArgs g, const void* __restrict__ Ylp_, int ldl,
                                                    double delta) {
    constexpr int NOP = ((OPS >> 0) & 1) + ((OPS >> 1) & 1) + ((OPS >> 2) & 1) +
                        ((OPS >> 3) & 1) + ((OPS >> 4) & 1);
    typedef bf16x8_t VT;
    __shared__ __align__(16) __bf16 zs[4][NOP][64][LPT_CH];    // also the combine buffers
    __shared__ double cst[NOP][64][5];     // per candidate: state, 1/sqrt(n var), kappa, variance, mean shift
    const __bf16* __restrict__ Ylp = (const __bf16*)Ylp_;
    const int2 tile = g.tiles[blockIdx.x];
    const int wave = wave_id();
    const int lane = threadIdx.x & 63;
    const int jc = tile.x;                                 // one j per tile
    const int i = tile.y + lane;
    const bool iok = i < g.i_end && i < jc;
    const int ic = i < g.Mc ? i : 0;
    const double mub = g.mu[jc], murb = g.mur[jc];
    const double mua = g.mu[ic], mura = g.mur[ic];
    double sh[NOP];
    {
        int k = 0;
        if (OPS & 1) sh[k++] = 0.0;
        if (OPS & 2) sh[k++] = 0.0;
        if (OPS & 4) sh[k++] = mua * mub;
        if (OPS & 8) sh[k++] = mua * murb;
        if (OPS & 16) sh[k++] = mura * mub;
    }
    const int nch = (g.n + LPT_CH - 1) / LPT_CH;
    const int cpw = (nch + 3) / 4;                         // chunks per wave
    const int c0 = wave * cpw, c1 = min(nch, c0 + cpw);
    double s1[NOP], s2[NOP];
    f32x4_t acc[NOP][4];
#pragma unroll
    for (int q = 0; q < NOP; q++) {
        s1[q] = 0.0;
        s2[q] = 0.0;
#pragma unroll
        for (int gq = 0; gq < 4; gq++) acc[q][gq] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    }
    const int col = lane & 15, kb = lane >> 4;
    for (int c = c0; c < c0 + cpw; c++) {                  // every wave runs cpw chunks
        if (c < c1) {
            for (int e0 = 0; e0 < LPT_CH; e0 += 4) {
                f32x4_t zf[NOP];
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const int s = c * LPT_CH + e0 + u;
                    double f[NOP];
                    if (s < g.n) {
                        const double b_ = g.Vf[(int64_t)jc * g.ldn + s];
                        const double rb = g.Rf[(int64_t)jc * g.ldn + s];
                        const double bc = g.Cf[(int64_t)jc * g.ldn + s];
                        const int64_t so = (int64_t)s * g.ldm + ic;
                        const double a = g.Vs[so], ra = g.Rs[so], ac = g.Cs[so];
                        int k = 0;
                        if (OPS & 1) { f[k] = ac + bc; k++; }
                        if (OPS & 2) { f[k] = ac - bc; k++; }
                        if (OPS & 4) { f[k] = fma(a, b_, -sh[k]); k++; }
                        if (OPS & 8) { f[k] = fma(a, rb, -sh[k]); k++; }
                        if (OPS & 16) { f[k] = fma(ra, b_, -sh[k]); k++; }
                    } else {
#pragma unroll
                        for (int q = 0; q < NOP; q++) f[q] = 0.0;
                    }
#pragma unroll
                    for (int q = 0; q < NOP; q++) {
                        s1[q] += f[q];
                        s2[q] = fma(f[q], f[q], s2[q]);
                        zf[q][u] = (float)f[q];
                    }
                }
#pragma unroll
                for (int q = 0; q < NOP; q++)
                    *(bf16x4_t*)&zs[wave][q][lane][e0] = __builtin_convertvector(zf[q], bf16x4_t);
            }
        }
        __syncthreads();                                   // chunk written
        if (c < c1) {
            const VT ya = *(const VT*)(Ylp + (int64_t)col * ldl + LPT_CH * c + 8 * kb);
#pragma unroll
            for (int q = 0; q < NOP; q++)
#pragma unroll
                for (int gq = 0; gq < 4; gq++) {
                    const VT bv = *(const VT*)&zs[wave][q][16 * gq + col][8 * kb];
                    acc[q][gq] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ya, bv, acc[q][gq], 0, 0, 0);
                }
        }
        __syncthreads();                                   // reads done before the next chunk
    }
    const double nn = (double)g.n;
    {
        // moments over the waves: (w0 + w1) + (w2 + w3)
        double* red = (double*)&zs[0][0][0][0];             // [4][NOP][2][64]
#pragma unroll
        for (int q = 0; q < NOP; q++) {
            red[((wave * NOP + q) * 2 + 0) * 64 + lane] = s1[q];
            red[((wave * NOP + q) * 2 + 1) * 64 + lane] = s2[q];
        }
        __syncthreads();
        if (wave == 0) {
            const int ws = NOP * 2 * 64;                   // stride between waves
#pragma unroll
            for (int q = 0; q < NOP; q++) {
                const double* r1 = red + (q * 2 + 0) * 64 + lane;
                const double* r2 = red + (q * 2 + 1) * 64 + lane;
                const double S1 = (r1[0] + r1[ws]) + (r1[2 * ws] + r1[3 * ws]);
                const double S2 = (r2[0] + r2[ws]) + (r2[2 * ws] + r2[3 * ws]);
                const double m1 = S1 / nn, varn = S2 - S1 * m1;
                const bool fin = (S2 < INFINITY) && (fabs(S1) < INFINITY);
                double kappa = varn > 0.0 ? S2 / varn : INFINITY;
                if ((OPS & 3) && q < ((OPS & 1) + ((OPS >> 1) & 1))) {   // add / sub
                    const bool isadd = (OPS & 1) && q == 0;
                    const double c0_ = isadd ? mua + mub : mua - mub;
                    const double ff = S2 + 2.0 * c0_ * S1 + nn * c0_ * c0_;
                    if (ff <= 1e-12 * nn * (g.msq[ic] + g.msq[jc])) kappa = INFINITY;
                }
                const bool ok = iok && g.valid[ic] && g.valid[jc] && fin;
                double shq = sh[q];
                if ((OPS & 1) && q == 0) shq = mua + mub;
                if ((OPS & 2) && q == (OPS & 1)) shq = mua - mub;
                const double mean = shq + m1;
                const bool nonconst = varn / nn > TAU_CONST * TAU_CONST * (varn / nn + mean * mean);
                // state: 0 invalid / constant, 1 precise, 2 upper bound, 3 fix-up
                double state = 0.0;
                if (ok && !(kappa <= KAPPA_MAX)) state = 3.0;
                else if (ok && nonconst) state = kappa <= LP1_KAPPA ? 1.0 : 2.0;
                cst[q][lane][0] = state;
                cst[q][lane][1] = state == 1.0 || state == 2.0 ? 1.0 / sqrt(nn * varn) : 0.0;
                cst[q][lane][2] = kappa;
                cst[q][lane][3] = varn / nn;
                cst[q][lane][4] = mean;
            }
        }
        __syncthreads();
    }
    // products over the waves (fixed order); wave w keeps group w
    float* fred = (float*)&zs[0][0][0][0];                 // [4 waves][NOP][4 groups][4][64]
#pragma unroll
    for (int q = 0; q < NOP; q++)
#pragma unroll
        for (int gq = 0; gq < 4; gq++)
#pragma unroll
            for (int e = 0; e < 4; e++)
                fred[(((wave * NOP + q) * 4 + gq) * 4 + e) * 64 + lane] = acc[q][gq][e];
    __syncthreads();
    const int gq = wave;
    float rs[NOP][4];
#pragma unroll
    for (int q = 0; q < NOP; q++)
#pragma unroll
        for (int e = 0; e < 4; e++) {
            float x[4];
#pragma unroll
            for (int w2 = 0; w2 < 4; w2++) x[w2] = fred[(((w2 * NOP + q) * 4 + gq) * 4 + e) * 64 + lane];
            rs[q][e] = (x[0] + x[1]) + (x[2] + x[3]);
        }
    // scores: lane holds the products for targets 4kb..4kb+3 of candidate 16gq + col
    unsigned cnt = 0;
    const int cl = 16 * gq + col;
    const int ii = tile.y + cl;
    const bool cok = ii < g.i_end && ii < jc;
    const int icl = ii < g.Mc ? ii : 0;
    int k = 0;
#pragma unroll
    for (int o = 0; o < 5; o++) {
        if (!((OPS >> o) & 1)) continue;
        const int q = k++;
        const double state = cst[q][cl][0], inv = cst[q][cl][1], kappa = cst[q][cl][2];
        double r[4];
        double mx = 0.0;
#pragma unroll
        for (int e = 0; e < 4; e++) {
            r[e] = fabs((double)rs[q][e]) * inv;
            if (4 * kb + e < g.T) mx = fmax(mx, r[e]);
        }
        mx = fmax(mx, __shfl_xor(mx, 16, 64));
        mx = fmax(mx, __shfl_xor(mx, 32, 64));
        if (!cok || !((g.opmask >> o) & 1)) continue;
        const int64_t id = pair_id(g.sd, g.r, OP_ADD + o, g.mat_raw[icl], g.mat_raw[jc]);
        const double nanv = __longlong_as_double(-1LL);
        if (state == 3.0) {
            if (kb == 0) {
                const unsigned long long slot = wave_slot(g.fix_cnt);
                if ((int64_t)slot < g.fix_cap) g.fix_ids[slot] = id;
                if (g.mode == DISCOVER_SCORE_MAX) g.scores[id] = nanv;
            }
            if (g.mode != DISCOVER_SCORE_MAX)
                for (int e = 0; e < 4; e++)
                    if (4 * kb + e < g.T) g.scores[(int64_t)(4 * kb + e) * g.N + id] = nanv;
            continue;
        }
        const bool ok = state == 1.0 || state == 2.0;
        const double ub = delta * sqrt(kappa);             // this candidate's error bound
        if (g.r2v && ok && kb == 0) {
            const double mean_ = cst[q][cl][4];
            const double var_ = cst[q][cl][3];
            g.r2v[id - g.sd.off[2]] = 1;
            g.r2m[id - g.sd.off[2]] = mean_;
            g.r2q[id - g.sd.off[2]] = var_ + mean_ * mean_;
        }
        if (g.mode == DISCOVER_SCORE_MAX) {
            if (kb == 0) {
                g.scores[id] = !ok ? nanv : state == 1.0 ? mx : -(mx + ub);
                cnt += ok;
            }
        } else {
            for (int e = 0; e < 4; e++)
                if (4 * kb + e < g.T)
                    g.scores[(int64_t)(4 * kb + e) * g.N + id] = !ok ? nanv : state == 1.0 ? r[e] : -(r[e] + ub);
            if (kb == 0) cnt += ok;
        }
    }
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor((int)cnt, o, 64);
    if (lane == 0 && cnt) atomicAdd(g.nscored, (unsigned long long)cnt);
}

// ------------------------------------------------------------ selection
// Pool = every candidate whose score may reach theta - margin.
__device__ __forceinline__ void d_compact(const double* __restrict__ sc, int64_t N,
                                                 const uint32_t* __restrict__ hist,
                                                 uint32_t* __restrict__ gsel,
                                                 int64_t* __restrict__ gst, double margin,
                                                 int64_t cap, int64_t* __restrict__ pool,
                                                 unsigned long long* __restrict__ cnt, int64_t K,
                                                 const SlotMap& sm, const SpaceDev& sd,
                                                 double* __restrict__ pscr) {
    uint32_t sel[3];
    int64_t st[2];
    radix_finish1(hist, K, gsel, gst, sel, st);        // one level: a lower bound suffices here
    const double th = select_threshold(sel, st);
    const double lo = st[1] ? 0.0 : th - 2.0 * margin;
    // Each wave gathers its hits in its own LDS queue (lane order within a
    // row) and appends the queue to the pool with one atomic when it is full
    // and once at the end, so a wave does not wait on a global atomic per
    // row that holds a hit; four strided rows of 64 scores are loaded before
    // any is tested, so the loads overlap (the pool's order does not matter:
    // it is sorted later).  The slots are decoded into IDs at the flush,
    // where the lanes' loads overlap too.
    constexpr unsigned QN = 256;
    __shared__ int64_t qs[4][QN];
    __shared__ double qx[4][QN];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const uint64_t below = (1ull << lane) - 1ull;
    const int64_t stride = (int64_t)gridDim.x * 256;
    unsigned qn = 0;                                      // queued (wave-uniform)
    auto flush = [&]() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(cnt, (unsigned long long)qn);
        base = __shfl(base, 0, 64);
        for (unsigned e = lane; e < qn; e += 64) {
            const unsigned long long slot = base + e;
            if ((int64_t)slot < cap) {
                pool[slot] = slot_id(sm, sd, qs[wv][e]);
                pscr[slot] = qx[wv][e];                   // the screening score, for the rescore
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        qn = 0;
    };
    for (int64_t i0 = (int64_t)blockIdx.x * 256 + (threadIdx.x & ~63); i0 < N; i0 += 4 * stride) {
        double xs[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int64_t i = i0 + q * stride + lane;
            xs[q] = i < N ? sc[i] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int64_t i = i0 + q * stride + lane;
            const double x = xs[q];
            const bool take = (x > 0.0 && x >= lo) || (x < 0.0 && -x >= lo);
            const uint64_t m = __builtin_amdgcn_ballot_w64(take);
            if (!m) continue;                             // (wave-uniform)
            const unsigned h = (unsigned)__popcll(m);
            if (qn + h > QN) flush();
            if (take) {
                const unsigned e = qn + (unsigned)__popcll(m & below);
                qs[wv][e] = i;
                qx[wv][e] = x;
            }
            qn += h;
        }
    }
    if (qn) flush();
}

// Exact FP64 rescore of the pool (one wave per entry); also flags entries
// whose ID is excluded.
// Values of the first cap pool entries as the exact rescoring evaluated
// them (row w of v, leading dimension ld), with their mean and centred sum
// of squares (NaN where the candidate is not valid): the duplicate-pair
// correlations then need one pass over two stored rows instead of two
// evaluations of each candidate.
struct PoolVals {
    double* v;
    int64_t ld, cap;
    double *mean, *sxx;
};

// ------------------------------------------------------ selection rules
// Per operand feature (compact index): its primaries (bits < 64), operator
// count, top operator and whether it and all its sub-expressions pass the
// hereditary rules.
struct RuleFeat {
    uint64_t vars;
    int32_t cplx;
    int8_t top;
    uint8_t ok;
    int16_t pad;
};

struct RuleTab {
    const RuleFeat* feat;
    const int32_t* unit;      // [Mc][B] unit vectors (scaled as the space's), for the target filter
    int B, max_cplx, target;
    uint32_t nest[10];
    int32_t tunit[8];
    uint64_t forb[64];
};

__device__ __forceinline__ bool pairs_forbidden(const RuleTab& R, uint64_t A, uint64_t B) {
    while (A) {
        const int u = __ffsll((long long)A) - 1;
        A &= A - 1;
        if (R.forb[u] & B) return true;
    }
    return false;
}

__device__ __forceinline__ bool nest_forbidden(const RuleTab& R, int op, int child_top) {
    return child_top != OP_NONE && ((R.nest[op] >> child_top) & 1u);
}

// Unit vector of op over operand vectors (the operator's rule holds: the
// candidate is unit-legal).
__device__ __forceinline__ void unit_apply(int op, int B, const int32_t* ua, const int32_t* ub, int32_t* out) {
    for (int k = 0; k < B; k++) {
        int32_t v = 0;
        switch (op) {
        case OP_EXP: case OP_LOG: v = 0; break;
        case OP_SQRT: v = ua[k] / 2; break;
        case OP_SQ: v = 2 * ua[k]; break;
        case OP_INV: v = -ua[k]; break;
        case OP_ADD: case OP_SUB: v = ua[k]; break;
        case OP_MUL: v = ua[k] + ub[k]; break;
        case OP_DIV: v = ua[k] - ub[k]; break;
        default: v = ub[k] - ua[k]; break;       // rdiv
        }
        out[k] = v;
    }
}

// Whether the rules allow candidate c (one lane's work; c decoded by
// cand_of_id, so its operands are operand features or, for kind 3, a
// rung-2 feature op2(cc, cd) over operand features).
__device__ __forceinline__ bool rules_pass(const RuleTab& R, const Cand& c) {
    const RuleFeat* F = R.feat;
    int32_t u[8], ug[8];
    int cplx;
    if (c.kind == 0) {
        const RuleFeat& f = F[c.ca];
        if (!f.ok) return false;
        if (R.target)
            for (int k = 0; k < R.B; k++)
                if (R.unit[(int64_t)c.ca * R.B + k] != R.tunit[k]) return false;
        return true;
    }
    const RuleFeat& fa = F[c.ca];
    if (!fa.ok || nest_forbidden(R, c.op, fa.top)) return false;
    const int32_t* ua = R.unit ? R.unit + (int64_t)c.ca * R.B : nullptr;
    if (c.kind == 1) {
        cplx = 1 + fa.cplx;
        if (R.target) unit_apply(c.op, R.B, ua, nullptr, u);
    } else {
        uint64_t vb;
        int cb, topb;
        const int32_t* ubp = ug;
        if (c.kind == 2) {
            const RuleFeat& fb = F[c.cb];
            if (!fb.ok) return false;
            vb = fb.vars;
            cb = fb.cplx;
            topb = fb.top;
            if (R.unit) ubp = R.unit + (int64_t)c.cb * R.B;
        } else {                                  // the rung-2 operand op2(cc, cd)
            const RuleFeat& f1 = F[c.cc];
            if (!f1.ok || nest_forbidden(R, c.op2, f1.top)) return false;
            vb = f1.vars;
            cb = 1 + f1.cplx;
            if (c.cd >= 0) {
                const RuleFeat& f2 = F[c.cd];
                if (!f2.ok || nest_forbidden(R, c.op2, f2.top) || pairs_forbidden(R, f1.vars, f2.vars))
                    return false;
                vb |= f2.vars;
                cb += f2.cplx;
            }
            if (R.max_cplx >= 0 && cb > R.max_cplx) return false;
            topb = c.op2;
            if (R.target)
                unit_apply(c.op2, R.B, R.unit + (int64_t)c.cc * R.B,
                           c.cd >= 0 ? R.unit + (int64_t)c.cd * R.B : nullptr, ug);
        }
        if (nest_forbidden(R, c.op, topb) || pairs_forbidden(R, fa.vars, vb)) return false;
        cplx = 1 + fa.cplx + cb;
        if (R.target) unit_apply(c.op, R.B, ua, ubp, u);
    }
    if (R.max_cplx >= 0 && cplx > R.max_cplx) return false;
    if (R.target)
        for (int k = 0; k < R.B; k++)
            if (u[k] != R.tunit[k]) return false;
    return true;
}

// The pool is rescored in two stages.  Stage 0 takes the entries whose
// screening score reaches the selection's lower bound th (at least K of
// them) and histograms their exact scores; the K-th largest of those, a
// lower bound theta1 of the K-th largest exact score, then spares stage 1
// every remaining entry whose score cannot reach it (|screening| + margin <
// theta1): those are marked not selectable, and the groups count the pool
// complete only down to max(th - margin, theta1).  d_split lists each
// stage's pool positions (pex = 2 marks a position left to stage 1).
__device__ __forceinline__ void d_split(int stage, const unsigned long long* __restrict__ Pp, int64_t cap,
                                        const uint32_t* __restrict__ sel, const int64_t* __restrict__ st,
                                        double margin, int64_t K, const uint32_t* __restrict__ hist1,
                                        uint32_t* __restrict__ th1d, double* __restrict__ perr,
                                        uint8_t* __restrict__ pex, double* __restrict__ ps,
                                        int32_t* __restrict__ rank, int32_t* __restrict__ order,
                                        const PoolVals pvs, int32_t* __restrict__ lst,
                                        unsigned long long* __restrict__ lcnt) {
    const int64_t P = min((int64_t)*Pp, cap);
    const bool all = st[1] != 0;
    const double th = select_threshold(sel, st);
    double th1 = 0.0;
    if (stage == 1) {
        const RadixDigit d = radix_digit(hist1, K, false);
        th1 = d.all ? 0.0 : (double)d.digit * 2.44140625e-4;          // digit * 2^-12
        if (blockIdx.x == 0 && threadIdx.x == 0) *th1d = d.all ? 0u : d.digit + 1u;
    }
    const int lane = threadIdx.x & 63;
    const uint64_t below = (1ull << lane) - 1ull;
    const int64_t l0 = stage == 0 ? 0 : (int64_t)lcnt[0];
    for (int64_t i0 = (int64_t)blockIdx.x * 256 + (threadIdx.x & ~63); i0 < P; i0 += (int64_t)gridDim.x * 256) {
        const int64_t w = i0 + lane;
        bool take = false;
        if (w < P) {
            const double x = fabs(perr[w]);               // the screening score (stage 0)
            if (stage == 0) {
                take = all || x >= th;
                if (!take) pex[w] = 2;
            } else if (pex[w] == 2) {
                take = x + margin >= th1;
                if (!take) {                              // cannot reach the K-th exact score
                    ps[w] = -1.0;
                    pex[w] = 0;
                    rank[w] = 0;
                    order[w] = (int32_t)w;
                    perr[w] = 0.0;
                    if (w < pvs.cap) {
                        pvs.mean[w] = __longlong_as_double(0x7FF8000000000000LL);
                        pvs.sxx[w] = __longlong_as_double(0x7FF8000000000000LL);
                    }
                }
            }
        }
        const uint64_t m = __builtin_amdgcn_ballot_w64(take);
        if (!m) continue;                                 // (wave-uniform)
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(&lcnt[stage], (unsigned long long)__popcll(m));
        base = __shfl(base, 0, 64);
        if (take) lst[l0 + (int64_t)(base + __popcll(m & below))] = (int32_t)w;
    }
}

// Exact scores of the pool, four entries per block (one per wave) in step:
// the first pass (values, mean, finiteness) per wave; in the second the
// block stages the centred targets of each 64-sample chunk in LDS once
// (double-buffered, one barrier per chunk) and every wave reads them there,
// so the T target rows are read from memory once per four entries instead
// of once per entry.  Per entry the arithmetic (and its order) is that of
// wave_exact_r.
template <int TMAX>
__device__ __forceinline__ void d_rescore(const int64_t* __restrict__ pool,
                                                 const unsigned long long* __restrict__ Pp, int64_t cap,
                                                 const EvalCtx& ev, Ops o, int n,
                                                 int T, int mode, int tlist,
                                                 const double* __restrict__ Yc,
                                                 const double* __restrict__ syy,
                                                 const int64_t* __restrict__ excl, int n_excl,
                                                 double* __restrict__ ps,
                                                 uint8_t* __restrict__ pex,
                                                 double* __restrict__ perr,
                                                 int32_t* __restrict__ rank,
                                                 int32_t* __restrict__ order,
                                                 const PoolVals pvs, const RuleTab* __restrict__ rules,
                                                 const int32_t* __restrict__ lst,
                                                 const unsigned long long* __restrict__ lcnt, int stage,
                                                 uint32_t* __restrict__ hist1) {
    // the entries of this stage: positions lst[l0 .. l0 + P) of the pool
    const int64_t l0 = stage == 0 ? 0 : (int64_t)lcnt[0];
    const int64_t P = min((int64_t)lcnt[stage], cap - l0);
    const int lane = threadIdx.x & 63;
    __shared__ double ys[2][TMAX][64];
    for (int64_t g = blockIdx.x; g * 4 < P; g += gridDim.x) {      // uniform over the block
    const int64_t wl = g * 4 + wave_id();
    const bool has = wl < P;
    const int64_t w = has ? lst[l0 + wl] : 0;
    const int64_t id = has ? pool[w] : 0;
    Cand c;
    bool ok = has && cand_of_id(ev, id, c);
    // a candidate the rules do not allow keeps its values but is never selected
    const bool allowed = !ok || !rules || rules_pass(*rules, c);
    const bool keep = has && w < pvs.cap;
    double* vals = keep ? pvs.v + w * pvs.ld : nullptr;
    // first pass: values, mean, finiteness, add/sub cancellation
    double m = 0.0;
    if (ok) {
        double s = 0.0;
        int bad = 0;
        const bool addsub = (c.kind == 2 || c.kind == 3) && (c.op == OP_ADD || c.op == OP_SUB);
        double ff = 0.0, ab = 0.0;
        for (int i = lane; i < n; i += 64) {
            const double f = cand_value(c, o, i);
            bad |= !isfinite(f);
            s += f;
            if (vals) vals[i] = f;
            if (addsub) {
                const double a = o.Vf[(int64_t)c.ca * o.ldn + i];
                double b;
                if (c.kind == 2) b = o.Vf[(int64_t)c.cb * o.ldn + i];
                else b = c.cd < 0 ? unary_value(c.op2, o, c.cc, i)
                                  : apply_op(c.op2, o.Vf[(int64_t)c.cc * o.ldn + i], o.Vf[(int64_t)c.cd * o.ldn + i]);
                ff += f * f;
                ab += a * a + b * b;
            }
        }
        if (__any(bad)) ok = false;
        if (ok && addsub) {                        // cancellation to rounding noise
            ff = wave_sum(ff);
            ab = wave_sum(ab);
            if (ff <= TAU_CANCEL * TAU_CANCEL * ab) ok = false;
        }
        if (ok) m = wave_sum(s) / n;
    }
    // second pass: centred sums against the targets staged in LDS
    double sxx = 0.0, sxy[TMAX];
#pragma unroll
    for (int t = 0; t < TMAX; t++) sxy[t] = 0.0;
    for (int i0 = 0, it = 0; i0 < n; i0 += 64, it++) {
        double(*yb)[64] = ys[it & 1];
        for (int q = threadIdx.x; q < T * 64; q += blockDim.x) {
            const int t = q >> 6, j = q & 63;
            yb[t][j] = i0 + j < n ? Yc[(int64_t)t * o.ldn + i0 + j] : 0.0;
        }
        __syncthreads();
        const int i = i0 + lane;
        if (ok && i < n) {
            // the first pass's values: stored (read back by the lane that
            // wrote them) or evaluated again
            const double d = (vals ? vals[i] : cand_value(c, o, i)) - m;
            sxx += d * d;
#pragma unroll
            for (int t = 0; t < TMAX; t++)
                if (t < T) sxy[t] += d * yb[t][lane];
        }
    }
    __syncthreads();                               // the buffers are refilled by the next group
    double r[TMAX];
    if (ok) {
        sxx = wave_sum(sxx);
        if (!isfinite(sxx)) ok = false;
    }
    if (ok) {
        const double sd = sqrt(sxx / n), rms = sqrt(sxx / n + m * m);
        if (!(sd > TAU_CONST * rms)) ok = false;
    }
    if (ok) {
#pragma unroll
        for (int t = 0; t < TMAX; t++)
            if (t < T) r[t] = wave_sum(sxy[t]) / sqrt(sxx * syy[t]);
    }
    if (!has) continue;
    if (keep && lane == 0) {                              // NaN: nothing stored for this entry
        pvs.mean[w] = ok ? m : __longlong_as_double(0x7FF8000000000000LL);
        pvs.sxx[w] = ok ? sxx : __longlong_as_double(0x7FF8000000000000LL);
    }
    int ex = 0;
    for (int e = lane; e < n_excl; e += 64) ex |= excl[e] == id;
    ex = __any(ex);
    if (lane == 0 && has) {
        double s = -1.0;
        if (ok) {
            if (mode == DISCOVER_SCORE_MAX) {
                s = 0.0;
                for (int t = 0; t < T; t++) s = fmax(s, fabs(r[t]));
            } else {
                s = fabs(r[tlist]);
            }
            if (!(s > 0.0) || !allowed) s = -1.0;
        }
        ps[w] = s;
        pex[w] = (uint8_t)ex;
        rank[w] = 0;                                      // counted by k_rankp or set by k_rk_rank
        order[w] = (int32_t)w;                            // (a valid index even before the scatter)
        const double x = perr[w];                         // screening-pass score (from the compaction)
        perr[w] = s > 0.0 && x > 0.0 ? fabs(x - s) : 0.0; // its maximum is taken by k_groups
        if (stage == 0 && s > 0.0) atomicAdd(&hist1[fx_key(s) >> 40], 1u);
    }
    }
}

// Exact two-pass score of the candidates whose shifted one-pass moments
// were ill-conditioned (one wave each), written back into the score slots
// (the list holds slots; below rung 3 a slot is the ID).
template <int TMAX>
__device__ __forceinline__ void d_fixup(const int64_t* __restrict__ ids,
                                               const unsigned long long* __restrict__ cnt,
                                               int64_t cap, const EvalCtx& ev, Ops o, int n,
                                               int T, int mode, const double* __restrict__ Yc,
                                               const double* __restrict__ syy, int64_t N,
                                               double* __restrict__ scores,
                                               unsigned long long* __restrict__ nscored,
                                               uint8_t* __restrict__ r2v, double* __restrict__ r2m,
                                               double* __restrict__ r2q) {
    const int64_t m = min((int64_t)*cnt, cap);
    unsigned nfix = 0;                                  // counted per wave, added once
    for (int64_t w = (int64_t)blockIdx.x * 4 + wave_id(); w < m; w += (int64_t)gridDim.x * 4) {
        const int64_t sl = ids[w];                      // a score slot (rung <= 2: the ID)
        const int64_t id = slot_id(ev.sm, ev.sd, sl);
        Cand c;
        bool ok = id >= 0 && cand_of_id(ev, id, c);
        double r[TMAX], mean = 0.0, msq = 0.0;
        ok = ok && wave_exact_r<TMAX>(c, o, n, T, Yc, syy, r, &mean, &msq);
        if ((threadIdx.x & 63) != 0 || !ok) continue;
        nfix++;
        if (r2v && id >= ev.sd.off[2] && id < ev.sd.off[3]) {     // rung-2 operand statistics
            r2v[id - ev.sd.off[2]] = 1;
            r2m[id - ev.sd.off[2]] = mean;
            r2q[id - ev.sd.off[2]] = msq;
        }
        if (mode == DISCOVER_SCORE_MAX) {
            double mx = 0.0;
            for (int t = 0; t < T; t++) mx = fmax(mx, fabs(r[t]));
            scores[sl] = mx;
        } else {
            for (int t = 0; t < T; t++) scores[(int64_t)t * N + sl] = fabs(r[t]);
        }
    }
    if ((threadIdx.x & 63) == 0 && nfix) atomicAdd(nscored, (unsigned long long)nfix);
}

// Sort of the pool by (-score, ID) as ranks: entry i's sorted position is
// the number of entries before it.  Blocks take a tile of 256 entries i and
// a chunk of RCH entries j staged in LDS (grid-strided over both, so any
// pool up to the capacity is covered) and add their counts with integer
// atomics, so the ranks do not depend on the order the blocks run in.
// Scores are -1 or positive (never NaN) and IDs are distinct, so the order
// is total and the ranks are a permutation.
constexpr int RCH = 256;

// (score, ID) of one entry, staged in LDS as one 16-byte read; a tile of
// them is scanned with a branch-free comparison, unrolled so that the LDS
// reads of several entries are in flight together.
struct __align__(16) SK {
    double s;
    long long id;
};
__device__ __forceinline__ int count_before(const SK* __restrict__ tile, int lim, double si, long long ii) {
    int c = 0;
    int j = 0;
    for (; j + 8 <= lim; j += 8) {
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const SK e = tile[j + u];
            c += (int)(e.s > si) | ((int)(e.s == si) & (int)(e.id < ii));
        }
    }
    for (; j < lim; j++) {
        const SK e = tile[j];
        c += (int)(e.s > si) | ((int)(e.s == si) & (int)(e.id < ii));
    }
    return c;
}

// Small pools: the rank of entry i is the number of entries j before it,
// counted over tiles of 256 entries i and chunks of RCH entries j staged in
// LDS (grid-strided over both) with integer atomics.
__device__ __forceinline__ void d_rankp(const double* __restrict__ ps, const int64_t* __restrict__ pool,
                                        const unsigned long long* __restrict__ Pp, int64_t cap,
                                        int32_t* __restrict__ rank) {
    const int64_t P = min((int64_t)*Pp, cap);
    __shared__ SK tile[RCH];
    for (int64_t j0 = (int64_t)blockIdx.y * RCH; j0 < P; j0 += (int64_t)gridDim.y * RCH) {
        __syncthreads();
        for (int q = threadIdx.x; q < RCH; q += 256)
            tile[q] = j0 + q < P ? SK{ps[j0 + q], (long long)pool[j0 + q]} : SK{-2.0, INT64_MAX};
        __syncthreads();
        const int lim = (int)min((int64_t)RCH, P - j0);
        for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i - threadIdx.x < P;
             i += (int64_t)gridDim.x * 256) {
            if (i >= P) continue;
            const int c = count_before(tile, lim, ps[i], (long long)pool[i]);
            if (c) atomicAdd(&rank[i], c);
        }
    }
}

// Large pools: ranks of the pool by (-score, ID) through buckets: an entry
// with a positive score goes to one of the first RK_NB / 2 buckets by its
// distance below the largest score, scaled so that the smallest positive
// score lands in the last of them (rounding is monotone, so a higher score
// never lands in a later bucket; scores are at most 1, so a stray tiny score
// only narrows the scale), an entry scored -1 to one of the last RK_NB / 2
// by its ID relative to the smallest such ID (the order among equal
// scores).  A bucket's entries all precede the next
// bucket's, so an entry's rank is the number of entries in earlier buckets
// (a prefix sum of the bucket counts) plus the number of its bucket-mates
// it follows (the same comparison as count_before).  The work is O(P) plus
// the squares of the bucket sizes, and nothing depends on the order the
// blocks run in.
constexpr int RK_NB = 65536;
constexpr int64_t RANK_PAIRS_MAX = 16384;   // pool capacity up to which all pairs are counted

// The buckets' scales: rkr[0] / rkr[1] hold the complement of the bits of
// the smallest and the bits of the largest positive score (positive
// doubles order as their bits), rkr[2] / rkr[3] the complement of the
// smallest and the largest ID of the entries scored -1 (all start at 0).
struct RkMap {
    double smax, inv;
    uint64_t i0;
    int shi;
};

__device__ __forceinline__ int rk_shift(uint64_t lo, uint64_t hi) {
    int sh = 0;
    if (hi < lo) return 0;                                 // none
    while (((hi - lo) >> sh) > (uint64_t)(RK_NB / 2 - 1)) sh++;
    return sh;
}

__device__ __forceinline__ RkMap rk_map(const unsigned long long* __restrict__ rkr) {
    RkMap m;
    const double smin = __longlong_as_double((long long)~rkr[0]);
    m.smax = __longlong_as_double((long long)rkr[1]);
    m.inv = m.smax > smin ? (double)(RK_NB / 2 - 1) / (m.smax - smin) : 0.0;
    m.i0 = ~(uint64_t)rkr[2];
    m.shi = rk_shift(m.i0, (uint64_t)rkr[3]);
    return m;
}

__device__ __forceinline__ int rk_bucket(double s, int64_t id, const RkMap& m) {
    return s > 0.0 ? min(RK_NB / 2 - 1, (int)((m.smax - s) * m.inv))
                   : RK_NB / 2 + (int)(((uint64_t)id - m.i0) >> m.shi);
}

__device__ __forceinline__ void d_rk_range(const double* __restrict__ ps, const int64_t* __restrict__ pool,
                                           const unsigned long long* __restrict__ Pp,
                                           int64_t cap, unsigned long long* __restrict__ rkr) {
    const int64_t P = min((int64_t)*Pp, cap);
    uint64_t v[4] = {0, 0, 0, 0};                          // as rkr
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x) {
        const double sv = ps[i];
        if (sv > 0.0) {
            const uint64_t k = (uint64_t)__double_as_longlong(sv);
            v[0] = max(v[0], ~k);
            v[1] = max(v[1], k);
        } else {
            const uint64_t k = (uint64_t)pool[i];
            v[2] = max(v[2], ~k);
            v[3] = max(v[3], k);
        }
    }
#pragma unroll
    for (int q = 0; q < 4; q++) {
        for (int o = 32; o > 0; o >>= 1) v[q] = max(v[q], (uint64_t)__shfl_xor((unsigned long long)v[q], o, 64));
        if ((threadIdx.x & 63) == 0 && v[q]) atomicMax(&rkr[q], (unsigned long long)v[q]);
    }
}

__device__ __forceinline__ void d_rk_hist(const double* __restrict__ ps, const int64_t* __restrict__ pool,
                                          const unsigned long long* __restrict__ Pp,
                                          int64_t cap, const unsigned long long* __restrict__ rkr,
                                          uint32_t* __restrict__ rkh) {
    const int64_t P = min((int64_t)*Pp, cap);
    const RkMap m = rk_map(rkr);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&rkh[rk_bucket(ps[i], pool[i], m)], 1u);
}

// Exclusive prefix sum of the bucket counts, in place (one block of 1024).
__device__ __forceinline__ void d_rk_scan(uint32_t* __restrict__ rkh) {
    constexpr int PER = RK_NB / 1024;
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    uint32_t sum = 0;
    for (int q = 0; q < PER; q++) sum += rkh[t * PER + q];
    part[t] = sum;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {                   // inclusive scan of the parts
        const uint32_t v = t >= o ? part[t - o] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = part[t] - sum;
    for (int q = 0; q < PER; q++) {
        const uint32_t c = rkh[t * PER + q];
        rkh[t * PER + q] = run;
        run += c;
    }
}

// Entries grouped by bucket: after this rkh[b] is the end of bucket b.
__device__ __forceinline__ void d_rk_scatter(const double* __restrict__ ps, const int64_t* __restrict__ pool,
                                             const unsigned long long* __restrict__ Pp,
                                             int64_t cap, const unsigned long long* __restrict__ rkr,
                                             uint32_t* __restrict__ rkh, int32_t* __restrict__ byb) {
    const int64_t P = min((int64_t)*Pp, cap);
    const RkMap m = rk_map(rkr);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x)
        byb[atomicAdd(&rkh[rk_bucket(ps[i], pool[i], m)], 1u)] = (int32_t)i;
}

// Ranks in bucket order: a block takes 256 consecutive positions of the
// bucket-grouped list, stages the entries of the buckets they touch (256 at
// a time, in LDS) and each thread counts its bucket-mates before it, so a
// bucket of many equal scores is compared from LDS rather than by one
// thread's chain of loads.
__device__ __forceinline__ void d_rk_rank(const double* __restrict__ ps, const int64_t* __restrict__ pool,
                                          const unsigned long long* __restrict__ Pp, int64_t cap,
                                          const unsigned long long* __restrict__ rkr,
                                          const uint32_t* __restrict__ rkh, const int32_t* __restrict__ byb,
                                          int32_t* __restrict__ rank) {
    const int64_t P = min((int64_t)*Pp, cap);
    const RkMap m = rk_map(rkr);
    __shared__ double ts[256];
    __shared__ long long tk[256];
    __shared__ uint32_t s_lo, s_hi;
    for (int64_t q0 = (int64_t)blockIdx.x * 256; q0 < P; q0 += (int64_t)gridDim.x * 256) {
        const int64_t q = q0 + threadIdx.x;
        const bool has = q < P;
        const int32_t i = has ? byb[q] : 0;
        const double si = has ? ps[i] : 0.0;
        const long long ii = has ? (long long)pool[i] : 0;
        uint32_t b0 = 0, b1 = 0;
        if (has) {
            const int b = rk_bucket(si, ii, m);
            b0 = b ? rkh[b - 1] : 0u;
            b1 = rkh[b];
        }
        if (threadIdx.x == 0) {
            s_lo = 0xFFFFFFFFu;
            s_hi = 0u;
        }
        __syncthreads();
        if (has) {
            atomicMin(&s_lo, b0);
            atomicMax(&s_hi, b1);
        }
        __syncthreads();
        const uint32_t lo = s_lo, hi = s_hi;
        int c = 0;
        for (uint32_t t0 = lo; t0 < hi; t0 += 256) {
            __syncthreads();
            const uint32_t j = t0 + threadIdx.x;
            if (j < hi) {
                const int32_t jj = byb[j];
                ts[threadIdx.x] = ps[jj];
                tk[threadIdx.x] = (long long)pool[jj];
            }
            __syncthreads();
            const uint32_t lim = min(256u, hi - t0);
            if (has)
                for (uint32_t k = 0; k < lim; k++) {
                    const uint32_t pos = t0 + k;
                    const bool mate = pos >= b0 && pos < b1;
                    c += (int)mate & ((int)(ts[k] > si) | ((int)(ts[k] == si) & (int)(tk[k] < ii)));
                }
        }
        if (has) rank[i] = (int32_t)(b0 + c);
        __syncthreads();                                   // s_lo, s_hi are set again
    }
}

// order[rank[i]] = i and the scores in sorted order.
__device__ __forceinline__ void d_scatter(const double* __restrict__ ps,
                                          const unsigned long long* __restrict__ Pp, int64_t cap,
                                          const int32_t* __restrict__ rank, int32_t* __restrict__ order,
                                          double* __restrict__ ss) {
    const int64_t P = min((int64_t)*Pp, cap);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = rank[i];
        order[r] = (int32_t)i;
        ss[r] = ps[i];
    }
}

// Near-tie clusters of the sorted pool.  Entries q-1 and q are chained when
// ss[q-1] - ss[q] <= TAU_NEAR ss[q-1]; a cluster is a maximal chain.  A
// group head h can only take entries of its own cluster: across a break,
// ss[h] - ss[q] exceeds TAU_NEAR ss[h].  Groups are formed over a prefix of
// the sorted pool: its first K entries, extended to the end of their last
// cluster (*pdp); entries past it cannot join a group that starts inside
// it, and the group pass checks that none of them could be selected.  (The
// pool of a precision form holds the whole guard band, most of which
// scores below the k-th group once rescored.)  Every valid entry of the
// prefix starts as its own head (parent[q] = q); entries whose exact score
// is not positive, and entries past the prefix, get -3.  The start of every
// cluster of two or more entries is listed for k_dedup (count in *ncl).
__device__ __forceinline__ bool chained(const double* __restrict__ ss, int64_t q) {
    const double sp = ss[q - 1], s = ss[q];
    return s > 0.0 && sp - s <= TAU_NEAR * sp;
}

__device__ __forceinline__ void d_clusters(const double* __restrict__ ss,
                                           const unsigned long long* __restrict__ Pp, int64_t cap,
                                           int64_t K, int dedup, int32_t* __restrict__ parent,
                                           int32_t* __restrict__ starts,
                                           unsigned long long* __restrict__ ncl,
                                           unsigned long long* __restrict__ pdp) {
    __shared__ int64_t s_pd;
    const int64_t P = min((int64_t)*Pp, cap);
    if (threadIdx.x == 0) {
        int64_t q = min(K, P);
        while (q > 0 && q < P && chained(ss, q)) q++;
        s_pd = q;
        if (blockIdx.x == 0) *pdp = (unsigned long long)q;
    }
    __syncthreads();
    const int64_t Pd = s_pd;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < P;
         q += (int64_t)gridDim.x * blockDim.x) {
        const bool valid = q < Pd && ss[q] > 0.0;
        parent[q] = valid ? (int32_t)q : -3;
        if (dedup && valid && (q == 0 || !chained(ss, q)) && q + 1 < Pd && chained(ss, q + 1))
            starts[atomicAdd(ncl, 1ull)] = (int32_t)q;
    }
}

// |corr(u, v)| >= 1 - TAU_DUP for the pool entries at slots iu and iv (one
// whole wave; every lane returns the flag).  Stored pool entries take the
// stored values, means and sums of squares (the same numbers the two-pass
// evaluation below forms, in the same order); others evaluate both.
__device__ __forceinline__ bool dup_pair(const int64_t* __restrict__ pool, int32_t iu, int32_t iv,
                                         const EvalCtx& ev, Ops o, int n, const PoolVals& pvs) {
    const int lane = threadIdx.x & 63;
    if (iu < pvs.cap && iv < pvs.cap && !isnan(pvs.sxx[iu]) && !isnan(pvs.sxx[iv])) {
        const double* u = pvs.v + (int64_t)iu * pvs.ld;
        const double* v = pvs.v + (int64_t)iv * pvs.ld;
        const double mu_ = pvs.mean[iu], mv = pvs.mean[iv];
        double uv = 0.0;
        for (int i = lane; i < n; i += 64) uv += (u[i] - mu_) * (v[i] - mv);
        uv = wave_sum(uv);
        return fabs(uv) / sqrt(pvs.sxx[iu] * pvs.sxx[iv]) >= 1.0 - TAU_DUP;
    }
    Cand cu, cv;
    if (!(cand_of_id(ev, pool[iu], cu) && cand_of_id(ev, pool[iv], cv))) return false;
    double su = 0.0, sv = 0.0;
    for (int i = lane; i < n; i += 64) {
        su += cand_value(cu, o, i);
        sv += cand_value(cv, o, i);
    }
    const double mu_ = wave_sum(su) / n, mv = wave_sum(sv) / n;
    double uu = 0.0, vv = 0.0, uv = 0.0;
    for (int i = lane; i < n; i += 64) {
        const double du = cand_value(cu, o, i) - mu_, dv = cand_value(cv, o, i) - mv;
        uu += du * du;
        vv += dv * dv;
        uv += du * dv;
    }
    uu = wave_sum(uu);
    vv = wave_sum(vv);
    uv = wave_sum(uv);
    return fabs(uv) / sqrt(uu * vv) >= 1.0 - TAU_DUP;
}

// The first q in [start, end) where pred holds, else end, found by the
// whole block in strides of its size (every thread calls it; slot is a
// shared int64 the search may use).
template <class Pred>
__device__ __forceinline__ int64_t block_first(int64_t start, int64_t end, Pred pred, int64_t& slot) {
    for (int64_t base = start; base < end; base += blockDim.x) {
        __syncthreads();
        if (threadIdx.x == 0) slot = end;
        __syncthreads();
        const int64_t q = base + threadIdx.x;
        if (q < end && pred(q)) atomicMin((unsigned long long*)&slot, (unsigned long long)q);
        __syncthreads();
        const int64_t f = slot;
        if (f < end) return f;
    }
    return end;
}

// First heads of the listed clusters, over the whole grid: a cluster's
// first entry always heads a group (no earlier entry can reach it), and
// takes every entry of its near-tie window that is its duplicate (all are
// free before it).  Work items are (cluster, slice of its window): the
// slices of one large group of equal scores run in many blocks instead of
// one.  The comparison is dup_pair's, the one the group pass below uses.
constexpr int DEDUP_SLICES = 16;

__device__ __forceinline__ void d_dedup_first(const int64_t* __restrict__ pool, const int32_t* __restrict__ order,
                                              const double* __restrict__ ss,
                                              const unsigned long long* __restrict__ Pp, int64_t cap,
                                              const EvalCtx& ev, Ops o, int n, int32_t* __restrict__ parent,
                                              const int32_t* __restrict__ starts,
                                              const unsigned long long* __restrict__ ncl, const PoolVals& pvs) {
    const int64_t P = min((int64_t)*Pp, cap);
    const int64_t nc = (int64_t)*ncl;
    const int w = wave_id(), nw = blockDim.x / 64;
    const int lane = threadIdx.x & 63;
    for (int64_t item = blockIdx.x; item < nc * DEDUP_SLICES; item += gridDim.x) {
        const int64_t h = starts[item / DEDUP_SLICES];
        const int sl = (int)(item % DEDUP_SLICES);
        const double sh = ss[h];
        const int32_t ih = order[h];
        for (int64_t q = h + 1 + (int64_t)sl * nw + w; q < P; q += (int64_t)DEDUP_SLICES * nw) {
            if (!(sh - ss[q] <= TAU_NEAR * sh)) break;      // past the window (scores sorted)
            if (parent[q] != (int32_t)q) continue;
            const bool dup = dup_pair(pool, ih, order[q], ev, o, n, pvs);
            if (dup && lane == 0) parent[q] = (int32_t)h;
        }
    }
}

// Duplicate heads of the listed clusters, one cluster at a time per block
// (blocks stride over the list), after the first-head pass: a cluster's
// first head has taken its duplicates, and the block goes on from the
// cluster's first free entry (the cluster's end and the next free entry are
// found by the whole block).  Inside a cluster the entries are visited
// in sorted order: an entry that no earlier head took is a head, and takes
// every later entry of its near-tie window (ss[h] - ss[q] <= TAU_NEAR ss[h])
// that is still free and is its duplicate.  So each entry joins the
// earliest head in its window of which it is a duplicate, and heads only
// are compared: a group of G equal scores costs G - 1 correlations, not a
// window of pairs.  The head's centred values are staged in LDS once (from
// its stored row, or evaluated); a member is read from its stored row, or
// evaluated once into registers (n <= 2048), so |corr| is formed with the
// same two-pass products as for two stored rows.
constexpr int DEDUP_LDS_N = 4096;     // longest head row staged in LDS
constexpr int DEDUP_REG = 32;         // member values per lane held in registers

__device__ __forceinline__ void d_dedup(const int64_t* __restrict__ pool, const int32_t* __restrict__ order,
                                        const double* __restrict__ ss,
                                        const unsigned long long* __restrict__ Pp, int64_t cap,
                                        const EvalCtx& ev, Ops o, int n, int32_t* __restrict__ parent,
                                        const int32_t* __restrict__ starts,
                                        const unsigned long long* __restrict__ ncl, const PoolVals& pvs) {
    __shared__ int64_t s_head, s_end, s_c1;
    __shared__ double s_huu;
    __shared__ int s_hok;
    __shared__ double hc[DEDUP_LDS_N];
    const int64_t P = min((int64_t)*Pp, cap);
    const int64_t nc = (int64_t)*ncl;
    const int w = wave_id(), nw = blockDim.x / 64;
    const int lane = threadIdx.x & 63;
    const bool staged = n <= DEDUP_LDS_N;
    volatile int32_t* vpar = parent;
    auto stored = [&](int32_t i) { return i < pvs.cap && !isnan(pvs.sxx[i]); };
    for (int64_t c = blockIdx.x; c < nc; c += gridDim.x) {
        const int64_t c0 = starts[c];
        // the cluster's end, and its first entry the first-head pass left
        // free (that pass took the first head's duplicates)
        const int64_t c1 = block_first(c0 + 1, P, [&](int64_t q) { return !chained(ss, q); }, s_c1);
        const int64_t h1 = block_first(c0 + 1, c1, [&](int64_t q) { return vpar[q] == (int32_t)q; }, s_head);
        __syncthreads();
        if (threadIdx.x == 0) s_head = h1;
        __syncthreads();
        for (;;) {
            const int64_t h = s_head;
            if (h >= c1) break;
            const int32_t ih = order[h];
            if (threadIdx.x == 0) {              // the head's window: a prefix of (h, c1)
                const double sh = ss[h];
                int64_t lo = h, hi = c1;         // in window up to lo, not from hi
                while (hi - lo > 1) {
                    const int64_t mid = lo + (hi - lo) / 2;
                    if (sh - ss[mid] <= TAU_NEAR * sh) lo = mid; else hi = mid;
                }
                s_end = lo + 1;
            }
            if (staged && w == 0) {              // head row, centred, into LDS
                if (stored(ih)) {
                    const double* u = pvs.v + (int64_t)ih * pvs.ld;
                    const double mu_ = pvs.mean[ih];
                    for (int i = lane; i < n; i += 64) hc[i] = u[i] - mu_;
                    if (lane == 0) { s_huu = pvs.sxx[ih]; s_hok = 1; }
                } else {
                    Cand ch;
                    const bool ok = cand_of_id(ev, pool[ih], ch);
                    double su = 0.0;
                    if (ok)
                        for (int i = lane; i < n; i += 64) {
                            const double x = cand_value(ch, o, i);
                            hc[i] = x;
                            su += x;
                        }
                    const double mu_ = wave_sum(su) / n;
                    double uu = 0.0;
                    if (ok)
                        for (int i = lane; i < n; i += 64) {
                            const double d = hc[i] - mu_;
                            hc[i] = d;
                            uu += d * d;
                        }
                    uu = wave_sum(uu);
                    if (lane == 0) { s_huu = uu; s_hok = ok ? 1 : 0; }
                }
            }
            __syncthreads();
            const int64_t e = s_end;
            for (int64_t q = h + 1 + w; q < e; q += nw) {
                if (vpar[q] != (int32_t)q) continue;          // taken by an earlier head
                const int32_t iv = order[q];
                bool dup;
                if (!staged) {
                    dup = dup_pair(pool, ih, iv, ev, o, n, pvs);
                } else if (!s_hok) {
                    dup = false;
                } else if (stored(iv)) {
                    const double* v = pvs.v + (int64_t)iv * pvs.ld;
                    const double mv = pvs.mean[iv];
                    double uv = 0.0;
                    for (int i = lane; i < n; i += 64) uv += hc[i] * (v[i] - mv);
                    uv = wave_sum(uv);
                    dup = fabs(uv) / sqrt(s_huu * pvs.sxx[iv]) >= 1.0 - TAU_DUP;
                } else {
                    Cand cv;
                    if (!cand_of_id(ev, pool[iv], cv)) {
                        dup = false;
                    } else if (n <= 64 * DEDUP_REG) {
                        double rv[DEDUP_REG];
                        double sv = 0.0;
#pragma unroll
                        for (int j = 0; j < DEDUP_REG; j++) {
                            const int i = lane + 64 * j;
                            rv[j] = i < n ? cand_value(cv, o, i) : 0.0;
                            sv += rv[j];
                        }
                        const double mv = wave_sum(sv) / n;
                        double vv = 0.0, uv = 0.0;
#pragma unroll
                        for (int j = 0; j < DEDUP_REG; j++) {
                            const int i = lane + 64 * j;
                            if (i < n) {
                                const double dv = rv[j] - mv;
                                vv += dv * dv;
                                uv += hc[i] * dv;
                            }
                        }
                        vv = wave_sum(vv);
                        uv = wave_sum(uv);
                        dup = fabs(uv) / sqrt(s_huu * vv) >= 1.0 - TAU_DUP;
                    } else {
                        double sv = 0.0;
                        for (int i = lane; i < n; i += 64) sv += cand_value(cv, o, i);
                        const double mv = wave_sum(sv) / n;
                        double vv = 0.0, uv = 0.0;
                        for (int i = lane; i < n; i += 64) {
                            const double dv = cand_value(cv, o, i) - mv;
                            vv += dv * dv;
                            uv += hc[i] * dv;
                        }
                        vv = wave_sum(vv);
                        uv = wave_sum(uv);
                        dup = fabs(uv) / sqrt(s_huu * vv) >= 1.0 - TAU_DUP;
                    }
                }
                if (dup && lane == 0) vpar[q] = (int32_t)h;
            }
            __threadfence_block();
            __syncthreads();
            // the next free entry heads the next group
            const int64_t hn = block_first(h + 1, c1, [&](int64_t q) { return vpar[q] == (int32_t)q; }, s_end);
            if (threadIdx.x == 0) s_head = hn;
            __syncthreads();
        }
    }
}

// Duplicate groups of the sorted pool, formed in parallel by one block of
// 1024 threads.  In sorted order, an entry joins the earliest group head in
// its near-tie window with which it is flagged a duplicate, otherwise it
// heads a new group (decided in rounds: an entry is decided once every
// flagged entry before it is).  Groups holding an excluded ID are blocked;
// each group is represented by its smallest ID; the first k unblocked
// groups in head order are returned in (-score, ID) order.  The result is
// complete when the pool reaches below the near-tie window of the k-th
// unblocked head, or when the pool holds every candidate.
// res: [0] selected, [1] complete, [2] merged duplicates.
constexpr int GRP_THREADS = 1024;

__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t* part) {
    const int t = threadIdx.x;
    part[t] = v;
    __syncthreads();
    for (int o = 1; o < GRP_THREADS; o <<= 1) {
        const int64_t x = t >= o ? part[t - o] : 0;
        __syncthreads();
        part[t] += x;
        __syncthreads();
    }
    const int64_t incl = part[t];
    __syncthreads();
    return incl - v;
}

__device__ __forceinline__ void d_groups(
    const int64_t* __restrict__ pool, const double* __restrict__ ps, const uint8_t* __restrict__ pex,
    const int32_t* __restrict__ order, const unsigned long long* __restrict__ Pp, int64_t cap,
    double tail, int k, const uint32_t* __restrict__ sel,
    const int64_t* __restrict__ st, double margin, const uint32_t* __restrict__ th1d,
    int32_t* __restrict__ parent, int32_t* __restrict__ blk, unsigned long long* __restrict__ repid, int32_t* __restrict__ reppos,
    int32_t* __restrict__ headpos, int64_t* __restrict__ out_ids, double* __restrict__ out_sc,
    int64_t* __restrict__ res) {
    __shared__ int64_t part[GRP_THREADS];
    const int64_t P = min((int64_t)*Pp, cap);
    const int t = threadIdx.x;
    const bool all = st[1] != 0;
    // the pool is complete down to th - margin, and down to theta1 where the
    // two-stage rescoring spared entries below it
    const double th_scan = all ? -1.0 : fmax(select_threshold(sel, st) - margin,
                                             *th1d ? (double)(*th1d - 1u) * 2.44140625e-4 : 0.0);
    const int32_t* vpar = parent;                          // heads, set by k_clusters / k_dedup
    for (int64_t q = t; q < P; q += GRP_THREADS) {
        blk[q] = 0;
        repid[q] = ~0ull;
        reppos[q] = -1;
    }
    __syncthreads();
    // aggregate groups onto their heads
    int64_t merged_loc = 0;
    for (int64_t q = t; q < P; q += GRP_THREADS) {
        const int32_t h = vpar[q];
        if (h < 0) continue;
        const int e = order[q];
        if (pex[e]) atomicOr(&blk[h], 1);
        atomicMin(&repid[h], (unsigned long long)pool[e]);
        merged_loc += h != (int32_t)q;
    }
    __syncthreads();
    for (int64_t q = t; q < P; q += GRP_THREADS) {
        const int32_t h = vpar[q];
        if (h >= 0 && (unsigned long long)pool[order[q]] == repid[h]) reppos[h] = (int32_t)q;
    }
    __syncthreads();
    // 4. rank the unblocked heads in sorted order (chunked block scan)
    const int64_t chunk = (P + GRP_THREADS - 1) / GRP_THREADS;
    const int64_t q0 = t * chunk, q1 = min(P, q0 + chunk);
    int64_t cnt = 0;
    for (int64_t q = q0; q < q1; q++) cnt += (vpar[q] == (int32_t)q && !blk[q]);
    int64_t r = block_excl_scan(cnt, part);
    const int64_t nunb = part[GRP_THREADS - 1];
    for (int64_t q = q0; q < q1; q++)
        if (vpar[q] == (int32_t)q && !blk[q]) {
            if (r < k) headpos[r] = (int32_t)q;
            r++;
        }
    const int64_t merged = block_excl_scan(merged_loc, part) + merged_loc;
    const int64_t merged_tot = part[GRP_THREADS - 1];
    (void)merged;
    __syncthreads();
    const int64_t ns = min((int64_t)k, nunb);
    // 5. representatives in (-score, ID) order (rank sort of <= k entries,
    // staged through LDS in tiles)
    __shared__ SK tile[GRP_THREADS];
    for (int64_t i0 = 0; i0 < ns; i0 += GRP_THREADS) {
        const int64_t i = i0 + t;
        double si = 0.0;
        int64_t ii = 0;
        if (i < ns) {
            const int32_t rp = reppos[headpos[i]];
            si = ps[order[rp]];
            ii = pool[order[rp]];
        }
        int64_t rank = 0;
        for (int64_t j0 = 0; j0 < ns; j0 += GRP_THREADS) {
            __syncthreads();
            if (j0 + t < ns) {
                const int32_t rq = reppos[headpos[j0 + t]];
                tile[t] = SK{ps[order[rq]], (long long)pool[order[rq]]};
            }
            __syncthreads();
            const int lim = (int)min((int64_t)GRP_THREADS, ns - j0);
            if (i < ns) rank += count_before(tile, lim, si, (long long)ii);
        }
        if (i < ns) {
            out_ids[rank] = ii;
            out_sc[rank] = si;
        }
    }
    for (int64_t i = ns + t; i < k; i += GRP_THREADS) {
        out_ids[i] = -1;
        out_sc[i] = __longlong_as_double(0x7FF8000000000000LL);
    }
    if (t == 0) {
        // the scan reached below the near-tie window of the k-th unblocked
        // head, both in the pool and in the grouped prefix (tail: the first
        // score past it)
        bool complete = all && !(tail > 0.0);
        if (nunb >= k) {
            const double lim = ps[order[headpos[k - 1]]];
            complete = (all || (1.0 - TAU_NEAR) * lim >= th_scan) && (1.0 - TAU_NEAR) * lim > tail;
        }
        res[0] = ns;
        res[1] = complete ? 1 : 0;
        res[2] = merged_tot;
        res[3] = 0;
        res[4] = (int64_t)*Pp;                  // pool size (capacity check)
    }
}

// The same for a pool of at most GRP_LDS entries, with the group state in
// LDS: parent (int32), the blocked flags (one bit per entry), and per head
// the 64-bit minimum of (ID << 12 | position), which gives the
// representative's ID and its sorted position at once (IDs stay below
// 2^51).  The tiles of the final rank sort reuse the parent array.
constexpr int GRP_LDS = 4096;

__device__ __forceinline__ void d_groups_lds(
    const int64_t* __restrict__ pool, const double* __restrict__ ps, const uint8_t* __restrict__ pex,
    const int32_t* __restrict__ order, const int32_t* __restrict__ parent, int64_t P, double tail, int k,
    const uint32_t* __restrict__ sel, const int64_t* __restrict__ st, double margin,
    const uint32_t* __restrict__ th1d, int32_t* __restrict__ headpos, int64_t* __restrict__ out_ids, double* __restrict__ out_sc,
    int64_t* __restrict__ res, const PoolVals pvs, int64_t* __restrict__ vrow) {
    __shared__ int64_t part[GRP_THREADS];
    __shared__ __align__(16) int32_t par[GRP_LDS];
    __shared__ __align__(16) unsigned long long rkey[GRP_LDS];   // also the sort array of phase 5
    __shared__ uint32_t blkb[GRP_LDS / 32];
    const int t = threadIdx.x;
    const bool all = st[1] != 0;
    // the pool is complete down to th - margin, and down to theta1 where the
    // two-stage rescoring spared entries below it
    const double th_scan = all ? -1.0 : fmax(select_threshold(sel, st) - margin,
                                             *th1d ? (double)(*th1d - 1u) * 2.44140625e-4 : 0.0);
    for (int q = t; q < P; q += GRP_THREADS) {             // heads, set by k_clusters / k_dedup
        par[q] = parent[q];
        rkey[q] = ~0ull;
    }
    for (int w = t; w < GRP_LDS / 32; w += GRP_THREADS) blkb[w] = 0u;
    __syncthreads();
    // aggregate groups onto their heads
    int64_t merged_loc = 0;
    for (int q = t; q < P; q += GRP_THREADS) {
        const int32_t h = par[q];
        if (h < 0) continue;
        const int e = order[q];
        if (pex[e]) atomicOr(&blkb[h >> 5], 1u << (h & 31));
        atomicMin(&rkey[h], ((unsigned long long)pool[e] << 12) | (unsigned long long)q);
        merged_loc += h != q;
    }
    __syncthreads();
    // 4. rank the unblocked heads in sorted order (chunked block scan)
    const int chunk = (int)((P + GRP_THREADS - 1) / GRP_THREADS);
    const int q0 = t * chunk, q1 = (int)min(P, (int64_t)q0 + chunk);
    auto unblocked_head = [&](int q) { return par[q] == q && !((blkb[q >> 5] >> (q & 31)) & 1u); };
    int64_t cnt = 0;
    for (int q = q0; q < q1; q++) cnt += unblocked_head(q);
    int64_t r = block_excl_scan(cnt, part);
    const int64_t nunb = part[GRP_THREADS - 1];
    for (int q = q0; q < q1; q++)
        if (unblocked_head(q)) {
            if (r < k) headpos[r] = q;
            r++;
        }
    block_excl_scan(merged_loc, part);
    const int64_t merged_tot = part[GRP_THREADS - 1];
    __syncthreads();
    const int64_t ns = min((int64_t)k, nunb);
    // 5. representatives in (-score, ID) order: up to 1024 by a bitonic
    // sort with one entry per thread (partners within a wave by register
    // shuffles, across waves through LDS, the key array's memory), more by
    // rank counting in tiles that reuse the parent array.  IDs are
    // distinct, so the order is strict and both give the same result.
    if (ns <= GRP_THREADS) {
        int N2 = 1;
        while (N2 < ns) N2 <<= 1;
        // the key keeps its sorted-position bits below the ID: distinct IDs
        // order the keys as they order the IDs
        SK e{-INFINITY, INT64_MAX};                               // padding sorts last
        if (t < ns) {
            const unsigned long long kk = rkey[headpos[t]];
            e = SK{ps[order[(int)(kk & 4095ull)]], (long long)kk};
        }
        SK* srt = (SK*)rkey;                                      // 1024 entries = 16 KB
        for (int kb = 2; kb <= N2; kb <<= 1)
            for (int j = kb >> 1; j > 0; j >>= 1) {
                SK o;
                if (j >= 64) {                                    // partner in another wave
                    __syncthreads();
                    srt[t] = e;
                    __syncthreads();
                    o = srt[t ^ j];
                } else {
                    o.s = __shfl_xor(e.s, j, 64);
                    o.id = __shfl_xor(e.id, j, 64);
                }
                const bool o_first = o.s > e.s || (o.s == e.s && o.id < e.id);
                // the lower index of a pair keeps the first entry in runs that
                // ascend (bit kb of the index clear), the later one otherwise
                const bool keep_first = ((t & j) == 0) == ((t & kb) == 0);
                if (o_first == keep_first) e = o;
            }
        if (t < ns) {
            const int32_t slot = order[(int)((unsigned long long)e.id & 4095ull)];
            out_ids[t] = e.id >> 12;
            out_sc[t] = e.s;
            vrow[t] = slot < pvs.cap ? (int64_t)(uintptr_t)(pvs.v + (int64_t)slot * pvs.ld) : 0;
        }
    } else {
    SK* tile = (SK*)par;                                          // 1024 entries = 16 KB
    for (int64_t i0 = 0; i0 < ns; i0 += GRP_THREADS) {
        const int64_t i = i0 + t;
        double si = 0.0;
        int64_t ii = 0;
        if (i < ns) {
            const unsigned long long kk = rkey[headpos[i]];
            si = ps[order[(int)(kk & 4095ull)]];
            ii = (int64_t)(kk >> 12);
        }
        int64_t rank = 0;
        for (int64_t j0 = 0; j0 < ns; j0 += GRP_THREADS) {
            __syncthreads();
            if (j0 + t < ns) {
                const unsigned long long kk = rkey[headpos[j0 + t]];
                tile[t] = SK{ps[order[(int)(kk & 4095ull)]], (long long)(kk >> 12)};
            }
            __syncthreads();
            const int lim = (int)min((int64_t)GRP_THREADS, ns - j0);
            if (i < ns) rank += count_before(tile, lim, si, (long long)ii);
        }
        if (i < ns) {
            out_ids[rank] = ii;
            out_sc[rank] = si;
            const int32_t slot = order[(int)(rkey[headpos[i]] & 4095ull)];
            vrow[rank] = slot < pvs.cap ? (int64_t)(uintptr_t)(pvs.v + (int64_t)slot * pvs.ld) : 0;
        }
    }
    }
    for (int64_t i = ns + t; i < k; i += GRP_THREADS) vrow[i] = 0;
    for (int64_t i = ns + t; i < k; i += GRP_THREADS) {
        out_ids[i] = -1;
        out_sc[i] = __longlong_as_double(0x7FF8000000000000LL);
    }
    if (t == 0) {
        // the scan reached below the near-tie window of the k-th unblocked
        // head, both in the pool and in the grouped prefix (tail: the first
        // score past it)
        bool complete = all && !(tail > 0.0);
        if (nunb >= k) {
            const double lim = ps[order[headpos[k - 1]]];
            complete = (all || (1.0 - TAU_NEAR) * lim >= th_scan) && (1.0 - TAU_NEAR) * lim > tail;
        }
        res[0] = ns;
        res[1] = complete ? 1 : 0;
        res[2] = merged_tot;
        res[3] = 0;
    }
}

// Values of the selected candidates: one wave per output row; a row whose
// values the exact rescoring kept (the same numbers) is copied.
__device__ __forceinline__ void d_values(const int64_t* __restrict__ ids, int64_t m,
                                                const EvalCtx& ev, Ops o, int n,
                                                double* __restrict__ out, int64_t ldv,
                                                const int64_t* __restrict__ vrow) {
    const int64_t w = (int64_t)blockIdx.x * 4 + wave_id();
    if (w >= m) return;
    const int lane = threadIdx.x & 63;
    const int64_t id = ids[w];
    const int64_t src = vrow && id >= 0 ? vrow[w] : 0;
    if (src) {                                          // (wave-uniform)
        const double* v = (const double*)(uintptr_t)src;
        for (int i = lane; i < n; i += 64) out[w * ldv + i] = v[i];
        return;
    }
    Cand c;
    const bool ok = id >= 0 && cand_of_id(ev, id, c);
    for (int i = lane; i < n; i += 64)
        out[w * ldv + i] = ok ? cand_value(c, o, i) : __longlong_as_double(0x7FF8000000000000LL);
}

// ------------------------------------------------- batched kernel entries
// Exact re-decisions of one problem (ill-conditioned shifted moments).
struct FixArgs {
    const int64_t* ids;
    const unsigned long long* cnt;
    int64_t cap;
    EvalCtx ev;
    Ops o;
    int n, T, mode;
    const double *Yc, *syy;
    int64_t N;
    double* scores;
    unsigned long long* nscored;
    uint8_t* r2v;
    double *r2m, *r2q;
};

// grid (persistent blocks, problems)
// TM: the most targets of any problem of the launch (1, 8 or 16).
template <int TM>
__global__ __launch_bounds__(256) void k_fixup(ctab<FixArgs> A) {
    const FixArgs& a = tab(A, blockIdx.y);
    DSC_GLOBAL(a.ids); DSC_GLOBAL(a.cnt); DSC_GLOBAL(a.ev.raw2c); DSC_GLOBAL(a.ev.valid); DSC_GLOBAL(a.o.Vf); DSC_GLOBAL(a.o.Rf); DSC_GLOBAL(a.Yc); DSC_GLOBAL(a.syy); DSC_GLOBAL(a.scores); DSC_GLOBAL(a.nscored);
    d_fixup<TM>(a.ids, a.cnt, a.cap, a.ev, a.o, a.n, a.T, a.mode, a.Yc, a.syy, a.N,
                                  a.scores, a.nscored, a.r2v, a.r2m, a.r2q);
}

static void launch_fixup(const std::vector<FixArgs>& fa, dim3 grid, ctab<FixArgs> d, hipStream_t st) {
    int Tm = 1;
    for (const FixArgs& x : fa) Tm = std::max(Tm, x.T);
    if (Tm <= 1) k_fixup<1><<<grid, 256, 0, st>>>(d);
    else if (Tm <= 8) k_fixup<8><<<grid, 256, 0, st>>>(d);
    else k_fixup<DISCOVER_MAX_TARGETS><<<grid, 256, 0, st>>>(d);
}

// Everything the exact top-k of one list (problem, target) works on.
struct SelArgs {
    const double* sc;         // score slots of the list
    int64_t N;
    uint32_t* sel;            // radix selection of the list
    int64_t* st;
    const uint32_t* hist;     // its two level histograms
    double margin;
    int64_t cap, fcap;        // pool and duplicate-pair capacities
    int64_t K;                // rank the radix selection bounds
    int64_t* pool;
    unsigned long long* cnt;  // pool entries found (may exceed cap)
    EvalCtx ev;
    Ops o;
    int n, T, mode, t, k, dedup;
    const double *Yc, *syy;
    const int64_t* excl;
    int n_excl;
    double* ps;
    uint8_t* pex;
    unsigned long long* maxerr;
    int32_t *order, *lo, *wc; // lo: pool positions grouped by rank bucket
    int32_t* rank;            // pool position -> sorted position (counted)
    uint32_t* rkh;            // rank buckets: counts, then starts, then ends
    unsigned long long* rkr;  // rank buckets' key range
    double* ss;               // scores in sorted order
    double* perr;             // per pool entry: its screening score, then |screening - exact|
    uint32_t* th1d;           // two-stage rescoring: digit of theta1 + 1 (0: none)
    int64_t* off;
    uint8_t* flag;
    unsigned long long* ncl;  // near-tie clusters listed in wc (starts)
    unsigned long long* pd;   // end of the grouped prefix of the sorted pool
    int32_t *parent, *blk;
    unsigned long long* repid;
    int32_t *reppos, *headpos;
    int64_t* out_ids;
    double* out_sc;
    int64_t* res;
    PoolVals pvs;             // stored values of the first pvs.cap pool entries
    int64_t* vrow;            // per selected rank: address of its stored value row, 0 for none
    const RuleTab* rules;     // selection rules, or NULL
};

// grid (blocks, lists) for the streaming kernels, (lists) for the one-block ones
__global__ __launch_bounds__(256) void k_compact(ctab<SelArgs> A) {
    const SelArgs& a = tab(A, blockIdx.y);
    DSC_GLOBAL(a.sc); DSC_GLOBAL(a.sel); DSC_GLOBAL(a.st); DSC_GLOBAL(a.pool); DSC_GLOBAL(a.cnt); DSC_GLOBAL(a.ev.raw2c); DSC_GLOBAL(a.ev.valid); DSC_GLOBAL(a.o.Vf); DSC_GLOBAL(a.o.Rf); DSC_GLOBAL(a.Yc); DSC_GLOBAL(a.syy); DSC_GLOBAL(a.ps); DSC_GLOBAL(a.pex); DSC_GLOBAL(a.maxerr); DSC_GLOBAL(a.order); DSC_GLOBAL(a.lo); DSC_GLOBAL(a.wc); DSC_GLOBAL(a.off); DSC_GLOBAL(a.flag); DSC_GLOBAL(a.parent); DSC_GLOBAL(a.blk); DSC_GLOBAL(a.repid); DSC_GLOBAL(a.reppos); DSC_GLOBAL(a.headpos); DSC_GLOBAL(a.out_ids); DSC_GLOBAL(a.out_sc); DSC_GLOBAL(a.res);
    d_compact(a.sc, a.N, a.hist, a.sel, a.st, a.margin, a.cap, a.pool, a.cnt, a.K, a.ev.sm, a.ev.sd, a.perr);
}

// TM: the most targets of any list of the launch (1, 8 or 16 registers of
// sums per lane).
template <int TM>
__global__ __launch_bounds__(256) void k_rescore(ctab<SelArgs> A, int stage) {
    const SelArgs& a = tab(A, blockIdx.y);
    DSC_GLOBAL(a.sc); DSC_GLOBAL(a.sel); DSC_GLOBAL(a.st); DSC_GLOBAL(a.pool); DSC_GLOBAL(a.cnt); DSC_GLOBAL(a.ev.raw2c); DSC_GLOBAL(a.ev.valid); DSC_GLOBAL(a.o.Vf); DSC_GLOBAL(a.o.Rf); DSC_GLOBAL(a.Yc); DSC_GLOBAL(a.syy); DSC_GLOBAL(a.ps); DSC_GLOBAL(a.pex); DSC_GLOBAL(a.maxerr); DSC_GLOBAL(a.order); DSC_GLOBAL(a.lo); DSC_GLOBAL(a.wc); DSC_GLOBAL(a.off); DSC_GLOBAL(a.flag); DSC_GLOBAL(a.parent); DSC_GLOBAL(a.blk); DSC_GLOBAL(a.repid); DSC_GLOBAL(a.reppos); DSC_GLOBAL(a.headpos); DSC_GLOBAL(a.out_ids); DSC_GLOBAL(a.out_sc); DSC_GLOBAL(a.res);
    d_rescore<TM>(a.pool, a.cnt, a.cap, a.ev, a.o, a.n, a.T, a.mode, a.t, a.Yc, a.syy,
                                    a.excl, a.n_excl, a.ps, a.pex, a.perr, a.rank, a.order, a.pvs,
                                    a.rules, a.lo, a.rkr + 4, stage, (uint32_t*)a.hist + 4096);
}

// grid (blocks, lists): the pool positions of one rescoring stage (the
// list in lo, its counts in rkr[4], rkr[5]; both free until the sort)
__global__ __launch_bounds__(256) void k_split(ctab<SelArgs> A, int stage) {
    const SelArgs& a = tab(A, blockIdx.y);
    d_split(stage, a.cnt, a.cap, a.sel, a.st, a.margin, a.K, a.hist + 4096, a.th1d, a.perr, a.pex, a.ps,
            a.rank, a.order, a.pvs, a.lo, a.rkr + 4);
}

// grid (i tiles, j chunks, lists)
__global__ __launch_bounds__(256) void k_rankp(ctab<SelArgs> A) {
    const SelArgs& a = tab(A, blockIdx.z);
    d_rankp(a.ps, a.pool, a.cnt, a.cap, a.rank);
}

__global__ __launch_bounds__(256) void k_rk_range(ctab<SelArgs> A) {
    const SelArgs& a = tab(A, blockIdx.y);
    d_rk_range(a.ps, a.pool, a.cnt, a.cap, a.rkr);
}

__global__ __launch_bounds__(256) void k_rk_hist(ctab<SelArgs> A) {
    const SelArgs& a = tab(A, blockIdx.y);
    d_rk_hist(a.ps, a.pool, a.cnt, a.cap, a.rkr, a.rkh);
}

__global__ __launch_bounds__(1024) void k_rk_scan(ctab<SelArgs> A) {
    const SelArgs& a = tab(A, blockIdx.x);
    d_rk_scan(a.rkh);
}

__global__ __launch_bounds__(256) void k_rk_scatter(ctab<SelArgs> A) {
    const SelArgs& a = tab(A, blockIdx.y);
    d_rk_scatter(a.ps, a.pool, a.cnt, a.cap, a.rkr, a.rkh, a.lo);
}

__global__ __launch_bounds__(256) void k_rk_rank(ctab<SelArgs> A) {
    const SelArgs& a = tab(A, blockIdx.y);
    d_rk_rank(a.ps, a.pool, a.cnt, a.cap, a.rkr, a.rkh, a.lo, a.rank);
}

__global__ __launch_bounds__(256) void k_scatter(ctab<SelArgs> A) {
    const SelArgs& a = tab(A, blockIdx.y);
    DSC_GLOBAL(a.ps); DSC_GLOBAL(a.pool); DSC_GLOBAL(a.cnt); DSC_GLOBAL(a.rank); DSC_GLOBAL(a.order); DSC_GLOBAL(a.ss); DSC_GLOBAL(a.lo); DSC_GLOBAL(a.wc); DSC_GLOBAL(a.off);
    d_scatter(a.ps, a.cnt, a.cap, a.rank, a.order, a.ss);
}

__global__ __launch_bounds__(256) void k_clusters(ctab<SelArgs> A) {
    const SelArgs& a = tab(A, blockIdx.y);
    DSC_GLOBAL(a.ss); DSC_GLOBAL(a.cnt); DSC_GLOBAL(a.parent); DSC_GLOBAL(a.wc); DSC_GLOBAL(a.ncl); DSC_GLOBAL(a.pd);
    d_clusters(a.ss, a.cnt, a.cap, a.K, a.dedup, a.parent, a.wc, a.ncl, a.pd);
}

constexpr int DEDUP_THREADS = 512;

__global__ __launch_bounds__(256) void k_dedup_first(ctab<SelArgs> A) {
    const SelArgs& a = tab(A, blockIdx.y);
    d_dedup_first(a.pool, a.order, a.ss, a.cnt, a.cap, a.ev, a.o, a.n, a.parent, a.wc, a.ncl, a.pvs);
}

__global__ __launch_bounds__(DEDUP_THREADS) void k_dedup(ctab<SelArgs> A) {
    const SelArgs& a = tab(A, blockIdx.y);
    DSC_GLOBAL(a.pool); DSC_GLOBAL(a.order); DSC_GLOBAL(a.ss); DSC_GLOBAL(a.cnt); DSC_GLOBAL(a.parent); DSC_GLOBAL(a.wc); DSC_GLOBAL(a.ncl); DSC_GLOBAL(a.ev.raw2c); DSC_GLOBAL(a.ev.valid); DSC_GLOBAL(a.o.Vf); DSC_GLOBAL(a.o.Rf);
    d_dedup(a.pool, a.order, a.ss, a.cnt, a.cap, a.ev, a.o, a.n, a.parent, a.wc, a.ncl, a.pvs);
}

__global__ __launch_bounds__(GRP_THREADS) void k_groups(ctab<SelArgs> A) {
    const SelArgs& a = tab(A, blockIdx.x);
    DSC_GLOBAL(a.sc); DSC_GLOBAL(a.sel); DSC_GLOBAL(a.st); DSC_GLOBAL(a.pool); DSC_GLOBAL(a.cnt); DSC_GLOBAL(a.ev.raw2c); DSC_GLOBAL(a.ev.valid); DSC_GLOBAL(a.o.Vf); DSC_GLOBAL(a.o.Rf); DSC_GLOBAL(a.Yc); DSC_GLOBAL(a.syy); DSC_GLOBAL(a.ps); DSC_GLOBAL(a.pex); DSC_GLOBAL(a.maxerr); DSC_GLOBAL(a.order); DSC_GLOBAL(a.lo); DSC_GLOBAL(a.wc); DSC_GLOBAL(a.off); DSC_GLOBAL(a.flag); DSC_GLOBAL(a.parent); DSC_GLOBAL(a.blk); DSC_GLOBAL(a.repid); DSC_GLOBAL(a.reppos); DSC_GLOBAL(a.headpos); DSC_GLOBAL(a.out_ids); DSC_GLOBAL(a.out_sc); DSC_GLOBAL(a.res);
    const int64_t P = min((int64_t)*a.cnt, a.cap);
    {
        // maximum |screening - exact| over the pool (one atomic per list)
        __shared__ double emax[GRP_THREADS / 64];
        double e = 0.0;
        for (int64_t q = threadIdx.x; q < P; q += GRP_THREADS) e = fmax(e, a.perr[q]);
        e = wave_max(e);
        if ((threadIdx.x & 63) == 0) emax[threadIdx.x >> 6] = e;
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < GRP_THREADS / 64; w++) e = fmax(e, emax[w]);
            if (e > 0.0) atomicMax(a.maxerr, (unsigned long long)__double_as_longlong(e));
        }
        __syncthreads();
    }
    // groups live in the prefix [0, Pd) of the sorted pool
    const int64_t Pd = min((int64_t)*a.pd, P);
    const double tail = Pd < P ? a.ps[a.order[Pd]] : -1.0;
    if (Pd <= GRP_LDS) {
        d_groups_lds(a.pool, a.ps, a.pex, a.order, a.parent, Pd, tail, a.k, a.sel, a.st, a.margin,
                     a.th1d, a.headpos, a.out_ids, a.out_sc, a.res, a.pvs, a.vrow);
        if (threadIdx.x == 0) a.res[4] = (int64_t)*a.cnt;     // pool size (capacity check)
        return;
    }
    for (int64_t i = threadIdx.x; i < a.k; i += GRP_THREADS) a.vrow[i] = 0;   // rows are evaluated
    d_groups(a.pool, a.ps, a.pex, a.order, a.cnt, a.cap, tail, a.k, a.sel, a.st, a.margin, a.th1d, a.parent, a.blk,
             a.repid, a.reppos, a.headpos, a.out_ids, a.out_sc, a.res);
}

// Values of the selected features of one list.
struct ValArgs {
    const int64_t* ids;
    int64_t m;
    EvalCtx ev;
    Ops o;
    int n;
    double* out;
    int64_t ldv;
    const int64_t* vrow;      // or NULL: per row, the address of its stored values (0: evaluate)
};

// grid (row blocks of 4, lists)
__global__ __launch_bounds__(256) void k_values(ctab<ValArgs> A) {
    const ValArgs& a = tab(A, blockIdx.y);
    DSC_GLOBAL(a.ids); DSC_GLOBAL(a.ev.raw2c); DSC_GLOBAL(a.ev.valid); DSC_GLOBAL(a.o.Vf); DSC_GLOBAL(a.o.Rf); DSC_GLOBAL(a.out);
    if ((int64_t)blockIdx.x * 4 >= a.m) return;
    d_values(a.ids, a.m, a.ev, a.o, a.n, a.out, a.ldv, a.vrow);
}

}  // namespace dsc

// ====================================================================== host
namespace dsc {

static int pad_targets(int T) { return T <= 1 ? 1 : T <= 2 ? 2 : T <= 4 ? 4 : T <= 8 ? 8 : 16; }

// Tile widths J (operand features j per wave) the dense kernel is built for.
static int max_J(int TP) { return TP == 1 ? 4 : TP == 2 ? 2 : 1; }

template <int OPS, int J, int TP>
static void launch_pairs_t(ctab<PairArgs> A, const int4* tiles, int64_t n, bool list,
                           unsigned long long* queue, hipStream_t st) {
    if (n == 0) return;
    if (list) {
        k_screen_pairs<OPS, 1, TP, true, false><<<(unsigned)n, 64 * pair_split<true>(), 0, st>>>(A, tiles, n, nullptr);
    } else if (queue) {                        // persistent: 8 blocks per CU at most
        const unsigned g = (unsigned)std::min<int64_t>(n, 8 * 256);
        k_screen_pairs<OPS, J, TP, false, true><<<g, 64 * pair_split<false>(), 0, st>>>(A, tiles, n, queue);
    } else {                                   // one block per tile
        k_screen_pairs<OPS, J, TP, false, false><<<(unsigned)n, 64 * pair_split<false>(), 0, st>>>(A, tiles, n, nullptr);
    }
}

template <int OPS>
static void launch_pairs_ops(ctab<PairArgs> A, const int4* tiles, int64_t n, bool list, int TP,
                             int J, unsigned long long* q, hipStream_t st) {
    switch (TP) {
    case 1:
        if (J == 4) launch_pairs_t<OPS, 4, 1>(A, tiles, n, list, q, st);
        else if (J == 2) launch_pairs_t<OPS, 2, 1>(A, tiles, n, list, q, st);
        else launch_pairs_t<OPS, 1, 1>(A, tiles, n, list, q, st);
        break;
    case 2:
        if (J == 2) launch_pairs_t<OPS, 2, 2>(A, tiles, n, list, q, st);
        else launch_pairs_t<OPS, 1, 2>(A, tiles, n, list, q, st);
        break;
    case 4: launch_pairs_t<OPS, 1, 4>(A, tiles, n, list, q, st); break;
    case 8: launch_pairs_t<OPS, 1, 8>(A, tiles, n, list, q, st); break;
    default: launch_pairs_t<OPS, 1, 16>(A, tiles, n, list, q, st); break;
    }
}

// queue: a zeroed device counter to run the dense tiles as one persistent
// launch over a work queue, or NULL for one block per tile.
static void launch_pairs(int OPS, ctab<PairArgs> A, const int4* tiles, int64_t n, bool list, int TP,
                         int J, hipStream_t st, unsigned long long* queue = nullptr) {
    switch (OPS) {
    case 31: launch_pairs_ops<31>(A, tiles, n, list, TP, J, queue, st); break;
    case 28: launch_pairs_ops<28>(A, tiles, n, list, TP, J, queue, st); break;
    case 3: launch_pairs_ops<3>(A, tiles, n, list, TP, J, queue, st); break;
    default: DSC_FAIL(DISCOVER_E_UNSUPPORTED, "operator class %d", OPS);
    }
}

template <bool FP16>
static void launch_lp(int cls, const PairArgs& a, const void* ylp, int ldl, double delta, hipStream_t st) {
    const unsigned blocks = (unsigned)a.n_tiles;           // one block per (j, 64 i) tile
    if (!blocks) return;
    if (!FP16) {                                           // BF16: single pass
        switch (cls) {
        case 31: k_screen_lp1<31><<<blocks, 256, 0, st>>>(a, ylp, ldl, delta); return;
        case 28: k_screen_lp1<28><<<blocks, 256, 0, st>>>(a, ylp, ldl, delta); return;
        default: DSC_FAIL(DISCOVER_E_UNSUPPORTED, "operator class %d", cls);
        }
    }
    switch (cls) {
    case 31: k_screen_lp<31, FP16><<<blocks, 256, 0, st>>>(a, ylp, ldl); break;
    case 28: k_screen_lp<28, FP16><<<blocks, 256, 0, st>>>(a, ylp, ldl); break;
    default: DSC_FAIL(DISCOVER_E_UNSUPPORTED, "operator class %d", cls);
    }
}

// Error bound of a low-precision score per unit of sqrt(kappa) (see
// k_screen_lp and k_screen_lp1): rounding both factors, u = 2^-8 (BF16) or
// 2^-11 (FP16), FP32 summation over n terms, and for BF16 the FP64 -> FP32
// step before the rounding (2^-23 for both factors).
static double lowprec_delta(int precision, int n) {
    const double u = precision == DISCOVER_FP16_GUARD ? std::ldexp(1.0, -11) : std::ldexp(1.0, -8);
    const double g = n * std::ldexp(1.0, -24);
    double d = 2 * u + u * u + 1.01 * g / (1 - g) + 1e-12;
    if (precision == DISCOVER_FP16_GUARD) d += std::ldexp(1.0, -24);
    else d += std::ldexp(1.0, -23);
    return d;
}

// Selection margin of a precision form: FP16 stores standardised values
// (kappa = 1); BF16 stores scores for kappa <= LP1_KAPPA.
static double lowprec_margin(int precision, int n) {
    const double d = lowprec_delta(precision, n);
    return precision == DISCOVER_FP16_GUARD ? d : d * std::sqrt(LP1_KAPPA);
}

// Description of one search space and its work lists, cached in the
// context: it depends only on (p, units, parameters, padded target count),
// not on the samples.  Device arrays hold what the kernels index directly;
// tile lists stay on the host and are merged per call across problems.
struct Plan {
    Space sp;
    int TP = 1, ldm = 0;
    std::vector<void*> allocs;
    int32_t* raw2c = nullptr;
    int64_t* mat_raw = nullptr;
    int8_t* mat_op = nullptr;
    int32_t *mat_a = nullptr, *mat_b = nullptr;
    ListItem* items = nullptr;
    int64_t n_items = 0;
    std::vector<int2> dtilesJ[3];             // dense (jc0, ic0) tiles for J = 1, 2, 4
    int tuned_J = 0;                          // 0: not tuned yet (single-problem calls)
    uint32_t dense_ops = 0;
    int dense_cls = 0;
    int2* ptiles = nullptr;                   // (j, i0) tiles of one j for the precision form
    int64_t n_ptiles = 0;
    std::vector<int4> ltiles;                 // list mode: (jc, list offset, count)
    int32_t* ilist = nullptr;
    uint32_t list_ops = 0;
    std::shared_ptr<R3Plan> r3;               // operator-limited rung 3 work lists
    uint32_t r3_ops = 0;
    SlotMap sm;                               // score slots of the candidates
    std::string key;

    template <class T>
    T* up(const std::vector<T>& v) {
        void* p = nullptr;
        const size_t bytes = std::max<size_t>(v.size() * sizeof(T), 16);
        if (hipMalloc(&p, bytes) != hipSuccess) DSC_FAIL(DISCOVER_E_NOMEM, "plan allocation failed");
        allocs.push_back(p);
        if (!v.empty()) DSC_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
        return (T*)p;
    }
    ~Plan() {
        for (void* p : allocs)
            if (hipFree(p) != hipSuccess) { /* nothing to do */ }
    }
};

static std::string plan_key(const discover_problem& pb, const discover_screen_params& prm) {
    std::string k((const char*)&prm.ops, sizeof prm.ops);
    k.append((const char*)&prm.rung, sizeof prm.rung);
    k.append((const char*)prm.rung_ops, sizeof prm.rung_ops);
    k.append((const char*)prm.rung_pool, sizeof prm.rung_pool);
    k.append((const char*)&prm.precision, sizeof prm.precision);
    const int32_t dims[3] = {pb.p, pb.B, pad_targets(pb.T)};
    k.append((const char*)dims, sizeof dims);
    if (pb.B && pb.units) k.append((const char*)pb.units, sizeof(int32_t) * pb.p * pb.B);
    return k;
}

static std::shared_ptr<Plan> get_plan(discover_ctx* ctx, const discover_problem& pb,
                                      const discover_screen_params& prm) {
    const std::string key = plan_key(pb, prm);
    auto it = ctx->plans.find(key);
    if (it != ctx->plans.end()) return std::static_pointer_cast<Plan>(it->second);
    if (ctx->capturing) DSC_FAIL(DISCOVER_E_CAPACITY, "search-space plan built during graph capture");
    ctx->evict_plans(64);
    auto P = std::make_shared<Plan>();
    P->key = key;
    Space& sp = P->sp;
    build_space(sp, pb.p, prm, pb.B, pb.units);
    const SpaceDev& sd = sp.d;
    P->TP = pad_targets(pb.T);
    const int Mc = sp.Mc();
    P->ldm = (int)((Mc + 63) / 64 * 64);
    P->raw2c = P->up(sp.raw2c);
    P->mat_raw = P->up(sp.mat_raw);
    P->mat_op = P->up(sp.mat_op);
    P->mat_a = P->up(sp.mat_a);
    P->mat_b = P->up(sp.mat_b);
    // operand features and unary candidates of the streamed rung: exact list
    std::vector<ListItem> items;
    for (int32_t c = 0; c < Mc; c++) items.push_back({sp.mat_raw[c], 0, OP_NONE, c, -1});
    const int R = sp.streamed;
    const int Bq = sp.B > 0 ? sp.B : 1;
    if (R) {
        const int32_t c0 = sp.rung_start[R - 1], c1 = sp.rung_start[R];
        std::vector<int32_t> tmp(Bq);
        for (int o = 0; o < OP_ADD; o++) {
            if (sd.block[R][o] < 0) continue;
            for (int32_t c = c0; c < c1; c++)
                if (unit_rule(o, sp.B, &sp.mat_unit[(size_t)c * Bq], nullptr, tmp.data()))
                    items.push_back({unary_id(sd, R, o, sp.mat_raw[c]), 1, o, c, -1});
        }
    }
    P->items = P->up(items);
    P->n_items = (int64_t)items.size();
    P->sm.s3 = P->sm.n = sp.n_raw();                     // slot = ID (rung 3 below)
    if (!R) return ctx->plans[key] = P, P;
    uint32_t bin = 0;
    for (int o = OP_ADD; o <= OP_RDIV; o++)
        if (sd.block[R][o] >= 0) bin |= 1u << (o - OP_ADD);
    const int32_t jc0 = sp.rung_start[R - 1], jc1 = sp.rung_start[R];
    const int pool = sd.pool[R];
    const int32_t i_end = pool == R - 1 ? Mc : sp.rung_start[pool + 1];
    const bool units = sp.B > 0;
    P->dense_ops = units ? (bin & 28u) : bin;
    P->list_ops = units ? (bin & 3u) : 0u;
    P->dense_cls = units ? 28 : 31;
    if (P->dense_ops) {
        for (int jx = 0; jx < 3; jx++) {
            const int J = 1 << jx;
            if (J > max_J(P->TP)) break;
            std::vector<int2>& tiles = P->dtilesJ[jx];
            for (int32_t j = jc0; j < jc1; j += J) {
                const int32_t ilim = std::min<int32_t>(i_end, std::min<int32_t>(j + J - 1, jc1 - 1));
                for (int32_t i0 = 0; i0 < ilim; i0 += 64) tiles.push_back(make_int2(j, i0));
            }
        }
        std::vector<int2> pt;
        for (int32_t j = jc0; j < jc1; j++) {
            const int32_t ilim = std::min<int32_t>(i_end, j);
            for (int32_t i0 = 0; i0 < ilim; i0 += 64) pt.push_back(make_int2(j, i0));
        }
        P->ptiles = P->up(pt);
        P->n_ptiles = (int64_t)pt.size();
    }
    std::vector<int32_t> il;
    if (P->list_ops) {
        std::map<std::string, std::vector<int32_t>> by_unit;
        auto key_of = [&](int32_t c) {
            return std::string((const char*)&sp.mat_unit[(size_t)c * Bq], sizeof(int32_t) * Bq);
        };
        if (pool != R - 1)
            for (int32_t c = 0; c < i_end; c++) by_unit[key_of(c)].push_back(c);
        for (int32_t c = 0; c < jc1; c++) {
            if (c >= jc0) {
                auto f = by_unit.find(key_of(c));
                if (f != by_unit.end()) {
                    const auto& v = f->second;
                    for (size_t q = 0; q < v.size(); q += 64) {
                        const int cnt = (int)std::min<size_t>(64, v.size() - q);
                        P->ltiles.push_back(make_int4(c, (int)il.size(), cnt, 0));
                        il.insert(il.end(), v.begin() + q, v.begin() + q + cnt);
                    }
                }
            }
            if (pool == R - 1) by_unit[key_of(c)].push_back(c);
        }
    }
    P->ilist = P->up(il);
    if (sp.stream3) {
        for (int o = OP_ADD; o <= OP_RDIV; o++)
            if (sd.block[3][o] >= 0) P->r3_ops |= 1u << (o - OP_ADD);
        P->r3 = build_r3_plan(sp, P->r3_ops);
    }
    // rung-3 slots over the plan's records (unit-legal rung-2 features)
    if (sp.stream3 && P->r3) {
        const R3Plan& r3 = *P->r3;
        P->sm.s3 = sd.off[3];
        P->sm.pe = std::max(r3.pe, 1);
        P->sm.grec = r3.grec;
        P->sm.mat_raw = P->mat_raw;
        P->sm.as_grec = r3.as_grec;
        P->sm.as_work = r3.as_work;
        P->sm.as_cols = r3.as_coldesc;
        int64_t s = sd.off[3];
        for (int q = 0; q < 5; q++) {
            const int64_t sz = q < 2 ? r3.n_as_work * 256 : r3.n_grec * r3.pe;
            if (sd.block[3][OP_ADD + q] >= 0 && sz > 0) {
                P->sm.sblk[q] = s;
                s += sz;
            }
        }
        P->sm.n = s;
    }
    ctx->plans[key] = P;
    return P;
}

struct Problem {
    std::shared_ptr<Plan> plan;
    int n, T, Tl, TP, ldn, ldm, Mc;
    int64_t N, fix_cap;
    unsigned long long* queues = nullptr;   // the call's work-queue counters (zeroed by its fills)
    double *Vf, *Rf, *Cf, *Vs, *Rs, *Cs, *mu, *mur, *msq, *Yc, *Yn, *syy, *ysum, *scores;
    uint8_t* valid;
    unsigned long long* ctr;                  // [0] bad target (int), [1] fix count, [2] scored, [3] rung-3 fix count
    int64_t *fix_ids, *fix_ids3;
    uint8_t* r2v = nullptr;                   // rung-2 operand statistics (streamed rung 3)
    double* r2m = nullptr;
    double* r2q = nullptr;
    void* ylp = nullptr;
    double* r3b = nullptr;                    // rung-3 right-hand operands
    double* r3p = nullptr;                    // rung-3 partner ranges
    int ldl = 0;
    int tile_j = 0;                           // dense pair kernel width used (0: not run)
    bool pairs = false;                       // streamed rung with pair operators
    EvalCtx ev() const {
        EvalCtx e;
        e.sd = plan->sp.d;
        e.streamed = plan->sp.streamed;
        e.stream3 = plan->sp.stream3 ? 1 : 0;
        e.raw2c = plan->raw2c;
        e.valid = valid;
        e.r2_valid = r2v;
        e.sm = plan->sm;
        return e;
    }
    Ops ops() const { return Ops{Vf, Rf, ldn}; }
};

// Per-list selection state carried across rounds (and into a captured run).
struct ListState {
    int b, t;
    int64_t K, cap, fcap;
    int n = 0;                // samples of the list's problem
    bool done = false;
};

// Pool entries whose values the rescoring keeps for the duplicate pairs:
// up to 4 GB of values per list (every entry of a pool of n = 2000 samples
// up to 268,435 entries; the pool's order is not the score order, so the
// entries the groups compare are spread over the whole pool).
static int64_t pool_vals_cap(int64_t cap, int n) {
    return std::min<int64_t>(cap, ((int64_t)1 << 32) / (8 * (int64_t)std::max(n, 1)));
}

// Allocate every problem's working memory for one call.
static void layout_problems(discover_ctx* ctx, const discover_problem* probs, int nb,
                            const discover_screen_params& prm, std::vector<Problem>& PS) {
    PS.resize(nb);
    Arena ar, ao;                                 // per call / operand features
    std::vector<std::vector<size_t>> o(nb), oo(nb);
    for (int b = 0; b < nb; b++) {
        const discover_problem& pb = probs[b];
        Problem& P = PS[b];
        P.plan = get_plan(ctx, pb, prm);
        const Plan& pl = *P.plan;
        const Space& sp = pl.sp;
        P.n = pb.n;
        P.T = pb.T;
        P.Tl = prm.score_mode == DISCOVER_SCORE_MAX ? 1 : pb.T;
        P.TP = pl.TP;
        P.ldn = (int)((pb.n + 63) / 64 * 64);
        P.ldm = pl.ldm;
        P.Mc = sp.Mc();
        P.N = pl.sm.n;
        P.fix_cap = std::min<int64_t>(P.N, ctx->fix_cap_min);
        P.pairs = sp.streamed && (pl.dense_ops || pl.list_ops);
        const size_t Mc = P.Mc, ldn = P.ldn, n = P.n, ldm = P.ldm;
        auto& v = o[b];
        auto& u = oo[b];
        for (int k = 0; k < 3; k++) u.push_back(ao.add(Mc * ldn * 8));          // Vf Rf Cf
        for (int k = 0; k < 3; k++) u.push_back(ao.add(Mc * 8));                // mu mur msq
        u.push_back(ao.add(Mc));                                               // valid
        for (int k = 0; k < 3; k++) u.push_back(ao.add(P.pairs ? n * ldm * 8 : 8));  // Vs Rs Cs
        v.push_back(ar.add((size_t)P.T * ldn * 8));                            // Yc
        v.push_back(ar.add((size_t)P.TP * ldn * 8));                           // Yn
        v.push_back(ar.add((size_t)P.T * 8));                                  // syy
        v.push_back(ar.add((size_t)P.TP * 8));                                 // ysum
        v.push_back(ar.add((size_t)P.Tl * P.N * 8));                           // scores
        v.push_back(ar.add((size_t)P.fix_cap * 8));                            // fix_ids
        v.push_back(ar.add(sp.stream3 ? (size_t)P.fix_cap * 8 : 8));           // fix_ids3
        const size_t L2 = sp.stream3 ? (size_t)sp.d.L[2] : 1;
        v.push_back(ar.add(L2));                                               // r2v
        v.push_back(ar.add(L2 * 8));                                           // r2m
        v.push_back(ar.add(L2 * 8));                                           // r2q
        P.ldl = (int)cdiv(P.n, 32) * 32;
        v.push_back(ar.add(prm.precision != DISCOVER_FP64 ? (size_t)16 * P.ldl * 2 : 8));  // Ylp
        const R3Plan* r3 = pl.r3.get();
        v.push_back(ar.add(r3 ? r3_bmat_bytes(*r3, P.TP, P.n) : 8));              // rung-3 operands
        v.push_back(ar.add(r3 ? r3_pstat_bytes(*r3, P.TP) : 8));                  // partner ranges, sums
    }
    char* base = (char*)ctx->raw("scr_arena", ar.total);
    char* obase = (char*)ctx->raw("scr_ops" + ctx->ops_tag, ao.total);
    // counters stay apart from the shared arena: a captured run checks the
    // bad-target flags after later calls have reused the arena
    unsigned long long* ctr = ctx->buf<unsigned long long>("scr_ctr" + ctx->tag, 4 * (size_t)nb);
    for (int b = 0; b < nb; b++) PS[b].ctr = ctr + 4 * b;
    for (int b = 0; b < nb; b++) {
        Problem& P = PS[b];
        const auto& v = o[b];
        const auto& u = oo[b];
        int q = 0, qo = 0;
        auto at = [&](void) { return base + v[q++]; };
        auto ato = [&](void) { return obase + u[qo++]; };
        P.Vf = (double*)ato(); P.Rf = (double*)ato(); P.Cf = (double*)ato();
        P.mu = (double*)ato(); P.mur = (double*)ato(); P.msq = (double*)ato();
        P.valid = (uint8_t*)ato();
        P.Vs = (double*)ato(); P.Rs = (double*)ato(); P.Cs = (double*)ato();
        P.Yc = (double*)at(); P.Yn = (double*)at(); P.syy = (double*)at(); P.ysum = (double*)at();
        P.scores = (double*)at();
        P.fix_ids = (int64_t*)at(); P.fix_ids3 = (int64_t*)at();
        uint8_t* r2v = (uint8_t*)at();
        double* r2m = (double*)at();
        double* r2q = (double*)at();
        if (P.plan->sp.stream3) { P.r2v = r2v; P.r2m = r2m; P.r2q = r2q; }
        P.ylp = at();
        P.r3b = (double*)at();
        P.r3p = (double*)at();
    }
}

// Merged dense / list tiles of a call: problems in decreasing n (the
// heaviest tiles first), each problem's tiles in plan order.
constexpr int MAX_QUEUES = 64;          // work-queue counters per screen (dense groups)

struct TileGroup {
    int cls, TP, J;
    bool list;
    std::vector<int4> tiles;
};

static std::vector<int> by_weight(const std::vector<Problem>& PS) {
    std::vector<int> order(PS.size());
    for (size_t b = 0; b < PS.size(); b++) order[b] = (int)b;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return PS[x].n > PS[y].n; });
    return order;
}

// Autotuned launch of a dense group: tile width J (operand features per
// wave: 1, 2, 4 as the target count allows) and schedule (one block per
// tile, or one persistent launch over a device work queue).  Each
// admissible variant is timed once for the group's shape class -- operator
// class, padded target count, and the power-of-two buckets of the largest
// sample count and of the tile count -- with the counter bumps of the trial
// runs undone (every variant writes the same scores), and the fastest is
// remembered for that class.  Returns J | queue << 8.
static int tune_dense(discover_ctx* ctx, const std::string& key, int cls, int TP,
                      ctab<PairArgs> dA, std::vector<Problem>& PS, const std::vector<int>& members,
                      int Jfix, int sched, hipStream_t st) {
    auto it = ctx->tuned.find(key);
    if (it != ctx->tuned.end()) return it->second;
    if (ctx->capturing) DSC_FAIL(DISCOVER_E_CAPACITY, "tile autotuning during graph capture");
    const std::vector<int> order = by_weight(PS);
    std::vector<unsigned long long*> saved;
    for (int b : members) {
        unsigned long long* sv = ctx->buf<unsigned long long>("tune_ctr_" + std::to_string(b), 4);
        DSC_HIP(hipMemcpyAsync(sv, PS[b].ctr, 32, hipMemcpyDeviceToDevice, st));
        saved.push_back(sv);
    }
    unsigned long long* q = ctx->buf<unsigned long long>("tune_queue", 1);
    double best = 1e30;
    int choice = 1;
    for (int jx = 0; jx < 3 && (1 << jx) <= max_J(TP); jx++) {
        if (Jfix > 0 && (1 << jx) != Jfix) continue;
        std::vector<int4> tiles;
        for (int b : order) {
            if (std::find(members.begin(), members.end(), b) == members.end()) continue;
            for (const int2& t : PS[b].plan->dtilesJ[jx]) tiles.push_back(make_int4(b, t.x, t.y, 0));
        }
        const int4* dt = ctx->upload("tune_tiles", tiles, st);
        for (int qv = 0; qv < 2; qv++) {
            if ((qv == 1 && sched < 0) || (qv == 0 && sched > 0)) continue;
            if (qv) fill_all(ctx, "tune_qfill", {fill_seg(q, 8, 0u)}, st);
            hipEvent_t e0 = ctx->event(), e1 = ctx->event();
            DSC_HIP(hipEventRecord(e0, st));
            launch_pairs(cls, dA, dt, (int64_t)tiles.size(), false, TP, 1 << jx, st, qv ? q : nullptr);
            DSC_HIP(hipEventRecord(e1, st));
            for (size_t m = 0; m < members.size(); m++)
                DSC_HIP(hipMemcpyAsync(PS[members[m]].ctr, saved[m], 32, hipMemcpyDeviceToDevice, st));
            DSC_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            DSC_HIP(hipEventElapsedTime(&ms, e0, e1));
            ctx->free_events.push_back(e0);
            ctx->free_events.push_back(e1);
            if (ms < best) { best = ms; choice = (1 << jx) | (qv << 8); }
        }
    }
    ctx->tuned[key] = choice;
    return choice;
}

static int log2_bucket(int64_t v) {
    int b = 0;
    while (v > 1) { v >>= 1; b++; }
    return b;
}

// Autotuned choice of the precision form for one problem's dense pair
// tiles: the MFMA kernel and the FP64 tiles (one operand feature per wave)
// are each timed once for this shape, their counter bumps undone, and the
// faster is remembered.  (Both give the same selection: the FP64 scores lie
// within the guard band of their own exact values.)
static bool tune_precision(discover_ctx* ctx, const std::string& key, Problem& P,
                           const std::function<void()>& run_lp, ctab<PairArgs> dA, int b, hipStream_t st) {
    auto it = ctx->tuned.find(key);
    if (it != ctx->tuned.end()) return it->second != 0;
    if (ctx->capturing) DSC_FAIL(DISCOVER_E_CAPACITY, "precision-form tuning during graph capture");
    unsigned long long* sv = ctx->buf<unsigned long long>("tune_lp_ctr", 4);
    DSC_HIP(hipMemcpyAsync(sv, P.ctr, 32, hipMemcpyDeviceToDevice, st));
    std::vector<int4> tiles;
    for (const int2& t : P.plan->dtilesJ[0]) tiles.push_back(make_int4(b, t.x, t.y, 0));
    const int4* dt = ctx->upload("tune_lp_tiles", tiles, st);
    float ms[2] = {0.f, 0.f};
    for (int v = 0; v < 2; v++) {
        hipEvent_t e0 = ctx->event(), e1 = ctx->event();
        DSC_HIP(hipEventRecord(e0, st));
        if (v == 0) run_lp();
        else launch_pairs(P.plan->dense_cls, dA, dt, (int64_t)tiles.size(), false, P.TP, 1, st);
        DSC_HIP(hipEventRecord(e1, st));
        DSC_HIP(hipMemcpyAsync(P.ctr, sv, 32, hipMemcpyDeviceToDevice, st));
        DSC_HIP(hipEventSynchronize(e1));
        DSC_HIP(hipEventElapsedTime(&ms[v], e0, e1));
        ctx->free_events.push_back(e0);
        ctx->free_events.push_back(e1);
    }
    const bool lp = ms[0] < ms[1];
    ctx->tuned[key] = lp ? 1 : 0;
    return lp;
}

// Materialise the operand features of every problem and screen every
// candidate into its score slots (no host synchronisation).
static void screen_all(discover_ctx* ctx, const discover_problem* probs, int nb,
                       const discover_screen_params& prm, std::vector<Problem>& PS, hipStream_t st,
                       const std::function<void(std::vector<FillSeg>&)>& more_fills = nullptr) {
    layout_problems(ctx, probs, nb, prm, PS);
    // 1. fills: counters, padded target rows, score slots (NaN pattern), rung-2 flags,
    // the work-queue counters of the dense groups
    std::vector<FillSeg> fills;
    unsigned long long* queues = ctx->buf<unsigned long long>("scr_queue" + ctx->tag, MAX_QUEUES);
    fills.push_back(fill_seg(queues, MAX_QUEUES * 8, 0u));
    for (Problem& P : PS) {
        P.queues = queues;
        fills.push_back(fill_seg(P.ctr, 32, 0u));
        fills.push_back(fill_seg(P.Yn, (size_t)P.TP * P.ldn * 8, 0u));
        fills.push_back(fill_seg(P.ysum, (size_t)P.TP * 8, 0u));
        fills.push_back(fill_seg(P.scores, (size_t)P.Tl * P.N * 8, 0xFFFFFFFFu));
        if (P.r2v) fills.push_back(fill_seg(P.r2v, ((size_t)P.plan->sp.d.L[2] + 3) & ~size_t(3), 0u));
    }
    if (more_fills) more_fills(fills);                  // e.g. the first selection round's counters
    fill_all(ctx, "scr_fills", fills, st);
    // 2. targets
    std::vector<TgtArgs> ta(nb);
    for (int b = 0; b < nb; b++) {
        const Problem& P = PS[b];
        ta[b] = TgtArgs{P.n, P.T, P.ldn, probs[b].Y, probs[b].ldy, P.Yc, P.Yn, P.syy, P.ysum, (int*)P.ctr};
    }
    k_targets<<<dim3(DISCOVER_MAX_TARGETS, nb), 256, 0, st>>>(ct(ctx->upload("scr_tgt", ta, st)));
    check_launch("k_targets");
    // 3. operand features, rung by rung
    std::vector<MatArgs> ma(nb);
    int nlev = 0, nmax = 0;
    std::vector<int> wmax(4, 0);
    for (int b = 0; b < nb; b++) {
        const Problem& P = PS[b];
        const Plan& pl = *P.plan;
        MatArgs& a = ma[b];
        a = MatArgs{};
        a.n = P.n; a.ldn = P.ldn;
        a.nlev = (int)pl.sp.rung_start.size() - 1;
        for (int r = 0; r <= a.nlev && r < 4; r++) a.rs[r] = pl.sp.rung_start[r];
        a.X = probs[b].X; a.ldx = probs[b].ldx;
        a.op = pl.mat_op; a.ca = pl.mat_a; a.cb = pl.mat_b; a.raw = pl.mat_raw;
        a.Vf = P.Vf; a.Rf = P.Rf; a.Cf = P.Cf; a.mu = P.mu; a.mur = P.mur; a.msq = P.msq;
        a.valid = P.valid;
        nlev = std::max(nlev, a.nlev);
        nmax = std::max(nmax, P.n);
        for (int r = 0; r < a.nlev; r++) wmax[r] = std::max(wmax[r], a.rs[r + 1] - a.rs[r]);
    }
    // the operands of these problems are already in place (same arena, same
    // layout, same X) when an earlier screen of the sequence made them
    std::vector<int64_t> sig;
    for (int b = 0; b < nb; b++) {
        const Problem& P = PS[b];
        sig.insert(sig.end(), {(int64_t)(uintptr_t)probs[b].X, probs[b].ldx, (int64_t)P.n, (int64_t)P.Mc,
                               (int64_t)P.ldn, (int64_t)P.ldm, (int64_t)P.pairs,
                               (int64_t)(uintptr_t)P.Vf, (int64_t)(uintptr_t)P.Vs});
        const auto& rs = P.plan->sp.rung_start;
        sig.insert(sig.end(), rs.begin(), rs.end());
    }
    const bool ops_ready = ctx->ops_reuse && sig == ctx->ops_sig;
    ctx->ops_sig = sig;
    const ctab<MatArgs> dma = ct(ctx->upload("scr_mat", ma, st));
    if (!ops_ready) {
        KTimer kt(ctx, st, "materialise");
        for (int r = 0; r < nlev; r++) {
            if (!wmax[r]) continue;
            k_mat_values<<<dim3((unsigned)cdiv(nmax, 256), (unsigned)wmax[r], nb), 256, 0, st>>>(dma, r);
            k_mat_stats<<<dim3((unsigned)cdiv(wmax[r], 4), nb), 256, 0, st>>>(dma, r);
        }
        check_launch("k_mat");
    }
    // 4. exact list: operand features and unary candidates of the streamed rung
    std::vector<ListArgs> la(nb);
    int64_t mmax = 0;
    for (int b = 0; b < nb; b++) {
        const Problem& P = PS[b];
        const Plan& pl = *P.plan;
        const SpaceDev& sd = pl.sp.d;
        ListArgs& a = la[b];
        a = ListArgs{};
        a.items = pl.items; a.m = pl.n_items; a.o = P.ops(); a.valid = P.valid;
        a.n = P.n; a.T = P.T; a.mode = prm.score_mode; a.Yc = P.Yc; a.syy = P.syy; a.N = P.N;
        a.scores = P.scores; a.nscored = P.ctr + 2;
        a.r2v = P.r2v; a.r2m = P.r2m; a.r2q = P.r2q;
        a.off2 = pl.sp.stream3 ? sd.off[2] : 0;
        a.off3 = pl.sp.stream3 ? sd.off[3] : 0;
        mmax = std::max(mmax, a.m);
    }
    {
        KTimer kt(ctx, st, "screen_list");
        k_score_list<<<dim3((unsigned)cdiv(mmax, 4), nb), 256, 0, st>>>(ct(ctx->upload("scr_list", la, st)));
        check_launch("k_score_list");
    }
    // 5. sample-major copies of the operands of the pair kernels
    std::vector<TrArgs> tr;
    std::vector<int> trb;
    int tn = 0, tm = 0;
    for (int b = 0; b < nb; b++) {
        const Problem& P = PS[b];
        if (!P.pairs) continue;
        tr.push_back(TrArgs{P.n, P.Mc, P.ldn, P.ldm, {P.Vf, P.Rf, P.Cf}, {P.Vs, P.Rs, P.Cs}});
        tn = std::max(tn, P.n);
        tm = std::max(tm, P.Mc);
    }
    if (!tr.empty() && !ops_ready) {
        k_transpose<<<dim3((unsigned)cdiv(tn, 32), (unsigned)cdiv(tm, 32), (unsigned)(3 * tr.size())),
                      dim3(32, 8), 0, st>>>(ct(ctx->upload("scr_tr", tr, st)));
        check_launch("k_transpose");
    }
    // 6. pair kernels
    std::vector<PairArgs> pa(nb);
    for (int b = 0; b < nb; b++) {
        const Problem& P = PS[b];
        const Plan& pl = *P.plan;
        const Space& sp = pl.sp;
        PairArgs& a = pa[b];
        a = PairArgs{};
        if (!P.pairs) continue;
        const int R = sp.streamed;
        const int pool = sp.d.pool[R];
        a.n = P.n; a.ldm = P.ldm; a.ldn = P.ldn; a.Mc = P.Mc; a.jc_end = sp.rung_start[R];
        a.i_end = pool == R - 1 ? P.Mc : sp.rung_start[pool + 1];
        a.Vs = P.Vs; a.Rs = P.Rs; a.Cs = P.Cs; a.Vf = P.Vf; a.Rf = P.Rf; a.Cf = P.Cf;
        a.mu = P.mu; a.mur = P.mur; a.valid = P.valid; a.mat_raw = pl.mat_raw;
        a.Yn = P.Yn; a.ysum = P.ysum; a.T = P.T; a.mode = prm.score_mode; a.r = R;
        a.sd = sp.d; a.N = P.N; a.scores = P.scores; a.nscored = P.ctr + 2;
        a.fix_cap = P.fix_cap; a.fix_ids = P.fix_ids; a.fix_cnt = P.ctr + 1;
        a.r2v = P.r2v; a.r2m = P.r2m; a.r2q = P.r2q; a.msq = P.msq;
        a.ilist = pl.ilist;
        a.opmask = pl.dense_ops;
    }
    const ctab<PairArgs> dpa = ct(ctx->upload("scr_pairs", pa, st));
    const std::vector<int> order = by_weight(PS);
    // 6a. precision form: per problem, MFMA screening with FP64 guard-band
    // rescore, where the autotuner found it faster than the FP64 tiles for
    // this problem's shape (either gives the same selection)
    std::vector<char> lp_used(nb, 0);
    for (int b = 0; b < nb; b++) {
        Problem& P = PS[b];
        const Plan& pl = *P.plan;
        if (!P.pairs || !pl.dense_ops || prm.precision == DISCOVER_FP64) continue;
        const bool fp16 = prm.precision == DISCOVER_FP16_GUARD;
        dim3 gy((unsigned)cdiv(P.ldl, 256), 16);
        if (fp16) k_targets_lp<true><<<gy, 256, 0, st>>>(P.n, P.T, P.ldn, P.ldl, P.Yn, (_Float16*)P.ylp);
        else k_targets_lp<false><<<gy, 256, 0, st>>>(P.n, P.T, P.ldn, P.ldl, P.Yn, (__bf16*)P.ylp);
        PairArgs a = pa[b];
        a.tiles = pl.ptiles; a.n_tiles = pl.n_ptiles;
        const double dl = lowprec_delta(prm.precision, P.n);
        auto run_lp = [&] {
            if (fp16) launch_lp<true>(pl.dense_cls, a, P.ylp, P.ldl, dl, st);
            else launch_lp<false>(pl.dense_cls, a, P.ylp, P.ldl, dl, st);
            check_launch("k_screen_lp");
        };
        if (prm.lp_pairs < 0 ||
            (prm.lp_pairs == 0 &&
             !tune_precision(ctx, "lp" + pl.key + std::to_string(P.n) + (fp16 ? "h" : "b"), P, run_lp, dpa, b, st)))
            continue;                            // FP64 tiles below
        lp_used[b] = 1;
        KTimer kt(ctx, st, "screen_lp");
        run_lp();
    }
    // 6b. FP64 dense tiles, merged per (operator class, padded targets)
    std::map<std::pair<int, int>, std::vector<int>> groups;
    for (int b : order) {
        const Problem& P = PS[b];
        if (P.pairs && P.plan->dense_ops && !lp_used[b])
            groups[{P.plan->dense_cls, P.TP}].push_back(b);
    }
    int gi = 0;
    unsigned long long* const gqueues = PS.empty() ? nullptr : PS[0].queues;
    for (auto& g : groups) {
        const int cls = g.first.first, TP = g.first.second;
        const std::vector<int>& mem = g.second;
        int J = 1;
        bool useq = prm.sched > 0;
        if (prm.tile_j > 0) {
            while (J * 2 <= std::min(prm.tile_j, max_J(TP))) J *= 2;
        }
        if (prm.tile_j == 0 || prm.sched == 0) {
            // shape class: operator class, padded targets, buckets of the
            // largest n and of the tile count
            int nmax = 0;
            int64_t nt = 0;
            for (int b : mem) {
                nmax = std::max(nmax, PS[b].n);
                nt += (int64_t)PS[b].plan->dtilesJ[0].size();
            }
            const std::string key = "dense|" + std::to_string(cls) + "|" + std::to_string(TP) + "|" +
                                    std::to_string(log2_bucket(nmax)) + "|" + std::to_string(log2_bucket(nt)) +
                                    "|" + std::to_string(prm.tile_j) + "|" + std::to_string(prm.sched);
            const int c = tune_dense(ctx, key, cls, TP, dpa, PS, mem, prm.tile_j > 0 ? J : 0, prm.sched, st);
            if (prm.tile_j == 0) J = c & 0xFF;
            if (prm.sched == 0) useq = (c >> 8) != 0;
        }
        const int jx = J == 4 ? 2 : J == 2 ? 1 : 0;
        std::vector<int4> tiles;
        for (int b : mem) {
            PS[b].tile_j = J;
            for (const int2& t : PS[b].plan->dtilesJ[jx]) tiles.push_back(make_int4(b, t.x, t.y, 0));
        }
        const int4* dt = ctx->upload("scr_dtiles" + std::to_string(gi), tiles, st);
        KTimer kt(ctx, st, "screen_pairs");
        if (useq && gi >= MAX_QUEUES) useq = false;   // (more groups than queue counters)
        launch_pairs(cls, dpa, dt, (int64_t)tiles.size(), false, TP, J, st, useq ? gqueues + gi : nullptr);
        check_launch("k_screen_pairs");
        gi++;
    }
    // 6c. same-unit add/sub partner lists (FP64 in every form), merged per TP
    std::map<int, std::vector<int4>> lgroups;
    for (int b : order) {
        const Problem& P = PS[b];
        if (!P.pairs || !P.plan->list_ops) continue;
        for (const int4& t : P.plan->ltiles) lgroups[P.TP].push_back(make_int4(b, t.x, t.y, t.z));
    }
    if (!lgroups.empty()) {
        // list-mode arguments differ from the dense ones only in the operator mask
        std::vector<PairArgs> pl2 = pa;
        for (int b = 0; b < nb; b++) pl2[b].opmask = PS[b].plan->list_ops;
        const ctab<PairArgs> dpl = ct(ctx->upload("scr_pairs_list", pl2, st));
        int li = 0;
        for (auto& g : lgroups) {
            const int4* dt = ctx->upload("scr_ltiles" + std::to_string(li++), g.second, st);
            KTimer kt(ctx, st, "screen_pairs_list");
            launch_pairs(3, dpl, dt, (int64_t)g.second.size(), true, g.first, 1, st);
            check_launch("k_screen_pairs(list)");
        }
    }
    // 7. exact decisions for the ill-conditioned candidates
    std::vector<FixArgs> fa(nb);
    for (int b = 0; b < nb; b++) {
        const Problem& P = PS[b];
        FixArgs& a = fa[b];
        a = FixArgs{};
        a.ids = P.fix_ids; a.cnt = P.ctr + 1; a.cap = P.fix_cap; a.ev = P.ev(); a.o = P.ops();
        a.n = P.n; a.T = P.T; a.mode = prm.score_mode; a.Yc = P.Yc; a.syy = P.syy; a.N = P.N;
        a.scores = P.scores; a.nscored = P.ctr + 2; a.r2v = P.r2v; a.r2m = P.r2m; a.r2q = P.r2q;
    }
    {
        KTimer kt(ctx, st, "screen_fixup");
        const unsigned fb = (unsigned)std::max(1, std::min(1024, 4096 / nb));
        launch_fixup(fa, dim3(fb, nb), ct(ctx->upload("scr_fix", fa, st)), st);
        check_launch("k_fixup");
    }
    // 8. operator-limited rung 3 on top of the rung-2 operand statistics
    std::vector<FixArgs> fa3;
    for (int b = 0; b < nb; b++) {
        Problem& P = PS[b];
        const Plan& pl = *P.plan;
        const Space& sp = pl.sp;
        const SpaceDev& sd = sp.d;
        if (!sp.stream3 || !pl.r3_ops || !pl.r3) continue;
        R3Launch g3{};
        g3.plan = pl.r3.get();
        g3.n = P.n; g3.ldn = P.ldn; g3.TP = P.TP; g3.T = P.T; g3.mode = prm.score_mode;
        g3.Vf = P.Vf; g3.Rf = P.Rf; g3.Cf = P.Cf; g3.mu = P.mu; g3.msq = P.msq;
        g3.valid = P.valid; g3.mat_raw = pl.mat_raw; g3.Yn = P.Yn; g3.ysum = P.ysum;
        g3.r2v = P.r2v; g3.r2m = P.r2m; g3.r2q = P.r2q; g3.sd = sd; g3.sm = pl.sm; g3.N = P.N;
        g3.scores = P.scores; g3.nscored = P.ctr + 2; g3.fix_ids = P.fix_ids3;
        g3.fix_cnt = P.ctr + 3; g3.fix_cap = P.fix_cap; g3.bmat = P.r3b; g3.pstat = P.r3p;
        // the precision form covers rung 3 in BF16 (FP16's range would need
        // per-row scaling; the FP16 form keeps rung 3 in FP64)
        g3.precision = prm.precision;
        g3.delta = prm.precision == DISCOVER_BF16_GUARD ? lowprec_delta(prm.precision, P.n) : 0.0;
        launch_r3(ctx, g3, st);
        FixArgs a = fa[b];
        a.ids = P.fix_ids3; a.cnt = P.ctr + 3; a.r2v = nullptr; a.r2m = nullptr; a.r2q = nullptr;
        fa3.push_back(a);
    }
    if (!fa3.empty()) {
        KTimer kt(ctx, st, "screen_fixup");
        launch_fixup(fa3, dim3(1024, (unsigned)fa3.size()), ct(ctx->upload("scr_fix3", fa3, st)), st);
        check_launch("k_fixup");
    }
}

// Launch one round of exact top-k for the given lists.  The pool of a list
// holds every candidate whose score can reach its K-th largest approximate
// score minus the error margin; it is rescored exactly and grouped in
// (-score, ID) order.
// Layout of one selection round's arena: per active list, the offsets of
// its arrays (pool, scores, ..., counters at SEL_MISC, histograms at
// SEL_HIST, stored pool values).
constexpr int SEL_MISC = 17, SEL_HIST = 18;

static char* sel_layout(discover_ctx* ctx, int k, const std::vector<ListState>& LS,
                        const std::vector<int>& act, std::vector<std::vector<size_t>>& o) {
    const int nl = (int)act.size();
    Arena ar;
    o.assign(nl, {});
    for (int q = 0; q < nl; q++) {
        const ListState& L = LS[act[q]];
        const size_t cap = (size_t)L.cap, fcap = (size_t)L.fcap;
        auto& v = o[q];
        v.push_back(ar.add(cap * 8));              // pool
        v.push_back(ar.add(cap * 8));              // ps
        v.push_back(ar.add(cap));                  // pex
        v.push_back(ar.add(cap * 4));              // order
        v.push_back(ar.add(cap * 4));              // lo
        v.push_back(ar.add(cap * 4));              // wc
        v.push_back(ar.add(cap * 4));              // rank
        v.push_back(ar.add(cap * 8));              // ss
        v.push_back(ar.add(cap * 8));              // perr
        v.push_back(ar.add((cap + 1) * 8));        // off
        v.push_back(ar.add(fcap));                 // flag
        v.push_back(ar.add((cap + 1) * 4));        // parent
        v.push_back(ar.add((cap + 1) * 4));        // blk
        v.push_back(ar.add((cap + 1) * 8));        // repid
        v.push_back(ar.add((cap + 1) * 4));        // reppos
        v.push_back(ar.add(((size_t)k + 1) * 4));  // headpos
        v.push_back(ar.add(64));                   // res
        v.push_back(ar.add(64));                   // cnt, maxerr, st[2], sel[4]
        v.push_back(ar.add(8192 * 4));             // hist (two levels)
        const size_t pvc = (size_t)pool_vals_cap(L.cap, L.n);
        v.push_back(ar.add(pvc * (size_t)L.n * 8)); // stored pool values
        v.push_back(ar.add(pvc * 8));              // their means
        v.push_back(ar.add(pvc * 8));              // their centred sums of squares
        v.push_back(ar.add(RK_NB * 4 + 64));       // rank buckets and their key range
    }
    return (char*)ctx->raw("sel_arena" + ctx->tag, ar.total);
}

// The rule table of one problem (NULL without rules): the operand
// features' metadata from the plan, uploaded with the rules.
static const RuleTab* rule_table(discover_ctx* ctx, const Problem& P, int b, hipStream_t st) {
    if (!ctx->has_rules) return nullptr;
    const Space& sp = P.plan->sp;
    const discover_rules& R = ctx->rules;
    const int Mc = sp.Mc(), B = sp.B;
    RuleTab t{};
    for (int i = 0; i + 1 < (int)ctx->rule_pairs.size(); i += 2) {
        const int u = ctx->rule_pairs[i], v = ctx->rule_pairs[i + 1];
        t.forb[u] |= 1ull << v;
        t.forb[v] |= 1ull << u;
    }
    for (int o = 0; o < 10; o++) t.nest[o] = R.forbid_nest[o];
    t.max_cplx = R.max_complexity;
    t.B = B;
    t.target = R.target_unit && B > 0 ? 1 : 0;
    for (int k = 0; k < B && k < 8; k++) t.tunit[k] = R.target_units[k] * (1 << sp.d.R);
    std::vector<RuleFeat> f(Mc);
    auto forbidden = [&](uint64_t A, uint64_t Bm) {
        for (int u = 0; u < 64; u++)
            if ((A >> u & 1ull) && (t.forb[u] & Bm)) return true;
        return false;
    };
    for (int c = 0; c < Mc; c++) {
        RuleFeat& x = f[c];
        const int op = sp.mat_op[c];
        if (op == OP_NONE) {
            const int64_t prim = sp.mat_raw[c];
            x.vars = prim < 64 ? 1ull << prim : 0;
            x.cplx = 0;
            x.top = (int8_t)OP_NONE;
            x.ok = 1;
            continue;
        }
        const int a = sp.mat_a[c], bb = sp.mat_b[c];
        x.cplx = 1 + f[a].cplx + (bb >= 0 ? f[bb].cplx : 0);
        x.vars = f[a].vars | (bb >= 0 ? f[bb].vars : 0);
        x.top = (int8_t)op;
        bool good = f[a].ok && (bb < 0 || f[bb].ok);
        if (R.max_complexity >= 0 && x.cplx > R.max_complexity) good = false;
        if (f[a].top != OP_NONE && (R.forbid_nest[op] >> f[a].top & 1u)) good = false;
        if (bb >= 0 && f[bb].top != OP_NONE && (R.forbid_nest[op] >> f[bb].top & 1u)) good = false;
        if (bb >= 0 && forbidden(f[a].vars, f[bb].vars)) good = false;
        x.ok = good ? 1 : 0;
    }
    const std::string sfx = std::to_string(b);
    t.feat = ctx->upload("sel_rule_feat" + sfx, f, st);
    t.unit = t.target ? ctx->upload("sel_rule_unit" + sfx, sp.mat_unit, st) : nullptr;
    return (const RuleTab*)ctx->upload("sel_rule_tab" + sfx, &t, sizeof t, st);
}

static void select_round(discover_ctx* ctx, const discover_problem* probs,
                         const discover_screen_params& prm, std::vector<Problem>& PS,
                         const std::vector<ListState>& LS, const std::vector<int>& act,
                         const std::vector<double>& margin, const std::vector<ScreenOut>& outs,
                         hipStream_t st, std::vector<SelArgs>& sa, bool prefilled = false) {
    const int nl = (int)act.size();
    const int k = prm.k;
    std::vector<std::vector<size_t>> o;
    char* base = sel_layout(ctx, k, LS, act, o);
    sa.assign(nl, SelArgs{});
    std::vector<RadixArgs> ra(nl);
    std::vector<FillSeg> fills;
    int64_t Nmax = 1, capmax = 1, Kmax = 1;
    std::vector<int64_t> vbase(PS.size() + 1, 0);              // value-row addresses, laid out as the IDs
    for (size_t b = 0; b < PS.size(); b++) vbase[b + 1] = vbase[b] + (int64_t)PS[b].Tl * k;
    int64_t* vrow = ctx->buf<int64_t>("scr_vrow" + ctx->tag, (size_t)vbase.back());
    std::map<int, const RuleTab*> rtab;      // one rule table per problem
    for (int q = 0; q < nl; q++) {
        const ListState& L = LS[act[q]];
        const Problem& P = PS[L.b];
        const discover_problem& pb = probs[L.b];
        const auto& v = o[q];
        SelArgs& a = sa[q];
        int j = 0;
        auto at = [&](void) { return base + v[j++]; };
        a.pool = (int64_t*)at(); a.ps = (double*)at(); a.pex = (uint8_t*)at();
        a.order = (int32_t*)at(); a.lo = (int32_t*)at(); a.wc = (int32_t*)at();
        a.rank = (int32_t*)at(); a.ss = (double*)at(); a.perr = (double*)at();
        a.off = (int64_t*)at(); a.flag = (uint8_t*)at();
        a.parent = (int32_t*)at(); a.blk = (int32_t*)at(); a.repid = (unsigned long long*)at();
        a.reppos = (int32_t*)at(); a.headpos = (int32_t*)at(); a.res = (int64_t*)at();
        char* misc = at();
        uint32_t* hist = (uint32_t*)at();
        a.pvs.v = (double*)at(); a.pvs.mean = (double*)at(); a.pvs.sxx = (double*)at();
        a.rkh = (uint32_t*)at(); a.rkr = (unsigned long long*)(a.rkh + RK_NB);
        a.pvs.ld = L.n; a.pvs.cap = pool_vals_cap(L.cap, L.n);
        a.cnt = (unsigned long long*)misc;
        a.maxerr = (unsigned long long*)(misc + 8);
        a.ncl = (unsigned long long*)(misc + 48);
        a.pd = (unsigned long long*)(misc + 56);
        int64_t* stv = (int64_t*)(misc + 16);
        uint32_t* sel = (uint32_t*)(misc + 32);
        a.th1d = (uint32_t*)(misc + 44);
        a.sel = sel; a.st = stv; a.hist = hist;
        a.sc = P.scores + (int64_t)L.t * P.N; a.N = P.N;
        a.margin = margin[L.b]; a.cap = L.cap; a.fcap = L.fcap; a.K = L.K;
        a.ev = P.ev(); a.o = P.ops(); a.n = P.n; a.T = P.T; a.mode = prm.score_mode; a.t = L.t;
        a.k = k; a.dedup = prm.dedup;
        a.Yc = P.Yc; a.syy = P.syy;
        a.excl = pb.exclude; a.n_excl = pb.exclude ? pb.n_exclude : 0;
        auto rt = rtab.find(L.b);
        if (rt == rtab.end()) rt = rtab.emplace(L.b, rule_table(ctx, P, L.b, st)).first;
        a.rules = rt->second;
        a.out_ids = outs[L.b].ids + (int64_t)L.t * k;
        a.out_sc = outs[L.b].sc + (int64_t)L.t * k;
        a.vrow = vrow + vbase[L.b] + (int64_t)L.t * k;
        ra[q] = RadixArgs{a.sc, P.N, L.K, hist, sel, stv, nullptr};
        fills.push_back(fill_seg(misc, 64, 0u));            // pool count, maximum error, st, sel, clusters, prefix
        fills.push_back(fill_seg(hist, 8192 * 4, 0u));
        fills.push_back(fill_seg(a.rkh, RK_NB * 4 + 64, 0u));
        Nmax = std::max(Nmax, P.N);
        capmax = std::max(capmax, L.cap);
        Kmax = std::max(Kmax, L.K);
    }
    if (!prefilled) fill_all(ctx, "sel_fills", fills, st);     // else cleared with the screen's fills
    const ctab<SelArgs> dsa = ct(ctx->upload("sel_args", sa, st));
    const RadixArgs* dra = ctx->upload("sel_radix", ra, st);
    {
        KTimer kt(ctx, st, "select");
        radix_select(dra, nl, Nmax, st, 1);
    }
    const unsigned hb = (unsigned)std::min<int64_t>(1024, std::max<int64_t>(1, cdiv(Nmax, 256 * 8)));
    k_compact<<<dim3(hb, nl), 256, 0, st>>>(dsa);
    check_launch("k_compact");
    {
        KTimer kt(ctx, st, "rescore");
        int Tm = 1;
        for (const SelArgs& x : sa) Tm = std::max(Tm, x.T);
        const dim3 rg((unsigned)std::min<int64_t>(std::max(64, 2048 / nl), cdiv(capmax, 4)), nl);
        const dim3 sg((unsigned)std::min<int64_t>(1024, cdiv(capmax, 256)), nl);
        for (int stage = 0; stage < 2; stage++) {
            k_split<<<sg, 256, 0, st>>>(dsa, stage);
            if (Tm <= 1) k_rescore<1><<<rg, 256, 0, st>>>(dsa, stage);
            else if (Tm <= 8) k_rescore<8><<<rg, 256, 0, st>>>(dsa, stage);
            else k_rescore<DISCOVER_MAX_TARGETS><<<rg, 256, 0, st>>>(dsa, stage);
        }
        check_launch("k_rescore");
    }
    {
        KTimer kt(ctx, st, "sort_dedup");
        if (capmax <= RANK_PAIRS_MAX) {
            // ranks by counting over all pairs (tiles of the expected pool size,
            // grid-strided beyond it): one launch, for pools of a few thousand
            const unsigned ri = (unsigned)std::max<int64_t>(1, std::min<int64_t>(64, cdiv(Kmax + 256, 256)));
            const unsigned rj = (unsigned)std::max<int64_t>(1, std::min<int64_t>(64, cdiv(Kmax + 256, RCH)));
            k_rankp<<<dim3(ri, rj, nl), 256, 0, st>>>(dsa);
        } else {
            // ranks through score buckets (grid-strided over the pool)
            const unsigned rb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(1024, cdiv(capmax, 256)));
            k_rk_range<<<dim3(rb, nl), 256, 0, st>>>(dsa);
            k_rk_hist<<<dim3(rb, nl), 256, 0, st>>>(dsa);
            k_rk_scan<<<nl, 1024, 0, st>>>(dsa);
            k_rk_scatter<<<dim3(rb, nl), 256, 0, st>>>(dsa);
            k_rk_rank<<<dim3(rb, nl), 256, 0, st>>>(dsa);
        }
        k_scatter<<<dim3((unsigned)std::min<int64_t>(1024, cdiv(capmax, 256)), nl), 256, 0, st>>>(dsa);
        k_clusters<<<dim3((unsigned)std::min<int64_t>(1024, cdiv(capmax, 256)), nl), 256, 0, st>>>(dsa);
        check_launch("k_sort");
    }
    if (prm.dedup) {
        KTimer kt(ctx, st, "dedup_pairs");
        k_dedup_first<<<dim3((unsigned)std::max(256, 4096 / nl), nl), 256, 0, st>>>(dsa);
        k_dedup<<<dim3((unsigned)std::max(64, 1024 / nl), nl), DEDUP_THREADS, 0, st>>>(dsa);
        check_launch("k_dedup");
    }
    {
        KTimer kt(ctx, st, "groups");
        k_groups<<<nl, GRP_THREADS, 0, st>>>(dsa);
        check_launch("k_groups");
    }
}

// Grow the result arena to what one round over every list needs.
static void select_reserve(discover_ctx* ctx, const discover_screen_params& prm,
                           const std::vector<ListState>& LS) {
    Arena ar;
    for (const ListState& L : LS) {
        const size_t cap = (size_t)L.cap, fcap = (size_t)L.fcap;
        const size_t pvc = (size_t)pool_vals_cap(L.cap, L.n);
        for (size_t b : {cap * 8, cap * 8, cap, cap * 4, cap * 4, cap * 4, cap * 4, cap * 8, cap * 8, (cap + 1) * 8, fcap,
                         (cap + 1) * 4, (cap + 1) * 4, (cap + 1) * 8, (cap + 1) * 4,
                         ((size_t)prm.k + 1) * 4, (size_t)64, (size_t)64, (size_t)8192 * 4,
                         pvc * (size_t)L.n * 8, pvc * 8, pvc * 8})
            ar.add(b);
    }
    ctx->raw("sel_arena" + ctx->tag, ar.total);
}

static void validate(const discover_problem* probs, int32_t nb, const discover_screen_params* prm,
                     const int64_t* out_ids, const double* out_sc, const double* out_values,
                     int64_t ldv) {
    DSC_REQUIRE(probs && prm && nb >= 1, "probs/prm must be non-NULL and n_problems >= 1");
    DSC_REQUIRE(nb <= 65535, "n_problems = %d > 65535", nb);
    DSC_REQUIRE(out_ids && out_sc, "out_ids and out_scores are required");
    DSC_REQUIRE(prm->rung >= 0 && prm->rung <= DISCOVER_MAX_RUNG, "rung %d outside 0..3", prm->rung);
    DSC_REQUIRE(prm->k >= 1, "k must be >= 1");
    DSC_REQUIRE((prm->ops & ~DISCOVER_OPS_ALL) == 0, "unknown operator bits 0x%x", prm->ops);
    DSC_REQUIRE(prm->score_mode == DISCOVER_SCORE_PER_TARGET || prm->score_mode == DISCOVER_SCORE_MAX,
                "score_mode %d", prm->score_mode);
    DSC_REQUIRE(prm->precision >= DISCOVER_FP64 && prm->precision <= DISCOVER_FP16_GUARD,
                "precision %d", prm->precision);
    DSC_REQUIRE(prm->tile_j >= 0 && prm->tile_j <= 4, "tile_j %d outside 0..4", prm->tile_j);
    DSC_REQUIRE(prm->lp_pairs >= -1 && prm->lp_pairs <= 1, "lp_pairs %d outside -1..1", prm->lp_pairs);
    DSC_REQUIRE(prm->sched >= -1 && prm->sched <= 1, "sched %d outside -1..1", prm->sched);
    for (int r = 1; r <= prm->rung; r++) {
        DSC_REQUIRE((prm->rung_ops[r] & ~DISCOVER_OPS_ALL) == 0, "unknown operator bits at rung %d", r);
        DSC_REQUIRE(prm->rung_pool[r] >= -1 && prm->rung_pool[r] < r, "rung_pool[%d]", r);
    }
    for (int b = 0; b < nb; b++) {
        const discover_problem& p = probs[b];
        DSC_REQUIRE(p.n >= 3, "problem %d: n = %d < 3", b, p.n);
        DSC_REQUIRE(p.p >= 1 && p.p <= 4096, "problem %d: p = %d", b, p.p);
        DSC_REQUIRE(p.T >= 1 && p.T <= DISCOVER_MAX_TARGETS, "problem %d: T = %d", b, p.T);
        DSC_REQUIRE(p.B >= 0 && p.B <= DISCOVER_MAX_UNITS, "problem %d: B = %d", b, p.B);
        DSC_REQUIRE(p.B == 0 || p.units, "problem %d: units required when B > 0", b);
        DSC_REQUIRE(p.X && p.Y, "problem %d: X and Y are required", b);
        DSC_REQUIRE(p.ldx >= p.n && p.ldy >= p.n, "problem %d: ldx/ldy < n", b);
        DSC_REQUIRE(p.n_exclude >= 0 && (p.n_exclude == 0 || p.exclude), "problem %d: exclude", b);
        DSC_REQUIRE(!out_values || ldv >= p.n, "problem %d: ldv < n", b);
    }
}

// Capacities of every list of a call, remembered so that a captured run of
// the same call starts from the sizes the eager run settled on.
struct SelMemo {
    std::vector<int64_t> K, cap, fcap;
};

// The shape of a call (parameters, sizes, units; not the data): the key of
// its remembered capacities.
static std::string call_key(const discover_problem* probs, int nb, const discover_screen_params& prm) {
    std::string k((const char*)&prm, sizeof prm);
    for (int b = 0; b < nb; b++) {
        const discover_problem& p = probs[b];
        const int64_t f[5] = {p.n, p.p, p.T, p.B, p.n_exclude};
        k.append((const char*)f, sizeof f);
        if (p.B && p.units) k.append((const char*)p.units, sizeof(int32_t) * p.p * p.B);
    }
    return k;
}

bool screen_sizes_known(discover_ctx* ctx, const discover_problem* probs, int nb,
                        const discover_screen_params& prm) {
    return ctx->batches.count("sel" + call_key(probs, nb, prm)) != 0;
}

// Host-known counters of one problem and where its lists' checks start.
struct StatBase {
    discover_screen_stats s;
    int32_t l0, nl;
};

// Stats of a call that did not wait for the stream: one thread per problem
// folds its lists' outcomes into the counters and the status.
__global__ __launch_bounds__(256) void k_screen_stats(ctab<StatBase> base, ctab<ListCheck> L, int nb,
                                                      discover_screen_stats* __restrict__ out) {
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= nb) return;
    const StatBase& B = tab(base, b);
    discover_screen_stats s = B.s;
    int status = DISCOVER_OK;
    for (int l = B.l0; l < B.l0 + B.nl; l++) {
        const ListCheck& c = tab(L, l);
        const int64_t* r = c.res;
        const unsigned long long* ctr = c.ctr;
        DSC_GLOBAL(r); DSC_GLOBAL(ctr); DSC_GLOBAL(c.maxerr);
        const int v = list_status(c, r, ctr);
        if (status == DISCOVER_OK) status = v;
        s.n_scored = (int64_t)ctr[2];
        s.pool_size += r[4];
        s.n_selected += r[0];
        s.n_merged += r[2];
        s.max_lowprec_err = fmax(s.max_lowprec_err, __longlong_as_double((long long)*c.maxerr));
    }
    s.status = status;
    out[b] = s;
}

struct FixRegrow {
    int64_t need;
};

static void generate_screen_once(discover_ctx* ctx, const discover_problem* probs, int nb,
                                 const discover_screen_params& prm, const std::vector<ScreenOut>& outs,
                                 discover_screen_stats* out_stats, hipStream_t st,
                                 std::vector<ListCheck>* checks, const std::vector<FillSeg>* extra_fills,
                                 discover_screen_stats* dev_stats) {
    // without host synchronisation one selection round runs at the sizes
    // an earlier call settled on, and its outcome is judged on the device
    const bool devmode = ctx->capturing || ctx->nosync;
    std::vector<Problem> PS;
    std::vector<ListState> LS;
    std::vector<int> act;
    const std::string ck = call_key(probs, nb, prm);
    // the lists and the first selection round's arena are laid out before
    // the screen, so that round's counters and histograms are cleared by the
    // screen's own fill launch
    auto first_round = [&](std::vector<FillSeg>& fills) {
        if (extra_fills) fills.insert(fills.end(), extra_fills->begin(), extra_fills->end());
        for (int b = 0; b < nb; b++) {
            const Problem& P = PS[b];
            for (int t = 0; t < P.Tl; t++) {
                ListState L;
                L.b = b; L.t = t; L.n = P.n;
                L.K = 2 * (int64_t)prm.k + probs[b].n_exclude + 64;
                L.cap = 4 * L.K + 4096;
                L.fcap = 64 * L.cap;
                LS.push_back(L);
            }
        }
        auto mit = ctx->batches.find("sel" + ck);
        if (mit != ctx->batches.end()) {        // start from the sizes a previous call settled on
            const SelMemo& m = *std::static_pointer_cast<SelMemo>(mit->second);
            if (m.K.size() == LS.size())
                for (size_t l = 0; l < LS.size(); l++) { LS[l].K = m.K[l]; LS[l].cap = m.cap[l]; LS[l].fcap = m.fcap[l]; }
        }
        act.resize(LS.size());
        for (size_t l = 0; l < LS.size(); l++) act[l] = (int)l;
        std::vector<std::vector<size_t>> o;
        char* base = sel_layout(ctx, prm.k, LS, act, o);
        for (size_t q = 0; q < act.size(); q++) {
            fills.push_back(fill_seg(base + o[q][SEL_MISC], 64, 0u));   // pool count, maximum error, st, sel, clusters, prefix
            fills.push_back(fill_seg(base + o[q][SEL_HIST], 8192 * 4, 0u));
            fills.push_back(fill_seg(base + o[q].back(), RK_NB * 4 + 64, 0u));   // rank buckets
        }
    };
    screen_all(ctx, probs, nb, prm, PS, st, first_round);
    std::vector<discover_screen_stats> stats(nb);
    std::vector<double> margin(nb);
    for (int b = 0; b < nb; b++) {
        const Problem& P = PS[b];
        discover_screen_stats& s = stats[b];
        s = discover_screen_stats{};
        s.n_raw = P.plan->sp.n_raw();
        s.n_unit_valid = P.plan->sp.n_unit_valid;
        s.tile_j = P.tile_j;
        margin[b] = 4.0 * P.n * EPS64 * KAPPA_MAX;
        if (prm.precision != DISCOVER_FP64) {
            s.guard_band = lowprec_margin(prm.precision, P.n);
            // rung 3 in BF16 carries its FP32 moments' error as well
            if (prm.precision == DISCOVER_BF16_GUARD && P.plan->sp.stream3)
                s.guard_band += 1.5 * r3_moment_err(P.n);
            margin[b] = std::max(margin[b], s.guard_band);
        }
    }
    std::vector<SelArgs> sa;
    std::vector<ListCheck> lc;
    bool checked_bad = false;
    bool prefilled = true;
    int rounds = 0;
    while (!act.empty()) {
        select_round(ctx, probs, prm, PS, LS, act, margin, outs, st, sa, prefilled);
        prefilled = false;
        rounds++;
        if (devmode) {                          // results are checked on the device
            for (size_t q = 0; q < act.size(); q++) {
                const ListState& L = LS[act[q]];
                lc.push_back(ListCheck{sa[q].res, L.cap, L.fcap, L.K, PS[L.b].N, PS[L.b].ctr, prm.dedup,
                                       PS[L.b].fix_cap, sa[q].maxerr, L.b});
            }
            if (checks) checks->insert(checks->end(), lc.begin(), lc.end());
            break;
        }
        // one synchronisation per round: outcome of every active list
        const int nl = (int)act.size();
        std::vector<int64_t> h_res(8 * (size_t)nl);
        std::vector<unsigned long long> h_err(nl);
        for (int q = 0; q < nl; q++) {
            DSC_HIP(hipMemcpyAsync(&h_res[8 * q], sa[q].res, 64, hipMemcpyDeviceToHost, st));
            DSC_HIP(hipMemcpyAsync(&h_err[q], sa[q].maxerr, 8, hipMemcpyDeviceToHost, st));
        }
        std::vector<unsigned long long> h_ctr(4 * (size_t)nb);
        if (!checked_bad)
            for (int b = 0; b < nb; b++)
                DSC_HIP(hipMemcpyAsync(&h_ctr[4 * b], PS[b].ctr, 32, hipMemcpyDeviceToHost, st));
        DSC_HIP(hipStreamSynchronize(st));
        if (!checked_bad) {
            int64_t need = 0;
            for (int b = 0; b < nb; b++) {
                if ((int)(h_ctr[4 * b] & 0xFFFFFFFFull))
                    DSC_FAIL(DISCOVER_E_NUMERIC, "problem %d: a target column is constant or not finite", b);
                stats[b].n_scored = (int64_t)h_ctr[4 * b + 2];
                const int64_t nf = (int64_t)std::max(h_ctr[4 * b + 1], h_ctr[4 * b + 3]);
                if (nf > PS[b].fix_cap) need = std::max(need, nf);
            }
            // a fix-up list overflowed: candidates past its end were neither
            // scored nor rescored, so the whole screen runs again with room
            // for every one of them
            if (need) throw FixRegrow{need};
            checked_bad = true;
        }
        std::vector<int> next;
        for (int q = 0; q < nl; q++) {
            ListState& L = LS[act[q]];
            discover_screen_stats& s = stats[L.b];
            const int64_t* r = &h_res[8 * q];
            const int64_t N = PS[L.b].N;
            if (r[4] > L.cap) {                       // pool overflow: enlarge and redo
                L.cap = r[4] + 1024;
                L.fcap = std::max(L.fcap, 64 * L.cap);
                s.pool_rounds += 1;
                next.push_back(act[q]);
                continue;
            }
            if (prm.dedup && r[3] > L.fcap) {         // pair-flag overflow
                L.fcap = r[3] + 1024;
                s.pool_rounds += 1;
                next.push_back(act[q]);
                continue;
            }
            s.pool_size += r[4];
            double e;
            std::memcpy(&e, &h_err[q], 8);
            s.max_lowprec_err = std::max(s.max_lowprec_err, e);
            if (r[1] || L.K >= N) {
                s.n_selected += r[0];
                s.n_merged += r[2];
                L.done = true;
                continue;
            }
            s.pool_rounds += 1;
            L.K = std::min<int64_t>(N, L.K * 4);
            L.cap = 4 * L.K + 4096;
            L.fcap = std::max(L.fcap, 64 * L.cap);
            next.push_back(act[q]);
        }
        act.swap(next);
    }
    const auto gen0 = ctx->generation;
    if (!devmode) {
        // size the result arena for a one-round run of every list at the final
        // capacities, as a captured run does
        select_reserve(ctx, prm, LS);
        auto m = std::make_shared<SelMemo>();
        for (const ListState& L : LS) { m->K.push_back(L.K); m->cap.push_back(L.cap); m->fcap.push_back(L.fcap); }
        if (ctx->batches.size() >= 256) ctx->batches.clear();
        ctx->batches["sel" + ck] = m;
    }
    if (outs[0].vals) {
        std::vector<ValArgs> va;
        int64_t mmax = 0;
        // after one selection round every list's stored pool values are still
        // in place (a later round lays the arena out anew, a regrown arena
        // is a new allocation)
        const int64_t* vrow = rounds == 1 && ctx->generation == gen0 ? ctx->buf<int64_t>("scr_vrow" + ctx->tag, 0) : nullptr;
        int64_t voff = 0;
        for (int b = 0; b < nb; b++) {
            const Problem& P = PS[b];
            ValArgs a{};
            a.ids = outs[b].ids; a.m = (int64_t)P.Tl * prm.k; a.ev = P.ev(); a.o = P.ops();
            a.n = P.n; a.out = outs[b].vals; a.ldv = outs[b].ldv;
            a.vrow = vrow ? vrow + voff : nullptr;
            voff += a.m;
            va.push_back(a);
            mmax = std::max(mmax, a.m);
        }
        KTimer kt(ctx, st, "values");
        k_values<<<dim3((unsigned)cdiv(mmax, 4), nb), 256, 0, st>>>(ct(ctx->upload("scr_values", va, st)));
        check_launch("k_values");
    }
    if (devmode) {
        if (dev_stats) {
            // lists are laid out problem by problem
            std::vector<StatBase> sb(nb);
            for (int b = 0; b < nb; b++) { sb[b].s = stats[b]; sb[b].l0 = -1; sb[b].nl = 0; }
            for (size_t l = 0; l < lc.size(); l++) {
                StatBase& x = sb[lc[l].b];
                if (x.l0 < 0) x.l0 = (int32_t)l;
                x.nl++;
            }
            for (StatBase& x : sb) x.l0 = std::max(x.l0, 0);
            k_screen_stats<<<(unsigned)cdiv(nb, 256), 256, 0, st>>>(
                ct(ctx->upload("scr_stats_base", sb, st)), ct(ctx->upload("scr_stats_lists", lc, st)), nb,
                dev_stats);
            check_launch("k_screen_stats");
        }
        return;
    }
    DSC_HIP(hipStreamSynchronize(st));
    ctx->resolve_timing();
    if (out_stats)
        for (int b = 0; b < nb; b++) out_stats[b] = stats[b];
}

void generate_screen(discover_ctx* ctx, const discover_problem* probs, int nb,
                     const discover_screen_params& prm, const std::vector<ScreenOut>& outs,
                     discover_screen_stats* out_stats, hipStream_t st, std::vector<ListCheck>* checks,
                     const std::vector<FillSeg>* extra_fills, discover_screen_stats* dev_stats) {
    for (;;) {
        try {
            generate_screen_once(ctx, probs, nb, prm, outs, out_stats, st, checks, extra_fills, dev_stats);
            return;
        } catch (const FixRegrow& r) {
            if (r.need >= ((int64_t)1 << 40))
                DSC_FAIL(DISCOVER_E_CAPACITY, "fix-up list of %lld entries", (long long)r.need);
            ctx->fix_cap_min = r.need + r.need / 4 + 4096;
        }
    }
}

}  // namespace dsc

extern "C" discover_status discover_generate_screen(discover_ctx* ctx, const discover_problem* probs,
                                                    int32_t n_problems, const discover_screen_params* prm,
                                                    int64_t* out_ids, double* out_scores,
                                                    double* out_values, int64_t ldv,
                                                    discover_screen_stats* out_stats, void* stream) {
    using namespace dsc;
    return guarded([&] {
        DSC_REQUIRE(ctx, "ctx is NULL");
        validate(probs, n_problems, prm, out_ids, out_scores, out_values, ldv);
        DSC_HIP(hipSetDevice(ctx->device));
        const hipStream_t st = (hipStream_t)stream;
        const bool cap = stream_capturing(st);
        const bool dev = device_memory(out_stats);
        DSC_REQUIRE(!cap || dev, "a call captured into a graph reports its outcome in device memory: "
                                 "out_stats must be a device pointer");
        std::vector<ScreenOut> outs(n_problems);
        int64_t row = 0;
        for (int b = 0; b < n_problems; b++) {
            outs[b] = ScreenOut{out_ids + row * prm->k, out_scores + row * prm->k,
                                out_values ? out_values + row * prm->k * ldv : nullptr, ldv};
            row += prm->score_mode == DISCOVER_SCORE_MAX ? 1 : probs[b].T;
        }
        if (dev && !screen_sizes_known(ctx, probs, n_problems, *prm)) {
            if (cap)
                DSC_FAIL(DISCOVER_E_CAPACITY, "no call of this shape has run outside capture: run it "
                                              "once (or discover_reserve) before capturing");
            // the first call of a shape settles its sizes, waiting for the stream
            std::vector<discover_screen_stats> hs(n_problems);
            generate_screen(ctx, probs, n_problems, *prm, outs, hs.data(), st);
            DSC_HIP(hipMemcpyAsync(out_stats, hs.data(), hs.size() * sizeof(discover_screen_stats),
                                   hipMemcpyHostToDevice, st));
            DSC_HIP(hipStreamSynchronize(st));
            return;
        }
        CallMode mode(ctx, cap, dev);
        generate_screen(ctx, probs, n_problems, *prm, outs, dev ? nullptr : out_stats, st, nullptr, nullptr,
                        dev ? out_stats : nullptr);
    });
}
