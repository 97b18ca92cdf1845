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
//   scores    [T'][N]       one FP64 slot per candidate ID:
//                             +s     score with |error| <= margin
//                             -u     error may be larger; u bounds s above
//                             NaN    invalid / unit-illegal / not computed
//
// The streamed rung is never materialised: each wave evaluates
// op(f_i, f_j) for its tile on the fly and keeps only moments in registers.
#include "dsc_select.h"
#include "dsc_space.h"

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
__global__ __launch_bounds__(256) void k_targets(int n, int T, const double* __restrict__ Y,
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
__global__ void k_mat_values(int n, int ldn, int c0, int c1, const double* __restrict__ X,
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
__global__ __launch_bounds__(256) void k_mat_stats(int n, int ldn, int c0, int c1,
                                                   const int8_t* __restrict__ mop,
                                                   const int32_t* __restrict__ ca,
                                                   const int32_t* __restrict__ cb,
                                                   double* __restrict__ Vf, double* __restrict__ Rf,
                                                   double* __restrict__ Cf, double* __restrict__ mu,
                                                   double* __restrict__ mur, double* __restrict__ msq,
                                                   uint8_t* __restrict__ valid) {
    const int c = c0 + blockIdx.x * 4 + (threadIdx.x >> 6);
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

// Feature-major [M][ldn] -> sample-major [n][ldm] (padding left as is).
__global__ void k_transpose(int n, int M, int ldn, int ldm, const double* __restrict__ src,
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

// Exact two-pass Pearson of one candidate against T centered targets by one
// wave.  Returns false when the candidate is not finite or is constant.
template <int TMAX>
__device__ bool wave_exact_r(const Cand& c, const Ops& o, int n, int T,
                             const double* __restrict__ Yc, const double* __restrict__ syy,
                             double* r, double* mean_out = nullptr, double* msq_out = nullptr) {
    const int lane = threadIdx.x & 63;
    double s = 0.0;
    int bad = 0;
    const bool addsub = (c.kind == 2 || c.kind == 3) && (c.op == OP_ADD || c.op == OP_SUB);
    double ff = 0.0, ab = 0.0;
    for (int i = lane; i < n; i += 64) {
        const double f = cand_value(c, o, i);
        bad |= !isfinite(f);
        s += f;
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
    return true;
}

// Exact scores of an explicit candidate list (operand features and unary
// candidates of the streamed rung), written into the score slots.
struct ListItem {
    int64_t id;
    int32_t kind, op, ca, cb;
};

__global__ __launch_bounds__(256) void k_score_list(const ListItem* __restrict__ items, int64_t m,
                                                    Ops o, const uint8_t* __restrict__ valid,
                                                    int n, int T, int mode,
                                                    const double* __restrict__ Yc,
                                                    const double* __restrict__ syy, int64_t N,
                                                    double* __restrict__ scores,
                                                    unsigned long long* __restrict__ nscored,
                                                    uint8_t* __restrict__ r2v, double* __restrict__ r2m,
                                                    double* __restrict__ r2q, int64_t off2, int64_t off3) {
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= m) return;
    const ListItem it = items[w];
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
        atomicAdd(nscored, 1ull);
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
    const int2* tiles;        // (jc0, ic0) per wave (dense) or (jc, list offset)
    const int32_t* ilist;     // explicit partner lists (list mode) or NULL
    const int32_t* icount;    // per-wave partner count (list mode)
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

// One block = one tile; its 4 waves take consecutive quarters of the samples
// and their partial moments are summed in LDS in a fixed order (wave 0 +
// wave 1 + wave 2 + wave 3), so results do not depend on scheduling.
constexpr int PAIR_SPLIT = 4;

template <int OPS, int J, int TP, bool LIST>
__global__ __launch_bounds__(256) void k_screen_pairs(PairArgs g) {
    constexpr int NOP = ((OPS >> 0) & 1) + ((OPS >> 1) & 1) + ((OPS >> 2) & 1) +
                        ((OPS >> 3) & 1) + ((OPS >> 4) & 1);
    constexpr int NV = J * NOP * (2 + TP);       // accumulators per lane
    constexpr int SL = 8;                        // accumulators combined per LDS round
    __shared__ double red[PAIR_SPLIT - 1][SL][64];
    const int64_t w = blockIdx.x;
    if (w >= g.n_tiles) return;
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int2 tile = g.tiles[w];
    const int jc0 = tile.x;
    int i;
    bool lane_ok;
    if (LIST) {
        lane_ok = lane < g.icount[w];
        i = g.ilist[tile.y + (lane_ok ? lane : 0)];
    } else {
        i = tile.y + lane;
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
    // combine the partial moments of the 4 waves into wave 0
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
                if (v0 + v < NV)
                    acc[v0 + v] = ((acc[v0 + v] + red[0][v][lane]) + red[1][v][lane]) + red[2][v][lane];
        }
        __syncthreads();
    }
    if (wave != 0) return;

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
                const unsigned long long slot = atomicAdd(g.fix_cnt, 1ull);
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

// ---------------------------------------------- operator-limited rung 3
// Candidates op3(f_i, f_j2): i in the materialised partner pool (uniform
// across the wave), j2 a rung-2 feature regenerated on the fly in every lane
// from two rung-1 operands (never stored).  The wave's 64 rung-2 features
// come from one rung-2 tile: (op2, l, 64 consecutive k) for binary op2,
// (op2, 64 consecutive l) for unary op2, or a same-unit partner list.
// Shifts: add/sub use centered operands, mul mu_i mu_j2, div mu_i / mu_j2,
// rdiv mu_j2 / mu_i-type estimates (mu_j2 from the rung-2 screening pass).
struct R3Args {
    const int4* tiles;        // (op2, l or l0, k0 or list offset, -1 dense | count | -2 unary)
    const int32_t* klist;
    int64_t n_tiles;
    int n, ldm, ldn, Mc, c1_lo, c1_hi, pe, B;
    const double *Vs, *Rs, *Cs, *Vf, *Rf, *Cf, *mu, *mur;
    const uint8_t* valid;
    const int64_t* mat_raw;
    const int32_t* mat_unit;
    const uint8_t* r2v;
    const double* r2m;
    const double* r2q;
    const double* msq;
    const double* Yn;
    const double* ysum;
    int T, mode;
    uint32_t opmask;          // rung-3 binary operators (bits 0..4 = add..rdiv)
    SpaceDev sd;
    int64_t N;
    double* scores;
    unsigned long long* nscored;
    int64_t* fix_ids;
    unsigned long long* fix_cnt;
    int64_t fix_cap;
};

__device__ __forceinline__ bool dev_unit_rule(int op, int B, const int32_t* ua, const int32_t* ub,
                                              int32_t* out) {
    switch (op) {
    case OP_EXP: case OP_LOG:
        for (int k = 0; k < B; k++) if (ua[k]) return false;
        for (int k = 0; k < B; k++) out[k] = 0;
        return true;
    case OP_SQRT:
        for (int k = 0; k < B; k++) if (ua[k] & 1) return false;
        for (int k = 0; k < B; k++) out[k] = ua[k] / 2;
        return true;
    case OP_SQ: for (int k = 0; k < B; k++) out[k] = 2 * ua[k]; return true;
    case OP_INV: for (int k = 0; k < B; k++) out[k] = -ua[k]; return true;
    case OP_ADD: case OP_SUB:
        for (int k = 0; k < B; k++) if (ua[k] != ub[k]) return false;
        for (int k = 0; k < B; k++) out[k] = ua[k];
        return true;
    case OP_MUL: for (int k = 0; k < B; k++) out[k] = ua[k] + ub[k]; return true;
    case OP_DIV: for (int k = 0; k < B; k++) out[k] = ua[k] - ub[k]; return true;
    default: for (int k = 0; k < B; k++) out[k] = ub[k] - ua[k]; return true;
    }
}

template <int OPS, int IC, int TP>
__global__ __launch_bounds__(256) void k_screen_r3(R3Args g) {
    constexpr int NOP = ((OPS >> 0) & 1) + ((OPS >> 1) & 1) + ((OPS >> 2) & 1) +
                        ((OPS >> 3) & 1) + ((OPS >> 4) & 1);
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= g.n_tiles) return;
    const int lane = threadIdx.x & 63;
    const int4 tile = g.tiles[w];
    const int op2 = tile.x;
    // this lane's rung-2 feature: operands (k, l) compact, raw id j2
    int k = -1, l = -1;
    bool lok;
    if (tile.w == -2) {                                   // unary op2 over 64 consecutive l
        l = tile.y + lane;
        lok = l < g.c1_hi;
    } else if (tile.w == -1) {                            // binary op2, k = k0 + lane < l
        l = tile.y;
        k = tile.z + lane;
        lok = k < l;
    } else {                                              // binary op2, explicit partner list
        l = tile.y;
        lok = lane < tile.w;
        k = g.klist[tile.z + (lok ? lane : 0)];
    }
    const int lc = lok ? l : g.c1_lo;
    const int kc = (k >= 0 && lok) ? k : 0;
    int64_t j2 = 0;
    if (lok) j2 = tile.w == -2 ? unary_id(g.sd, 2, op2, g.mat_raw[lc])
                              : pair_id(g.sd, 2, op2, g.mat_raw[kc], g.mat_raw[lc]);
    const int64_t o2 = j2 - g.sd.off[2];
    const bool ok2 = lok && g.r2v[o2];
    const double mu2 = ok2 ? g.r2m[o2] : 1.0;
    const double q2 = ok2 ? g.r2q[o2] : 1.0;
    int32_t u2[DISCOVER_MAX_UNITS];
    if (g.B > 0) {
        bool leg = dev_unit_rule(op2, g.B, g.mat_unit + (int64_t)(tile.w == -2 ? lc : kc) * g.B,
                                 g.mat_unit + (int64_t)lc * g.B, u2);
        (void)leg;                                        // ok2 already implies legality
    }
    const bool want_rcp = (OPS & 8) != 0;
    const int nn_i = g.n;
    const double nn = (double)g.n;
    unsigned cnt = 0;
    for (int i0 = 0; i0 < g.pe; i0 += IC) {
        // per-lane legality of add/sub partners (unit exponents must agree)
        bool addok[IC];
        bool any_add = false;
#pragma unroll
        for (int ii = 0; ii < IC; ii++) {
            const int i = min(i0 + ii, g.pe - 1);
            bool eq = true;
            for (int b = 0; b < g.B; b++) eq = eq && (g.mat_unit[(int64_t)i * g.B + b] == u2[b]);
            addok[ii] = ok2 && (i0 + ii < g.pe) && eq;
            any_add |= addok[ii];
        }
        const bool wave_add = (OPS & 3) && __any(any_add);
        double sh[IC][NOP];
#pragma unroll
        for (int ii = 0; ii < IC; ii++) {
            const int i = min(i0 + ii, g.pe - 1);
            const double mi = g.mu[i], mri = g.mur[i];
            int q = 0;
            if (OPS & 1) sh[ii][q++] = 0.0;
            if (OPS & 2) sh[ii][q++] = 0.0;
            if (OPS & 4) sh[ii][q++] = mi * mu2;
            if (OPS & 8) sh[ii][q++] = mu2 != 0.0 ? mi / mu2 : 0.0;
            if (OPS & 16) sh[ii][q++] = mu2 * mri;
        }
        double acc[IC][NOP][2 + TP];
#pragma unroll
        for (int ii = 0; ii < IC; ii++)
#pragma unroll
            for (int q = 0; q < NOP; q++)
#pragma unroll
                for (int v = 0; v < 2 + TP; v++) acc[ii][q][v] = 0.0;
        for (int s = 0; s < nn_i; s++) {
            double f2;
            if (tile.w == -2) {
                const int64_t so = (int64_t)s * g.ldm + lc;
                const double a = g.Vs[so];
                f2 = op2 == OP_INV ? g.Rs[so] : op2 == OP_SQ ? a * a : apply_op(op2, a, 0.0);
            } else {
                const double a = g.Vs[(int64_t)s * g.ldm + kc];
                const double b = g.Vf[(int64_t)lc * g.ldn + s];
                switch (op2) {
                case OP_ADD: f2 = a + b; break;
                case OP_SUB: f2 = a - b; break;
                case OP_MUL: f2 = a * b; break;
                case OP_DIV: f2 = a * g.Rf[(int64_t)lc * g.ldn + s]; break;
                default: f2 = b * g.Rs[(int64_t)s * g.ldm + kc]; break;
                }
            }
            const double f2c = f2 - mu2;
            double rf2 = 0.0;
            if (want_rcp) {
                double r = __builtin_amdgcn_rcp(f2);
                r = fma(r, fma(-f2, r, 1.0), r);
                rf2 = fma(r, fma(-f2, r, 1.0), r);
            }
            double y[TP];
#pragma unroll
            for (int t = 0; t < TP; t++) y[t] = g.Yn[(int64_t)t * g.ldn + s];
#pragma unroll
            for (int ii = 0; ii < IC; ii++) {
                const int i = min(i0 + ii, g.pe - 1);
                const double x = g.Vf[(int64_t)i * g.ldn + s];
                const double xc = (OPS & 3) ? g.Cf[(int64_t)i * g.ldn + s] : 0.0;
                const double rx = (OPS & 16) ? g.Rf[(int64_t)i * g.ldn + s] : 0.0;
                double f[NOP];
                int q = 0;
                if (OPS & 1) { f[q] = xc + f2c; q++; }
                if (OPS & 2) { f[q] = xc - f2c; q++; }
                if (OPS & 4) { f[q] = fma(x, f2, -sh[ii][q]); q++; }
                if (OPS & 8) { f[q] = fma(x, rf2, -sh[ii][q]); q++; }
                if (OPS & 16) { f[q] = fma(f2, rx, -sh[ii][q]); q++; }
#pragma unroll
                for (int qq = 0; qq < NOP; qq++) {
                    if (qq < ((OPS & 1) + ((OPS >> 1) & 1)) && !wave_add) continue;   // uniform
                    acc[ii][qq][0] += f[qq];
                    acc[ii][qq][1] = fma(f[qq], f[qq], acc[ii][qq][1]);
#pragma unroll
                    for (int t = 0; t < TP; t++) acc[ii][qq][2 + t] = fma(f[qq], y[t], acc[ii][qq][2 + t]);
                }
            }
        }
        // finalise the IC x NOP candidates of this chunk
#pragma unroll
        for (int ii = 0; ii < IC; ii++) {
            const int i = i0 + ii;
            if (i >= g.pe) continue;
            int q = 0;
#pragma unroll
            for (int o = 0; o < 5; o++) {
                if (!((OPS >> o) & 1)) continue;
                const int qq = q++;
                // score slots start as NaN: unit-illegal or invalid candidates are
                // simply not written
                if (!((g.opmask >> o) & 1) || !ok2 || !g.valid[i]) continue;
                if (o < 2 && !addok[ii]) continue;
                const int64_t id = pair_id(g.sd, 3, OP_ADD + o, g.mat_raw[i], j2);
                const double nanv = __longlong_as_double(-1LL);
                const double S1v = acc[ii][qq][0], S2v = acc[ii][qq][1];
                const double m1 = S1v / nn, varn = S2v - S1v * m1;
                if (!(S2v < INFINITY) || !(fabs(S1v) < INFINITY)) continue;
                double kappa = varn > 0.0 ? S2v / varn : INFINITY;
                if (o < 2) {                                      // possible cancellation
                    const double c0 = o == 0 ? g.mu[i] + mu2 : g.mu[i] - mu2;
                    const double ff = S2v + 2.0 * c0 * S1v + nn * c0 * c0;
                    if (ff <= 1e-12 * nn * (g.msq[i] + q2)) kappa = INFINITY;
                }
                if (!(kappa <= KAPPA_MAX)) {
                    const unsigned long long slot = atomicAdd(g.fix_cnt, 1ull);
                    if ((int64_t)slot < g.fix_cap) {
                        g.fix_ids[slot] = id;
                        for (int t = 0; t < (g.mode ? 1 : g.T); t++) g.scores[(int64_t)t * g.N + id] = nanv;
                        continue;
                    }
                }
                double shift = sh[ii][qq];
                if (o == 0) shift = g.mu[i] + mu2;
                if (o == 1) shift = g.mu[i] - mu2;
                const double mean = shift + m1;
                const bool nonconst = varn / nn > TAU_CONST * TAU_CONST * (varn / nn + mean * mean);
                if (kappa <= KAPPA_MAX && !nonconst) {
                    for (int t = 0; t < (g.mode ? 1 : g.T); t++) g.scores[(int64_t)t * g.N + id] = nanv;
                    continue;
                }
                const double isd = 1.0 / sqrt(varn);
                double out[TP], best = 0.0;
#pragma unroll
                for (int t = 0; t < TP; t++) {
                    out[t] = fabs((acc[ii][qq][2 + t] - S1v * g.ysum[t] / nn) * isd);
                    if (t < g.T) best = fmax(best, out[t]);
                }
                const double err = 4.0 * nn * EPS64 * kappa;
                const bool precise = kappa <= KAPPA_MAX;
                cnt++;
                if (g.mode == DISCOVER_SCORE_MAX) {
                    g.scores[id] = precise ? best : -(best + err);
                } else {
#pragma unroll
                    for (int t = 0; t < TP; t++)
                        if (t < g.T) g.scores[(int64_t)t * g.N + id] = precise ? out[t] : -(out[t] + err);
                }
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor((int)cnt, o, 64);
    if (lane == 0 && cnt) atomicAdd(g.nscored, (unsigned long long)cnt);
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
constexpr int LP_IB = 1;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8_t;
typedef __attribute__((ext_vector_type(8))) _Float16 f16x8_t;
typedef __attribute__((ext_vector_type(4))) float f32x4_t;

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

template <int OPS, bool FP16>
__global__ __launch_bounds__(256) void k_screen_lp(PairArgs g, const void* __restrict__ Ylp_, int ldl) {
    constexpr int NOP = ((OPS >> 0) & 1) + ((OPS >> 1) & 1) + ((OPS >> 2) & 1) +
                        ((OPS >> 3) & 1) + ((OPS >> 4) & 1);
    constexpr int IB = LP_IB;                              // LP_IB x 16 operand features i per wave
    constexpr int G = IB * NOP;
    typedef typename LpVec<FP16>::T VT;
    typedef typename std::conditional<FP16, _Float16, __bf16>::type ET;
    const ET* __restrict__ Ylp = (const ET*)Ylp_;
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= g.n_tiles) return;
    const int lane = threadIdx.x & 63;
    const int col = lane & 15, kb = lane >> 4;
    const int2 tile = g.tiles[w];
    const int jc = tile.x;                                 // one j per tile
    const double mub = g.mu[jc], murb = g.mur[jc];
    int ic[IB];
    bool iok[IB];
    double sh[IB][NOP];
#pragma unroll
    for (int b = 0; b < IB; b++) {
        const int i = tile.y + 16 * b + col;
        iok[b] = i < g.i_end && i < jc;
        ic[b] = i < g.Mc ? i : 0;
        const double mua = g.mu[ic[b]], mura = g.mur[ic[b]];
        int k = 0;
        if (OPS & 1) sh[b][k++] = 0.0;
        if (OPS & 2) sh[b][k++] = 0.0;
        if (OPS & 4) sh[b][k++] = mua * mub;
        if (OPS & 8) sh[b][k++] = mua * murb;
        if (OPS & 16) sh[b][k++] = mura * mub;
    }
    auto values = [&](int s, double f[IB][NOP]) {
        const double b_ = g.Vf[(int64_t)jc * g.ldn + s];
        const double rb = g.Rf[(int64_t)jc * g.ldn + s];
        const double bc = g.Cf[(int64_t)jc * g.ldn + s];
#pragma unroll
        for (int b = 0; b < IB; b++) {
            const int64_t so = (int64_t)s * g.ldm + ic[b];
            const double a = g.Vs[so], ra = g.Rs[so], ac = g.Cs[so];
            int k = 0;
            if (OPS & 1) { f[b][k] = ac + bc; k++; }
            if (OPS & 2) { f[b][k] = ac - bc; k++; }
            if (OPS & 4) { f[b][k] = fma(a, b_, -sh[b][k]); k++; }
            if (OPS & 8) { f[b][k] = fma(a, rb, -sh[b][k]); k++; }
            if (OPS & 16) { f[b][k] = fma(ra, b_, -sh[b][k]); k++; }
        }
    };
    // pass 1: shifted moments over this lane's samples, then across the 4
    // lanes that share a candidate
    double s1[G], s2[G];
#pragma unroll
    for (int q = 0; q < G; q++) { s1[q] = 0.0; s2[q] = 0.0; }
    const int nch = (g.n + 31) / 32;
    for (int c = 0; c < nch; c++) {
        for (int e = 0; e < 8; e++) {
            const int s = 32 * c + 8 * kb + e;
            if (s >= g.n) break;
            double f[IB][NOP];
            values(s, f);
#pragma unroll
            for (int b = 0; b < IB; b++)
#pragma unroll
                for (int k = 0; k < NOP; k++) {
                    s1[b * NOP + k] += f[b][k];
                    s2[b * NOP + k] = fma(f[b][k], f[b][k], s2[b * NOP + k]);
                }
        }
    }
#pragma unroll
    for (int q = 0; q < G; q++) {
        // fixed order: (kb0 + kb1) + (kb2 + kb3) in every lane
        const double a1 = s1[q] + __shfl_xor(s1[q], 16, 64);
        s1[q] = a1 + __shfl_xor(a1, 32, 64);
        const double a2 = s2[q] + __shfl_xor(s2[q], 16, 64);
        s2[q] = a2 + __shfl_xor(a2, 32, 64);
    }
    const double nn = (double)g.n;
    double isd[G], cz[G];
    unsigned okmask = 0, fixmask = 0;
#pragma unroll
    for (int b = 0; b < IB; b++)
#pragma unroll
        for (int k = 0; k < NOP; k++) {
            const int q = b * NOP + k;
            const double m1 = s1[q] / nn, varn = s2[q] - s1[q] * m1;
            const bool fin = (s2[q] < INFINITY) && (fabs(s1[q]) < INFINITY);
            double kappa = varn > 0.0 ? s2[q] / varn : INFINITY;
            if ((OPS & 3) && k < ((OPS & 1) + ((OPS >> 1) & 1))) {   // add / sub
                const bool isadd = (OPS & 1) && k == 0;
                const double c0 = isadd ? g.mu[ic[b]] + mub : g.mu[ic[b]] - mub;
                const double ff = s2[q] + 2.0 * c0 * s1[q] + nn * c0 * c0;
                if (ff <= 1e-12 * nn * (g.msq[ic[b]] + g.msq[jc])) kappa = INFINITY;
            }
            bool ok = iok[b] && g.valid[ic[b]] && g.valid[jc] && fin;
            if (ok && !(kappa <= KAPPA_MAX)) { fixmask |= 1u << q; ok = false; }
            isd[q] = ok ? sqrt(nn / varn) : 0.0;           // 1 / population sd
            cz[q] = m1 * isd[q];
            if (ok) okmask |= 1u << q;
        }
    // pass 2: low-precision products on the matrix cores
    f32x4_t acc[G];
#pragma unroll
    for (int q = 0; q < G; q++) acc[q] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    for (int c = 0; c < nch; c++) {
        const VT ya = *(const VT*)(Ylp + (int64_t)col * ldl + 32 * c + 8 * kb);
        VT bv[G];
#pragma unroll
        for (int e = 0; e < 8; e++) {
            const int s = 32 * c + 8 * kb + e;
            double f[IB][NOP];
            if (s < g.n) values(s, f);
#pragma unroll
            for (int q = 0; q < G; q++) {
                const double z = s < g.n ? fma(f[q / NOP][q % NOP], isd[q], -cz[q]) : 0.0;
                bv[q][e] = LpVec<FP16>::cvt((float)z);
            }
        }
#pragma unroll
        for (int q = 0; q < G; q++) acc[q] = LpVec<FP16>::mma(ya, bv[q], acc[q]);
    }
    // scores: lane holds r for targets 4kb..4kb+3 of candidate col
    unsigned cnt = 0;
#pragma unroll
    for (int b = 0; b < IB; b++) {
        const int i = tile.y + 16 * b + col;
        int k = 0;
#pragma unroll
        for (int o = 0; o < 5; o++) {
            if (!((OPS >> o) & 1)) continue;
            const int q = b * NOP + k++;
            double r[4];
            double mx = 0.0;
#pragma unroll
            for (int e = 0; e < 4; e++) {
                r[e] = fabs((double)acc[q][e]) / nn;
                if (4 * kb + e < g.T) mx = fmax(mx, r[e]);
            }
            mx = fmax(mx, __shfl_xor(mx, 16, 64));
            mx = fmax(mx, __shfl_xor(mx, 32, 64));
            if (!iok[b] || !((g.opmask >> o) & 1)) continue;
            const int64_t id = pair_id(g.sd, g.r, OP_ADD + o, g.mat_raw[ic[b]], g.mat_raw[jc]);
            const double nanv = __longlong_as_double(-1LL);
            const bool ok = (okmask >> q) & 1;
            if ((fixmask >> q) & 1) {
                if (kb == 0) {
                    const unsigned long long slot = atomicAdd(g.fix_cnt, 1ull);
                    if ((int64_t)slot < g.fix_cap) g.fix_ids[slot] = id;
                    if (g.mode == DISCOVER_SCORE_MAX) g.scores[id] = nanv;
                }
                if (g.mode != DISCOVER_SCORE_MAX)
                    for (int e = 0; e < 4; e++)
                        if (4 * kb + e < g.T) g.scores[(int64_t)(4 * kb + e) * g.N + id] = nanv;
                continue;
            }
            if (g.r2v && ok && kb == 0) {
                const double sh_ = (o == 0) ? g.mu[ic[b]] + mub : (o == 1) ? g.mu[ic[b]] - mub : sh[b][k - 1];
                const double mean_ = sh_ + s1[q] / nn;
                const double var_ = (s2[q] - s1[q] * s1[q] / nn) / nn;
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
    }
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor((int)cnt, o, 64);
    if (lane == 0 && cnt) atomicAdd(g.nscored, (unsigned long long)cnt);
}

// ------------------------------------------------------------ selection
// Pool = every candidate whose score may reach theta - margin.
__global__ __launch_bounds__(256) void k_compact(const double* __restrict__ sc, int64_t N,
                                                 const uint32_t* __restrict__ sel,
                                                 const int64_t* __restrict__ st, double margin,
                                                 int64_t cap, int64_t* __restrict__ pool,
                                                 unsigned long long* __restrict__ cnt) {
    const double th = select_threshold(sel, st);
    const double lo = st[1] ? 0.0 : th - 2.0 * margin;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256) {
        const double x = sc[i];
        const bool take = (x > 0.0 && x >= lo) || (x < 0.0 && -x >= lo);
        if (take) {
            const unsigned long long slot = atomicAdd(cnt, 1ull);
            if ((int64_t)slot < cap) pool[slot] = i;
        }
    }
}

// Exact FP64 rescore of the pool (one wave per entry); also flags entries
// whose ID is excluded.
template <int TMAX>
__global__ __launch_bounds__(256) void k_rescore(const int64_t* __restrict__ pool,
                                                 const unsigned long long* __restrict__ Pp, int64_t cap,
                                                 EvalCtx ev, Ops o, int n,
                                                 int T, int mode, int tlist,
                                                 const double* __restrict__ Yc,
                                                 const double* __restrict__ syy,
                                                 const int64_t* __restrict__ excl, int n_excl,
                                                 double* __restrict__ ps,
                                                 uint8_t* __restrict__ pex,
                                                 const double* __restrict__ sc_row,
                                                 unsigned long long* __restrict__ maxerr) {
    const int64_t P = min((int64_t)*Pp, cap);
    const int lane = threadIdx.x & 63;
    for (int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); w < P; w += (int64_t)gridDim.x * 4) {
    const int64_t id = pool[w];
    Cand c;
    bool ok = cand_of_id(ev, id, c);
    double r[TMAX];
    ok = ok && wave_exact_r<TMAX>(c, o, n, T, Yc, syy, r);
    int ex = 0;
    for (int e = lane; e < n_excl; e += 64) ex |= excl[e] == id;
    ex = __any(ex);
    if (lane == 0) {
        double s = -1.0;
        if (ok) {
            if (mode == DISCOVER_SCORE_MAX) {
                s = 0.0;
                for (int t = 0; t < T; t++) s = fmax(s, fabs(r[t]));
            } else {
                s = fabs(r[tlist]);
            }
            if (!(s > 0.0)) s = -1.0;
        }
        ps[w] = s;
        pex[w] = (uint8_t)ex;
        const double x = sc_row[id];                      // screening-pass score
        if (s > 0.0 && x > 0.0)
            atomicMax(maxerr, (unsigned long long)__double_as_longlong(fabs(x - s)));
    }
    }
}

// Exact two-pass score of the candidates whose shifted one-pass moments
// were ill-conditioned (one wave each), written back into the score slots.
template <int TMAX>
__global__ __launch_bounds__(256) void k_fixup(const int64_t* __restrict__ ids,
                                               const unsigned long long* __restrict__ cnt,
                                               int64_t cap, EvalCtx ev, Ops o, int n,
                                               int T, int mode, const double* __restrict__ Yc,
                                               const double* __restrict__ syy, int64_t N,
                                               double* __restrict__ scores,
                                               unsigned long long* __restrict__ nscored,
                                               uint8_t* __restrict__ r2v, double* __restrict__ r2m,
                                               double* __restrict__ r2q) {
    const int64_t m = min((int64_t)*cnt, cap);
    for (int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); w < m; w += (int64_t)gridDim.x * 4) {
        const int64_t id = ids[w];
        Cand c;
        bool ok = cand_of_id(ev, id, c);
        double r[TMAX], mean = 0.0, msq = 0.0;
        ok = ok && wave_exact_r<TMAX>(c, o, n, T, Yc, syy, r, &mean, &msq);
        if ((threadIdx.x & 63) != 0 || !ok) continue;
        atomicAdd(nscored, 1ull);
        if (r2v && id >= ev.sd.off[2] && id < ev.sd.off[3]) {     // rung-2 operand statistics
            r2v[id - ev.sd.off[2]] = 1;
            r2m[id - ev.sd.off[2]] = mean;
            r2q[id - ev.sd.off[2]] = msq;
        }
        if (mode == DISCOVER_SCORE_MAX) {
            double mx = 0.0;
            for (int t = 0; t < T; t++) mx = fmax(mx, fabs(r[t]));
            scores[id] = mx;
        } else {
            for (int t = 0; t < T; t++) scores[(int64_t)t * N + id] = fabs(r[t]);
        }
    }
}

// Rank sort of the pool by (-score, ID).
__global__ __launch_bounds__(256) void k_rank(const double* __restrict__ ps,
                                              const int64_t* __restrict__ pool,
                                              const unsigned long long* __restrict__ Pp, int64_t cap,
                                              int32_t* __restrict__ order) {
    const int64_t P = min((int64_t)*Pp, cap);
    if (P <= 4096) return;                      // handled by k_bitonic
    __shared__ double ts[1024];
    __shared__ int64_t ti[1024];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const double si = i < P ? ps[i] : 0.0;
    const int64_t ii = i < P ? pool[i] : 0;
    int64_t rank = 0;
    for (int64_t base = 0; base < P; base += 1024) {
        __syncthreads();
        for (int k = threadIdx.x; k < 1024; k += 256) {
            ts[k] = base + k < P ? ps[base + k] : -2.0;
            ti[k] = base + k < P ? pool[base + k] : INT64_MAX;
        }
        __syncthreads();
        const int lim = (int)min((int64_t)1024, P - base);
        for (int k = 0; k < lim; k++) rank += (ts[k] > si) || (ts[k] == si && ti[k] < ii);
    }
    if (i < P) order[rank] = (int32_t)i;
}

// Near-tie window of each sorted entry: lo[q] = first earlier position whose
// score is within TAU_NEAR (relative) of entry q, scanning backwards.
__global__ void k_window(const double* __restrict__ ps, const int32_t* __restrict__ order,
                         const unsigned long long* __restrict__ Pp, int64_t cap,
                         int32_t* __restrict__ lo, int32_t* __restrict__ cnt) {
    const int64_t P = min((int64_t)*Pp, cap);
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < P;
         q += (int64_t)gridDim.x * blockDim.x) {
    const double s = ps[order[q]];
    int64_t l = q;
    if (s > 0.0)
        while (l > 0 && q - l < 1024) {
            const double sp = ps[order[l - 1]];
            if (!(sp - s <= TAU_NEAR * sp)) break;
            l--;
        }
    lo[q] = (int32_t)l;
    cnt[q] = (int32_t)(q - l);
    }
}

// Exclusive prefix sum of cnt (single block).
__global__ __launch_bounds__(1024) void k_scan_offsets(const int32_t* __restrict__ cnt,
                                                       const unsigned long long* __restrict__ Pp,
                                                       int64_t cap, int64_t* __restrict__ off) {
    const int64_t P = min((int64_t)*Pp, cap);
    __shared__ int64_t part[1024];
    const int64_t per = (P + 1023) / 1024;
    const int64_t b = threadIdx.x * per, e = min(P, b + per);
    int64_t s = 0;
    for (int64_t q = b; q < e; q++) s += cnt[q];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t acc = 0;
        for (int k = 0; k < 1024; k++) {
            const int64_t v = part[k];
            part[k] = acc;
            acc += v;
        }
        off[P] = acc;
    }
    __syncthreads();
    int64_t acc = part[threadIdx.x];
    for (int64_t q = b; q < e; q++) {
        off[q] = acc;
        acc += cnt[q];
    }
}

// One wave per near-tie pair (earlier position lo[q]+k, later position q):
// duplicate flag = |corr| >= 1 - TAU_DUP.
__global__ __launch_bounds__(256) void k_pairs(const int64_t* __restrict__ pool,
                                               const int32_t* __restrict__ order,
                                               const int32_t* __restrict__ lo,
                                               const int64_t* __restrict__ off,
                                               const unsigned long long* __restrict__ Pp, int64_t cap,
                                               EvalCtx ev, Ops o, int n,
                                               uint8_t* __restrict__ flag, int64_t flag_cap) {
    const int64_t P = min((int64_t)*Pp, cap);
    const int64_t total = min(off[P], flag_cap);
    const int lane = threadIdx.x & 63;
    for (int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); w < total;
         w += (int64_t)gridDim.x * 4) {
    // find q with off[q] <= w < off[q+1]
    int64_t a = 0, b = P;
    while (b - a > 1) {
        const int64_t mid = (a + b) / 2;
        if (off[mid] <= w) a = mid; else b = mid;
    }
    const int64_t q = a;
    const int64_t pe = lo[q] + (w - off[q]);
    Cand cu, cv;
    const bool okp = cand_of_id(ev, pool[order[pe]], cu) && cand_of_id(ev, pool[order[q]], cv);
    if (!okp) {
        if (lane == 0) flag[w] = 0;
        continue;
    }
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
    if (lane == 0) flag[w] = fabs(uv) / sqrt(uu * vv) >= 1.0 - TAU_DUP;
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

__global__ __launch_bounds__(GRP_THREADS) void k_groups(
    const int64_t* __restrict__ pool, const double* __restrict__ ps, const uint8_t* __restrict__ pex,
    const int32_t* __restrict__ order, const int32_t* __restrict__ lo, const int64_t* __restrict__ off,
    const uint8_t* __restrict__ flag, const unsigned long long* __restrict__ Pp, int64_t cap,
    int64_t flag_cap, int k, int dedup, const uint32_t* __restrict__ sel,
    const int64_t* __restrict__ st, double margin, int32_t* __restrict__ parent,
    int32_t* __restrict__ blk, unsigned long long* __restrict__ repid, int32_t* __restrict__ reppos,
    int32_t* __restrict__ headpos, int64_t* __restrict__ out_ids, double* __restrict__ out_sc,
    int64_t* __restrict__ res) {
    __shared__ int64_t part[GRP_THREADS];
    __shared__ int changed, undecided;
    const int64_t P = min((int64_t)*Pp, cap);
    const int t = threadIdx.x;
    const bool all = st[1] != 0;
    const double th_scan = all ? -1.0 : select_threshold(sel, st) - margin;
    volatile int32_t* vpar = parent;
    // 1. initial decisions
    for (int64_t q = t; q < P; q += GRP_THREADS) {
        const double sq = ps[order[q]];
        int32_t v = (int32_t)q;
        if (!(sq > 0.0)) v = -3;                           // invalid after exact rescoring
        else if (dedup) {
            for (int64_t p2 = lo[q]; p2 < q; p2++)
                if (off[q] + (p2 - lo[q]) < flag_cap && flag[off[q] + (p2 - lo[q])]) { v = -2; break; }
        }
        parent[q] = v;
        blk[q] = 0;
        repid[q] = ~0ull;
        reppos[q] = -1;
    }
    __syncthreads();
    // 2. rounds
    for (;;) {
        if (t == 0) { changed = 0; undecided = 0; }
        __syncthreads();
        for (int64_t q = t; q < P; q += GRP_THREADS) {
            if (vpar[q] != -2) continue;
            int32_t dec = (int32_t)q;                       // head unless a flagged head comes first
            bool wait = false;
            for (int64_t p2 = lo[q]; p2 < q; p2++) {
                if (off[q] + (p2 - lo[q]) >= flag_cap || !flag[off[q] + (p2 - lo[q])]) continue;
                const int32_t sp2 = vpar[p2];
                if (sp2 == -2) { wait = true; break; }
                if (sp2 == (int32_t)p2) { dec = (int32_t)p2; break; }
            }
            if (wait) { atomicAdd(&undecided, 1); continue; }
            vpar[q] = dec;
            atomicAdd(&changed, 1);
        }
        __syncthreads();
        const int ch = changed, un = undecided;
        __syncthreads();
        if (un == 0 || ch == 0) break;
    }
    // 3. aggregate groups onto their heads
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
    __shared__ double tsc[GRP_THREADS];
    __shared__ int64_t tid_[GRP_THREADS];
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
                tsc[t] = ps[order[rq]];
                tid_[t] = pool[order[rq]];
            }
            __syncthreads();
            const int64_t lim = min((int64_t)GRP_THREADS, ns - j0);
            if (i < ns)
                for (int64_t j = 0; j < lim; j++)
                    rank += (tsc[j] > si) || (tsc[j] == si && tid_[j] < ii);
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
        bool complete = all;
        if (!all && nunb >= k) {
            const double lim = ps[order[headpos[k - 1]]];
            complete = (1.0 - TAU_NEAR) * lim >= th_scan;
        }
        res[0] = ns;
        res[1] = complete ? 1 : 0;
        res[2] = merged_tot;
        res[3] = P > 0 ? off[P] : 0;            // duplicate-check pairs (capacity check)
        res[4] = (int64_t)*Pp;                  // pool size (capacity check)
    }
}

// Sort of a pool of at most 4096 entries by (-score, ID): bitonic network
// in LDS, one block of 1024 threads.
constexpr int BITONIC_MAX = 4096;

__global__ __launch_bounds__(1024) void k_bitonic(const double* __restrict__ ps,
                                                  const int64_t* __restrict__ pool,
                                                  const unsigned long long* __restrict__ Pp,
                                                  int64_t cap, int32_t* __restrict__ order) {
    const int64_t P = min((int64_t)*Pp, cap);
    if (P > BITONIC_MAX) return;                // handled by k_rank
    __shared__ double ks[BITONIC_MAX];
    __shared__ int64_t ki[BITONIC_MAX];
    __shared__ int32_t kx[BITONIC_MAX];
    int N2 = 1;
    while (N2 < P) N2 <<= 1;
    for (int i = threadIdx.x; i < N2; i += 1024) {
        ks[i] = i < P ? ps[i] : -INFINITY;
        ki[i] = i < P ? pool[i] : INT64_MAX;
        kx[i] = i;
    }
    __syncthreads();
    for (int size = 2; size <= N2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int u = threadIdx.x; u < N2 / 2; u += 1024) {
                const int i = 2 * stride * (u / stride) + (u % stride);
                const int j = i + stride;
                const bool up = (i & size) == 0;
                // "before(a, b)": a.s > b.s, ties by smaller ID
                const bool jb = ks[j] > ks[i] || (ks[j] == ks[i] && ki[j] < ki[i]);
                if (jb == up) {
                    const double ts = ks[i]; ks[i] = ks[j]; ks[j] = ts;
                    const int64_t ti = ki[i]; ki[i] = ki[j]; ki[j] = ti;
                    const int32_t tx = kx[i]; kx[i] = kx[j]; kx[j] = tx;
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < P; i += 1024) order[i] = kx[i];
}

// Values of the selected candidates: one wave per output row.
__global__ __launch_bounds__(256) void k_values(const int64_t* __restrict__ ids, int64_t m,
                                                EvalCtx ev, Ops o, int n,
                                                double* __restrict__ out, int64_t ldv) {
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= m) return;
    const int lane = threadIdx.x & 63;
    const int64_t id = ids[w];
    Cand c;
    const bool ok = id >= 0 && cand_of_id(ev, id, c);
    for (int i = lane; i < n; i += 64)
        out[w * ldv + i] = ok ? cand_value(c, o, i) : __longlong_as_double(0x7FF8000000000000LL);
}

}  // namespace dsc

// ====================================================================== host
namespace dsc {

template <class T>
static T download1(const T* src, hipStream_t st) {
    T v;
    DSC_HIP(hipMemcpyAsync(&v, src, sizeof(T), hipMemcpyDeviceToHost, st));
    DSC_HIP(hipStreamSynchronize(st));
    return v;
}

static int pad_targets(int T) { return T <= 1 ? 1 : T <= 2 ? 2 : T <= 4 ? 4 : T <= 8 ? 8 : 16; }

template <int OPS, int J, int TP>
static void launch_pairs_t(const PairArgs& a, bool list, hipStream_t st) {
    const int64_t blocks = a.n_tiles;          // one 256-thread block per tile
    if (blocks == 0) return;
    if (list) k_screen_pairs<OPS, 1, TP, true><<<(unsigned)blocks, 256, 0, st>>>(a);
    else k_screen_pairs<OPS, J, TP, false><<<(unsigned)blocks, 256, 0, st>>>(a);
}

template <int OPS>
static void launch_pairs_ops(const PairArgs& a, bool list, int TP, int J, hipStream_t st) {
    switch (TP) {
    case 1:
        if (J == 4) launch_pairs_t<OPS, 4, 1>(a, list, st);
        else if (J == 2) launch_pairs_t<OPS, 2, 1>(a, list, st);
        else launch_pairs_t<OPS, 1, 1>(a, list, st);
        break;
    case 2:
        if (J == 2) launch_pairs_t<OPS, 2, 2>(a, list, st);
        else launch_pairs_t<OPS, 1, 2>(a, list, st);
        break;
    case 4: launch_pairs_t<OPS, 1, 4>(a, list, st); break;
    case 8: launch_pairs_t<OPS, 1, 8>(a, list, st); break;
    default: launch_pairs_t<OPS, 1, 16>(a, list, st); break;
    }
}

// Tile widths J (operand features j per wave) the dense kernel is built for.
static int max_J(int TP) { return TP == 1 ? 4 : TP == 2 ? 2 : 1; }

static void launch_pairs(int OPS, const PairArgs& a, bool list, int TP, int J, hipStream_t st) {
    switch (OPS) {
    case 31: launch_pairs_ops<31>(a, list, TP, J, st); break;
    case 28: launch_pairs_ops<28>(a, list, TP, J, st); break;
    case 3: launch_pairs_ops<3>(a, list, TP, J, st); break;
    default: DSC_FAIL(DISCOVER_E_UNSUPPORTED, "operator class %d", OPS);
    }
}

template <bool FP16>
static void launch_lp(int cls, const PairArgs& a, const void* ylp, int ldl, hipStream_t st) {
    const unsigned blocks = (unsigned)cdiv(a.n_tiles, 4);
    if (!blocks) return;
    switch (cls) {
    case 31: k_screen_lp<31, FP16><<<blocks, 256, 0, st>>>(a, ylp, ldl); break;
    case 28: k_screen_lp<28, FP16><<<blocks, 256, 0, st>>>(a, ylp, ldl); break;
    default: DSC_FAIL(DISCOVER_E_UNSUPPORTED, "operator class %d", cls);
    }
}

// Guard half-width of the precision forms (see k_screen_lp).
static double lowprec_delta(int precision, int n) {
    const double u = precision == DISCOVER_FP16_GUARD ? std::ldexp(1.0, -11) : std::ldexp(1.0, -8);
    const double g = n * std::ldexp(1.0, -24);
    double d = 2 * u + u * u + 1.01 * g / (1 - g) + 1e-12;
    if (precision == DISCOVER_FP16_GUARD) d += std::ldexp(1.0, -24);
    return d;
}

// Device-resident description of one search space and its work lists,
// cached in the context: it depends only on (p, n, units, parameters).
struct Plan {
    Space sp;
    int n = 0, TP = 1, ldn = 0, ldm = 0;
    std::vector<void*> allocs;
    int32_t* raw2c = nullptr;
    int64_t* mat_raw = nullptr;
    int8_t* mat_op = nullptr;
    int32_t *mat_a = nullptr, *mat_b = nullptr;
    ListItem* items = nullptr;
    int64_t n_items = 0;
    int2* dtilesJ[3] = {nullptr, nullptr, nullptr};   // dense tiles for J = 1, 2, 4
    int64_t n_dtilesJ[3] = {0, 0, 0};
    int tuned_J = 0;                                     // 0: not tuned yet
    double tune_ms[3] = {0, 0, 0};
    uint32_t dense_ops = 0;
    int dense_cls = 0;
    int2* ptiles = nullptr;                   // (j, i0) tiles of one j for the precision form
    int64_t n_ptiles = 0;
    int2* ltiles = nullptr;
    int32_t *ilist = nullptr, *icount = nullptr;
    int64_t n_ltiles = 0;
    uint32_t list_ops = 0;
    int4* r3tiles = nullptr;                  // rung-3 tiles over rung-2 operands
    int64_t n_r3tiles = 0;
    int32_t* mat_unit = nullptr;
    uint32_t r3_ops = 0;
    std::vector<int2> h_ltiles;               // host copies used to derive rung-3 tiles
    std::vector<int32_t> h_icount;

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
    const int32_t dims[4] = {pb.p, pb.n, pb.B, pad_targets(pb.T)};
    k.append((const char*)dims, sizeof dims);
    if (pb.B && pb.units) k.append((const char*)pb.units, sizeof(int32_t) * pb.p * pb.B);
    return k;
}

static std::shared_ptr<Plan> get_plan(discover_ctx* ctx, const discover_problem& pb,
                                      const discover_screen_params& prm) {
    const std::string key = plan_key(pb, prm);
    auto it = ctx->plans.find(key);
    if (it != ctx->plans.end()) return std::static_pointer_cast<Plan>(it->second);
    if (ctx->plans.size() >= 16) ctx->plans.clear();
    auto P = std::make_shared<Plan>();
    Space& sp = P->sp;
    build_space(sp, pb.p, prm, pb.B, pb.units);
    const SpaceDev& sd = sp.d;
    P->n = pb.n;
    P->TP = pad_targets(pb.T);
    P->ldn = (int)((pb.n + 63) / 64 * 64);
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
            std::vector<int2> tiles;
            for (int32_t j = jc0; j < jc1; j += J) {
                const int32_t ilim = std::min<int32_t>(i_end, std::min<int32_t>(j + J - 1, jc1 - 1));
                for (int32_t i0 = 0; i0 < ilim; i0 += 64) tiles.push_back(make_int2(j, i0));
            }
            P->dtilesJ[jx] = P->up(tiles);
            P->n_dtilesJ[jx] = (int64_t)tiles.size();
        }
        std::vector<int2> pt;
        for (int32_t j = jc0; j < jc1; j++) {
            const int32_t ilim = std::min<int32_t>(i_end, j);
            for (int32_t i0 = 0; i0 < ilim; i0 += 16 * LP_IB) pt.push_back(make_int2(j, i0));
        }
        P->ptiles = P->up(pt);
        P->n_ptiles = (int64_t)pt.size();
    }
    if (P->list_ops) {
        std::vector<int2> tiles;
        std::vector<int32_t> il, ic;
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
                        tiles.push_back(make_int2(c, (int)il.size()));
                        const int cnt = (int)std::min<size_t>(64, v.size() - q);
                        ic.push_back(cnt);
                        il.insert(il.end(), v.begin() + q, v.begin() + q + cnt);
                    }
                }
            }
            if (pool == R - 1) by_unit[key_of(c)].push_back(c);
        }
        P->ltiles = P->up(tiles);
        P->ilist = P->up(il);
        P->icount = P->up(ic);
        P->n_ltiles = (int64_t)tiles.size();
        if (sp.stream3) {            // keep the host copies for the rung-3 list tiles
            P->h_ltiles = tiles;
            P->h_icount = ic;
        }
    }
    if (sp.stream3) {
        // rung-3 candidates op3(i, j2): one wave per 64 rung-2 features j2
        std::vector<int4> t3;
        const int32_t c0 = sp.rung_start[1], c1 = sp.rung_start[2];
        for (int o = 0; o < OP_ADD; o++) {
            if (sd.block[2][o] < 0) continue;
            for (int32_t l0 = c0; l0 < c1; l0 += 64) t3.push_back(make_int4(o, l0, 0, -2));
        }
        for (int o = OP_ADD; o <= OP_RDIV; o++) {
            if (sd.block[2][o] < 0) continue;
            const bool addcls = o <= OP_SUB;
            if (units && addcls) {
                for (size_t q = 0; q < P->h_ltiles.size(); q++)
                    t3.push_back(make_int4(o, P->h_ltiles[q].x, P->h_ltiles[q].y, P->h_icount[q]));
            } else {
                for (int32_t l = c0; l < c1; l++)
                    for (int32_t k0 = 0; k0 < l; k0 += 64) t3.push_back(make_int4(o, l, k0, -1));
            }
        }
        P->r3tiles = P->up(t3);
        P->n_r3tiles = (int64_t)t3.size();
        std::vector<int32_t> mu(sp.mat_unit.begin(), sp.mat_unit.end());
        if (mu.empty()) mu.push_back(0);
        P->mat_unit = P->up(mu);
        for (int o = OP_ADD; o <= OP_RDIV; o++)
            if (sd.block[3][o] >= 0) P->r3_ops |= 1u << (o - OP_ADD);
    }
    ctx->plans[key] = P;
    return P;
}

struct Problem {
    std::shared_ptr<Plan> plan;
    int n, T, Tl, TP, ldn, ldm, Mc;
    double *Vf, *Rf, *Cf, *Vs, *Rs, *Cs, *mu, *mur, *msq, *Yc, *Yn, *syy, *ysum, *scores;
    uint8_t* valid;
    int* bad;
    unsigned long long* nscored;
    uint8_t* r2v = nullptr;                   // rung-2 operand statistics (streamed rung 3)
    double* r2m = nullptr;
    double* r2q = nullptr;
    int tile_j = 0;                           // dense pair kernel width used (0: not run)
    EvalCtx ev() const {
        EvalCtx e;
        e.sd = plan->sp.d;
        e.streamed = plan->sp.streamed;
        e.stream3 = plan->sp.stream3 ? 1 : 0;
        e.raw2c = plan->raw2c;
        e.valid = valid;
        e.r2_valid = r2v;
        return e;
    }
};

// Materialise the operand features and screen every candidate into the
// score slots (no host synchronisation).
static void screen_problem(discover_ctx* ctx, const discover_problem& pb,
                           const discover_screen_params& prm, Problem& P, hipStream_t st) {
    P.plan = get_plan(ctx, pb, prm);
    const Plan& pl = *P.plan;
    const Space& sp = pl.sp;
    const SpaceDev& sd = sp.d;
    const int n = pb.n;
    P.n = n;
    P.T = pb.T;
    P.Tl = prm.score_mode == DISCOVER_SCORE_MAX ? 1 : pb.T;
    P.TP = pl.TP;
    P.ldn = pl.ldn;
    P.ldm = pl.ldm;
    P.Mc = sp.Mc();
    const int Mc = P.Mc, ldn = P.ldn, ldm = P.ldm;
    const int64_t N = sp.n_raw();

    P.Vf = ctx->buf<double>("Vf", (size_t)Mc * ldn);
    P.Rf = ctx->buf<double>("Rf", (size_t)Mc * ldn);
    P.Cf = ctx->buf<double>("Cf", (size_t)Mc * ldn);
    P.mu = ctx->buf<double>("mu", Mc);
    P.mur = ctx->buf<double>("mur", Mc);
    P.msq = ctx->buf<double>("msq", Mc);
    P.valid = ctx->buf<uint8_t>("valid", Mc);
    P.Yc = ctx->buf<double>("Yc", (size_t)pb.T * ldn);
    P.Yn = ctx->buf<double>("Yn", (size_t)P.TP * ldn);
    P.syy = ctx->buf<double>("syy", pb.T);
    P.ysum = ctx->buf<double>("ysum", P.TP);
    // counters: [0] bad target, [1] fix-up count, [2] scored (as u64 slots)
    unsigned long long* ctr = ctx->buf<unsigned long long>("screen_ctr", 4);
    P.bad = (int*)ctr;
    P.nscored = ctr + 2;
    unsigned long long* fix_cnt = ctr + 1;
    DSC_HIP(hipMemsetAsync(ctr, 0, 32, st));
    DSC_HIP(hipMemsetAsync(P.Yn, 0, (size_t)P.TP * ldn * 8, st));
    DSC_HIP(hipMemsetAsync(P.ysum, 0, (size_t)P.TP * 8, st));
    k_targets<<<pb.T, 256, 0, st>>>(n, pb.T, pb.Y, pb.ldy, ldn, P.Yc, P.Yn, P.syy, P.ysum, P.bad);
    check_launch("k_targets");
    {
        KTimer kt(ctx, st, "materialise");
        for (size_t r = 0; r + 1 < sp.rung_start.size(); r++) {
            const int c0 = sp.rung_start[r], c1 = sp.rung_start[r + 1];
            if (c1 <= c0) continue;
            dim3 g((unsigned)cdiv(n, 256), (unsigned)(c1 - c0));
            k_mat_values<<<g, 256, 0, st>>>(n, ldn, c0, c1, pb.X, pb.ldx, pl.mat_op, pl.mat_a,
                                            pl.mat_b, pl.mat_raw, P.Vf);
            k_mat_stats<<<(unsigned)cdiv(c1 - c0, 4), 256, 0, st>>>(
                n, ldn, c0, c1, pl.mat_op, pl.mat_a, pl.mat_b, P.Vf, P.Rf, P.Cf, P.mu, P.mur, P.msq,
                P.valid);
        }
        check_launch("k_mat");
    }
    P.scores = ctx->buf<double>("scores", (size_t)P.Tl * N);
    DSC_HIP(hipMemsetAsync(P.scores, 0xFF, (size_t)P.Tl * N * 8, st));
    Ops ops{P.Vf, P.Rf, ldn};
    const int64_t off2 = sp.stream3 ? sd.off[2] : 0, off3 = sp.stream3 ? sd.off[3] : 0;
    if (sp.stream3) {
        P.r2v = ctx->buf<uint8_t>("r2v", sd.L[2]);
        P.r2m = ctx->buf<double>("r2m", sd.L[2]);
        P.r2q = ctx->buf<double>("r2q", sd.L[2]);
        DSC_HIP(hipMemsetAsync(P.r2v, 0, (size_t)sd.L[2], st));
    }
    {
        KTimer kt(ctx, st, "screen_list");
        k_score_list<<<(unsigned)cdiv(pl.n_items, 4), 256, 0, st>>>(
            pl.items, pl.n_items, ops, P.valid, n, pb.T, prm.score_mode, P.Yc, P.syy, N, P.scores,
            P.nscored, P.r2v, P.r2m, P.r2q, off2, off3);
        check_launch("k_score_list");
    }
    const int R = sp.streamed;
    if (!R || (!pl.dense_ops && !pl.list_ops)) return;
    P.Vs = ctx->buf<double>("Vs", (size_t)n * ldm);
    P.Rs = ctx->buf<double>("Rs", (size_t)n * ldm);
    P.Cs = ctx->buf<double>("Cs", (size_t)n * ldm);
    {
        dim3 g((unsigned)cdiv(n, 32), (unsigned)cdiv(Mc, 32)), b(32, 8);
        k_transpose<<<g, b, 0, st>>>(n, Mc, ldn, ldm, P.Vf, P.Vs);
        k_transpose<<<g, b, 0, st>>>(n, Mc, ldn, ldm, P.Rf, P.Rs);
        k_transpose<<<g, b, 0, st>>>(n, Mc, ldn, ldm, P.Cf, P.Cs);
        check_launch("k_transpose");
    }
    const int pool = sd.pool[R];
    PairArgs a{};
    a.n = n; a.ldm = ldm; a.ldn = ldn; a.Mc = Mc; a.jc_end = sp.rung_start[R];
    a.i_end = pool == R - 1 ? Mc : sp.rung_start[pool + 1];
    a.Vs = P.Vs; a.Rs = P.Rs; a.Cs = P.Cs; a.Vf = P.Vf; a.Rf = P.Rf; a.Cf = P.Cf;
    a.mu = P.mu; a.mur = P.mur; a.valid = P.valid; a.mat_raw = pl.mat_raw;
    a.Yn = P.Yn; a.ysum = P.ysum; a.T = pb.T; a.mode = prm.score_mode; a.r = R;
    a.sd = sd; a.N = N; a.scores = P.scores; a.nscored = P.nscored;
    a.fix_cap = std::min<int64_t>(N, (int64_t)1 << 24);
    a.fix_ids = ctx->buf<int64_t>("fix_ids", a.fix_cap);
    a.fix_cnt = fix_cnt;
    a.r2v = P.r2v;
    a.r2m = P.r2m;
    a.r2q = P.r2q;
    a.msq = P.msq;
    if (pl.dense_ops && prm.precision != DISCOVER_FP64) {
        const int ldl = (int)cdiv(n, 32) * 32;
        void* ylp = ctx->raw("Ylp", (size_t)16 * ldl * 2);
        dim3 gy((unsigned)cdiv(ldl, 256), 16);
        const bool fp16 = prm.precision == DISCOVER_FP16_GUARD;
        if (fp16) k_targets_lp<true><<<gy, 256, 0, st>>>(n, pb.T, ldn, ldl, P.Yn, (_Float16*)ylp);
        else k_targets_lp<false><<<gy, 256, 0, st>>>(n, pb.T, ldn, ldl, P.Yn, (__bf16*)ylp);
        a.tiles = pl.ptiles; a.ilist = nullptr; a.icount = nullptr;
        a.n_tiles = pl.n_ptiles; a.opmask = pl.dense_ops;
        KTimer kt(ctx, st, "screen_lp");
        if (fp16) launch_lp<true>(pl.dense_cls, a, ylp, ldl, st);
        else launch_lp<false>(pl.dense_cls, a, ylp, ldl, st);
        check_launch("k_screen_lp");
    } else if (pl.dense_ops) {
        a.ilist = nullptr; a.icount = nullptr; a.opmask = pl.dense_ops;
        Plan& mp = *P.plan;
        if (prm.tile_j <= 0 && mp.tuned_J == 0) {
            // autotune the tile width once per plan: every variant writes the same
            // scores (each candidate's sums run in the same order), so the timing
            // runs only repeat idempotent stores; the counters they bump are
            // restored after each run, and the fastest J is cached in the plan
            unsigned long long* saved = ctx->buf<unsigned long long>("screen_ctr_tune", 4);
            DSC_HIP(hipMemcpyAsync(saved, ctr, 32, hipMemcpyDeviceToDevice, st));
            double best = 1e30;
            for (int jx = 0; jx < 3 && (1 << jx) <= max_J(P.TP); jx++) {
                a.tiles = mp.dtilesJ[jx];
                a.n_tiles = mp.n_dtilesJ[jx];
                hipEvent_t e0 = ctx->event(), e1 = ctx->event();
                DSC_HIP(hipEventRecord(e0, st));
                launch_pairs(pl.dense_cls, a, false, P.TP, 1 << jx, st);
                DSC_HIP(hipEventRecord(e1, st));
                DSC_HIP(hipMemcpyAsync(ctr, saved, 32, hipMemcpyDeviceToDevice, st));
                DSC_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                DSC_HIP(hipEventElapsedTime(&ms, e0, e1));
                ctx->free_events.push_back(e0);
                ctx->free_events.push_back(e1);
                mp.tune_ms[jx] = ms;
                if (ms < best) { best = ms; mp.tuned_J = 1 << jx; }
            }
        }
        int J = mp.tuned_J;
        if (prm.tile_j > 0) {
            // caller-forced width, rounded down to a power of two built for this TP
            J = 1;
            while (J * 2 <= std::min(prm.tile_j, max_J(P.TP))) J *= 2;
        }
        P.tile_j = J;
        const int jx = J == 4 ? 2 : J == 2 ? 1 : 0;
        a.tiles = mp.dtilesJ[jx];
        a.n_tiles = mp.n_dtilesJ[jx];
        KTimer kt(ctx, st, "screen_pairs");
        launch_pairs(pl.dense_cls, a, false, P.TP, J, st);
        check_launch("k_screen_pairs");
    }
    if (pl.list_ops && pl.n_ltiles) {
        a.tiles = pl.ltiles; a.ilist = pl.ilist; a.icount = pl.icount;
        a.n_tiles = pl.n_ltiles; a.opmask = pl.list_ops;
        KTimer kt(ctx, st, "screen_pairs_list");
        launch_pairs(3, a, true, P.TP, 1, st);
        check_launch("k_screen_pairs(list)");
    }
    const EvalCtx ev = P.ev();
    {
        // exact decision for the ill-conditioned ones (persistent waves over
        // the device-side count)
        KTimer kt(ctx, st, "screen_fixup");
        k_fixup<DISCOVER_MAX_TARGETS><<<1024, 256, 0, st>>>(
            a.fix_ids, a.fix_cnt, a.fix_cap, ev, ops, n, pb.T, prm.score_mode, P.Yc, P.syy, N,
            P.scores, P.nscored, P.r2v, P.r2m, P.r2q);
        check_launch("k_fixup");
    }
    if (!sp.stream3 || !pl.r3_ops || !pl.n_r3tiles) return;
    // operator-limited rung 3 on top of the rung-2 operand statistics
    unsigned long long* fix3 = ctr + 3;
    R3Args g3{};
    g3.tiles = pl.r3tiles; g3.klist = pl.ilist; g3.n_tiles = pl.n_r3tiles;
    g3.n = n; g3.ldm = ldm; g3.ldn = ldn; g3.Mc = Mc;
    g3.c1_lo = sp.rung_start[1]; g3.c1_hi = sp.rung_start[2];
    g3.pe = sp.rung_start[sd.pool[3] + 1];
    g3.B = sp.B;
    g3.Vs = P.Vs; g3.Rs = P.Rs; g3.Cs = P.Cs; g3.Vf = P.Vf; g3.Rf = P.Rf; g3.Cf = P.Cf;
    g3.mu = P.mu; g3.mur = P.mur; g3.valid = P.valid; g3.mat_raw = pl.mat_raw;
    g3.mat_unit = pl.mat_unit; g3.r2v = P.r2v; g3.r2m = P.r2m; g3.r2q = P.r2q; g3.msq = P.msq;
    g3.Yn = P.Yn; g3.ysum = P.ysum; g3.T = pb.T; g3.mode = prm.score_mode;
    g3.opmask = pl.r3_ops; g3.sd = sd; g3.N = N; g3.scores = P.scores; g3.nscored = P.nscored;
    g3.fix_cap = a.fix_cap;
    g3.fix_ids = ctx->buf<int64_t>("fix_ids3", g3.fix_cap);
    g3.fix_cnt = fix3;
    {
        KTimer kt(ctx, st, "screen_r3");
        const unsigned blocks = (unsigned)cdiv(g3.n_tiles, 4);
        switch (P.TP) {
        case 1: k_screen_r3<31, 2, 1><<<blocks, 256, 0, st>>>(g3); break;
        case 2: k_screen_r3<31, 2, 2><<<blocks, 256, 0, st>>>(g3); break;
        case 4: k_screen_r3<31, 1, 4><<<blocks, 256, 0, st>>>(g3); break;
        case 8: k_screen_r3<31, 1, 8><<<blocks, 256, 0, st>>>(g3); break;
        default: k_screen_r3<31, 1, 16><<<blocks, 256, 0, st>>>(g3); break;
        }
        check_launch("k_screen_r3");
    }
    {
        KTimer kt(ctx, st, "screen_fixup");
        k_fixup<DISCOVER_MAX_TARGETS><<<1024, 256, 0, st>>>(
            g3.fix_ids, g3.fix_cnt, g3.fix_cap, ev, ops, n, pb.T, prm.score_mode, P.Yc, P.syy, N,
            P.scores, P.nscored, nullptr, nullptr, nullptr);
        check_launch("k_fixup");
    }
}

// Exact top-k of list t (pool, rescore, sort, duplicate groups).  The
// pool holds every candidate whose score can reach the K-th largest
// approximate score minus the error margin; it is rescored exactly and
// grouped in (-score, ID) order.  If the pool does not reach below the
// near-tie window of the k-th group, K grows and the selection repeats.
static void select_list(discover_ctx* ctx, const discover_problem& pb,
                        const discover_screen_params& prm, Problem& P, int t, double margin,
                        int64_t* out_ids, double* out_sc, discover_screen_stats& stats,
                        hipStream_t st) {
    const Plan& pl = *P.plan;
    const Space& sp = pl.sp;
    const int64_t N = sp.n_raw();
    const double* sc = P.scores + (int64_t)t * N;
    const int k = prm.k;
    int64_t K = 2 * (int64_t)k + pb.n_exclude + 64;
    uint32_t* hist = ctx->buf<uint32_t>("hist", 4096);
    uint32_t* sel = ctx->buf<uint32_t>("sel", 4);
    int64_t* stv = ctx->buf<int64_t>("selst", 2);
    unsigned long long* cnt = ctx->buf<unsigned long long>("poolcnt", 1);
    int64_t* res = ctx->buf<int64_t>("groupres", 8);
    unsigned long long* maxerr = ctx->buf<unsigned long long>("maxerr", 1);
    DSC_HIP(hipMemsetAsync(maxerr, 0, 8, st));
    Ops ops{P.Vf, P.Rf, P.ldn};
    int64_t cap = 4 * K + 4096;
    int64_t fcap = 64 * cap;
    for (;;) {
        {
            KTimer kt(ctx, st, "select");
            radix_select(sc, N, K, hist, sel, stv, st);
        }
        int64_t* pool = ctx->buf<int64_t>("pool", cap);
        double* ps = ctx->buf<double>("ps", cap);
        uint8_t* pex = ctx->buf<uint8_t>("pex", cap);
        int32_t* order = ctx->buf<int32_t>("order", cap);
        int32_t* lo = ctx->buf<int32_t>("wlo", cap);
        int32_t* wc = ctx->buf<int32_t>("wcnt", cap);
        int64_t* off = ctx->buf<int64_t>("woff", cap + 1);
        uint8_t* flag = ctx->buf<uint8_t>("dupflag", fcap);
        int32_t* parent = ctx->buf<int32_t>("gparent", cap + 1);
        int32_t* blk = ctx->buf<int32_t>("gblk", cap + 1);
        unsigned long long* repid = ctx->buf<unsigned long long>("grepid", cap + 1);
        int32_t* reppos = ctx->buf<int32_t>("greppos", cap + 1);
        int32_t* headpos = ctx->buf<int32_t>("gheadpos", (size_t)k + 1);
        DSC_HIP(hipMemsetAsync(cnt, 0, 8, st));
        const unsigned hb = (unsigned)std::min<int64_t>(1024, std::max<int64_t>(1, cdiv(N, 256 * 8)));
        k_compact<<<hb, 256, 0, st>>>(sc, N, sel, stv, margin, cap, pool, cnt);
        check_launch("k_compact");
        {
            KTimer kt(ctx, st, "rescore");
            k_rescore<DISCOVER_MAX_TARGETS><<<(unsigned)std::min<int64_t>(2048, cdiv(cap, 4)), 256, 0, st>>>(
                pool, cnt, cap, P.ev(), ops, P.n, P.T, prm.score_mode, t,
                P.Yc, P.syy, pb.exclude, pb.exclude ? pb.n_exclude : 0, ps, pex, sc, maxerr);
            check_launch("k_rescore");
        }
        {
            KTimer kt(ctx, st, "sort_dedup");
            k_bitonic<<<1, 1024, 0, st>>>(ps, pool, cnt, cap, order);
            k_rank<<<(unsigned)cdiv(cap, 256), 256, 0, st>>>(ps, pool, cnt, cap, order);
            k_window<<<(unsigned)std::min<int64_t>(1024, cdiv(cap, 256)), 256, 0, st>>>(ps, order, cnt, cap, lo, wc);
            k_scan_offsets<<<1, 1024, 0, st>>>(wc, cnt, cap, off);
            check_launch("k_sort");
        }
        if (prm.dedup) {
            KTimer kt(ctx, st, "dedup_pairs");
            k_pairs<<<2048, 256, 0, st>>>(pool, order, lo, off, cnt, cap, P.ev(), ops, P.n, flag, fcap);
            check_launch("k_pairs");
        }
        {
            KTimer kt(ctx, st, "groups");
            k_groups<<<1, GRP_THREADS, 0, st>>>(pool, ps, pex, order, lo, off, flag, cnt, cap, fcap, k,
                                                prm.dedup, sel, stv, margin, parent, blk, repid,
                                                reppos, headpos, out_ids, out_sc, res);
            check_launch("k_groups");
        }
        int64_t h_res[8];
        int h_bad = 0;
        double h_err = 0.0;
        DSC_HIP(hipMemcpyAsync(h_res, res, sizeof h_res, hipMemcpyDeviceToHost, st));
        DSC_HIP(hipMemcpyAsync(&h_err, maxerr, 8, hipMemcpyDeviceToHost, st));
        DSC_HIP(hipMemcpyAsync(&h_bad, P.bad, sizeof h_bad, hipMemcpyDeviceToHost, st));
        DSC_HIP(hipStreamSynchronize(st));
        if (h_bad) DSC_FAIL(DISCOVER_E_NUMERIC, "a target column is constant or not finite");
        if (h_res[4] > cap) {                       // pool overflow: enlarge and redo
            cap = h_res[4] + 1024;
            fcap = std::max(fcap, 64 * cap);
            stats.pool_rounds += 1;
            continue;
        }
        if (prm.dedup && h_res[3] > fcap) {         // pair-flag overflow
            fcap = h_res[3] + 1024;
            stats.pool_rounds += 1;
            continue;
        }
        stats.pool_size += h_res[4];
        stats.max_lowprec_err = std::max(stats.max_lowprec_err, h_err);
        if (h_res[1] || K >= N) {
            stats.n_selected += h_res[0];
            stats.n_merged += h_res[2];
            return;
        }
        stats.pool_rounds += 1;
        K = std::min<int64_t>(N, K * 4);
        cap = 4 * K + 4096;
        fcap = std::max(fcap, 64 * cap);
    }
}

static void validate(const discover_problem* probs, int32_t nb, const discover_screen_params* prm,
                     const int64_t* out_ids, const double* out_sc, const double* out_values,
                     int64_t ldv) {
    DSC_REQUIRE(probs && prm && nb >= 1, "probs/prm must be non-NULL and n_problems >= 1");
    DSC_REQUIRE(out_ids && out_sc, "out_ids and out_scores are required");
    DSC_REQUIRE(prm->rung >= 0 && prm->rung <= DISCOVER_MAX_RUNG, "rung %d outside 0..3", prm->rung);
    DSC_REQUIRE(prm->k >= 1, "k must be >= 1");
    DSC_REQUIRE((prm->ops & ~DISCOVER_OPS_ALL) == 0, "unknown operator bits 0x%x", prm->ops);
    DSC_REQUIRE(prm->score_mode == DISCOVER_SCORE_PER_TARGET || prm->score_mode == DISCOVER_SCORE_MAX,
                "score_mode %d", prm->score_mode);
    DSC_REQUIRE(prm->precision >= DISCOVER_FP64 && prm->precision <= DISCOVER_FP16_GUARD,
                "precision %d", prm->precision);
    DSC_REQUIRE(prm->tile_j >= 0 && prm->tile_j <= 4, "tile_j %d outside 0..4", prm->tile_j);
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

}  // namespace dsc

extern "C" discover_status discover_generate_screen(discover_ctx* ctx, const discover_problem* probs,
                                                    int32_t n_problems,
                                                    const discover_screen_params* prm,
                                                    int64_t* out_ids, double* out_scores,
                                                    double* out_values, int64_t ldv,
                                                    discover_screen_stats* out_stats, void* stream) {
    using namespace dsc;
    return guarded([&] {
        DSC_REQUIRE(ctx, "ctx is NULL");
        validate(probs, n_problems, prm, out_ids, out_scores, out_values, ldv);
        DSC_HIP(hipSetDevice(ctx->device));
        hipStream_t st = (hipStream_t)stream;
        int64_t row = 0;
        for (int b = 0; b < n_problems; b++) {
            const discover_problem& pb = probs[b];
            Problem P{};
            discover_screen_stats stats{};
            screen_problem(ctx, pb, *prm, P, st);
            stats.n_raw = P.plan->sp.n_raw();
            stats.n_unit_valid = P.plan->sp.n_unit_valid;
            stats.tile_j = P.tile_j;
            double margin = 4.0 * P.n * EPS64 * KAPPA_MAX;
            if (prm->precision != DISCOVER_FP64) {
                stats.guard_band = lowprec_delta(prm->precision, P.n);
                margin = std::max(margin, stats.guard_band);
            }
            const int Tl = P.Tl;
            for (int t = 0; t < Tl; t++) {
                select_list(ctx, pb, *prm, P, t, margin, out_ids + (row + t) * prm->k,
                            out_scores + (row + t) * prm->k, stats, st);
            }
            if (out_values) {
                KTimer kt(ctx, st, "values");
                Ops ops{P.Vf, P.Rf, P.ldn};
                const int64_t m = (int64_t)Tl * prm->k;
                k_values<<<(unsigned)cdiv(m, 4), 256, 0, st>>>(out_ids + row * prm->k, m, P.ev(), ops, P.n,
                                                               out_values + row * prm->k * ldv, ldv);
                check_launch("k_values");
            }
            stats.n_scored = (int64_t)download1(P.nscored, st);
            DSC_HIP(hipStreamSynchronize(st));
            ctx->resolve_timing();
            if (out_stats) out_stats[b] = stats;
            row += Tl;
        }
    });
}
