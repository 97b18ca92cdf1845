// Operator-limited rung 3 on gfx950: screening of op3(f_i, g) for every
// partner f_i of the pool and every rung-2 feature g, without storing g
// (candidate generation by operators, Software Description; screening, the
// SIS step of the cited SISSO method, Summary).
//
// mul / div / rdiv: the per-candidate sums are matrix products over samples.
// A wave holds GT blocks of 16 rung-2 features (rows, regenerated in
// registers from their two rung-1 operands, 4 consecutive samples per lane)
// and one tile of 16 partner columns.  For every target t, the products
// sum_s a_s (x_s y_ts) give P_t, sum_s a_s x_s gives S1 and sum_s a_s^2 x_s^2
// gives S2, where a = g (mul, and rdiv with x replaced by 1/x) or a = 1/g
// (div).  The right-hand operands [x y_t | x | x^2] of every column tile are
// laid out once per call by k_r3_bmat, in the lane order of
// v_mfma_f64_16x16x4f64 (B[k][j] from lane j + 16k, four samples per lane),
// so a wave reads each as one 32-byte load per lane.
//
// The one-pass moments are unshifted: with kappa = S2 / (S2 - S1^2/n) the
// rounding error of every score is below 2.5 n u kappa (u = 2^-53; n sums
// of rounded products, plus the variance's cancellation), inside the
// selection margin 4 n u KAPPA_MAX for kappa <= KAPPA_MAX.  Candidates with
// a larger kappa, or whose values might overflow, are listed for the exact
// two-pass fix-up; candidates whose values are certainly not finite (a
// division by an exact zero) are left invalid.
#include "dsc_r3.h"

#include <algorithm>
#include <map>
#include <string>
#include <type_traits>

namespace dsc {

namespace {

constexpr double R3_KAPPA_MAX = 64.0;   // same bound as the other fast screens
constexpr double R3_BIG = 1e150;        // |f| below this: f and n f^2 stay finite
constexpr double R3_TINY = 1e-300;      // |g| above this: 1/g is finite
constexpr double R3_TAU_CONST = 1e-8;
constexpr double R3_TAU_CANCEL_FAST = 1e-12;

typedef double r3_v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int r3_wave() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Workgroups are dealt to the 8 XCDs in turn (block b to XCD b % 8); this
// numbering gives each XCD a contiguous range of the grid's logical blocks,
// so that the row tiles one XCD works on at a time are neighbours in the
// record order and share their operand rows in that XCD's L2.
__device__ __forceinline__ int r3_xcd_block() {
    const int nb = (int)gridDim.x, b = (int)blockIdx.x;
    const int per = nb >> 3, rem = nb & 7, x = b & 7, pos = b >> 3;
    return x < rem ? x * (per + 1) + pos : rem * (per + 1) + (x - rem) * per + pos;
}

// Slot of each active lane in a list (lane order), one atomic per wave.
__device__ __forceinline__ unsigned long long r3_slot(unsigned long long* ctr) {
    const uint64_t m = __builtin_amdgcn_ballot_w64(true);
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)m) - 1;
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(ctr, (unsigned long long)__popcll(m));
    base = __shfl(base, leader, 64);
    return base + (unsigned long long)__popcll(m & ((1ull << lane) - 1ull));
}

__device__ __forceinline__ double r3_un(int op, double a) {
    switch (op) {
    case OP_EXP: return exp(a);
    case OP_LOG: return log(a);
    case OP_SQRT: return sqrt(a);
    default: return a * a;               // OP_SQ (OP_INV reads the reciprocal row)
    }
}

// Rung-2 operator applied to operands already loaded: x from row p1, y from
// row p2 of r3_rows (reciprocal rows where the operator divides).
__device__ __forceinline__ r3_v4d r3_combine(int op2, r3_v4d x, r3_v4d y) {
    switch (op2) {
    case OP_EXP: return r3_v4d{exp(x.x), exp(x.y), exp(x.z), exp(x.w)};
    case OP_LOG: return r3_v4d{log(x.x), log(x.y), log(x.z), log(x.w)};
    case OP_SQRT: return r3_v4d{sqrt(x.x), sqrt(x.y), sqrt(x.z), sqrt(x.w)};
    case OP_SQ: return x * x;
    case OP_INV: return x;
    case OP_ADD: return x + y;
    case OP_SUB: return x - y;
    default: return x * y;               // OP_MUL, OP_DIV, OP_RDIV
    }
}

// Operand rows of rung-2 feature (k, l, op2): the combine above of rows p1
// and p2 gives its values (the formulas of the rung-2 screen: a division
// multiplies by the stored reciprocal).
__device__ __forceinline__ void r3_rows(const double* Vf, const double* Rf, int64_t ldn, int k, int l,
                                        int op2, const double*& p1, const double*& p2) {
    const int64_t kk = k < 0 ? 0 : k;
    if (op2 < OP_ADD) {
        p1 = (op2 == OP_INV ? Rf : Vf) + (int64_t)l * ldn;
        p2 = p1;
    } else if (op2 == OP_RDIV) {
        p1 = Vf + (int64_t)l * ldn;
        p2 = Rf + kk * ldn;
    } else {
        p1 = Vf + kk * ldn;
        p2 = (op2 == OP_DIV ? Rf : Vf) + (int64_t)l * ldn;
    }
}

__device__ __forceinline__ double r3_regen1(const double* __restrict__ Vf, const double* __restrict__ Rf,
                                            int64_t ldn, int k, int l, int op2, int s) {
    const double b = Vf[(int64_t)l * ldn + s];
    if (k < 0) return op2 == OP_INV ? Rf[(int64_t)l * ldn + s] : r3_un(op2, b);
    const double a = Vf[(int64_t)k * ldn + s];
    switch (op2) {
    case OP_ADD: return a + b;
    case OP_SUB: return a - b;
    case OP_MUL: return a * b;
    case OP_DIV: return a * Rf[(int64_t)l * ldn + s];
    default: return b * Rf[(int64_t)k * ldn + s];
    }
}

__device__ __forceinline__ double r3_rcp(double g) {
    double r = __builtin_amdgcn_rcp(g);
    r = fma(r, fma(-g, r, 1.0), r);
    return fma(r, fma(-g, r, 1.0), r);
}

__device__ __forceinline__ void r3_rec(int2 rc, int& k, int& l, int& op2) {
    k = rc.x;
    l = rc.y & 0x0FFFFFFF;
    op2 = (int)((unsigned)rc.y >> 28);
}

__device__ __forceinline__ int64_t r3_j2(const SpaceDev& sd, const int64_t* mat_raw, int k, int l, int op2) {
    return k < 0 ? unary_id(sd, 2, op2, mat_raw[l]) : pair_id(sd, 2, op2, mat_raw[k], mat_raw[l]);
}

// ------------------------------------------------------------ set-up
// max |x| and min |x| of every partner over the n samples.
__global__ __launch_bounds__(256) void k_r3_pstat(int n, int64_t ldn, int pe, const double* __restrict__ Vf,
                                                  double* __restrict__ pstat) {
    const int p = blockIdx.x;
    double mx = 0.0, mn = INFINITY;
    for (int s = threadIdx.x; s < n; s += 256) {
        const double v = fabs(Vf[(int64_t)p * ldn + s]);
        mx = fmax(mx, v);
        mn = fmin(mn, v);
    }
    __shared__ double smx[256], smn[256];
    smx[threadIdx.x] = mx;
    smn[threadIdx.x] = mn;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            smx[threadIdx.x] = fmax(smx[threadIdx.x], smx[threadIdx.x + o]);
            smn[threadIdx.x] = fmin(smn[threadIdx.x], smn[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pstat[p] = smx[0];
        pstat[pe + p] = smn[0];
    }
}

// Per-partner sums for add / sub: pc[p (TP + 2) + t] = sum_s x_s y_ts (t <
// TP), sum x (t = TP), sum x^2 (t = TP + 1); one block per partner, a fixed
// reduction order.
__global__ __launch_bounds__(256) void k_r3_pconst(int n, int64_t ldn, int TP, const double* __restrict__ Vf,
                                                   const double* __restrict__ Yn, double* __restrict__ pc) {
    const int p = blockIdx.x;
    __shared__ double part[256];
    for (int t = 0; t < TP + 2; t++) {
        double a = 0.0;
        for (int s = threadIdx.x; s < n; s += 256) {
            const double x = Vf[(int64_t)p * ldn + s];
            a += t < TP ? x * Yn[(int64_t)t * ldn + s] : t == TP ? x : x * x;
        }
        part[threadIdx.x] = a;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) pc[(int64_t)p * (TP + 2) + t] = part[0];
        __syncthreads();
    }
}

// Right-hand operands: bmat[((c TK + t) NQ + q) 64 + 4 j + e] = column j of
// tile c, kind t, sample 4q + e; kinds t < TP: x y_t, t = TP: x, TP+1: x^2,
// with x = f_p (mul, div and add/sub columns), 1/f_p (rdiv columns) or 1
// (the column of ones of an add/sub tile); zero for padding columns and
// samples >= n.
__global__ __launch_bounds__(256) void k_r3_bmat(int n, int64_t ldn, int TP, int NQ, int nct,
                                                 const int32_t* __restrict__ coldesc,
                                                 const double* __restrict__ Vf, const double* __restrict__ Rf,
                                                 const double* __restrict__ Yn, double* __restrict__ bmat) {
    const int TK = TP + 2;
    const int64_t total = (int64_t)nct * TK * NQ * 64;
    for (int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x; f < total; f += (int64_t)gridDim.x * 256) {
        const int e = (int)(f & 3), j = (int)((f >> 2) & 15);
        const int64_t r = f >> 6;
        const int q = (int)(r % NQ);
        const int64_t ct_t = r / NQ;
        const int t = (int)(ct_t % TK), c = (int)(ct_t / TK);
        const int s = 4 * q + e;
        const int32_t d = coldesc[c * 16 + j];
        double v = 0.0;
        if (d >= 0 && s < n) {
            const int p = d & 0xFFFF, kind = d >> 16;
            const double x = kind == 3 ? 1.0 : kind == 1 ? Rf[(int64_t)p * ldn + s] : Vf[(int64_t)p * ldn + s];
            v = t < TP ? x * Yn[(int64_t)t * ldn + s] : t == TP ? x : x * x;
        }
        bmat[f] = v;
    }
}

// The targets in the B lane order: yb[q 64 + 4 j + e] = y_j at sample 4q + e
// (0 for j >= TP and samples >= n).
__global__ __launch_bounds__(256) void k_r3_ybmat(int n, int64_t ldn, int TP, int NQ,
                                                  const double* __restrict__ Yn, double* __restrict__ yb) {
    const int64_t total = (int64_t)NQ * 64;
    for (int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x; f < total; f += (int64_t)gridDim.x * 256) {
        const int e = (int)(f & 3), j = (int)((f >> 2) & 15);
        const int s = 4 * (int)(f >> 6) + e;
        yb[f] = j < TP && s < n ? Yn[(int64_t)j * ldn + s] : 0.0;
    }
}

// ------------------------------------------------------------ MFMA screen
struct R3mArgs {
    const int2* grec;
    int64_t n_grec;
    const int2* work;         // add / sub: (row tile, column tile) per wave
    int64_t n_work;
    const double* pconst;     // add / sub: per-partner sums (k_r3_pconst)
    const int32_t* coldesc;
    int n_gct, n_gblk, NQ, n, T, mode;
    int64_t ldn;
    const double* bmat;
    const double* ybmat;      // add / sub: the targets (k_r3_ybmat)
    const double *Vf, *Rf;
    const double* pstat;
    int pe;
    uint32_t ops;
    const uint8_t* valid;
    const int64_t* mat_raw;
    const uint8_t* r2v;
    const double* ysum;
    SpaceDev sd;
    SlotMap sm;
    int64_t N;
    double* scores;
    unsigned long long* nscored;
    int64_t* fix_ids;         // score slots
    unsigned long long* fix_cnt;
    int64_t fix_cap;
};

template <int TP, int GT, bool AS>
__global__ __launch_bounds__(256) void k_r3_mm(R3mArgs g) {
    constexpr int TK = TP + 2;
    static_assert(!AS || GT == 1, "add/sub tiles come one per wave");
    const int lane = threadIdx.x & 63;
    const int r16 = lane & 15, kq = lane >> 4;
    int ct;
    int64_t tile0;
    const int64_t w = (int64_t)blockIdx.x * 4 + r3_wave();   // add / sub: the work item
    if (AS) {                                          // explicit (row tile, column tile) list
        if (w >= g.n_work) return;
        const int2 wk = g.work[w];
        tile0 = wk.x;
        ct = wk.y;
    } else {
        const int lb = r3_xcd_block();
        ct = lb / g.n_gblk;                            // column tile (slowest: its operands stay in L2)
        const int gb = lb - ct * g.n_gblk;
        tile0 = ((int64_t)gb * 4 + r3_wave()) * GT;
        if (tile0 * 16 >= g.n_grec) return;
    }
    const bool hk = !AS && ct >= g.n_gct;              // rows hold 1/g (div columns)
    const double* __restrict__ Vf = g.Vf;
    const double* __restrict__ Rf = g.Rf;

    // every tile's records share one operator (runs are padded to 16), so
    // the regeneration's branches are uniform; absent rows read feature 0
    int kk[GT], ll[GT], oo[GT];
    bool rok[GT];
    int64_t j2[GT];
#pragma unroll
    for (int u = 0; u < GT; u++) {
        const int64_t t16 = min(tile0 + u, (g.n_grec >> 4) - 1) * 16;
        const int64_t rec = (tile0 + u) * 16 + r16;
        int k = -2, l = 0, op2;
        r3_rec(g.grec[rec < g.n_grec ? rec : t16], k, l, op2);
        oo[u] = __builtin_amdgcn_readfirstlane(op2);
        rok[u] = rec < g.n_grec && k != -2;
        j2[u] = rok[u] ? r3_j2(g.sd, g.mat_raw, k, l, op2) : 0;
        rok[u] = rok[u] && g.r2v[j2[u] - g.sd.off[2]];
        kk[u] = oo[u] < OP_ADD ? -1 : (rok[u] ? k : 0);
        ll[u] = rok[u] ? l : 0;
    }
    const double* p1[GT];
    const double* p2[GT];
#pragma unroll
    for (int u = 0; u < GT; u++) r3_rows(Vf, Rf, g.ldn, kk[u], ll[u], oo[u], p1[u], p2[u]);
    r3_v4d acc[GT][TK];
#pragma unroll
    for (int u = 0; u < GT; u++)
#pragma unroll
        for (int t = 0; t < TK; t++) acc[u][t] = r3_v4d{0.0, 0.0, 0.0, 0.0};
    double gmx[GT], gmn[GT];
#pragma unroll
    for (int u = 0; u < GT; u++) { gmx[u] = 0.0; gmn[u] = INFINITY; }

    const double* bp = g.bmat + (int64_t)ct * TK * g.NQ * 64 + lane * 4;
    const int nm = g.NQ >> 2;
    if constexpr (AS) {
        // add / sub need per row only sum g y_t, sum g, sum g^2 and per pair
        // sum x g: three product streams, g against [x | 1] (acc[0][TP]),
        // against the targets (acc[0][0], column t = target t) and g^2
        // against [x^2 | 1] (acc[0][TP + 1], its column of ones)
        const double* yp = g.ybmat + lane * 4;
        for (int m = 0; m < nm; m++) {
            const int s = 16 * m + 4 * kq;
            r3_v4d v = r3_combine(oo[0], *(const r3_v4d*)(p1[0] + s), *(const r3_v4d*)(p2[0] + s));
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const bool in = rok[0] && s + e < g.n;
                v[e] = in ? v[e] : 0.0;
            }
            const r3_v4d v2 = v * v;
            const r3_v4d bx = *(const r3_v4d*)(bp + ((int64_t)TP * g.NQ + 4 * m) * 64);
            const r3_v4d bq = *(const r3_v4d*)(bp + ((int64_t)(TP + 1) * g.NQ + 4 * m) * 64);
            const r3_v4d by = *(const r3_v4d*)(yp + (int64_t)(4 * m) * 64);
#pragma unroll
            for (int e = 0; e < 4; e++) {
                acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[e], by[e], acc[0][0], 0, 0, 0);
                acc[0][TP] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[e], bx[e], acc[0][TP], 0, 0, 0);
                acc[0][TP + 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(v2[e], bq[e], acc[0][TP + 1], 0, 0, 0);
            }
        }
    } else {
    for (int m = 0; m < nm; m++) {
        const int s = 16 * m + 4 * kq;
        r3_v4d A[GT], A2[GT];
#pragma unroll
        for (int u = 0; u < GT; u++) {
            r3_v4d v = r3_combine(oo[u], *(const r3_v4d*)(p1[u] + s), *(const r3_v4d*)(p2[u] + s));
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const bool in = rok[u] && s + e < g.n;
                const double x = in ? v[e] : 0.0;
                v[e] = x;
                if (in) {
                    gmx[u] = fmax(gmx[u], fabs(x));
                    gmn[u] = fmin(gmn[u], fabs(x));
                }
                if (hk) v[e] = in ? r3_rcp(x) : 0.0;
            }
            A[u] = v;
            A2[u] = v * v;
        }
#pragma unroll
        for (int t = 0; t < TK; t++) {
            const r3_v4d b = *(const r3_v4d*)(bp + ((int64_t)t * g.NQ + 4 * m) * 64);
#pragma unroll
            for (int u = 0; u < GT; u++) {
                const r3_v4d a = t == TK - 1 ? A2[u] : A[u];
                acc[u][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, acc[u][t], 0, 0, 0);
                acc[u][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.y, acc[u][t], 0, 0, 0);
                acc[u][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.z, b.z, acc[u][t], 0, 0, 0);
                acc[u][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.w, b.w, acc[u][t], 0, 0, 0);
            }
        }
    }
    }
    // row ranges over the four sample groups of each row
#pragma unroll
    for (int u = 0; u < GT; u++) {
        gmx[u] = fmax(gmx[u], __shfl_xor(gmx[u], 16, 64));
        gmx[u] = fmax(gmx[u], __shfl_xor(gmx[u], 32, 64));
        gmn[u] = fmin(gmn[u], __shfl_xor(gmn[u], 16, 64));
        gmn[u] = fmin(gmn[u], __shfl_xor(gmn[u], 32, 64));
    }
    // this lane's column: D[i][j] sits in lane j + 16 (i mod 4), register i / 4
    const double nn = (double)g.n;
    unsigned cnt = 0;
    if (AS) {
        // column 15 holds the ones: sum g y_t, sum g, sum g^2 of each row; a
        // partner column holds sum x g.  The add / sub moments follow from
        // these and the partner's own sums:
        //   S1 = Sx +- Sg, S2 = Sx2 +- 2 Sxg + Sg2, P_t = Sxy_t +- Sgy_t.
        // Their rounding error is below 3.2 n u kappa' with kappa' =
        // (Sx2 + Sg2) / (S2 - S1^2/n), so kappa' <= KAPPA_MAX keeps every
        // score inside the selection margin; other pairs go to the fix-up.
        const int32_t cd = g.coldesc[ct * 16 + r16];
        const int p = cd & 0xFFFF;
        const bool colok = cd >= 0 && (cd >> 16) == 0 && g.valid[p];
        const int src = (lane & 48) | 15;
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int i = kq + 4 * r;
            double gs[TK];                             // sum g y_t, sum g, sum g^2 of row i
#pragma unroll
            for (int t = 0; t < TP; t++) gs[t] = __shfl(acc[0][0][r], (lane & 48) | t, 64);
            gs[TP] = __shfl(acc[0][TP][r], src, 64);
            gs[TP + 1] = __shfl(acc[0][TP + 1][r], src, 64);
            const bool ok = __shfl((int)rok[0], i, 64) != 0 && colok;
            if (!ok) continue;
            const double* pc = g.pconst + (int64_t)p * TK;
            const double Sxg = acc[0][TP][r];
            const double A = pc[TP + 1] + gs[TP + 1];
#pragma unroll
            for (int o = 0; o < 2; o++) {
                if (!((g.ops >> o) & 1u)) continue;
                const double sg = o == 0 ? 1.0 : -1.0;
                const int64_t id = slot3as(g.sm, OP_ADD + o, w, i, r16);   // score slot
                const double S1 = pc[TP] + sg * gs[TP];
                const double S2 = pc[TP + 1] + 2.0 * sg * Sxg + gs[TP + 1];
                const double varn = S2 - S1 * (S1 / nn);
                const double kappa = varn > 0.0 ? A / varn : INFINITY;
                if (!(S2 < INFINITY) || !(kappa <= R3_KAPPA_MAX) || S2 <= R3_TAU_CANCEL_FAST * A) {
                    const unsigned long long slot = r3_slot(g.fix_cnt);
                    if ((int64_t)slot < g.fix_cap) g.fix_ids[slot] = id;
                    continue;
                }
                const double isd = 1.0 / sqrt(varn);
                cnt++;
                if (g.mode == DISCOVER_SCORE_MAX) {
                    double best = 0.0;
#pragma unroll
                    for (int t = 0; t < TP; t++)
                        if (t < g.T) best = fmax(best, fabs((pc[t] + sg * gs[t] - S1 * (g.ysum[t] / nn)) * isd));
                    g.scores[id] = best;
                } else {
#pragma unroll
                    for (int t = 0; t < TP; t++)
                        if (t < g.T)
                            g.scores[(int64_t)t * g.N + id] = fabs((pc[t] + sg * gs[t] - S1 * (g.ysum[t] / nn)) * isd);
                }
            }
        }
    } else {
        const int32_t cd = g.coldesc[ct * 16 + r16];
        const int p = cd & 0xFFFF, kind = cd >> 16;
        const int op3 = kind == 0 ? OP_MUL : kind == 1 ? OP_RDIV : OP_DIV;
        const bool colok = cd >= 0 && ((g.ops >> (op3 - OP_ADD)) & 1u) && g.valid[p];
        const double xmx = colok ? g.pstat[p] : 0.0, xmn = colok ? g.pstat[g.pe + p] : 1.0;
    #pragma unroll
        for (int u = 0; u < GT; u++) {
    #pragma unroll
            for (int r = 0; r < 4; r++) {
                const int i = kq + 4 * r;                      // row of this register
                const bool ok = __shfl((int)rok[u], i, 64) != 0 && colok;
                const double rmx = __shfl(gmx[u], i, 64), rmn = __shfl(gmn[u], i, 64);
                if (!ok) continue;
                const int64_t id = slot3(g.sm, op3, (tile0 + u) * 16 + i, p);   // score slot
                // finiteness of the candidate's values
                bool sure = true;
                if (op3 == OP_MUL) {
                    sure = rmx * xmx < R3_BIG;
                } else if (op3 == OP_DIV) {
                    if (rmn == 0.0) continue;                  // x / 0: not finite
                    sure = rmn >= R3_TINY && xmx < R3_BIG * rmn;
                } else {
                    if (xmn == 0.0) continue;                  // g / 0: not finite
                    sure = xmn >= R3_TINY && rmx < R3_BIG * xmn;
                }
                const double S1 = acc[u][TP][r], S2 = acc[u][TP + 1][r];
                const double varn = S2 - S1 * (S1 / nn);
                const double kappa = varn > 0.0 ? S2 / varn : INFINITY;
                if (!sure || !(kappa <= R3_KAPPA_MAX)) {
                    const unsigned long long slot = r3_slot(g.fix_cnt);
                    if ((int64_t)slot < g.fix_cap) g.fix_ids[slot] = id;
                    continue;
                }
                const double isd = 1.0 / sqrt(varn);
                cnt++;
                if (g.mode == DISCOVER_SCORE_MAX) {
                    double best = 0.0;
    #pragma unroll
                    for (int t = 0; t < TP; t++)
                        if (t < g.T) best = fmax(best, fabs((acc[u][t][r] - S1 * (g.ysum[t] / nn)) * isd));
                    g.scores[id] = best;
                } else {
    #pragma unroll
                    for (int t = 0; t < TP; t++)
                        if (t < g.T)
                            g.scores[(int64_t)t * g.N + id] = fabs((acc[u][t][r] - S1 * (g.ysum[t] / nn)) * isd);
                }
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor((int)cnt, o, 64);
    if (lane == 0 && cnt) atomicAdd(g.nscored, (unsigned long long)cnt);
}

// ------------------------------------------------------------ precision form
// BF16 numerators, split-BF16 moments.  Per 32-sample chunk a lane
// regenerates 8 consecutive samples of its row (rows 16 rung-2 features, as
// above) in FP64 and rounds them to FP32 (a) and BF16 (a_h).  Every product
// is a v_mfma_f32_16x16x32_bf16 (lane l supplies row l%16 at samples
// 8(l/16)..+7 of the chunk and column l%16 at the same samples, and
// receives D[4(l/16)+e][l%16] in slot e): the T numerators against x y_t
// rounded to BF16, and the moments S1 = sum a x and S2 = sum a^2 x^2 each
// from three products of two-term splits a = a_h + a_l (a_h = BF16(a), a_l
// = BF16(a - a_h)): a_h x_h + (a_h x_l + a_l x_h), the cross terms in an
// accumulator of their own.
//
// Error: with u = 2^-8 (plus the FP64 -> FP32 -> BF16 double rounding) the
// product of two rounded values is within 2u + u^2 of the true product and
// the FP32 sum adds gamma_n, so |P_lp - P| <= delta ||f|| ||y_t|| and
// |r_lp - r| <= delta sqrt(kappa) with kappa = S2 / (S2 - S1^2/n): delta is
// the precision form's BF16 bound.  A split product misses a_l x_l and the
// splits' own rounding: within 3 2^-16 of a x (plus the FP32 roundings of a,
// x, a^2 and x^2, 8 v, v = 2^-24); the FP32 accumulation adds at most
// (n + 42) v of the summed magnitudes (at most 31 roundings inside one
// product's 32-term sum, one per accumulation).  So |dS1| <= e sqrt(n)
// ||f|| and |dS2| <= e S2 with e = (n + 50) v + 3 2^-16, the variance moves
// by at most 3 e kappa of itself and the score (targets centred, unit norm)
// by at most cm kappa with cm = 3 e (r3_moment_err); kappa itself is then
// known within a factor 1 +- 4/3 cm kappa, which the bound below absorbs.
// Scores with kappa <= LP_KAPPA are stored (error within the selection
// margin 1.1 delta + 1.5 cm); others store the upper bound -(s + delta
// sqrt(kappa)(1 + cm kappa) + 1.1 cm kappa) and are rescored exactly when
// they can reach the pool.  Rows or partners whose values leave a safe FP32
// range (products above LP_BIG, squares above LP_BIG2, a norm below
// LP_SMALL2 where subnormals would matter) or whose kappa makes cm kappa
// exceed 0.05 go to the exact fix-up.
constexpr double LP_BIG = 1e30;
constexpr double LP_BIG2 = 1e16;        // |f|, |g|, |x| below this: n f^2 stays finite in FP32
constexpr double LP_SMALL2 = 1e-10;     // ||f|| above this: FP32 subnormals are negligible
constexpr double LP_KAPPA = 1.21;

typedef __attribute__((ext_vector_type(8))) __bf16 r3_bf16x8;
typedef __attribute__((ext_vector_type(4))) float r3_f32x4;
typedef __attribute__((ext_vector_type(4))) unsigned r3_u32x4;

// Two FP32 values rounded to BF16 (nearest, ties to even: gfx950's packed
// conversion) and packed, lo in bits 0..15, hi in bits 16..31; the layout
// kernel and the screen round the same way.
__device__ __forceinline__ unsigned r3_bf16_pack(float lo, float hi) {
    typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
    bf2 v;
    v[0] = (__bf16)lo;
    v[1] = (__bf16)hi;
    return __builtin_bit_cast(unsigned, v);
}

// Two-term BF16 splits of two FP32 values: hi = their BF16 roundings
// (packed as r3_bf16_pack), lo = the BF16 roundings of the exact remainders
// v - hi.
__device__ __forceinline__ void r3_split(float v0, float v1, unsigned& hi, unsigned& lo) {
    hi = r3_bf16_pack(v0, v1);
    __asm__("" : "+v"(hi));              // (the compiler would otherwise convert v0 twice)
    const float h0 = __uint_as_float(hi << 16), h1 = __uint_as_float(hi & 0xFFFF0000u);
    lo = r3_bf16_pack(v0 - h0, v1 - h1);
}

// Right-hand operands of the precision form, per column tile c and 32-sample
// chunk ch (512 entries each, lane-major: entry 8 l + e belongs to column
// l%16 at sample 32 ch + 8 (l/16) + e): b32[(c NC + ch) 512 + 8 l + e] =
// FP32(x), blp[((c TP + t) NC + ch) 512 + 8 l + e] = BF16(x y_t).
__global__ __launch_bounds__(256) void k_r3_bmat_lp(int n, int64_t ldn, int TP, int NC, int nct,
                                                    const int32_t* __restrict__ coldesc,
                                                    const double* __restrict__ Vf, const double* __restrict__ Rf,
                                                    const double* __restrict__ Yn, float* __restrict__ b32,
                                                    __bf16* __restrict__ blp) {
    const int64_t per = (int64_t)NC * 512;
    const int64_t total = (int64_t)nct * (1 + TP) * per;
    for (int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x; f < total; f += (int64_t)gridDim.x * 256) {
        const int64_t r = f % per, ck = f / per;
        const int c = (int)(ck / (1 + TP)), v = (int)(ck % (1 + TP));
        const int ch = (int)(r / 512), w = (int)(r % 512);
        const int l = w >> 3, e = w & 7;
        const int j = l & 15, s = 32 * ch + 8 * (l >> 4) + e;
        const int32_t d = coldesc[c * 16 + j];
        double x = 0.0;
        if (d >= 0 && s < n) {
            const int p = d & 0xFFFF, kind = d >> 16;
            x = kind == 3 ? 1.0 : kind == 1 ? Rf[(int64_t)p * ldn + s] : Vf[(int64_t)p * ldn + s];
        }
        if (v == 0) {
            b32[(int64_t)c * per + r] = (float)x;
        } else {
            const int t = v - 1;
            const double yv = (s < n) ? Yn[(int64_t)t * ldn + s] : 0.0;
            const unsigned pk = r3_bf16_pack((float)(x * yv), 0.0f);
            blp[((int64_t)c * TP + t) * per + r] = __builtin_bit_cast(__bf16, (unsigned short)(pk & 0xFFFFu));
        }
    }
}

struct R3lpArgs {
    R3mArgs m;
    const float* b32;
    const __bf16* blp;
    const double* r2q;        // mean square of each rung-2 feature (by id - off[2])
    int NC;
    int ct0, ct1;             // column tiles of the launch
    double delta;
    double cm;                // FP32-moment error coefficient (r3_moment_err)
};

typedef float r3_f32x2 __attribute__((ext_vector_type(2)));

// A block's four waves take four row tiles (16 rung-2 features each)
// against CT column tiles (16 partner columns each): a wave regenerates its
// row values once per chunk and issues the products of every column tile
// from them.  The column tiles' operands of a chunk (x, x^2 and the TP
// products x y_t: 4 + TP KB per tile) are staged once per block in LDS,
// double-buffered, and each wave reads them there (16 contiguous bytes per
// lane per read).  The next chunk's operands are loaded into registers (a
// share of 8 + 16 TP/4 bytes per tile per thread) and the next chunk's row
// operands per wave while the current chunk's products are issued.
// HK: the launch's column tiles multiply 1/g (div), else g (mul, rdiv);
// the two kinds are separate launches, so that neither carries the
// other's per-sample work.  Column tiles past the launch's range (the last
// group may be short) repeat its last tile and store nothing.
template <int TP, int CT, bool HK>
__global__ __launch_bounds__(256, (TP * CT <= 16 ? 2 : 1)) void k_r3_lp(R3lpArgs a) {
    const R3mArgs& g = a.m;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int r16 = lane & 15, kq = lane >> 4;
    const int lb = r3_xcd_block();
    const int cb = lb / g.n_gblk;
    const int ctb = a.ct0 + cb * CT;                     // first column tile of the block
    const int64_t tile0 = (int64_t)(lb - cb * g.n_gblk) * 4 + r3_wave();
    // a wave without a row tile still stages its share and meets every barrier
    const bool active = tile0 * 16 < g.n_grec;
    constexpr bool hk = HK;
    bool rok;
    int64_t j2;
    int oo;
    const double* p1;
    const double* p2;
    {
        const int64_t t16 = min(tile0, (g.n_grec >> 4) - 1) * 16;
        const int64_t rec = tile0 * 16 + r16;
        int k = -2, l = 0, op2;
        r3_rec(g.grec[rec < g.n_grec ? rec : t16], k, l, op2);
        op2 = __builtin_amdgcn_readfirstlane(op2);
        oo = op2;
        rok = rec < g.n_grec && k != -2;
        j2 = rok ? r3_j2(g.sd, g.mat_raw, k, l, op2) : 0;
        rok = rok && g.r2v[j2 - g.sd.off[2]];
        r3_rows(g.Vf, g.Rf, g.ldn, op2 < OP_ADD ? -1 : (rok ? k : 0), rok ? l : 0, op2, p1, p2);
    }
    r3_f32x4 s1[CT], s2[CT], c1[CT], c2[CT];              // moments: a_h x_h and cross terms
    r3_f32x4 pa[CT][TP];
    double hmx = 0.0;                                    // div tiles: max |1/g| of the lane's samples
#pragma unroll
    for (int c = 0; c < CT; c++) {
        s1[c] = r3_f32x4{0.f, 0.f, 0.f, 0.f};
        s2[c] = r3_f32x4{0.f, 0.f, 0.f, 0.f};
        c1[c] = r3_f32x4{0.f, 0.f, 0.f, 0.f};
        c2[c] = r3_f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < TP; t++) pa[c][t] = r3_f32x4{0.f, 0.f, 0.f, 0.f};
    }
    // LDS buffer: per column tile the splits x_h, x_l, (x^2)_h, (x^2)_l
    // (512 BF16 each), then the TP x y_t blocks (512 BF16 each), all
    // lane-major as in b32 and blp
    constexpr int TB = (4 + TP) * 1024;
    constexpr int BUF = CT * TB;
    __shared__ __attribute__((aligned(16))) char smem[2 * BUF];
    constexpr int NPB = (TP * 64 + 255) / 256;           // 16-byte pieces of x y_t per thread and tile
    const float* gx[CT];
    const __bf16* gb[CT];
#pragma unroll
    for (int c = 0; c < CT; c++) {
        const int ctc = min(ctb + c, a.ct1 - 1);
        gx[c] = a.b32 + (int64_t)ctc * a.NC * 512;
        gb[c] = a.blp + (int64_t)ctc * TP * a.NC * 512;
    }
    r3_f32x2 sx[CT];
    r3_u32x4 sb[CT][NPB];
    // piece i of thread tid: q = tid + 256 i (with fewer than 256 pieces,
    // threads share pieces and write the same bytes); every thread loads and
    // stores on every chunk, so that no load sits behind a branch
    auto piece = [&](int i) { return TP * 64 >= 256 ? tid + 256 * i : (tid & (TP * 64 - 1)); };
    auto stage_load = [&](int ch) {
#pragma unroll
        for (int c = 0; c < CT; c++) {
            sx[c] = *(const r3_f32x2*)(gx[c] + (int64_t)ch * 512 + 2 * tid);
#pragma unroll
            for (int i = 0; i < NPB; i++) {
                const int q = piece(i);
                sb[c][i] = *(const r3_u32x4*)(gb[c] + ((int64_t)(q >> 6) * a.NC + ch) * 512 + (q & 63) * 8);
            }
        }
    };
    auto stage_store = [&](int buf) {
#pragma unroll
        for (int c = 0; c < CT; c++) {
            // thread tid holds entries 2 tid, 2 tid + 1: one 4-byte BF16 pair
            // per split
            char* xs = smem + buf * BUF + c * TB + 4 * tid;
            const float x0 = sx[c].x, x1 = sx[c].y;
            const float q0 = x0 * x0, q1 = x1 * x1;
            unsigned hi, lo;
            r3_split(x0, x1, hi, lo);
            *(unsigned*)xs = hi;
            *(unsigned*)(xs + 1024) = lo;
            r3_split(q0, q1, hi, lo);
            *(unsigned*)(xs + 2048) = hi;
            *(unsigned*)(xs + 3072) = lo;
            char* bs = smem + buf * BUF + c * TB + 4096;
#pragma unroll
            for (int i = 0; i < NPB; i++) {
                const int q = piece(i);
                *(r3_u32x4*)(bs + (q >> 6) * 1024 + (q & 63) * 16) = sb[c][i];
            }
        }
    };
    // row operands of chunk ch: 8 samples of two operand rows
    struct Ld {
        r3_v4d x1[2], x2[2];
    };
    auto load_rows = [&](int ch, Ld& L) {
        const int s = 32 * ch + 8 * kq;
#pragma unroll
        for (int h = 0; h < 2; h++) {
            L.x1[h] = *(const r3_v4d*)(p1 + s + 4 * h);
            L.x2[h] = *(const r3_v4d*)(p2 + s + 4 * h);
        }
    };
    Ld cur, nxt;
    stage_load(0);
    load_rows(0, cur);
    stage_store(0);
    __syncthreads();
    // Only the last chunk holds samples >= n: there the row values are set
    // to 0 (the right-hand operands are 0 too, but a row value there may be
    // inf or NaN).  A row whose feature is invalid only reaches its own row
    // of the products, whose scores are never stored, so it is not masked.
    // The products of chunk ch from buffer ch & 1 and the rows in cur; the
    // last chunk (samples >= n masked) runs after the loop as a copy of its
    // own, so that no other chunk carries the mask.
    auto chunk = [&](int ch, auto tail_c) {
        constexpr bool tail = decltype(tail_c)::value;
        const int s = 32 * ch + 8 * kq;
        double v[8];
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const r3_v4d w = r3_combine(oo, cur.x1[h], cur.x2[h]);
#pragma unroll
            for (int e = 0; e < 4; e++) v[4 * h + e] = w[e];
        }
        float vf[8];
#pragma unroll
        for (int e = 0; e < 8; e++) {
            double x = v[e];
            if (hk) x = r3_rcp(x);
            if (tail && s + e >= g.n) x = 0.0;
            if (hk) hmx = fabs(x) > hmx ? fabs(x) : hmx;   // NaN leaves it unchanged
            // FP64 -> FP32 here and FP32 -> BF16 in the pack: two
            // hardware roundings (the error bound counts both); the
            // empty asm keeps the compiler from fusing them into one
            // correctly rounded (and much longer) conversion
            vf[e] = (float)x;
            __asm__("" : "+v"(vf[e]));
        }
        // av = a_h (also the numerators' operand), al = a_l, qh / ql:
        // the splits of a^2
        r3_u32x4 ah, al, qh, ql;
#pragma unroll
        for (int e = 0; e < 4; e++) {
            unsigned h, l;
            r3_split(vf[2 * e], vf[2 * e + 1], h, l);
            ah[e] = h;
            al[e] = l;
            r3_split(vf[2 * e] * vf[2 * e], vf[2 * e + 1] * vf[2 * e + 1], h, l);
            qh[e] = h;
            ql[e] = l;
        }
        const r3_bf16x8 av = __builtin_bit_cast(r3_bf16x8, ah);
        const r3_bf16x8 avl = __builtin_bit_cast(r3_bf16x8, al);
        const r3_bf16x8 aq = __builtin_bit_cast(r3_bf16x8, qh);
        const r3_bf16x8 aql = __builtin_bit_cast(r3_bf16x8, ql);
#pragma unroll
        for (int c = 0; c < CT; c++) {
            const char* xs = smem + (ch & 1) * BUF + c * TB + 16 * lane;
            const char* bs = smem + (ch & 1) * BUF + c * TB + 4096;
            const r3_bf16x8 xh = *(const r3_bf16x8*)xs, xl = *(const r3_bf16x8*)(xs + 1024);
            const r3_bf16x8 x2h = *(const r3_bf16x8*)(xs + 2048), x2l = *(const r3_bf16x8*)(xs + 3072);
            s1[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, xh, s1[c], 0, 0, 0);
            s2[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aq, x2h, s2[c], 0, 0, 0);
            c1[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, xl, c1[c], 0, 0, 0);
            c2[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aq, x2l, c2[c], 0, 0, 0);
            c1[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(avl, xh, c1[c], 0, 0, 0);
            c2[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aql, x2h, c2[c], 0, 0, 0);
#pragma unroll
            for (int t = 0; t < TP; t++) {
                const r3_bf16x8 bv = *(const r3_bf16x8*)(bs + t * 1024 + lane * 16);
                pa[c][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, pa[c][t], 0, 0, 0);
            }
        }
    };
    for (int ch = 0; ch + 1 < a.NC; ch++) {
        stage_load(ch + 1);
        load_rows(ch + 1, nxt);
        if (active) chunk(ch, std::false_type{});
        stage_store((ch + 1) & 1);
        __syncthreads();
        cur = nxt;
    }
    if (active) chunk(a.NC - 1, std::true_type{});
    if (!active) return;
    if (hk) {
        hmx = fmax(hmx, __shfl_xor(hmx, 16, 64));
        hmx = fmax(hmx, __shfl_xor(hmx, 32, 64));
    }
    const double nn = (double)g.n;
    unsigned cnt = 0;
#pragma unroll
    for (int c = 0; c < CT; c++) {
        if (ctb + c >= a.ct1) continue;                  // repeated tile: stores nothing
        const int ct = ctb + c;
        const int32_t cd = g.coldesc[ct * 16 + r16];
        const int p = cd & 0xFFFF, kind = cd >> 16;
        const int op3 = kind == 0 ? OP_MUL : kind == 1 ? OP_RDIV : OP_DIV;
        const bool colok = cd >= 0 && ((g.ops >> (op3 - OP_ADD)) & 1u) && g.valid[p];
        const double xmx = colok ? g.pstat[p] : 0.0, xmn = colok ? g.pstat[g.pe + p] : 1.0;
        double S1[4], S2[4];                             // row 4 kq + e in slot e
#pragma unroll
        for (int e = 0; e < 4; e++) {
            S1[e] = (double)s1[c][e] + (double)c1[c][e];
            S2[e] = (double)s2[c][e] + (double)c2[c][e];
        }
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int i = 4 * kq + e;                      // row of slot e
            const bool ok = __shfl((int)rok, i, 64) != 0 && colok;
            const int64_t gj = __shfl(j2, i, 64);
            const double hx = hk ? __shfl(hmx, i, 64) : 0.0;
            if (!ok) continue;
            // max |g| <= sqrt(sum g^2) = sqrt(n E[g^2]) (E[g^2] recorded by the
            // rung-2 screen; 1 % margin for its rounding): only compared with
            // range limits many orders of magnitude away; min |g| = 1 / max
            // |1/g| (div tiles only)
            const double rmx = sqrt(nn * a.r2q[gj - g.sd.off[2]]) * 1.01;
            const double rmn = hk ? 1.0 / hx : 0.0;
            const int64_t id = slot3(g.sm, op3, tile0 * 16 + i, p);   // score slot
            bool sure;
            double amx, fmx, bmx;                          // largest |A|, |f|, |B| of the products
            if (op3 == OP_MUL) {
                sure = rmx * xmx < R3_BIG;
                amx = rmx; fmx = rmx * xmx; bmx = xmx;
            } else if (op3 == OP_DIV) {
                if (rmn == 0.0) continue;                  // x / 0: not finite
                sure = rmn >= R3_TINY && xmx < R3_BIG * rmn;
                amx = 1.0 / rmn; fmx = xmx / rmn; bmx = xmx;
            } else {
                if (xmn == 0.0) continue;                  // g / 0: not finite
                sure = xmn >= R3_TINY && rmx < R3_BIG * xmn;
                amx = rmx; fmx = rmx / xmn; bmx = 1.0 / xmn;
            }
            const double varn = S2[e] - S1[e] * (S1[e] / nn);
            const double kappa = varn > 0.0 ? S2[e] / varn : INFINITY;
            const bool lp_ok = amx < LP_BIG2 && fmx < LP_BIG2 && bmx < LP_BIG2 &&
                               S2[e] > LP_SMALL2 * LP_SMALL2 && a.cm * kappa <= 0.05;
            if (!sure || !lp_ok || !(kappa <= R3_KAPPA_MAX)) {
                const unsigned long long slot = r3_slot(g.fix_cnt);
                if ((int64_t)slot < g.fix_cap) g.fix_ids[slot] = id;
                continue;
            }
            const double isd = 1.0 / sqrt(varn);
            const bool precise = kappa <= LP_KAPPA;
            const double ub = a.delta * sqrt(kappa) * (1.0 + a.cm * kappa) + 1.1 * a.cm * kappa;
            cnt++;
            if (g.mode == DISCOVER_SCORE_MAX) {
                double best = 0.0;
#pragma unroll
                for (int t = 0; t < TP; t++)
                    if (t < g.T) best = fmax(best, fabs(((double)pa[c][t][e] - S1[e] * (g.ysum[t] / nn)) * isd));
                g.scores[id] = precise ? best : -(best + ub);
            } else {
#pragma unroll
                for (int t = 0; t < TP; t++)
                    if (t < g.T) {
                        const double r = fabs(((double)pa[c][t][e] - S1[e] * (g.ysum[t] / nn)) * isd);
                        g.scores[(int64_t)t * g.N + id] = precise ? r : -(r + ub);
                    }
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor((int)cnt, o, 64);
    if (lane == 0 && cnt) atomicAdd(g.nscored, (unsigned long long)cnt);
}

// One launch over the mul / rdiv column tiles [0, n_gct), one over the div
// tiles [n_gct, nct); each in groups of CT tiles per block.
template <int TP, int CT, bool HK>
void launch_lp_range(R3lpArgs l, int ct0, int ct1, hipStream_t st) {
    if (ct1 <= ct0) return;
    l.ct0 = ct0;
    l.ct1 = ct1;
    const int64_t groups = (ct1 - ct0 + CT - 1) / CT;
    DSC_REQUIRE((int64_t)l.m.n_gblk * groups < ((int64_t)1 << 31), "rung-3 grid too large");
    k_r3_lp<TP, CT, HK><<<(unsigned)((int64_t)l.m.n_gblk * groups), 256, 0, st>>>(l);
}

// Column tiles per wave: up to 3 at <= 4 targets and 2 at 8 (3 tiles at 8
// targets hold 266 VGPRs, one wave per SIMD; measured on gfx950 at 8
// targets: 2 tiles 19.3 ms, 3 tiles 22.8 ms per dimension of the large
// workload), as many as the range holds; the rest in smaller groups.
template <int TP>
void launch_lp(R3lpArgs l, int n_gct, int nct, int64_t n_grec, hipStream_t st) {
    l.m.n_gblk = (int)((n_grec / 16 + 3) / 4);
    constexpr int CMAX = TP <= 4 ? 3 : TP <= 8 ? 2 : 1;
    auto range = [&](int c0, int c1, auto hk) {
        constexpr bool HK = decltype(hk)::value;
        int c = c0;
        if constexpr (CMAX >= 3) {
            const int m = (c1 - c) / 3 * 3;
            launch_lp_range<TP, 3, HK>(l, c, c + m, st);
            c += m;
        }
        if constexpr (CMAX >= 2) {
            const int m = (c1 - c) / 2 * 2;
            launch_lp_range<TP, 2, HK>(l, c, c + m, st);
            c += m;
        }
        launch_lp_range<TP, 1, HK>(l, c, c1, st);
    };
    range(0, n_gct, std::false_type{});
    range(n_gct, nct, std::true_type{});
}

template <class T>
T* r3_up(R3Plan& P, const std::vector<T>& v) {
    void* p = nullptr;
    const size_t bytes = std::max<size_t>(v.size() * sizeof(T), 16);
    if (hipMalloc(&p, bytes) != hipSuccess) DSC_FAIL(DISCOVER_E_NOMEM, "rung-3 plan allocation failed");
    P.allocs.push_back(p);
    if (!v.empty()) DSC_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return (T*)p;
}

template <int TP, int GT>
void launch_mm(R3mArgs a, int nct, hipStream_t st) {
    const int64_t ntl = (a.n_grec + 15) / 16;
    a.n_gblk = (int)((ntl + 4 * GT - 1) / (4 * GT));
    const int64_t blocks = (int64_t)a.n_gblk * nct;
    DSC_REQUIRE(blocks < ((int64_t)1 << 31), "rung-3 grid too large");
    k_r3_mm<TP, GT, false><<<(unsigned)blocks, 256, 0, st>>>(a);
}

template <int TP>
void launch_as(const R3mArgs& a, hipStream_t st) {
    const int64_t blocks = (a.n_work + 3) / 4;
    DSC_REQUIRE(blocks < ((int64_t)1 << 31), "rung-3 add/sub grid too large");
    k_r3_mm<TP, 1, true><<<(unsigned)blocks, 256, 0, st>>>(a);
}

}  // namespace

std::shared_ptr<R3Plan> build_r3_plan(const Space& sp, uint32_t r3_ops) {
    auto P = std::make_shared<R3Plan>();
    const SpaceDev& d = sp.d;
    const int B = sp.B, Bq = B > 0 ? B : 1;
    P->ops = r3_ops;
    P->pe = sp.rung_start[d.pool[3] + 1];
    DSC_REQUIRE(P->pe < 65536, "rung-3 partner pool too large");
    const int32_t c0 = sp.rung_start[1], c1 = sp.rung_start[2];
    DSC_REQUIRE(c1 < (1 << 28), "rung-1 operand count too large");
    const int pool2 = d.pool[2];
    const bool addsub = (r3_ops & 3u) != 0;
    // every unit-legal rung-2 feature with its unit vector (unary operators
    // in ID order, binary ones in windows of operands, below)
    std::vector<int2> rec;
    std::vector<int32_t> gunit;
    std::vector<int32_t> u2(Bq, 0);
    auto push = [&](int k, int l, int o) {
        rec.push_back(make_int2(k, l | (o << 28)));
        if (addsub) gunit.insert(gunit.end(), u2.begin(), u2.end());
    };
    // each operator's run is padded to a multiple of 16 records (k = -2:
    // no feature), so that the rows of a 16-row tile share one operator
    auto pad16 = [&](int o) {
        while (rec.size() % 16) {
            rec.push_back(make_int2(-2, o << 28));
            if (addsub) gunit.insert(gunit.end(), Bq, INT32_MIN);
        }
    };
    for (int o = 0; o < OP_ADD; o++) {
        if (d.block[2][o] < 0) continue;
        for (int32_t l = c0; l < c1; l++)
            if (unit_rule(o, B, &sp.mat_unit[(size_t)l * Bq], nullptr, u2.data())) push(-1, l, o);
        pad16(o);
    }
    // binary records in windows of R3_SW operands l by R3_SW operands k: the
    // tiles of a window need 2 R3_SW operand rows, which stay in L2 while
    // its tiles run (the kernels keep neighbouring blocks on one XCD)
    constexpr int32_t R3_SW = 64;
    const int32_t kend = pool2 == 1 ? c1 : sp.rung_start[pool2 + 1];
    for (int o = OP_ADD; o <= OP_RDIV; o++) {
        if (d.block[2][o] < 0) continue;
        for (int32_t l0 = c0; l0 < c1; l0 += R3_SW)
            for (int32_t k0 = 0; k0 < kend; k0 += R3_SW)
                for (int32_t l = l0; l < std::min(l0 + R3_SW, c1); l++) {
                    const int32_t kmax = std::min(pool2 == 1 ? l : sp.rung_start[pool2 + 1], k0 + R3_SW);
                    for (int32_t k = k0; k < kmax; k++)
                        if (unit_rule(o, B, &sp.mat_unit[(size_t)k * Bq], &sp.mat_unit[(size_t)l * Bq], u2.data()))
                            push(k, l, o);
                }
        pad16(o);
    }
    P->n_grec = (int64_t)rec.size();
    DSC_REQUIRE(P->n_grec < ((int64_t)1 << 31), "rung-3 record list too large");
    // partner column tiles: per group of 8 partners, 8 mul then 8 rdiv
    // columns (both against g); then the div columns (against 1/g)
    const bool mul = (r3_ops >> (OP_MUL - OP_ADD)) & 1u, div = (r3_ops >> (OP_DIV - OP_ADD)) & 1u,
               rdiv = (r3_ops >> (OP_RDIV - OP_ADD)) & 1u;
    std::vector<int32_t> cols;
    for (int g8 = 0; g8 < (P->pe + 7) / 8; g8++)
        for (int kind = 0; kind < 2; kind++) {
            if (kind == 0 ? !mul : !rdiv) continue;
            for (int q = 0; q < 8; q++) {
                const int p = 8 * g8 + q;
                cols.push_back(p < P->pe ? (p | (kind << 16)) : -1);
            }
        }
    while (cols.size() % 16) cols.push_back(-1);
    P->n_gct = (int)(cols.size() / 16);
    if (div) {
        for (int p = 0; p < P->pe; p++) cols.push_back(p | (2 << 16));
        while (cols.size() % 16) cols.push_back(-1);
    }
    P->n_ctiles = (int)(cols.size() / 16);
    P->h_coldesc = cols;
    if (P->n_grec) P->grec = r3_up(*P, rec);            // also what the score slots decode
    if (P->n_grec && P->n_ctiles) P->coldesc = r3_up(*P, cols);
    // add / sub: records grouped by unit vector and operator, against
    // column tiles of the partners with the same unit vector (15 at most)
    // and a column of ones
    if (addsub && P->n_grec) {
        auto key = [&](const int32_t* u) { return std::string((const char*)u, sizeof(int32_t) * Bq); };
        std::map<std::string, std::vector<int32_t>> pg;
        for (int p = 0; p < P->pe; p++) pg[key(&sp.mat_unit[(size_t)p * Bq])].push_back(p);
        std::map<std::string, std::map<int, std::vector<int64_t>>> byk;
        for (int64_t r = 0; r < P->n_grec; r++) {
            if (rec[r].x == -2) continue;
            const std::string kk = B > 0 ? key(&gunit[(size_t)r * Bq]) : key(u2.data());
            if (pg.count(kk)) byk[kk][(int)((unsigned)rec[r].y >> 28)].push_back(r);
        }
        std::vector<int2> arec, work;
        std::vector<int32_t> acols;
        for (auto& e : byk) {
            const std::vector<int32_t>& pl = pg[e.first];
            const int ct0 = (int)(acols.size() / 16);
            for (size_t q = 0; q < pl.size(); q += 15) {
                for (size_t z = 0; z < 15; z++) acols.push_back(q + z < pl.size() ? pl[q + z] : -1);
                acols.push_back(3 << 16);                        // the ones
            }
            const int ct1 = (int)(acols.size() / 16);
            for (auto& ro : e.second) {
                const int64_t rt0 = (int64_t)arec.size() / 16;
                for (int64_t r : ro.second) arec.push_back(rec[r]);
                while (arec.size() % 16) arec.push_back(make_int2(-2, ro.first << 28));
                const int64_t rt1 = (int64_t)arec.size() / 16;
                for (int64_t rt = rt0; rt < rt1; rt++)
                    for (int c = ct0; c < ct1; c++) work.push_back(make_int2((int)rt, c));
            }
        }
        DSC_REQUIRE(arec.size() < ((size_t)1 << 35), "rung-3 add/sub list too large");
        P->n_as_grec = (int64_t)arec.size();
        P->n_as_ctiles = (int)(acols.size() / 16);
        P->n_as_work = (int64_t)work.size();
        if (P->n_as_work) {
            P->as_grec = r3_up(*P, arec);
            P->as_coldesc = r3_up(*P, acols);
            P->as_work = r3_up(*P, work);
        }
    }
    return P;
}

void launch_r3(discover_ctx* ctx, const R3Launch& a, hipStream_t st) {
    const R3Plan& P = *a.plan;
    const int NQ = r3_quads(a.n);
    if (P.n_grec && P.n_ctiles && a.precision == DISCOVER_BF16_GUARD) {
        k_r3_pstat<<<(unsigned)P.pe, 256, 0, st>>>(a.n, a.ldn, P.pe, a.Vf, a.pstat);
        check_launch("k_r3_pstat");
        const int NC = r3_chunks(a.n);
        float* b32 = (float*)a.bmat;
        __bf16* blp = (__bf16*)(b32 + (size_t)P.n_ctiles * NC * 512);
        const int64_t tot = (int64_t)P.n_ctiles * (a.TP + 1) * NC * 512;
        k_r3_bmat_lp<<<(unsigned)std::min<int64_t>(cdiv(tot, 256), 16384), 256, 0, st>>>(
            a.n, a.ldn, a.TP, NC, P.n_ctiles, P.coldesc, a.Vf, a.Rf, a.Yn, b32, blp);
        check_launch("k_r3_bmat_lp");
        R3lpArgs l{};
        R3mArgs& m = l.m;
        m.grec = P.grec; m.n_grec = P.n_grec; m.coldesc = P.coldesc; m.n_gct = P.n_gct;
        m.NQ = NQ; m.n = a.n; m.T = a.T; m.mode = a.mode; m.ldn = a.ldn; m.bmat = a.bmat;
        m.Vf = a.Vf; m.Rf = a.Rf; m.pstat = a.pstat; m.pe = P.pe; m.ops = P.ops;
        m.valid = a.valid; m.mat_raw = a.mat_raw; m.r2v = a.r2v; m.ysum = a.ysum; m.sd = a.sd;
        m.sm = a.sm; m.N = a.N; m.scores = a.scores; m.nscored = a.nscored; m.fix_ids = a.fix_ids;
        m.fix_cnt = a.fix_cnt; m.fix_cap = a.fix_cap;
        l.b32 = b32; l.blp = blp; l.r2q = a.r2q; l.NC = NC; l.delta = a.delta; l.cm = r3_moment_err(a.n);
        KTimer kt(ctx, st, "screen_r3");
        switch (a.TP) {
        case 1: launch_lp<1>(l, P.n_gct, P.n_ctiles, P.n_grec, st); break;
        case 2: launch_lp<2>(l, P.n_gct, P.n_ctiles, P.n_grec, st); break;
        case 4: launch_lp<4>(l, P.n_gct, P.n_ctiles, P.n_grec, st); break;
        case 8: launch_lp<8>(l, P.n_gct, P.n_ctiles, P.n_grec, st); break;
        default: launch_lp<16>(l, P.n_gct, P.n_ctiles, P.n_grec, st); break;
        }
        check_launch("k_r3_lp");
    } else if (P.n_grec && P.n_ctiles) {
        k_r3_pstat<<<(unsigned)P.pe, 256, 0, st>>>(a.n, a.ldn, P.pe, a.Vf, a.pstat);
        check_launch("k_r3_pstat");
        const int64_t tot = (int64_t)P.n_ctiles * (a.TP + 2) * NQ * 64;
        k_r3_bmat<<<(unsigned)std::min<int64_t>(cdiv(tot, 256), 16384), 256, 0, st>>>(
            a.n, a.ldn, a.TP, NQ, P.n_ctiles, P.coldesc, a.Vf, a.Rf, a.Yn, a.bmat);
        check_launch("k_r3_bmat");
        R3mArgs m{};
        m.grec = P.grec; m.n_grec = P.n_grec; m.coldesc = P.coldesc; m.n_gct = P.n_gct;
        m.NQ = NQ; m.n = a.n; m.T = a.T; m.mode = a.mode; m.ldn = a.ldn; m.bmat = a.bmat;
        m.Vf = a.Vf; m.Rf = a.Rf; m.pstat = a.pstat; m.pe = P.pe; m.ops = P.ops;
        m.valid = a.valid; m.mat_raw = a.mat_raw; m.r2v = a.r2v; m.ysum = a.ysum; m.sd = a.sd;
        m.sm = a.sm; m.N = a.N; m.scores = a.scores; m.nscored = a.nscored; m.fix_ids = a.fix_ids;
        m.fix_cnt = a.fix_cnt; m.fix_cap = a.fix_cap;
        KTimer kt(ctx, st, "screen_r3");
        switch (a.TP) {
        // row tiles per wave: as many as keep two or three waves per SIMD
        // with the accumulators in VGPRs (measured on gfx950: one tile per
        // wave at 8 targets beats two tiles at one wave per SIMD)
        case 1: launch_mm<1, 2>(m, P.n_ctiles, st); break;
        case 2: launch_mm<2, 2>(m, P.n_ctiles, st); break;
        case 4: launch_mm<4, 1>(m, P.n_ctiles, st); break;
        case 8: launch_mm<8, 1>(m, P.n_ctiles, st); break;
        default: launch_mm<16, 1>(m, P.n_ctiles, st); break;
        }
        check_launch("k_r3_mm");
    }
    if (P.n_as_work) {
        double* bm = (double*)((char*)a.bmat + r3_as_offset(P, a.TP, a.n));
        double* pc = a.pstat + 2 * P.pe;
        k_r3_pconst<<<(unsigned)P.pe, 256, 0, st>>>(a.n, a.ldn, a.TP, a.Vf, a.Yn, pc);
        check_launch("k_r3_pconst");
        const int64_t tot = (int64_t)P.n_as_ctiles * (a.TP + 2) * NQ * 64;
        k_r3_bmat<<<(unsigned)std::min<int64_t>(cdiv(tot, 256), 16384), 256, 0, st>>>(
            a.n, a.ldn, a.TP, NQ, P.n_as_ctiles, P.as_coldesc, a.Vf, a.Rf, a.Yn, bm);
        check_launch("k_r3_bmat");
        double* yb = (double*)((char*)a.bmat + r3_asy_offset(P, a.TP, a.n));
        k_r3_ybmat<<<(unsigned)std::min<int64_t>(cdiv((int64_t)NQ * 64, 256), 4096), 256, 0, st>>>(
            a.n, a.ldn, a.TP, NQ, a.Yn, yb);
        check_launch("k_r3_ybmat");
        R3mArgs m{};
        m.grec = P.as_grec; m.n_grec = P.n_as_grec; m.work = P.as_work; m.n_work = P.n_as_work;
        m.pconst = pc; m.coldesc = P.as_coldesc; m.n_gct = 0; m.ybmat = yb;
        m.NQ = NQ; m.n = a.n; m.T = a.T; m.mode = a.mode; m.ldn = a.ldn; m.bmat = bm;
        m.Vf = a.Vf; m.Rf = a.Rf; m.pstat = a.pstat; m.pe = P.pe; m.ops = P.ops;
        m.valid = a.valid; m.mat_raw = a.mat_raw; m.r2v = a.r2v; m.ysum = a.ysum; m.sd = a.sd;
        m.sm = a.sm; m.N = a.N; m.scores = a.scores; m.nscored = a.nscored; m.fix_ids = a.fix_ids;
        m.fix_cnt = a.fix_cnt; m.fix_cap = a.fix_cap;
        KTimer kt(ctx, st, "screen_r3_addsub");
        switch (a.TP) {
        case 1: launch_as<1>(m, st); break;
        case 2: launch_as<2>(m, st); break;
        case 4: launch_as<4>(m, st); break;
        case 8: launch_as<8>(m, st); break;
        default: launch_as<16>(m, st); break;
        }
        check_launch("k_r3_mm(add/sub)");
    }
}

R3Plan::~R3Plan() {
    for (void* p : allocs)
        if (hipFree(p) != hipSuccess) { /* nothing to do */ }
}

}  // namespace dsc
