// Sparsifying step on gfx950: exhaustive L0 over all D-subsets of a
// subspace (Eq. (1), Core Optimization Objective, with an intercept) and
// orthogonal matching pursuit (cited OMP, Software Description).
//
// L0 plan per problem:
//   1. Z = centered, unit-norm rows of F and of y (row S) -> Gram G = Z Z^T
//      ((S+1) x (S+1) FP64; G[a][S] is the correlation of row a with y).
//   2. Sweep: every D-subset's explained fraction q = c^T C^{-1} c from G by
//      per-lane Schur/Cholesky updates (D = 3: one wave per (a, 64 c's),
//      looping over b; uniform per-(a, b) factors staged in LDS).  Each wave
//      keeps only its best q (b packed into the low mantissa bits).
//   3. thr = m-th largest wave best - DELTA; waves whose best reaches thr
//      are swept again and every subset with q >= thr is collected.
//   4. The collected band is refitted by FP64 Householder QR on the raw
//      data (one workgroup per subset) and ranked by RSS with the tie rule.
#include "dsc_internal.h"
#include "dsc_select.h"

#include <algorithm>

namespace dsc {

constexpr double SW3_RCP_DELTA = 4.76837158203125e-7;  // 2^-21: D = 3 sweep values use a bare rcp

// ------------------------------------------------------------------ prep
// One wave per row (rows 0..S-1 of F, row S = y): Z = (f - mean) / ||f - mean||,
// and when nrm is given, nrm[row] = |Z row|^2 for the rows of F (0 for a
// constant row).
__device__ __forceinline__ void d_l0_prep(int n, int S, const double* __restrict__ F,
                                                 int64_t ldf, const double* __restrict__ y,
                                                 int ldz, double* __restrict__ Z,
                                                 double* __restrict__ yy,
                                                 double* __restrict__ nrm = nullptr) {
    const int row = blockIdx.x * 4 + wave_id();
    const int lane = threadIdx.x & 63;
    if (row > S) return;
    const double* f = row < S ? F + (int64_t)row * ldf : y;
    double s = 0.0;
    for (int i = lane; i < n; i += 64) s += f[i];
    const double m = wave_sum(s) / n;
    double q = 0.0;
    for (int i = lane; i < n; i += 64) {
        const double d = f[i] - m;
        q += d * d;
    }
    q = wave_sum(q);
    const double inv = q > 0.0 ? 1.0 / sqrt(q) : 0.0;
    double* z = Z + (int64_t)row * ldz;
    double zz = 0.0;
    for (int i = lane; i < ldz; i += 64) {
        const double zi = i < n ? (f[i] - m) * inv : 0.0;
        z[i] = zi;
        zz += zi * zi;
    }
    if (nrm && row < S) {
        zz = wave_sum(zz);
        if (lane == 0) nrm[row] = zz;
    }
    if (row == S && lane == 0) *yy = q;
}

// G = Z Z^T for M = S + 1 rows on the FP64 matrix cores.  A block covers a
// 32 x 32 tile of the upper triangle (mirrored when written) as 2 x 2
// products of v_mfma_f64_16x16x4f64, and its four waves split the sum over
// samples into four runs of whole 16-sample chunks; the partial tiles meet
// in LDS and are added in wave order, so the result does not depend on
// timing.  (Each wave owning a whole chain keeps the MFMA pipe busy between
// loads; a 64 x 64 tile per block left small Gram matrices to a few dozen
// blocks, each waiting on its loads.)  The instruction takes A[i][k] from
// lane i + 16 k and B[k][j] from lane j + 16 k and leaves D[i][j] in lane
// j + 16 (i mod 4), register i / 4.  The sum over samples may run in any
// order, so lane l takes samples k0 + 4 (l / 16) + s at step s of a chunk
// of 16: its four samples of a row are one 32-byte load, and the four lanes
// of a row read 128 contiguous bytes.  The next chunk's fragments are
// loaded while the current chunk's 16 products run.  ldz is a multiple of
// 16 and Z is zero past n, rows are 32-byte aligned.
typedef double dsc_v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void d_gram(int M, int ldz, int nk, const double* __restrict__ Z,
                                       double* __restrict__ G, int ldg, int bi, int bj,
                                       double* __restrict__ dg) {
    __shared__ dsc_v4d part[3][4][64];        // waves 1..3: their 2 x 2 partial tiles
    const int wv = wave_id();
    const int lane = threadIdx.x & 63;
    const int r16 = lane & 15, kg = 4 * (lane >> 4);
    const int nch = nk >> 4;                  // chunks of 16 samples; wave wv takes [ch0, ch1)
    const int ch0 = (nch * wv) >> 2, ch1 = (nch * (wv + 1)) >> 2;
    dsc_v4d acc[2][2];
#pragma unroll
    for (int u = 0; u < 2; u++)
#pragma unroll
        for (int v = 0; v < 2; v++) acc[u][v] = dsc_v4d{0.0, 0.0, 0.0, 0.0};
    if (ch1 > ch0) {                          // (wave-uniform)
        const double* pa[2];
        const double* pb[2];
#pragma unroll
        for (int t = 0; t < 2; t++) {
            pa[t] = Z + (int64_t)min(bi + 16 * t + r16, M - 1) * ldz + kg;
            pb[t] = Z + (int64_t)min(bj + 16 * t + r16, M - 1) * ldz + kg;
        }
        double4 A[2], B[2];
        const int kbeg = ch0 * 16, klast = ch1 * 16 - 16;
#pragma unroll
        for (int t = 0; t < 2; t++) { A[t] = *(const double4*)(pa[t] + kbeg); B[t] = *(const double4*)(pb[t] + kbeg); }
        for (int k0 = kbeg; k0 <= klast; k0 += 16) {
            double4 An[2], Bn[2];
            const int kn = min(k0 + 16, klast);   // the last chunk reloads itself
#pragma unroll
            for (int t = 0; t < 2; t++) {
                An[t] = *(const double4*)(pa[t] + kn);
                Bn[t] = *(const double4*)(pb[t] + kn);
            }
#pragma unroll
            for (int u = 0; u < 2; u++)
#pragma unroll
                for (int v = 0; v < 2; v++) {
                    acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[u].x, B[v].x, acc[u][v], 0, 0, 0);
                    acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[u].y, B[v].y, acc[u][v], 0, 0, 0);
                    acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[u].z, B[v].z, acc[u][v], 0, 0, 0);
                    acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[u].w, B[v].w, acc[u][v], 0, 0, 0);
                }
            // the loaded fragments pass through an empty asm: without it the
            // compiler folds this load into a load at the top of the next
            // chunk that waits for its own result
#pragma unroll
            for (int t = 0; t < 2; t++) {
                asm("" : "+v"(An[t].x), "+v"(An[t].y), "+v"(An[t].z), "+v"(An[t].w));
                asm("" : "+v"(Bn[t].x), "+v"(Bn[t].y), "+v"(Bn[t].z), "+v"(Bn[t].w));
                A[t] = An[t]; B[t] = Bn[t];
            }
        }
    }
    if (wv > 0)
#pragma unroll
        for (int u = 0; u < 2; u++)
#pragma unroll
            for (int v = 0; v < 2; v++) part[wv - 1][2 * u + v][lane] = acc[u][v];
    __syncthreads();
    if (wv != 0) return;
#pragma unroll
    for (int u = 0; u < 2; u++)
#pragma unroll
        for (int v = 0; v < 2; v++) {
            dsc_v4d t = acc[u][v];
#pragma unroll
            for (int w = 0; w < 3; w++) t += part[w][2 * u + v][lane];
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int i = bi + 16 * u + (lane >> 4) + 4 * r, j = bj + 16 * v + r16;
                if (i < M && j < M && i <= j) {
                    G[(int64_t)i * ldg + j] = t[r];
                    G[(int64_t)j * ldg + i] = t[r];
                    if (i == j) dg[i] = t[r];
                }
            }
        }
}

// ----------------------------------------------------------------- sweep
// Every sweep writes, per lane, the best explained fraction q of the
// subsets that lane owns (D = 1, 2: exactly one subset per lane; D = 3: the
// lane's (a, c) pair over its block's range of b).  A radix selection over
// these lane values gives the m-th best, and only lanes reaching the band
// threshold are expanded again.
struct SweepArgs {
    const double* G;
    const double* dg;         // G's diagonal, contiguous
    int ldg, S, D;
    const double4* E;         // D = 3: (a, b) factor table, E[b * lde + a]
    int lde;
    const int2* items;        // D = 1, 2: (a, first b) per wave; a < 0: padding
    const int4* items3;       // D = 3: (a0, c0, b_lo, b_hi) per block
    int64_t n_items;
    double* lane_q;           // [n_items][64] (D = 1, 2) or [n_items][256] (D = 3)
    int64_t item0;            // first merged block (D = 3) or merged block of 4 waves (D = 1, 2)
    const double* theta;      // D = 3: the bound th of the table's shifted Q_ab
    // bounded D = 3: lanes holding a value (a subset above th) are listed
    // here instead of writing every lane: lane index within lane_q's
    // layout, value; capacity = every lane, count zeroed by k_sw3_theta
    int32_t* lidx;
    double* lval;
    unsigned long long* lcnt;
};

// 1/x by the hardware reciprocal and one Newton step.  The residual e = 1 -
// x r (one FMA, exact to its rounding) is r's relative error, and the
// Newton step leaves about e^2: when |e| exceeds 2^-20 (never seen on
// gfx950) the correctly rounded quotient is taken instead, so the result
// is within 2^-40 of 1/x whatever the hardware reciprocal's accuracy.
__device__ __forceinline__ double fast_rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, r, 1.0);
    if (!(fabs(e) <= 9.5367431640625e-7)) return 1.0 / x;
    return fma(r, e, r);
}

// The sweeps of every problem of a call run as one launch: block i of the
// grid belongs to problem bprob[i]; a problem's blocks are contiguous.
// D = 1: lane a.
__global__ __launch_bounds__(256) void k_sweep1(ctab<SweepArgs> A, const int* __restrict__ bprob) {
    const SweepArgs& g = tab(A, bprob[blockIdx.x]);
    DSC_GLOBAL(g.G); DSC_GLOBAL(g.items); DSC_GLOBAL(g.lane_q);
    const int64_t it = ((int64_t)blockIdx.x - g.item0) * 4 + wave_id();
    if (it >= g.n_items) return;
    const int lane = threadIdx.x & 63;
    const int a = g.items[it].y + lane;
    double q = -1.0;
    if (a < g.S) {
        const double caa = g.G[(int64_t)a * g.ldg + a], ca = g.G[(int64_t)a * g.ldg + g.S];
        if (caa > PIV_TOL) q = ca * ca / caa;
    }
    g.lane_q[it * 64 + lane] = q;
}

// D = 2: fixed a per wave, lane b.
__device__ __forceinline__ double q2(const double* G, int ldg, int S, int a, int b) {
    const double* Ga = G + (int64_t)a * ldg;
    const double caa = Ga[a], ca = Ga[S];
    if (!(caa > PIV_TOL)) return -1.0;
    const double cab = Ga[b], cbb = G[(int64_t)b * ldg + b], cb = G[(int64_t)b * ldg + S];
    const double w = cab / caa;
    const double piv = cbb - cab * w;
    const double e = cb - ca * w;
    return piv > PIV_TOL ? ca * ca / caa + e * e / piv : -1.0;
}

__global__ __launch_bounds__(256) void k_sweep2(ctab<SweepArgs> A, const int* __restrict__ bprob) {
    const SweepArgs& g = tab(A, bprob[blockIdx.x]);
    DSC_GLOBAL(g.G); DSC_GLOBAL(g.items); DSC_GLOBAL(g.lane_q);
    const int64_t it = ((int64_t)blockIdx.x - g.item0) * 4 + wave_id();
    if (it >= g.n_items) return;
    const int lane = threadIdx.x & 63;
    const int a = g.items[it].x, b = g.items[it].y + lane;
    g.lane_q[it * 64 + lane] = (b < g.S && b > a) ? q2(g.G, g.ldg, g.S, a, b) : -1.0;
}

// D = 3.  One block = 16 consecutive a (4 per wave) x 64 consecutive c (one
// per lane) x a range of b.  Each G[b][c] load serves the wave's 4 values
// of a.  Per (a, b), the same for every lane of a wave: u_b = G[a][b],
// g_b = z'_b / d_b, h_b = 1 / d_b, Q_ab = c_a^2 / G_aa + z'_b^2 / d_b with
// d_b = G_bb - u_b^2 / G_aa and z'_b = c_b - u_b c_a / G_aa.  Per subset:
//   C'  = G[b][c] - u_b u_c / G_aa
//   den = d_c - C'^2 / d_b            (third Cholesky pivot)
//   e   = z'_c - C' g_b
//   q   = Q_ab + e^2 / den.
// The (a, b) factors are tabulated once per call, b-major (E[b][a]), so a
// wave's four entries for one b are 128 contiguous bytes at a wave-uniform
// address: they arrive through scalar loads into SGPRs and enter the FP64
// FMAs as scalar operands, leaving LDS and the vector memory path to the
// per-lane G[b][c] stream.
//
// Bounded sweep.  Before the sweep, a lower bound theta on the m-th best
// subset is taken from m subsets in distinct lanes (k_sw3_rows/k_sw3_theta)
// and lowered by every allowance of the band (th = theta - GRAM_DELTA -
// 4 SW3_RCP_DELTA - 2^-24 - 1e-8).  The table stores Q_ab - th, so the test
//   e^2 + (Q_ab - th) den > 0   <=>   q > th      (den > 0)
// costs one FMA and two 32-bit compares per subset; only when some lane of
// the wave passes it are the wave's exact values (reciprocal, pivot test,
// minimum) computed.  A lane whose best subset lies above th therefore
// reports that subset's exact sweep value, as an unbounded sweep would, and
// every other lane reports a value below th (or -1), which no band
// threshold can reach: the m lanes that define theta report at least theta,
// the radix selection's bound of the m-th lane value is at most 2^-24 below
// it, so the threshold is at least theta - 2^-24 - GRAM_DELTA -
// SW3_RCP_DELTA - 1e-12, and a lane is expanded only from that threshold
// minus another SW3_RCP_DELTA + 1e-9 on.
constexpr int SW3_A = 4;              // values of a per wave
constexpr int SW3_MMAX = 16;          // bounded sweep for m up to this
// (2^-24: the radix selection's threshold may lie that far below the m-th lane value)
constexpr double SW3_TH_SLACK = GRAM_DELTA + 4.0 * SW3_RCP_DELTA + 5.9604644775390625e-8 + 1e-8;

struct Sw3Lane {
    double upc, dc, zc;
};

// Entry of the factor table for (a, b); w = Q_ab - th.  A singular a or
// pair (a, b), and every (a, b) that cannot start a triple, carries
// (0, 0, 0, -inf): h_b = 0 leaves den = d_c, and w = -inf makes q = -inf
// in every form of the sweep (the bounded test fails, the exact value is
// +inf in negated form, which the minimum skips).  ub = G[a][b]; G[b][b]
// comes from the diagonal copy dg and G[b][y] from row S (G is written
// mirrored, so both equal the transposed entries bit for bit), so that
// lanes with consecutive b read consecutive addresses.
__device__ __forceinline__ double4 sw3_b_entry(const double* G, int ldg, int S, const double* dg, double ub,
                                               double ica, double ca, int b) {
    const double db = dg[b] - ub * ub * ica;
    const double zb = G[(int64_t)S * ldg + b] - ub * ca * ica;
    if (db > PIV_TOL) {
        const double hb = 1.0 / db;
        return make_double4(ub, zb * hb, hb, ca * ca * ica + zb * zb * hb);
    }
    return make_double4(0.0, 0.0, 0.0, -__builtin_inf());
}

__device__ __forceinline__ Sw3Lane sw3_lane(const double* G, int ldg, int S, const double* dg, const double* Ga,
                                            double caa, double ca, int c, bool cok) {
    Sw3Lane L;
    const double uc = Ga[c];
    L.upc = uc * (1.0 / caa);
    // an out-of-range c gets a negative d_c, so none of its triples passes
    L.dc = cok ? dg[c] - uc * L.upc : -1.0;
    L.zc = G[(int64_t)S * ldg + c] - ca * L.upc;
    return L;
}

__device__ __forceinline__ double sw3_q(const double4& e, const Sw3Lane& L, double Cbc,
                                        double& den) {
    const double Cp = fma(-e.x, L.upc, Cbc);
    const double ee = fma(-Cp, e.y, L.zc);
    const double t = Cp * e.z;
    den = fma(-Cp, t, L.dc);
    return fma(ee * ee, fast_rcp(den), e.w);
}

// Table of (a, b) factors, E[b * lde + a], lde >= S + 16.  Row b holds every
// a < b and the entries a = b .. b + 15 that a block starting below b may
// also read (a wave's a values reach at most 15 past the block's first a).
__device__ __forceinline__ void d_sw3_table(const double* __restrict__ G, int ldg, int S,
                                            const double* __restrict__ dg,
                                            double4* __restrict__ E, int lde, double th) {
    const int b = blockIdx.y;
    const int a = blockIdx.x * 256 + threadIdx.x;
    if (a >= lde || a > b + 15) return;
    double4 e = make_double4(0.0, 0.0, 0.0, -__builtin_inf());
    if (a < S - 2 && b > a) {
        const double caa = dg[a];                       // lanes take consecutive a: row reads
        if (caa > PIV_TOL) {
            e = sw3_b_entry(G, ldg, S, dg, G[(int64_t)b * ldg + a], 1.0 / caa, G[(int64_t)S * ldg + a], b);
            e.w -= th;
        }
    }
    E[(int64_t)b * lde + a] = e;
}

// min(low, ok ? x : +huge): the mask selects only the high word (a value
// with high word 0x7FEFFFFF is a large positive finite number whatever its
// low word), and the minimum is one v_min_f64.  In IEEE mode v_min_f64
// returns the other operand when one is a quiet NaN and never prefers
// +inf, which the sweep's marked entries rely on; the instruction is written
// out to leave out the input quieting the compiler adds around fmin.
__device__ __forceinline__ double sw3_keep(double low, double x, bool ok) {
    const int hi = ok ? __double2hiint(x) : (int)0x7FEFFFFF;
    const double v = __hiloint2double(hi, __double2loint(x));
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(low), "v"(v));
    return r;
}

// The sweep's own value, -q~ with q~ = e^2 * rcp(den) + Q_ab, where rcp is
// the bare hardware reciprocal; SW3_RCP_DELTA allows 2^-21 of the explained
// fraction for its error.  The residual 1 - den rcp (one FMA, exact to its
// rounding) is that error: a reciprocal further than 2^-22 off (never seen
// on gfx950, whose error stays below 2^-24.3) is replaced by the correctly
// rounded quotient, so the allowance holds by construction.  w is the
// table's Q_ab - th; adding th back costs one rounding of Q_ab, far inside
// the band's allowances.
__device__ __forceinline__ double sw3_negq(double ee2, double den, double w, double th) {
    double r = __builtin_amdgcn_rcp(den);
    if (!(fabs(fma(-den, r, 1.0)) <= 2.384185791015625e-7)) r = 1.0 / den;
    return fma(-ee2, r, -(w + th));
}

// One row b of a wave, from its loaded G entry C and factor entries E.  In
// the bounded form a lane passes when e^2 + w den > 0 (w = Q_ab - th); only
// when some lane of the wave passes are the exact values of all its lanes
// formed.  Diagonal lanes with c <= b are cut from the pass mask (lmask)
// and from the exact update (live); a singular or ill-conditioned triple
// (den <= PIV_TOL) may pass the test but fails the exact update.
template <bool BOUND>
__device__ __forceinline__ void sw3_row(const double4 (&E)[SW3_A], double C, uint64_t lmask, bool live,
                                        double th, const Sw3Lane (&L)[SW3_A], double (&low)[SW3_A]) {
    double den[SW3_A], ee2[SW3_A];
    uint64_t hit = 0;
#pragma unroll
    for (int k = 0; k < SW3_A; k++) {
        const double Cp = fma(-E[k].x, L[k].upc, C);
        const double ee = fma(-Cp, E[k].y, L[k].zc);
        const double t = Cp * E[k].z;
        den[k] = fma(-Cp, t, L[k].dc);
        ee2[k] = ee * ee;
        if (BOUND) hit |= __builtin_amdgcn_ballot_w64(__double2hiint(fma(E[k].w, den[k], ee2[k])) > 0);
    }
    if (!BOUND || (hit & lmask)) {
#pragma unroll
        for (int k = 0; k < SW3_A; k++)
            low[k] = sw3_keep(low[k], sw3_negq(ee2[k], den[k], E[k].w, th), live && den[k] > PIV_TOL);
    }
}

// Rows b .. bend - 1 of a wave.  DIAG: the block's diagonal part, b >= c0,
// where lanes with c <= b own no triple.  Per row the G entry of the lane's
// c (a vector load from the row's scalar base) and the wave's four factor
// entries (scalar loads) are read; eight waves per SIMD cover their latency
// (issuing the next row's loads ahead needs a second set of 32 SGPRs,
// which the compiler then spills).
template <bool DIAG, bool BOUND>
__device__ __forceinline__ void sw3_run(const double4* __restrict__ Ew, int lde, const double* G,
                                        int ldg, uint32_t cc, int c0, int b, int bend, double th,
                                        const Sw3Lane (&L)[SW3_A], double (&low)[SW3_A]) {
    const int lane = threadIdx.x & 63;
    const double4* Eb = Ew + (int64_t)b * lde;
    const double* Gb = G + (int64_t)b * ldg;
    for (; b < bend; b++, Eb += lde, Gb += ldg) {
        const double C = Gb[cc];
        double4 E[SW3_A];
#pragma unroll
        for (int k = 0; k < SW3_A; k++) E[k] = Eb[k];
        // lanes c = c0 + lane > b keep their triples
        sw3_row<BOUND>(E, C, DIAG ? ~0ull << (b - c0 + 1) : ~0ull, !DIAG || c0 + lane > b, th, L, low);
    }
}

// Eight waves per SIMD (64 VGPRs; the few spills sit outside the row loops).
template <bool BOUND>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_sweep3(ctab<SweepArgs> A, const int* __restrict__ bprob) {
    const SweepArgs& g = tab(A, bprob[blockIdx.x]);
    DSC_GLOBAL(g.G); DSC_GLOBAL(g.dg); DSC_GLOBAL(g.E); DSC_GLOBAL(g.items3); DSC_GLOBAL(g.lane_q); DSC_GLOBAL(g.theta);
    const int64_t li = (int64_t)blockIdx.x - g.item0;   // block within its problem
    const int4 item = g.items3[li];
    const int a0 = item.x, c0 = item.y;                  // block: a0..a0+15, c0..c0+63, b in [z, w)
    const int wv = wave_id();
    const int lane = threadIdx.x & 63;
    const int c = c0 + lane;
    double* out = g.lane_q + (li * 4 + wv) * (SW3_A * 64);
    if (a0 < 0) {                                        // padding block (uniform)
        // (the bounded form lists lanes instead; its lane_q holds the list)
        if (!BOUND)
            for (int k = 0; k < SW3_A; k++) out[k * 64 + lane] = -1.0;
        return;
    }
    const double th = *g.theta;
    const int aw = a0 + wv * SW3_A;                      // the wave's first a
    // a lane past the last column evaluates column S - 1 (c > b holds
    // there) and reports no triple
    const bool cok = c < g.S;
    const int cc = cok ? c : g.S - 1;
    Sw3Lane L[SW3_A];
    double low[SW3_A];                                   // min over b of -q~
#pragma unroll
    for (int k = 0; k < SW3_A; k++) {
        const int ac = min(aw + k, g.S - 1);
        const double* Ga = g.G + (int64_t)ac * g.ldg;
        L[k] = sw3_lane(g.G, g.ldg, g.S, g.dg, Ga, Ga[ac], Ga[g.S], cc, true);
        low[k] = 1.0;
    }
    const double4* Ew = g.E + aw;
    const int bstart = max(aw + 1, item.z);
    const int bend = min(min(g.S - 1, c0 + 63), item.w); // b < largest c of the block
    // b < c0: every lane has c > b; from c0 on, lanes with c <= b are cut
    sw3_run<false, BOUND>(Ew, g.lde, g.G, g.ldg, (uint32_t)cc, c0, bstart, min(bend, c0), th, L, low);
    sw3_run<true, BOUND>(Ew, g.lde, g.G, g.ldg, (uint32_t)cc, c0, max(bstart, c0), bend, th, L, low);
    if (!BOUND) {
#pragma unroll
        for (int k = 0; k < SW3_A; k++) out[k * 64 + lane] = cok ? -low[k] : -1.0;   // -1: no valid triple
        return;
    }
    // bounded: append the lanes that hold a value (one atomic per wave)
    uint64_t keep[SW3_A];
    int tot = 0;
#pragma unroll
    for (int k = 0; k < SW3_A; k++) {
        keep[k] = __builtin_amdgcn_ballot_w64(cok && low[k] < 0.5);
        tot += __popcll(keep[k]);
    }
    if (tot == 0) return;                               // (wave-uniform)
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(g.lcnt, (unsigned long long)tot);
    base = __shfl(base, 0, 64);
    const uint64_t below = (1ull << lane) - 1ull;
    const int64_t lane0 = (li * 4 + wv) * (SW3_A * 64);
#pragma unroll
    for (int k = 0; k < SW3_A; k++) {
        if ((keep[k] >> lane) & 1ull) {
            const unsigned long long pos = base + __popcll(keep[k] & below);
            g.lidx[pos] = (int32_t)(lane0 + k * 64 + lane);
            g.lval[pos] = -low[k];
        }
        base += __popcll(keep[k]);
    }
}

// Lower bound for the bounded sweep, step 1: one wave per row a.  b(a) is
// the partner with the largest Q_ab (ties: smaller b) among b <= S - 2, and
// rowq[a] the largest sweep value of the triples (a, b(a), c), c > b(a), or
// -1.  Distinct rows give subsets in distinct sweep lanes (a, c).
struct ThetaArgs {
    const double* G;
    const double* dg;         // G's diagonal, contiguous
    int ldg, S;
    double* rowq;
    double* theta;
    unsigned long long* lcnt;     // the bounded sweep's lane-list count, zeroed here
};

__device__ __forceinline__ void wave_argmax(double& v, int& i) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const double ov = __shfl_xor(v, o);
        const int oi = __shfl_xor(i, o);
        if (ov > v || (ov == v && oi < i)) { v = ov; i = oi; }
    }
}

// grid (rows, problems): the block's 256 threads share the row's b and c
// ranges; the arg-max (ties to the smaller b) and the maximum do not depend
// on how the range is split.
__global__ __launch_bounds__(256) void k_sw3_rows(ctab<ThetaArgs> A) {
    const ThetaArgs& g = tab(A, blockIdx.y);
    DSC_GLOBAL(g.G); DSC_GLOBAL(g.dg); DSC_GLOBAL(g.rowq);
    __shared__ double sv[4];
    __shared__ int si[4];
    const int a = blockIdx.x;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    if (a >= g.S) return;                               // (block-uniform)
    const double* Ga = g.G + (int64_t)a * g.ldg;
    const double caa = Ga[a], ca = Ga[g.S];
    double best = -1.0;
    if (a < g.S - 2 && caa > PIV_TOL) {
        const double ica = 1.0 / caa;
        double qb = -1.0;
        int bb = 0x7fffffff;
        for (int b = a + 1 + t; b < g.S - 1; b += 256) {
            const double4 e = sw3_b_entry(g.G, g.ldg, g.S, g.dg, Ga[b], ica, ca, b);
            if (e.w > qb) { qb = e.w; bb = b; }
        }
        wave_argmax(qb, bb);
        if (lane == 0) { sv[wv] = qb; si[wv] = bb; }
        __syncthreads();
        for (int w = 0; w < 4; w++)
            if (sv[w] > qb || (sv[w] == qb && si[w] < bb)) { qb = sv[w]; bb = si[w]; }
        __syncthreads();                                // sv/si are read before their reuse
        if (qb >= 0.0) {
            const int b = bb;
            const double4 e = sw3_b_entry(g.G, g.ldg, g.S, g.dg, Ga[b], ica, ca, b);
            const double* Gb = g.G + (int64_t)b * g.ldg;
            for (int c = b + 1 + t; c < g.S; c += 256) {
                const Sw3Lane L = sw3_lane(g.G, g.ldg, g.S, g.dg, Ga, caa, ca, c, true);
                const double Cp = fma(-e.x, L.upc, Gb[c]);
                const double ee = fma(-Cp, e.y, L.zc);
                const double den = fma(-Cp, Cp * e.z, L.dc);
                if (den > PIV_TOL) best = fmax(best, -sw3_negq(ee * ee, den, e.w, 0.0));
            }
            best = wave_max(best);
            if (lane == 0) sv[wv] = best;
            __syncthreads();
            best = fmax(fmax(sv[0], sv[1]), fmax(sv[2], sv[3]));
        }
    }
    if (t == 0) g.rowq[a] = best;
}

// Step 2, one block per problem: theta = the m-th largest row value (m
// rounds of a block-wide arg-max, ties to the smaller row), th = theta -
// SW3_TH_SLACK; with fewer than m rows holding a triple, th = -1 (every
// subset passes the bounded test).
__global__ __launch_bounds__(256) void k_sw3_theta(ctab<ThetaArgs> A, int m) {
    const ThetaArgs& g = tab(A, blockIdx.x);
    DSC_GLOBAL(g.rowq); DSC_GLOBAL(g.theta); DSC_GLOBAL(g.lcnt);
    __shared__ double sv[4];
    __shared__ int si[4];
    double pv = __builtin_inf();
    int pi = -1;
    for (int r = 0; r < m; r++) {
        double v = -__builtin_inf();
        int i = 0x7fffffff;
        for (int a = threadIdx.x; a < g.S; a += 256) {
            const double x = g.rowq[a];
            const bool below = x < pv || (x == pv && a > pi);
            if (below && (x > v || (x == v && a < i))) { v = x; i = a; }
        }
        wave_argmax(v, i);
        __syncthreads();
        if ((threadIdx.x & 63) == 0) { sv[threadIdx.x >> 6] = v; si[threadIdx.x >> 6] = i; }
        __syncthreads();
        v = sv[0]; i = si[0];
        for (int w = 1; w < 4; w++)
            if (sv[w] > v || (sv[w] == v && si[w] < i)) { v = sv[w]; i = si[w]; }
        pv = v; pi = i;
    }
    if (threadIdx.x == 0) {
        *g.theta = pv >= 0.0 ? pv - SW3_TH_SLACK : -1.0;
        *g.lcnt = 0;
    }
}

// Band expansion.  thr = (m-th best lane value) * (1 - 1e-12) - GRAM_DELTA.
struct BandArgs {
    const double* G;
    const double* dg;         // G's diagonal, contiguous
    int ldg, S, D;
    const double4* E;         // D = 3 factor table (as in SweepArgs)
    int lde;
    const int2* items;
    int64_t n_lanes;
    const double* lane_q;
    uint32_t* sel;            // radix selection of the problem's lanes
    int64_t* st;
    const uint32_t* hist;     // its two level histograms
    int4* band;
    unsigned long long* bcnt;
    int64_t bcap;
    const int4* items3;
    int4* pairs;              // D = 3: (a, c, b_lo, b_hi) lanes to expand
    unsigned long long* pcnt;
    int64_t pcap;
    const double* theta;      // D = 3: the table's shift th
    const int32_t* lidx;      // bounded D = 3: listed lanes (lane index, value) instead of lane_q
    const double* lval;
    const unsigned long long* lcnt;
};

// For D = 3 the lane values carry the sweep's reciprocal error (at most
// SW3_RCP_DELTA): the m lanes at or above the selected value hold m distinct
// subsets whose exact q is at least that value minus SW3_RCP_DELTA, so the
// threshold drops by it; and a lane whose exact best reaches the threshold
// shows a sweep value no lower than threshold - SW3_RCP_DELTA.
__device__ __forceinline__ double band_thr(const uint32_t* sel, const int64_t* st, int D) {
    if (st[1]) return -0.5;                              // fewer than m valid lanes: take all
    return select_threshold(sel, st) * (1.0 - 1e-12) - GRAM_DELTA - (D == 3 ? SW3_RCP_DELTA : 0.0);
}

__device__ __forceinline__ double band_thr(const BandArgs& g) { return band_thr(g.sel, g.st, g.D); }

__device__ __forceinline__ void band_push(const BandArgs& g, int a, int b, int c) {
    const unsigned long long slot = atomicAdd(g.bcnt, 1ull);
    if ((int64_t)slot < g.bcap) g.band[slot] = make_int4(a, b, c, 0);
}

// grid (blocks, problems)
__global__ __launch_bounds__(256) void k_band_lanes(ctab<BandArgs> A) {
    const BandArgs& g = tab(A, blockIdx.y);
    DSC_GLOBAL(g.lane_q); DSC_GLOBAL(g.items); DSC_GLOBAL(g.items3); DSC_GLOBAL(g.sel); DSC_GLOBAL(g.st); DSC_GLOBAL(g.band); DSC_GLOBAL(g.bcnt); DSC_GLOBAL(g.pairs); DSC_GLOBAL(g.pcnt); DSC_GLOBAL(g.lidx); DSC_GLOBAL(g.lval); DSC_GLOBAL(g.lcnt); DSC_GLOBAL(g.hist);
    uint32_t sel[3];
    int64_t st[2];
    radix_finish(g.hist, g.sel, g.st, sel, st);
    const double thr = band_thr(sel, st, g.D);
    const int per = g.D == 3 ? 4 * SW3_A * 64 : 64;
    const int64_t nl = g.lidx ? min((int64_t)*g.lcnt, g.n_lanes) : g.n_lanes;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nl; e += (int64_t)gridDim.x * 256) {
        const int64_t i = g.lidx ? (int64_t)g.lidx[e] : e;
        const double q = g.lidx ? g.lval[e] : g.lane_q[i];
        if (!(q > -0.5) || q < thr - (g.D == 3 ? SW3_RCP_DELTA : 0.0) - 1e-9) continue;
        const int lane = (int)(i % per);
        if (g.D == 1) band_push(g, g.items[i / per].y + lane, -1, -1);
        else if (g.D == 2) band_push(g, g.items[i / per].x, g.items[i / per].y + lane, -1);
        else {
            // lane index within a D = 3 block: ((wave * SW3_A) + k) * 64 + c lane
            const int4 it = g.items3[i / per];
            const int wk = lane / 64, cl = lane % 64;
            const unsigned long long slot = atomicAdd(g.pcnt, 1ull);
            if ((int64_t)slot < g.pcap) g.pairs[slot] = make_int4(it.x + wk, it.y + cl, it.z, it.w);
        }
    }
}

// D = 3: one wave per listed (a, c) lane; its lanes split the b range.
__global__ __launch_bounds__(256) void k_band_expand3(ctab<BandArgs> A) {
    const BandArgs& g = tab(A, blockIdx.y);
    DSC_GLOBAL(g.G); DSC_GLOBAL(g.dg); DSC_GLOBAL(g.E); DSC_GLOBAL(g.sel); DSC_GLOBAL(g.st); DSC_GLOBAL(g.band); DSC_GLOBAL(g.bcnt); DSC_GLOBAL(g.pairs); DSC_GLOBAL(g.pcnt); DSC_GLOBAL(g.theta);
    const double thr = band_thr(g);
    const double th = *g.theta;
    const int64_t np = min((int64_t)*g.pcnt, g.pcap);
    const int lane = threadIdx.x & 63;
    for (int64_t i = (int64_t)blockIdx.x * 4 + wave_id(); i < np; i += (int64_t)gridDim.x * 4) {
        const int a = g.pairs[i].x, c = g.pairs[i].y;
        const int blo = max(a + 1, g.pairs[i].z), bhi = min(c, g.pairs[i].w);
        const double* Ga = g.G + (int64_t)a * g.ldg;
        const double caa = Ga[a], ca = Ga[g.S];
        const Sw3Lane L = sw3_lane(g.G, g.ldg, g.S, g.dg, Ga, caa, ca, c, true);   // as in the sweep
        for (int b = blo + lane; b < bhi; b += 64) {
            double4 e = g.E[(int64_t)b * g.lde + a];
            e.w += th;
            double den;
            const double q = sw3_q(e, L, g.G[(int64_t)b * g.ldg + c], den);
            if (den > PIV_TOL && q >= thr) band_push(g, a, b, c);
        }
    }
}

// ------------------------------------------------------------ QR refit
// Least squares of y on [1, F rows idx[0..d-1]] by Householder QR in one
// 256-thread workgroup; A holds the M + 1 columns of n (intercept, the d
// features, the right-hand side), in LDS (dynamic shared memory) or a
// global slab — the function is inlined into each caller's branches, so
// each copy addresses its own memory directly.  The column count M = d + 1
// is fixed at compile time: each Householder step j forms, in one pass,
// the norm of column j and its raw products with the later columns and the
// right-hand side (the reflector v differs from column j only in element j,
// a_jj - alpha, so v . a_c = a_j . a_c + (v_j - a_jj) a_c[j]) and reduces
// them together; every loop is unrolled, so a step costs one block
// reduction and one update pass.  (With run-time counts the same scheme
// was slower than a reduction per column.)
template <int M>
__device__ __forceinline__ void block_lsq_t(int n, const int* idx, const double* __restrict__ F, int64_t ldf,
                                            const double* __restrict__ y, double* A, double* coef,
                                            double* rss, double* resid) {
    constexpr int d = M - 1;
    __shared__ double redm[M + 1][4];
    __shared__ double R[M][M + 1];
    double* w = A + (int64_t)M * n;
    for (int i = threadIdx.x; i < n; i += 256) {
        A[i] = 1.0;
#pragma unroll
        for (int j = 0; j < d; j++) A[(int64_t)(j + 1) * n + i] = F[(int64_t)idx[j] * ldf + i];
        w[i] = y[i];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < M; j++) {
        const double* aj = A + (int64_t)j * n;
        double sums[M + 1];                           // [0] |a_j|^2, [q] a_j . a_{j+q} (q = M - j: rhs)
#pragma unroll
        for (int q = 0; q <= M - j; q++) sums[q] = 0.0;
        for (int i = j + threadIdx.x; i < n; i += 256) {
            const double a = aj[i];
            sums[0] += a * a;
#pragma unroll
            for (int q = 1; q <= M - j; q++) sums[q] += a * A[(int64_t)(j + q) * n + i];
        }
#pragma unroll
        for (int q = 0; q <= M - j; q++) sums[q] = wave_sum(sums[q]);
        if ((threadIdx.x & 63) == 0)
#pragma unroll
            for (int q = 0; q <= M - j; q++) redm[q][threadIdx.x >> 6] = sums[q];
        __syncthreads();
#pragma unroll
        for (int q = 0; q <= M - j; q++) sums[q] = (redm[q][0] + redm[q][1]) + (redm[q][2] + redm[q][3]);
        const double nrm = sqrt(sums[0]);
        const double ajj = aj[j];
        const double alpha = ajj > 0 ? -nrm : nrm;
        const double v0 = ajj - alpha;
        const double vv = 2.0 * nrm * (nrm + fabs(ajj));   // v^T v
        double gm[M + 1];
#pragma unroll
        for (int q = 1; q <= M - j; q++) {
            const double dot = fma(v0 - ajj, A[(int64_t)(j + q) * n + j], sums[q]);
            gm[q] = vv > 0.0 ? 2.0 * dot / vv : 0.0;
        }
        __syncthreads();                              // a_cj and a_jj read; redm free
        for (int i = j + threadIdx.x; i < n; i += 256) {
            const double vi = i == j ? v0 : aj[i];
#pragma unroll
            for (int q = 1; q <= M - j; q++) A[(int64_t)(j + q) * n + i] -= gm[q] * vi;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            R[j][j] = alpha;
#pragma unroll
            for (int c = j + 1; c < M; c++) R[j][c] = A[(int64_t)c * n + j];
            R[j][M] = w[j];
        }
    }
    double loc = 0.0;
    for (int i = M + threadIdx.x; i < n; i += 256) loc += w[i] * w[i];
    loc = wave_sum(loc);
    if ((threadIdx.x & 63) == 0) redm[0][threadIdx.x >> 6] = loc;
    __syncthreads();
    const double r2 = (redm[0][0] + redm[0][1]) + (redm[0][2] + redm[0][3]);
    if (threadIdx.x == 0) {
        for (int j = M - 1; j >= 0; j--) {
            double acc = R[j][M];
            for (int c = j + 1; c < M; c++) acc -= R[j][c] * coef[c];
            coef[j] = acc / R[j][j];
        }
        *rss = r2;
    }
    __syncthreads();
    if (resid) {
        for (int i = threadIdx.x; i < n; i += 256) {
            double p = coef[0];
#pragma unroll
            for (int j = 0; j < d; j++) p = fma(coef[j + 1], F[(int64_t)idx[j] * ldf + i], p);
            resid[i] = y[i] - p;
        }
    }
}

__device__ __forceinline__ void block_lsq(int n, int d, const int* idx, const double* __restrict__ F,
                                                int64_t ldf, const double* __restrict__ y, double* A,
                                                double* coef, double* rss, double* resid) {
    switch (d + 1) {
    case 1: block_lsq_t<1>(n, idx, F, ldf, y, A, coef, rss, resid); return;
    case 2: block_lsq_t<2>(n, idx, F, ldf, y, A, coef, rss, resid); return;
    case 3: block_lsq_t<3>(n, idx, F, ldf, y, A, coef, rss, resid); return;
    case 4: block_lsq_t<4>(n, idx, F, ldf, y, A, coef, rss, resid); return;
    case 5: block_lsq_t<5>(n, idx, F, ldf, y, A, coef, rss, resid); return;
    case 6: block_lsq_t<6>(n, idx, F, ldf, y, A, coef, rss, resid); return;
    case 7: block_lsq_t<7>(n, idx, F, ldf, y, A, coef, rss, resid); return;
    case 8: block_lsq_t<8>(n, idx, F, ldf, y, A, coef, rss, resid); return;
    default: block_lsq_t<9>(n, idx, F, ldf, y, A, coef, rss, resid); return;
    }
}

// Rank the band: repeatedly take the minimum RSS; entries within
// TAU_TIE * yy of it are tied and the smallest sorted-ID tuple wins.  The
// 256 threads of the block scan the band in parallel: the minimum RSS does
// not depend on the order of the scan, and band subsets are distinct, so
// the winning tuple is unique and every order of the scan finds it.
struct RankKey {
    int64_t k[3];                 // sorted IDs (unused places 0)
    int64_t e;                    // band entry, -1 for none
};

__device__ __forceinline__ bool rank_before(const RankKey& x, const RankKey& y) {
    if (y.e < 0) return x.e >= 0;
    if (x.e < 0) return false;
    for (int j = 0; j < 3; j++)
        if (x.k[j] != y.k[j]) return x.k[j] < y.k[j];
    return x.e < y.e;
}

// The same ranking by one thread, for short bands (fewer barriers).
constexpr int64_t RANK_SERIAL = 512;

__device__ __forceinline__ void rank_models_serial(const int4* __restrict__ band, const double* __restrict__ brss,
                              const double* __restrict__ bcoef, int64_t nb, int D, int m,
                              const int64_t* __restrict__ ids, double yy, int n, uint8_t* __restrict__ taken,
                              int32_t* __restrict__ out_sub, double* __restrict__ out_rmse,
                              double* __restrict__ out_coef, int32_t* __restrict__ chosen, int sub_ld,
                              int coef_ld) {
    for (int64_t e = 0; e < nb; e++) taken[e] = !(brss[e] >= 0.0);
    for (int q = 0; q < m; q++) {
        double rmin = INFINITY;
        for (int64_t e = 0; e < nb; e++)
            if (!taken[e] && brss[e] < rmin) rmin = brss[e];
        RankKey best{{0, 0, 0}, -1};
        if (rmin < INFINITY) {
            for (int64_t e = 0; e < nb; e++) {
                if (taken[e] || !(brss[e] <= rmin + TAU_TIE * yy)) continue;
                const int4 sv = band[e];
                const int pos[3] = {sv.x, sv.y, sv.z};
                RankKey c{{0, 0, 0}, e};
                for (int j = 0; j < D; j++) c.k[j] = ids[pos[j]];
                for (int u = 1; u < D; u++)
                    for (int v = u; v > 0 && c.k[v - 1] > c.k[v]; v--) {
                        const int64_t tt = c.k[v]; c.k[v] = c.k[v - 1]; c.k[v - 1] = tt;
                    }
                if (rank_before(c, best)) best = c;
            }
        }
        const int64_t pick = best.e;
        chosen[q] = (int32_t)pick;
        if (pick < 0) {
            for (int j = 0; j < D; j++) out_sub[q * sub_ld + j] = -1;
            out_rmse[q] = __longlong_as_double(0x7FF8000000000000LL);
            for (int j = 0; j <= D; j++) out_coef[q * coef_ld + j] = __longlong_as_double(0x7FF8000000000000LL);
            continue;
        }
        taken[pick] = 1;
        const int4 sv = band[pick];
        const int pos[3] = {sv.x, sv.y, sv.z};
        for (int j = 0; j < D; j++) out_sub[q * sub_ld + j] = pos[j];
        out_rmse[q] = sqrt(brss[pick] / n);
        for (int j = 0; j <= D; j++) out_coef[q * coef_ld + j] = bcoef[pick * (D + 1) + j];
    }
}

__device__ __forceinline__ void d_rank_models(const int4* __restrict__ band, const double* __restrict__ brss,
                              const double* __restrict__ bcoef,
                              const unsigned long long* __restrict__ bcnt, int64_t bcap, int D, int m,
                              const int64_t* __restrict__ ids, const double* __restrict__ yyp,
                              int n, uint8_t* __restrict__ taken, int32_t* __restrict__ out_sub,
                              double* __restrict__ out_rmse, double* __restrict__ out_coef,
                              int32_t* __restrict__ chosen, int sub_ld, int coef_ld) {
    __shared__ double smin[4];
    __shared__ RankKey skey[4];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const double yy = *yyp;
    const int64_t nb = min((int64_t)*bcnt, bcap);
    if (nb <= RANK_SERIAL) {                         // (block-uniform) a short band: one thread
        if (t == 0) rank_models_serial(band, brss, bcoef, nb, D, m, ids, yy, n, taken, out_sub, out_rmse,
                                       out_coef, chosen, sub_ld, coef_ld);
        __syncthreads();
        return;
    }
    for (int64_t e = t; e < nb; e += 256) taken[e] = !(brss[e] >= 0.0);
    __syncthreads();
    for (int q = 0; q < m; q++) {
        double rmin = INFINITY;
        for (int64_t e = t; e < nb; e += 256)
            if (!taken[e]) rmin = fmin(rmin, brss[e]);
        rmin = wave_min(rmin);
        if (lane == 0) smin[wv] = rmin;
        __syncthreads();
        rmin = fmin(fmin(smin[0], smin[1]), fmin(smin[2], smin[3]));
        RankKey best{{0, 0, 0}, -1};
        if (rmin < INFINITY) {
            for (int64_t e = t; e < nb; e += 256) {
                if (taken[e] || !(brss[e] <= rmin + TAU_TIE * yy)) continue;
                const int4 sv = band[e];
                const int pos[3] = {sv.x, sv.y, sv.z};
                RankKey c{{0, 0, 0}, e};
                for (int j = 0; j < D; j++) c.k[j] = ids[pos[j]];
                for (int u = 1; u < D; u++)          // sort the ID tuple
                    for (int v = u; v > 0 && c.k[v - 1] > c.k[v]; v--) {
                        const int64_t tt = c.k[v]; c.k[v] = c.k[v - 1]; c.k[v - 1] = tt;
                    }
                if (rank_before(c, best)) best = c;
            }
        }
        const uint64_t has = __builtin_amdgcn_ballot_w64(best.e >= 0);
        if (__popcll(has) > 1) {
            for (int o = 32; o > 0; o >>= 1) {       // wave minimum in the tuple order
                RankKey x;
                for (int j = 0; j < 3; j++) x.k[j] = __shfl_xor(best.k[j], o, 64);
                x.e = __shfl_xor(best.e, o, 64);
                if (rank_before(x, best)) best = x;
            }
        } else if (has) {                            // one lane holds the wave's only candidate
            const int src = __builtin_ctzll(has);
            for (int j = 0; j < 3; j++) best.k[j] = __shfl(best.k[j], src, 64);
            best.e = __shfl(best.e, src, 64);
        }
        if (lane == 0) skey[wv] = best;
        __syncthreads();
        if (t == 0) {
            for (int w = 0; w < 4; w++)
                if (rank_before(skey[w], best)) best = skey[w];
            const int64_t pick = best.e;
            chosen[q] = (int32_t)pick;
            if (pick < 0) {
                for (int j = 0; j < D; j++) out_sub[q * sub_ld + j] = -1;
                out_rmse[q] = __longlong_as_double(0x7FF8000000000000LL);
                for (int j = 0; j <= D; j++) out_coef[q * coef_ld + j] = __longlong_as_double(0x7FF8000000000000LL);
            } else {
                taken[pick] = 1;
                const int4 sv = band[pick];
                const int pos[3] = {sv.x, sv.y, sv.z};
                for (int j = 0; j < D; j++) out_sub[q * sub_ld + j] = pos[j];
                out_rmse[q] = sqrt(brss[pick] / n);
                for (int j = 0; j <= D; j++) out_coef[q * coef_ld + j] = bcoef[pick * (D + 1) + j];
            }
        }
        __syncthreads();                             // taken and the shared slots are settled
    }
}

// Residual of chosen model q (NaN for a missing model), by the 256 threads
// of a block.
__device__ __forceinline__ void d_resid(int q, int n, int D, const double* __restrict__ F,
                                               int64_t ldf, const double* __restrict__ y,
                                               const int32_t* __restrict__ sub,
                                               const double* __restrict__ coef,
                                               double* __restrict__ out, int64_t ldr, int sub_ld, int coef_ld) {
    const int32_t* s = sub + q * sub_ld;
    const double* c = coef + q * coef_ld;
    for (int i = threadIdx.x; i < n; i += 256) {
        if (s[0] < 0) {
            out[q * ldr + i] = __longlong_as_double(0x7FF8000000000000LL);
            continue;
        }
        double p = c[0];
        for (int j = 0; j < D; j++) p = fma(c[j + 1], F[(int64_t)s[j] * ldf + i], p);
        out[q * ldr + i] = y[i] - p;
    }
}

// ------------------------------------------------ batched kernel entries
struct PrepArgs {
    int n, S, ldz, ldg;
    const double* F;
    int64_t ldf;
    const double* y;
    double *Z, *G, *yy;
    double* dg;               // G's diagonal, contiguous (written by the Gram kernel)
    uint32_t* clr;            // words the standardising kernel clears (the band's first-round counters)
    int64_t clr_n32;
    double4* E;               // D = 3 factor table
    int lde;
    const double* theta;      // D = 3: shift th of the table's Q_ab
};

// grid (row blocks of 4, problems)
__global__ __launch_bounds__(256) void k_l0_prep(ctab<PrepArgs> A) {
    const PrepArgs& a = tab(A, blockIdx.y);
    DSC_GLOBAL(a.F); DSC_GLOBAL(a.y); DSC_GLOBAL(a.Z); DSC_GLOBAL(a.yy);
    for (int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x; w < a.clr_n32; w += (int64_t)gridDim.x * 256)
        a.clr[w] = 0u;
    if ((int)blockIdx.x * 4 > a.S) return;
    d_l0_prep(a.n, a.S, a.F, a.ldf, a.y, a.ldz, a.Z, a.yy);
}

// OMP set-up for one problem: grid (row blocks of 4).  Standardised rows,
// their squared norms, and (block 0) the starting active set.
// Warm start: the rows of init that lie in 0..S-1, first occurrences only,
// in order; a missing or repeated row leaves the model one row shorter.
__global__ __launch_bounds__(256) void k_omp_prep(int n, int S, const double* __restrict__ F,
                                                  int64_t ldf, const double* __restrict__ y, int ldz,
                                                  double* __restrict__ Z, double* __restrict__ yy,
                                                  double* __restrict__ nrm,
                                                  int32_t* __restrict__ active, int D_max,
                                                  const int32_t* __restrict__ init, int n_init,
                                                  int32_t* __restrict__ nact) {
    d_l0_prep(n, S, F, ldf, y, ldz, Z, yy, nrm);
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int c = 0;
    for (int q = 0; q < n_init; q++) {
        const int r = init[q];
        bool keep = r >= 0 && r < S;
        for (int t = 0; t < c; t++) keep = keep && active[t] != r;
        if (keep) active[c++] = r;
    }
    for (int q = c; q < D_max; q++) active[q] = -1;
    *nact = c;
}

// grid (8 x the tiles of the busiest XCD, 1, problems).  Block p runs on
// XCD p mod 8; XCD x takes the tile rows x, x + 8, x + 16, ... of the upper
// triangle and walks its tiles column by column, so its band of Z rows
// stays in its L2 while each column tile is read once.
__global__ __launch_bounds__(256) void k_gram(ctab<PrepArgs> A) {
    const PrepArgs& a = tab(A, blockIdx.z);
    DSC_GLOBAL(a.Z); DSC_GLOBAL(a.G); DSC_GLOBAL(a.dg);
    const int M = a.S + 1;
    const int gt = (M + 31) / 32;
    const int x = blockIdx.x & 7, l = blockIdx.x >> 3;
    int bj = x, cum = 0;
    for (; bj < gt; bj++) {                   // column bj holds rows x + 8m <= bj
        const int c = (bj - x) / 8 + 1;
        if (l < cum + c) break;
        cum += c;
    }
    if (bj >= gt) return;                     // (block-uniform) past this XCD's tiles
    const int bi = x + 8 * (l - cum);
    d_gram(M, a.ldz, a.ldz, a.Z, a.G, a.ldg, 32 * bi, 32 * bj, a.dg);
}

// Blocks per XCD of the Gram launch for gt tile rows (XCD 0 has the most).
static int gram_xcd_tiles(int gt) {
    int c = 0;
    for (int bj = 0; bj < gt; bj++) c += bj / 8 + 1;
    return c;
}

// grid (a blocks, b rows, problems)
__global__ __launch_bounds__(256) void k_sw3_table(ctab<PrepArgs> A) {
    const PrepArgs& a = tab(A, blockIdx.z);
    DSC_GLOBAL(a.G); DSC_GLOBAL(a.dg); DSC_GLOBAL(a.E); DSC_GLOBAL(a.theta);
    if ((int)blockIdx.y >= a.S || (int)blockIdx.x * 256 >= a.lde) return;
    d_sw3_table(a.G, a.ldg, a.S, a.dg, a.E, a.lde, *a.theta);
}

struct RefitArgs {
    int n, D, m;
    const double* F;
    int64_t ldf;
    const double* y;
    const int4* band;
    const unsigned long long* bcnt;
    int64_t bcap;
    double *scratch, *brss, *bcoef;
    const int64_t* ids;
    const double* yy;
    uint8_t* taken;
    int32_t* out_sub;
    double *out_rmse, *out_coef;
    int32_t* chosen;
    double* out_resid;
    int64_t ldr;
    int sub_ld, coef_ld;      // row strides of out_sub and out_coef
};

// Offsets of every problem's band in one merged work list: boff[p] =
// sum of min(count, capacity) over problems before p (one block).
__global__ __launch_bounds__(256) void k_band_offsets(ctab<RefitArgs> A, int na, int64_t* __restrict__ boff) {
    __shared__ int64_t part[256];
    const int per = (na + 255) / 256;
    const int b0 = threadIdx.x * per, b1 = min(na, b0 + per);
    int64_t s = 0;
    for (int b = b0; b < b1; b++) {
        const RefitArgs& a = tab(A, b);
        s += min((int64_t)*a.bcnt, a.bcap);
    }
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t acc = 0;
        for (int t = 0; t < 256; t++) {
            const int64_t v = part[t];
            part[t] = acc;
            acc += v;
        }
        boff[na] = acc;
    }
    __syncthreads();
    int64_t acc = part[threadIdx.x];
    for (int b = b0; b < b1; b++) {
        boff[b] = acc;
        const RefitArgs& a = tab(A, b);
        acc += min((int64_t)*a.bcnt, a.bcap);
    }
}

constexpr int REFIT_LDS_NA = 256;     // problems whose band offsets the refit forms itself

// QR refit of every band entry of every problem: persistent workgroups
// take entries from the merged list, so one problem with a large band is
// spread over the whole GPU.
__global__ __launch_bounds__(256) void k_refit_all(ctab<RefitArgs> A, int na,
                                                   const int64_t* __restrict__ boff,
                                                   double* __restrict__ scratch, int64_t sld,
                                                   int use_lds) {
    __shared__ double coef[DISCOVER_MAX_D + 1];
    __shared__ double rss;
    extern __shared__ double dsm[];              // sld doubles when use_lds
    double* S = scratch + (int64_t)blockIdx.x * sld;
    // up to REFIT_LDS_NA problems, every block forms the band offsets itself
    // (an exclusive sum of the band sizes) instead of a launch of their own
    __shared__ int64_t lboff[REFIT_LDS_NA + 1];
    if (na <= REFIT_LDS_NA) {
        if (threadIdx.x < na) {
            const RefitArgs& a = tab(A, threadIdx.x);
            lboff[threadIdx.x + 1] = min((int64_t)*a.bcnt, a.bcap);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            lboff[0] = 0;
            for (int b = 1; b <= na; b++) lboff[b] += lboff[b - 1];
        }
        __syncthreads();
        boff = lboff;
    }
    const int64_t total = boff[na];
    for (int64_t e = blockIdx.x; e < total; e += gridDim.x) {
        int lo = 0, hi = na;                     // boff[lo] <= e < boff[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) / 2;
            if (boff[mid] <= e) lo = mid; else hi = mid;
        }
        const RefitArgs& a = tab(A, lo);
        DSC_GLOBAL(a.F); DSC_GLOBAL(a.y); DSC_GLOBAL(a.band); DSC_GLOBAL(a.brss); DSC_GLOBAL(a.bcoef);
        const int64_t le = e - boff[lo];
        const int4 s = a.band[le];
        const int idx[3] = {s.x, s.y, s.z};
        if (use_lds) block_lsq(a.n, a.D, idx, a.F, a.ldf, a.y, dsm, coef, &rss, nullptr);
        else block_lsq(a.n, a.D, idx, a.F, a.ldf, a.y, S, coef, &rss, nullptr);
        if (threadIdx.x == 0) {
            a.brss[le] = rss;
            for (int j = 0; j <= a.D; j++) a.bcoef[le * (a.D + 1) + j] = coef[j];
        }
        __syncthreads();
    }
}

// grid (problems): the m best models of each problem's band (one thread),
// then their residuals when asked for (the whole block).
__global__ __launch_bounds__(256) void k_rank_models(ctab<RefitArgs> A) {
    const RefitArgs& a = tab(A, blockIdx.x);
    DSC_GLOBAL(a.F); DSC_GLOBAL(a.y); DSC_GLOBAL(a.band); DSC_GLOBAL(a.bcnt); DSC_GLOBAL(a.scratch); DSC_GLOBAL(a.brss); DSC_GLOBAL(a.bcoef); DSC_GLOBAL(a.ids); DSC_GLOBAL(a.yy); DSC_GLOBAL(a.taken); DSC_GLOBAL(a.out_sub); DSC_GLOBAL(a.out_rmse); DSC_GLOBAL(a.out_coef); DSC_GLOBAL(a.chosen); DSC_GLOBAL(a.out_resid);
    d_rank_models(a.band, a.brss, a.bcoef, a.bcnt, a.bcap, a.D, a.m, a.ids, a.yy, a.n, a.taken,
                  a.out_sub, a.out_rmse, a.out_coef, a.chosen, a.sub_ld, a.coef_ld);
    if (!a.out_resid) return;
    __syncthreads();                             // the chosen models are written
    for (int q = 0; q < a.m; q++)
        d_resid(q, a.n, a.D, a.F, a.ldf, a.y, a.out_sub, a.out_coef, a.out_resid, a.ldr, a.sub_ld,
                a.coef_ld);
}

// ------------------------------------------------------------------ OMP
// g_j = |Z_j . r| for inactive rows (one wave per row).
__global__ __launch_bounds__(256) void k_omp_corr(int n, int S, const double* __restrict__ Z, int ldz,
                                                  const double* __restrict__ r,
                                                  const int32_t* __restrict__ active,
                                                  const int32_t* __restrict__ nact,
                                                  double* __restrict__ g) {
    const int j = blockIdx.x * 4 + wave_id();
    const int lane = threadIdx.x & 63;
    if (j >= S) return;
    double s = 0.0;
    for (int i = lane; i < n; i += 64) s += Z[(int64_t)j * ldz + i] * r[i];
    s = fabs(wave_sum(s));
    if (lane == 0) {
        bool act = false;
        for (int q = 0; q < *nact; q++) act |= active[q] == j;
        double zz = 0.0;
        (void)zz;
        g[j] = act ? -1.0 : s;
    }
}

// One OMP step in one workgroup.  With g given, first the argmax of g by
// (-g, ID) over the non-constant rows is appended to the active list (none
// when every row is taken); then the least-squares fit on the active rows,
// its residual r and, with out_rmse given, sqrt(RSS / n).
__global__ __launch_bounds__(256) void k_omp_fit(int n, const double* __restrict__ F, int64_t ldf,
                                                 const double* __restrict__ y,
                                                 int32_t* __restrict__ active,
                                                 int32_t* __restrict__ nact,
                                                 double* __restrict__ A, double* __restrict__ coef,
                                                 double* __restrict__ rss, double* __restrict__ r,
                                                 int use_lds, int S, const double* __restrict__ g,
                                                 const int64_t* __restrict__ ids,
                                                 const double* __restrict__ rownorm,
                                                 double* __restrict__ out_rmse) {
    __shared__ int idx[DISCOVER_MAX_D];
    __shared__ double cf[DISCOVER_MAX_D + 1];
    __shared__ double rs;
    __shared__ double bg[256];
    __shared__ int bj[256];
    __shared__ int s_d;
    extern __shared__ double dsm[];              // (D_max + 2) * n doubles when use_lds
    if (threadIdx.x == 0) s_d = *nact;
    __syncthreads();
    const int d0 = s_d;
    int pick = -1;
    if (g) {
        double best = -2.0;
        int bi = -1;
        // four rows per thread are loaded before any is compared, so the
        // loads overlap; rows are visited in increasing j as before
        for (int j0 = threadIdx.x; j0 < S; j0 += 4 * 256) {
            double nv[4], gv[4];
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int j = j0 + q * 256;
                nv[q] = j < S ? rownorm[j] : 0.0;
                gv[q] = j < S ? g[j] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int j = j0 + q * 256;
                if (!(nv[q] > 0.0)) continue;
                const double v = gv[q];
                if (v > best || (v == best && bi >= 0 && ids[j] < ids[bi])) {
                    best = v;
                    bi = j;
                }
            }
        }
        bg[threadIdx.x] = best;
        bj[threadIdx.x] = bi;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (threadIdx.x < o) {
                const double v = bg[threadIdx.x + o];
                const int j = bj[threadIdx.x + o];
                const int cj = bj[threadIdx.x];
                if (j >= 0 && (cj < 0 || v > bg[threadIdx.x] || (v == bg[threadIdx.x] && ids[j] < ids[cj]))) {
                    bg[threadIdx.x] = v;
                    bj[threadIdx.x] = j;
                }
            }
            __syncthreads();
        }
        pick = bj[0] >= 0 && bg[0] >= 0.0 ? bj[0] : -1;
        if (threadIdx.x == 0 && pick >= 0) {
            active[d0] = pick;
            *nact = d0 + 1;
        }
    }
    const int d = pick >= 0 ? d0 + 1 : d0;
    if (threadIdx.x < d) idx[threadIdx.x] = threadIdx.x < d0 ? active[threadIdx.x] : pick;
    __syncthreads();
    if (use_lds) block_lsq(n, d, idx, F, ldf, y, dsm, cf, &rs, r);
    else block_lsq(n, d, idx, F, ldf, y, A, cf, &rs, r);
    if (threadIdx.x == 0) {
        for (int j = 0; j <= d; j++) coef[j] = cf[j];
        *rss = rs;
        if (out_rmse) *out_rmse = sqrt(rs / n);
    }
}

// ================================================================== host
// D = 3 blocks (16 consecutive a, 64 consecutive c, a range of b).  A block
// reads the factor-table tile E[b range][a rows] (32 bytes per (a, b)) and
// the G tile [b range][c columns] (8 bytes per (b, c)).  Groups of 16 a rows
// are dealt to the 8 XCDs by longest-processing-time on their total work,
// and block p of the grid runs on XCD p mod 8, so each XCD reads only its
// own rows of E (72 MB at S = 1500, which every XCD read in full when the
// XCDs were given column groups instead).  The b ranges are cut on a common
// grid of 96 rows, so blocks of different a groups with the same (b range,
// c columns) read the same G tile; each XCD runs its blocks in (b range, c
// columns, a group) order, so that tile and the E tiles of its a groups for
// that b range are in its L2 when the next blocks need them.  The C(1500, 3)
// sweep has about 7600 blocks, some 30 per CU.
constexpr int SW3_BMAX = 96;          // b iterations per block (and the grid of b ranges)

static std::vector<int4> sweep3_blocks(int S) {
    const int ngrp = (S + 15) / 16;
    std::vector<std::vector<int4>> per_grp(ngrp);
    std::vector<int64_t> gwork(ngrp, 0);
    for (int cg = 0; cg < (S + 63) / 64; cg++) {
        const int c0 = 64 * cg, ch = std::min(S, c0 + 64);
        for (int a0 = 0; a0 < S - 2 && a0 + 2 < ch; a0 += 16) {
            const int bend = std::min(S - 1, c0 + 63);
            const int g = a0 / 16;
            for (int b0 = a0 + 1; b0 < bend;) {
                const int b1 = std::min(bend, (b0 / SW3_BMAX + 1) * SW3_BMAX);
                per_grp[g].push_back(make_int4(a0, c0, b0, b1));
                gwork[g] += (int64_t)(b1 - b0) * 16;
                b0 = b1;
            }
        }
    }
    std::vector<int> order(ngrp);
    for (int g = 0; g < ngrp; g++) order[g] = g;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return gwork[x] > gwork[y]; });
    std::vector<std::vector<int4>> q(8);
    std::vector<int64_t> xwork(8, 0);
    for (int g : order) {
        const int x = (int)(std::min_element(xwork.begin(), xwork.end()) - xwork.begin());
        xwork[x] += gwork[g];
        q[x].insert(q[x].end(), per_grp[g].begin(), per_grp[g].end());
    }
    size_t mx = 0;
    for (auto& v : q) {
        std::stable_sort(v.begin(), v.end(), [](const int4& x, const int4& y) {
            const int bx = x.z / SW3_BMAX, by = y.z / SW3_BMAX;
            if (bx != by) return bx < by;
            if (x.y != y.y) return x.y < y.y;
            return x.x < y.x;
        });
        mx = std::max(mx, v.size());
    }
    std::vector<int4> out;
    out.reserve(mx * 8);
    for (size_t i = 0; i < mx; i++)
        for (int x = 0; x < 8; x++) out.push_back(i < q[x].size() ? q[x][i] : make_int4(-1, 0, 0, 0));
    return out;
}

// Sweep work items of one subspace size (cached: they depend on S and D only).
struct L0Items {
    std::vector<int2> items;      // D = 1, 2
    std::vector<int4> items3;     // D = 3
};

static std::shared_ptr<L0Items> l0_items(discover_ctx* ctx, int S, int D) {
    const std::string key = "l0items:" + std::to_string(S) + ":" + std::to_string(D);
    auto it = ctx->plans.find(key);
    if (it != ctx->plans.end()) return std::static_pointer_cast<L0Items>(it->second);
    auto P = std::make_shared<L0Items>();
    if (D == 1) {
        for (int a0 = 0; a0 < S; a0 += 64) P->items.push_back(make_int2(0, a0));
    } else if (D == 2) {
        for (int a = 0; a < S - 1; a++)
            for (int b0 = a + 1; b0 < S; b0 += 64) P->items.push_back(make_int2(a, b0));
    } else {
        P->items3 = sweep3_blocks(S);
    }
    ctx->evict_plans(64);
    ctx->plans[key] = P;
    return P;
}

struct BandMemo {
    std::vector<int64_t> cap;
};

static size_t band_arena_bytes(const std::vector<int>& act, const std::vector<int64_t>& cap, int D,
                               int m, std::vector<std::vector<size_t>>* offs) {
    Arena br;
    for (int b : act) {
        const size_t c = (size_t)cap[b];
        std::vector<size_t> v;
        v.push_back(br.add(c * 16));                                   // band
        v.push_back(br.add(c * 16));                                   // pairs
        v.push_back(br.add(c * 8));                                    // brss
        v.push_back(br.add(c * (D + 1) * 8));                          // bcoef
        v.push_back(br.add(c));                                        // taken
        v.push_back(br.add((size_t)m * 4));                            // chosen
        v.push_back(br.add(64));                                       // bcnt, pcnt, st[2], sel[4]
        v.push_back(br.add(8192 * 4));                                 // hist (two levels)
        if (offs) offs->push_back(v);
    }
    return br.total;
}

// Exhaustive L0 of every problem of a call, one launch per phase.
// Stats of a call that did not wait for the stream (one thread per problem).
__global__ __launch_bounds__(256) void k_l0_stats(ctab<BandCheck> B, ctab<discover_l0_stats> base, int nb,
                                                  discover_l0_stats* __restrict__ out) {
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= nb) return;
    const BandCheck& c = tab(B, b);
    DSC_GLOBAL(c.cnt);
    discover_l0_stats s = tab(base, b);
    s.n_band = (int64_t)c.cnt[0];
    s.status = band_status(c, c.cnt);
    out[b] = s;
}

void l0_batch(discover_ctx* ctx, const discover_l0_problem* probs, int nb, int D, int m,
              const std::vector<L0Out>& outs, std::vector<discover_l0_stats>& stats,
              hipStream_t st, std::vector<BandCheck>* checks, discover_l0_stats* dev_stats) {
    const bool devmode = ctx->capturing || ctx->nosync;
    // 1. layout
    std::vector<std::shared_ptr<L0Items>> its(nb);
    std::vector<PrepArgs> pa(nb);
    std::vector<int64_t> ni(nb), nblk(nb), lane0(nb), blk0(nb);
    const int per = D == 3 ? 4 * SW3_A * 64 : 64;
    Arena ar;
    std::vector<std::vector<size_t>> o(nb);
    int64_t tot_blk = 0, tot_items = 0, tot_items3 = 0, tot_lanes = 0;
    int Smax = 0, ldemax = 0;
    for (int b = 0; b < nb; b++) {
        const discover_l0_problem& pb = probs[b];
        its[b] = l0_items(ctx, pb.S, D);
        ni[b] = D == 3 ? (int64_t)its[b]->items3.size() : (int64_t)its[b]->items.size();
        nblk[b] = D == 3 ? ni[b] : cdiv(ni[b], 4);
        blk0[b] = tot_blk;
        tot_blk += nblk[b];
        lane0[b] = tot_lanes;
        tot_lanes += ni[b] * per;
        PrepArgs& a = pa[b];
        a = PrepArgs{};
        a.n = pb.n; a.S = pb.S; a.ldz = (int)cdiv(pb.n, 16) * 16; a.ldg = (int)cdiv(pb.S + 1, 2) * 2;
        a.F = pb.F; a.ldf = pb.ldf; a.y = pb.y;
        a.lde = D == 3 ? (int)cdiv(pb.S + 16, 4) * 4 : 0;
        auto& v = o[b];
        v.push_back(ar.add((size_t)(pb.S + 1) * a.ldz * 8));               // Z
        v.push_back(ar.add((size_t)(pb.S + 1) * a.ldg * 8));               // G
        v.push_back(ar.add(8));                                            // yy
        v.push_back(ar.add(D == 3 ? (size_t)pb.S * a.lde * 32 : 32));      // E
        v.push_back(ar.add(8));                                            // th
        v.push_back(ar.add(D == 3 ? (size_t)pb.S * 8 : 8));                // row values
        v.push_back(ar.add(8));                                            // lane-list count
        v.push_back(ar.add((size_t)(pb.S + 1) * 8));                       // G's diagonal
        Smax = std::max(Smax, pb.S);
        ldemax = std::max(ldemax, a.lde);
        if (D == 3) tot_items3 += ni[b]; else tot_items += ni[b];
    }
    char* base = (char*)ctx->raw("l0_arena", ar.total);
    for (int b = 0; b < nb; b++) {
        pa[b].Z = (double*)(base + o[b][0]);
        pa[b].G = (double*)(base + o[b][1]);
        pa[b].yy = (double*)(base + o[b][2]);
        pa[b].E = (double4*)(base + o[b][3]);
        pa[b].theta = (const double*)(base + o[b][4]);
        pa[b].dg = (double*)(base + o[b][7]);
    }
    // the band's first-round arena is laid out now, so that its counters and
    // radix histograms are cleared by the standardising kernel
    std::vector<int64_t> cap(nb, std::max<int64_t>(1 << 16, 256 * (int64_t)m));
    std::string ck((const char*)&D, sizeof D);
    ck.append((const char*)&m, sizeof m);
    for (int b = 0; b < nb; b++) {                      // the call's shape, not its data
        const int32_t f[2] = {probs[b].n, probs[b].S};
        ck.append((const char*)f, sizeof f);
    }
    auto mit = ctx->batches.find("band" + ck);
    if (mit != ctx->batches.end()) {
        const BandMemo& bm = *std::static_pointer_cast<BandMemo>(mit->second);
        if ((int)bm.cap.size() == nb) cap = bm.cap;
    }
    std::vector<int> act(nb);
    for (int b = 0; b < nb; b++) act[b] = b;
    {
        std::vector<std::vector<size_t>> bo0;
        char* bb0 = (char*)ctx->raw("l0_band_arena" + ctx->tag, band_arena_bytes(act, cap, D, m, &bo0));
        for (int b = 0; b < nb; b++) {                  // counters and histograms are adjacent
            pa[b].clr = (uint32_t*)(bb0 + bo0[b][6]);
            pa[b].clr_n32 = (int64_t)(bo0[b][7] + 8192 * 4 - bo0[b][6]) / 4;
        }
    }
    const ctab<PrepArgs> dpa = ct(ctx->upload("l0_prep", pa, st));
    const bool bound = D == 3 && m <= SW3_MMAX;
    // 2. Gram matrices (and the D = 3 factor tables)
    {
        KTimer kt(ctx, st, "l0_gram");
        k_l0_prep<<<dim3((unsigned)cdiv(Smax + 1, 4), nb), 256, 0, st>>>(dpa);
        const int gt = (int)cdiv(Smax + 1, 32);
        k_gram<<<dim3(8u * (unsigned)gram_xcd_tiles(gt), 1, nb), 256, 0, st>>>(dpa);
        check_launch("k_gram");
    }
    if (D == 3) {
        KTimer kt(ctx, st, "l0_table");
        if (bound) {                            // the lower bound th of each problem
            std::vector<ThetaArgs> ta(nb);
            for (int b = 0; b < nb; b++)
                ta[b] = ThetaArgs{pa[b].G, pa[b].dg, pa[b].ldg, probs[b].S, (double*)(base + o[b][5]),
                                  (double*)(base + o[b][4]), (unsigned long long*)(base + o[b][6])};
            const ctab<ThetaArgs> dta = ct(ctx->upload("l0_theta", ta, st));
            k_sw3_rows<<<dim3((unsigned)Smax, nb), 256, 0, st>>>(dta);
            k_sw3_theta<<<nb, 256, 0, st>>>(dta, m);
        } else {                                // unbounded: th = 0
            std::vector<FillSeg> fz;
            for (int b = 0; b < nb; b++) fz.push_back(fill_seg(base + o[b][4], 8, 0u));
            fill_all(ctx, "l0_theta_fill", fz, st);
        }
        k_sw3_table<<<dim3((unsigned)cdiv(ldemax, 256), (unsigned)Smax, nb), 256, 0, st>>>(dpa);
        check_launch("k_sw3_table");
    }
    // 3. sweep over the merged work items
    std::vector<int2> items;
    std::vector<int4> items3;
    std::vector<int> bprob;
    std::vector<int64_t> item_off(nb);
    for (int b = 0; b < nb; b++) {
        item_off[b] = D == 3 ? (int64_t)items3.size() : (int64_t)items.size();
        if (D == 3) items3.insert(items3.end(), its[b]->items3.begin(), its[b]->items3.end());
        else items.insert(items.end(), its[b]->items.begin(), its[b]->items.end());
        bprob.insert(bprob.end(), (size_t)nblk[b], b);
    }
    const int2* d_items = D == 3 ? nullptr : ctx->upload("l0_items", items, st);
    const int4* d_items3 = D == 3 ? ctx->upload("l0_items3", items3, st) : nullptr;
    const int* d_bprob = ctx->upload("l0_bprob", bprob, st);
    double* lane_q = ctx->buf<double>("l0_laneq", (size_t)tot_lanes);
    // bounded D = 3: listed lanes (indices here, values in lane_q's slice)
    int32_t* lane_idx = bound ? ctx->buf<int32_t>("l0_laneidx", (size_t)tot_lanes) : nullptr;
    std::vector<SweepArgs> sa(nb);
    for (int b = 0; b < nb; b++) {
        SweepArgs& g = sa[b];
        g = SweepArgs{};
        g.G = pa[b].G; g.dg = pa[b].dg; g.ldg = pa[b].ldg; g.S = probs[b].S; g.D = D; g.E = pa[b].E; g.lde = pa[b].lde;
        g.items = d_items ? d_items + item_off[b] : nullptr;
        g.items3 = d_items3 ? d_items3 + item_off[b] : nullptr;
        g.n_items = ni[b];
        g.lane_q = lane_q + lane0[b];
        g.item0 = blk0[b];
        g.theta = pa[b].theta;
        if (bound) {
            g.lidx = lane_idx + lane0[b];
            g.lval = g.lane_q;
            g.lcnt = (unsigned long long*)(base + o[b][6]);
        }
    }
    const ctab<SweepArgs> dsa = ct(ctx->upload("l0_sweep", sa, st));
    {
        KTimer kt(ctx, st, D == 3 ? "l0_sweep3" : "l0_sweep");
        if (tot_blk) {
            if (D == 1) k_sweep1<<<(unsigned)tot_blk, 256, 0, st>>>(dsa, d_bprob);
            else if (D == 2) k_sweep2<<<(unsigned)tot_blk, 256, 0, st>>>(dsa, d_bprob);
            else if (bound) k_sweep3<true><<<(unsigned)tot_blk, 256, 0, st>>>(dsa, d_bprob);
            else k_sweep3<false><<<(unsigned)tot_blk, 256, 0, st>>>(dsa, d_bprob);
        }
        check_launch("k_sweep");
    }
    // 4. band: radix selection of the m-th best lane, expansion, QR refit, ranking
    constexpr int NREFIT = 2048;                // persistent refit workgroups (all problems)
    int nmax = 0;
    for (int b = 0; b < nb; b++) nmax = std::max(nmax, probs[b].n);
    const int64_t sld = (int64_t)(D + 2) * nmax;
    double* rscratch = ctx->buf<double>("l0_refit_scratch", (size_t)NREFIT * sld);
    int64_t* boff = ctx->buf<int64_t>("l0_boff" + ctx->tag, (size_t)nb + 1);
    bool prefilled = true;                      // the first round's counters: cleared by k_l0_prep
    std::vector<BandCheck> bcl;
    while (!act.empty()) {
        const int na = (int)act.size();
        std::vector<std::vector<size_t>> bo;
        const size_t btot = band_arena_bytes(act, cap, D, m, &bo);
        char* bb = (char*)ctx->raw("l0_band_arena" + ctx->tag, btot);
        std::vector<BandArgs> ba(na);
        std::vector<RadixArgs> ra(na);
        std::vector<RefitArgs> fa(na);
        std::vector<FillSeg> fills;
        int64_t lanes_max = 1;
        for (int q = 0; q < na; q++) {
            const int b = act[q];
            const auto& v = bo[q];
            char* misc = bb + v[6];
            BandArgs& g = ba[q];
            g = BandArgs{};
            g.G = pa[b].G; g.dg = pa[b].dg; g.ldg = pa[b].ldg; g.S = probs[b].S; g.D = D; g.E = pa[b].E; g.lde = pa[b].lde;
            g.items = sa[b].items; g.items3 = sa[b].items3;
            g.n_lanes = ni[b] * per;
            g.lane_q = sa[b].lane_q;
            g.sel = (uint32_t*)(misc + 32); g.st = (int64_t*)(misc + 16); g.hist = (const uint32_t*)(bb + v[7]);
            g.band = (int4*)(bb + v[0]); g.bcnt = (unsigned long long*)misc; g.bcap = cap[b];
            g.pairs = (int4*)(bb + v[1]); g.pcnt = (unsigned long long*)misc + 1; g.pcap = cap[b];
            g.theta = pa[b].theta;
            g.lidx = sa[b].lidx; g.lval = sa[b].lval; g.lcnt = sa[b].lcnt;
            ra[q] = RadixArgs{g.lidx ? g.lval : g.lane_q, g.n_lanes, m, (uint32_t*)(bb + v[7]),
                              (uint32_t*)(misc + 32), (int64_t*)(misc + 16), g.lidx ? g.lcnt : nullptr};
            fills.push_back(fill_seg(misc, 48, 0u));              // bcnt, pcnt, st, sel
            fills.push_back(fill_seg(bb + v[7], 8192 * 4, 0u));   // radix histograms
            lanes_max = std::max(lanes_max, g.n_lanes);
            RefitArgs& f = fa[q];
            f = RefitArgs{};
            f.n = probs[b].n; f.D = D; f.m = m; f.F = probs[b].F; f.ldf = probs[b].ldf; f.y = probs[b].y;
            f.band = g.band; f.bcnt = g.bcnt; f.bcap = cap[b];
            f.scratch = nullptr; f.brss = (double*)(bb + v[2]); f.bcoef = (double*)(bb + v[3]);
            f.ids = probs[b].ids; f.yy = pa[b].yy; f.taken = (uint8_t*)(bb + v[4]);
            f.out_sub = outs[b].sub; f.sub_ld = outs[b].sub_ld; f.out_rmse = outs[b].rmse;
            f.out_coef = outs[b].coef; f.coef_ld = outs[b].coef_ld; f.chosen = (int32_t*)(bb + v[5]);
            f.out_resid = outs[b].resid;
            f.ldr = outs[b].ldr;
        }
        if (!prefilled) fill_all(ctx, "l0_fills", fills, st);
        prefilled = false;
        const ctab<BandArgs> dba = ct(ctx->upload("l0_band", ba, st));
        const RadixArgs* dra = ctx->upload("l0_radix", ra, st);
        const ctab<RefitArgs> dfa = ct(ctx->upload("l0_refit", fa, st));
        {
            KTimer kt(ctx, st, "l0_band");
            // the bounded sweep's lane lists are short: fewer blocks (grid-strided)
            const int64_t scan = bound ? std::min<int64_t>(lanes_max, 1 << 16) : lanes_max;
            radix_select(dra, na, scan, st);
            const unsigned lb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(std::max(8, 1024 / na),
                                                                                cdiv(scan, 256)));
            k_band_lanes<<<dim3(lb, na), 256, 0, st>>>(dba);
            if (D == 3) k_band_expand3<<<dim3((unsigned)std::max(8, 1024 / na), na), 256, 0, st>>>(dba);
            check_launch("k_band");
        }
        {
            KTimer kt(ctx, st, "l0_refit");
            if (na > REFIT_LDS_NA) k_band_offsets<<<1, 256, 0, st>>>(dfa, na, boff);
            const int rl = sld * (int64_t)sizeof(double) <= 65536 ? 1 : 0;   // QR columns in LDS
            k_refit_all<<<NREFIT, 256, rl ? (size_t)sld * sizeof(double) : 0, st>>>(dfa, na, boff, rscratch,
                                                                                   sld, rl);
            check_launch("k_refit");
        }
        k_rank_models<<<na, 256, 0, st>>>(dfa);
        check_launch("k_rank_models");
        if (devmode) {                          // capacities are checked on the device
            for (int q = 0; q < na; q++) bcl.push_back(BandCheck{ba[q].bcnt, cap[act[q]]});
            if (checks) checks->insert(checks->end(), bcl.begin(), bcl.end());
            break;
        }
        std::vector<unsigned long long> cnt(2 * (size_t)na);
        for (int q = 0; q < na; q++)
            DSC_HIP(hipMemcpyAsync(&cnt[2 * q], ba[q].bcnt, 16, hipMemcpyDeviceToHost, st));
        DSC_HIP(hipStreamSynchronize(st));
        std::vector<int> next;
        for (int q = 0; q < na; q++) {
            const int b = act[q];
            if ((int64_t)cnt[2 * q] <= cap[b] && (int64_t)cnt[2 * q + 1] <= cap[b]) {
                stats[b].n_band = (int64_t)cnt[2 * q];
                if (cnt[2 * q] == 0) DSC_FAIL(DISCOVER_E_NUMERIC, "problem %d: no non-singular %d-subset", b, D);
                continue;
            }
            cap[b] = (int64_t)std::max(cnt[2 * q], cnt[2 * q + 1]) + 1024;
            next.push_back(b);
        }
        act.swap(next);
    }
    if (devmode) {
        if (dev_stats) {
            k_l0_stats<<<(unsigned)cdiv(nb, 256), 256, 0, st>>>(ct(ctx->upload("l0_stats_chk", bcl, st)),
                                                               ct(ctx->upload("l0_stats_base", stats, st)),
                                                               nb, dev_stats);
            check_launch("k_l0_stats");
        }
        return;
    }
    std::vector<int> all(nb);
    for (int b = 0; b < nb; b++) all[b] = b;
    ctx->raw("l0_band_arena" + ctx->tag, band_arena_bytes(all, cap, D, m, nullptr));
    auto bm = std::make_shared<BandMemo>();
    bm->cap = cap;
    if (ctx->batches.size() >= 256) ctx->batches.clear();
    ctx->batches["band" + ck] = bm;
}

}  // namespace dsc

static int64_t binom(int64_t n, int k) {
    if (k < 0 || n < k) return 0;
    int64_t r = 1;
    for (int i = 0; i < k; i++) r = r * (n - i) / (i + 1);
    return r;
}

extern "C" discover_status discover_l0_fit(discover_ctx* ctx, const discover_l0_problem* probs,
                                           int32_t n_problems, int32_t D, int32_t m,
                                           int32_t* out_subsets, double* out_rmse, double* out_coef,
                                           double* out_resid, int64_t ldr,
                                           discover_l0_stats* out_stats, void* stream) {
    using namespace dsc;
    return guarded([&] {
        DSC_REQUIRE(ctx && probs && n_problems >= 1, "ctx/probs");
        DSC_REQUIRE(n_problems <= 65535, "n_problems = %d > 65535", n_problems);
        DSC_REQUIRE(D >= 1 && D <= 3, "D = %d outside 1..3", D);
        DSC_REQUIRE(m >= 1 && m <= 64, "m = %d outside 1..64", m);
        DSC_REQUIRE(out_subsets && out_rmse && out_coef, "outputs required");
        for (int b = 0; b < n_problems; b++) {
            const discover_l0_problem& p = probs[b];
            DSC_REQUIRE(p.n >= D + 2, "problem %d: n = %d < D + 2", b, p.n);
            DSC_REQUIRE(p.S >= D && p.S < 65536, "problem %d: S = %d", b, p.S);
            DSC_REQUIRE(p.F && p.ids && p.y && p.ldf >= p.n, "problem %d: F/ids/y/ldf", b);
            DSC_REQUIRE(!out_resid || ldr >= p.n, "problem %d: ldr < n", b);
        }
        DSC_HIP(hipSetDevice(ctx->device));
        hipStream_t st = (hipStream_t)stream;
        std::vector<discover_l0_stats> stats(n_problems);
        for (int b = 0; b < n_problems; b++) {
            stats[b] = discover_l0_stats{};
            stats[b].n_subsets = binom(probs[b].S, D);
        }
        std::vector<L0Out> outs(n_problems);
        for (int b = 0; b < n_problems; b++)
            outs[b] = L0Out{out_subsets + (int64_t)b * m * D, D, out_rmse + (int64_t)b * m,
                            out_coef + (int64_t)b * m * (D + 1), D + 1,
                            out_resid ? out_resid + (int64_t)b * m * ldr : nullptr, ldr};
        const bool cap = stream_capturing(st);
        const bool dev = device_memory(out_stats);
        DSC_REQUIRE(!cap || dev, "a call captured into a graph reports its outcome in device memory: "
                                 "out_stats must be a device pointer");
        CallMode mode(ctx, cap, dev);
        l0_batch(ctx, probs, n_problems, D, m, outs, stats, st, nullptr, dev ? out_stats : nullptr);
        if (!dev) {
            DSC_HIP(hipStreamSynchronize(st));
            ctx->resolve_timing();
            if (out_stats)
                for (int b = 0; b < n_problems; b++) out_stats[b] = stats[b];
        }
    });
}

namespace dsc {

// Work buffers of one problem's OMP (byte sizes, each a multiple of 256):
// standardised rows Z, |y - mean|^2, active count, scores, row norms,
// residual (when the caller keeps none), QR columns, RSS.
static void omp_sizes(const discover_l0_problem& pb, int D_max, bool resid, size_t sz[8]) {
    auto r256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t ldz = (size_t)cdiv(pb.n, 16) * 16;
    sz[0] = r256((size_t)(pb.S + 1) * ldz * 8);
    sz[1] = 256;
    sz[2] = 256;
    sz[3] = r256((size_t)pb.S * 8);
    sz[4] = r256((size_t)pb.S * 8);
    sz[5] = resid ? 0 : r256((size_t)pb.n * 8);
    sz[6] = r256((size_t)(D_max + 2) * pb.n * 8);
    sz[7] = 256;
}

size_t omp_scratch_bytes(const discover_l0_problem* probs, int nb, int D_max, bool resid) {
    size_t t = 0;
    for (int b = 0; b < nb; b++) {
        size_t sz[8];
        omp_sizes(probs[b], D_max, resid, sz);
        for (size_t v : sz) t += v;
    }
    return t;
}

void omp_batch(discover_ctx* ctx, const discover_l0_problem* probs, int nb, int D_max,
               const int32_t* init_active, int n_init, int64_t init_ld, int32_t* out_active,
               double* out_coef, double* out_rmse, double* out_resid, int64_t ldr, hipStream_t st,
               char* scratch) {
    static const char* const names[8] = {"ompZ", "ompyy", "ompn", "ompg", "ompnrm", "ompr", "ompA", "omprss"};
    size_t off = 0;
    for (int b = 0; b < nb; b++) {
        const discover_l0_problem& pb = probs[b];
        const int ldz = (int)cdiv(pb.n, 16) * 16;
        size_t sz[8];
        omp_sizes(pb, D_max, out_resid != nullptr, sz);
        char* w[8] = {};
        for (int q = 0; q < 8; q++) {
            if (!sz[q]) continue;
            if (scratch) {                       // the caller's scratch, laid out in order
                w[q] = scratch + off;
                off += sz[q];
            } else {
                w[q] = (char*)ctx->raw(names[q] + std::to_string(b), sz[q]);
            }
        }
        double* Z = (double*)w[0];
        double* yy = (double*)w[1];
        int32_t* active = out_active + (int64_t)b * D_max;
        int32_t* nact = (int32_t*)w[2];
        double* g = (double*)w[3];
        double* nrm = (double*)w[4];
        double* r = out_resid ? out_resid + (int64_t)b * ldr : (double*)w[5];
        double* A = (double*)w[6];
        double* rss = (double*)w[7];
        double* coef = out_coef + (int64_t)b * (D_max + 1);
        // (no timer events in the scratch form: it creates nothing)
        std::unique_ptr<KTimer> kt(scratch ? nullptr : new KTimer(ctx, st, "omp"));
        k_omp_prep<<<(unsigned)cdiv(pb.S + 1, 4), 256, 0, st>>>(
            pb.n, pb.S, pb.F, pb.ldf, pb.y, ldz, Z, yy, nrm, active, D_max,
            n_init ? init_active + (int64_t)b * init_ld : nullptr, n_init, nact);
        // the QR's columns in LDS when they fit in 64 KB
        const size_t qr_bytes = (size_t)(D_max + 2) * pb.n * sizeof(double);
        const int qr_lds = qr_bytes <= 65536 ? 1 : 0;
        const size_t dyn = qr_lds ? qr_bytes : 0;
        k_omp_fit<<<1, 256, dyn, st>>>(pb.n, pb.F, pb.ldf, pb.y, active, nact, A, coef, rss, r, qr_lds,
                                       pb.S, nullptr, pb.ids, nrm, n_init < D_max ? nullptr : out_rmse + b);
        for (int step = n_init; step < D_max; step++) {
            k_omp_corr<<<(unsigned)cdiv(pb.S, 4), 256, 0, st>>>(pb.n, pb.S, Z, ldz, r, active,
                                                                nact, g);
            k_omp_fit<<<1, 256, dyn, st>>>(pb.n, pb.F, pb.ldf, pb.y, active, nact, A, coef, rss, r,
                                           qr_lds, pb.S, g, pb.ids, nrm,
                                           step + 1 == D_max ? out_rmse + b : nullptr);
        }
        check_launch("omp");
    }
}

// Householder QR fit of y on [1, the D given rows] for every problem (the
// OMP fit kernel with no pick): coefficients (intercept first, then the rows
// in the given order), sqrt(RSS / n), residuals when resid is given.
void fit_rows(discover_ctx* ctx, const discover_l0_problem* probs, int nb, int D, const int32_t* rows,
              int64_t rows_ld, double* coef, int64_t coef_ld, double* rmse, double* resid, int64_t ldr,
              hipStream_t st) {
    int32_t* cnt = ctx->buf<int32_t>("fit_rows_d" + ctx->tag, 1);
    fill_all(ctx, "fit_rows_fill", {fill_seg(cnt, 4, (uint32_t)D)}, st);
    for (int b = 0; b < nb; b++) {
        const discover_l0_problem& pb = probs[b];
        double* A = ctx->buf<double>("fit_rows_A" + std::to_string(b) + ctx->tag, (size_t)(D + 2) * pb.n);
        double* rs = ctx->buf<double>("fit_rows_rss" + std::to_string(b) + ctx->tag, 1);
        double* r = resid ? resid + (int64_t)b * ldr
                          : ctx->buf<double>("fit_rows_r" + std::to_string(b) + ctx->tag, pb.n);
        const size_t qr_bytes = (size_t)(D + 2) * pb.n * sizeof(double);
        const int qr_lds = qr_bytes <= 65536 ? 1 : 0;
        // the rows are not modified: the kernel only appends when it picks
        k_omp_fit<<<1, 256, qr_lds ? qr_bytes : 0, st>>>(pb.n, pb.F, pb.ldf, pb.y, (int32_t*)rows + b * rows_ld,
                                                       cnt, A, coef + b * coef_ld, rs, r, qr_lds, pb.S, nullptr,
                                                       pb.ids, nullptr, rmse + b);
    }
    check_launch("k_omp_fit (rows)");
}

GramOut l0_gram_one(discover_ctx* ctx, const discover_l0_problem& pb, const std::string& name,
                    hipStream_t st) {
    PrepArgs a{};
    a.n = pb.n; a.S = pb.S; a.ldz = (int)cdiv(pb.n, 16) * 16; a.ldg = (int)cdiv(pb.S + 1, 2) * 2;
    a.F = pb.F; a.ldf = pb.ldf; a.y = pb.y;
    a.Z = ctx->buf<double>(name + "_Z" + ctx->tag, (size_t)(pb.S + 1) * a.ldz);
    a.G = ctx->buf<double>(name + "_G" + ctx->tag, (size_t)(pb.S + 1) * a.ldg);
    a.yy = ctx->buf<double>(name + "_yy" + ctx->tag, 1);
    a.dg = ctx->buf<double>(name + "_dg" + ctx->tag, (size_t)pb.S + 1);
    const ctab<PrepArgs> dpa = ct((const PrepArgs*)ctx->upload(name + "_prep", &a, sizeof a, st));
    KTimer kt(ctx, st, "l0_gram");
    k_l0_prep<<<dim3((unsigned)cdiv(pb.S + 1, 4), 1), 256, 0, st>>>(dpa);
    const int gt = (int)cdiv(pb.S + 1, 32);
    k_gram<<<dim3(8u * (unsigned)gram_xcd_tiles(gt), 1, 1), 256, 0, st>>>(dpa);
    check_launch("k_gram");
    return GramOut{a.G, a.ldg, a.yy, a.dg};
}

// QR residual sum of squares of each listed D-subset (block-stride over the
// list; the work space of a block is in LDS when it fits).
__global__ __launch_bounds__(256) void k_refit_list(int n, int D, const double* __restrict__ F, int64_t ldf,
                                                    const double* __restrict__ y,
                                                    const int32_t* __restrict__ subs, int64_t count,
                                                    double* __restrict__ rss_out, double* __restrict__ scratch,
                                                    int64_t sld, int use_lds) {
    __shared__ double coef[DISCOVER_MAX_D + 1];
    __shared__ double rss;
    extern __shared__ double dsm[];
    double* A = use_lds ? dsm : scratch + (int64_t)blockIdx.x * sld;
    for (int64_t e = blockIdx.x; e < count; e += gridDim.x) {
        block_lsq(n, D, subs + e * D, F, ldf, y, A, coef, &rss, nullptr);
        if (threadIdx.x == 0) rss_out[e] = rss;
        __syncthreads();
    }
}

void refit_list(discover_ctx* ctx, const discover_l0_problem& pb, int D, const int32_t* subs, int64_t count,
                double* rss, hipStream_t st) {
    if (count <= 0) return;
    const int64_t sld = (int64_t)(D + 2) * pb.n;
    const int use_lds = sld * 8 <= 65536 ? 1 : 0;
    const unsigned grid = (unsigned)std::min<int64_t>(count, 2048);
    double* scr = use_lds ? nullptr : ctx->buf<double>("refit_list_A" + ctx->tag, (size_t)grid * sld);
    k_refit_list<<<grid, 256, use_lds ? sld * 8 : 0, st>>>(pb.n, D, pb.F, pb.ldf, pb.y, subs, count, rss, scr,
                                                          sld, use_lds);
    check_launch("k_refit_list");
}

void validate_omp(const discover_l0_problem* probs, int32_t n_problems, int32_t D_max,
                  const int32_t* init_active, int32_t n_init, const int32_t* out_active,
                  const double* out_coef, const double* out_rmse, const double* out_resid, int64_t ldr) {
    DSC_REQUIRE(probs && n_problems >= 1, "probs/n_problems");
    DSC_REQUIRE(D_max >= 1 && D_max <= DISCOVER_MAX_D, "D_max = %d outside 1..%d", D_max, DISCOVER_MAX_D);
    DSC_REQUIRE(n_init >= 0 && n_init <= D_max && (n_init == 0 || init_active), "init_active");
    DSC_REQUIRE(out_active && out_coef && out_rmse, "outputs required");
    for (int b = 0; b < n_problems; b++) {
        const discover_l0_problem& p = probs[b];
        DSC_REQUIRE(p.S >= D_max, "problem %d: S = %d < D_max", b, p.S);
        DSC_REQUIRE(p.n >= D_max + 2, "problem %d: n too small", b);
        DSC_REQUIRE(p.F && p.ids && p.y && p.ldf >= p.n, "problem %d: F/ids/y/ldf", b);
        DSC_REQUIRE(!out_resid || ldr >= p.n, "problem %d: ldr < n", b);
    }
}

}  // namespace dsc

extern "C" discover_status discover_omp(discover_ctx* ctx, const discover_l0_problem* probs,
                                        int32_t n_problems, int32_t D_max, const int32_t* init_active,
                                        int32_t n_init, int32_t* out_active, double* out_coef,
                                        double* out_rmse, double* out_resid, int64_t ldr,
                                        void* stream) {
    using namespace dsc;
    return guarded([&] {
        DSC_REQUIRE(ctx, "ctx is NULL");
        validate_omp(probs, n_problems, D_max, init_active, n_init, out_active, out_coef, out_rmse,
                     out_resid, ldr);
        DSC_HIP(hipSetDevice(ctx->device));
        const hipStream_t st = (hipStream_t)stream;
        CallMode mode(ctx, stream_capturing(st), false);
        omp_batch(ctx, probs, n_problems, D_max, init_active, n_init, n_init, out_active, out_coef,
                  out_rmse, out_resid, ldr, st);
    });
}
