// Exact L0 (Eq. (1), Core Optimization Objective, with an intercept) by
// branch and bound on the correlation matrix: the exact search the paper
// names beside enumeration and the stochastic searches (Software
// Description), for D up to 8.
//
// Tree.  A node is a prefix P = (p_1 < ... < p_a) of rows; its children
// append a row j > p_a, the leaves are the D-subsets.  Every subset below
// child P + j uses rows from P + {rows >= j}, and the explained fraction of
// a least-squares fit never falls when rows are added, so
//     bound(P, j) = R^2(P + {rows >= j})
// bounds the whole branch.  It falls as j grows: the first child whose
// bound is below the threshold ends the scan of its siblings.
//
// Bounds.  With L the Cholesky factor of the correlation matrix in reverse
// row order (row S-1 first) and y appended last, the leading m columns
// span the m trailing rows {S-m, ..., S-1} = {rows >= S-m}.  Row p's
// entries w_p[u] = L[rev(p)][u] (u < m) are its coordinates in that span
// and v[u] = L[y][u] are y's, so for m = S - j
//     R^2({rows >= j}) = sum_{u<m} v_u^2,
//     K = G_PP - sum_{u<m} w_P w_P^T,  h = c_P - sum_{u<m} w_P v_u,
//     bound(P, j) = sum_{u<m} v_u^2 + h^T K^{-1} h,
// where the three prefix sums over u are tabulated once per problem for
// every pair of rows (a few hundred MB at S = 1024), so a bound costs a
// handful of table reads and an a x a Cholesky.  The factor stops at the
// first pivot <= 1e-6 of its row's diagonal (a row nearly in the span of
// the rows after it); bounds needing more than those m0 columns, or whose
// K has a pivot that small, are taken as 2 (nothing is cut on them).
//
// Exactness.  A branch is cut when its bound is below thr - 1e-6 - 1e-7,
// thr a value that never exceeds the m-th best explained fraction: the
// m-th largest of the per-prefix best leaves found so far (distinct
// prefixes give distinct subsets).  Every leaf within 1e-7 of the m-th
// best therefore survives, is evaluated (row-order Cholesky, the same
// singular-pivot rule as the exhaustive sweep) and listed; the list is cut
// to the final thr - 1e-7, refitted by Householder QR and ranked by RSS
// with the tie rule of the exhaustive L0, so the models equal the
// exhaustive search's (under the same assumption that the explained
// fraction from the correlation matrix is within 1e-7 of QR's).  The order
// in which the GPU visits the tree changes thr on the way, so the counts of
// nodes and leaves may vary from run to run; the band and the result do
// not.
//
// GPU mapping.  The host runs a chunked depth-first walk over levels:
// level a holds prefixes of length a; a launch takes a chunk from the
// front of the deepest non-empty level and expands it into the next level
// (one wave per prefix, 64 children per step, a ballot finds the cut) or,
// at level D - 1, evaluates its leaves (one wave per prefix, one leaf per
// lane, the prefix's factor in registers).  A one-block kernel then merges
// the chunk's per-prefix maxima into the running top m and sets thr.
#include "dsc_internal.h"

#include <algorithm>
#include <cstddef>
#include <cstring>
#include <string>

namespace dsc {
namespace {

constexpr double BNB_TAU = 1e-6;                    // trusted pivot, relative to the row's diagonal
constexpr double BNB_CUT = 1e-6 + GRAM_DELTA;       // margin below thr at which a branch is cut
constexpr int BNB_PANEL = 32;
constexpr int BNB_MAX_S = 1024;
constexpr int BNB_MAX_M = 64;
constexpr int64_t BNB_LEVEL_CAP = 1 << 24;          // prefixes per level buffer
constexpr int64_t BNB_CAND_CAP = 1 << 26;           // listed leaves
constexpr double NO_CUT = 2.0;                      // a bound that cuts nothing

struct Node {
    int16_t r[8];
};

// Device state of one problem's search.
struct BnbState {
    double thr;                  // cut threshold base: <= the m-th best explained fraction
    double seed_thr;             // the local search's m-th best
    int32_t m0;                  // columns of the reverse factor
    int32_t stop;                // the factor has stopped
    unsigned long long out;      // prefixes written by an expansion
    unsigned long long ncand;    // listed leaves
    unsigned long long nbounds;
    unsigned long long nleaves;
    unsigned long long qhead;    // next parent of a pair launch (reset by the threshold update)
    double top[BNB_MAX_M];       // running top m of the per-prefix maxima, descending
};

struct BnbTab {
    const double* G;             // correlation matrix, (S + 1) rows of ldg (row S: y)
    const double* dg;            // its diagonal
    int ldg, S, m0;
    const double* PW;            // pair prefix sums
    const int64_t* off;          // [S] start of row q's pairs
    const double* PV;            // [S][m0 + 1]
    const double* VV;            // [m0 + 1]
};

__device__ __forceinline__ int rev(int t, int S) { return t < S ? S - 1 - t : S; }

// Reverse-ordered copy of G (lower triangle): A[t][u] = G[rev t][rev u].
__global__ __launch_bounds__(256) void k_bnb_load(const double* __restrict__ G, int ldg, int S,
                                                  double* __restrict__ A, int lda) {
    const int t = blockIdx.y;
    const int rt = rev(t, S);
    for (int u = blockIdx.x * 256 + threadIdx.x; u <= t; u += gridDim.x * 256)
        A[(int64_t)t * lda + u] = G[(int64_t)rt * ldg + rev(u, S)];
}

// Columns u0 .. u0 + BNB_PANEL - 1 of the factor, all rows below them (one
// block).  A pivot <= BNB_TAU of the row's own diagonal stops the factor:
// m0 = that column.  A row that is exactly zero (a constant feature) spans
// nothing: its column stays zero and is passed over.
__global__ __launch_bounds__(1024) void k_bnb_panel(double* __restrict__ A, int lda, int S, int u0,
                                                    const double* __restrict__ G, int ldg,
                                                    BnbState* __restrict__ st) {
    if (st->stop) return;
    const int u1 = min(S, u0 + BNB_PANEL);
    for (int u = u0; u < u1; u++) {
        const double orig = G[(int64_t)rev(u, S) * ldg + rev(u, S)];
        const double d = A[(int64_t)u * lda + u];
        if (orig == 0.0) {                      // uniform: every thread reads the same values
            for (int t = u + threadIdx.x; t <= S; t += blockDim.x) A[(int64_t)t * lda + u] = 0.0;
            __syncthreads();
            continue;
        }
        if (!(d > BNB_TAU * orig)) {
            __syncthreads();
            if (threadIdx.x == 0) {
                st->stop = 1;
                st->m0 = u;
            }
            return;
        }
        const double l = sqrt(d);
        __syncthreads();
        for (int t = u + 1 + threadIdx.x; t <= S; t += blockDim.x) A[(int64_t)t * lda + u] /= l;
        if (threadIdx.x == 0) A[(int64_t)u * lda + u] = l;
        __syncthreads();
        // the rest of the panel: A[t][c] -= L[t][u] L[c][u], u < c < u1, t >= c
        const int w = u1 - u - 1;
        if (w > 0) {
            const int64_t rows = S - u;          // t = u + 1 .. S
            for (int64_t e = threadIdx.x; e < rows * w; e += blockDim.x) {
                const int t = u + 1 + (int)(e / w);
                const int c = u + 1 + (int)(e % w);
                if (c <= t) A[(int64_t)t * lda + c] -= A[(int64_t)t * lda + u] * A[(int64_t)c * lda + u];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && u1 == S) st->m0 = S;
}

// Trailing update after panel u0: A[t][c] -= sum_u L[t][u] L[c][u] over the
// panel's columns, for u0 + BNB_PANEL <= c <= t <= S.  grid (column blocks,
// rows).
__global__ __launch_bounds__(256) void k_bnb_update(double* __restrict__ A, int lda, int S, int u0,
                                                    const BnbState* __restrict__ st) {
    if (st->stop) return;
    const int c0 = u0 + BNB_PANEL;
    const int t = c0 + blockIdx.y;
    if (t > S) return;
    const int c = c0 + blockIdx.x * 256 + threadIdx.x;
    if (c > t) return;
    const double* at = A + (int64_t)t * lda + u0;
    const double* ac = A + (int64_t)c * lda + u0;
    double s = 0.0;
#pragma unroll 8
    for (int u = 0; u < BNB_PANEL; u++) s = fma(at[u], ac[u], s);
    A[(int64_t)t * lda + c] -= s;
}

// Inclusive prefix sum over the 64 lanes.
__device__ __forceinline__ double wave_incl_scan(double x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

// Prefix-sum tables, one wave per sequence: waves 0 .. npair-1 the pairs
// p <= q (q-major), then S waves for PV, then one for VV.
__global__ __launch_bounds__(256) void k_bnb_tables(const double* __restrict__ A, int lda, int S, int m0,
                                                    const int64_t* __restrict__ off, double* __restrict__ PW,
                                                    double* __restrict__ PV, double* __restrict__ VV,
                                                    int64_t npair) {
    const int64_t w = (int64_t)blockIdx.x * 4 + wave_id();
    const int lane = threadIdx.x & 63;
    const double* vy = A + (int64_t)S * lda;
    const double *x1, *x2;
    double* out;
    int len;                                     // entries m = 0 .. len - 1
    if (w < npair) {
        // q = the largest with q (q + 1) / 2 <= w
        int q = (int)((sqrt(8.0 * (double)w + 1.0) - 1.0) * 0.5);
        while ((int64_t)(q + 1) * (q + 2) / 2 <= w) q++;
        while ((int64_t)q * (q + 1) / 2 > w) q--;
        const int p = (int)(w - (int64_t)q * (q + 1) / 2);
        len = min(m0, S - 1 - q) + 1;
        x1 = A + (int64_t)(S - 1 - p) * lda;
        x2 = A + (int64_t)(S - 1 - q) * lda;
        out = PW + off[q] + (int64_t)p * len;
    } else if (w < npair + S) {
        const int p = (int)(w - npair);
        len = min(m0, S - 1 - p) + 1;
        x1 = A + (int64_t)(S - 1 - p) * lda;
        x2 = vy;
        out = PV + (int64_t)p * (m0 + 1);
    } else if (w == npair + S) {
        len = m0 + 1;
        x1 = vy;
        x2 = vy;
        out = VV;
    } else {
        return;
    }
    if (lane == 0) out[0] = 0.0;
    double carry = 0.0;
    for (int u0 = 0; u0 < len - 1; u0 += 64) {
        const int u = u0 + lane;
        const double term = u < len - 1 ? x1[u] * x2[u] : 0.0;
        const double s = wave_incl_scan(term) + carry;
        if (u < len - 1) out[u + 1] = s;
        carry = __shfl(s, 63, 64);
    }
}

// R^2(P + {rows >= S - m}) for a prefix of A rows (NO_CUT where untrusted).
template <int A>
__device__ __forceinline__ double bnb_bound(const BnbTab& T, const int* P, int m) {
    if (m > T.m0) return NO_CUT;
    double z = T.VV[m];
    if constexpr (A > 0) {
        double L[A][A], h[A];
        const int S = T.S;
#pragma unroll
        for (int k = 0; k < A; k++) {
            const int pk = P[k];
            h[k] = T.G[(int64_t)pk * T.ldg + S] - T.PV[(int64_t)pk * (T.m0 + 1) + m];
#pragma unroll
            for (int l = k; l < A; l++) {
                const int pl = P[l];
                const int len = min(T.m0, S - 1 - pl) + 1;
                L[l][k] = T.G[(int64_t)pk * T.ldg + pl] - T.PW[T.off[pl] + (int64_t)pk * len + m];
            }
        }
#pragma unroll
        for (int k = 0; k < A; k++) {
            double d = L[k][k];
#pragma unroll
            for (int i = 0; i < k; i++) d -= L[k][i] * L[k][i];
            const double orig = T.G[(int64_t)P[k] * T.ldg + P[k]];
            if (!(d > BNB_TAU * orig)) return NO_CUT;
            const double lk = sqrt(d);
            L[k][k] = lk;
#pragma unroll
            for (int l = k + 1; l < A; l++) {
                double e = L[l][k];
#pragma unroll
                for (int i = 0; i < k; i++) e -= L[l][i] * L[k][i];
                L[l][k] = e / lk;
            }
            double hk = h[k];
#pragma unroll
            for (int i = 0; i < k; i++) hk -= L[k][i] * h[i];
            h[k] = hk / lk;
            z += h[k] * h[k];
        }
    }
    return z;
}

struct BnbLaunch {
    BnbTab T;
    BnbState* st;
    const Node* in;
    int64_t nin;
    int D;
    // expansion
    Node* out;                   // the next level
    int32_t* cut;                // [nin] first child cut (children last+1 .. cut-1 survive)
    int64_t* cnt;                // [nin] surviving (non-constant) children, then their offsets
    int32_t* nbw;                // [nin] bound evaluations
    const int32_t* vpre;         // [S + 1] non-constant rows below j
    // leaves
    Node* cand;                  // listed subsets
    double* cval;
    double* blk_best;            // [grid] best leaf of the block's prefixes
    unsigned long long* blk_cnt; // [grid] leaves evaluated by the block
};

__device__ __forceinline__ unsigned long long wave_slots(unsigned long long* ctr, uint64_t mask) {
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)mask) - 1;
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(ctr, (unsigned long long)__popcll(mask));
    base = __shfl(base, leader, 64);
    return base + (unsigned long long)__popcll(mask & ((1ull << lane) - 1ull));
}

// vpre[j] = non-constant rows below j (one block).
__global__ __launch_bounds__(1024) void k_bnb_vpre(const double* __restrict__ dg, int S, int32_t* __restrict__ vpre) {
    __shared__ int32_t part[1024];
    const int per = (S + 1023) / 1024;
    const int j0 = threadIdx.x * per, j1 = min(S, j0 + per);
    int c = 0;
    for (int j = j0; j < j1; j++) c += dg[j] > 0.0;
    part[threadIdx.x] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int t = 0; t < 1024; t++) { const int v = part[t]; part[t] = acc; acc += v; }
    }
    __syncthreads();
    int acc = part[threadIdx.x];
    for (int j = j0; j < j1; j++) { vpre[j] = acc; acc += dg[j] > 0.0; }
    if (j1 == S && j0 < j1) vpre[S] = acc;
    if (S == 0 && threadIdx.x == 0) vpre[0] = 0;
}

// Expansion, pass 1: the cut of each prefix of length A (one wave per
// prefix, 64 children per step; the first child whose bound is below the
// threshold ends the scan).  No atomics: counts go to per-prefix slots.
template <int A>
__global__ __launch_bounds__(256) void k_bnb_expand(BnbLaunch g) {
    const int lane = threadIdx.x & 63;
    const BnbTab& T = g.T;
    const int S = T.S;
    const int jmax = S - (g.D - A);             // D - A - 1 rows must follow j
    const double cut = g.st->thr - BNB_CUT;
    for (int64_t w = (int64_t)blockIdx.x * 4 + wave_id(); w < g.nin; w += (int64_t)gridDim.x * 4) {
        int P[8];
#pragma unroll
        for (int k = 0; k < 8; k++) P[k] = k < A ? g.in[w].r[k] : 0;
        const int last = A > 0 ? P[A - 1] : -1;
        int nb = 0;
        int end = jmax + 1;
        for (int j0 = last + 1; j0 <= jmax; j0 += 64) {
            const int j = j0 + lane;
            const bool in = j <= jmax;
            const double b = in ? bnb_bound<A>(T, P, S - j) : NO_CUT;
            const uint64_t fail = __builtin_amdgcn_ballot_w64(in && b < cut);
            const int first = fail ? __builtin_ctzll(fail) : 64;
            nb += __popcll(__builtin_amdgcn_ballot_w64(in && lane <= first));
            if (fail) {
                end = j0 + first;
                break;
            }
        }
        if (lane == 0) {
            g.cut[w] = end;
            g.cnt[w] = end > last + 1 ? g.vpre[end] - g.vpre[last + 1] : 0;
            g.nbw[w] = nb;
        }
    }
}

// Expansion, scan (one block): cnt -> exclusive offsets, the total to
// st->out, the bound evaluations added to st->nbounds.
__global__ __launch_bounds__(1024) void k_bnb_scan(int64_t n, int64_t* __restrict__ cnt, const int32_t* __restrict__ nbw,
                                                   BnbState* __restrict__ st) {
    __shared__ int64_t part[1024];
    __shared__ unsigned long long nbs[1024];
    const int64_t per = (n + 1023) / 1024;
    const int64_t e0 = threadIdx.x * per, e1 = min(n, e0 + per);
    int64_t c = 0;
    unsigned long long b = 0;
    for (int64_t e = e0; e < e1; e++) { c += cnt[e]; b += (unsigned long long)nbw[e]; }
    part[threadIdx.x] = c;
    nbs[threadIdx.x] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t acc = 0;
        unsigned long long bs = 0;
        for (int t = 0; t < 1024; t++) { const int64_t v = part[t]; part[t] = acc; acc += v; bs += nbs[t]; }
        st->out = (unsigned long long)acc;
        st->nbounds += bs;
    }
    __syncthreads();
    int64_t acc = part[threadIdx.x];
    for (int64_t e = e0; e < e1; e++) { const int64_t v = cnt[e]; cnt[e] = acc; acc += v; }
}

// Expansion, pass 2: the surviving non-constant children of each prefix at
// its offset (one wave per prefix).
template <int A>
__global__ __launch_bounds__(256) void k_bnb_emit(BnbLaunch g) {
    const int lane = threadIdx.x & 63;
    for (int64_t w = (int64_t)blockIdx.x * 4 + wave_id(); w < g.nin; w += (int64_t)gridDim.x * 4) {
        int P[8];
#pragma unroll
        for (int k = 0; k < 8; k++) P[k] = k < A ? g.in[w].r[k] : 0;
        const int last = A > 0 ? P[A - 1] : -1;
        const int end = g.cut[w];
        const int64_t base = g.cnt[w] - g.vpre[last + 1];
        for (int j = last + 1 + lane; j < end; j += 64)
            if (g.T.dg[j] > 0.0) {
                Node nd;
#pragma unroll
                for (int k = 0; k < 8; k++) nd.r[k] = (int16_t)(k < A ? P[k] : (k == A ? j : 0));
                g.out[base + g.vpre[j]] = nd;
            }
    }
}

// Leaves of prefixes of length A = D - 1 (one wave per prefix at a time, a
// leaf per lane); the block's best leaf and leaf count go to per-block slots.
template <int A>
__global__ __launch_bounds__(256) void k_bnb_leaves(BnbLaunch g) {
    __shared__ double wbest[4];
    __shared__ unsigned long long wcnt[4];
    const int lane = threadIdx.x & 63;
    const BnbTab& T = g.T;
    const int S = T.S;
    const double* G = T.G;
    const int64_t ldg = T.ldg;
    const double* cy = G + (int64_t)S * ldg;   // row S: the correlations with y
    const double thr = g.st->thr;
    const double cut = thr - BNB_CUT;
    unsigned long long nl = 0;
    double best = -1.0;
    for (int64_t w = (int64_t)blockIdx.x * 4 + wave_id(); w < g.nin; w += (int64_t)gridDim.x * 4) {
        int P[8];
#pragma unroll
        for (int k = 0; k < 8; k++) P[k] = k < A ? g.in[w].r[k] : 0;
        const int last = A > 0 ? P[A - 1] : -1;
        // the prefix's factor in row order (every lane), as the exhaustive sweep
        double L[A > 0 ? A : 1][A > 0 ? A : 1], u[A > 0 ? A : 1];
        double base = 0.0;
        bool singular = false;
#pragma unroll
        for (int k = 0; k < A; k++) {
            double d = G[(int64_t)P[k] * ldg + P[k]];
#pragma unroll
            for (int i = 0; i < k; i++) d -= L[k][i] * L[k][i];
            if (!(d > PIV_TOL)) singular = true;
            const double lk = sqrt(fmax(d, 1e-300));
            L[k][k] = lk;
#pragma unroll
            for (int l = k + 1; l < A; l++) {
                double e = G[(int64_t)P[l] * ldg + P[k]];
#pragma unroll
                for (int i = 0; i < k; i++) e -= L[l][i] * L[k][i];
                L[l][k] = e / lk;
            }
            double c = G[(int64_t)P[k] * ldg + S];
#pragma unroll
            for (int i = 0; i < k; i++) c -= L[k][i] * u[i];
            u[k] = c / lk;
            base += u[k] * u[k];
        }
        if (singular) continue;                  // uniform over the wave
        for (int j0 = last + 1; j0 < S; j0 += 64) {
            if (bnb_bound<A>(T, P, S - j0) < cut) break;     // uniform over the wave
            const int j = j0 + lane;
            double val = -1.0;
            if (j < S) {
                // G is symmetric: row P[k] read at column j is coalesced over the lanes
                double e = cy[j];
                double piv = T.dg[j];
                double l[A > 0 ? A : 1];
#pragma unroll
                for (int k = 0; k < A; k++) {
                    double x = G[(int64_t)P[k] * ldg + j];
#pragma unroll
                    for (int i = 0; i < k; i++) x -= L[k][i] * l[i];
                    l[k] = x / L[k][k];
                    piv -= l[k] * l[k];
                    e -= l[k] * u[k];
                }
                if (piv > PIV_TOL) val = base + e * e / piv;
            }
            nl += min(64, S - j0);
            best = fmax(best, val);
            const bool keep = val >= 0.0 && val >= thr - GRAM_DELTA;
            const uint64_t km = __builtin_amdgcn_ballot_w64(keep);
            if (km) {
                const unsigned long long s = wave_slots(&g.st->ncand, km);
                if (keep) {
                    Node nd;
#pragma unroll
                    for (int k = 0; k < 8; k++) nd.r[k] = (int16_t)(k < A ? P[k] : (k == A ? j : 0));
                    g.cand[s] = nd;
                    g.cval[s] = val;
                }
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) best = fmax(best, __shfl_xor(best, o, 64));
    if (lane == 0) {
        wbest[wave_id()] = best;
        wcnt[wave_id()] = nl;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        g.blk_best[blockIdx.x] = fmax(fmax(wbest[0], wbest[1]), fmax(wbest[2], wbest[3]));
        g.blk_cnt[blockIdx.x] = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    }
}

// The last two levels at once, for parents P of length A = D - 2 (one
// block per parent at a time).  With L the parent's factor (row order), each
// later row r gets w_r = L^{-1} G[P][r], its residual norm gt_r = G_rr -
// |w_r|^2 and residual correlation ct_r = c_r - w_r . u, kept in LDS; the
// leaf P + (p, j), p < j, then needs only
//     g = G_pj - w_p . w_j,  piv = gt_j - g^2 / gt_p,  e = ct_j - g ct_p / gt_p,
//     R^2 = R^2(P) + ct_p^2 / gt_p + e^2 / piv
// (pivots gt_p and piv are the row-order Cholesky pivots of p and j: <=
// PIV_TOL is singular).  The children p of P are cut by bound(P, p) as an
// expansion cuts them; each child's leaves j in steps of 64 by bound(P + p,
// j).  A leaf list that would overflow is counted, not written (the host
// redoes the launch after compacting).
template <int A>
__global__ __launch_bounds__(256) void k_bnb_pairs(BnbLaunch g, int64_t cap) {
    extern __shared__ double lds[];              // [A + 2][S]: w_r, gt_r, ct_r by row r - r0 (lanes contiguous)
    __shared__ int pcut_s;
    __shared__ int64_t next_s;
    __shared__ double wbest[4];
    __shared__ unsigned long long wcnt[4];
    const int lane = threadIdx.x & 63;
    const int wv = wave_id();
    const BnbTab& T = g.T;
    const int S = T.S;
    const double* G = T.G;
    const int64_t ldg = T.ldg;
    const double* cy = G + (int64_t)S * ldg;
    const double thr = g.st->thr;
    const double cut = thr - BNB_CUT;
    unsigned long long nl = 0;
    double best = -1.0;
    // parents are taken from a queue: their work varies with the rows after them
    for (;;) {
        if (threadIdx.x == 0) next_s = (int64_t)atomicAdd(&g.st->qhead, 1ull);
        __syncthreads();
        const int64_t w = next_s;
        __syncthreads();
        if (w >= g.nin) break;
        int P[8];
#pragma unroll
        for (int k = 0; k < 8; k++) P[k] = k < A ? g.in[w].r[k] : 0;
        const int last = A > 0 ? P[A - 1] : -1;
        const int r0 = last + 1;
        double L[A > 0 ? A : 1][A > 0 ? A : 1], u[A > 0 ? A : 1];
        double base = 0.0;
        bool singular = false;
#pragma unroll
        for (int k = 0; k < A; k++) {
            double d = G[(int64_t)P[k] * ldg + P[k]];
#pragma unroll
            for (int i = 0; i < k; i++) d -= L[k][i] * L[k][i];
            if (!(d > PIV_TOL)) singular = true;
            const double lk = sqrt(fmax(d, 1e-300));
            L[k][k] = lk;
#pragma unroll
            for (int l = k + 1; l < A; l++) {
                double e = G[(int64_t)P[l] * ldg + P[k]];
#pragma unroll
                for (int i = 0; i < k; i++) e -= L[l][i] * L[k][i];
                L[l][k] = e / lk;
            }
            double c = G[(int64_t)P[k] * ldg + S];
#pragma unroll
            for (int i = 0; i < k; i++) c -= L[k][i] * u[i];
            u[k] = c / lk;
            base += u[k] * u[k];
        }
        if (singular) continue;                  // uniform over the block
        // 1. the later rows, residualised against P; the cut of the children
        if (threadIdx.x == 0) pcut_s = S - 1;
        __syncthreads();
        for (int r = r0 + threadIdx.x; r < S; r += 256) {
            double* x = lds + (r - r0);
            double gt = T.dg[r], ct = cy[r];
            double v[A > 0 ? A : 1];
#pragma unroll
            for (int k = 0; k < A; k++) {
                double t = G[(int64_t)P[k] * ldg + r];
#pragma unroll
                for (int i = 0; i < k; i++) t -= L[k][i] * v[i];
                t /= L[k][k];
                v[k] = t;
                x[k * S] = t;
                gt -= t * t;
                ct -= t * u[k];
            }
            x[A * S] = gt;
            x[(A + 1) * S] = ct;
            if (r <= S - 2 && bnb_bound<A>(T, P, S - r) < cut) atomicMin(&pcut_s, r);
        }
        __syncthreads();
        const int pcut = pcut_s;                 // children p < pcut survive
        // 2. the leaves of each surviving child, one child per wave at a time
        for (int p = r0 + wv; p < pcut; p += 4) {
            const double* xp = lds + (p - r0);
            const double gtp = xp[A * S], ctp = xp[(A + 1) * S];
            if (!(gtp > PIV_TOL)) continue;
            double wp[A > 0 ? A : 1];
#pragma unroll
            for (int k = 0; k < A; k++) wp[k] = xp[k * S];
            const double base_p = base + ctp * ctp / gtp;
            const double rg = 1.0 / gtp;
            int Pp[8];
#pragma unroll
            for (int k = 0; k < 8; k++) Pp[k] = k < A ? P[k] : (k == A ? p : 0);
            const double* gp = G + (int64_t)p * ldg;
            // 128 leaves per step, two per lane (independent chains); the
            // bound at the step's first leaf covers both.  The first step's
            // bound, R^2(P + p + rows > p) = bound(P, p), passed the cut above.
            for (int j0 = p + 1; j0 < S; j0 += 128) {
                if (j0 > p + 1 && bnb_bound<A + 1>(T, Pp, S - j0) < cut) break;   // uniform over the wave
                double val[2];
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    const int j = j0 + 64 * h + lane;
                    const int jj = min(j, S - 1);            // in-bounds read; j >= S is discarded
                    const double* xj = lds + (jj - r0);
                    double gpj = gp[jj];
#pragma unroll
                    for (int k = 0; k < A; k++) gpj -= wp[k] * xj[k * S];
                    const double piv = xj[A * S] - gpj * gpj * rg;
                    const double e = xj[(A + 1) * S] - gpj * ctp * rg;
                    // e^2 / piv by a reciprocal refined twice (Newton), a few
                    // ulps from the quotient
                    double r = __builtin_amdgcn_rcp(piv);
                    r = fma(fma(-piv, r, 1.0), r, r);
                    r = fma(fma(-piv, r, 1.0), r, r);
                    const double v = fma(e * e, r, base_p);
                    val[h] = (j < S && piv > PIV_TOL) ? v : -1.0;
                }
                nl += min(128, S - j0);
                best = fmax(best, fmax(val[0], val[1]));
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    const bool keep = val[h] >= 0.0 && val[h] >= thr - GRAM_DELTA;
                    const uint64_t km = __builtin_amdgcn_ballot_w64(keep);
                    if (km) {
                        const unsigned long long s = wave_slots(&g.st->ncand, km);
                        if (keep && (int64_t)s < cap) {
                            const int j = j0 + 64 * h + lane;
                            Node nd;
#pragma unroll
                            for (int k = 0; k < 8; k++)
                                nd.r[k] = (int16_t)(k < A ? P[k] : (k == A ? p : (k == A + 1 ? j : 0)));
                            g.cand[s] = nd;
                            g.cval[s] = val[h];
                        }
                    }
                }
            }
        }
        __syncthreads();                         // the rows of the next parent overwrite LDS
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) best = fmax(best, __shfl_xor(best, o, 64));
    if (lane == 0) {
        wbest[wv] = best;
        wcnt[wv] = nl;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        g.blk_best[blockIdx.x] = fmax(fmax(wbest[0], wbest[1]), fmax(wbest[2], wbest[3]));
        g.blk_cnt[blockIdx.x] = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    }
}

// Merge a leaf launch's per-block maxima (each the best leaf of its own
// prefixes, so distinct blocks give distinct subsets) into the running top m
// (one block):
// m rounds of a block arg-max in the order (value desc, index asc) over the
// old top m (indices 0..m-1) and the new maxima (m..), each round taking
// the largest entry after the previous pick.  thr = the m-th entry (-1
// while fewer than m are known).
__global__ __launch_bounds__(256) void k_bnb_topm(BnbState* __restrict__ st, const double* __restrict__ best,
                                                  int64_t nb, int m, const unsigned long long* __restrict__ cnt) {
    if (threadIdx.x == 0) st->qhead = 0;         // the next pair launch starts its queue anew
    if (cnt) {                                   // the leaf launch's per-block counts
        __shared__ unsigned long long cs[256];
        unsigned long long c = 0;
        for (int64_t e = threadIdx.x; e < nb; e += 256) c += cnt[e];
        cs[threadIdx.x] = c;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long t = 0;
            for (int i = 0; i < 256; i++) t += cs[i];
            st->nleaves += t;
        }
    }
    __shared__ double sv[256];
    __shared__ int64_t si[256];
    __shared__ double newtop[BNB_MAX_M];
    double pv = INFINITY;
    int64_t pi = -1;
    const int64_t tot = m + nb;
    for (int r = 0; r < m; r++) {
        double bv = -INFINITY;
        int64_t bi = INT64_MAX;
        for (int64_t e = threadIdx.x; e < tot; e += 256) {
            const double v = e < m ? st->top[e] : best[e - m];
            if (!(v >= 0.0)) continue;
            const bool after = v < pv || (v == pv && e > pi);
            const bool better = v > bv || (v == bv && e < bi);
            if (after && better) { bv = v; bi = e; }
        }
        sv[threadIdx.x] = bv;
        si[threadIdx.x] = bi;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (threadIdx.x < o) {
                const double v = sv[threadIdx.x + o];
                const int64_t i = si[threadIdx.x + o];
                if (v > sv[threadIdx.x] || (v == sv[threadIdx.x] && i < si[threadIdx.x])) {
                    sv[threadIdx.x] = v;
                    si[threadIdx.x] = i;
                }
            }
            __syncthreads();
        }
        pv = sv[0];
        pi = si[0];
        if (threadIdx.x == 0) newtop[r] = pi == INT64_MAX ? -1.0 : pv;
        __syncthreads();
        if (pi == INT64_MAX) {                   // fewer than m known: the rest stay empty
            for (int q = r + 1 + threadIdx.x; q < m; q += 256) newtop[q] = -1.0;
            break;
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < m; q += 256) st->top[q] = newtop[q];
    // the search's and the local search's m-th best each bound the m-th best
    // (they may share subsets, so they are not merged)
    if (threadIdx.x == 0) st->thr = fmax(st->seed_thr, newtop[m - 1]);
}

// Explained fraction of the rows r[0..D-1] (ascending) from G by a Cholesky
// in row order; -1 when a pivot is <= PIV_TOL (singular) or a row repeats.
__device__ double seed_r2(const double* __restrict__ G, int64_t ldg, int S, const int* r, int D) {
    double L[DISCOVER_MAX_D][DISCOVER_MAX_D], u[DISCOVER_MAX_D];
    double z = 0.0;
    for (int k = 0; k < D; k++) {
        double d = G[(int64_t)r[k] * ldg + r[k]];
        for (int i = 0; i < k; i++) d -= L[k][i] * L[k][i];
        if (!(d > PIV_TOL)) return -1.0;
        const double lk = sqrt(d);
        L[k][k] = lk;
        for (int l = k + 1; l < D; l++) {
            double e = G[(int64_t)r[l] * ldg + r[k]];
            for (int i = 0; i < k; i++) e -= L[l][i] * L[k][i];
            L[l][k] = e / lk;
        }
        double c = G[(int64_t)r[k] * ldg + S];
        for (int i = 0; i < k; i++) c -= L[k][i] * u[i];
        u[k] = c / lk;
        z += u[k] * u[k];
    }
    return z;
}

// The subset cur with position p replaced by row x, ascending, in out;
// false when x is already in cur.
__device__ __forceinline__ bool swapped(const int* cur, int D, int p, int x, int* out) {
    int c = 0;
    bool placed = false;
    for (int k = 0; k < D; k++) {
        if (cur[k] == x) return false;
        if (k == p) continue;
        if (!placed && x < cur[k]) { out[c++] = x; placed = true; }
        out[c++] = cur[k];
    }
    if (!placed) out[c++] = x;
    return true;
}

// A starting threshold (one block): from the D rows of largest |c|, single-
// row swaps that raise the explained fraction are taken (best first) until
// none does; the subset reached and its D (S - D) swap neighbours are
// distinct feasible subsets, so the m-th largest of their fractions is at
// most the m-th best: it becomes seed_thr and thr.
__global__ __launch_bounds__(256) void k_bnb_seed(const double* __restrict__ G, int ldg, int S, int D, int m,
                                                  double* __restrict__ nv, BnbState* __restrict__ st) {
    __shared__ double sv[256];
    __shared__ int si[256];
    __shared__ int cur[DISCOVER_MAX_D];
    __shared__ double cval;
    __shared__ double newtop[BNB_MAX_M];
    const int t = threadIdx.x;
    // start: the D rows of largest |c| (ties to the smaller row), then sorted
    for (int k = 0; k < D; k++) {
        double bv = -1.0;
        int bi = S;
        for (int j = t; j < S; j += 256) {
            bool used = false;
            for (int i = 0; i < k; i++) used = used || cur[i] == j;
            const double v = G[(int64_t)j * ldg + j] > 0.0 ? fabs(G[(int64_t)j * ldg + S]) : -1.0;
            if (!used && (v > bv || (v == bv && j < bi))) { bv = v; bi = j; }
        }
        sv[t] = bv;
        si[t] = bi;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (t < o && (sv[t + o] > sv[t] || (sv[t + o] == sv[t] && si[t + o] < si[t]))) {
                sv[t] = sv[t + o];
                si[t] = si[t + o];
            }
            __syncthreads();
        }
        if (t == 0) cur[k] = si[0] < S ? si[0] : k;
        __syncthreads();
    }
    if (t == 0) {
        for (int a = 1; a < D; a++)
            for (int b = a; b > 0 && cur[b - 1] > cur[b]; b--) {
                const int x = cur[b]; cur[b] = cur[b - 1]; cur[b - 1] = x;
            }
        cval = seed_r2(G, ldg, S, cur, D);
    }
    __syncthreads();
    const int64_t ns = (int64_t)D * S;
    // at most 256 improving swaps; the last round (round 256, or the one that
    // finds no improvement) only lists the neighbours of the final subset
    for (int round = 0; round <= 256; round++) {
        double bv = -1.0;
        int bi = -1;
        int c[DISCOVER_MAX_D], r[DISCOVER_MAX_D];
        for (int k = 0; k < D; k++) c[k] = cur[k];
        for (int64_t e = t; e < ns; e += 256) {
            double v = -1.0;
            if (G[(int64_t)(e % S) * ldg + (e % S)] > 0.0 && swapped(c, D, (int)(e / S), (int)(e % S), r))
                v = seed_r2(G, ldg, S, r, D);
            nv[e] = v;
            if (v > bv) { bv = v; bi = (int)e; }
        }
        if (round == 256) break;                 // uniform
        sv[t] = bv;
        si[t] = bi;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (t < o && (sv[t + o] > sv[t] || (sv[t + o] == sv[t] && si[t + o] >= 0 && (si[t] < 0 || si[t + o] < si[t])))) {
                sv[t] = sv[t + o];
                si[t] = si[t + o];
            }
            __syncthreads();
        }
        const bool better = si[0] >= 0 && sv[0] > cval;
        __syncthreads();
        if (!better) break;
        if (t == 0) {
            swapped(c, D, si[0] / S, si[0] % S, r);
            for (int k = 0; k < D; k++) cur[k] = r[k];
            cval = sv[0];
        }
        __syncthreads();
    }
    __syncthreads();
    // nv holds the neighbours of the final subset: top m of {cur} + nv
    double pv = INFINITY;
    int64_t pi = -2;
    for (int q = 0; q < m; q++) {
        double bv = -INFINITY;
        int64_t bi = INT64_MAX;
        for (int64_t e = (int64_t)t - 1; e < ns; e += 256) {
            const double v = e < 0 ? cval : nv[e];
            if (!(v >= 0.0)) continue;
            const bool after = v < pv || (v == pv && e > pi);
            if (after && (v > bv || (v == bv && e < bi))) { bv = v; bi = e; }
        }
        sv[t] = bv;
        __shared__ int64_t sl[256];
        sl[t] = bi;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (t < o && (sv[t + o] > sv[t] || (sv[t + o] == sv[t] && sl[t + o] < sl[t]))) {
                sv[t] = sv[t + o];
                sl[t] = sl[t + o];
            }
            __syncthreads();
        }
        pv = sv[0];
        pi = sl[0];
        if (t == 0) newtop[q] = pi == INT64_MAX ? -1.0 : pv;
        __syncthreads();
    }
    if (t == 0) {
        st->seed_thr = newtop[m - 1];
        st->thr = fmax(st->thr, newtop[m - 1]);
    }
}

// Listed leaves with value >= thr - GRAM_DELTA, copied to the other buffer.
__global__ __launch_bounds__(256) void k_bnb_compact(BnbState* __restrict__ st, const Node* __restrict__ cin,
                                                     const double* __restrict__ vin, int64_t n,
                                                     Node* __restrict__ cout, double* __restrict__ vout,
                                                     unsigned long long* __restrict__ cnt) {
    const double lim = st->thr - GRAM_DELTA;
    for (int64_t e0 = (int64_t)blockIdx.x * 256; e0 < n; e0 += (int64_t)gridDim.x * 256) {
        const int64_t e = e0 + threadIdx.x;
        const bool keep = e < n && vin[e] >= lim;
        const uint64_t km = __builtin_amdgcn_ballot_w64(keep);
        if (km) {
            const unsigned long long s = wave_slots(cnt, km);
            if (keep) {
                cout[s] = cin[e];
                vout[s] = vin[e];
            }
        }
    }
}

// Listed subsets as int32 rows [count][D] for the QR refit.
__global__ __launch_bounds__(256) void k_bnb_rows(const Node* __restrict__ c, int64_t n, int D,
                                                  int32_t* __restrict__ rows) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
        for (int k = 0; k < D; k++) rows[e * D + k] = c[e].r[k];
}

// Tuple order of the tie rule: sorted candidate IDs, lexicographic.
__device__ __forceinline__ bool ids_before(const int64_t* a, const int64_t* b, int D) {
    for (int k = 0; k < D; k++)
        if (a[k] != b[k]) return a[k] < b[k];
    return false;
}

// The m best models of the refitted list (one block): each round takes the
// smallest RSS among the untaken entries, then among the entries within
// TAU_TIE * yy of it the smallest sorted ID tuple.
__global__ __launch_bounds__(256) void k_bnb_rank(const int32_t* __restrict__ rows, const double* __restrict__ rss,
                                                  int64_t n, int D, int m, const int64_t* __restrict__ ids,
                                                  const double* __restrict__ yy, uint8_t* __restrict__ taken,
                                                  int32_t* __restrict__ out_sub, int32_t* __restrict__ nfound) {
    __shared__ double smin[256];
    __shared__ int64_t sidx[256];
    __shared__ int found;
    if (threadIdx.x == 0) found = 0;
    for (int64_t e = threadIdx.x; e < n; e += 256) taken[e] = 0;
    __syncthreads();
    const double tol = TAU_TIE * *yy;
    for (int q = 0; q < m; q++) {
        double mn = INFINITY;
        for (int64_t e = threadIdx.x; e < n; e += 256)
            if (!taken[e] && rss[e] < mn) mn = rss[e];
        smin[threadIdx.x] = mn;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (threadIdx.x < o) smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + o]);
            __syncthreads();
        }
        const double lim = smin[0] + tol;
        __syncthreads();
        int64_t bi = -1;
        int64_t bk[DISCOVER_MAX_D];
        for (int64_t e = threadIdx.x; e < n; e += 256) {
            if (taken[e] || !(rss[e] <= lim)) continue;
            int64_t k[DISCOVER_MAX_D];
            for (int j = 0; j < D; j++) k[j] = ids[rows[e * D + j]];
            for (int a = 1; a < D; a++)
                for (int b = a; b > 0 && k[b - 1] > k[b]; b--) {
                    const int64_t t = k[b]; k[b] = k[b - 1]; k[b - 1] = t;
                }
            if (bi < 0 || ids_before(k, bk, D)) {
                bi = e;
                for (int j = 0; j < D; j++) bk[j] = k[j];
            }
        }
        sidx[threadIdx.x] = bi;
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t pick = -1;
            int64_t pk[DISCOVER_MAX_D];
            for (int t = 0; t < 256; t++) {
                const int64_t e = sidx[t];
                if (e < 0) continue;
                int64_t k[DISCOVER_MAX_D];
                for (int j = 0; j < D; j++) k[j] = ids[rows[e * D + j]];
                for (int a = 1; a < D; a++)
                    for (int b = a; b > 0 && k[b - 1] > k[b]; b--) {
                        const int64_t tt = k[b]; k[b] = k[b - 1]; k[b - 1] = tt;
                    }
                if (pick < 0 || ids_before(k, pk, D)) {
                    pick = e;
                    for (int j = 0; j < D; j++) pk[j] = k[j];
                }
            }
            if (pick >= 0) {
                taken[pick] = 1;
                for (int j = 0; j < D; j++) out_sub[q * D + j] = rows[pick * D + j];
                found = q + 1;
                sidx[0] = pick;
            } else {
                sidx[0] = -1;
                for (int j = 0; j < D; j++) out_sub[q * D + j] = -1;
            }
        }
        __syncthreads();
        // a subset listed more than once is taken once
        const int64_t pk = sidx[0];
        if (pk >= 0)
            for (int64_t e = threadIdx.x; e < n; e += 256) {
                bool same = !taken[e];
                for (int j = 0; j < D && same; j++) same = rows[e * D + j] == rows[pk * D + j];
                if (same) taken[e] = 1;
            }
        __syncthreads();
    }
    if (threadIdx.x == 0) *nfound = found;
}

__global__ void k_bnb_nan(double* __restrict__ p, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
        p[e] = __longlong_as_double(0x7FF8000000000000LL);
}

constexpr int64_t BNB_GRID = 8192;                 // blocks of an expansion launch (waves loop)
constexpr int64_t BNB_LEAF_GRID = 2048;            // blocks of a leaf launch: one round of resident waves

template <int A>
void expand_a(const BnbLaunch& g, unsigned grid, hipStream_t st) {
    k_bnb_expand<A><<<grid, 256, 0, st>>>(g);
    k_bnb_scan<<<1, 1024, 0, st>>>(g.nin, g.cnt, g.nbw, g.st);
    k_bnb_emit<A><<<grid, 256, 0, st>>>(g);
}

// The children of g.nin prefixes of length a written to g.out; their
// number to st->out.
void launch_expand(int a, const BnbLaunch& g, hipStream_t st) {
    const unsigned grid = (unsigned)std::min<int64_t>(cdiv(g.nin, 4), BNB_GRID);
    switch (a) {
    case 0: expand_a<0>(g, grid, st); break;
    case 1: expand_a<1>(g, grid, st); break;
    case 2: expand_a<2>(g, grid, st); break;
    case 3: expand_a<3>(g, grid, st); break;
    case 4: expand_a<4>(g, grid, st); break;
    case 5: expand_a<5>(g, grid, st); break;
    default: expand_a<6>(g, grid, st); break;
    }
    check_launch("k_bnb_expand");
}

constexpr int64_t BNB_PAIR_GRID = 2048;            // blocks of a pair launch

// The leaves of g.nin parents of length a = D - 2 by the pair form, then
// the threshold update.
void launch_pairs(discover_ctx* ctx, int a, const BnbLaunch& g, int m, int64_t cap, hipStream_t st) {
    const unsigned grid = (unsigned)std::min<int64_t>(g.nin, BNB_PAIR_GRID);
    const size_t lds = (size_t)(a + 2) * g.T.S * sizeof(double);
    {
    KTimer kt(ctx, st, "bnb_pairs");
    switch (a) {
    case 0: k_bnb_pairs<0><<<grid, 256, lds, st>>>(g, cap); break;
    case 1: k_bnb_pairs<1><<<grid, 256, lds, st>>>(g, cap); break;
    case 2: k_bnb_pairs<2><<<grid, 256, lds, st>>>(g, cap); break;
    case 3: k_bnb_pairs<3><<<grid, 256, lds, st>>>(g, cap); break;
    case 4: k_bnb_pairs<4><<<grid, 256, lds, st>>>(g, cap); break;
    case 5: k_bnb_pairs<5><<<grid, 256, lds, st>>>(g, cap); break;
    default: k_bnb_pairs<6><<<grid, 256, lds, st>>>(g, cap); break;
    }
    }
    k_bnb_topm<<<1, 256, 0, st>>>(g.st, g.blk_best, grid, m, g.blk_cnt);
    check_launch("k_bnb_pairs");
}

// The leaves of g.nin prefixes of length a, then the threshold update.
void launch_leaves(int a, const BnbLaunch& g, int m, hipStream_t st) {
    const unsigned grid = (unsigned)std::min<int64_t>(cdiv(g.nin, 4), BNB_LEAF_GRID);
    switch (a) {
    case 0: k_bnb_leaves<0><<<grid, 256, 0, st>>>(g); break;
    case 1: k_bnb_leaves<1><<<grid, 256, 0, st>>>(g); break;
    case 2: k_bnb_leaves<2><<<grid, 256, 0, st>>>(g); break;
    case 3: k_bnb_leaves<3><<<grid, 256, 0, st>>>(g); break;
    case 4: k_bnb_leaves<4><<<grid, 256, 0, st>>>(g); break;
    case 5: k_bnb_leaves<5><<<grid, 256, 0, st>>>(g); break;
    case 6: k_bnb_leaves<6><<<grid, 256, 0, st>>>(g); break;
    default: k_bnb_leaves<7><<<grid, 256, 0, st>>>(g); break;
    }
    k_bnb_topm<<<1, 256, 0, st>>>(g.st, g.blk_best, grid, m, g.blk_cnt);
    check_launch("k_bnb_leaves");
}

int64_t binom_sat(int64_t n, int k) {
    double r = 1.0;
    for (int i = 1; i <= k; i++) r = r * (double)(n - k + i) / (double)i;
    return r >= 9.2e18 ? INT64_MAX : (int64_t)(r + 0.5);
}

// Host mirror of the counters read after each launch.
struct HostCounts {
    unsigned long long out, ncand, nbounds, nleaves;
    int32_t m0, stop;
    double thr;
    int32_t nfound;
};

void read_counts(discover_ctx* ctx, BnbState* dst, int32_t* nfound, HostCounts& h, hipStream_t st) {
    char* pin = (char*)ctx->pinned_buf("bnb_counts", 128);
    DSC_HIP(hipMemcpyAsync(pin, dst, offsetof(BnbState, top), hipMemcpyDeviceToHost, st));
    if (nfound) DSC_HIP(hipMemcpyAsync(pin + 96, nfound, 4, hipMemcpyDeviceToHost, st));
    DSC_HIP(hipStreamSynchronize(st));
    BnbState s;
    std::memcpy(&s, pin, offsetof(BnbState, top));
    h.out = s.out; h.ncand = s.ncand; h.nbounds = s.nbounds; h.nleaves = s.nleaves;
    h.m0 = s.m0; h.stop = s.stop; h.thr = s.thr;
    if (nfound) std::memcpy(&h.nfound, pin + 96, 4);
}

// One problem's search; returns its status.
discover_status bnb_one(discover_ctx* ctx, const discover_l0_problem& pb, int D, int m, int64_t max_nodes,
                        int32_t* out_sub, double* out_rmse, double* out_coef, double* out_resid, int64_t ldr,
                        discover_bnb_stats& stats, hipStream_t st) {
    const int S = pb.S;
    const std::string tg = ctx->tag;
    stats = discover_bnb_stats{};
    stats.n_subsets = binom_sat(S, D);
    const GramOut go = l0_gram_one(ctx, pb, "bnb", st);
    // state: thr = -1 (nothing known), top = -1, counters 0
    BnbState* dst = ctx->buf<BnbState>("bnb_state" + tg, 1);
    {
        BnbState h{};
        h.thr = -1.0;
        h.seed_thr = -1.0;
        for (int q = 0; q < BNB_MAX_M; q++) h.top[q] = -1.0;
        BnbState* up = (BnbState*)ctx->upload("bnb_state_init", &h, sizeof h, st);
        DSC_HIP(hipMemcpyAsync(dst, up, sizeof h, hipMemcpyDeviceToDevice, st));
    }
    // 1. reverse-order factor (y last) and m0
    const int lda = (int)cdiv(S + 1, 2) * 2;
    double* Aw = ctx->buf<double>("bnb_A" + tg, (size_t)(S + 1) * lda);
    {
        KTimer kt(ctx, st, "bnb_factor");
        k_bnb_load<<<dim3((unsigned)cdiv(S + 1, 256), (unsigned)(S + 1)), 256, 0, st>>>(go.G, go.ldg, S, Aw, lda);
        for (int u0 = 0; u0 < S; u0 += BNB_PANEL) {
            k_bnb_panel<<<1, 1024, 0, st>>>(Aw, lda, S, u0, go.G, go.ldg, dst);
            const int c0 = u0 + BNB_PANEL;
            if (c0 <= S)
                k_bnb_update<<<dim3((unsigned)cdiv(S + 1 - c0, 256), (unsigned)(S + 1 - c0)), 256, 0, st>>>(
                    Aw, lda, S, u0, dst);
        }
        check_launch("k_bnb_panel");
    }
    HostCounts hc{};
    read_counts(ctx, dst, nullptr, hc, st);
    {
        double yy = 0.0;
        DSC_HIP(hipMemcpy(&yy, go.yy, 8, hipMemcpyDeviceToHost));
        if (!(yy > 0.0)) {
            stats.status = DISCOVER_E_NUMERIC;
            return DISCOVER_E_NUMERIC;
        }
    }
    const int m0 = hc.m0;
    stats.m0 = m0;
    // 2. prefix-sum tables
    std::vector<int64_t> off(S + 1, 0);
    for (int q = 0; q < S; q++) off[q + 1] = off[q] + (int64_t)(q + 1) * (std::min(m0, S - 1 - q) + 1);
    BnbTab T{};
    T.G = go.G; T.dg = go.dg; T.ldg = go.ldg; T.S = S; T.m0 = m0;
    double* PW = ctx->buf<double>("bnb_PW" + tg, (size_t)std::max<int64_t>(off[S], 1));
    double* PV = ctx->buf<double>("bnb_PV" + tg, (size_t)S * (m0 + 1));
    double* VV = ctx->buf<double>("bnb_VV" + tg, (size_t)m0 + 1);
    T.off = ctx->upload("bnb_off", off, st);
    T.PW = PW; T.PV = PV; T.VV = VV;
    {
        KTimer kt(ctx, st, "bnb_tables");
        const int64_t npair = (int64_t)S * (S + 1) / 2;
        k_bnb_tables<<<(unsigned)cdiv(npair + S + 1, 4), 256, 0, st>>>(Aw, lda, S, m0, T.off, PW, PV, VV, npair);
        check_launch("k_bnb_tables");
    }
    // 3. a starting threshold from a local search, then the walk
    {
        KTimer kt(ctx, st, "bnb_seed");
        double* nv = ctx->buf<double>("bnb_seed_nv" + tg, (size_t)D * S);
        k_bnb_seed<<<1, 256, 0, st>>>(go.G, go.ldg, S, D, m, nv, dst);
        check_launch("k_bnb_seed");
    }
    std::vector<Node*> lvl(D, nullptr);
    std::vector<int64_t> head(D, 0), tail(D, 0);
    for (int a = 1; a < D - 1; a++) lvl[a] = ctx->buf<Node>("bnb_lvl" + std::to_string(a) + tg, BNB_LEVEL_CAP);
    Node* cand[2] = {ctx->buf<Node>("bnb_cand0" + tg, BNB_CAND_CAP), ctx->buf<Node>("bnb_cand1" + tg, BNB_CAND_CAP)};
    double* cval[2] = {ctx->buf<double>("bnb_cval0" + tg, BNB_CAND_CAP),
                       ctx->buf<double>("bnb_cval1" + tg, BNB_CAND_CAP)};
    int cur = 0;
    const int64_t chunk_max = std::min<int64_t>(BNB_LEVEL_CAP / std::max(1, S), 1 << 17);
    Node* root = ctx->buf<Node>("bnb_root" + tg, 1);
    {
        Node z{};
        Node* up = (Node*)ctx->upload("bnb_root_init", &z, sizeof z, st);
        DSC_HIP(hipMemcpyAsync(root, up, sizeof z, hipMemcpyDeviceToDevice, st));
    }
    BnbLaunch g{};
    g.T = T; g.st = dst; g.D = D;
    g.cut = ctx->buf<int32_t>("bnb_cut" + tg, (size_t)chunk_max);
    g.cnt = ctx->buf<int64_t>("bnb_cnt" + tg, (size_t)chunk_max);
    g.nbw = ctx->buf<int32_t>("bnb_nbw" + tg, (size_t)chunk_max);
    int32_t* vpre = ctx->buf<int32_t>("bnb_vpre" + tg, (size_t)S + 1);
    k_bnb_vpre<<<1, 1024, 0, st>>>(go.dg, S, vpre);
    g.vpre = vpre;
    g.blk_best = ctx->buf<double>("bnb_blk_best" + tg, (size_t)BNB_LEAF_GRID);
    g.blk_cnt = ctx->buf<unsigned long long>("bnb_blk_cnt" + tg, (size_t)BNB_LEAF_GRID);
    int64_t ncand = 0;
    int64_t nodes = 0;
    // keep the listed leaves within GRAM_DELTA of thr (the list's counter
    // restarts at the compacted length)
    auto compact = [&]() {
        fill_all(ctx, "bnb_ncand_fill", {fill_seg(&dst->ncand, 8, 0u)}, st);
        k_bnb_compact<<<(unsigned)std::min<int64_t>(cdiv(std::max<int64_t>(ncand, 1), 256), 4096), 256, 0, st>>>(
            dst, cand[cur], cval[cur], ncand, cand[1 - cur], cval[1 - cur], &dst->ncand);
        check_launch("k_bnb_compact");
        read_counts(ctx, dst, nullptr, hc, st);
        cur = 1 - cur;
        ncand = (int64_t)hc.ncand;
    };
    // the pair form over parents [in, in + nin); when the leaf list
    // overflowed, what was written is compacted and the launch redone (a
    // leaf listed twice is taken once by the ranking)
    auto pairs = [&](int a, const Node* in, int64_t nin) {
        for (;;) {
            g.in = in;
            g.nin = nin;
            g.cand = cand[cur];
            g.cval = cval[cur];
            launch_pairs(ctx, a, g, m, BNB_CAND_CAP, st);
            read_counts(ctx, dst, nullptr, hc, st);
            ncand = (int64_t)hc.ncand;
            if (ncand <= BNB_CAND_CAP) return;
            ncand = BNB_CAND_CAP;
            compact();
            if (ncand > BNB_CAND_CAP / 2)
                DSC_FAIL(DISCOVER_E_CAPACITY, "the band of near-best subsets exceeds %lld entries",
                         (long long)(BNB_CAND_CAP / 2));
        }
    };
    // the root (the empty prefix): its leaves (D = 1), its pairs (D = 2), or
    // its children; then the walk over levels 1 .. D - 2
    {
        KTimer kt(ctx, st, "bnb_search");
        g.in = root;
        g.nin = 1;
        if (D == 1) {
            g.cand = cand[cur]; g.cval = cval[cur];
            launch_leaves(0, g, m, st);
            read_counts(ctx, dst, nullptr, hc, st);
            ncand = (int64_t)hc.ncand;
        } else if (D == 2) {
            pairs(0, root, 1);
        } else {
            g.out = lvl[1];
            launch_expand(0, g, st);
            read_counts(ctx, dst, nullptr, hc, st);
            tail[1] = (int64_t)hc.out;
        }
        nodes = 1;
        for (;;) {
            int a = D - 2;
            while (a >= 1 && head[a] == tail[a]) a--;
            if (a < 1) break;
            if (max_nodes > 0 && nodes >= max_nodes) {
                stats.status = DISCOVER_E_CAPACITY;
                break;
            }
            int64_t ch = std::min(tail[a] - head[a], chunk_max);
            if (a == D - 2) {
                if (max_nodes > 0) ch = std::min(ch, std::max<int64_t>(1, max_nodes - nodes));
                pairs(a, lvl[a] + head[a], ch);
            } else {
                g.in = lvl[a] + head[a];
                g.nin = ch;
                g.out = lvl[a + 1];
                launch_expand(a, g, st);
                read_counts(ctx, dst, nullptr, hc, st);
                head[a + 1] = 0;
                tail[a + 1] = (int64_t)hc.out;
            }
            head[a] += ch;
            nodes += ch;
            if (head[a] == tail[a]) head[a] = tail[a] = 0;
        }
    }
    stats.n_nodes = nodes;
    stats.n_bounds = (int64_t)hc.nbounds;
    stats.n_leaves = (int64_t)hc.nleaves;
    if (stats.status == DISCOVER_E_CAPACITY) return DISCOVER_E_CAPACITY;
    // 4. the band: listed leaves within GRAM_DELTA of the final thr, by QR
    if (ncand > 0) compact();
    stats.n_refit = ncand;
    int32_t* rows = ctx->buf<int32_t>("bnb_rows" + tg, (size_t)std::max<int64_t>(ncand, 1) * D);
    double* rss = ctx->buf<double>("bnb_rss" + tg, (size_t)std::max<int64_t>(ncand, 1));
    uint8_t* taken = ctx->buf<uint8_t>("bnb_taken" + tg, (size_t)std::max<int64_t>(ncand, 1));
    int32_t* nfound = ctx->buf<int32_t>("bnb_nfound" + tg, 1);
    {
        KTimer kt(ctx, st, "bnb_refit");
        if (ncand > 0) {
            k_bnb_rows<<<(unsigned)std::min<int64_t>(cdiv(ncand, 256), 4096), 256, 0, st>>>(cand[cur], ncand, D, rows);
            refit_list(ctx, pb, D, rows, ncand, rss, st);
        }
        k_bnb_rank<<<1, 256, 0, st>>>(rows, rss, ncand, D, m, pb.ids, go.yy, taken, out_sub, nfound);
        check_launch("k_bnb_rank");
    }
    read_counts(ctx, dst, nfound, hc, st);
    const int found = hc.nfound;
    if (found == 0) {
        stats.status = DISCOVER_E_NUMERIC;
        return DISCOVER_E_NUMERIC;
    }
    std::vector<discover_l0_problem> reps(found, pb);
    fit_rows(ctx, reps.data(), found, D, out_sub, D, out_coef, D + 1, out_rmse, out_resid, ldr, st);
    if (found < m) {
        k_bnb_nan<<<1, 256, 0, st>>>(out_rmse + found, m - found);
        k_bnb_nan<<<1, 256, 0, st>>>(out_coef + (int64_t)found * (D + 1), (int64_t)(m - found) * (D + 1));
        if (out_resid)
            for (int q = found; q < m; q++) k_bnb_nan<<<1, 256, 0, st>>>(out_resid + q * ldr, pb.n);
        check_launch("k_bnb_nan");
    }
    DSC_HIP(hipStreamSynchronize(st));
    stats.status = DISCOVER_OK;
    return DISCOVER_OK;
}

}  // namespace
}  // namespace dsc

extern "C" discover_status discover_l0_bnb(discover_ctx* ctx, const discover_l0_problem* probs,
                                           int32_t n_problems, int32_t D, int32_t m,
                                           const discover_bnb_params* prm, int32_t* out_subsets,
                                           double* out_rmse, double* out_coef, double* out_resid, int64_t ldr,
                                           discover_bnb_stats* out_stats, void* stream) {
    using namespace dsc;
    return guarded([&] {
        DSC_REQUIRE(ctx && probs && n_problems >= 1, "ctx/probs/n_problems");
        DSC_REQUIRE(D >= 1 && D <= DISCOVER_MAX_D, "D = %d outside 1..%d", D, DISCOVER_MAX_D);
        DSC_REQUIRE(m >= 1 && m <= BNB_MAX_M, "m = %d outside 1..%d", m, BNB_MAX_M);
        DSC_REQUIRE(!prm || (prm->max_nodes >= 0 && prm->reserved == 0), "prm");
        DSC_REQUIRE(out_subsets && out_rmse && out_coef, "outputs required");
        for (int b = 0; b < n_problems; b++) {
            const discover_l0_problem& p = probs[b];
            DSC_REQUIRE(p.S >= D && p.S <= BNB_MAX_S, "problem %d: S = %d outside D..%d", b, p.S, BNB_MAX_S);
            DSC_REQUIRE(p.n >= D + 2, "problem %d: n = %d < D + 2", b, p.n);
            DSC_REQUIRE(p.F && p.ids && p.y && p.ldf >= p.n, "problem %d: F/ids/y/ldf", b);
            DSC_REQUIRE(!out_resid || ldr >= p.n, "problem %d: ldr < n", b);
        }
        DSC_HIP(hipSetDevice(ctx->device));
        const hipStream_t st = (hipStream_t)stream;
        DSC_REQUIRE(!stream_capturing(st), "the branch-and-bound search steers itself from the host and "
                                           "cannot be captured");
        discover_status worst = DISCOVER_OK;
        std::string msg;
        for (int b = 0; b < n_problems; b++) {
            discover_bnb_stats s{};
            const discover_status r =
                bnb_one(ctx, probs[b], D, m, prm ? prm->max_nodes : 0, out_subsets + (int64_t)b * m * D,
                        out_rmse + (int64_t)b * m, out_coef + (int64_t)b * m * (D + 1),
                        out_resid ? out_resid + (int64_t)b * m * ldr : nullptr, ldr, s, st);
            if (out_stats) out_stats[b] = s;
            if (r != DISCOVER_OK && worst == DISCOVER_OK) {
                worst = r;
                msg = r == DISCOVER_E_CAPACITY ? "problem " + std::to_string(b) + ": max_nodes reached"
                                               : "problem " + std::to_string(b) +
                                                     ": constant y or no non-singular subset";
            }
        }
        if (worst != DISCOVER_OK) DSC_FAIL(worst, "%s", msg.c_str());
    });
}
