// Radix selection of a lower bound of the K-th largest positive value: one
// or two 12-bit levels of a fixed-point key.  Its users need only a bound
// at most the K-th value (the screening pool and the L0 band reach below it
// by their own margins); one level bounds it within 2^-12 (the screening
// pool), two within 2^-24 (the L0 band, whose refits grow with the band).
#pragma once

#include <algorithm>

#include "dsc_common.h"

namespace dsc {

// Key of a score in [0, 1): its 52-bit fixed-point value (monotone, uniform
// resolution; values >= 1 saturate).  The two 12-bit levels cover bits
// 51..28, so the selected threshold is exact in double, at most the K-th
// largest value and within 2^-24 of it.
constexpr int RADIX_LEVELS = 2;

static __device__ __forceinline__ uint64_t fx_key(double x) {
    const double c = x < 0.9999999999999999 ? x : 0.9999999999999999;
    return (uint64_t)(c * 4503599627370496.0);          // * 2^52
}

// One radix selection per list: x[0..N) holds the values (entries <= 0 are
// ignored), K the rank wanted; hist holds two 4096-bin histograms (one per
// level), sel the selected 12-bit digits (sel[2] stays 0), st[0] the
// remaining rank and st[1] the take-all flag (fewer than K positive
// entries).  Before the selection, hist, st and sel must be zero (the
// callers clear them with their other counters).  A level's digit is read
// from its finished histogram by every block of the next kernel (the
// level-1 histogram for level 0, the selection's consumer for level 1), so
// no launch is spent on it; block 0 of that kernel publishes it.
struct RadixArgs {
    const double* x;
    int64_t N;
    int64_t K;
    uint32_t* hist;
    uint32_t* sel;
    int64_t* st;
    const unsigned long long* Nd;   // or NULL: device count of entries (at most N)
};

struct RadixDigit {
    uint32_t digit;
    int64_t rank;                   // rank left within the digit's bin
    bool all;                       // fewer than the wanted rank: take all
};

// The digit holding rank K of a finished histogram, by the 256 threads of a
// block (every thread gets it): thread t owns bins [16t, 16t+16) and a
// suffix scan over threads gives the count above each range.
static __device__ __forceinline__ RadixDigit radix_digit(const uint32_t* __restrict__ hist, int64_t K,
                                                         bool all_in) {
    __shared__ int64_t part[256];
    __shared__ uint32_t s_digit;
    __shared__ int64_t s_rank;
    const int t = threadIdx.x;
    int64_t loc = 0;
    uint32_t hb[16];
    for (int q = 0; q < 16; q++) {
        hb[q] = hist[t * 16 + q];
        loc += hb[q];
    }
    part[t] = loc;
    if (t == 0) {
        s_digit = 0;
        s_rank = K;
    }
    __syncthreads();
    // inclusive suffix sums (Hillis-Steele over 256 entries)
    for (int o = 1; o < 256; o <<= 1) {
        const int64_t v = t + o < 256 ? part[t + o] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    const bool all = all_in || part[0] < K;
    const int64_t above = t + 1 < 256 ? part[t + 1] : 0;     // count in bins above my range
    if (!all && above < K && above + loc >= K) {              // exactly one thread
        int64_t cum = above;
        for (int q = 15; q >= 0; q--) {
            if (cum + hb[q] >= K) {
                s_digit = (uint32_t)(t * 16 + q);
                s_rank = K - cum;
                break;
            }
            cum += hb[q];
        }
    }
    __syncthreads();
    const RadixDigit r{s_digit, s_rank, all};
    __syncthreads();                                          // part and s_* free again
    return r;
}

// grid (blocks, lists).  Level 1 first reads the level-0 digit.
static __global__ __launch_bounds__(256) void k_hist(ctab<RadixArgs> A, int level) {
    const RadixArgs& a = tab(A, blockIdx.y);
    DSC_GLOBAL(a.x); DSC_GLOBAL(a.hist); DSC_GLOBAL(a.sel); DSC_GLOBAL(a.st); DSC_GLOBAL(a.Nd);
    __shared__ uint32_t h[4096];
    uint32_t p0 = 0;
    if (level == 1) {
        const RadixDigit d0 = radix_digit(a.hist, a.K, false);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            a.sel[0] = d0.digit;
            a.st[0] = d0.rank;
            a.st[1] = d0.all ? 1 : 0;
        }
        if (d0.all) return;                               // (block-uniform) nothing left to split
        p0 = d0.digit;
    }
    for (int b = threadIdx.x; b < 4096; b += 256) h[b] = 0;
    __syncthreads();
    const double* __restrict__ sc = a.x;
    const int64_t N = a.Nd ? min((int64_t)*a.Nd, a.N) : a.N;
    // four strided values per thread are loaded before any is counted, so
    // the loads overlap instead of each waiting for the one before
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i0 = (int64_t)blockIdx.x * 256 + threadIdx.x; i0 < N; i0 += 4 * stride) {
        double xs[4];
#pragma unroll
        for (int q = 0; q < 4; q++) xs[q] = i0 + q * stride < N ? sc[i0 + q * stride] : 0.0;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            if (!(xs[q] > 0.0)) continue;
            const uint64_t u = fx_key(xs[q]);
            if (level == 1 && ((u >> 40) & 0xFFF) != p0) continue;
            atomicAdd(&h[(u >> (40 - 12 * level)) & 0xFFF], 1u);
        }
    }
    __syncthreads();
    uint32_t* hout = a.hist + level * 4096;
    for (int b = threadIdx.x; b < 4096; b += 256)
        if (h[b]) atomicAdd(&hout[b], h[b]);
}

// One level only: the consumer reads the level-0 digit for rank K (a lower
// bound within 2^-12 of the K-th value); sel[1] stays 0.
static __device__ __forceinline__ void radix_finish1(const uint32_t* __restrict__ hist, int64_t K,
                                                     uint32_t* __restrict__ gsel, int64_t* __restrict__ gst,
                                                     uint32_t (&sel)[3], int64_t (&st)[2]) {
    const RadixDigit d0 = radix_digit(hist, K, false);
    sel[0] = d0.all ? 0u : d0.digit;
    sel[1] = 0u;
    sel[2] = 0u;
    st[0] = d0.rank;
    st[1] = d0.all ? 1 : 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        gsel[0] = sel[0];
        gst[0] = st[0];
        gst[1] = st[1];
    }
}

// The selection's consumer: every block reads the level-1 digit into sel
// and st (its own copies); block 0 publishes them for later kernels.
static __device__ __forceinline__ void radix_finish(const uint32_t* __restrict__ hist,
                                                    uint32_t* __restrict__ gsel, int64_t* __restrict__ gst,
                                                    uint32_t (&sel)[3], int64_t (&st)[2]) {
    const bool all0 = gst[1] != 0;
    const RadixDigit d1 = radix_digit(hist + 4096, gst[0], all0);
    sel[0] = gsel[0];
    sel[1] = d1.all ? 0u : d1.digit;
    sel[2] = 0u;
    st[0] = d1.rank;
    st[1] = d1.all ? 1 : 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        gsel[1] = sel[1];
        gst[0] = st[0];
        gst[1] = st[1];
    }
}

static __device__ __forceinline__ double select_threshold(const uint32_t* sel, const int64_t* st) {
    if (st[1]) return 0.0;
    const uint64_t key = ((uint64_t)sel[0] << 40) | ((uint64_t)sel[1] << 28) | ((uint64_t)sel[2] << 16);
    return (double)key * 2.220446049250313e-16;          // * 2^-52 (exact)
}

// Launch the histograms of the selections of nl lists (device table A;
// each list's hist, st and sel zero); the consumer's radix_finish then
// gives the K-th largest positive entry of each list.
static inline void radix_select(const RadixArgs* Ad, int nl, int64_t Nmax, hipStream_t s,
                                int levels = RADIX_LEVELS) {
    if (nl <= 0) return;
    const ctab<RadixArgs> A = ct(Ad);
    const unsigned hb = (unsigned)std::min<int64_t>(1024, std::max<int64_t>(1, cdiv(Nmax, 256 * 8)));
    for (int level = 0; level < levels; level++) k_hist<<<dim3(hb, nl), 256, 0, s>>>(A, level);
    check_launch("radix_select");
}

}  // namespace dsc
