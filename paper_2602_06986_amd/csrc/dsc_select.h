// Radix selection of a lower bound of the K-th largest positive value: two
// 12-bit levels of a fixed-point key.  Its users need only a bound at most
// the K-th value (the screening pool and the L0 band reach below it by
// their own margins), and two levels bound it within 2^-24.  Shared by the
// screening pool and the L0 band.
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
// ignored), K the rank wanted; hist is a 4096-bin scratch histogram, sel
// the selected 12-bit digits (sel[2] stays 0), st[0] the remaining rank and
// st[1] the take-all flag (fewer than K positive entries).  Before the
// selection, hist, st and sel must be zero (the callers clear them with
// their other counters, which saves a launch).
struct RadixArgs {
    const double* x;
    int64_t N;
    int64_t K;
    uint32_t* hist;
    uint32_t* sel;
    int64_t* st;
    const unsigned long long* Nd;   // or NULL: device count of entries (at most N)
};

// grid (blocks, lists)
static __global__ __launch_bounds__(256) void k_hist(ctab<RadixArgs> A, int level) {
    const RadixArgs& a = tab(A, blockIdx.y);
    DSC_GLOBAL(a.x); DSC_GLOBAL(a.hist); DSC_GLOBAL(a.sel); DSC_GLOBAL(a.Nd);
    __shared__ uint32_t h[4096];
    for (int b = threadIdx.x; b < 4096; b += 256) h[b] = 0;
    __syncthreads();
    uint32_t p0 = 0, p1 = 0;
    if (level > 0) p0 = a.sel[0];
    if (level > 1) p1 = a.sel[1];
    const double* __restrict__ sc = a.x;
    const int64_t N = a.Nd ? min((int64_t)*a.Nd, a.N) : a.N;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256) {
        const double x = sc[i];
        if (!(x > 0.0)) continue;
        const uint64_t u = fx_key(x);
        if (level > 0 && ((u >> 40) & 0xFFF) != p0) continue;
        if (level > 1 && ((u >> 28) & 0xFFF) != p1) continue;
        atomicAdd(&h[(u >> (40 - 12 * level)) & 0xFFF], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < 4096; b += 256)
        if (h[b]) atomicAdd(&a.hist[b], h[b]);
}

// One block of 256 threads per list: thread t owns bins [16t, 16t+16); a
// suffix scan over threads gives the count above each range.  The
// histogram is cleared for the next level after it has been read.  Level 0
// starts from rank K, later levels from the rank left in st[0].
static __global__ __launch_bounds__(256) void k_find(ctab<RadixArgs> A, int level) {
    const RadixArgs& a = tab(A, blockIdx.x);
    DSC_GLOBAL(a.hist); DSC_GLOBAL(a.sel); DSC_GLOBAL(a.st);
    uint32_t* __restrict__ hist = a.hist;
    uint32_t* __restrict__ sel = a.sel;
    int64_t* __restrict__ st = a.st;
    __shared__ int64_t part[256];
    const int t = threadIdx.x;
    int64_t loc = 0;
    uint32_t hb[16];
    for (int q = 0; q < 16; q++) {
        hb[q] = hist[t * 16 + q];
        loc += hb[q];
    }
    for (int q = 0; q < 16; q++) hist[t * 16 + q] = 0;
    part[t] = loc;
    __syncthreads();
    // inclusive suffix sums (Hillis-Steele over 256 entries)
    for (int o = 1; o < 256; o <<= 1) {
        const int64_t v = t + o < 256 ? part[t + o] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    const int64_t K = level == 0 ? a.K : st[0];
    const int64_t total = part[0];
    const bool all = (level > 0 && st[1] != 0) || total < K;
    __syncthreads();
    if (all) {
        if (t == 0) {
            st[1] = 1;
            sel[level] = 0;
        }
        return;
    }
    const int64_t above = t + 1 < 256 ? part[t + 1] : 0;     // count in bins above my range
    if (above < K && above + loc >= K) {                      // exactly one thread
        int64_t cum = above;
        for (int q = 15; q >= 0; q--) {
            if (cum + hb[q] >= K) {
                sel[level] = (uint32_t)(t * 16 + q);
                st[0] = K - cum;
                break;
            }
            cum += hb[q];
        }
    }
}

static __device__ __forceinline__ double select_threshold(const uint32_t* sel, const int64_t* st) {
    if (st[1]) return 0.0;
    const uint64_t key = ((uint64_t)sel[0] << 40) | ((uint64_t)sel[1] << 28) | ((uint64_t)sel[2] << 16);
    return (double)key * 2.220446049250313e-16;          // * 2^-52 (exact)
}

// Launch the selections of nl lists (device table A; each list's hist, st
// and sel zero); afterwards each list's sel/st describe its K-th largest
// positive entry.
static inline void radix_select(const RadixArgs* Ad, int nl, int64_t Nmax, hipStream_t s) {
    if (nl <= 0) return;
    const ctab<RadixArgs> A = ct(Ad);
    const unsigned hb = (unsigned)std::min<int64_t>(1024, std::max<int64_t>(1, cdiv(Nmax, 256 * 8)));
    for (int level = 0; level < RADIX_LEVELS; level++) {
        k_hist<<<dim3(hb, nl), 256, 0, s>>>(A, level);
        k_find<<<nl, 256, 0, s>>>(A, level);
    }
    check_launch("radix_select");
}

}  // namespace dsc
