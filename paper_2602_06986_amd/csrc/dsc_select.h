// Radix selection of the K-th largest positive double (bits of a positive
// double are monotone in its value): three 12-bit levels below the sign
// bit.  Shared by the screening pool and the L0 band.
#pragma once

#include <algorithm>

#include "dsc_common.h"

namespace dsc {

// Key of a score in [0, 1): its 52-bit fixed-point value (monotone, uniform
// resolution; values >= 1 saturate).  Three 12-bit levels cover bits 51..16,
// so the selected threshold is exact in double and within 2^-36 of the
// K-th largest value.
static __device__ __forceinline__ uint64_t fx_key(double x) {
    const double c = x < 0.9999999999999999 ? x : 0.9999999999999999;
    return (uint64_t)(c * 4503599627370496.0);          // * 2^52
}

static __global__ __launch_bounds__(256) void k_hist(const double* __restrict__ sc, int64_t N,
                                                     int level, const uint32_t* __restrict__ sel,
                                                     uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[4096];
    for (int b = threadIdx.x; b < 4096; b += 256) h[b] = 0;
    __syncthreads();
    uint32_t p0 = 0, p1 = 0;
    if (level > 0) p0 = sel[0];
    if (level > 1) p1 = sel[1];
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
        if (h[b]) atomicAdd(&hist[b], h[b]);
}

// st[0] = remaining rank K, st[1] = take-all flag.  One block of 256
// threads: thread t owns bins [16t, 16t+16); a suffix scan over threads
// gives the count above each range.
static __global__ __launch_bounds__(256) void k_find(const uint32_t* __restrict__ hist, int level,
                                                     uint32_t* __restrict__ sel,
                                                     int64_t* __restrict__ st) {
    __shared__ int64_t part[256];
    const int t = threadIdx.x;
    int64_t loc = 0;
    uint32_t hb[16];
    for (int q = 0; q < 16; q++) {
        hb[q] = hist[t * 16 + q];
        loc += hb[q];
    }
    part[t] = loc;
    __syncthreads();
    // inclusive suffix sums (Hillis-Steele over 256 entries)
    for (int o = 1; o < 256; o <<= 1) {
        const int64_t v = t + o < 256 ? part[t + o] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    const int64_t K = st[0];
    const int64_t total = part[0];
    const bool all = st[1] != 0 || total < K;
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

static inline double host_threshold(const uint32_t* sel, const int64_t* st) {
    if (st[1]) return 0.0;
    const uint64_t key = ((uint64_t)sel[0] << 40) | ((uint64_t)sel[1] << 28) | ((uint64_t)sel[2] << 16);
    return (double)key * 2.220446049250313e-16;
}

// Launch the three levels; afterwards sel/st describe the K-th largest
// positive entry of x (st[1] = 1 when fewer than K positive entries exist).
static inline void radix_select(const double* x, int64_t N, int64_t K, uint32_t* hist,
                                uint32_t* sel, int64_t* st, hipStream_t s) {
    const int64_t init[2] = {K, 0};
    DSC_HIP(hipMemcpyAsync(st, init, sizeof init, hipMemcpyHostToDevice, s));
    DSC_HIP(hipMemsetAsync(sel, 0, 16, s));
    const unsigned hb = (unsigned)std::min<int64_t>(1024, std::max<int64_t>(1, cdiv(N, 256 * 8)));
    for (int level = 0; level < 3; level++) {
        DSC_HIP(hipMemsetAsync(hist, 0, 4096 * 4, s));
        k_hist<<<hb, 256, 0, s>>>(x, N, level, sel, hist);
        k_find<<<1, 256, 0, s>>>(hist, level, sel, st);
    }
    check_launch("radix_select");
}

}  // namespace dsc
