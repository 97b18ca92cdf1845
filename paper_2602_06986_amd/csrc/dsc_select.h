// Radix selection of the K-th largest positive double (bits of a positive
// double are monotone in its value): three 12-bit levels below the sign
// bit.  Shared by the screening pool and the L0 band.
#pragma once

#include <algorithm>

#include "dsc_common.h"

namespace dsc {

static __global__ __launch_bounds__(256) void k_hist(const double* __restrict__ sc, int64_t N, int level,
                                              const uint32_t* __restrict__ sel,
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
        const uint64_t u = (uint64_t)__double_as_longlong(x);
        if (level > 0 && ((u >> 51) & 0xFFF) != p0) continue;
        if (level > 1 && ((u >> 39) & 0xFFF) != p1) continue;
        atomicAdd(&h[(u >> (51 - 12 * level)) & 0xFFF], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < 4096; b += 256)
        if (h[b]) atomicAdd(&hist[b], h[b]);
}

// st[0] = remaining rank K, st[1] = take-all flag
static __global__ void k_find(const uint32_t* __restrict__ hist, int level, uint32_t* __restrict__ sel,
                       int64_t* __restrict__ st) {
    if (threadIdx.x != 0) return;
    int64_t K = st[0];
    int64_t cum = 0, total = 0;
    for (int b = 0; b < 4096; b++) total += hist[b];
    if (st[1] || total < K) {          // fewer candidates than requested: take all
        st[1] = 1;
        sel[level] = 0;
        return;
    }
    for (int b = 4095; b >= 0; b--) {
        if (cum + hist[b] >= K) {
            sel[level] = b;
            st[0] = K - cum;
            return;
        }
        cum += hist[b];
    }
}

static __device__ __forceinline__ double select_threshold(const uint32_t* sel, const int64_t* st) {
    if (st[1]) return 0.0;
    const uint64_t key = ((uint64_t)sel[0] << 51) | ((uint64_t)sel[1] << 39) | ((uint64_t)sel[2] << 27);
    return __longlong_as_double((long long)key);
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
        k_find<<<1, 64, 0, s>>>(hist, level, sel, st);
    }
    check_launch("radix_select");
}

}  // namespace dsc
