// Shared host/device plumbing of the discover library: error reporting,
// the context (device workspace arena, kernel timing) and wave/block
// reductions for 64-wide CDNA wavefronts.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "../../include/discover.h"

namespace dsc {

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
const char* get_error();

struct Error {
    discover_status code;
};

#define DSC_FAIL(code, ...)                         \
    do {                                            \
        ::dsc::set_error(__VA_ARGS__);              \
        throw ::dsc::Error{code};                   \
    } while (0)

#define DSC_HIP(call)                                                        \
    do {                                                                     \
        hipError_t e_ = (call);                                              \
        if (e_ != hipSuccess)                                                \
            DSC_FAIL(DISCOVER_E_HIP, "%s failed: %s (%s:%d)", #call,         \
                     hipGetErrorString(e_), __FILE__, __LINE__);             \
    } while (0)

#define DSC_REQUIRE(cond, ...)                                               \
    do {                                                                     \
        if (!(cond)) DSC_FAIL(DISCOVER_E_ARG, __VA_ARGS__);                  \
    } while (0)

// Run a body that may throw dsc::Error and convert to a status code.
template <class F>
discover_status guarded(F&& f) {
    try {
        f();
        return DISCOVER_OK;
    } catch (const Error& e) {
        return e.code;
    } catch (const std::exception& e) {
        set_error("internal error: %s", e.what());
        return DISCOVER_E_HIP;
    } catch (...) {
        set_error("internal error");
        return DISCOVER_E_HIP;
    }
}

constexpr int WAVE = 64;

}  // namespace dsc

// ---------------------------------------------------------------- context
struct discover_ctx {
    int device = 0;
    struct Buf {
        void* p = nullptr;
        size_t cap = 0;
    };
    std::map<std::string, Buf> bufs;
    bool timing = false;
    std::map<std::string, std::pair<int64_t, double>> times;
    struct Pending {
        std::string name;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> free_events;
    std::map<std::string, std::shared_ptr<void>> plans;   // cached search-space plans

    // Grow-only named device buffer of at least `bytes` bytes.
    void* raw(const std::string& name, size_t bytes) {
        Buf& b = bufs[name];
        if (bytes == 0) bytes = 256;
        if (b.cap < bytes) {
            if (b.p) {
                hipError_t e = hipFree(b.p);
                (void)e;
                b.p = nullptr;
                b.cap = 0;
            }
            size_t want = bytes + bytes / 4;
            want = (want + 4095) & ~size_t(4095);
            if (hipMalloc(&b.p, want) != hipSuccess) {
                b.p = nullptr;
                DSC_FAIL(DISCOVER_E_NOMEM, "device allocation of %zu bytes (%s) failed", want,
                         name.c_str());
            }
            b.cap = want;
        }
        return b.p;
    }
    template <class T>
    T* buf(const std::string& name, size_t count) {
        return static_cast<T*>(raw(name, count * sizeof(T)));
    }

    hipEvent_t event() {
        if (!free_events.empty()) {
            hipEvent_t e = free_events.back();
            free_events.pop_back();
            return e;
        }
        hipEvent_t e;
        DSC_HIP(hipEventCreate(&e));
        return e;
    }
    // Accumulate the pending kernel times (the stream must be synchronised).
    void resolve_timing() {
        for (auto& p : pending) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
                auto& t = times[p.name];
                t.first += 1;
                t.second += ms;
            }
            free_events.push_back(p.a);
            free_events.push_back(p.b);
        }
        pending.clear();
    }
};

namespace dsc {

// Brackets one kernel launch with HIP events on its stream when timing is on.
struct KTimer {
    discover_ctx* c;
    hipStream_t s;
    const char* name;
    hipEvent_t a = nullptr, b = nullptr;
    KTimer(discover_ctx* c_, hipStream_t s_, const char* n) : c(c_), s(s_), name(n) {
        if (c->timing) {
            a = c->event();
            b = c->event();
            DSC_HIP(hipEventRecord(a, s));
        }
    }
    ~KTimer() {
        if (a && hipEventRecord(b, s) == hipSuccess) c->pending.push_back({name, a, b});
    }
};

inline void check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        DSC_FAIL(DISCOVER_E_HIP, "launch of %s failed: %s", what, hipGetErrorString(e));
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ------------------------------------------------------- device helpers
// Wave-wide sum in a fixed butterfly order; every lane returns lane 0's
// result so that all lanes agree bit for bit.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return __shfl(v, 0, 64);
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return __shfl(v, 0, 64);
}

__host__ __device__ __forceinline__ int64_t choose2(int64_t m) { return m * (m - 1) / 2; }

}  // namespace dsc
