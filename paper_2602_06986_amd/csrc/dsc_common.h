// Shared host/device plumbing of the discover library: error reporting,
// the context (device workspace arena, kernel timing) and wave/block
// reductions for 64-wide CDNA wavefronts.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <map>
#include <set>
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
        bool bound = false;    // referenced by a graph a caller captured: never freed
    };
    std::map<std::string, Buf> bufs;
    // small pinned host buffers (hipHostMalloc) that kernels write and the
    // host reads after a synchronisation, kept until the context is destroyed
    std::map<std::string, void*> pinned;
    void* pinned_buf(const std::string& name, size_t bytes) {
        auto it = pinned.find(name);
        if (it != pinned.end()) return it->second;
        if (capturing)
            DSC_FAIL(DISCOVER_E_CAPACITY, "pinned buffer %s would be made during graph capture", name.c_str());
        void* p = nullptr;
        DSC_HIP(hipHostMalloc(&p, bytes, hipHostMallocDefault));
        pinned[name] = p;
        return p;
    }
    bool timing = false;
    std::map<std::string, std::pair<int64_t, double>> times;
    struct Pending {
        std::string name;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> free_events;
    // Timer names whose kernels are bracketed by events inside captured
    // graphs too (each replay then reports their time), and the event pairs
    // recorded by the capture in progress.
    std::set<std::string> graph_timed;
    std::vector<Pending> graph_pending;
    std::map<std::string, std::shared_ptr<void>> plans;   // cached search-space plans
    std::map<std::string, std::shared_ptr<void>> batches; // cached batch plans / graphs
    std::map<std::string, std::vector<char>> shadows;     // host copies of uploaded arguments
    std::map<std::string, int> tuned;                     // autotuned tile choices
    // While a launch sequence is being captured into a graph nothing may
    // allocate, synchronise or copy from the host: buffers must already be
    // large enough and argument tables already uploaded.
    bool capturing = false;
    // The capture in progress is the caller's (a public call made on a
    // stream the caller is capturing): buffers it touches become bound, and
    // new ones may be allocated, which a capture in relaxed mode permits.
    bool caller_capture = false;
    // Set once a caller has captured a call: search-space plans are then
    // never evicted (their device tables may be referenced by that graph).
    bool frozen = false;
    int64_t capture_seq = 0;
    // The call reports its outcome in device memory and must not wait for
    // the stream: one selection round at the remembered sizes, checked on
    // the device.
    bool nosync = false;
    // Suffix of argument-table and result-buffer names, so that the calls of
    // one captured sequence keep tables of their own.
    std::string tag;
    // Operand features of a screen (values, reciprocals, centred copies,
    // their moments and sample-major copies) depend on X alone: a sequence
    // of screens over the same problems keeps them in an arena named by
    // ops_tag and, with ops_reuse set, skips materialising them again when
    // the problems' layout signature matches the one stored in ops_sig.
    std::string ops_tag;
    bool ops_reuse = false;
    std::vector<int64_t> ops_sig;
    // Bumped whenever device memory that a captured graph may reference is
    // released (a buffer regrown, plans evicted); graphs of an older
    // generation are discarded instead of replayed.
    uint64_t generation = 0;
    // Entries of a screen's exact fix-up lists (candidates whose one-pass
    // score is not trusted); a screen that needs more grows this and runs
    // again.
    int64_t fix_cap_min = (int64_t)1 << 22;
    hipStream_t side = nullptr;            // private stream for uploads during capture
    // Selection rules (discover_set_rules): the copied parameters and pairs.
    bool has_rules = false;
    discover_rules rules{};
    std::vector<int32_t> rule_pairs;

    // Grow-only named device buffer of at least `bytes` bytes.
    void* raw(const std::string& name, size_t bytes) {
        Buf& b = bufs[name];
        if (bytes == 0) bytes = 256;
        if (b.cap < bytes) {
            if (b.bound)
                DSC_FAIL(DISCOVER_E_CAPACITY,
                         "buffer %s is referenced by a graph captured from this context and cannot "
                         "grow (reserve larger sizes before capturing, or use another context)",
                         name.c_str());
            if (capturing && !(caller_capture && !b.p))
                DSC_FAIL(DISCOVER_E_CAPACITY,
                         "buffer %s would grow during graph capture (run the call, or "
                         "discover_reserve, outside capture first)", name.c_str());
            if (b.p) {
                hipError_t e = hipFree(b.p);
                (void)e;
                b.p = nullptr;
                b.cap = 0;
                generation++;
            }
            size_t want = bytes + bytes / 4;
            want = (want + 4095) & ~size_t(4095);
            if (hipMalloc(&b.p, want) != hipSuccess) {
                b.p = nullptr;
                (void)hipGetLastError();
                if (capturing)
                    DSC_FAIL(DISCOVER_E_CAPACITY,
                             "allocation of %zu bytes (%s) during graph capture failed: capture in "
                             "relaxed mode, or size the workspace (discover_reserve) first",
                             want, name.c_str());
                DSC_FAIL(DISCOVER_E_NOMEM, "device allocation of %zu bytes (%s) failed", want,
                         name.c_str());
            }
            b.cap = want;
        }
        if (caller_capture) b.bound = true;
        return b.p;
    }
    template <class T>
    T* buf(const std::string& name, size_t count) {
        return static_cast<T*>(raw(name, count * sizeof(T)));
    }

    // Device copy of a host argument table.  The copy is skipped when the
    // device buffer already holds exactly these bytes (so a captured
    // sequence reuses the tables of the eager run that preceded it).
    // While capturing, a table that differs is written at once through a
    // private stream (not part of the graph): the graph's kernels read it
    // when they run.
    void* upload(const std::string& name0, const void* data, size_t bytes, hipStream_t st) {
        const std::string name = name0 + tag;
        void* d = raw(name, bytes);
        std::vector<char>& sh = shadows[name];
        const bool same = sh.size() == bytes && bytes && std::memcmp(sh.data(), data, bytes) == 0 &&
                          shadow_ptr[name] == d;
        if (!same) {
            if (bytes) {
                if (capturing) {
                    if (!side) DSC_HIP(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
                    DSC_HIP(hipMemcpyAsync(d, data, bytes, hipMemcpyHostToDevice, side));
                    DSC_HIP(hipStreamSynchronize(side));
                } else {
                    DSC_HIP(hipMemcpyAsync(d, data, bytes, hipMemcpyHostToDevice, st));
                }
            }
            sh.assign((const char*)data, (const char*)data + bytes);
            shadow_ptr[name] = d;
        }
        return d;
    }
    template <class T>
    T* upload(const std::string& name, const std::vector<T>& v, hipStream_t st) {
        return static_cast<T*>(upload(name, v.data(), v.size() * sizeof(T), st));
    }
    std::map<std::string, void*> shadow_ptr;

    // Drops the cached search-space plans when there are too many, unless a
    // captured graph may reference their tables.
    void evict_plans(size_t limit) {
        if (frozen || plans.size() < limit) return;
        plans.clear();
        generation++;
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
    // Accumulate the pending kernel times (waits for the kernels still running).
    void resolve_timing() {
        for (auto& p : pending) {
            float ms = 0.f;
            if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
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

// Records ev as a node of the graph being captured on s (a plain
// hipEventRecord during a capture does not become a graph node).
inline hipError_t capture_event_record(hipStream_t s, hipEvent_t ev) {
    hipStreamCaptureStatus cs;
    unsigned long long id = 0;
    hipGraph_t g = nullptr;
    const hipGraphNode_t* deps = nullptr;
    size_t nd = 0;
    hipError_t e = hipStreamGetCaptureInfo_v2(s, &cs, &id, &g, &deps, &nd);
    if (e != hipSuccess) return e;
    if (cs != hipStreamCaptureStatusActive || !g) return hipErrorStreamCaptureInvalidated;
    hipGraphNode_t node;
    e = hipGraphAddEventRecordNode(&node, g, deps, nd, ev);
    if (e != hipSuccess) return e;
    return hipStreamUpdateCaptureDependencies(s, &node, 1, hipStreamSetCaptureDependencies);
}

// Brackets one kernel launch with HIP events on its stream when timing is on.
struct KTimer {
    discover_ctx* c;
    hipStream_t s;
    const char* name;
    hipEvent_t a = nullptr, b = nullptr;
    bool graph = false;
    KTimer(discover_ctx* c_, hipStream_t s_, const char* n) : c(c_), s(s_), name(n) {
        if (c->timing && !c->capturing) {
            a = c->event();
            b = c->event();
            DSC_HIP(hipEventRecord(a, s));
        } else if (c->capturing && !c->caller_capture && c->graph_timed.count(name)) {
            // event-record nodes of the graph: the pair belongs to the graph
            graph = true;
            DSC_HIP(hipEventCreate(&a));
            if (hipEventCreate(&b) != hipSuccess) {
                if (hipEventDestroy(a) != hipSuccess) { /* ignore */ }
                a = nullptr;
                DSC_FAIL(DISCOVER_E_HIP, "event creation failed");
            }
            c->graph_pending.push_back({name, a, b});
            DSC_HIP(capture_event_record(s, a));
        }
    }
    ~KTimer() {
        if (!a) return;
        if (graph) {
            if (capture_event_record(s, b) != hipSuccess) { /* the capture reports it */ }
        } else if (hipEventRecord(b, s) == hipSuccess) {
            c->pending.push_back({name, a, b});
        }
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
// Wave reductions (every lane active; every lane gets the result, combined
// in a fixed order).  Within each row of 16 lanes, DPP lane permutations
// (quad_perm [1,0,3,2] and [2,3,0,1], row_half_mirror, row_mirror) combine
// lanes i and i^1, i^2, then the mirrored half and mirrored row, leaving the
// row's result in all 16 lanes; the four row results are then read from
// lanes 0, 16, 32 and 48.  This avoids a chain of LDS permutes.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo));
}

__device__ __forceinline__ double lane_f64(double v, int l) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const int hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo));
}

__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_f64<0xB1>(v);       // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);       // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);      // row_half_mirror
    v += dpp_f64<0x140>(v);      // row_mirror
    return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}

__device__ __forceinline__ double wave_min(double v) {
    v = fmin(v, dpp_f64<0xB1>(v));
    v = fmin(v, dpp_f64<0x4E>(v));
    v = fmin(v, dpp_f64<0x141>(v));
    v = fmin(v, dpp_f64<0x140>(v));
    return fmin(fmin(lane_f64(v, 0), lane_f64(v, 16)), fmin(lane_f64(v, 32), lane_f64(v, 48)));
}

__device__ __forceinline__ double wave_max(double v) {
    v = fmax(v, dpp_f64<0xB1>(v));
    v = fmax(v, dpp_f64<0x4E>(v));
    v = fmax(v, dpp_f64<0x141>(v));
    v = fmax(v, dpp_f64<0x140>(v));
    return fmax(fmax(lane_f64(v, 0), lane_f64(v, 16)), fmax(lane_f64(v, 32), lane_f64(v, 48)));
}

__host__ __device__ __forceinline__ int64_t choose2(int64_t m) { return m * (m - 1) / 2; }

// Index of the calling wave in its 256-thread block, as a wave-uniform
// value (the compiler then keeps per-wave work indices, their loads and
// their branches on the scalar unit).
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// ------------------------------------------------------ argument tables
// Per-problem argument tables live in device memory and are read through
// the constant address space, as kernel arguments are: uniform fields become
// scalar loads, and structures indexed with run-time subscripts (the search
// space description) are read in place rather than copied to scratch.
template <class T>
using ctab = const __attribute__((address_space(4))) T*;

template <class T>
inline ctab<T> ct(const T* p) { return (ctab<T>)p; }

template <class T>
__device__ __forceinline__ const T& tab(ctab<T> A, int64_t i) { return *(const T*)(A + i); }

// Pointers read from a table are generic; this tells the compiler that one
// addresses global memory (not LDS or scratch), so that it emits global
// rather than flat memory instructions.
#if defined(__HIP_DEVICE_COMPILE__)
#define DSC_GLOBAL(p)                                                                         \
    __builtin_assume(!__builtin_amdgcn_is_shared((const void*)(p)) &&                          \
                     !__builtin_amdgcn_is_private((const void*)(p)))
#else
#define DSC_GLOBAL(p) ((void)0)   // the host pass does not generate device code
#endif

// ------------------------------------------------------------ fills
// Device-side fills of many buffers in one launch (used instead of
// hipMemsetAsync so that the sequence can be captured into a graph).
struct FillSeg {
    void* p;
    int64_t n32;      // 32-bit words
    uint32_t v;
    uint32_t pad;
};

static __global__ __launch_bounds__(256) void k_fill(ctab<FillSeg> segs) {
    const FillSeg& f = tab(segs, blockIdx.y);
    uint32_t* p = (uint32_t*)f.p;
    DSC_GLOBAL(p);
    const int64_t t0 = (int64_t)blockIdx.x * 256 + threadIdx.x, stride = (int64_t)gridDim.x * 256;
    if (((uintptr_t)p & 15) == 0) {                       // 16-byte stores, then the tail
        const int64_t n4 = f.n32 >> 2;
        uint4* q = (uint4*)p;
        const uint4 v = make_uint4(f.v, f.v, f.v, f.v);
        for (int64_t i = t0; i < n4; i += stride) q[i] = v;
        for (int64_t i = 4 * n4 + t0; i < f.n32; i += stride) p[i] = f.v;
    } else {
        for (int64_t i = t0; i < f.n32; i += stride) p[i] = f.v;
    }
}

// Launch the fills of `segs` (each size a multiple of 4 bytes).
inline void fill_all(discover_ctx* ctx, const std::string& name, const std::vector<FillSeg>& segs,
                     hipStream_t st) {
    if (segs.empty()) return;
    int64_t mx = 1;
    for (const FillSeg& f : segs) mx = std::max<int64_t>(mx, f.n32);
    const FillSeg* d = ctx->upload(name, segs, st);
    dim3 g((unsigned)std::min<int64_t>(2048, cdiv(mx, 1024)), (unsigned)segs.size());
    k_fill<<<g, 256, 0, st>>>(ct(d));
    check_launch("k_fill");
}

inline FillSeg fill_seg(void* p, size_t bytes, uint32_t v) {
    return FillSeg{p, (int64_t)(bytes / 4), v, 0};
}

// Slices of one named device buffer, one per problem or list (256-byte
// aligned), so that every problem of a call keeps its own data.
struct Arena {
    std::vector<size_t> off;
    size_t total = 0;
    size_t add(size_t bytes) {
        const size_t o = total;
        total += (std::max<size_t>(bytes, 1) + 255) & ~size_t(255);
        off.push_back(o);
        return o;
    }
};

}  // namespace dsc
