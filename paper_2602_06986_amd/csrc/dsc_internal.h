// Internal interfaces shared by the library's sources: the batched
// screening and L0 passes that the public calls and the captured SISSO loop
// are built from.
#pragma once

#include "dsc_common.h"

namespace dsc {

// Where the results of one screened problem go: list t of the problem
// writes its k IDs and scores at ids + t * k and sc + t * k, and (if vals)
// the values of the selected features at vals + (t * k + j) * ldv.
struct ScreenOut {
    int64_t* ids;
    double* sc;
    double* vals;
    int64_t ldv;
};

// What a captured replay checks afterwards for one selection list: the
// pool and duplicate-pair capacities held, the selection was complete and
// the targets were usable.
struct ListCheck {
    const int64_t* res;
    int64_t cap, fcap, K, N;
    const unsigned long long* ctr;
    int dedup;
    int64_t fix_cap;          // entries of the problem's two fix-up lists (ctr[1], ctr[3])
    const unsigned long long* maxerr;   // precision forms: max |s_lowprec - s_fp64| (bits)
    int b;                    // problem of the list
};

// Outcome of one list, as a discover_status: the capacities held, the
// selection is complete and the targets were usable.
__host__ __device__ inline int list_status(const ListCheck& c, const int64_t* r,
                                           const unsigned long long* ctr) {
    if ((ctr[0] & 0xFFFFFFFFull) != 0) return DISCOVER_E_NUMERIC;
    if (r[4] > c.cap || (c.dedup && r[3] > c.fcap) || !(r[1] || c.K >= c.N) ||
        (int64_t)ctr[1] > c.fix_cap || (int64_t)ctr[3] > c.fix_cap)
        return DISCOVER_E_CAPACITY;
    return DISCOVER_OK;
}

// Where the models of one L0 problem go: model q at sub + q * sub_ld (D row
// indices), rmse[q], coef + q * coef_ld (D + 1 values), resid + q * ldr.
struct L0Out {
    int32_t* sub;
    int sub_ld;
    double* rmse;
    double* coef;
    int coef_ld;
    double* resid;
    int64_t ldr;
};

// What a captured replay checks afterwards for one L0 problem.
struct BandCheck {
    const unsigned long long* cnt;   // band and pair counts
    int64_t cap;
};

__host__ __device__ inline int band_status(const BandCheck& c, const unsigned long long* cnt) {
    if ((int64_t)cnt[0] > c.cap || (int64_t)cnt[1] > c.cap) return DISCOVER_E_CAPACITY;
    if (cnt[0] == 0) return DISCOVER_E_NUMERIC;
    return DISCOVER_OK;
}

// How a public call runs.  On a stream that the caller is capturing, the
// call is recorded with argument tables of its own (a fresh tag), nothing
// it references can later be freed, and its outcome goes to device memory;
// with device stats (nosync) it runs without waiting for the stream.  The
// previous state is restored when the call ends.
struct CallMode {
    discover_ctx* c;
    bool cap, nosync;
    std::string prev_tag;
    CallMode(discover_ctx* ctx, bool capture, bool device_stats)
        : c(ctx), cap(capture), nosync(device_stats), prev_tag(ctx->tag) {
        if (cap) {
            c->capturing = true;
            c->caller_capture = true;
            c->frozen = true;
            c->tag = "#c" + std::to_string(++c->capture_seq);
        }
        c->nosync = nosync;
    }
    ~CallMode() {
        if (cap) {
            c->capturing = false;
            c->caller_capture = false;
        }
        c->nosync = false;
        c->tag = prev_tag;
    }
};

// Whether work enqueued on st is being captured into a graph.
inline bool stream_capturing(hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    DSC_HIP(hipStreamIsCapturing(st, &cs));
    if (cs == hipStreamCaptureStatusInvalidated)
        DSC_FAIL(DISCOVER_E_HIP, "the capture on this stream has been invalidated");
    return cs == hipStreamCaptureStatusActive;
}

// Whether p is device memory (hipMalloc); host memory, pinned or not, is not.
inline bool device_memory(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();          // plain host memory: not an error of the call
        return false;
    }
    return a.type == hipMemoryTypeDevice;
}

// Screening of every problem of a call (validated arguments).  Outside
// capture the call synchronises and fills out_stats; while capturing it
// records the checks instead.
// extra_fills: more buffers to clear with the screen's own fill launch.
// dev_stats: device memory for the stats of a call that does not wait for
// the stream (ctx->nosync or a capture); each problem's status field then
// reports its outcome.
void generate_screen(discover_ctx* ctx, const discover_problem* probs, int nb,
                     const discover_screen_params& prm, const std::vector<ScreenOut>& outs,
                     discover_screen_stats* out_stats, hipStream_t st,
                     std::vector<ListCheck>* checks = nullptr,
                     const std::vector<FillSeg>* extra_fills = nullptr,
                     discover_screen_stats* dev_stats = nullptr);

// Whether an earlier call of this shape settled the selection sizes that a
// call without host synchronisation starts from.
bool screen_sizes_known(discover_ctx* ctx, const discover_problem* probs, int nb,
                        const discover_screen_params& prm);

// Exhaustive L0 of every problem of a call (validated arguments).
// dev_stats as for generate_screen.
void l0_batch(discover_ctx* ctx, const discover_l0_problem* probs, int nb, int D, int m,
              const std::vector<L0Out>& outs, std::vector<discover_l0_stats>& stats,
              hipStream_t st, std::vector<BandCheck>* checks = nullptr,
              discover_l0_stats* dev_stats = nullptr);

// Orthogonal matching pursuit of every problem of a call (validated
// arguments); problem b starts from the n_init rows init_active + b *
// init_ld.  The call does not wait for the stream.
// With scratch (omp_scratch_bytes bytes of device memory) the call takes
// its work buffers from there and allocates and creates nothing.
void omp_batch(discover_ctx* ctx, const discover_l0_problem* probs, int nb, int D_max,
               const int32_t* init_active, int n_init, int64_t init_ld, int32_t* out_active,
               double* out_coef, double* out_rmse, double* out_resid, int64_t ldr, hipStream_t st,
               char* scratch = nullptr);
// Looks up this device's address of the allocation-free OMP's scratch
// (the device must be current).
void noalloc_init(int device);
size_t omp_scratch_bytes(const discover_l0_problem* probs, int nb, int D_max, bool resid);
void fit_rows(discover_ctx* ctx, const discover_l0_problem* probs, int nb, int D, const int32_t* rows,
              int64_t rows_ld, double* coef, int64_t coef_ld, double* rmse, double* resid, int64_t ldr,
              hipStream_t st);
// Explained fractions (Eq. (1) through the normal equations) share these
// with every L0 search: the singular-pivot rule, the band of the QR refit
// and the RSS tie tolerance.
constexpr double PIV_TOL = 1e-10;     // normalized Cholesky pivot at/below which a subset is singular
constexpr double GRAM_DELTA = 1e-7;   // band width in explained fraction
constexpr double TAU_TIE = 1e-11;     // RSS tie tolerance relative to ||y - mean||^2

// Standardised rows and the (S + 1) x (S + 1) correlation matrix of one L0
// problem (row S: y), G[a * ldg + b]; yy = ||y - mean||^2.  Buffers are
// named from `name`.
struct GramOut {
    double* G;
    int ldg;
    double* yy;
    double* dg;               // G's diagonal, contiguous
};
GramOut l0_gram_one(discover_ctx* ctx, const discover_l0_problem& pb, const std::string& name,
                    hipStream_t st);
// QR residual sum of squares of `count` D-subsets subs[count][D] (device).
void refit_list(discover_ctx* ctx, const discover_l0_problem& pb, int D, const int32_t* subs, int64_t count,
                double* rss, hipStream_t st);
void validate_omp(const discover_l0_problem* probs, int32_t n_problems, int32_t D_max,
                  const int32_t* init_active, int32_t n_init, const int32_t* out_active,
                  const double* out_coef, const double* out_rmse, const double* out_resid, int64_t ldr);

}  // namespace dsc
