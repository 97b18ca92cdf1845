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
};

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

// Screening of every problem of a call (validated arguments).  Outside
// capture the call synchronises and fills out_stats; while capturing it
// records the checks instead.
// extra_fills: more buffers to clear with the screen's own fill launch.
void generate_screen(discover_ctx* ctx, const discover_problem* probs, int nb,
                     const discover_screen_params& prm, const std::vector<ScreenOut>& outs,
                     discover_screen_stats* out_stats, hipStream_t st,
                     std::vector<ListCheck>* checks = nullptr,
                     const std::vector<FillSeg>* extra_fills = nullptr);

// Exhaustive L0 of every problem of a call (validated arguments).
void l0_batch(discover_ctx* ctx, const discover_l0_problem* probs, int nb, int D, int m,
              const std::vector<L0Out>& outs, std::vector<discover_l0_stats>& stats,
              hipStream_t st, std::vector<BandCheck>* checks = nullptr);

// Orthogonal matching pursuit of every problem of a call (validated
// arguments); problem b starts from the n_init rows init_active + b *
// init_ld.  Outside capture the call synchronises.
void omp_batch(discover_ctx* ctx, const discover_l0_problem* probs, int nb, int D_max,
               const int32_t* init_active, int n_init, int64_t init_ld, int32_t* out_active,
               double* out_coef, double* out_rmse, double* out_resid, int64_t ldr, hipStream_t st);

}  // namespace dsc
