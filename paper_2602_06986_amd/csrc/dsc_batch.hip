// The SISSO dimension loop over a batch of datasets as one launch sequence
// (the batched form of the screening + sparsifying steps of the cited SISSO
// method, Summary and Software Description): for d = 1..D every dataset is
// screened against its residuals, the selected features are appended to its
// subspace, and exhaustive L0 refits its target.  The first call with a
// given set of inputs runs eagerly (sizing every buffer and settling every
// capacity), then captures the same sequence into a hipGraph; later calls
// with the same inputs replay the graph and check, on the device, that
// every capacity held and every selection was complete (else they run
// eagerly again).
#include "dsc_internal.h"

#include <string>

namespace dsc {

// One thread per check; any failure sets *out (a plain store: out is in
// pinned host memory, read by the host after the replay).
__global__ __launch_bounds__(256) void k_verdict(ctab<ListCheck> L, int nl, ctab<BandCheck> B, int nbc,
                                                 int* __restrict__ out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    bool bad = false;
    if (i < nl) {
        const ListCheck& c = tab(L, i);
        DSC_GLOBAL(c.res); DSC_GLOBAL(c.ctr);
        bad = list_status(c, c.res, c.ctr) != DISCOVER_OK;
    } else if (i < nl + nbc) {
        const BandCheck& c = tab(B, i - nl);
        DSC_GLOBAL(c.cnt);
        bad = band_status(c, c.cnt) != DISCOVER_OK;
    }
    if (bad) *(volatile int*)out = 1;
}

struct SissoGraph {
    int id = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t generation = 0;
    std::vector<discover_ctx::Pending> timers;   // event pairs recorded inside the graph
    void drop_timers() {
        for (auto& t : timers) {
            if (hipEventDestroy(t.a) != hipSuccess) { /* ignore */ }
            if (hipEventDestroy(t.b) != hipSuccess) { /* ignore */ }
        }
        timers.clear();
    }
    ~SissoGraph() {
        if (exec && hipGraphExecDestroy(exec) != hipSuccess) { /* ignore */ }
        if (graph && hipGraphDestroy(graph) != hipSuccess) { /* ignore */ }
        drop_timers();
    }
};

struct SissoCall {
    const discover_problem* probs;
    int nb;
    discover_screen_params prm;
    int D, m, k, ldf;
    int64_t* ids;
    double* sc;
    int32_t* sub;
    double* rmse;
    double* coef;
    int omp_D;
    int32_t* omp_active;
    double* omp_coef;
    double* omp_rmse;
};

// The whole loop on stream st; while capturing, the checks of every
// selection list and band are collected and judged by k_verdict.
static void sisso_sequence(discover_ctx* ctx, const SissoCall& c, const std::string& gtag,
                           hipStream_t st) {
    const int nb = c.nb, D = c.D, m = c.m, k = c.k;
    const size_t ldf = (size_t)c.ldf;
    ctx->tag = gtag;
    double* F = ctx->buf<double>("sisF" + gtag, (size_t)nb * D * k * ldf);
    double* R = ctx->buf<double>("sisR" + gtag, (size_t)nb * m * ldf);
    int* verdict = (int*)ctx->pinned_buf("sisV" + gtag, 64);
    std::vector<FillSeg> fills;
    fills.push_back(fill_seg(verdict, 4, 0u));
    fills.push_back(fill_seg(c.sub, (size_t)nb * D * m * 3 * 4, 0xFFFFFFFFu));
    fills.push_back(fill_seg(c.coef, (size_t)nb * D * m * 4 * 8, 0xFFFFFFFFu));   // NaN
    // (cleared by dimension 1's screen fill launch, which precedes every use)
    std::vector<ListCheck> lc;
    std::vector<BandCheck> bc;
    std::vector<discover_l0_stats> l0st(nb);
    ctx->ops_tag = gtag;                  // the operand features are made once, by d = 1
    struct OpsScope {                     // no reuse outside this sequence, also on an error
        discover_ctx* c;
        ~OpsScope() { c->ops_reuse = false; c->ops_tag.clear(); }
    } ops_scope{ctx};
    for (int d = 1; d <= D; d++) {
        ctx->tag = gtag + "d" + std::to_string(d);
        ctx->ops_reuse = d > 1;
        std::vector<discover_problem> sp(c.probs, c.probs + nb);
        std::vector<ScreenOut> so(nb);
        for (int b = 0; b < nb; b++) {
            if (d > 1) {
                sp[b].Y = R + (size_t)b * m * ldf;
                sp[b].ldy = (int64_t)ldf;
                sp[b].T = m;
            }
            sp[b].exclude = d > 1 ? c.ids + (int64_t)b * D * k : nullptr;
            sp[b].n_exclude = (d - 1) * k;
            const int64_t row = (int64_t)b * D + (d - 1);
            so[b] = ScreenOut{c.ids + row * k, c.sc + row * k, F + ((size_t)b * D * k + (size_t)(d - 1) * k) * ldf,
                              (int64_t)ldf};
        }
        discover_screen_params q = c.prm;
        if (d > 1 && m > 1) q.score_mode = DISCOVER_SCORE_MAX;
        generate_screen(ctx, sp.data(), nb, q, so, nullptr, st, ctx->capturing ? &lc : nullptr,
                        d == 1 ? &fills : nullptr);
        std::vector<discover_l0_problem> lp(nb);
        std::vector<L0Out> lo(nb);
        for (int b = 0; b < nb; b++) {
            lp[b].n = c.probs[b].n;
            lp[b].S = d * k;
            lp[b].F = F + (size_t)b * D * k * ldf;
            lp[b].ldf = (int64_t)ldf;
            lp[b].ids = c.ids + (int64_t)b * D * k;
            lp[b].y = c.probs[b].Y;
            const int64_t row = (int64_t)b * D + (d - 1);
            lo[b] = L0Out{c.sub + row * m * 3, 3, c.rmse + row * m, c.coef + row * m * 4, 4,
                          R + (size_t)b * m * ldf, (int64_t)ldf};
        }
        l0_batch(ctx, lp.data(), nb, d, m, lo, l0st, st, ctx->capturing ? &bc : nullptr);
    }
    ctx->ops_reuse = false;
    if (c.omp_D > D) {
        // the best D-model of each dataset, extended by OMP over its subspace
        ctx->tag = gtag + "omp";
        std::vector<discover_l0_problem> op(nb);
        for (int b = 0; b < nb; b++) {
            op[b].n = c.probs[b].n;
            op[b].S = D * k;
            op[b].F = F + (size_t)b * D * k * ldf;
            op[b].ldf = (int64_t)ldf;
            op[b].ids = c.ids + (int64_t)b * D * k;
            op[b].y = c.probs[b].Y;
        }
        omp_batch(ctx, op.data(), nb, c.omp_D, c.sub + (int64_t)(D - 1) * m * 3, D, (int64_t)D * m * 3,
                  c.omp_active, c.omp_coef, c.omp_rmse, nullptr, 0, st);
    }
    ctx->tag = gtag;
    if (!ctx->capturing) {
        // one selection list and one band per dataset and dimension: size the
        // check tables now, a capture may not allocate
        ctx->raw("sis_lchecks" + gtag, (size_t)D * nb * sizeof(ListCheck));
        ctx->raw("sis_bchecks" + gtag, (size_t)D * nb * sizeof(BandCheck));
    } else {
        const ListCheck* dl = ctx->upload("sis_lchecks", lc, st);
        const BandCheck* db = ctx->upload("sis_bchecks", bc, st);
        const int n = (int)(lc.size() + bc.size());
        k_verdict<<<(unsigned)cdiv(std::max(n, 1), 256), 256, 0, st>>>(ct(dl), (int)lc.size(), ct(db),
                                                                       (int)bc.size(), verdict);
        check_launch("k_verdict");
    }
    ctx->tag.clear();
}

static std::string sisso_key(const SissoCall& c) {
    std::string key((const char*)&c.prm, sizeof c.prm);
    const int64_t f[13] = {c.nb, c.D, c.m, c.k, (int64_t)(intptr_t)c.ids, (int64_t)(intptr_t)c.sc,
                           (int64_t)(intptr_t)c.sub, (int64_t)(intptr_t)c.rmse, (int64_t)(intptr_t)c.coef,
                           c.omp_D, (int64_t)(intptr_t)c.omp_active, (int64_t)(intptr_t)c.omp_coef,
                           (int64_t)(intptr_t)c.omp_rmse};
    key.append((const char*)f, sizeof f);
    for (int b = 0; b < c.nb; b++) {
        const discover_problem& p = c.probs[b];
        const int64_t g[7] = {p.n, p.p, p.B, (int64_t)(intptr_t)p.X, p.ldx, (int64_t)(intptr_t)p.Y, p.ldy};
        key.append((const char*)g, sizeof g);
        if (p.B && p.units) key.append((const char*)p.units, sizeof(int32_t) * p.p * p.B);
    }
    return key;
}

}  // namespace dsc

extern "C" discover_status discover_sisso_batch(discover_ctx* ctx, const discover_problem* probs,
                                                int32_t n_problems, const discover_screen_params* prm,
                                                int32_t D, int32_t m, int32_t use_graph,
                                                int64_t* out_ids, double* out_scores,
                                                int32_t* out_subsets, double* out_rmse, double* out_coef,
                                                int32_t omp_D, int32_t* out_omp_active,
                                                double* out_omp_coef, double* out_omp_rmse,
                                                int32_t* out_replayed, void* stream) {
    using namespace dsc;
    return guarded([&] {
        DSC_REQUIRE(ctx && probs && prm && n_problems >= 1 && n_problems <= 65535, "ctx/probs/prm");
        DSC_REQUIRE(D >= 1 && D <= 3, "D = %d outside 1..3", D);
        DSC_REQUIRE(m >= 1 && m <= DISCOVER_MAX_TARGETS, "m = %d outside 1..%d", m, DISCOVER_MAX_TARGETS);
        DSC_REQUIRE(out_ids && out_scores && out_subsets && out_rmse && out_coef, "outputs required");
        DSC_REQUIRE(omp_D == 0 || (omp_D > D && omp_D <= DISCOVER_MAX_D), "omp_D = %d: 0 or %d..%d",
                    omp_D, D + 1, DISCOVER_MAX_D);
        DSC_REQUIRE(omp_D == 0 || (out_omp_active && out_omp_coef && out_omp_rmse),
                    "OMP outputs required");
        DSC_REQUIRE(omp_D == 0 || (int64_t)D * prm->k >= omp_D, "omp_D exceeds the subspace");
        DSC_REQUIRE(prm->rung >= 0 && prm->rung <= DISCOVER_MAX_RUNG && prm->k >= 1, "rung/k");
        DSC_REQUIRE(prm->tile_j >= 0 && prm->tile_j <= 4 && prm->lp_pairs >= -1 && prm->lp_pairs <= 1 &&
                    prm->sched >= -1 && prm->sched <= 1, "tile_j / lp_pairs / sched");
        DSC_REQUIRE(prm->score_mode == DISCOVER_SCORE_PER_TARGET, "the first dimension screens one target");
        int nmax = 0;
        for (int b = 0; b < n_problems; b++) {
            const discover_problem& p = probs[b];
            DSC_REQUIRE(p.T == 1, "problem %d: T must be 1 (the target)", b);
            DSC_REQUIRE(p.n_exclude == 0, "problem %d: exclude lists are built by the loop", b);
            DSC_REQUIRE(p.n >= D + 2 && p.n >= 3 && p.X && p.Y && p.ldx >= p.n && p.ldy >= p.n,
                        "problem %d: n/X/Y", b);
            DSC_REQUIRE(p.p >= 1 && p.p <= 4096 && p.B >= 0 && p.B <= DISCOVER_MAX_UNITS &&
                        (p.B == 0 || p.units), "problem %d: p/B/units", b);
            nmax = std::max(nmax, p.n);
        }
        DSC_HIP(hipSetDevice(ctx->device));
        hipStream_t caller = (hipStream_t)stream;
        DSC_REQUIRE(!stream_capturing(caller), "discover_sisso_batch captures and replays graphs of its "
                                               "own and cannot itself be captured");
        if (out_replayed) *out_replayed = 0;
        SissoCall c{probs, n_problems, *prm, D, m, prm->k, (int)cdiv(nmax, 64) * 64,
                    out_ids, out_scores, out_subsets, out_rmse, out_coef, omp_D, out_omp_active,
                    out_omp_coef, out_omp_rmse};
        // all work runs on the context's own stream (a capture needs a
        // non-default stream); the call returns with its results ready
        hipStream_t gs = nullptr;
        {
            auto it = ctx->batches.find("sisso_stream");
            if (it == ctx->batches.end()) {
                hipStream_t s2;
                DSC_HIP(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
                auto holder = std::shared_ptr<void>((void*)s2, [](void* p) {
                    if (hipStreamDestroy((hipStream_t)p) != hipSuccess) { /* ignore */ }
                });
                ctx->batches["sisso_stream"] = holder;
                gs = s2;
            } else {
                gs = (hipStream_t)it->second.get();
            }
        }
        DSC_HIP(hipStreamSynchronize(caller));
        const std::string key = "sisso" + sisso_key(c);
        auto git = ctx->batches.find(key);
        std::shared_ptr<SissoGraph> G;
        if (git != ctx->batches.end()) G = std::static_pointer_cast<SissoGraph>(git->second);
        if (use_graph && G && G->exec && G->generation == ctx->generation) {
            const std::string gtag = "#s" + std::to_string(G->id);
            const volatile int* verdict = (const volatile int*)ctx->pinned_buf("sisV" + gtag, 64);
            DSC_HIP(hipGraphLaunch(G->exec, gs));
            DSC_HIP(hipStreamSynchronize(gs));
            const int h = *verdict;                    // written by the replay's k_verdict
            if (ctx->timing)
                for (auto& t : G->timers) {
                    float ms = 0.f;
                    if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
                        auto& acc = ctx->times[t.name];
                        acc.first += 1;
                        acc.second += ms;
                    }
                }
            if (h == 0) {
                if (out_replayed) *out_replayed = 1;
                return;
            }
            G->exec = nullptr;                  // fall back to an eager run below
        }
        if (!G) {
            static int next_id = 0;
            G = std::make_shared<SissoGraph>();
            G->id = next_id++;
            if (ctx->batches.size() >= 256) {
                ctx->batches.clear();
                ctx->generation++;
            }
            ctx->batches[key] = G;
        }
        const std::string gtag = "#s" + std::to_string(G->id);
        sisso_sequence(ctx, c, gtag, gs);
        DSC_HIP(hipStreamSynchronize(gs));
        ctx->resolve_timing();
        if (!use_graph) return;
        // capture the same sequence for later calls
        if (G->exec) { if (hipGraphExecDestroy(G->exec) != hipSuccess) { } G->exec = nullptr; }
        if (G->graph) { if (hipGraphDestroy(G->graph) != hipSuccess) { } G->graph = nullptr; }
        G->drop_timers();
        const uint64_t gen0 = ctx->generation;
        ctx->capturing = true;
        ctx->graph_pending.clear();
        DSC_HIP(hipStreamBeginCapture(gs, hipStreamCaptureModeRelaxed));
        discover_status cap_status = guarded([&] { sisso_sequence(ctx, c, gtag, gs); });
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(gs, &graph);
        ctx->capturing = false;
        ctx->tag.clear();
        G->timers.swap(ctx->graph_pending);
        ctx->graph_pending.clear();
        if (cap_status != DISCOVER_OK || ec != hipSuccess || !graph || ctx->generation != gen0) {
            G->drop_timers();
            if (graph && hipGraphDestroy(graph) != hipSuccess) { }
            if (cap_status == DISCOVER_OK) {
                if (ec != hipSuccess) set_error("graph capture failed: %s", hipGetErrorString(ec));
                else set_error("device memory was reallocated during graph capture");
            }
            if (out_replayed) *out_replayed = -1;
            return;                             // results of the eager run stand; no graph
        }
        hipGraphExec_t exec = nullptr;
        DSC_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        G->graph = graph;
        G->exec = exec;
        G->generation = ctx->generation;
    });
}

namespace dsc {

// Values of the stand-in subspaces that size the L0 workspace: uniform on
// [0.5, 2) from a counter hash (splitmix64), so that every subset is
// non-singular and the band keeps its default size.
__global__ __launch_bounds__(256) void k_reserve_fill(double* __restrict__ v, int64_t count, uint64_t seed) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256) {
        uint64_t z = seed + (uint64_t)i * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        v[i] = 0.5 + 1.5 * (double)(z >> 11) * 0x1.0p-53;
    }
}

__global__ __launch_bounds__(256) void k_reserve_iota(int64_t* __restrict__ v, const int64_t* __restrict__ start,
                                                      const int32_t* __restrict__ len, int nb) {
    const int b = blockIdx.y;
    if (b >= nb) return;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < len[b]; i += (int64_t)gridDim.x * 256)
        v[start[b] + i] = i;
}

}  // namespace dsc

static void rethrow(discover_status s) {
    if (s != DISCOVER_OK) throw dsc::Error{s};
}

extern "C" discover_status discover_reserve(discover_ctx* ctx, const discover_problem* probs,
                                            int32_t n_problems, const discover_screen_params* prm,
                                            int32_t D_max, int32_t m, void* stream) {
    using namespace dsc;
    return guarded([&] {
        DSC_REQUIRE(ctx && probs && prm && n_problems >= 1, "ctx/probs/prm");
        DSC_REQUIRE(n_problems <= 65535, "n_problems = %d > 65535", n_problems);
        DSC_REQUIRE(D_max >= 0 && D_max <= 3, "D_max = %d outside 0..3", D_max);
        DSC_REQUIRE(D_max == 0 || (m >= 1 && m <= 64), "m = %d outside 1..64", m);
        DSC_REQUIRE(prm->k >= 1, "k must be >= 1");
        DSC_HIP(hipSetDevice(ctx->device));
        const hipStream_t st = (hipStream_t)stream;
        DSC_REQUIRE(!stream_capturing(st), "discover_reserve cannot run inside a graph capture");
        // 1. the screen itself, eagerly: plans, tile choices, selection sizes
        int64_t rows = 0;
        int nmax = 0;
        std::vector<int> tl(n_problems);
        for (int b = 0; b < n_problems; b++) {
            tl[b] = prm->score_mode == DISCOVER_SCORE_MAX ? 1 : probs[b].T;
            rows += tl[b];
            nmax = std::max(nmax, probs[b].n);
        }
        DSC_REQUIRE(nmax >= 1, "n");
        int64_t* ids = ctx->buf<int64_t>("rsv_ids", (size_t)rows * prm->k);
        double* sc = ctx->buf<double>("rsv_sc", (size_t)rows * prm->k);
        double* vals = ctx->buf<double>("rsv_vals", (size_t)rows * prm->k * nmax);
        std::vector<discover_screen_stats> ss(n_problems);
        rethrow(discover_generate_screen(ctx, probs, n_problems, prm, ids, sc, vals, nmax, ss.data(), stream));
        // 2. L0 of every dimension up to D_max over D * k * T' rows, then OMP,
        // on stand-in subspaces of the same sizes
        for (int D = 1; D <= D_max; D++) {
            std::vector<discover_l0_problem> lp;
            std::vector<int64_t> fo, io;
            int64_t ftot = 0, itot = 0, ytot = 0;
            std::vector<int64_t> yo;
            for (int b = 0; b < n_problems; b++) {
                const int64_t S = std::min<int64_t>(65535, (int64_t)D * prm->k * tl[b]);
                if (S < D || probs[b].n < D + 2) continue;
                discover_l0_problem q{};
                q.n = probs[b].n;
                q.S = (int32_t)S;
                q.ldf = q.n;
                lp.push_back(q);
                fo.push_back(ftot); io.push_back(itot); yo.push_back(ytot);
                ftot += S * q.n; itot += S; ytot += q.n;
            }
            if (lp.empty()) continue;
            const int nl = (int)lp.size();
            double* F = ctx->buf<double>("rsv_F", (size_t)ftot);
            double* y = ctx->buf<double>("rsv_y", (size_t)ytot);
            int64_t* rid = ctx->buf<int64_t>("rsv_rid", (size_t)itot);
            k_reserve_fill<<<(unsigned)std::min<int64_t>(4096, cdiv(ftot, 256)), 256, 0, st>>>(F, ftot, 0x5EEDull + D);
            k_reserve_fill<<<(unsigned)std::min<int64_t>(4096, cdiv(ytot, 256)), 256, 0, st>>>(y, ytot, 0xF00Dull + D);
            std::vector<int32_t> len(nl);
            int32_t lmax = 1;
            for (int q = 0; q < nl; q++) { len[q] = lp[q].S; lmax = std::max(lmax, len[q]); }
            const int64_t* dio = ctx->upload("rsv_io", io, st);
            const int32_t* dlen = ctx->upload("rsv_len", len, st);
            k_reserve_iota<<<dim3((unsigned)cdiv(lmax, 256), nl), 256, 0, st>>>(rid, dio, dlen, nl);
            check_launch("k_reserve");
            for (int q = 0; q < nl; q++) {
                lp[q].F = F + fo[q];
                lp[q].y = y + yo[q];
                lp[q].ids = rid + io[q];
            }
            int32_t* sub = ctx->buf<int32_t>("rsv_sub", (size_t)nl * m * D);
            double* rmse = ctx->buf<double>("rsv_rmse", (size_t)nl * m);
            double* coef = ctx->buf<double>("rsv_coef", (size_t)nl * m * (D + 1));
            double* res = ctx->buf<double>("rsv_res", (size_t)nl * m * nmax);
            std::vector<discover_l0_stats> ls(nl);
            rethrow(discover_l0_fit(ctx, lp.data(), nl, D, m, sub, rmse, coef, res, nmax, ls.data(), stream));
            if (D == D_max) {
                int Do = DISCOVER_MAX_D;
                for (const auto& q : lp) Do = std::min({Do, q.S, q.n - 2});
                if (Do >= 1) {
                    int32_t* act = ctx->buf<int32_t>("rsv_oact", (size_t)nl * Do);
                    double* oc = ctx->buf<double>("rsv_ocoef", (size_t)nl * (Do + 1));
                    double* orm = ctx->buf<double>("rsv_ormse", (size_t)nl);
                    double* ores = ctx->buf<double>("rsv_ores", (size_t)nl * nmax);
                    rethrow(discover_omp(ctx, lp.data(), nl, Do, nullptr, 0, act, oc, orm, ores, nmax, stream));
                }
            }
        }
        DSC_HIP(hipStreamSynchronize(st));
    });
}
