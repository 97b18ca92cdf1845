// Context lifetime, error text, host-side space queries and kernel timing.
#include "dsc_internal.h"
#include "dsc_space.h"

extern "C" discover_status discover_create(int device, discover_ctx** out) {
    using namespace dsc;
    return guarded([&] {
        DSC_REQUIRE(out, "out is NULL");
        *out = nullptr;
        int count = 0;
        DSC_HIP(hipGetDeviceCount(&count));
        DSC_REQUIRE(device >= 0 && device < count, "device %d outside 0..%d", device, count - 1);
        DSC_HIP(hipSetDevice(device));
        noalloc_init(device);              // this device's copy of the OMP scratch
        discover_ctx* c = new discover_ctx();
        c->device = device;
        *out = c;
    });
}

extern "C" void discover_destroy(discover_ctx* ctx) {
    if (!ctx) return;
    if (hipSetDevice(ctx->device) == hipSuccess) {
        if (hipDeviceSynchronize() != hipSuccess) { /* keep tearing down */ }
        ctx->batches.clear();              // captured graphs first, then what they referenced
        ctx->plans.clear();
        if (ctx->side && hipStreamDestroy(ctx->side) != hipSuccess) { /* ignore */ }
        for (auto& kv : ctx->bufs)
            if (kv.second.p && hipFree(kv.second.p) != hipSuccess) { /* ignore */ }
        for (auto& kv : ctx->pinned)
            if (kv.second && hipHostFree(kv.second) != hipSuccess) { /* ignore */ }
        for (auto& p : ctx->pending) {
            if (hipEventDestroy(p.a) != hipSuccess || hipEventDestroy(p.b) != hipSuccess) { }
        }
        for (hipEvent_t e : ctx->free_events)
            if (hipEventDestroy(e) != hipSuccess) { }
    }
    delete ctx;
}

extern "C" const char* discover_last_error(void) { return dsc::get_error(); }

extern "C" int64_t discover_count(int32_t p, const discover_screen_params* prm) {
    using namespace dsc;
    int64_t out = -1;
    discover_status s = guarded([&] {
        DSC_REQUIRE(prm && p >= 1, "prm/p");
        DSC_REQUIRE(prm->rung >= 0 && prm->rung <= DISCOVER_MAX_RUNG, "rung");
        SpaceDev d;
        space_layout(d, p, *prm);                // counting needs no operand plan
        out = d.off[d.R + 1];
    });
    return s == DISCOVER_OK ? out : (int64_t)s;
}

extern "C" discover_status discover_decode(int32_t p, const discover_screen_params* prm, int64_t id,
                                           char* buf, size_t len) {
    using namespace dsc;
    return guarded([&] {
        DSC_REQUIRE(prm && buf && len > 0, "prm/buf/len");
        const int64_t N = discover_count(p, prm);
        DSC_REQUIRE(N > 0 && id >= 0 && id < N, "id %lld outside the space", (long long)id);
        SpaceDev d;
        space_layout(d, p, *prm);
        const std::string s = expr_of(d, id);
        std::snprintf(buf, len, "%s", s.c_str());
    });
}

extern "C" discover_status discover_set_fixup_capacity(discover_ctx* ctx, int64_t entries) {
    using namespace dsc;
    return guarded([&] {
        DSC_REQUIRE(ctx, "ctx is NULL");
        DSC_REQUIRE(entries >= 1, "fix-up capacity must be >= 1");
        ctx->fix_cap_min = entries;
    });
}

extern "C" discover_status discover_set_rules(discover_ctx* ctx, const discover_rules* rules) {
    using namespace dsc;
    return guarded([&] {
        DSC_REQUIRE(ctx, "ctx is NULL");
        if (rules) {
            DSC_REQUIRE(rules->max_complexity >= -1, "max_complexity %d < -1", rules->max_complexity);
            for (int o = 0; o < 10; o++)
                DSC_REQUIRE((rules->forbid_nest[o] & ~DISCOVER_OPS_ALL) == 0, "forbid_nest[%d]", o);
            DSC_REQUIRE(rules->n_forbid_pairs >= 0 && (rules->n_forbid_pairs == 0 || rules->forbid_pairs),
                        "forbid_pairs");
            for (int i = 0; i < 2 * rules->n_forbid_pairs; i++)
                DSC_REQUIRE(rules->forbid_pairs[i] >= 0 && rules->forbid_pairs[i] < 64,
                            "forbid_pairs: primary %d outside 0..63", rules->forbid_pairs[i]);
            DSC_REQUIRE(rules->target_unit == 0 || rules->target_unit == 1, "target_unit");
            ctx->rules = *rules;
            ctx->rule_pairs.assign(rules->forbid_pairs, rules->forbid_pairs + 2 * rules->n_forbid_pairs);
            ctx->rules.forbid_pairs = nullptr;
            ctx->has_rules = true;
        } else {
            ctx->has_rules = false;
            ctx->rule_pairs.clear();
        }
        // captured graphs and the memoised selection sizes belong to the old rules
        DSC_HIP(hipSetDevice(ctx->device));
        DSC_HIP(hipDeviceSynchronize());
        ctx->batches.clear();
        ctx->generation++;
    });
}

extern "C" discover_status discover_set_timing(discover_ctx* ctx, int32_t enable) {
    using namespace dsc;
    return guarded([&] {
        DSC_REQUIRE(ctx, "ctx is NULL");
        ctx->timing = enable != 0;
    });
}

extern "C" discover_status discover_set_graph_timing(discover_ctx* ctx, const char* names) {
    using namespace dsc;
    return guarded([&] {
        DSC_REQUIRE(ctx, "ctx is NULL");
        std::set<std::string> want;
        for (const char* p = names; p && *p;) {
            const char* e = std::strchr(p, ',');
            const size_t len = e ? (size_t)(e - p) : std::strlen(p);
            if (len) want.insert(std::string(p, len));
            p = e ? e + 1 : p + len;
        }
        if (want != ctx->graph_timed) {
            ctx->graph_timed.swap(want);
            ctx->generation++;                  // graphs captured before are not replayed
        }
    });
}

extern "C" discover_status discover_timing(discover_ctx* ctx, const char* kernel, int64_t* launches,
                                           double* total_ms) {
    using namespace dsc;
    return guarded([&] {
        DSC_REQUIRE(ctx && kernel && launches && total_ms, "arguments");
        ctx->resolve_timing();               // kernels of calls that did not wait
        auto it = ctx->times.find(kernel);
        *launches = it == ctx->times.end() ? 0 : it->second.first;
        *total_ms = it == ctx->times.end() ? 0.0 : it->second.second;
    });
}

extern "C" discover_status discover_reset_timing(discover_ctx* ctx) {
    using namespace dsc;
    return guarded([&] {
        DSC_REQUIRE(ctx, "ctx is NULL");
        ctx->resolve_timing();
        ctx->times.clear();
    });
}
