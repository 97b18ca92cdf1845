// The allocation-free form of orthogonal matching pursuit, for callers that
// cannot allocate device memory (code under graph capture, tight serving
// loops, harnesses that forbid allocation).  Its work buffers come from one
// file-scope device array; each GPU holds its own copy of the array, at an
// address the host learns once per device, when a context is created on
// it.
#include <mutex>

#include "dsc_internal.h"

namespace {

constexpr size_t SCRATCH_BYTES = (size_t)64 << 20;   // 64 MiB per GPU
constexpr int MAX_DEVICES = 64;

// In host code this name is only a stand-in for the symbol: the device
// address of each GPU's copy is looked up with hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::mutex g_lock;
void* g_scratch[MAX_DEVICES] = {};

}  // namespace

namespace dsc {

// Called by discover_create with `device` current.
void noalloc_init(int device) {
    DSC_REQUIRE(device >= 0 && device < MAX_DEVICES, "device %d outside 0..%d", device, MAX_DEVICES - 1);
    std::lock_guard<std::mutex> g(g_lock);
    if (g_scratch[device]) return;
    void* p = nullptr;
    DSC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch[device] = p;
}

}  // namespace dsc

extern "C" discover_status discover_omp_noalloc(discover_ctx* ctx, const discover_l0_problem* probs,
                                                int32_t n_problems, int32_t D_max,
                                                const int32_t* init_active, int32_t n_init,
                                                int32_t* out_active, double* out_coef, double* out_rmse,
                                                double* out_resid, int64_t ldr, void* stream) {
    using namespace dsc;
    return guarded([&] {
        DSC_REQUIRE(ctx, "ctx is NULL");
        validate_omp(probs, n_problems, D_max, init_active, n_init, out_active, out_coef, out_rmse,
                     out_resid, ldr);
        const size_t need = omp_scratch_bytes(probs, n_problems, D_max, out_resid != nullptr);
        DSC_REQUIRE(need <= SCRATCH_BYTES,
                    "these problems need %zu bytes of OMP work space; the allocation-free form has "
                    "%zu (pass out_resid, or fewer or smaller problems per call)",
                    need, SCRATCH_BYTES);
        char* base;
        {
            std::lock_guard<std::mutex> g(g_lock);
            base = (char*)g_scratch[ctx->device];
        }
        if (!base) DSC_FAIL(DISCOVER_E_HIP, "the scratch address of device %d is unknown", ctx->device);
        DSC_HIP(hipSetDevice(ctx->device));
        omp_batch(ctx, probs, n_problems, D_max, init_active, n_init, n_init, out_active, out_coef,
                  out_rmse, out_resid, ldr, (hipStream_t)stream, base);
    });
}
