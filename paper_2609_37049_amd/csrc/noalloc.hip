// disco_dirac_apply_noalloc: disco_dirac_apply for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops).
//
// disco_dirac_apply converts the canonical fields to the native layout in two
// workspace blocks that grow with hipMalloc.  Here those two blocks live in
// one file-scope device array of fixed size, `scratch`, which every GPU the
// library runs on holds (its own copy, at its own address) until the process
// ends.  Its device address is resolved once per device when a context is
// created there; host code uses only that address, never the array's name.
// Nothing in it needs to start at zero: the layout conversion writes the
// whole input block and the stencil every site of the output block.
#include <algorithm>
#include <mutex>

#include "common.h"

namespace {

constexpr size_t kScratchBytes = 256ull << 20;   // 256 MiB per GPU
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex scratch_mu;
void* scratch_ptr[kMaxDevices] = {};

}  // namespace

namespace disco {

void scratch_bind(int device) {
    REQUIRE(device >= 0 && device < kMaxDevices, DISCO_EINVAL, "device %d: at most %d devices", device, kMaxDevices);
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (scratch_ptr[device]) return;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    REQUIRE(e == hipSuccess && p, DISCO_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", device,
            hipGetErrorString(e));
    scratch_ptr[device] = p;
}

}  // namespace disco

extern "C" int disco_dirac_apply_noalloc(disco_ctx* ctx, int prec, int dagger, int nrhs, const void* in, void* out) {
    if (!ctx) return DISCO_EINVAL;
    return guarded(ctx, [&] {
        REQUIRE(in && out, DISCO_EINVAL, "NULL spinor");
        REQUIRE(in != out, DISCO_EINVAL, "in and out must differ");
        REQUIRE(prec >= 0 && prec <= 2, DISCO_EINVAL, "bad precision %d", prec);
        REQUIRE(nrhs >= 0, DISCO_EINVAL, "nrhs < 0");
        // right-hand sides per launch: both native blocks (the second at a
        // 256-byte boundary) must fit in the scratch array
        const size_t per = disco::native_bytes(ctx, prec, 1);
        const long long fit = (long long)((kScratchBytes / 2 - 256) / per);
        REQUIRE(fit >= 1, DISCO_EINVAL,
                "one right-hand side of %ld sites needs 2 x %zu bytes of scratch in precision %d; the no-allocation "
                "entry point has %zu bytes",
                ctx->V, per, prec, kScratchBytes);
        REQUIRE(ctx->have_clover, DISCO_ESTATE, "operator applied before clover_setup");
        REQUIRE(ctx->device >= 0 && ctx->device < kMaxDevices && scratch_ptr[ctx->device], DISCO_ESTATE,
                "no scratch bound on device %d", ctx->device);
        activate(ctx);
        if (nrhs == 0) return;
        // not profiled: a profiled launch may create HIP events
        struct NoProfile {
            disco_ctx* c;
            bool was;
            ~NoProfile() { c->prof_on = was; }
        } np{ctx, ctx->prof_on};
        ctx->prof_on = false;
        char* base = (char*)scratch_ptr[ctx->device];
        const int cap = (int)std::min<long long>({fit, 64LL, (long long)disco::plane_rhs_limit(ctx)});
        const size_t off = (disco::native_bytes(ctx, prec, cap) + 255) & ~(size_t)255;
        const size_t field = (size_t)ctx->V * 12 * sizeof(double2);
        for (int r0 = 0; r0 < nrhs; r0 += cap) {
            const int n = std::min(cap, nrhs - r0);
            void* a = base;
            void* b = base + off;
            disco::to_native(ctx, prec, n, (const char*)in + r0 * field, a);
            disco::StencilCall c{prec, dagger ? 1 : 0, n, a, b, nullptr, nullptr, nullptr, nullptr, disco::EPI_NONE};
            disco::stencil_launch(ctx, c);
            disco::from_native(ctx, prec, n, b, (char*)out + r0 * field);
        }
    });
}
