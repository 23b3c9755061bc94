// Operator product without device allocation (vie_apply_noalloc), for callers
// that cannot allocate: code under stream capture, tight serving loops.
//
// The FFT intermediates of the product (the only scratch memory it needs
// beyond the caller's x and y and the context's resident operator and
// contrast) live in one fixed, file-scope device array, `scratch`, of
// VIE_NOALLOC_SCRATCH_BYTES.  Every GPU the library is loaded on holds its
// own copy of the array until the process ends.  The host never uses the
// array's name as an address: vie_create looks its device address up once
// per device, with that device current, and every launch takes that address.
// Calls on one GPU share the array, so products issued at the same time on
// one GPU (from any context or stream) overwrite each other's intermediates:
// the caller must order them.  Nothing in the array has to start at zero
// (every intermediate is written before it is read), so nothing is cleared.
#include <mutex>

#include "ctx.hpp"

namespace vie {

constexpr size_t kNoallocBytes = VIE_NOALLOC_SCRATCH_BYTES;
constexpr int kNoallocDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

static std::mutex g_noalloc_m;
static void* g_noalloc_ptr[kNoallocDevices] = {};   // device address of `scratch` per device

void noalloc_init(int device) {
    std::lock_guard<std::mutex> g(g_noalloc_m);
    VIE_REQUIRE(device >= 0 && device < kNoallocDevices, VIE_EINVAL, "device index above the supported 64");
    if (g_noalloc_ptr[device]) return;
    int cur = -1;
    VIE_HIP(hipGetDevice(&cur));
    VIE_REQUIRE(cur == device, VIE_EDEVICE, "no-allocation workspace looked up with another device current");
    void* p = nullptr;
    VIE_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    VIE_REQUIRE(p != nullptr, VIE_EDEVICE, "no device address for the no-allocation workspace");
    g_noalloc_ptr[device] = p;
}

static void* noalloc_ptr(int device) {
    std::lock_guard<std::mutex> g(g_noalloc_m);
    return (device >= 0 && device < kNoallocDevices) ? g_noalloc_ptr[device] : nullptr;
}

}  // namespace vie

using namespace vie;

extern "C" int vie_apply_noalloc(vie_ctx* ctx, int op, int precision, int nrhs, const void* x, void* y) {
    return guarded([&] {
        VIE_REQUIRE(ctx != nullptr, VIE_EINVAL, "null context");
        Ctx& c = ctx->c;
        VIE_HIP(hipSetDevice(c.device));
        VIE_REQUIRE(op == VIE_OP_PREC || op == VIE_OP_A || op == VIE_OP_N, VIE_EINVAL, "unknown operator");
        VIE_REQUIRE(nrhs >= 1 && x && y, VIE_EINVAL, "bad arguments");
        VIE_REQUIRE(precision == VIE_C64 || precision == VIE_C128, VIE_EINVAL,
                    "precision must be VIE_C64 or VIE_C128");
        VIE_REQUIRE(c.has_grid, VIE_ESTATE, "vie_apply_noalloc before vie_set_grid");
        const size_t bytes = (size_t)nrhs * c.nc * c.V * (precision == VIE_C64 ? 8 : 16);
        const uintptr_t px = reinterpret_cast<uintptr_t>(x), py = reinterpret_cast<uintptr_t>(y);
        VIE_REQUIRE(!(px < py + bytes && py < px + bytes), VIE_EINVAL, "x and y must not overlap");
        void* ws = noalloc_ptr(c.device);
        VIE_REQUIRE(ws != nullptr, VIE_ESTATE, "no-allocation workspace not set up for this device");
        // the launch profiler takes events from a pool that may grow: off here
        const bool prof = c.prof.on;
        c.prof.on = false;
        try {
            if (precision == VIE_C64)
                apply_op<float>(c, op, nrhs, static_cast<const float2*>(x), static_cast<float2*>(y), nullptr, ws,
                                kNoallocBytes);
            else
                apply_op<double>(c, op, nrhs, static_cast<const double2*>(x), static_cast<double2*>(y), nullptr, ws,
                                 kNoallocBytes);
        } catch (...) {
            c.prof.on = prof;
            throw;
        }
        c.prof.on = prof;
    });
}
