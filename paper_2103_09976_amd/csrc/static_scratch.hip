// The one entry point of the library that allocates nothing at all:
// dmrg_heff_apply_static, the product dmrg_heff_apply with the partial tiles
// of split tasks in a static device array instead of the context arena.
//
// `scratch` is a file-scope device array of kScratchBytes on every GPU the
// library runs on (held until the process ends).  Its name in host code is a
// host-side stand-in, never a device address: the device address is taken
// once per device with hipGetSymbolAddress (with that device current) and
// kept in g_scratch; only that pointer is passed to kernels.  Every call on
// one GPU shares the array, so calls that overlap on one GPU race; the array
// holds nothing that must start at zero (each split task writes its whole
// partial tile before the reduction reads it).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "core.hpp"

namespace {
constexpr int64_t kScratchBytes = int64_t(256) << 20;   // 256 MiB per device
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) char scratch[kScratchBytes];

static void* g_scratch[kMaxDevices];
static std::mutex g_scratch_mu;

// Device address of `scratch` on the current device (looked up at the first
// call on each device).
static dmrg_status scratch_address(void** out) {
    int dev = -1;
    DMRG_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return dmrg::fail(DMRG_E_UNSUPPORTED, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return dmrg::hip_fail((int)e, "hipGetSymbolAddress(scratch)");
        if (!p) return dmrg::fail(DMRG_E_HIP, "hipGetSymbolAddress(scratch) returned no address");
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return DMRG_OK;
}

dmrg_status heff_apply_impl(dmrg_heff* H, int32_t precision, int32_t n_vec, const void* psi, void* sigma,
                            void* partial, int64_t partial_bytes, void* stream);

extern "C" dmrg_status dmrg_heff_apply_static(dmrg_heff* H, int32_t precision, int32_t n_vec, const void* psi,
                                              void* sigma, void* stream) {
    if (!H || !psi || !sigma) return dmrg::fail(DMRG_E_ARG, "null argument");
    void* p = nullptr;
    const dmrg_status st = scratch_address(&p);
    if (st != DMRG_OK) return st;
    return heff_apply_impl(H, precision, n_vec, psi, sigma, p, kScratchBytes, stream);
}
