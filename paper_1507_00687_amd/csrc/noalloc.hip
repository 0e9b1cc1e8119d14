// fastmm_gemm_noalloc: fastmm_gemm with its workspace in a fixed device array of the library,
// for callers that cannot allocate device memory.
//
// `scratch` below is a file-scope device array: every GPU the library runs on holds its own
// copy, at its own address, from the first use on that GPU until the process ends.  In host
// code the name `scratch` is only a host-side stand-in, so the device address of each GPU's
// copy is looked up once per device with hipGetSymbolAddress (with that device current) and
// kept; kernels receive that address, never the name.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "fastmm.h"
#include "fastmm_internal.h"

namespace fastmm {
namespace {

constexpr size_t kScratchBytes = FASTMM_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch` (looked up once per device).
fastmm_status scratch_of_current_device(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_error(std::string("hipGetDevice: ") + hipGetErrorString(e));
        return FASTMM_EHIP;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("fastmm_gemm_noalloc: device index " + std::to_string(dev) + " beyond the supported " +
                  std::to_string(kMaxDevices));
        return FASTMM_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return FASTMM_EHIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return FASTMM_OK;
}

}  // namespace
}  // namespace fastmm

using namespace fastmm;

extern "C" fastmm_status fastmm_gemm_noalloc(fastmm_plan_t plan, const void *A, const void *B, void *C, int64_t m,
                                             int64_t k, int64_t n, void *stream) {
    if (!plan) {
        set_error("null plan");
        return FASTMM_EINVAL;
    }
    size_t need = 0;
    fastmm_status st = fastmm_workspace_size(plan, m, k, n, &need);
    if (st != FASTMM_OK) return st;
    if (need > kScratchBytes) {
        set_error("fastmm_gemm_noalloc: this product needs " + std::to_string(need) +
                  " bytes of workspace; the fixed scratch array holds " + std::to_string(kScratchBytes));
        return FASTMM_EWORKSPACE;
    }
    void *ws = nullptr;
    if ((st = scratch_of_current_device(&ws)) != FASTMM_OK) return st;
    set_no_alloc(true);
    st = fastmm_gemm(plan, A, B, C, m, k, n, ws, kScratchBytes, stream);
    set_no_alloc(false);
    return st;
}
