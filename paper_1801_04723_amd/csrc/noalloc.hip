// spin_invert_noalloc: the FP64 inversion of spin_invert without any device
// allocation, for callers that cannot allocate (code under stream capture,
// serving loops that forbid allocation).  Its workspace is `scratch`, a
// fixed array in device memory that every GPU the library runs on holds
// until the process ends.  The host resolves the array's device address once
// per device (hipGetSymbolAddress, with that device current) and passes only
// that address to the kernels; the array's name in host code is not a device
// address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "spin.h"
#include "spin_plan.hpp"

namespace {

constexpr size_t kScratchBytes = size_t(SPIN_NOALLOC_SCRATCH_MB) << 20;
__device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char *g_ptr[kMaxDevices];  // device address of `scratch` on each device

// The address of the current device's scratch, or nullptr on failure.
char *scratch_ptr() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_ptr[dev] = static_cast<char *>(p);
    }
    return g_ptr[dev];
}

}  // namespace

extern "C" int spin_invert_noalloc(const double *A, int64_t n, int64_t lda, double *Ainv,
                                   int64_t ldx, int64_t leaf, int *info, spin_stream_t stream) {
    char *ws = scratch_ptr();
    if (!ws) return SPIN_E_HIP;
    return spin::invert_on_workspace(A, n, lda, Ainv, ldx, leaf, ws, kScratchBytes, info,
                                     reinterpret_cast<hipStream_t>(stream));
}
