// noalloc.hip -- the library's own device scratch, for callers that cannot
// allocate (code under HIP graph capture, serving loops, harnesses that forbid
// hipMalloc).  psp_solve_batched_noalloc runs the step-schedule path with its
// per-system solutions (batch x K x n doubles when the batch is too small for
// one workgroup per Jacobian) in this array instead of a caller workspace.
//
// The array is a file-scope __device__ variable: every GPU the library runs on
// holds its own copy until the process ends.  In host code its name is only a
// host-side stand-in, so the device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and only that address is ever
// passed to kernels.  Every call on a GPU shares that GPU's copy and leaves its
// contents behind; nothing in it needs to start at zero (each solution entry
// is written before the combine reads it).  Calls that overlap on one GPU race.
#include <mutex>

#include "sparse.h"

namespace psp {

namespace {

constexpr size_t kScratchBytes = 16u << 20;   // 16 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

// Device address of the current device's scratch (looked up on first use per device).
hipError_t noalloc_scratch(void** out) {
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

}  // namespace psp
