// Device scratch of the no-allocation entry point (kde_eval_noalloc).
//
// Callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc) get the estimate's
// workspace from this file-scope array instead of a caller buffer. Each GPU
// the library runs on holds its own copy at its own address until the process
// ends. In host code the array's name stands for a host-side shadow, not a
// device address, so the host never uses it directly: the device address of
// each GPU's copy is looked up once, with that GPU current, and kept.
//
// Every call on a GPU shares that GPU's copy, which keeps the previous call's
// contents; calls that overlap on one GPU race.

#include <mutex>

#include "kde_internal.h"

namespace kde {
namespace {

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

hipError_t scratch_address(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices || !out) return hipErrorInvalidValue;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        const hipError_t back = cur != dev ? hipSetDevice(cur) : hipSuccess;
        if (e != hipSuccess) return e;
        if (back != hipSuccess) return back;
        if (!ptr || reinterpret_cast<uintptr_t>(ptr) % 256 != 0) return hipErrorInvalidValue;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace kde
