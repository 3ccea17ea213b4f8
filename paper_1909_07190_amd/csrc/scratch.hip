// The library's fixed device workspace, for wt_plan_run_batch_static: the
// entry point for callers that cannot allocate device memory.  It is one
// file-scope array of WT_STATIC_SCRATCH_BYTES; every GPU the library uses it
// on holds its own copy, at its own address, from the first lookup until
// the process ends.  Host code never passes the array's name to a kernel
// (in host code it is only a stand-in for the symbol): the device address
// comes from hipGetSymbolAddress, once per device, with that device current.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/wt.h"

namespace {

__device__ __align__(256) unsigned char scratch[WT_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};

}  // namespace

namespace wt {

// Device address of `device`'s copy of the workspace, which must be the
// current device; looked up on its first use and kept.  On failure returns
// nullptr and the HIP error in *err.
void* static_scratch(int device, hipError_t* err) {
    *err = hipSuccess;
    if (device < 0 || device >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess || cur != device) {
            *err = e != hipSuccess ? e : hipErrorInvalidDevice;
            return nullptr;
        }
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
            return nullptr;
        }
        g_addr[device] = p;
    }
    return g_addr[device];
}

}  // namespace wt
