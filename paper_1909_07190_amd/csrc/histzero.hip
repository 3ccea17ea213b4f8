// Clears histogram outputs before the kernel that accumulates them.  A
// kernel rather than a memset, so that a hipGraph capturing the launch
// sequence replays the clearing like any other node.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "wt_runtime.h"

namespace {

__global__ void __launch_bounds__(256) zero_planes(unsigned int* base, long long cs, int n) {
    unsigned int* p = base + (long long)blockIdx.y * cs;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = 0u;
}

// image blockIdx.z of a batch: output `d` of its argument table entry
__global__ void __launch_bounds__(256) zero_planes_batch(const wt::WtArgsHost* __restrict__ ab, int d, int n) {
    const wt::WtArgsHost& a = ab[blockIdx.z];
    unsigned int* p = (unsigned int*)a.dst[d] + (long long)blockIdx.y * a.dst_cs[d];
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = 0u;
}

unsigned blocks_for(int n) { return (unsigned)std::min(16, (n + 255) / 256); }

}  // namespace

namespace wt {

hipError_t zero_hist(void* base, long long cs, int n, int planes, hipStream_t s) {
    hipLaunchKernelGGL(zero_planes, dim3(blocks_for(n), (unsigned)planes), dim3(256), 0, s, (unsigned int*)base, cs, n);
    return hipGetLastError();
}

hipError_t zero_hist_batch(const void* table, int nimg, int d, int n, int planes, hipStream_t s) {
    hipLaunchKernelGGL(zero_planes_batch, dim3(blocks_for(n), (unsigned)planes, (unsigned)nimg), dim3(256), 0, s,
                       (const WtArgsHost*)table, d, n);
    return hipGetLastError();
}

}  // namespace wt
