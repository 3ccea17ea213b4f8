// Streaming device copy: the achievable-bandwidth reference that the
// benchmark reports beside the pipeline kernels.  One 16-byte element per
// thread, nontemporal loads and stores (the data is touched once), 256
// threads per workgroup; the byte tail past the last whole element goes
// through a second one-byte-per-thread kernel.  Not part of any pipeline.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace {

typedef unsigned int u4v __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) copy16_nt(const u4v* __restrict__ src, u4v* __restrict__ dst, long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

__global__ void __launch_bounds__(256) copy1(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst,
                                             long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

}  // namespace

namespace wt {

// Copies `bytes` bytes from src to dst (device pointers, 16-byte aligned,
// not overlapping) on `stream`; returns the launch status.
hipError_t stream_copy(const void* src, void* dst, size_t bytes, hipStream_t stream) {
    const long long n16 = (long long)(bytes / 16);
    if (n16 > 0) {
        const long long blocks = (n16 + 255) / 256;
        hipLaunchKernelGGL(copy16_nt, dim3((unsigned)blocks), dim3(256), 0, stream, (const u4v*)src, (u4v*)dst, n16);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const long long tail = (long long)(bytes - (size_t)n16 * 16);
    if (tail > 0) {
        hipLaunchKernelGGL(copy1, dim3(1), dim3(256), 0, stream, (const unsigned char*)src + n16 * 16,
                           (unsigned char*)dst + n16 * 16, tail);
        return hipGetLastError();
    }
    return hipSuccess;
}

}  // namespace wt
