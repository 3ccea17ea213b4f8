// Device kernels of the learned cost model: a small fully connected network
// (ReLU hidden layers, one linear output) trained with MSE on log kernel
// time and Adam.  FP32 on the vector ALUs (these products are far too small
// for matrix cores to matter), LDS-tiled.
#include <hip/hip_runtime.h>

namespace {

constexpr int TM = 64, TN = 64, TK = 16;  // workgroup tile; 256 threads, 4x4 outputs each

// C[M x N] = op(A) * op(B) (+ bias[n]) with op(X) = X or X^T, then optional
// ReLU, then optional mask: C[m][n] *= (mask[m*ldm + n] > 0).
//   A: M x K (TA = 0, row-major, lda) or K x M (TA = 1)
//   B: K x N (TB = 0, row-major, ldb) or N x K (TB = 1)
template <int TA, int TB>
__global__ void __launch_bounds__(256)
gemm_kernel(const float* __restrict__ A, int lda, const float* __restrict__ B, int ldb,
            float* __restrict__ C, int ldc, int M, int N, int K, const float* __restrict__ bias,
            int relu, const float* __restrict__ mask, int ldm, int accumulate) {
    __shared__ float As[TK][TM + 1];
    __shared__ float Bs[TK][TN + 1];
    const int tid = threadIdx.x;
    const int tm = (tid / 16) * 4, tn = (tid % 16) * 4;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    float acc[4][4] = {};
    for (int k0 = 0; k0 < K; k0 += TK) {
        for (int i = tid; i < TK * TM; i += 256) {
            int kk = i / TM, mm = i % TM;
            int m = m0 + mm, k = k0 + kk;
            float v = 0.f;
            if (m < M && k < K) v = TA ? A[(size_t)k * lda + m] : A[(size_t)m * lda + k];
            As[kk][mm] = v;
        }
        for (int i = tid; i < TK * TN; i += 256) {
            int kk = i / TN, nn = i % TN;
            int n = n0 + nn, k = k0 + kk;
            float v = 0.f;
            if (n < N && k < K) v = TB ? B[(size_t)n * ldb + k] : B[(size_t)k * ldb + n];
            Bs[kk][nn] = v;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TK; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][tm + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tn + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int m = m0 + tm + i, n = n0 + tn + j;
            if (m >= M || n >= N) continue;
            float v = acc[i][j];
            if (bias) v += bias[n];
            if (relu) v = v > 0.f ? v : 0.f;
            if (mask && !(mask[(size_t)m * ldm + n] > 0.f)) v = 0.f;
            if (accumulate) v += C[(size_t)m * ldc + n];
            C[(size_t)m * ldc + n] = v;
        }
}

// out[n] = sum_m X[m][n] (column sums, the bias gradient); one thread per column.
__global__ void colsum_kernel(const float* __restrict__ X, int ld, int M, int N, float* __restrict__ out) {
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int m = 0; m < M; ++m) s += X[(size_t)m * ld + n];
    out[n] = s;
}

// Mean squared error of y against t over B samples: dy = 2 (y - t) / B and
// loss = mean (y - t)^2 (one workgroup, fixed-order reduction).
__global__ void __launch_bounds__(256) mse_kernel(const float* __restrict__ y, const float* __restrict__ t, int B,
                                                  float* __restrict__ dy, float* __restrict__ loss) {
    __shared__ float red[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < B; i += 256) {
        float d = y[i] - t[i];
        dy[i] = 2.f * d / B;
        s += d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0] / B;
}

// Adam (Kingma & Ba 2015) with bias-corrected moments.
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float bc1,
                            float bc2) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float gi = g[i];
    float mi = b1 * m[i] + (1.f - b1) * gi;
    float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    float mh = mi / bc1, vh = vi / bc2;
    p[i] -= lr * mh / (sqrtf(vh) + eps);
}

}  // namespace

// Host-side launchers (C++ linkage inside the library).
namespace wt {

hipError_t mlp_gemm(hipStream_t st, int ta, int tb, const float* A, int lda, const float* B, int ldb, float* C,
                    int ldc, int M, int N, int K, const float* bias, int relu, const float* mask, int ldm,
                    int accumulate) {
    dim3 grid((N + TN - 1) / TN, (M + TM - 1) / TM), block(256);
    if (!ta && !tb)
        gemm_kernel<0, 0><<<grid, block, 0, st>>>(A, lda, B, ldb, C, ldc, M, N, K, bias, relu, mask, ldm, accumulate);
    else if (!ta && tb)
        gemm_kernel<0, 1><<<grid, block, 0, st>>>(A, lda, B, ldb, C, ldc, M, N, K, bias, relu, mask, ldm, accumulate);
    else if (ta && !tb)
        gemm_kernel<1, 0><<<grid, block, 0, st>>>(A, lda, B, ldb, C, ldc, M, N, K, bias, relu, mask, ldm, accumulate);
    else
        gemm_kernel<1, 1><<<grid, block, 0, st>>>(A, lda, B, ldb, C, ldc, M, N, K, bias, relu, mask, ldm, accumulate);
    return hipGetLastError();
}

hipError_t mlp_colsum(hipStream_t st, const float* X, int ld, int M, int N, float* out) {
    colsum_kernel<<<(N + 127) / 128, 128, 0, st>>>(X, ld, M, N, out);
    return hipGetLastError();
}

hipError_t mlp_mse(hipStream_t st, const float* y, const float* t, int B, float* dy, float* loss) {
    mse_kernel<<<1, 256, 0, st>>>(y, t, B, dy, loss);
    return hipGetLastError();
}

hipError_t mlp_adam(hipStream_t st, float* p, const float* g, float* m, float* v, int n, float lr, float b1,
                    float b2, float eps, float bc1, float bc2) {
    adam_kernel<<<(n + 255) / 256, 256, 0, st>>>(p, g, m, v, n, lr, b1, b2, eps, bc1, bc2);
    return hipGetLastError();
}

}  // namespace wt
