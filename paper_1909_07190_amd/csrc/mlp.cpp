// Learned cost model: a fully connected network over the 40 group/schedule
// features predicting log kernel time, trained on the device by the kernels
// in mlp.hip (forward, backward, MSE, Adam).  Used by WT_SCHED_MLP to rank
// candidate configurations; the analytical model stays the fallback when a
// candidate's features fall outside the training range.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <fstream>
#include <numeric>
#include <sstream>

#include "wt_mlp.h"
#include "wt_runtime.h"

namespace wt {

hipError_t mlp_gemm(hipStream_t st, int ta, int tb, const float* A, int lda, const float* B, int ldb, float* C,
                    int ldc, int M, int N, int K, const float* bias, int relu, const float* mask, int ldm,
                    int accumulate);
hipError_t mlp_colsum(hipStream_t st, const float* X, int ld, int M, int N, float* out);
hipError_t mlp_mse(hipStream_t st, const float* y, const float* t, int B, float* dy, float* loss);
hipError_t mlp_adam(hipStream_t st, float* p, const float* g, float* m, float* v, int n, float lr, float b1,
                    float b2, float eps, float bc1, float bc2);

namespace {
uint64_t splitmix(uint64_t& s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
double uniform01(uint64_t& s) { return (splitmix(s) >> 11) * (1.0 / 9007199254740992.0); }

float* dalloc(size_t n) {
    void* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(float)) != hipSuccess) fail(WT_E_NOMEM, "mlp device buffer");
    hip_check(hipMemset(p, 0, std::max<size_t>(n, 1) * sizeof(float)), "hipMemset");
    return static_cast<float*>(p);
}
void ck(hipError_t e, const char* w) { hip_check(e, w); }
}  // namespace

Mlp::Mlp(const std::vector<int>& d, uint64_t seed) : dims(d) {
    if (dims.size() < 2) fail(WT_E_INVALID, "mlp needs at least an input and an output layer");
    for (int v : dims)
        if (v < 1 || v > 4096) fail(WT_E_INVALID, "mlp layer width out of range");
    size_t off = 0;
    for (size_t l = 0; l + 1 < dims.size(); ++l) {
        woff.push_back(off);
        off += (size_t)dims[l] * dims[l + 1];
        boff.push_back(off);
        off += dims[l + 1];
    }
    nparams = off;
    host.assign(nparams, 0.f);
    // He initialisation (normal via Box-Muller), zero biases
    uint64_t s = seed;
    for (size_t l = 0; l + 1 < dims.size(); ++l) {
        double sd = std::sqrt(2.0 / dims[l]);
        for (size_t i = 0; i < (size_t)dims[l] * dims[l + 1]; ++i) {
            double u1 = std::max(uniform01(s), 1e-300), u2 = uniform01(s);
            host[woff[l] + i] = (float)(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2));
        }
    }
    in_mean.assign(dims[0], 0.f);
    in_std.assign(dims[0], 1.f);
}

Mlp::~Mlp() {
    release();
    if (stream && own_stream) hipStreamDestroy(stream);
}

void Mlp::use_stream(hipStream_t s) {
    if (dparams) fail(WT_E_INVALID, "the model's stream is set before its first device operation");
    stream = s;
    own_stream = false;
}

void Mlp::release() {
    for (float* p : {dparams, dgrads, dm, dv, dx, dt, dy, dloss})
        if (p) hipFree(p);
    for (float* p : dact)
        if (p) hipFree(p);
    for (float* p : ddz)
        if (p) hipFree(p);
    dparams = dgrads = dm = dv = dx = dt = dy = dloss = nullptr;
    dact.clear();
    ddz.clear();
    cap = 0;
}

void Mlp::ensure_device(int batch) {
    if (!dparams) {
        if (!stream) {
            hip_check(hipStreamCreate(&stream), "hipStreamCreate");
            own_stream = true;
        }
        dparams = dalloc(nparams);
        dgrads = dalloc(nparams);
        dm = dalloc(nparams);
        dv = dalloc(nparams);
        dloss = dalloc(1);
        upload_params();
    }
    if (batch <= cap) return;
    for (float* p : {dx, dt, dy})
        if (p) hipFree(p);
    for (float* p : dact)
        if (p) hipFree(p);
    for (float* p : ddz)
        if (p) hipFree(p);
    dact.clear();
    ddz.clear();
    cap = std::max(batch, 256);
    dx = dalloc((size_t)cap * dims[0]);
    dt = dalloc(cap);
    dy = dalloc(cap);
    for (size_t l = 1; l < dims.size(); ++l) {
        dact.push_back(dalloc((size_t)cap * dims[l]));
        ddz.push_back(dalloc((size_t)cap * dims[l]));
    }
}

void Mlp::upload_params() {
    ck(hipMemcpy(dparams, host.data(), nparams * sizeof(float), hipMemcpyHostToDevice), "hipMemcpy");
}
void Mlp::download_params() {
    ck(hipMemcpy(host.data(), dparams, nparams * sizeof(float), hipMemcpyDeviceToHost), "hipMemcpy");
}

// Activations for a batch already in dx: act[l] = relu(act[l-1] W_l + b_l)
// for hidden layers, the last layer linear.
void Mlp::forward_dev(int B) {
    const float* a = dx;
    int L = (int)dims.size() - 1;
    for (int l = 0; l < L; ++l) {
        ck(mlp_gemm(stream, 0, 0, a, dims[l], dparams + woff[l], dims[l + 1], dact[l], dims[l + 1], B, dims[l + 1],
                    dims[l], dparams + boff[l], l + 1 < L, nullptr, 0, 0),
           "mlp forward");
        a = dact[l];
    }
}

// Gradients of the MSE of act[L-1] against dt into dgrads (and the loss).
void Mlp::backward_dev(int B) {
    int L = (int)dims.size() - 1;
    ck(mlp_mse(stream, dact[L - 1], dt, B, ddz[L - 1], dloss), "mlp mse");
    for (int l = L - 1; l >= 0; --l) {
        const float* a_in = l == 0 ? dx : dact[l - 1];
        // dW_l = a_in^T dZ_l ; db_l = column sums of dZ_l
        ck(mlp_gemm(stream, 1, 0, a_in, dims[l], ddz[l], dims[l + 1], dgrads + woff[l], dims[l + 1], dims[l],
                    dims[l + 1], B, nullptr, 0, nullptr, 0, 0),
           "mlp dW");
        ck(mlp_colsum(stream, ddz[l], dims[l + 1], B, dims[l + 1], dgrads + boff[l]), "mlp db");
        if (l > 0)  // dZ_{l-1} = (dZ_l W_l^T) * [act_{l-1} > 0]
            ck(mlp_gemm(stream, 0, 1, ddz[l], dims[l + 1], dparams + woff[l], dims[l + 1], ddz[l - 1], dims[l], B,
                        dims[l], dims[l + 1], nullptr, 0, dact[l - 1], dims[l], 0),
               "mlp dX");
    }
}

void Mlp::forward(const float* x, int B, float* y) {
    ensure_device(B);
    ck(hipMemcpyAsync(dx, x, (size_t)B * dims[0] * sizeof(float), hipMemcpyHostToDevice, stream), "hipMemcpyAsync");
    forward_dev(B);
    ck(hipMemcpyAsync(y, dact.back(), (size_t)B * dims.back() * sizeof(float), hipMemcpyDeviceToHost, stream),
       "hipMemcpyAsync");
    ck(hipStreamSynchronize(stream), "hipStreamSynchronize");
}

float Mlp::forward_backward(const float* x, const float* t, int B, float* grads) {
    if (dims.back() != 1) fail(WT_E_UNSUPPORTED, "training needs one output");
    ensure_device(B);
    ck(hipMemcpyAsync(dx, x, (size_t)B * dims[0] * sizeof(float), hipMemcpyHostToDevice, stream), "hipMemcpyAsync");
    ck(hipMemcpyAsync(dt, t, (size_t)B * sizeof(float), hipMemcpyHostToDevice, stream), "hipMemcpyAsync");
    forward_dev(B);
    backward_dev(B);
    float loss = 0;
    ck(hipMemcpyAsync(&loss, dloss, sizeof(float), hipMemcpyDeviceToHost, stream), "hipMemcpyAsync");
    if (grads)
        ck(hipMemcpyAsync(grads, dgrads, nparams * sizeof(float), hipMemcpyDeviceToHost, stream), "hipMemcpyAsync");
    ck(hipStreamSynchronize(stream), "hipStreamSynchronize");
    return loss;
}

void Mlp::adam_step(float lr) {
    ++step;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    float bc1 = 1.f - std::pow(b1, (float)step), bc2 = 1.f - std::pow(b2, (float)step);
    ck(mlp_adam(stream, dparams, dgrads, dm, dv, (int)nparams, lr, b1, b2, eps, bc1, bc2), "mlp adam");
}

void Mlp::adam_from_host(const float* g, float lr) {
    ensure_device(1);
    ck(hipMemcpy(dgrads, g, nparams * sizeof(float), hipMemcpyHostToDevice), "hipMemcpy");
    adam_step(lr);
    ck(hipStreamSynchronize(stream), "hipStreamSynchronize");
    download_params();
}

float Mlp::train(const float* x, const float* t, int n, int epochs, int batch, float lr, uint64_t seed) {
    if (n < 2) fail(WT_E_INVALID, "training needs at least two samples");
    const int F = dims[0];
    // z-score features and target on the training set
    for (int f = 0; f < F; ++f) {
        double s = 0, s2 = 0;
        for (int i = 0; i < n; ++i) s += x[(size_t)i * F + f];
        double m = s / n;
        for (int i = 0; i < n; ++i) s2 += (x[(size_t)i * F + f] - m) * (x[(size_t)i * F + f] - m);
        double sd = std::sqrt(s2 / n);
        in_mean[f] = (float)m;
        in_std[f] = sd > 1e-12 ? (float)sd : 1.f;
    }
    double ts = 0, ts2 = 0;
    for (int i = 0; i < n; ++i) ts += t[i];
    t_mean = (float)(ts / n);
    for (int i = 0; i < n; ++i) ts2 += (t[i] - t_mean) * (t[i] - t_mean);
    t_std = std::max(1e-6f, (float)std::sqrt(ts2 / n));
    std::vector<float> xn((size_t)n * F), tn(n);
    for (int i = 0; i < n; ++i) {
        for (int f = 0; f < F; ++f) xn[(size_t)i * F + f] = (x[(size_t)i * F + f] - in_mean[f]) / in_std[f];
        tn[i] = (t[i] - t_mean) / t_std;
    }
    batch = std::max(1, std::min(batch, n));
    ensure_device(batch);
    std::vector<int> perm(n);
    std::iota(perm.begin(), perm.end(), 0);
    uint64_t s = seed;
    std::vector<float> bx((size_t)batch * F), bt(batch);
    float last = 0;
    for (int ep = 0; ep < epochs; ++ep) {
        for (int i = n - 1; i > 0; --i) std::swap(perm[i], perm[splitmix(s) % (uint64_t)(i + 1)]);
        double sum = 0;
        int nb = 0;
        for (int b0 = 0; b0 + batch <= n; b0 += batch) {
            for (int j = 0; j < batch; ++j) {
                std::memcpy(&bx[(size_t)j * F], &xn[(size_t)perm[b0 + j] * F], F * sizeof(float));
                bt[j] = tn[perm[b0 + j]];
            }
            ck(hipMemcpyAsync(dx, bx.data(), bx.size() * sizeof(float), hipMemcpyHostToDevice, stream), "copy");
            ck(hipMemcpyAsync(dt, bt.data(), bt.size() * sizeof(float), hipMemcpyHostToDevice, stream), "copy");
            forward_dev(batch);
            backward_dev(batch);
            adam_step(lr);
            float l = 0;
            ck(hipMemcpyAsync(&l, dloss, sizeof(float), hipMemcpyDeviceToHost, stream), "copy");
            ck(hipStreamSynchronize(stream), "sync");
            sum += l;
            ++nb;
        }
        last = nb ? (float)(sum / nb) : 0.f;
    }
    download_params();
    trained = true;
    return last;
}

void Mlp::predict(const float* x, int n, float* y) {
    const int F = dims[0];
    std::vector<float> xn((size_t)n * F);
    for (int i = 0; i < n; ++i)
        for (int f = 0; f < F; ++f) xn[(size_t)i * F + f] = (x[(size_t)i * F + f] - in_mean[f]) / in_std[f];
    std::vector<float> raw(n);
    forward(xn.data(), n, raw.data());
    for (int i = 0; i < n; ++i) y[i] = raw[i] * t_std + t_mean;
}

double Mlp::max_abs_z(const float* x) const {
    double z = 0;
    for (size_t f = 0; f < in_mean.size(); ++f) z = std::max(z, (double)std::fabs((x[f] - in_mean[f]) / in_std[f]));
    return z;
}

void Mlp::save(const std::string& path) const {
    std::ofstream f(path);
    if (!f) fail(WT_E_INVALID, "cannot write model file " + path);
    f.precision(9);
    f << "wavetile-mlp 1\n" << dims.size();
    for (int d : dims) f << " " << d;
    f << "\n" << t_mean << " " << t_std << "\n";
    for (size_t i = 0; i < in_mean.size(); ++i) f << in_mean[i] << " " << in_std[i] << "\n";
    for (float v : host) f << v << "\n";
}

std::unique_ptr<Mlp> Mlp::load(const std::string& path) {
    std::ifstream f(path);
    std::string magic;
    int ver = 0;
    if (!(f >> magic >> ver) || magic != "wavetile-mlp" || ver != 1) fail(WT_E_INVALID, "not a model file: " + path);
    size_t nl = 0;
    f >> nl;
    if (nl < 2 || nl > 16) fail(WT_E_INVALID, "bad model file");
    std::vector<int> d(nl);
    for (auto& v : d) f >> v;
    auto m = std::make_unique<Mlp>(d, 1);
    f >> m->t_mean >> m->t_std;
    for (size_t i = 0; i < m->in_mean.size(); ++i) f >> m->in_mean[i] >> m->in_std[i];
    for (auto& v : m->host) f >> v;
    if (!f) fail(WT_E_INVALID, "truncated model file " + path);
    m->trained = true;
    return m;
}

}  // namespace wt
