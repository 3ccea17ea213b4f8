// Learned cost model (see mlp.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <memory>
#include <string>
#include <vector>

#include "wt_internal.h"

namespace wt {

// Streaming device copy, the benchmark's achievable-bandwidth reference
// (copyref.hip).
hipError_t stream_copy(const void* src, void* dst, size_t bytes, hipStream_t stream);

struct Mlp {
    std::vector<int> dims;              // layer widths, input first
    std::vector<size_t> woff, boff;     // offsets of W_l (dims[l] x dims[l+1], row-major) and b_l
    size_t nparams = 0;
    std::vector<float> host;            // parameters (host copy)
    std::vector<float> in_mean, in_std; // feature normalisation
    float t_mean = 0, t_std = 1;        // target normalisation
    bool trained = false;
    int step = 0;                       // Adam step count

    Mlp(const std::vector<int>& dims, uint64_t seed);
    ~Mlp();
    void forward(const float* x, int B, float* y);                  // raw network
    float forward_backward(const float* x, const float* t, int B, float* grads);
    void adam_from_host(const float* g, float lr);
    float train(const float* x, const float* t, int n, int epochs, int batch, float lr, uint64_t seed);
    void predict(const float* x, int n, float* y);                  // normalised in, target units out
    double max_abs_z(const float* x) const;
    // Device work runs on `s` (the caller's, kept) instead of a stream of
    // the model's own; call before the first device operation.
    void use_stream(hipStream_t s);
    void upload_params();
    void download_params();
    void save(const std::string& path) const;
    static std::unique_ptr<Mlp> load(const std::string& path);

   private:
    hipStream_t stream = nullptr;
    bool own_stream = false;
    float *dparams = nullptr, *dgrads = nullptr, *dm = nullptr, *dv = nullptr;
    float *dx = nullptr, *dt = nullptr, *dy = nullptr, *dloss = nullptr;
    std::vector<float*> dact, ddz;
    int cap = 0;
    void ensure_device(int batch);
    void forward_dev(int B);
    void backward_dev(int B);
    void adam_step(float lr);
    void release();
};

// Rows of a measurement database (JSON lines): the 40 features (row-major
// into x) and log(measured microseconds) (into t) of every usable line;
// returns the row count.
int read_measure_db(const std::string& path, std::vector<float>& x, std::vector<float>& t);
// Trains the cost network (40-128-128-128-1, 200 epochs of Adam, batch 256,
// lr 1e-3, seed 1) on every usable row of `db` and saves it to `out_model`.
void train_model_from_db(const std::string& db, const std::string& out_model, hipStream_t stream);

}  // namespace wt
