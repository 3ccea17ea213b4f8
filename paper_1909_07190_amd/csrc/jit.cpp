// Run-time compilation of generated kernels with hipRTC for gfx950, with an
// in-process cache and an optional on-disk code-object cache keyed by a hash
// of the source and the compile options.
#include <hip/hiprtc.h>

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <mutex>
#include <sstream>
#include <sys/stat.h>
#include <unistd.h>
#include <unordered_map>

#include "wt_internal.h"

namespace wt {

namespace {
// Packed-FP32 VALU forms are disabled for all generated code.
const char* kOpts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17",
                       "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
const int kNumOpts = sizeof(kOpts) / sizeof(kOpts[0]);

uint64_t fnv1a(const std::string& s, uint64_t h = 1469598103934665603ull) {
    for (unsigned char c : s) {
        h ^= c;
        h *= 1099511628211ull;
    }
    return h;
}

std::mutex g_mu;
std::unordered_map<uint64_t, std::vector<char>> g_cache;
}  // namespace

std::vector<char> compile_hip(const std::string& src, const std::string& name,
                              const std::string& cache_dir) {
    std::string key = src;
    for (int i = 0; i < kNumOpts; ++i) key += std::string("\n//opt ") + kOpts[i];
    uint64_t h = fnv1a(key);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_cache.find(h);
        if (it != g_cache.end()) return it->second;
    }
    char hex[32];
    std::snprintf(hex, sizeof hex, "%016llx", (unsigned long long)h);
    std::string path;
    if (!cache_dir.empty()) {
        path = cache_dir + "/wt_" + hex + ".co";
        std::ifstream f(path, std::ios::binary);
        if (f) {
            std::vector<char> code((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
            // A cached object is trusted only if it carries the source hash
            // trailer written below (a torn or foreign file is recompiled).
            if (code.size() > 16 && std::string(code.end() - 16, code.end()) == hex) {
                code.resize(code.size() - 16);
                std::lock_guard<std::mutex> lk(g_mu);
                g_cache[h] = code;
                return code;
            }
        }
    }
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), (name + ".hip").c_str(), 0, nullptr, nullptr) !=
        HIPRTC_SUCCESS)
        fail(WT_E_COMPILE, "hiprtcCreateProgram failed");
    hiprtcResult rc = hiprtcCompileProgram(prog, kNumOpts, kOpts);
    if (rc != HIPRTC_SUCCESS) {
        size_t n = 0;
        hiprtcGetProgramLogSize(prog, &n);
        std::string log(n, '\0');
        if (n) hiprtcGetProgramLog(prog, &log[0]);
        hiprtcDestroyProgram(&prog);
        fail(WT_E_COMPILE, "compiling " + name + ": " + log.substr(0, 4000));
    }
    size_t n = 0;
    hiprtcGetCodeSize(prog, &n);
    std::vector<char> code(n);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    if (!path.empty()) {
        mkdir(cache_dir.c_str(), 0755);
        std::string tmp = path + ".tmp" + std::to_string(::getpid());
        std::ofstream f(tmp, std::ios::binary);
        if (f) {
            f.write(code.data(), code.size());
            f.write(hex, 16);
            f.close();
            std::rename(tmp.c_str(), path.c_str());
        }
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[h] = code;
    return code;
}

}  // namespace wt
