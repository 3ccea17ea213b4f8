// Pre-profiling of stages (the paper, Section 6): before the fusion search,
// every stage's body is timed on the device as a microbenchmark -- one
// workgroup, a single active lane, operands read from LDS, many iterations --
// giving the time of one evaluation, and the VGPRs its unfused kernel
// allocates are read from the compiled code object.  The analytical model
// uses both (compute time per wave and the register tile); results are cached
// per stage signature for the life of the process.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <mutex>
#include <sstream>

#include "wt_cost.h"
#include "wt_runtime.h"

namespace wt {

namespace {

std::mutex g_mu;
std::map<std::string, StageProfile> g_prof;

constexpr int kIters = 1 << 16;

// Everything that determines the stage body's code.
std::string stage_key(const Pipeline& p, int id) {
    const Node& n = p.nodes[id];
    std::ostringstream os;
    os.precision(17);
    os << (int)n.kind << "|" << n.dtype << "|" << n.kw << "x" << n.kh << "|" << n.scale << "|" << n.divisor << "|"
       << n.expr_text << "|";
    for (double w : n.weights) os << w << ",";
    for (int s : n.srcs) os << "d" << p.nodes[s].dtype;
    return os.str();
}

// C expression of a pointwise expression tree, sources given as strings.
std::string emit_expr(const Expr& e, bool in, const std::vector<std::string>& src) {
    auto K = [&](int i) { return emit_expr(e.kids[i], in, src); };
    char b[64];
    switch (e.op) {
        case Expr::Const:
            if (in) return "(" + std::to_string((long long)e.value) + ")";
            std::snprintf(b, sizeof b, "(%.9ef)", e.value);
            return b;
        case Expr::Src: return src[e.src];
        case Expr::Neg: return "(-" + K(0) + ")";
        case Expr::Add: return "(" + K(0) + " + " + K(1) + ")";
        case Expr::Sub: return "(" + K(0) + " - " + K(1) + ")";
        case Expr::Mul: return "(" + K(0) + " * " + K(1) + ")";
        case Expr::Div: return "(" + K(0) + " / " + K(1) + ")";
        case Expr::Lt: return "(" + K(0) + " < " + K(1) + ")";
        case Expr::Le: return "(" + K(0) + " <= " + K(1) + ")";
        case Expr::Gt: return "(" + K(0) + " > " + K(1) + ")";
        case Expr::Ge: return "(" + K(0) + " >= " + K(1) + ")";
        case Expr::Abs: return (in ? "wt_abs(" : "fabsf(") + K(0) + ")";
        case Expr::Min: return (in ? "wt_min(" : "fminf(") + K(0) + ", " + K(1) + ")";
        case Expr::Max: return (in ? "wt_max(" : "fmaxf(") + K(0) + ", " + K(1) + ")";
        case Expr::Sqrt: return "sqrtf(" + K(0) + ")";
        case Expr::Floor: return "floorf(" + K(0) + ")";
        case Expr::Select: return "(" + K(0) + " ? " + K(1) + " : " + K(2) + ")";
    }
    fail(WT_E_INTERNAL, "bad expression node");
}

// Microbenchmark of one stage body (or, with id < 0, of the bare loop: one
// LDS operand per iteration), `kname(out, iters)`.
std::string bench_source(const Pipeline& p, int id, const std::string& kname) {
    const bool in = id >= 0 && p.nodes[id].is_int();
    const std::string T = in ? "int" : "float";
    std::ostringstream o;
    o << device_prelude() << "\n";
    o << "extern \"C\" __global__ void __launch_bounds__(64) " << kname << "(float* out, int iters) {\n";
    o << "    __shared__ " << T << " L[256];\n";
    o << "    for (int i = threadIdx.x; i < 256; i += 64) L[i] = (" << T << ")(i % 17) "
      << (in ? "+ 1" : "* 0.25f + 1.0f") << ";\n";
    o << "    __syncthreads();\n";
    o << "    if (threadIdx.x != 0) return;\n";
    o << "    " << (in ? "unsigned" : "float") << " acc = 0;\n";
    o << "    for (int it = 0; it < iters; ++it) {\n";
    o << "        const int b = it & 127;\n";
    std::string v;
    if (id < 0) {
        v = "L[b]";
    } else {
        const Node& n = p.nodes[id];
        if (n.kind == Kind::Stencil) {
            std::string acc;
            int t = 0;
            for (size_t k = 0; k < n.weights.size(); ++k) {
                if (n.weights[k] == 0.0) continue;
                std::string r = "L[(b + " + std::to_string(t++) + ") & 255]";
                if (in) {
                    std::string term = "(" + std::to_string((long long)n.weights[k]) + ") * " + r;
                    acc = acc.empty() ? term : acc + " + " + term;
                } else {
                    char w[64];
                    std::snprintf(w, sizeof w, "(%.9ef)", n.weights[k] * n.scale);
                    acc = acc.empty() ? std::string(w) + " * " + r : "fmaf(" + std::string(w) + ", " + r + ", " + acc + ")";
                }
            }
            if (acc.empty()) acc = "0";
            if (in) {
                auto rg = dtype_range(n.dtype);
                acc = "wt_sat(wt_rdiv(" + acc + ", " + std::to_string(n.divisor) + "), " + std::to_string(rg.first) +
                      ", " + std::to_string(rg.second) + ")";
            }
            v = acc;
        } else {
            std::vector<std::string> src;
            for (size_t i = 0; i < n.srcs.size(); ++i)
                src.push_back("L[(b + " + std::to_string(16 * i) + ") & 255]");
            v = emit_expr(n.expr, in, src);
        }
    }
    o << "        const " << T << " v = " << v << ";\n";
    if (in) o << "        acc = acc * 3u + (unsigned)v;\n";
    else o << "        acc += v;\n";
    o << "    }\n";
    o << "    out[0] = (float)acc;\n";
    o << "}\n";
    return o.str();
}

double time_kernel_ns(hipFunction_t fn, float* out, hipStream_t st) {
    OwnedEvents ev;
    hipEvent_t e0 = ev.e0, e1 = ev.e1;
    int iters = kIters;
    void* params[] = {&out, &iters};
    double best = INFINITY;
    for (int s = 0; s < 4; ++s) {  // first run warms up
        hip_check(hipEventRecord(e0, st), "hipEventRecord");
        hip_check(hipModuleLaunchKernel(fn, 1, 1, 1, 64, 1, 1, 0, st, params, nullptr), "hipModuleLaunchKernel");
        hip_check(hipEventRecord(e1, st), "hipEventRecord");
        hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
        float ms = 0;
        hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        if (s > 0) best = std::min(best, (double)ms * 1e6);
    }
    return best;
}

}  // namespace

bool preprofile_enabled() {
    const char* e = std::getenv("WT_PREPROFILE");
    return !(e && e[0] == '0');
}

bool lookup_profile(const Pipeline& p, int id, StageProfile& out) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_prof.find(stage_key(p, id));
    if (it == g_prof.end()) return false;
    out = it->second;
    return true;
}

void preprofile(const Plan& plan) {
    const Pipeline& p = plan.p;
    std::vector<int> todo;
    std::vector<std::string> keys;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (const Node& n : p.nodes) {
            if (n.kind != Kind::Stencil && n.kind != Kind::Pointwise) continue;
            std::string k = stage_key(p, n.id);
            if (g_prof.count(k) || std::find(keys.begin(), keys.end(), k) != keys.end()) continue;
            todo.push_back(n.id);
            keys.push_back(k);
        }
    }
    if (todo.empty()) return;
    // microbenchmarks (plus the bare loop) and each stage's unfused kernel
    std::vector<GroupRt> benches(todo.size() + 1), units(todo.size());
    for (size_t i = 0; i <= todo.size(); ++i) {
        int id = i < todo.size() ? todo[i] : -1;
        char name[64];
        std::snprintf(name, sizeof name, "wt_prof_%zu", i);
        std::string src = bench_source(p, id, "wt_kernel_name_placeholder");
        uint64_t h = 1469598103934665603ull;
        for (unsigned char c : src) h = (h ^ c) * 1099511628211ull;
        std::snprintf(name, sizeof name, "wt_prof_%012llx", (unsigned long long)(h & 0xffffffffffffull));
        benches[i].kname = name;
        std::string body = bench_source(p, id, name);
        benches[i].src = benches[i].src_single = body;
    }
    for (size_t i = 0; i < todo.size(); ++i) {
        units[i].g.nodes = {todo[i]};
        units[i].g.fp16 = false;
        // the stage's unfused kernel at the widths the cost models were
        // fitted with: one column per lane for a stage that reads a
        // pipeline input or writes an output, four otherwise
        bool user = p.is_output(todo[i]);
        for (int s : p.nodes[todo[i]].srcs)
            if (p.nodes[s].kind == Kind::Input) user = true;
        units[i].g.V = user ? 1 : 4;
        prepare_group(plan, units[i], 0);
    }
    std::vector<GroupRt*> all;
    for (auto& b : benches) all.push_back(&b);
    for (auto& u : units) all.push_back(&u);
    compile_groups(plan, all);
    if (plan.no_device) return;  // compile check only

    float* out = nullptr;
    if (hipMalloc(&out, 256) != hipSuccess) fail(WT_E_NOMEM, "profile scratch");
    OwnedStream ost(plan.setup_stream);
    hipStream_t st = ost.s;
    std::vector<StageProfile> res(todo.size());
    try {
        double base = time_kernel_ns(benches.back().fn, out, st) / kIters;
        for (size_t i = 0; i < todo.size(); ++i) {
            double t = time_kernel_ns(benches[i].fn, out, st) / kIters;
            StageProfile sp = estimate_stage(p, todo[i], plan.machine);
            sp.ns_per_point = std::max(0.05, t - base);
            int regs = 0;
            if (hipFuncGetAttribute(&regs, HIP_FUNC_ATTRIBUTE_NUM_REGS, units[i].fn) == hipSuccess && regs > 0) {
                // the unfused kernel's VGPRs less its input rings and the
                // addressing registers every wave-tile kernel holds
                int ring = 0;
                for (const NodeGeom& ng : units[i].geo.nodes)
                    if (!ng.member) ring += ng.win * ng.nch * units[i].g.V;
                sp.vgprs = std::max(2, regs - ring - 12);
            }
            sp.measured = true;
            res[i] = sp;
        }
    } catch (...) {
        hipFree(out);
        for (auto& b : benches) unload_group(b);
        for (auto& u : units) unload_group(u);
        throw;
    }
    hipFree(out);
    for (auto& b : benches) unload_group(b);
    for (auto& u : units) unload_group(u);
    std::lock_guard<std::mutex> lk(g_mu);
    for (size_t i = 0; i < todo.size(); ++i) g_prof[keys[i]] = res[i];
}

StageProfile stage_profile(const Pipeline& p, int id, int W, int H, bool measure) {
    Plan plan;
    plan.p = p;
    plan.W = W;
    plan.H = H;
    const char* env_cache = std::getenv("WT_CACHE_DIR");
    plan.cache_dir = env_cache ? env_cache : "";
    plan.no_device = !measure;
    if (measure) {
        hip_check(hipGetDevice(&plan.device), "hipGetDevice");
        plan.machine = machine_from_device(plan.device);
    }
    preprofile(plan);
    return estimate_stage(p, id, plan.machine);
}

}  // namespace wt

