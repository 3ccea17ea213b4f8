// Autotuner: measures candidate configurations of every fused group on the
// device and keeps the fastest (the project's replacement for PolyMage's
// measured autotuner, restricted to the candidates the models rank best).
//
// Candidates per group: the top-k by predicted time, the top-k by
// Algorithm 2's score, a few gfx950 defaults, and the current choice.  Each
// is compiled (in parallel, through the code cache) and timed with the
// paper's protocol: 3 samples of R back-to-back launches, minimum of the
// sample means.  Every measurement is appended to the measurement database
// ($WT_MEASURE_DB, JSON lines) with the configuration's 40 model features;
// the database trains the learned cost model and refits Algorithm 2's
// weights.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <set>
#include <sstream>

#include "wt_cost.h"
#include "wt_runtime.h"

namespace wt {

namespace {

struct DeviceScratch {
    std::vector<void*> ptrs;
    ~DeviceScratch() {
        for (void* p : ptrs) hipFree(p);
    }
    void* alloc(size_t bytes) {
        void* p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess) fail(WT_E_NOMEM, "autotune scratch");
        ptrs.push_back(p);
        hip_check(hipMemset(p, 0, std::max<size_t>(bytes, 256)), "hipMemset");
        return p;
    }
};

std::string json_escape(const std::string& s) {
    std::string o;
    for (char c : s) {
        if (c == '"' || c == '\\') o += '\\';
        o += c;
    }
    return o;
}

}  // namespace

// Measured time (microseconds) of one launch of `gr`: 3 samples of `reps`
// launches, minimum of the sample means.
double time_group_us(const Plan& plan, const GroupRt& gr, const std::map<int, ImgRef>& mem, hipStream_t st,
                     int reps) {
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "hipEventCreate");
    hip_check(hipEventCreate(&e1), "hipEventCreate");
    for (int i = 0; i < 3; ++i) launch_group(plan, gr, mem, st);
    double best = INFINITY;
    for (int s = 0; s < 3; ++s) {
        hip_check(hipEventRecord(e0, st), "hipEventRecord");
        for (int i = 0; i < reps; ++i) launch_group(plan, gr, mem, st);
        hip_check(hipEventRecord(e1, st), "hipEventRecord");
        hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
        float ms = 0;
        hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        best = std::min(best, (double)ms * 1e3 / reps);
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return best;
}

std::map<int, ImgRef> scratch_memory(const Plan& plan, DeviceScratch& sc) {
    const Pipeline& p = plan.p;
    std::map<int, ImgRef> mem;
    for (int id : p.inputs) {
        size_t n = (size_t)plan.W * plan.H * p.nodes[id].channels;
        mem[id] = {sc.alloc(n * 4), plan.W, (int64_t)plan.W * plan.H};
    }
    for (int id : p.outputs) {
        auto d = level_dims(plan.W, plan.H, p.nodes[id].level);
        int64_t rs = (d.first + 63) / 64 * 64;
        mem[id] = {sc.alloc((size_t)rs * d.second * p.nodes[id].channels * 4), rs, rs * d.second};
    }
    for (auto& kv : plan.bufs) mem[kv.first] = {kv.second.ptr, kv.second.rs, kv.second.cs};
    return mem;
}

void autotune_plan(Plan& plan, int topk) {
    const Pipeline& p = plan.p;
    DeviceScratch sc;
    std::map<int, ImgRef> mem = scratch_memory(plan, sc);
    hipStream_t st;
    hip_check(hipStreamCreate(&st), "hipStreamCreate");
    const char* dbp = std::getenv("WT_MEASURE_DB");
    std::ofstream db;
    if (dbp && *dbp) db.open(dbp, std::ios::app);
    SchedRequest req;
    req.W = plan.W;
    req.H = plan.H;
    req.fp16 = plan.fp16;
    req.any_width = plan.any_width;
    uint64_t phash = 1469598103934665603ull;
    for (auto& g : plan.groups)
        for (unsigned char c : g.kname) phash = (phash ^ c) * 1099511628211ull;

    for (size_t gi = 0; gi < plan.sched.groups.size(); ++gi) {
        if (plan.groups[gi].resample) continue;
        const GroupSched cur = plan.sched.groups[gi];
        std::vector<ScoredConfig> all = score_configs(p, plan.machine, req, cur.nodes);
        std::vector<const ScoredConfig*> by_pred, by_score;
        for (auto& c : all) {
            by_pred.push_back(&c);
            by_score.push_back(&c);
        }
        std::sort(by_pred.begin(), by_pred.end(), [](auto a, auto b) { return a->cost.pred_us < b->cost.pred_us; });
        std::sort(by_score.begin(), by_score.end(),
                  [](auto a, auto b) { return a->cost.alg2.score < b->cost.alg2.score; });
        std::vector<GroupSched> cands;
        std::set<std::string> seen;
        auto add = [&](const GroupSched& g) {
            if (seen.insert(describe_group(g)).second) cands.push_back(g);
        };
        add(cur);
        for (int i = 0; i < topk && i < (int)by_pred.size(); ++i) add(by_pred[i]->g);
        for (int i = 0; i < topk && i < (int)by_score.size(); ++i) add(by_score[i]->g);
        int vmax = max_vector_width(p, cur, plan.W, plan.H, plan.any_width);
        for (int V : {4, 2})
            for (int TX : {1, 2})
                for (int TY : {16, 32}) {
                    if (V > vmax) continue;
                    GroupSched g = cur;
                    g.V = V;
                    g.TX = TX;
                    g.SX = 0;
                    g.TY = TY;
                    g.PF = 2;
                    g.WPB = 1;
                    add(g);
                }
        std::vector<GroupRt> trials;
        for (auto& g : cands) {
            GroupRt gr;
            gr.g = g;
            try {
                prepare_group(plan, gr, (int)gi);
            } catch (const Error&) {
                continue;
            }
            trials.push_back(std::move(gr));
        }
        std::vector<GroupRt*> ptrs;
        for (auto& t : trials) ptrs.push_back(&t);
        compile_groups(plan, ptrs);
        double best_t = INFINITY;
        GroupSched best = cur;
        for (auto& t : trials) {
            double us = time_group_us(plan, t, mem, st, 20);
            if (us < best_t) {
                best_t = us;
                best = t.g;
            }
            if (db.is_open()) {
                // model quantities of the measured configuration
                GroupCost c;
                int txs = 128;
                for (const auto& s : all)
                    if (describe_group(s.g) == describe_group(t.g)) {
                        c = s.cost;
                        txs = s.tx_size;
                        break;
                    }
                std::vector<double> f = group_features(p, t.g, t.geo, c, plan.W, plan.H, txs);
                std::ostringstream os;
                os.precision(9);
                char h[32];
                std::snprintf(h, sizeof h, "%016llx", (unsigned long long)phash);
                os << "{\"pipeline\": \"" << h << "\", \"W\": " << plan.W << ", \"H\": " << plan.H
                   << ", \"group\": \"" << json_escape(describe_group(t.g)) << "\", \"measured_us\": " << us
                   << ", \"pred_us\": " << c.pred_us << ", \"score\": " << c.alg2.score << ", \"terms\": [";
                for (int i = 0; i < 7; ++i) os << (i ? ", " : "") << c.alg2.terms[i];
                os << "], \"features\": [";
                for (size_t i = 0; i < f.size(); ++i) os << (i ? ", " : "") << f[i];
                os << "]}\n";
                db << os.str();
            }
        }
        for (auto& t : trials)
            if (t.mod) {
                hipModuleUnload(t.mod);
                t.mod = nullptr;
            }
        plan.sched.groups[gi] = best;
    }
    hipStreamDestroy(st);
    build_groups(plan);
}

}  // namespace wt
