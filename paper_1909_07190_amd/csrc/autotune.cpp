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
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <set>
#include <sstream>

#include "wt_cost.h"
#include "wt_mlp.h"
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

// Analytical quantities of one configuration as the scheduler sees them
// (the transaction size with the better Algorithm 2 score).
ScoredConfig score_one(const Pipeline& p, const Machine& m, const GroupSched& g, const GroupGeom& geo, int W,
                       int H) {
    std::map<int, StageProfile> prof;
    for (int n : g.nodes) prof[n] = estimate_stage(p, n, m);
    ScoredConfig best;
    best.g = g;
    bool have = false;
    for (int tx : {m.tx_sizes[0], m.tx_sizes[1]}) {
        GroupCost c = group_cost(p, g, geo, m, W, H, prof, tx, kGfx950Weights);
        if (!have || c.alg2.score < best.cost.alg2.score) {
            best.cost = c;
            best.tx_size = tx;
            have = true;
        }
    }
    return best;
}

// One measurement database line: the configuration, its measured and
// predicted time, Algorithm 2's terms and the 40 model features.
void write_db_line(std::ofstream& db, const std::string& tag, const Plan& plan, const GroupRt& gr, double us) {
    ScoredConfig sc = score_one(plan.p, plan.machine, gr.g, gr.geo, plan.W, plan.H);
    std::vector<double> f = group_features(plan.p, gr.g, gr.geo, sc.cost, plan.W, plan.H, sc.tx_size);
    std::ostringstream os;
    os.precision(9);
    // JSON has no infinity: non-finite model quantities are written as null
    auto num = [](double v) {
        std::ostringstream t;
        t.precision(9);
        if (std::isfinite(v)) t << v;
        else t << "null";
        return t.str();
    };
    os << "{\"pipeline\": \"" << json_escape(tag) << "\", \"W\": " << plan.W << ", \"H\": " << plan.H
       << ", \"group\": \"" << json_escape(describe_group(gr.g)) << "\", \"measured_us\": " << num(us)
       << ", \"pred_us\": " << num(sc.cost.pred_us) << ", \"score\": " << num(sc.cost.alg2.score)
       << ", \"terms\": [";
    for (int i = 0; i < 7; ++i) os << (i ? ", " : "") << num(sc.cost.alg2.terms[i]);
    os << "], \"features\": [";
    for (size_t i = 0; i < f.size(); ++i) os << (i ? ", " : "") << num(f[i]);
    os << "]}\n";
    db << os.str();
    db.flush();
}

}  // namespace

// Measured time (microseconds) of one launch of `gr`: 3 samples of `reps`
// launches, minimum of the sample means.  Consecutive launches use the
// memory sets in turn, so with sets spanning more than the last-level cache
// every launch reads its inputs from HBM, as a pipeline run on fresh images
// does.
double time_group_us(const Plan& plan, const GroupRt& gr, const std::vector<std::map<int, ImgRef>>& sets,
                     hipStream_t st, int reps) {
    OwnedEvents ev;
    hipEvent_t e0 = ev.e0, e1 = ev.e1;
    const size_t n = sets.size();
    size_t next = 0;
    for (int i = 0; i < 3; ++i) launch_group(plan, gr, sets[next++ % n], st);
    double best = INFINITY;
    for (int s = 0; s < 3; ++s) {
        hip_check(hipEventRecord(e0, st), "hipEventRecord");
        for (int i = 0; i < reps; ++i) launch_group(plan, gr, sets[next++ % n], st);
        hip_check(hipEventRecord(e1, st), "hipEventRecord");
        hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
        float ms = 0;
        hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        best = std::min(best, (double)ms * 1e3 / reps);
    }
    return best;
}

double time_group_us(const Plan& plan, const GroupRt& gr, const std::map<int, ImgRef>& mem, hipStream_t st,
                     int reps) {
    return time_group_us(plan, gr, std::vector<std::map<int, ImgRef>>{mem}, st, reps);
}

std::map<int, ImgRef> scratch_memory(const Plan& plan, DeviceScratch& sc) {
    const Pipeline& p = plan.p;
    std::map<int, ImgRef> mem;
    for (int id : p.inputs) {
        size_t n = (size_t)plan.W * plan.H * p.nodes[id].channels;
        mem[id] = {sc.alloc(n * 4), plan.W, (int64_t)plan.W * plan.H};
    }
    for (int id : p.outputs) {
        auto d = node_dims(p, id, plan.W, plan.H);
        int64_t rs = (d.first + 63) / 64 * 64;
        mem[id] = {sc.alloc((size_t)rs * d.second * p.nodes[id].channels * 4), rs, rs * d.second};
    }
    for (auto& kv : plan.bufs) mem[kv.first] = {kv.second.ptr, kv.second.rs, kv.second.cs};
    return mem;
}

// Copies of every buffer of a plan (its inputs, outputs and materialised
// intermediates, the first copy being scratch_memory's) until the copies
// hold at least 1 GiB (at most 8), more than the MI355X's 256 MB Infinity
// Cache.
std::vector<std::map<int, ImgRef>> scratch_sets(const Plan& plan, DeviceScratch& sc) {
    const Pipeline& p = plan.p;
    std::vector<std::map<int, ImgRef>> sets{scratch_memory(plan, sc)};
    size_t bytes = 0;
    for (auto& kv : sets[0]) bytes += (size_t)kv.second.cs * p.nodes[kv.first].channels * 4;
    const size_t want = (size_t)1 << 30;
    const int n = (int)std::min<size_t>(8, std::max<size_t>(1, (want + std::max<size_t>(bytes, 1) - 1) / std::max<size_t>(bytes, 1)));
    for (int c = 1; c < n; ++c) {
        std::map<int, ImgRef> m;
        for (auto& kv : sets[0]) {
            const ImgRef& r = kv.second;
            m[kv.first] = {sc.alloc((size_t)r.cs * p.nodes[kv.first].channels * 4), r.rs, r.cs};
        }
        sets.push_back(std::move(m));
    }
    return sets;
}

namespace {

// Buffers a group reads and writes, each at its level's size for a W x H
// image: (node id, bytes of one plane, channels).
std::vector<std::array<int64_t, 3>> group_planes(const Plan& plan, const GroupRt& gr, int W, int H) {
    std::vector<std::array<int64_t, 3>> out;
    std::set<int> seen;
    auto add = [&](int id) {
        if (!seen.insert(id).second) return;
        auto d = node_dims(plan.p, id, W, H);
        int64_t rs = (d.first + 63) / 64 * 64;
        out.push_back({id, rs * d.second * 4, plan.p.nodes[id].channels});
    };
    for (int id : gr.loaded) add(id);
    for (int id : gr.liveouts) add(id);
    return out;
}

// How many images' worth of rows a batched plan's candidates are timed on:
// up to the batch size, with the group's buffers within 4 GiB and every
// plane under 1 GiB.
int stack_count(const Plan& plan, const GroupRt& gr, int batch) {
    if (batch <= 1) return 1;
    int64_t total = 0, plane = 1;
    for (auto& b : group_planes(plan, gr, plan.W, plan.H)) {
        total += b[1] * b[2];
        plane = std::max(plane, b[1]);
    }
    int64_t k = std::min<int64_t>(batch, std::max<int64_t>(1, (int64_t(4) << 30) / std::max<int64_t>(1, total)));
    k = std::min<int64_t>(k, std::max<int64_t>(1, (int64_t(1) << 30) / plane));
    k = std::min<int64_t>(k, std::max(1, (1 << 24) / std::max(1, plan.H)));
    return (int)std::max<int64_t>(1, k);
}

// Sets a plan's height for the lifetime of the guard.
struct PlanHeight {
    Plan& plan;
    int saved;
    PlanHeight(Plan& p, int h) : plan(p), saved(p.H) { plan.H = h; }
    ~PlanHeight() { plan.H = saved; }
};

}  // namespace

// One step from `best` along one configuration axis: V, TX, TY, WPB and PF
// halved or doubled within their ranges, or V and TX traded at one tile
// width.
std::vector<GroupSched> config_neighbours(const GroupSched& best, int vmax) {
    std::vector<GroupSched> nb;
    auto step = [&](int GroupSched::*f, int v, int lo, int hi) {
        if (v < lo || v > hi) return;
        GroupSched g = best;
        g.*f = v;
        if (g.SX > g.TX) g.SX = g.TX;
        nb.push_back(g);
    };
    step(&GroupSched::V, best.V * 2, 1, vmax);
    step(&GroupSched::V, best.V / 2, 1, vmax);
    step(&GroupSched::TX, best.TX * 2, 1, 4);
    step(&GroupSched::TX, best.TX / 2, 1, 4);
    step(&GroupSched::TY, best.TY * 2, 8, 64);
    step(&GroupSched::TY, best.TY / 2, 8, 64);
    step(&GroupSched::WPB, best.WPB * 2, 1, 4);
    step(&GroupSched::WPB, best.WPB / 2, 1, 4);
    step(&GroupSched::PF, best.PF * 2, 1, 4);
    step(&GroupSched::PF, best.PF / 2, 1, 4);
    for (int f : {2, -2}) {
        GroupSched g = best;
        g.V = f > 0 ? best.V * 2 : best.V / 2;
        g.TX = f > 0 ? best.TX / 2 : best.TX * 2;
        if (g.V < 1 || g.V > vmax || g.TX < 1 || g.TX > 4 || (f > 0 ? best.TX % 2 : best.V % 2)) continue;
        g.SX = std::min(g.SX, g.TX);
        nb.push_back(g);
    }
    return nb;
}

namespace {

// What a group computes, independent of which nodes it computes it for: each
// member's stage (kind, channels, level, type and parameters) with its
// sources as members (by position) or as outside nodes (their kind, level
// and channels), and its decimated, expanded and counted stages likewise.
// Two groups with one signature run the same kernel on different images.
std::string group_signature(const Pipeline& p, const GroupSched& g) {
    std::map<int, int> pos;
    for (size_t i = 0; i < g.nodes.size(); ++i) pos[g.nodes[i]] = (int)i;
    std::ostringstream os;
    os.precision(17);
    auto stage = [&](int id) {
        const Node& n = p.nodes[id];
        os << (int)n.kind << ':' << n.channels << ':' << n.level << ':' << n.dtype << ':' << n.kw << 'x' << n.kh << ':'
           << n.ax << ',' << n.ay << ':' << n.scale << ':' << n.divisor << ':' << n.bins << ':' << n.hlo << ':' << n.hhi
           << ':' << n.expr_text << '[';
        for (double w : n.weights) os << w << ',';
        for (long long w : n.iweights) os << w << ',';
        os << "](";
        for (int s : n.srcs) {
            auto it = pos.find(s);
            if (it != pos.end()) os << 'm' << it->second << ',';
            else os << 'x' << (int)p.nodes[s].kind << '.' << p.nodes[s].level << '.' << p.nodes[s].channels << ',';
        }
        os << ')';
    };
    for (int m : g.nodes) stage(m);
    for (const auto* list : {&g.dec, &g.exp, &g.hst}) {
        os << '|';
        for (int d : *list) stage(d);
    }
    return os.str();
}

void copy_config(const GroupSched& from, GroupSched& to) {
    to.V = from.V;
    to.TX = from.TX;
    to.SX = from.SX;
    to.TY = from.TY;
    to.WPB = from.WPB;
    to.PF = from.PF;
    to.XCD = from.XCD;
    to.ORD = from.ORD;
    to.NT = from.NT;
    to.align = from.align;
    to.fp16 = from.fp16;
    to.BLK = from.BLK;
    to.GH = from.GH;
}

}  // namespace

double autotune_plan(Plan& plan, int topk, const std::string& model_path, int batch, TuneMemo* memo) {
    const Pipeline& p = plan.p;
    DeviceScratch sc;
    std::vector<std::map<int, ImgRef>> sets = scratch_sets(plan, sc);
    OwnedStream ost(plan.setup_stream);
    hipStream_t st = ost.s;
    const char* dbp = std::getenv("WT_MEASURE_DB");
    std::ofstream db;
    if (dbp && *dbp) db.open(dbp, std::ios::app);
    std::unique_ptr<Mlp> model;
    if (!model_path.empty()) model = Mlp::load(model_path);
    SchedRequest req;
    req.W = plan.W;
    req.H = plan.H;
    req.fp16 = plan.fp16;
    req.any_width = plan.any_width;
    // the network was trained on single images; the analytical ranking takes
    // the batch size
    req.batch = model ? 1 : std::max(1, batch);
    uint64_t phash = 1469598103934665603ull;
    for (auto& g : plan.groups)
        for (unsigned char c : g.kname) phash = (phash ^ c) * 1099511628211ull;
    char hbuf[32];
    std::snprintf(hbuf, sizeof hbuf, "%016llx", (unsigned long long)phash);
    const std::string tag = hbuf;

    double total_us = 0;  // the chosen configurations' times per image
    const size_t G = plan.sched.groups.size();
    std::vector<double> gtime(G, -1.0);  // each tuned group's time per image
    std::vector<std::string> gkey(G);
    for (size_t gi = 0; gi < G; ++gi) {
        if (plan.groups[gi].resample) {
            total_us += time_group_us(plan, plan.groups[gi], sets, st, 20);
            continue;
        }
        const GroupSched cur = plan.sched.groups[gi];
        // a group tuned before (for another grouping of the same plan)
        std::ostringstream key;
        for (int v : cur.nodes) key << v << ',';
        key << '|';
        for (int v : cur.dec) key << v << ',';
        key << '|';
        for (int v : cur.exp) key << v << ',';
        key << '|';
        for (int v : cur.hst) key << v << ',';
        gkey[gi] = key.str();
        if (memo) {
            auto hit = memo->find(key.str());
            if (hit != memo->end()) {
                plan.sched.groups[gi] = hit->second.first;
                total_us += hit->second.second;
                gtime[gi] = hit->second.second;
                continue;
            }
        }
        std::vector<ScoredConfig> all = score_configs(p, plan.machine, req, cur.nodes, cur.dec);
        std::vector<const ScoredConfig*> by_pred, by_score;
        for (auto& c : all) {
            by_pred.push_back(&c);
            by_score.push_back(&c);
        }
        if (model) {
            // rank by the learned model (analytical time outside its range)
            std::vector<float> feats;
            for (auto& c : all) {
                std::vector<double> f = group_features(p, c.g, *c.geo, c.cost, plan.W, plan.H, c.tx_size);
                for (double v : f) feats.push_back((float)v);
            }
            std::vector<float> pred(all.size());
            if (!all.empty()) model->predict(feats.data(), (int)all.size(), pred.data());
            std::vector<double> t(all.size());
            for (size_t i = 0; i < all.size(); ++i)
                t[i] = model->max_abs_z(&feats[i * kNumFeatures]) <= 4.0 ? std::exp((double)pred[i]) : all[i].cost.cal_us;
            std::vector<size_t> idx(all.size());
            for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
            std::sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return t[a] < t[b]; });
            by_pred.clear();
            for (size_t i : idx) by_pred.push_back(&all[i]);
        } else {
            std::sort(by_pred.begin(), by_pred.end(),
                      [](auto a, auto b) { return a->cost.cal_us < b->cost.cal_us; });
        }
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
        for (int V : {4, 2, 1})
            for (int TX : {1, 2})
                for (int TY : {16, 32, 64}) {
                    // the widest vector only; 64-row tiles only for batches
                    if (V != vmax || (TY == 64 && batch <= 1)) continue;
                    GroupSched g = cur;
                    g.V = V;
                    g.TX = TX;
                    g.SX = 0;
                    g.TY = TY;
                    g.PF = 2;
                    g.WPB = 1;
                    add(g);
                }
        // A batched plan runs each group over the tiles of every image at
        // once; one image of the planning size gives too few waves to rank
        // tall tiles as they run there, so its candidates are timed on an
        // image as tall as several of them.
        const int k = stack_count(plan, plan.groups[gi], batch);
        PlanHeight tall(plan, plan.H * k);
        DeviceScratch tall_scratch;
        std::map<int, ImgRef> tall_mem;
        std::vector<GroupRt> trials;
        for (auto& g : cands) {
            GroupRt gr;
            gr.g = g;
            gr.g.dec = cur.dec;  // decimated outputs and expanded inputs stay with the group
            gr.g.exp = cur.exp;
            gr.g.hst = cur.hst;
            try {
                prepare_group(plan, gr, (int)gi);
            } catch (const Error&) {
                continue;
            }
            trials.push_back(std::move(gr));
        }
        std::vector<GroupRt*> ptrs;
        for (auto& t : trials) ptrs.push_back(&t);
        std::vector<bool> bad;
        compile_groups(plan, ptrs, false, &bad);  // a candidate that does not compile is dropped
        {
            std::vector<GroupRt> kept;
            for (size_t i = 0; i < trials.size(); ++i)
                if (!bad[i]) kept.push_back(std::move(trials[i]));
            trials = std::move(kept);
        }
        if (k > 1)
            for (auto& t : trials)
                for (auto& b : group_planes(plan, t, plan.W, plan.H)) {
                    if (tall_mem.count((int)b[0])) continue;
                    auto d = node_dims(p, (int)b[0], plan.W, plan.H);
                    int64_t rs = (d.first + 63) / 64 * 64;
                    tall_mem[(int)b[0]] = {tall_scratch.alloc((size_t)b[1] * b[2]), rs, rs * d.second};
                }
        double best_t = INFINITY;
        GroupSched best = cur;
        const int reps = std::max(5, 20 / k);  // tall images: fewer, longer launches
        for (auto& t : trials) {
            double us = k > 1 ? time_group_us(plan, t, tall_mem, st, reps) : time_group_us(plan, t, sets, st, reps);
            if (us < best_t) {
                best_t = us;
                best = t.g;
            }
            if (db.is_open()) write_db_line(db, tag, plan, t, us);
        }
        for (auto& t : trials) unload_group(t);
        // Local search around the winner: one configuration parameter at a
        // time (vector width, sub-tiles, tile height, waves per workgroup,
        // prefetch depth up to 4 rows), or vector width and sub-tiles
        // together at the same tile width, while a step still helps.  The grid above samples
        // each axis coarsely; the optimum often sits one step from its best.
        for (int round = 0; round < 2 && std::isfinite(best_t); ++round) {
            std::vector<GroupSched> nb;
            for (const GroupSched& g : config_neighbours(best, vmax))
                if (seen.insert(describe_group(g)).second) nb.push_back(g);
            std::vector<GroupRt> more;
            for (auto& g : nb) {
                GroupRt gr;
                gr.g = g;
                gr.g.dec = cur.dec;
                gr.g.exp = cur.exp;
                gr.g.hst = cur.hst;
                try {
                    prepare_group(plan, gr, (int)gi);
                } catch (const Error&) {
                    continue;
                }
                more.push_back(std::move(gr));
            }
            if (more.empty()) break;
            std::vector<GroupRt*> mp;
            for (auto& t : more) mp.push_back(&t);
            std::vector<bool> bad;
            compile_groups(plan, mp, false, &bad);
            {
                std::vector<GroupRt> kept;
                for (size_t i = 0; i < more.size(); ++i)
                    if (!bad[i]) kept.push_back(std::move(more[i]));
                more = std::move(kept);
            }
            if (more.empty()) break;
            if (k > 1)
                for (auto& t : more)
                    for (auto& b : group_planes(plan, t, plan.W, plan.H)) {
                        if (tall_mem.count((int)b[0])) continue;
                        auto d = node_dims(p, (int)b[0], plan.W, plan.H);
                        int64_t rs = (d.first + 63) / 64 * 64;
                        tall_mem[(int)b[0]] = {tall_scratch.alloc((size_t)b[1] * b[2]), rs, rs * d.second};
                    }
            bool improved = false;
            for (auto& t : more) {
                double us = k > 1 ? time_group_us(plan, t, tall_mem, st, reps) : time_group_us(plan, t, sets, st, reps);
                if (db.is_open()) write_db_line(db, tag, plan, t, us);
                if (us < best_t) {
                    best_t = us;
                    best = t.g;
                    improved = true;
                }
            }
            for (auto& t : more) unload_group(t);
            if (!improved) break;
        }
        plan.sched.groups[gi] = best;
        total_us += best_t / k;
        gtime[gi] = best_t / k;
        if (memo) (*memo)[key.str()] = {best, best_t / k};
        if (verbose())
            std::fprintf(stderr, "wavetile autotune: group %zu of %zu, %zu candidates, best %.1f us on %d image(s): %s\n",
                         gi + 1, plan.sched.groups.size(), trials.size(), best_t, k, describe_group(best).c_str());
    }
    // Groups that compute the same stages on different images (a pyramid's
    // blurs of each input) are tuned one by one, each from its own
    // candidates; every one of them takes the fastest configuration any of
    // them found.
    std::map<std::string, size_t> fastest;
    std::vector<std::string> sig(G);
    for (size_t gi = 0; gi < G; ++gi) {
        if (gtime[gi] < 0) continue;
        sig[gi] = group_signature(p, plan.sched.groups[gi]);
        auto it = fastest.find(sig[gi]);
        if (it == fastest.end() || gtime[gi] < gtime[it->second]) fastest[sig[gi]] = gi;
    }
    for (size_t gi = 0; gi < G; ++gi) {
        if (gtime[gi] < 0) continue;
        const size_t j = fastest[sig[gi]];
        if (j == gi) continue;
        copy_config(plan.sched.groups[j], plan.sched.groups[gi]);
        total_us += gtime[j] - gtime[gi];
        if (memo) (*memo)[gkey[gi]] = {plan.sched.groups[gi], gtime[j]};
        if (verbose())
            std::fprintf(stderr, "wavetile autotune: group %zu of %zu takes group %zu's configuration (%.1f against %.1f us per image)\n",
                         gi + 1, G, j + 1, gtime[j], gtime[gi]);
    }
    build_groups(plan);
    return total_us;
}

// Times arbitrary candidate groups of a pipeline on scratch images (every
// node's image allocated at its level's size, zero-filled), for building the
// measurement database.  Groups that cannot be built get +inf.
void measure_groups(const Pipeline& p, int W, int H, bool fp16, const std::vector<std::string>& descs, int reps,
                    const std::string& tag, double* out_us) {
    Plan plan;
    plan.p = p;
    plan.W = W;
    plan.H = H;
    plan.fp16 = fp16;
    const char* env_cache = std::getenv("WT_CACHE_DIR");
    plan.cache_dir = env_cache ? env_cache : "";
    plan.no_device = reps == 0;  // compile only (fills the code cache)
    if (!plan.no_device) {
        hip_check(hipGetDevice(&plan.device), "hipGetDevice");
        plan.machine = machine_from_device(plan.device);
    }
    std::vector<GroupRt> trials(descs.size());
    std::vector<GroupRt*> ok;
    std::vector<size_t> idx;
    for (size_t i = 0; i < descs.size(); ++i) {
        out_us[i] = INFINITY;
        try {
            Schedule sc = parse_schedule(descs[i], p, true);
            if (sc.groups.size() != 1) fail(WT_E_INVALID, "one group per entry");
            trials[i].g = sc.groups[0];
            trials[i].g.fp16 = fp16;
            prepare_group(plan, trials[i], 0);
        } catch (const Error&) {
            continue;
        }
        ok.push_back(&trials[i]);
        idx.push_back(i);
    }
    std::vector<bool> bad;
    compile_groups(plan, ok, false, &bad);
    {
        std::vector<GroupRt*> okc;
        std::vector<size_t> idxc;
        for (size_t j = 0; j < ok.size(); ++j)
            if (!bad[j]) {
                okc.push_back(ok[j]);
                idxc.push_back(idx[j]);
            }
        ok = std::move(okc);
        idx = std::move(idxc);
    }
    if (!plan.no_device && preprofile_enabled()) preprofile(plan);
    if (plan.no_device) {
        for (size_t i : idx) out_us[i] = 0.0;
        return;
    }
    DeviceScratch scr;
    std::vector<std::map<int, ImgRef>> mem(1);
    size_t bytes = 0;
    for (const Node& n : p.nodes) {
        auto d = node_dims(p, n.id, W, H);
        int64_t rs = (d.first + 63) / 64 * 64;
        mem[0][n.id] = {scr.alloc((size_t)rs * d.second * n.channels * 4), rs, rs * d.second};
        bytes += (size_t)rs * d.second * n.channels * 4;
    }
    // copies spanning more than the last-level cache (see scratch_sets)
    const int nsets = (int)std::min<size_t>(8, std::max<size_t>(1, (((size_t)1 << 30) + bytes - 1) / std::max<size_t>(bytes, 1)));
    for (int c = 1; c < nsets; ++c) {
        std::map<int, ImgRef> m;
        for (auto& kv : mem[0])
            m[kv.first] = {scr.alloc((size_t)kv.second.cs * p.nodes[kv.first].channels * 4), kv.second.rs, kv.second.cs};
        mem.push_back(std::move(m));
    }
    OwnedStream ost;
    const char* dbp = std::getenv("WT_MEASURE_DB");
    std::ofstream db;
    if (dbp && *dbp) db.open(dbp, std::ios::app);
    try {
        for (size_t k = 0; k < ok.size(); ++k) {
            double us = time_group_us(plan, *ok[k], mem, ost.s, reps);
            out_us[idx[k]] = us;
            if (db.is_open() && !ok[k]->resample) write_db_line(db, tag, plan, *ok[k], us);
        }
    } catch (...) {
        for (auto* t : ok) unload_group(*t);
        throw;
    }
    for (auto* t : ok) unload_group(*t);
}

}  // namespace wt
