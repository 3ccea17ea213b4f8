// Fusion search: which stages run fused in one kernel and with which tile
// configuration (the paper, Section 6: DP-Fusion driven by the GPU cost
// function, and the argmin over tile sizes, block sizes, register fraction
// and transaction size).
//
// The paper uses PolyMage's Bounded DP-Fusion without specifying it.  This
// search is a dynamic program over down-closed sets S of already scheduled
// stages (memoised on a bitmask): from S it may schedule any group G of
// unscheduled stages that is ready (every producer of a member is in S or G,
// which also makes G convex), connected, on one pyramid level, and of at most
// K stages; resampling stages form groups of their own.  The cost of a group
// is the time of its best configuration over the configuration grid, and the
// DP minimises the sum over groups.  With the analytical model both the
// argmin and the sum use the calibrated time: Algorithm 2's terms and the
// roofline-style predicted time, combined with coefficients refitted on
// gfx950 measurements (the paper's score alone ranks configurations but has
// no unit to sum); with the learned model, its predicted time.
#include <string>
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <functional>
#include <map>
#include <set>
#include <unordered_map>

#include "wt_cost.h"
#include "wt_mlp.h"

namespace wt {

namespace {


struct Search {
    const Pipeline& p;
    const Machine& m;
    const SchedRequest& r;
    std::vector<int> stages;           // stage node ids (non-inputs), ascending
    std::map<int, int> pos;            // node id -> bit
    std::vector<uint64_t> prod, adj;   // per bit: producer bits / undirected neighbours
    std::vector<bool> fusable;         // may be a member of a multi-stage group
    std::vector<int> flevel;           // pyramid level of the group it may join
    uint64_t resample_bits = 0;        // down2 / up2 stages
    std::map<int, StageProfile> prof;
    std::unordered_map<uint64_t, std::pair<double, GroupSched>> gcache;
    std::unordered_map<uint64_t, std::pair<double, uint64_t>> memo;
    int K;
    long long groups_costed = 0;

    Search(const Pipeline& pp, const Machine& mm, const SchedRequest& rr) : p(pp), m(mm), r(rr) {
        for (const Node& n : p.nodes)
            if (n.kind != Kind::Input) {
                pos[n.id] = (int)stages.size();
                stages.push_back(n.id);
            }
        if (stages.size() > 64) fail(WT_E_UNSUPPORTED, "fusion search handles at most 64 stages");
        prod.assign(stages.size(), 0);
        adj.assign(stages.size(), 0);
        fusable.assign(stages.size(), false);
        flevel.assign(stages.size(), 0);
        for (size_t i = 0; i < stages.size(); ++i) {
            const Node& n = p.nodes[stages[i]];
            flevel[i] = n.level;
            if (n.kind == Kind::Stencil || n.kind == Kind::Pointwise || n.kind == Kind::Equalize) {
                fusable[i] = true;
            } else if (n.kind == Kind::Down2 || n.kind == Kind::Hist) {
                // written decimated, or counted, by the group of its source
                resample_bits |= 1ull << i;
                const Node& src = p.nodes[n.srcs[0]];
                fusable[i] = src.kind == Kind::Stencil || src.kind == Kind::Pointwise;
                flevel[i] = src.level;
            } else {
                // folded into the group of the stage whose decimation it expands
                resample_bits |= 1ull << i;
                fusable[i] = r.fold && p.fold_source(n.id) >= 0;
            }
            for (int s : n.srcs)
                if (pos.count(s)) {
                    prod[i] |= 1ull << pos[s];
                    adj[i] |= 1ull << pos[s];
                    adj[pos[s]] |= 1ull << i;
                }
        }
        // stages reading the same pipeline input are neighbours too: fused,
        // they share one load of it
        for (int in : p.inputs) {
            uint64_t readers = 0;
            for (size_t i = 0; i < stages.size(); ++i)
                for (int s : p.nodes[stages[i]].srcs)
                    if (s == in) readers |= 1ull << i;
            for (size_t i = 0; i < stages.size(); ++i)
                if (readers >> i & 1) adj[i] |= readers & ~(1ull << i);
        }
        for (size_t i = 0; i < stages.size(); ++i) {
            prof[stages[i]] = estimate_stage(p, stages[i], m);
        }
        K = r.max_group > 0 ? r.max_group : 12;
    }

    // Stages of a group that count towards its size bound (a decimated
    // store is not a stage of the kernel's body).
    int group_size(uint64_t g) const {
        uint64_t down = 0;
        for (size_t i = 0; i < stages.size(); ++i)
            if ((g >> i & 1) && (p.nodes[stages[i]].kind == Kind::Down2 || p.nodes[stages[i]].kind == Kind::Hist))
                down |= 1ull << i;
        return __builtin_popcountll(g & ~down);
    }
    // A multi-stage group may hold a down2 only with its source, and an up2
    // only with the down2 it expands (hence with the stage it folds).
    bool admissible(uint64_t g) const {
        if (__builtin_popcountll(g) == 1) return true;
        bool body = false;
        for (size_t i = 0; i < stages.size(); ++i) {
            if (!(g >> i & 1)) continue;
            if (!fusable[i]) return false;
            const Node& n = p.nodes[stages[i]];
            if (n.kind == Kind::Stencil || n.kind == Kind::Pointwise || n.kind == Kind::Equalize) body = true;
            // a histogram's counts are complete only after the kernel that
            // accumulates them: no stage of that kernel may read them
            if (n.kind == Kind::Equalize) {
                auto h = pos.find(n.srcs[1]);
                if (h != pos.end() && (g >> h->second & 1)) return false;
            }
            if (n.kind == Kind::Down2 || n.kind == Kind::Up2 || n.kind == Kind::Hist) {
                auto it = pos.find(n.srcs[0]);
                if (it == pos.end() || !(g >> it->second & 1)) return false;
            }
        }
        return body;
    }

    // Best configuration of one group and its time.
    std::pair<double, GroupSched> cost_of(uint64_t g) {
        auto it = gcache.find(g);
        if (it != gcache.end()) return it->second;
        ++groups_costed;
        std::vector<int> nodes, dec, hst;
        for (size_t i = 0; i < stages.size(); ++i) {
            if (!(g >> i & 1)) continue;
            const Kind k = p.nodes[stages[i]].kind;
            const bool multi = __builtin_popcountll(g) > 1;
            (multi && k == Kind::Down2 ? dec : multi && k == Kind::Hist ? hst : nodes).push_back(stages[i]);
        }
        GroupSched base;
        base.nodes = nodes;
        base.dec = dec;
        base.hst = hst;
        base.fp16 = r.fp16;
        if (!admissible(g)) {
            auto res = std::make_pair((double)INFINITY, base);
            gcache[g] = res;
            return res;
        }
        if (nodes.size() == 1 && (resample_bits >> pos[nodes[0]] & 1)) {
            int src = p.nodes[nodes[0]].srcs[0];
            double t = resample_pred_us(p, nodes[0], m, r.W, r.H,
                                        r.fp16 && p.half_storable(src) && !p.is_output(src),
                                        r.fp16 && p.half_storable(nodes[0]) && !p.is_output(nodes[0]));
            auto res = std::make_pair(t, base);
            gcache[g] = res;
            return res;
        }
        double best_score = INFINITY, best_pred = INFINITY;
        GroupSched best = base;
        std::vector<ScoredConfig> cfgs = score_configs(p, m, r, nodes, dec);
        if (r.model && !cfgs.empty()) {
            // learned model: predicted time of every configuration; the
            // analytical prediction stands in outside the training range
            std::vector<float> feats;
            feats.reserve(cfgs.size() * kNumFeatures);
            for (const auto& sc : cfgs) {
                std::vector<double> f = group_features(p, sc.g, *sc.geo, sc.cost, r.W, r.H, sc.tx_size);
                for (double v : f) feats.push_back((float)v);
            }
            std::vector<float> pred(cfgs.size());
            r.model->predict(feats.data(), (int)cfgs.size(), pred.data());
            for (size_t i = 0; i < cfgs.size(); ++i) {
                bool inside = r.model->max_abs_z(&feats[i * kNumFeatures]) <= 4.0;
                double t = inside ? std::exp((double)pred[i]) : cfgs[i].cost.cal_us;
                if (t < best_pred) {
                    best_pred = t;
                    best = cfgs[i].g;
                }
            }
        } else {
            // the refitted analytical model: argmin of the calibrated time
            for (const ScoredConfig& sc : cfgs)
                if (sc.cost.cal_us < best_score) {
                    best_score = sc.cost.cal_us;
                    best_pred = sc.cost.cal_us;
                    best = sc.g;
                }
        }
        best.hst = hst;
        auto res = std::make_pair(best_pred, best);
        gcache[g] = res;
        return res;
    }

    // Ready, connected groups of at most K stages whose lowest stage is `seed`.
    void enumerate(uint64_t S, int seed, std::vector<uint64_t>& out) {
        uint64_t all = stages.size() == 64 ? ~0ull : ((1ull << stages.size()) - 1);
        uint64_t avail = all & ~S;
        int lvl = flevel[seed];
        std::function<void(uint64_t, uint64_t)> grow = [&](uint64_t G, uint64_t ext) {
            // G is connected; record it if ready
            bool ready = true;
            for (size_t i = 0; i < stages.size() && ready; ++i)
                if ((G >> i & 1) && (prod[i] & ~(S | G))) ready = false;
            if (ready) out.push_back(G);
            while (ext) {
                int v = __builtin_ctzll(ext);
                ext &= ext - 1;
                uint64_t ng = G | (1ull << v);
                if (group_size(ng) > K) continue;  // (a decimated store always fits)
                uint64_t next = ext;
                uint64_t nb = adj[v] & avail & ~ng & ~((1ull << seed) - 1) & ~(1ull << seed);
                for (size_t i = 0; i < stages.size(); ++i)
                    if ((nb >> i & 1) && (!fusable[i] || flevel[i] != lvl)) nb &= ~(1ull << i);
                // neighbours of v not adjacent to G before (ESU extension)
                uint64_t gadj = 0;
                for (size_t i = 0; i < stages.size(); ++i)
                    if (G >> i & 1) gadj |= adj[i];
                next |= nb & ~gadj & ~G;
                grow(ng, next);
            }
        };
        if (!fusable[seed] || (resample_bits >> seed & 1)) {
            // a resampling stage on its own (a larger group holding it has
            // a lower stage: the one it decimates or folds)
            if (!(prod[seed] & ~S)) out.push_back(1ull << seed);
            return;
        }
        uint64_t ext = adj[seed] & avail & ~((1ull << seed) - 1) & ~(1ull << seed);
        for (size_t i = 0; i < stages.size(); ++i)
            if ((ext >> i & 1) && (!fusable[i] || flevel[i] != lvl)) ext &= ~(1ull << i);
        grow(1ull << seed, ext);
    }

    double solve(uint64_t S) {
        uint64_t all = stages.size() == 64 ? ~0ull : ((1ull << stages.size()) - 1);
        if (S == all) return 0.0;
        auto it = memo.find(S);
        if (it != memo.end()) return it->second.first;
        double best = INFINITY;
        uint64_t best_g = 0;
        std::vector<uint64_t> cands;
        for (size_t v = 0; v < stages.size(); ++v)
            if (!(S >> v & 1) && !(prod[v] & ~S)) enumerate(S, (int)v, cands);
        for (uint64_t G : cands) {
            double c = cost_of(G).first;
            if (!std::isfinite(c)) continue;
            double t = c + solve(S | G);
            if (t < best) {
                best = t;
                best_g = G;
            }
        }
        memo[S] = {best, best_g};
        return best;
    }

    Schedule extract() {
        Schedule s;
        uint64_t S = 0;
        uint64_t all = stages.size() == 64 ? ~0ull : ((1ull << stages.size()) - 1);
        while (S != all) {
            uint64_t G = memo.at(S).second;
            if (!G) fail(WT_E_INTERNAL, "fusion search found no feasible schedule");
            s.groups.push_back(cost_of(G).second);
            S |= G;
        }
        return s;
    }
};

}  // namespace

// Table 3's V100 weights (Algorithm 2's score in the paper's form).
const double kGfx950Weights[7] = {50, 0.5, 60, 10, 2, 100, 1};

// Refit on gfx950 (learn.py fit-analytic: bounded least squares of log
// measured time over the measurement database's training pipelines: 4444
// timed candidate groups of 93 random pipelines, seeds 4..119 less the
// held-out fifth).  Only the normalised global-memory transactions and the
// lost occupancy keep a weight; on the 23 held-out pipelines the calibrated time
// has log-correlation 0.84 with the measurements, Kendall tau 0.58 over
// each group's candidates and a top-1 regret of 1.17 (geomean).
const AnalyticFit kGfx950Fit = {-0.34099, 0.61802, {0.30606, 1.35482, 0.0, 0.0, 0.0, 0.0, 0.0}};

const AnalyticFit& active_fit() {
    static const AnalyticFit fit = [] {
        AnalyticFit f = kGfx950Fit;
        const char* e = std::getenv("WT_ANALYTIC_FIT");
        if (!e || !*e) return f;
        double v[9];
        int n = 0;
        std::string text(e);
        size_t pos = 0;
        while (n < 9 && pos <= text.size()) {
            size_t q = text.find(',', pos);
            std::string tok = text.substr(pos, q == std::string::npos ? std::string::npos : q - pos);
            char* end = nullptr;
            v[n] = std::strtod(tok.c_str(), &end);
            if (tok.empty() || end != tok.c_str() + tok.size() || !std::isfinite(v[n])) break;
            ++n;
            if (q == std::string::npos) break;
            pos = q + 1;
        }
        if (n != 9) {
            std::fprintf(stderr, "wavetile: WT_ANALYTIC_FIT needs 9 comma-separated numbers; using the built-in fit\n");
            return f;
        }
        f.c0 = v[0];
        f.c1 = v[1];
        for (int k = 0; k < 7; ++k) f.w[k] = v[2 + k];
        return f;
    }();
    return fit;
}

std::vector<ScoredConfig> score_configs(const Pipeline& p, const Machine& m, const SchedRequest& r,
                                        const std::vector<int>& nodes, const std::vector<int>& dec) {
    std::vector<ScoredConfig> out;
    std::map<int, StageProfile> prof;
    for (int n : nodes) prof[n] = estimate_stage(p, n, m);
    GroupSched base;
    base.nodes = nodes;
    base.dec = dec;
    base.fp16 = r.fp16;
    int vmax = max_vector_width(p, base, r.W, r.H, r.any_width);
    const double* w = r.weights ? r.weights : kGfx950Weights;
    for (int V : {4, 2, 1}) {
        if (V > vmax) continue;
        for (int TX : {1, 2, 4})
            for (int SX = 0; SX <= TX; ++SX)
                for (int PF : {1, 2}) {
                    GroupSched s = base;
                    s.V = V;
                    s.TX = TX;
                    s.SX = SX;
                    s.PF = PF;
                    GroupGeom geo;
                    try {
                        geo = group_geometry(p, s);
                    } catch (const Error&) {
                        continue;
                    }
                    for (auto& ng : geo.nodes)
                        ng.mem_half = r.fp16 && p.half_storable(ng.id) && !p.is_output(ng.id) &&
                                      (!ng.member || ng.liveout);
                    auto shared = std::make_shared<const GroupGeom>(geo);
                    for (int TY : {8, 16, 32, 64})
                        for (int WPB : {1, 2, 4}) {
                            s.TY = TY;
                            s.WPB = WPB;
                            GroupGeom gg = geo;
                            gg.lds_bytes_per_wg = geo.lds_bytes * WPB;
                            for (int tx : {m.tx_sizes[0], m.tx_sizes[1]}) {
                                // the network was trained on single images: it
                                // sees single-image features
                                GroupCost c = group_cost(p, s, gg, m, r.W, r.H, prof, tx, w,
                                                         r.mode == WT_SCHED_MLP ? 1 : r.batch);
                                if (!c.alg2.feasible || c.nwaves <= 0) continue;
                                out.push_back({s, c, tx, shared});
                            }
                        }
                }
    }
    return out;
}

Schedule schedule_analytic(const Pipeline& p, const Machine& m, const SchedRequest& r) {
    Search srch(p, m, r);
    auto t0 = std::chrono::steady_clock::now();
    double t = srch.solve(0);
    if (std::getenv("WT_DEBUG_SEARCH"))
        fprintf(stderr, "search: %zu stages, %lld groups costed, %zu states, %.3f s\n", srch.stages.size(),
                srch.groups_costed, srch.memo.size(),
                std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
    if (!std::isfinite(t)) fail(WT_E_UNSUPPORTED, "no feasible schedule for this pipeline");
    return srch.extract();
}

// Minimum total predicted time by the DP and by exhaustive enumeration of all
// partitions into ready groups under the same group costs (test hook; the
// exhaustive search is exponential and refuses more than 10 stages).
void fusion_costs(const Pipeline& p, const Machine& m, const SchedRequest& r, double* dp, double* brute) {
    Search srch(p, m, r);
    *dp = srch.solve(0);
    *brute = INFINITY;
    size_t n = srch.stages.size();
    if (n > 10) return;
    // assign each stage a group label (restricted growth strings), then test
    // that the group graph is acyclic and every group is fusable/connected
    std::vector<int> lab(n, 0);
    std::function<void(size_t, int)> rec = [&](size_t i, int k) {
        if (i == n) {
            std::vector<uint64_t> gs(k, 0);
            for (size_t j = 0; j < n; ++j) gs[lab[j]] |= 1ull << j;
            double tot = 0;
            // order groups: repeatedly pick a ready group
            uint64_t S = 0;
            std::vector<bool> used(k, false);
            for (int step = 0; step < k; ++step) {
                int pick = -1;
                for (int g = 0; g < k && pick < 0; ++g) {
                    if (used[g]) continue;
                    bool ready = true;
                    for (size_t j = 0; j < n; ++j)
                        if ((gs[g] >> j & 1) && (srch.prod[j] & ~(S | gs[g]))) ready = false;
                    if (ready) pick = g;
                }
                if (pick < 0) return;  // cyclic group graph
                used[pick] = true;
                S |= gs[pick];
                // group admissibility as in the DP
                uint64_t G = gs[pick];
                int cnt = __builtin_popcountll(G);
                if (srch.group_size(G) > srch.K) return;
                if (!srch.admissible(G)) return;
                int lvl = -1;
                for (size_t j = 0; j < n; ++j)
                    if (G >> j & 1) {
                        if (cnt > 1 && !srch.fusable[j]) return;
                        int l = cnt > 1 ? srch.flevel[j] : p.nodes[srch.stages[j]].level;
                        if (lvl >= 0 && l != lvl) return;
                        lvl = l;
                    }
                // connected
                uint64_t seen = G & (~G + 1), frontier = seen;
                while (frontier) {
                    uint64_t nf = 0;
                    for (size_t j = 0; j < n; ++j)
                        if (frontier >> j & 1) nf |= srch.adj[j] & G & ~seen;
                    seen |= nf;
                    frontier = nf;
                }
                if (seen != G) return;
                double c = srch.cost_of(G).first;
                if (!std::isfinite(c)) return;
                tot += c;
            }
            *brute = std::min(*brute, tot);
            return;
        }
        for (int l = 0; l <= k; ++l) {
            lab[i] = l;
            rec(i + 1, std::max(k, l + 1));
        }
    };
    rec(0, 0);
}

}  // namespace wt
