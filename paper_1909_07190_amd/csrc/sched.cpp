// Schedules: which stages are fused and with which tile configuration.
#include <algorithm>
#include <set>

#include "wt_internal.h"
#include "wt_mlp.h"

namespace wt {

// One kernel per stage; every intermediate round-trips through HBM.
Schedule schedule_unfused(const Pipeline& p, bool fp16) {
    Schedule s;
    for (const Node& n : p.nodes) {
        if (n.kind == Kind::Input) continue;
        GroupSched g;
        g.nodes = {n.id};
        g.V = 4;
        g.TX = 1;
        g.SX = 0;
        g.TY = 16;
        g.WPB = 1;
        g.fp16 = fp16;
        s.groups.push_back(g);
    }
    return s;
}

Schedule schedule_analytic(const Pipeline& p, const Machine& m, const SchedRequest& r);

// Largest vector width a group may use.  Loads and stores of 32-bit
// elements need only 4-byte alignment, so rows of any width and stride take
// any V; groups that read or write the caller's images of narrower integer
// elements address its dense rows in vectors of V elements aligned to V, so
// V must divide that level's width (intermediate buffers are padded by the
// library).
int max_vector_width(const Pipeline& p, const GroupSched& g, int W, int H, bool any_width) {
    bool user = false;
    auto narrow = [&](int id) { return p.nodes[id].is_int() && dtype_size(p.nodes[id].dtype) < 4; };
    for (int n : g.nodes) {
        if (p.is_output(n) && narrow(n)) user = true;
        for (int s : p.nodes[n].srcs)
            if (p.nodes[s].kind == Kind::Input && narrow(s)) user = true;
    }
    if (!user) return 4;
    if (any_width) return 1;
    int lw = W;
    for (int i = 0; i < p.nodes[g.nodes[0]].level; ++i) lw = (lw + 1) / 2;
    (void)H;
    return lw % 4 == 0 ? 4 : (lw % 2 == 0 ? 2 : 1);
}

// A down2 whose source is computed in a fused (non-resampling) group is
// written by that group directly, decimated: its own launch and the
// full-resolution read of its source disappear.  Its consumers still come
// after the producing group, so the order stays valid.
void absorb_downsamples(const Pipeline& p, Schedule& s) {
    std::vector<GroupSched> out;
    for (const GroupSched& g : s.groups) {
        bool absorbed = false;
        if (g.nodes.size() == 1 && p.nodes[g.nodes[0]].kind == Kind::Down2) {
            int src = p.nodes[g.nodes[0]].srcs[0];
            for (GroupSched& h : out)
                if (!is_resample_group(p, h) && std::binary_search(h.nodes.begin(), h.nodes.end(), src)) {
                    h.dec.push_back(g.nodes[0]);
                    absorbed = true;
                    break;
                }
        }
        if (!absorbed) out.push_back(g);
    }
    s.groups = out;
}

// An up2 that is not a pipeline output and whose every consumer is fused
// in a (non-resampling) group is read by expansion inside those groups: its
// launch and its full-resolution image disappear.
void absorb_upsamples(const Pipeline& p, Schedule& s) {
    auto cons = p.consumers();
    std::vector<GroupSched> out;
    std::vector<int> drop;
    for (const GroupSched& g : s.groups) {
        if (g.nodes.size() != 1 || p.nodes[g.nodes[0]].kind != Kind::Up2 || p.is_output(g.nodes[0])) continue;
        int u = g.nodes[0];
        bool ok = !cons[u].empty();
        for (int c : cons[u]) {
            bool found = false;
            for (const GroupSched& h : s.groups)
                if (!is_resample_group(p, h) && std::binary_search(h.nodes.begin(), h.nodes.end(), c)) found = true;
            ok = ok && found;
        }
        if (ok) drop.push_back(u);
    }
    for (GroupSched g : s.groups) {
        if (g.nodes.size() == 1 && std::count(drop.begin(), drop.end(), g.nodes[0])) continue;
        if (!is_resample_group(p, g))
            for (int u : drop)
                for (int c : cons[u])
                    if (std::binary_search(g.nodes.begin(), g.nodes.end(), c) &&
                        !std::count(g.exp.begin(), g.exp.end(), u))
                        g.exp.push_back(u);
        out.push_back(g);
    }
    s.groups = out;
}

Schedule make_schedule(const Pipeline& p, const Machine& m, const SchedRequest& r) {
    switch (r.mode) {
        case WT_SCHED_UNFUSED: {
            Schedule s = schedule_unfused(p, r.fp16);
            for (auto& g : s.groups) g.V = std::min(g.V, max_vector_width(p, g, r.W, r.H, r.any_width));
            return s;
        }
        case WT_SCHED_FIXED: {
            if (r.fixed.empty()) fail(WT_E_INVALID, "WT_SCHED_FIXED needs fixed_schedule");
            Schedule s = parse_schedule(r.fixed, p);
            return s;
        }
        case WT_SCHED_MLP: {
            if (r.model_path.empty()) fail(WT_E_INVALID, "WT_SCHED_MLP needs model_path");
            std::unique_ptr<Mlp> model = Mlp::load(r.model_path);
            SchedRequest rr = r;
            rr.model = model.get();
            Schedule s = schedule_analytic(p, m, rr);
            for (auto& g : s.groups) g.V = std::min(g.V, max_vector_width(p, g, r.W, r.H, r.any_width));
            absorb_downsamples(p, s);
            absorb_upsamples(p, s);
            return s;
        }
        case WT_SCHED_ANALYTIC:
        case WT_SCHED_AUTOTUNE: {
            // the autotuner starts from the learned model's schedule when
            // given one, else from the analytical model's
            std::unique_ptr<Mlp> model;
            SchedRequest rr = r;
            if (r.mode == WT_SCHED_AUTOTUNE && !r.model_path.empty()) {
                model = Mlp::load(r.model_path);
                rr.model = model.get();
            }
            Schedule s = schedule_analytic(p, m, rr);
            for (auto& g : s.groups) g.V = std::min(g.V, max_vector_width(p, g, r.W, r.H, r.any_width));
            absorb_downsamples(p, s);
            absorb_upsamples(p, s);
            return s;
        }
        default: fail(WT_E_INVALID, "unknown schedule mode");
    }
}

}  // namespace wt
