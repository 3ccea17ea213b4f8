// Schedules: which stages are fused and with which tile configuration.
#include <set>

#include "wt_internal.h"

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

Schedule make_schedule(const Pipeline& p, const Machine& m, const SchedRequest& r) {
    switch (r.mode) {
        case WT_SCHED_UNFUSED: return schedule_unfused(p, r.fp16);
        case WT_SCHED_FIXED: {
            if (r.fixed.empty()) fail(WT_E_INVALID, "WT_SCHED_FIXED needs fixed_schedule");
            Schedule s = parse_schedule(r.fixed, p);
            return s;
        }
        case WT_SCHED_ANALYTIC:
        case WT_SCHED_MLP:
        case WT_SCHED_AUTOTUNE: return schedule_analytic(p, m, r);
        default: fail(WT_E_INVALID, "unknown schedule mode");
    }
}

}  // namespace wt
