// Fusion search (placeholder: maximal same-level fusion; replaced by the
// bounded DP over convex groups with the analytical cost).
#include <set>

#include "wt_internal.h"

namespace wt {

Schedule schedule_analytic(const Pipeline& p, const Machine& m, const SchedRequest& r) {
    (void)m;
    Schedule s;
    GroupSched cur;
    int level = -1;
    auto flush = [&] {
        if (!cur.nodes.empty()) s.groups.push_back(cur);
        cur = GroupSched{};
        cur.fp16 = r.fp16;
    };
    cur.fp16 = r.fp16;
    for (const Node& n : p.nodes) {
        if (n.kind == Kind::Input) continue;
        bool fusable = n.kind == Kind::Stencil || n.kind == Kind::Pointwise;
        if (!fusable) {
            flush();
            GroupSched g;
            g.nodes = {n.id};
            s.groups.push_back(g);
            level = -1;
            continue;
        }
        if (n.level != level) flush();
        level = n.level;
        cur.nodes.push_back(n.id);
    }
    flush();
    return s;
}

}  // namespace wt
