// Group geometry: the warp(wave)-overlapped tile of a fused group (the
// paper, Section 4) and the skewed sub-tiles of hybrid tiling (Section 5,
// Algorithm 1), laid out for 64-lane wavefronts.
//
// Layout of one wave tile.  Lanes run along x; lane t holds V contiguous
// columns of each of TX sub-tiles (sub-tile k covers slots 64*V*k ..
// 64*V*(k+1)-1), so a row of a stage has N = TX*64*V slots.  Sub-tiles
// 0..SX-1 live in LDS, SX..TX-1 in VGPRs (the paper's left shared-memory and
// right register tiles).  The tile streams down y: at step k every stage holds
// its row k + lead, so consecutive rows are the skewed parallelogram sub-tiles
// of the split dimension and only a window of `win` rows is kept per stage.
//
// Alignment (Section 5, "alignment and scaling"): slot j of node n holds
// x = x0 + a_n + j.  With align=1 each node n gets an x skew a_n with
// a_p >= a_c + dx for every dependence (dx, dy) of consumer c on p (producers
// shifted right, parallel to the right hyperplane), so that in slot space
// every producer read is at offset dx - (a_p - a_c) <= 0:
// a read comes from the same slot or from the left, which gives exactly the
// four load types (own register / LDS / other lane of the same sub-tile /
// other lane of the previous sub-tile).  The same rule on y gives the leads.
// With align=0 (the default) all skews are 0 and reads may also come from
// the right: because a whole stage row is resident before its consumers run,
// the next sub-tile plays the role of the previous one for those reads.
#include <algorithm>
#include <numeric>
#include <set>
#include <sstream>

#include "wt_internal.h"

namespace wt {

bool is_resample_group(const Pipeline& p, const GroupSched& g) {
    if (g.nodes.size() != 1) return false;
    Kind k = p.nodes[g.nodes[0]].kind;
    return k == Kind::Down2 || k == Kind::Up2;
}

bool is_hist_group(const Pipeline& p, const GroupSched& g) {
    return g.nodes.size() == 1 && p.nodes[g.nodes[0]].kind == Kind::Hist;
}

static int round_up(int v, int m) { return (v + m - 1) / m * m; }

GroupGeom group_geometry(const Pipeline& p, const GroupSched& g) {
    if (g.nodes.empty()) fail(WT_E_INVALID, "empty group");
    if (g.V != 1 && g.V != 2 && g.V != 4) fail(WT_E_INVALID, "V must be 1, 2 or 4");
    if (g.TX < 1 || g.TX > 16) fail(WT_E_INVALID, "TX must be in 1..16");
    if (g.SX < 0 || g.SX > g.TX) fail(WT_E_INVALID, "SX must be in 0..TX");
    if (g.TY < 1 || g.TY > 1024) fail(WT_E_INVALID, "TY must be in 1..1024");
    if (g.WPB < 1 || g.WPB > 16) fail(WT_E_INVALID, "WPB must be in 1..16");
    if (g.PF < 0 || g.PF > 8) fail(WT_E_INVALID, "PF must be in 0..8");
    if (g.GH != 0 && g.GH != 1) fail(WT_E_INVALID, "GH must be 0 or 1");

    GroupGeom geo;
    std::set<int> mem(g.nodes.begin(), g.nodes.end());
    std::set<int> dec(g.dec.begin(), g.dec.end());
    std::set<int> hst(g.hst.begin(), g.hst.end());
    int level = p.nodes[g.nodes[0]].level;
    for (size_t i = 0; i < g.nodes.size(); ++i) {
        const Node& n = p.nodes[g.nodes[i]];
        if (n.kind == Kind::Up2) {
            // a folded up2: the group holds the stage it folds and writes
            // the down2 between them decimated
            int f = p.fold_source(n.id);
            if (f < 0 || !mem.count(f) || !dec.count(n.srcs[0]))
                fail(WT_E_INVALID, "up2 node " + std::to_string(n.id) +
                                       " can only be fused with the stage whose decimation it expands");
        } else if (n.kind == Kind::Equalize) {
            if (hst.count(n.srcs[1]))
                fail(WT_E_INVALID, "equalize node " + std::to_string(n.id) +
                                       " reads a histogram its own group accumulates");
        } else if (n.kind != Kind::Stencil && n.kind != Kind::Pointwise) {
            fail(WT_E_INVALID, "node " + std::to_string(n.id) + " cannot be fused");
        }
        if (n.level != level) fail(WT_E_INVALID, "group spans pyramid levels");
        if (i && g.nodes[i] <= g.nodes[i - 1]) fail(WT_E_INVALID, "group nodes must be sorted");
    }
    // the group's dependence graph: a folded up2 reads the stage it folds
    auto gsrcs = [&](int m) -> std::vector<int> {
        if (p.nodes[m].kind == Kind::Up2) return {p.fold_source(m)};
        if (p.nodes[m].kind == Kind::Equalize) return {p.nodes[m].srcs[0]};  // its histogram is a table
        return p.nodes[m].srcs;
    };
    for (int m : g.nodes)
        if (p.nodes[m].kind == Kind::Equalize &&
            std::find(geo.tables.begin(), geo.tables.end(), p.nodes[m].srcs[1]) == geo.tables.end())
            geo.tables.push_back(p.nodes[m].srcs[1]);
    auto cons = p.consumers();
    for (int m : g.nodes)
        if (p.nodes[m].kind == Kind::Up2) cons[p.fold_source(m)].push_back(m);

    // loaded nodes and live-outs
    std::set<int> loaded;
    for (int m : g.nodes)
        for (int s : gsrcs(m))
            if (!mem.count(s)) loaded.insert(s);
    geo.loaded.assign(loaded.begin(), loaded.end());
    for (int d : g.dec) {
        if (d < 0 || d >= (int)p.nodes.size() || p.nodes[d].kind != Kind::Down2)
            fail(WT_E_INVALID, "dec names a node that is not a down2 stage");
        int s = p.nodes[d].srcs[0];
        if (!mem.count(s)) fail(WT_E_INVALID, "dec node " + std::to_string(d) + " decimates a non-member");
        geo.dec.push_back({d, s});
    }
    for (int h : g.hst) {
        if (h < 0 || h >= (int)p.nodes.size() || p.nodes[h].kind != Kind::Hist)
            fail(WT_E_INVALID, "hst names a node that is not a histogram stage");
        int s = p.nodes[h].srcs[0];
        if (!mem.count(s)) fail(WT_E_INVALID, "hst node " + std::to_string(h) + " counts a non-member");
        geo.hist.push_back({h, s});
    }
    for (int m : g.nodes) {
        bool lo = p.is_output(m);
        for (int c : cons[m])
            if (!mem.count(c) && !dec.count(c) && !hst.count(c)) lo = true;
        if (lo) geo.liveouts.push_back(m);
    }
    geo.outs = geo.liveouts;
    for (auto& ds : geo.dec)
        if (std::find(geo.outs.begin(), geo.outs.end(), ds.second) == geo.outs.end()) geo.outs.push_back(ds.second);
    for (auto& hs : geo.hist)
        if (std::find(geo.outs.begin(), geo.outs.end(), hs.second) == geo.outs.end()) geo.outs.push_back(hs.second);
    std::sort(geo.outs.begin(), geo.outs.end());
    if (geo.outs.empty()) fail(WT_E_INVALID, "group has no live-out");

    // channel mode
    int C = p.nodes[g.nodes[0]].channels;
    bool par = true;
    for (int m : g.nodes) {
        const Node& n = p.nodes[m];
        if (n.channels != C) par = false;
        if (n.kind == Kind::Pointwise && expr_has_explicit_channel(n.expr)) par = false;
    }
    for (int l : geo.loaded)
        if (p.nodes[l].channels != C && p.nodes[l].channels != 1) par = false;
    geo.chan_parallel = par;
    geo.C = par ? C : 1;

    // nodes: loaded first, then members in topological order
    for (int l : geo.loaded) geo.nodes.push_back({l, false, false});
    for (int m : g.nodes) geo.nodes.push_back({m, true, false});
    for (int u : g.exp) {
        if (u < 0 || u >= (int)p.nodes.size() || p.nodes[u].kind != Kind::Up2)
            fail(WT_E_INVALID, "exp names a node that is not an up2 stage");
        if (!loaded.count(u)) fail(WT_E_INVALID, "exp node " + std::to_string(u) + " is not read by the group");
    }
    for (size_t i = 0; i < geo.nodes.size(); ++i) {
        NodeGeom& ng = geo.nodes[i];
        if (!ng.member && std::find(g.exp.begin(), g.exp.end(), ng.id) != g.exp.end())
            ng.expand_src = p.nodes[ng.id].srcs[0];
        geo.index[ng.id] = (int)i;
        ng.liveout = std::find(geo.liveouts.begin(), geo.liveouts.end(), ng.id) != geo.liveouts.end();
        ng.out = std::find(geo.outs.begin(), geo.outs.end(), ng.id) != geo.outs.end();
        ng.skew = ng.lead = 0;
        ng.win = 1;
        ng.nch = par ? 1 : p.nodes[ng.id].channels;
        ng.fix_top = ng.fix_bot = ng.fix_x = false;
        ng.vlo = ng.vhi = 0;
        ng.consumed = false;
        ng.lds_off = 0;
        ng.half = g.fp16 && ng.member && p.half_storable(ng.id);
        ng.mem_half = false;
    }

    // skews and leads, consumers before producers (reverse creation order)
    std::vector<int> order;
    for (auto& ng : geo.nodes) order.push_back(ng.id);
    std::sort(order.rbegin(), order.rend());
    for (int id : order) {
        NodeGeom& ng = geo.nodes[geo.index[id]];
        int a = 0, L = 0, oldest = 0;
        bool any = false;
        for (int c : cons[id]) {
            if (!mem.count(c)) continue;
            const NodeGeom& cg = geo.nodes[geo.index[c]];
            for (const Tap& t : p.taps(c, id)) {
                a = std::max(a, cg.skew + t.dx);
                L = std::max(L, cg.lead + std::max(t.dy, 0));
                if (t.dy < 0) ng.fix_top = true;
                if (t.dy > 0) ng.fix_bot = true;
                if (t.dx != 0) ng.fix_x = true;
                any = true;
            }
        }
        if (g.align == 0) a = 0;
        if ((ng.out || !ng.member) && a % g.V) a = round_up(a, g.V);
        ng.skew = a;
        ng.lead = L;
        ng.consumed = any;
        if (any) {
            oldest = L;
            for (int c : cons[id]) {
                if (!mem.count(c)) continue;
                const NodeGeom& cg = geo.nodes[geo.index[c]];
                for (const Tap& t : p.taps(c, id)) oldest = std::min(oldest, cg.lead + t.dy);
            }
            ng.win = L - oldest + 1;
        }
        if (!ng.member) ng.fix_top = ng.fix_bot = ng.fix_x = false;  // clamped loads
        if (ng.fix_bot) ng.win = std::max(ng.win, 2);  // keeps row r-1 for the copy
    }

    // members whose rows are used only on even rows: decimated (and not
    // otherwise stored) or read only by folded up2s
    for (auto& ng : geo.nodes) {
        if (!ng.member || ng.liveout) continue;
        bool uses = false, only_even = true;
        for (int c : cons[ng.id]) {
            if (hst.count(c)) {
                uses = true;
                only_even = false;
            } else if (dec.count(c)) {
                uses = true;
            } else if (mem.count(c)) {
                uses = true;
                if (p.nodes[c].kind != Kind::Up2) only_even = false;
            }
        }
        ng.even_rows = uses && only_even;
    }

    // loads run PF rows ahead of their first use (software prefetch)
    for (auto& ng : geo.nodes)
        if (!ng.member) {
            ng.lead += g.PF;
            ng.win += g.PF;
        }

    // ghost columns (GH=1): a plain loaded node carries, beyond its slots,
    // the columns its member consumers read there, so it is valid on
    // [-ghl, N + ghr) and those consumers on every slot
    if (g.GH) {
        if (g.SX != 0 || g.align != 0 || g.BLK) fail(WT_E_UNSUPPORTED, "GH=1 needs SX=0, align=0 and BLK=0");
        for (auto& ng : geo.nodes) {
            if (ng.member || ng.expand_src >= 0) continue;
            int l = 0, r = 0;
            for (int c : cons[ng.id]) {
                if (!mem.count(c)) continue;
                const NodeGeom& cg = geo.nodes[geo.index[c]];
                for (const Tap& t : p.taps(c, ng.id)) {
                    int delta = t.dx - (ng.skew - cg.skew);
                    l = std::max(l, -delta);
                    r = std::max(r, delta);
                }
            }
            if (l > 64 * g.V || r > 64 * g.V) fail(WT_E_UNSUPPORTED, "ghost columns exceed one sub-tile");
            ng.ghl = l;
            ng.ghr = r;
            ng.vlo = -l;
            ng.vhi = -r;
        }
    }

    // valid slot range [vlo, N - vhi), producers before consumers: a read at
    // slot offset delta = dx - (a_p - a_c) needs slot j + delta valid.
    for (auto& ng : geo.nodes) {
        if (!ng.member) continue;
        int lo = 0, hi = 0;
        for (int s : gsrcs(ng.id)) {
            const NodeGeom& pg = geo.nodes[geo.index[s]];
            for (const Tap& t : p.taps(ng.id, s)) {
                int delta = t.dx - (pg.skew - ng.skew);
                lo = std::max(lo, pg.vlo - delta);
                hi = std::max(hi, pg.vhi + delta);
            }
        }
        ng.vlo = lo;
        ng.vhi = hi;
    }

    geo.N = g.TX * 64 * g.V;
    int vlo = 0, vhi = 0, amax = 0;
    for (int lo : geo.outs) {
        const NodeGeom& ng = geo.nodes[geo.index[lo]];
        vlo = std::max(vlo, ng.vlo);
        vhi = std::max(vhi, ng.vhi);
        amax = std::max(amax, ng.skew);
    }
    geo.S0 = round_up(vlo, g.V);
    geo.X = (geo.N - vhi - geo.S0) / g.V * g.V;
    if (geo.X <= 0)
        fail(WT_E_UNSUPPORTED, "tile too narrow for the group's halo (" + std::to_string(vlo + vhi) +
                                   " columns); raise TX or V");
    // slot j of node n holds x = x0 + a_n + j; tile 0 starts the live-out
    // with the largest skew at x = 0 (the others start left of it)
    geo.base = -amax - geo.S0;

    // warm-up: the earliest step at which some node must hold a valid row
    std::map<int, int> first;  // first needed row relative to y0
    for (int lo : geo.outs) first[lo] = 0;
    for (int id : order) {
        if (!first.count(id)) first[id] = 0;
        for (int c : cons[id]) {
            if (!mem.count(c)) continue;
            for (const Tap& t : p.taps(c, id)) first[id] = std::min(first[id], first[c] + t.dy);
        }
    }
    int kmin = 0;
    for (auto& ng : geo.nodes) kmin = std::min(kmin, first[ng.id] - ng.lead);
    geo.D = -kmin;
    for (auto& ng : geo.nodes) ng.first_step = geo.D + first[ng.id] - ng.lead;

    // unroll period: ring slots become compile-time register names
    std::vector<int> wins;
    for (auto& ng : geo.nodes) wins.push_back(ng.win);
    int U = 1;
    for (int w : wins) U = std::lcm(U, w);
    if (U > 12) {
        U = *std::max_element(wins.begin(), wins.end());
        for (auto& ng : geo.nodes) {
            int w = ng.win;
            while (U % w) ++w;
            ng.win = w;
        }
    }
    // a folded up2 weighs its source's rows by their parity: an even period
    // fixes every step's row parity at compile time (with even TY)
    bool folds = false;
    for (int m : g.nodes)
        if (p.nodes[m].kind == Kind::Up2) folds = true;
    if (folds && U % 2 && 2 * U <= 24) U *= 2;
    geo.U = U;
    // main loop of whole periods; the epilogue holds the rest and at least
    // the last PF steps, whose loads would fetch rows past the tile
    geo.E = g.TY % U;
    while (geo.E < g.PF && geo.E + U <= g.TY) geo.E += U;
    if (geo.E < g.PF) geo.E = g.TY;
    geo.NMAIN = (g.TY - geo.E) / U;

    // LDS rings: rows x channels x (SX*64*V) values per consumed node
    int off = 0;
    int per_row = g.SX * 64 * g.V;
    for (auto& ng : geo.nodes) {
        ng.lds_off = off;
        if (g.SX == 0 || !ng.consumed) continue;
        int bytes = ng.win * ng.nch * per_row * (ng.half ? 2 : 4);
        off += round_up(bytes, 16);
    }
    // then each accumulated histogram's bins (32-bit counts per channel slot)
    geo.hist_lds_off = off;
    for (auto& hs : geo.hist) {
        const int words = p.nodes[hs.first].bins * geo.nodes[geo.index.at(hs.second)].nch;
        off += round_up((words + 1) * hist_replicas(words) * 4, 16);
    }
    // then the cumulative counts of the tables equalize members read, and 64
    // words for the lanes' partial sums while they are formed
    geo.table_lds_off = off;
    for (int t : geo.tables) off += round_up(p.nodes[t].bins * (par ? 1 : p.nodes[t].channels) * 4, 16);
    if (!geo.tables.empty()) off += 256;
    geo.lds_bytes = off;
    geo.lds_bytes_per_wg = off * g.WPB;
    return geo;
}

std::string describe_group(const GroupSched& g) {
    std::ostringstream os;
    os << "nodes=";
    for (size_t i = 0; i < g.nodes.size(); ++i) os << (i ? "," : "") << g.nodes[i];
    os << " V=" << g.V << " TX=" << g.TX << " SX=" << g.SX << " TY=" << g.TY
       << " WPB=" << g.WPB << " PF=" << g.PF << " fp16=" << (g.fp16 ? 1 : 0) << " align=" << g.align
       << " XCD=" << g.XCD << " NT=" << g.NT;
    if (g.ORD) os << " ORD=" << g.ORD;
    if (g.BLK) os << " BLK=" << g.BLK;
    if (g.GH) os << " GH=" << g.GH;
    if (!g.dec.empty()) {
        os << " dec=";
        for (size_t i = 0; i < g.dec.size(); ++i) os << (i ? "," : "") << g.dec[i];
    }
    if (!g.exp.empty()) {
        os << " exp=";
        for (size_t i = 0; i < g.exp.size(); ++i) os << (i ? "," : "") << g.exp[i];
    }
    if (!g.hst.empty()) {
        os << " hst=";
        for (size_t i = 0; i < g.hst.size(); ++i) os << (i ? "," : "") << g.hst[i];
    }
    return os.str();
}

Schedule parse_schedule(const std::string& text, const Pipeline& p, bool partial) {
    Schedule s;
    std::string t = text;
    std::replace(t.begin(), t.end(), ';', '\n');
    std::istringstream lines(t);
    std::string line;
    std::set<int> seen, expanded;
    while (std::getline(lines, line)) {
        std::istringstream ws(line);
        std::string tok;
        GroupSched g;
        bool any = false;
        while (ws >> tok) {
            auto eq = tok.find('=');
            if (eq == std::string::npos) continue;  // e.g. a "g0" label
            std::string k = tok.substr(0, eq), v = tok.substr(eq + 1);
            if (k.rfind("batch_", 0) == 0) continue;  // launch facts in a plan description
            try {
                if (k == "nodes") {
                    std::istringstream vs(v);
                    std::string n;
                    while (std::getline(vs, n, ',')) g.nodes.push_back(std::stoi(n));
                } else if (k == "V") g.V = std::stoi(v);
                else if (k == "TX") g.TX = std::stoi(v);
                else if (k == "SX") g.SX = std::stoi(v);
                else if (k == "TY") g.TY = std::stoi(v);
                else if (k == "WPB") g.WPB = std::stoi(v);
                else if (k == "fp16") g.fp16 = std::stoi(v) != 0;
                else if (k == "align") g.align = std::stoi(v);
                else if (k == "PF") g.PF = std::stoi(v);
                else if (k == "XCD") g.XCD = std::stoi(v);
                else if (k == "ORD") g.ORD = std::stoi(v);
                else if (k == "BLK") g.BLK = std::stoi(v);
                else if (k == "GH") g.GH = std::stoi(v);
                else if (k == "dec" || k == "exp" || k == "hst") {
                    std::istringstream vs(v);
                    std::string n;
                    while (std::getline(vs, n, ','))
                        (k == "dec" ? g.dec : k == "exp" ? g.exp : g.hst).push_back(std::stoi(n));
                }
                else if (k == "NT") g.NT = std::stoi(v);
                else fail(WT_E_INVALID, "unknown schedule key '" + k + "'");
            } catch (const std::logic_error&) {
                fail(WT_E_INVALID, "bad schedule value '" + tok + "'");
            }
            any = true;
        }
        if (!any) continue;
        std::sort(g.nodes.begin(), g.nodes.end());
        for (int n : g.nodes) {
            if (n < 0 || n >= (int)p.nodes.size() || p.nodes[n].kind == Kind::Input)
                fail(WT_E_INVALID, "schedule names a non-stage node " + std::to_string(n));
            if (!seen.insert(n).second)
                fail(WT_E_INVALID, "node " + std::to_string(n) + " in two groups");
        }
        for (int d : g.dec) {  // a decimated down2 is produced by this group
            if (d < 0 || d >= (int)p.nodes.size()) fail(WT_E_INVALID, "dec names an unknown node");
            if (!seen.insert(d).second) fail(WT_E_INVALID, "node " + std::to_string(d) + " in two groups");
        }
        for (int h : g.hst) {  // an accumulated histogram is produced by this group
            if (h < 0 || h >= (int)p.nodes.size()) fail(WT_E_INVALID, "hst names an unknown node");
            if (!seen.insert(h).second) fail(WT_E_INVALID, "node " + std::to_string(h) + " in two groups");
        }
        for (int u : g.exp) expanded.insert(u);  // may be expanded by several groups
        s.groups.push_back(g);
    }
    if (!partial)
        for (const Node& n : p.nodes)
            if (n.kind != Kind::Input && !seen.count(n.id) && !expanded.count(n.id))
                fail(WT_E_INVALID, "schedule misses node " + std::to_string(n.id));
    return s;
}

}  // namespace wt
