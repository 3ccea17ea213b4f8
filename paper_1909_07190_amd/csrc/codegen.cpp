// HIP code generation for fused wave-tile groups.
//
// One generated kernel per group.  Each wavefront computes one overlapped
// tile (OTPW, the paper's Section 4) and synchronises its stages at wave
// level only.  Every producer load inside the group is classified at
// generation time into the four load types of hybrid tiling (Section 5,
// Fig. 4; Algorithm 1 and its generalisation in Appendix A) and emitted as:
//   (1) a VGPR of the same lane       -> a named register
//   (2) a value in the LDS sub-tiles  -> ds_read
//   (3) a VGPR of another lane of the same register sub-tile and
//   (4) a VGPR of another lane of the previous register sub-tile
//                                      -> DPP wavefront shift (one-lane
//                                         distance) or ds_bpermute.
// Register tiles are fully unrolled into compile-time-indexed arrays (the
// paper's explicit register naming), and the y direction is streamed with a
// per-stage ring of rows whose slots are fixed per unrolled step.
#include <cmath>
#include <cstdio>
#include <functional>
#include <set>
#include <sstream>

#include "wt_internal.h"
#include "wt_device_src.inc"  // kWtDeviceSrc: device/wt_device.h as a string

namespace wt {

std::string device_prelude() { return kWtDeviceSrc; }

namespace {

std::string flit(double v) {
    char b[64];
    std::snprintf(b, sizeof b, "%.9e", (double)(float)v);
    return std::string("(") + b + "f)";
}

int pmod(int a, int m) { return ((a % m) + m) % m; }

struct Gen {
    const Pipeline& P;
    const GroupSched& g;
    const GroupGeom& geo;
    std::ostringstream o;
    int V, SX, RX, N, SUB;
    std::map<std::string, std::string> memo;  // per unrolled step
    int tmp = 0;
    std::string ind = "    ";

    Gen(const Pipeline& p, const GroupSched& gs, const GroupGeom& ge)
        : P(p), g(gs), geo(ge), V(gs.V), SX(gs.SX), RX(gs.TX - gs.SX), N(ge.N), SUB(64 * gs.V) {}

    const NodeGeom& G(int id) const { return geo.nodes.at(geo.index.at(id)); }
    std::string I(int v) { return std::to_string(v); }
    void line(const std::string& s) { o << ind << s << "\n"; }

    bool isint(int id) const { return P.nodes[id].is_int(); }
    // register / LDS type of a node's values, and its element type in memory
    std::string ctype(int id) const { return isint(id) ? "int" : "float"; }
    std::string mtype(const NodeGeom& n) const {
        return isint(n.id) ? dtype_ctype(P.nodes[n.id].dtype) : (n.mem_half ? "_Float16" : "float");
    }
    int msize(const NodeGeom& n) const { return isint(n.id) ? dtype_size(P.nodes[n.id].dtype) : (n.mem_half ? 2 : 4); }
    // ext_vector type of V elements of C type `t`
    static std::string vec(const std::string& t, int V) {
        std::string b = t == "float" ? "wt_f" : t == "_Float16" ? "wt_h" : t == "int" ? "wt_i" :
                        t == "unsigned char" ? "wt_b" : t == "unsigned short" ? "wt_us" : "wt_s";
        return b + std::to_string(V);
    }
    // vector type for a global load of V elements of C type `t`: 32-bit
    // elements need only their own alignment (rows may start anywhere)
    static std::string gvec(const std::string& t, int V) {
        if (t == "float") return "wt_f" + std::to_string(V) + "d";
        if (t == "int") return "wt_i" + std::to_string(V) + "d";
        return vec(t, V);
    }
    // unsigned type of `bytes` bytes and the buffer store of that width
    static std::string store_ty(int bytes) {
        switch (bytes) {
            case 1: return "unsigned char";
            case 2: return "unsigned short";
            case 4: return "unsigned int";
            case 8: return "wt_u2";
            default: return "wt_u4";
        }
    }
    static std::string store_fn(int bytes) {
        return "__builtin_amdgcn_raw_buffer_store_b" + std::to_string(bytes * 8);
    }

    bool has_regs(const NodeGeom& n) const { return RX > 0 && (n.consumed || !n.member); }
    // ghost registers of a loaded node (GH=1): lanes 64-nl..63 of `gl` hold
    // the nl*V columns left of slot 0 (as lanes of a sub-tile -1 would), lanes
    // 0..nr-1 of `gr` the nr*V columns right of the last slot; a single ghost
    // lane is kept where its one-lane shift lands instead (lane 0 of `gl`,
    // lane 63 of `gr`)
    int ghost_lanes_l(const NodeGeom& n) const { return (n.ghl + V - 1) / V; }
    int ghost_lanes_r(const NodeGeom& n) const { return (n.ghr + V - 1) / V; }
    std::string ghost(int id, bool left, int slot, int ch, int e) {
        return "g" + I(id) + (left ? "l" : "r") + "[" + I(slot) + "][" + I(ch) + "][" + I(e) + "]";
    }
    bool has_lds(const NodeGeom& n) const { return SX > 0 && (n.consumed || !n.member); }
    // FP16 members with an even number of elements per lane keep their
    // register rows as packed pairs, two values per VGPR (wt_h2); they are
    // converted to FP32 when read (the arithmetic stays FP32).
    bool packed(int id) const {
        const NodeGeom& n = G(id);
        return n.half && V % 2 == 0 && has_regs(n);
    }
    // The packed pair holding element e, as an lvalue.
    std::string preg(int id, int slot, int ch, int kr, int e) {
        return "w" + I(id) + "[" + I(slot) + "][" + I(ch) + "][" + I(kr) + "][" + I(e / 2) + "]";
    }
    // Element e of a register row: an lvalue, or for packed rows the
    // element converted to FP32 (an rvalue; writes go through preg).
    std::string reg(int id, int slot, int ch, int kr, int e) {
        if (packed(id)) return "((float)" + preg(id, slot, ch, kr, e) + "[" + I(e % 2) + "])";
        return "w" + I(id) + "[" + I(slot) + "][" + I(ch) + "][" + I(kr) + "][" + I(e) + "]";
    }
    // LDS element index of (slot, ch, j) of node id
    std::string lidx(int id, int slot, int ch, const std::string& j) {
        const NodeGeom& n = G(id);
        return "L" + I(id) + "[" + I((slot * n.nch + ch) * SX * SUB) + " + (" + j + ")]";
    }
    std::string lread(int id, int slot, int ch, const std::string& j) {
        return "(" + ctype(id) + ")" + lidx(id, slot, ch, j);
    }
    std::string fresh(const std::string& pfx) { return pfx + I(tmp++); }
    std::string memoize(const std::string& expr, bool opaque = false) {
        auto it = memo.find(expr);
        if (it != memo.end()) return it->second;
        std::string n = fresh("t");
        if (opaque) {
            // An integer lane exchange, kept opaque to the compiler: without
            // this the backend folds the DPP move into the following integer
            // add / subtract (v_add_u32_dpp, v_subrev_u32_dpp), and those
            // folded forms gave wrong values on gfx950, while the separate
            // move is exact.  (Float arithmetic here is never folded: its
            // operands are literal constants.)
            line("auto " + n + " = " + expr + ";");
            line("asm volatile(\"\" : \"+v\"(" + n + "));");
        } else {
            line("const auto " + n + " = " + expr + ";");
        }
        memo[expr] = n;
        return n;
    }
    // memoize for a lane exchange of node p's values
    std::string xchg(int p, const std::string& expr) { return memoize(expr, isint(p)); }

    // Producer value for consumer c (channel slot of the producer chp) at
    // sub-tile k, element e, through dependence (dx, dy), at unrolled step ph.
    // Slot offset delta = dx - (a_p - a_c); q = e + delta locates the source
    // element relative to this lane's first element.
    std::string read(int c, int p, int chp, int k, int e, int dx, int dy, int ph) {
        const NodeGeom& cg = G(c);
        const NodeGeom& pg = G(p);
        int drow = pg.lead - cg.lead - dy;
        if (drow < 0 || drow >= pg.win) fail(WT_E_INTERNAL, "ring window too small");
        int slot = pmod(ph - drow, pg.win);
        int delta = dx - (pg.skew - cg.skew);
        if (g.align == 1 && delta > 0) fail(WT_E_INTERNAL, "skew invariant violated");
        int q = e + delta;
        std::string own = I(k * SUB) + " + lane * " + I(V);
        if (q >= 0 && q < V) {
            if (k >= SX) return reg(p, slot, chp, k - SX, q);                 // type 1
            return memoize(lread(p, slot, chp, own + " + " + I(q)));            // type 2
        }
        if ((q < 0 && (-q + V - 1) / V > 63) || q / V > 63) return read_far(p, slot, chp, k, q);
        if (q < 0) {
            int d = (-q + V - 1) / V;
            int ep = q + d * V;
            if (k < SX)  // whole read inside the LDS sub-tiles: type 2 for every lane
                return memoize(lread(p, slot, chp, "max(" + own + " + " + I(q) + ", 0)"));
            std::string cur = reg(p, slot, chp, k - SX, ep);
            if (d == 1) {
                if (k - 1 >= SX)  // types 3 (lanes 1..63) + 4 (lane 0)
                    return xchg(p, "wt_shift1(" + cur + ", " + reg(p, slot, chp, k - 1 - SX, ep) + ")");
                if (k - 1 >= 0) {  // types 3 + 2: lane 0 reads the last LDS sub-tile
                    std::string b = memoize(lread(p, slot, chp, I((k - 1) * SUB + 63 * V + ep)));
                    return xchg(p, "wt_shr1(" + cur + ", " + b + ")");
                }
                if (pg.ghl > 0) {
                    // one ghost lane: it sits in lane 0 already, so a single
                    // DPP shift keeps it there as the shift's old value
                    std::string gv = ghost(p, true, slot, chp, ep);
                    if (ghost_lanes_l(pg) == 1) return xchg(p, "wt_shr1(" + cur + ", " + gv + ")");
                    return xchg(p, "wt_shift1(" + cur + ", " + gv + ")");
                }
                // lane 0 belongs to the overlap: any value
                return xchg(p, "wt_mov_shr1(" + cur + ")");
            }
            if (k - 1 >= SX) {
                std::string prv = reg(p, slot, chp, k - 1 - SX, ep);
                if (d == 2) return xchg(p, "wt_shift2(" + cur + ", " + prv + ")");
                return xchg(p, "wt_shiftd(" + cur + ", " + prv + ", " + I(d) + ", lane)");
            }
            if (k - 1 >= 0) {
                std::string pv = memoize(lread(p, slot, chp, I((k - 1) * SUB) + " + ((lane - " + I(d) +
                                                               ") & 63) * " + I(V) + " + " + I(ep)));
                return xchg(p, "wt_shiftd_l(" + cur + ", " + pv + ", " + I(d) + ", lane)");
            }
            if (pg.ghl > 0) {  // lanes t < d read the ghost lanes 64-d+t
                std::string gv = ghost(p, true, slot, chp, ep);
                if (d == 2) return xchg(p, "wt_shift2(" + cur + ", " + gv + ")");
                return xchg(p, "wt_shiftd(" + cur + ", " + gv + ", " + I(d) + ", lane)");
            }
            if (d == 2) return xchg(p, "wt_shift2(" + cur + ", " + cur + ")");
            return xchg(p, "wt_shiftd(" + cur + ", " + cur + ", " + I(d) + ", lane)");
        }
        // q >= V: source to the right (lane t + d, or the next sub-tile)
        int d = q / V;
        int ep = q - d * V;
        if (k < SX) {
            std::string lv = memoize(lread(p, slot, chp, "min(" + own + " + " + I(q) + ", " + I(SX * SUB - 1) + ")"));
            if (k + 1 < SX || SX == g.TX) return lv;  // type 2 (or overlap past the strip)
            // last LDS sub-tile: lanes t >= 64-d read the first register sub-tile
            std::string nx = reg(p, slot, chp, 0, ep);
            std::string rot = d == 1 ? "wt_rol1(" + nx + ")"
                                     : "wt_bperm(((lane + " + I(d) + ") & 63) << 2, " + nx + ")";
            std::string rv = xchg(p, rot);
            return memoize("(lane >= " + I(64 - d) + " ? " + rv + " : " + lv + ")");
        }
        std::string cur = reg(p, slot, chp, k - SX, ep);
        if (k + 1 >= g.TX && pg.ghr > 0) {  // lanes t >= 64-d read the ghost lanes t+d-64
            std::string gv = ghost(p, false, slot, chp, ep);
            if (d == 1 && ghost_lanes_r(pg) == 1) return xchg(p, "wt_shl1(" + cur + ", " + gv + ")");
            if (d == 1) return xchg(p, "wt_shift1n(" + cur + ", " + gv + ")");
            if (d == 2) return xchg(p, "wt_shift2n(" + cur + ", " + gv + ")");
            return xchg(p, "wt_shiftdn(" + cur + ", " + gv + ", " + I(d) + ", lane)");
        }
        if (k + 1 >= g.TX) {  // lanes past the strip belong to the overlap: any value
            if (d == 1) return xchg(p, "wt_mov_shl1(" + cur + ")");
            if (d == 2) return xchg(p, "wt_shift2n(" + cur + ", " + cur + ")");
            return xchg(p, "wt_shiftdn(" + cur + ", " + cur + ", " + I(d) + ", lane)");
        }
        std::string next = reg(p, slot, chp, k + 1 - SX, ep);
        if (d == 1) return xchg(p, "wt_shift1n(" + cur + ", " + next + ")");
        if (d == 2) return xchg(p, "wt_shift2n(" + cur + ", " + next + ")");
        return xchg(p, "wt_shiftdn(" + cur + ", " + next + ", " + I(d) + ", lane)");
    }

    // A source 64 or more lanes to the left (Appendix A's lookback across
    // several sub-tiles: under the right-hyperplane skew the offsets of a
    // deep group add up along its chains).  With the lane distance
    // d = 64 j + r, lane t reads lane t - r of sub-tile k - j, and lanes
    // t < r read lane t - r + 64 of sub-tile k - j - 1; register sub-tiles
    // exchange across lanes, LDS sub-tiles are indexed directly.  Sub-tiles
    // left of the strip hold overlap columns, whose values no valid output
    // depends on; ghost columns (a few lanes wide) cannot stand in for them.
    std::string read_far(int p, int slot, int chp, int k, int q) {
        const NodeGeom& pg = G(p);
        const std::string own = I(k * SUB) + " + lane * " + I(V);
        const std::string any = "((" + ctype(p) + ")0)";
        if (q < 0) {
            const int d = (-q + V - 1) / V, ep = q + d * V, j = d / 64, r = d % 64;
            const int A = k - j, B = A - 1;
            if (pg.ghl > 0 && (A < 0 || (r > 0 && B < 0)))
                fail(WT_E_UNSUPPORTED, "ghost columns do not reach a dependence spanning sub-tiles");
            if (A < 0) return any;
            if (A < SX) {  // every source position lies in the LDS sub-tiles
                if (r == 0) return memoize(lread(p, slot, chp, I(A * SUB) + " + lane * " + I(V) + " + " + I(ep)));
                return memoize(lread(p, slot, chp, "max(" + own + " + " + I(q) + ", 0)"));
            }
            const std::string cur = reg(p, slot, chp, A - SX, ep);
            if (r == 0) return cur;
            if (B >= SX) {
                const std::string prv = reg(p, slot, chp, B - SX, ep);
                if (r == 1) return xchg(p, "wt_shift1(" + cur + ", " + prv + ")");
                if (r == 2) return xchg(p, "wt_shift2(" + cur + ", " + prv + ")");
                return xchg(p, "wt_shiftd(" + cur + ", " + prv + ", " + I(r) + ", lane)");
            }
            if (B >= 0) {
                const std::string pv = memoize(lread(p, slot, chp, I(B * SUB) + " + ((lane - " + I(r) + ") & 63) * " +
                                                                    I(V) + " + " + I(ep)));
                return xchg(p, "wt_shiftd_l(" + cur + ", " + pv + ", " + I(r) + ", lane)");
            }
            return xchg(p, "wt_shiftd(" + cur + ", " + cur + ", " + I(r) + ", lane)");  // lanes t < r: overlap
        }
        // to the right a source is at most 14 columns away (stencil sides are
        // at most 15 and right-hyperplane tiles read only from the left)
        fail(WT_E_INTERNAL, "dependence distance to the right exceeds one wavefront");
        return {};
    }

    int src_chan(const NodeGeom& p, int ch_c, int explicit_ch) {
        if (explicit_ch >= 0) return explicit_ch;
        return p.nch == 1 ? 0 : ch_c;
    }

    std::string expr(const Expr& e, int c, int ch, int k, int el, int ph) {
        const Node& n = P.nodes[c];
        const bool in = n.is_int();
        auto K = [&](int i) { return expr(e.kids[i], c, ch, k, el, ph); };
        switch (e.op) {
            case Expr::Const: return in ? "(" + std::to_string((long long)e.value) + ")" : flit(e.value);
            case Expr::Src: {
                int p = n.srcs[e.src];
                std::string r = read(c, p, src_chan(G(p), ch, e.chan), k, el, 0, 0, ph);
                // a float stage sees integer values converted (exactly, in range)
                return (!in && isint(p)) ? "(float)" + r : r;
            }
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

    std::string value(int c, int ch, int k, int e, int ph) {
        const Node& n = P.nodes[c];
        std::string sat;
        if (n.is_int()) {
            auto r = dtype_range(n.dtype);
            sat = ", " + std::to_string(r.first) + ", " + std::to_string(r.second) + ")";
            if (n.dtype == WT_I32) sat.clear();  // 32-bit values never leave the type
        }
        if (n.kind == Kind::Pointwise) {
            std::string v = expr(n.expr, c, ch, k, e, ph);
            return sat.empty() ? v : "wt_sat(" + v + sat;
        }
        int p = n.srcs[0];
        int chp = src_chan(G(p), ch, -1);
        if (n.kind == Kind::Equalize) {  // the cumulative count of the value's bin, scaled
            const Node& h = P.nodes[n.srcs[1]];
            std::string v = read(c, p, chp, k, e, 0, 0, ph);
            if (isint(p)) v = "(float)" + v;
            const int tk = table_index(h.id), ts = geo.chan_parallel ? 0 : chp;
            const std::string lo = flit((double)(float)h.hlo), sc = flit((double)(float)(h.bins / (h.hhi - h.hlo)));
            return "((float)ht" + I(tk) + "[" + I(ts * h.bins) + " + wt_hist_bin(" + v + ", " + lo + ", " + sc + ", " +
                   I(h.bins) + ")] * rn" + I(tk) + "_" + I(ts) + ")";
        }
        if (n.is_int()) {
            // exact integer sum, quotient rounded half up, saturation
            std::string acc;
            for (int j = 0; j < n.kh; ++j)
                for (int i = 0; i < n.kw; ++i) {
                    long long w = n.iweights[(size_t)j * n.kw + i];
                    if (!w) continue;
                    std::string r = read(c, p, chp, k, e, i - n.ax, j - n.ay, ph);
                    std::string term = w == 1 ? r : "(" + std::to_string(w) + ") * " + r;
                    acc = acc.empty() ? term : acc + " + " + term;
                }
            if (acc.empty()) acc = "0";
            long long d = n.divisor;
            std::string q = "(" + acc + ")";
            if (d > 1) {
                int sh = 0;
                while ((1LL << sh) < d) ++sh;
                q = (1LL << sh) == d ? "wt_rshift(" + q + ", " + I(sh) + ")" : "wt_rdiv(" + q + ", " + std::to_string(d) + ")";
            }
            return sat.empty() ? q : "wt_sat(" + q + sat;
        }
        std::string acc;
        for (const Tap& t : P.taps(c, p)) {
            std::string r = read(c, p, chp, k, e, t.dx, t.dy, ph);
            if (acc.empty()) acc = flit(t.w) + " * " + r;
            else acc = "fmaf(" + flit(t.w) + ", " + r + ", " + acc + ")";
        }
        return acc;
    }

    std::string chan_off(int id, bool dst, int slot_idx, int ch) {
        const NodeGeom& n = G(id);
        std::string cs = std::string(dst ? "A.dst_cs[" : "A.src_cs[") + I(slot_idx) + "]";
        if (geo.chan_parallel) return P.nodes[id].channels == 1 ? "0" : "(long long)cp * " + cs;
        (void)n;
        return "(long long)" + I(ch) + " * " + cs;
    }

    // ------------------------------------------------------------ loads --
    // Row kk + lead of an up2 node read by expansion: every element is the
    // separable 2x expansion of the coarse source at the clamped fine point
    // (x first, then y: even index 2i -> (P(i-1) + 6 P(i) + P(i+1)) / 8, odd
    // 2i+1 -> (P(i) + P(i+1)) / 2, coarse indices clamped), gathered from the
    // coarse image (a quarter of the fine one, mostly served by the caches).
    // Expanded inputs in interior waves with one column per lane keep the
    // three coarse rows they blend (lane t: coarse column bc + t) in
    // registers across steps: the row index advances by at most one per
    // step, so each step loads only the lowest row and shifts the others
    // when the index has moved.
    bool coarse_ring(const NodeGeom& n) const { return !border && n.expand_src >= 0 && (V == 1 || V == 2 || V == 4); }
    // Even V: lane t of sub-tile k holds coarse columns bc_k + t*V/2 .. +V/2-1
    // (its fine columns' own coarse columns, one aligned-to-dword vector load
    // per coarse row); the columns just left and right of a sub-tile (for its
    // edge lanes) are ghosts every lane loads at one address.
    std::string cvec(int id, int ch, int k, char which) { return "xv" + I(id) + "_" + I(ch) + "_" + I(k) + which; }
    std::string cghost(int id, int ch, int k, char side, char which) {
        return "xg" + I(id) + "_" + I(ch) + "_" + I(k) + side + which;
    }
    // Emits the loads of coarse row `row` (an expression, already clamped)
    // for sub-tile k of an even-V ring into rows `which`.
    void load_coarse_even(const NodeGeom& n, int li, int ch, int k, const std::string& rowp, char which) {
        const int h = V / 2;
        const std::string bc = "((x0 + " + I(n.skew) + " + " + I(k * SUB) + ") >> 1)";
        if (h == 1) {
            line("  " + cvec(n.id, ch, k, which) + "[0] = (float)" + rowp + "[wt_clampi(" + bc + " + lane, 0, Wc - 1)];");
        } else if (n.mem_half) {
            line("  { const int c0 = " + bc + " + lane * 2;");
            line("    " + cvec(n.id, ch, k, which) + "[0] = (float)" + rowp + "[min(c0, Wc - 1)]; " +
                 cvec(n.id, ch, k, which) + "[1] = (float)" + rowp + "[min(c0 + 1, Wc - 1)]; }");
        } else {
            // interior waves: both coarse columns of every lane lie inside
            // the coarse row
            line("  { const wt_f2d q = *(const wt_f2d*)(" + rowp + " + " + bc + " + lane * 2); " +
                 cvec(n.id, ch, k, which) + "[0] = q[0]; " + cvec(n.id, ch, k, which) + "[1] = q[1]; }");
        }
        if (k == 0)
            line("  " + cghost(n.id, ch, k, 'l', which) + " = (float)" + rowp + "[wt_clampi(" + bc + " - 1, 0, Wc - 1)];");
        if (k == g.TX - 1)
            line("  " + cghost(n.id, ch, k, 'r', which) + " = (float)" + rowp + "[min(" + bc + " + " + I(64 * h) +
                 ", Wc - 1)];");
        (void)li;
    }
    std::string cring(int id, int ch, int k, char which) {
        return "xr" + I(id) + "_" + I(ch) + "_" + I(k) + which;
    }
    void prime_coarse_rings() {
        int li = 0;
        for (auto& n : geo.nodes) {
            if (n.member) continue;
            const int l = li++;
            if (!coarse_ring(n)) continue;
            const std::string ty = n.mem_half ? "_Float16" : "float";
            for (int ch = 0; ch < n.nch; ++ch)
                for (int k = 0; k < g.TX; ++k) {
                    if (V == 1) {
                        line("float " + cring(n.id, ch, k, 'p') + ", " + cring(n.id, ch, k, 'c') + ", " +
                             cring(n.id, ch, k, 'n') + ";");
                        continue;
                    }
                    for (char w : {'p', 'c', 'n'}) {
                        line("float " + cvec(n.id, ch, k, w) + "[" + I(V / 2) + "];");
                        if (k == 0) line("float " + cghost(n.id, ch, k, 'l', w) + ";");
                        if (k == g.TX - 1) line("float " + cghost(n.id, ch, k, 'r', w) + ";");
                    }
                }
            line("int xj" + I(n.id) + ";  // coarse row held in the middle of node " + I(n.id) + "'s ring");
            line("{ const int Wc = (W + 1) >> 1, Hc = (H + 1) >> 1;");
            line("  const int jf = wt_clampi(y0 - " + I(geo.D - n.first_step) + " + " + I(n.lead) + ", 0, H - 1) >> 1;");
            line("  xj" + I(n.id) + " = jf;");
            for (int ch = 0; ch < n.nch; ++ch) {
                line("  { const " + ty + "* cb = (const " + ty + "*)A.src[" + I(l) + "] + " + chan_off(n.id, false, l, ch) + ";");
                line("    const " + ty + "* r0 = cb + (long long)wt_clampi(jf - 1, 0, Hc - 1) * A.src_rs[" + I(l) + "];");
                line("    const " + ty + "* r1 = cb + (long long)jf * A.src_rs[" + I(l) + "];");
                line("    const " + ty + "* r2 = cb + (long long)min(jf + 1, Hc - 1) * A.src_rs[" + I(l) + "];");
                if (V > 1) {
                    for (int k = 0; k < g.TX; ++k) {
                        load_coarse_even(n, l, ch, k, "r0", 'p');
                        load_coarse_even(n, l, ch, k, "r1", 'c');
                        load_coarse_even(n, l, ch, k, "r2", 'n');
                    }
                    line("  }");
                    continue;
                }
                for (int k = 0; k < g.TX; ++k) {
                    line("    { const int cl = wt_clampi(((x0 + " + I(n.skew) + " + " + I(k * SUB) + ") >> 1) - 1 + lane, 0, Wc - 1);");
                    line("      " + cring(n.id, ch, k, 'p') + " = (float)r0[cl];");
                    line("      " + cring(n.id, ch, k, 'c') + " = (float)r1[cl];");
                    line("      " + cring(n.id, ch, k, 'n') + " = (float)r2[cl]; }");
                }
                line("  }");
            }
            line("}");
        }
    }
    void emit_expand_load(int li, const NodeGeom& n, int ph) {
        const std::string ty = n.mem_half ? "_Float16" : "float";
        int slot = pmod(ph, n.win);
        if (coarse_ring(n)) {
            line("const bool adv" + I(n.id) + " = (wt_clampi(kk + " + I(n.lead) + ", 0, H - 1) >> 1) != xj" + I(n.id) + ";");
            line("xj" + I(n.id) + " = wt_clampi(kk + " + I(n.lead) + ", 0, H - 1) >> 1;");
        }
        for (int ch = 0; ch < n.nch; ++ch) {
            line("{  // expand node " + I(n.expand_src) + " into node " + I(n.id) + " channel slot " + I(ch) +
                 ", row kk + " + I(n.lead));
            ind += "    ";
            line("const int Wc = (W + 1) >> 1, Hc = (H + 1) >> 1;");
            line("const int yr = wt_clampi(kk + " + I(n.lead) + ", 0, H - 1);");
            line("const int jr = yr >> 1;");
            line("const float wy0 = (yr & 1) ? 0.0f : 0.125f, wy1 = (yr & 1) ? 0.5f : 0.75f, wy2 = (yr & 1) ? 0.5f : 0.125f;");
            line("const " + ty + "* cb = (const " + ty + "*)A.src[" + I(li) + "] + " + chan_off(n.id, false, li, ch) + ";");
            line("const " + ty + "* r0 = cb + (long long)wt_clampi(jr - 1, 0, Hc - 1) * A.src_rs[" + I(li) + "];");
            line("const " + ty + "* r1 = cb + (long long)min(jr, Hc - 1) * A.src_rs[" + I(li) + "];");
            line("const " + ty + "* r2 = cb + (long long)min(jr + 1, Hc - 1) * A.src_rs[" + I(li) + "];");
            // even V, interior wave: advance the ring, load the lowest coarse
            // row, blend the three rows per coarse column; fine column 2c
            // takes 1/8, 3/4, 1/8 of coarse columns c-1, c, c+1 and 2c+1
            // half of c and c+1, the neighbours of a lane's edge columns
            // coming from the next lanes by DPP (the sub-tile's edge lanes
            // from the neighbouring sub-tile or the ghosts)
            std::vector<std::vector<std::string>> ev;  // [k][e] fine values
            if (coarse_ring(n) && V > 1) {
                const int h = V / 2;
                std::vector<std::vector<std::string>> q(g.TX, std::vector<std::string>(h));
                std::string ql, qr;
                auto blend = [&](const std::string& P, const std::string& C, const std::string& N) {
                    std::string t = fresh("q");
                    line("const float " + t + " = fmaf(wy2, " + N + ", fmaf(wy1, " + C + ", wy0 * " + P + "));");
                    return t;
                };
                const std::string a = "adv" + I(n.id);
                for (int k = 0; k < g.TX; ++k) {
                    for (int m = 0; m < h; ++m) {
                        const std::string P = cvec(n.id, ch, k, 'p') + "[" + I(m) + "]",
                                          C = cvec(n.id, ch, k, 'c') + "[" + I(m) + "]",
                                          N = cvec(n.id, ch, k, 'n') + "[" + I(m) + "]";
                        line(P + " = " + a + " ? " + C + " : " + P + ";");
                        line(C + " = " + a + " ? " + N + " : " + C + ";");
                    }
                    for (char side : {'l', 'r'}) {
                        if ((side == 'l' && k != 0) || (side == 'r' && k != g.TX - 1)) continue;
                        const std::string P = cghost(n.id, ch, k, side, 'p'), C = cghost(n.id, ch, k, side, 'c'),
                                          N = cghost(n.id, ch, k, side, 'n');
                        line(P + " = " + a + " ? " + C + " : " + P + ";");
                        line(C + " = " + a + " ? " + N + " : " + C + ";");
                    }
                    load_coarse_even(n, li, ch, k, "r2", 'n');
                    for (int m = 0; m < h; ++m)
                        q[k][m] = blend(cvec(n.id, ch, k, 'p') + "[" + I(m) + "]", cvec(n.id, ch, k, 'c') + "[" + I(m) + "]",
                                        cvec(n.id, ch, k, 'n') + "[" + I(m) + "]");
                    if (k == 0)
                        ql = blend(cghost(n.id, ch, k, 'l', 'p'), cghost(n.id, ch, k, 'l', 'c'), cghost(n.id, ch, k, 'l', 'n'));
                    if (k == g.TX - 1)
                        qr = blend(cghost(n.id, ch, k, 'r', 'p'), cghost(n.id, ch, k, 'r', 'c'), cghost(n.id, ch, k, 'r', 'n'));
                }
                ev.assign(g.TX, std::vector<std::string>(V));
                for (int k = 0; k < g.TX; ++k) {
                    std::string L = fresh("ql"), R = fresh("qr");
                    if (k > 0)
                        line("const float " + L + " = wt_shift1(" + q[k][h - 1] + ", " + q[k - 1][h - 1] + ");");
                    else
                        line("const float " + L + " = wt_shr1(" + q[k][h - 1] + ", " + ql + ");");
                    if (k + 1 < g.TX)
                        line("const float " + R + " = wt_shift1n(" + q[k][0] + ", " + q[k + 1][0] + ");");
                    else
                        line("const float " + R + " = wt_shl1(" + q[k][0] + ", " + qr + ");");
                    for (int e = 0; e < V; ++e) {
                        const int m = e / 2;
                        const std::string qa = m > 0 ? q[k][m - 1] : L, qb = m + 1 < h ? q[k][m + 1] : R;
                        ev[k][e] = e % 2 == 0 ? "fmaf(0.125f, " + qb + ", fmaf(0.75f, " + q[k][m] + ", 0.125f * " + qa + "))"
                                              : "fmaf(0.5f, " + qb + ", 0.5f * " + q[k][m] + ")";
                    }
                }
            }
            for (int k = 0; k < g.TX; ++k) {
                std::vector<std::string> dst;
                std::string v;
                if (k >= SX) {
                    for (int e = 0; e < V; ++e) dst.push_back(reg(n.id, slot, ch, k - SX, e));
                } else {
                    v = fresh("ld");
                    line("float " + v + "[" + I(V) + "];");
                    for (int e = 0; e < V; ++e) dst.push_back(v + "[" + I(e) + "]");
                }
                if (coarse_ring(n) && V > 1) {
                    for (int e = 0; e < V; ++e) line(dst[e] + " = " + ev[k][e] + ";");
                    if (k < SX) emit_lds_store(n, slot, ch, k, v);
                    continue;
                }
                if (coarse_ring(n)) {
                    // interior wave, one column per lane: lane t holds coarse
                    // column bc + t of the three coarse rows in its ring (one
                    // new row loaded per step), blends them vertically, forms
                    // both horizontal phases with its DPP neighbours (even:
                    // 1/8, 3/4, 1/8 of columns c-1, c, c+1; odd: 1/2, 1/2 of
                    // c, c+1), and each lane picks its phase of column x/2
                    // from lane x/2 - bc through the LDS crossbar
                    const std::string P = cring(n.id, ch, k, 'p'), C = cring(n.id, ch, k, 'c'), N = cring(n.id, ch, k, 'n');
                    line("{ const int xs0 = x0 + " + I(n.skew) + " + " + I(k * SUB) + ";");
                    line("  const int bc = (xs0 >> 1) - 1;");
                    line("  const int cl = wt_clampi(bc + lane, 0, Wc - 1);");
                    line("  const float nl = (float)r2[cl];");
                    line("  " + P + " = adv" + I(n.id) + " ? " + C + " : " + P + ";");
                    line("  " + C + " = adv" + I(n.id) + " ? " + N + " : " + C + ";");
                    line("  " + N + " = nl;");
                    line("  const float q = fmaf(wy2, " + N + ", fmaf(wy1, " + C + ", wy0 * " + P + "));");
                    line("  const float qm = wt_mov_shr1(q), qp = wt_mov_shl1(q);");
                    line("  const float ev = fmaf(0.125f, qp, fmaf(0.75f, q, 0.125f * qm));");
                    line("  const float od = fmaf(0.5f, qp, 0.5f * q);");
                    line("  const int x = xs0 + lane;");
                    line("  const int sa = (((x >> 1) - bc) & 63) << 2;");
                    line("  const float e2 = wt_bperm(sa, ev), o2 = wt_bperm(sa, od);");
                    line("  " + dst[0] + " = (x & 1) ? o2 : e2;");
                    line("}");
                    if (k < SX) emit_lds_store(n, slot, ch, k, v);
                    continue;
                }
                if (!border && V % 2 == 0) {
                    // interior wave, even V: a lane's first column is even
                    // (tile origins, skews and sub-tile widths are multiples
                    // of V), so its V columns share coarse columns
                    // ib-1 .. ib+V/2 (V/2 + 2 loads per coarse row instead
                    // of 3 per column) and each column's parity, hence its
                    // horizontal weights, is known here
                    const int nc = V / 2 + 2;
                    line("{ const int ib = (x0 + " + I(n.skew) + " + " + I(k * SUB) + " + lane * " + I(V) + ") >> 1;");
                    for (int c = 0; c < nc; ++c)
                        line("  const int xc" + I(c) + " = wt_clampi(ib + " + I(c - 1) + ", 0, Wc - 1);");
                    const char* rows[3] = {"r0", "r1", "r2"};
                    for (int r = 0; r < 3; ++r)
                        for (int c = 0; c < nc; ++c)
                            line("  const float c" + I(r) + "_" + I(c) + " = (float)" + rows[r] + "[xc" + I(c) + "];");
                    for (int e = 0; e < V; ++e) {
                        const int m = e / 2;
                        std::string h[3];
                        for (int r = 0; r < 3; ++r) {
                            std::string a = "c" + I(r) + "_" + I(m), b = "c" + I(r) + "_" + I(m + 1),
                                        cc = "c" + I(r) + "_" + I(m + 2);
                            h[r] = (e % 2 == 0) ? "fmaf(0.125f, " + cc + ", fmaf(0.75f, " + b + ", 0.125f * " + a + "))"
                                                : "fmaf(0.5f, " + cc + ", 0.5f * " + b + ")";
                        }
                        line("  " + dst[e] + " = fmaf(wy2, " + h[2] + ", fmaf(wy1, " + h[1] + ", wy0 * " + h[0] + "));");
                    }
                    line("}");
                    if (k < SX) emit_lds_store(n, slot, ch, k, v);
                    continue;
                }
                for (int e = 0; e < V; ++e) {
                    line("{ const int xf = wt_clampi(x0 + " + I(n.skew) + " + " + I(k * SUB) + " + lane * " + I(V) +
                         " + " + I(e) + ", 0, W - 1);");
                    line("  const int i = xf >> 1;");
                    line("  const int xa = wt_clampi(i - 1, 0, Wc - 1), xb = min(i, Wc - 1), xc = min(i + 1, Wc - 1);");
                    line("  const float wx0 = (xf & 1) ? 0.0f : 0.125f, wx1 = (xf & 1) ? 0.5f : 0.75f, "
                         "wx2 = (xf & 1) ? 0.5f : 0.125f;");
                    line("  const float h0 = fmaf(wx2, (float)r0[xc], fmaf(wx1, (float)r0[xb], wx0 * (float)r0[xa]));");
                    line("  const float h1 = fmaf(wx2, (float)r1[xc], fmaf(wx1, (float)r1[xb], wx0 * (float)r1[xa]));");
                    line("  const float h2 = fmaf(wx2, (float)r2[xc], fmaf(wx1, (float)r2[xb], wx0 * (float)r2[xa]));");
                    line("  " + dst[e] + " = fmaf(wy2, h2, fmaf(wy1, h1, wy0 * h0));");
                    line("}");
                }
                if (k < SX) emit_lds_store(n, slot, ch, k, v);
            }
            ind.resize(ind.size() - 4);
            line("}");
        }
        if (SX > 0) line("wt_wave_sync();");
    }

    void emit_load(int li, const NodeGeom& n, int ph) {
        if (n.expand_src >= 0) return emit_expand_load(li, n, ph);
        const std::string ty = mtype(n), ct = ctype(n.id);
        int slot = pmod(ph, n.win);
        for (int ch = 0; ch < n.nch; ++ch) {
            line("{  // load node " + I(n.id) + " channel slot " + I(ch) + ", row kk + " + I(n.lead));
            ind += "    ";
            line("const int yr = wt_clampi(kk + " + I(n.lead) + ", 0, H - 1);");
            line("const " + ty + "* rp = (const " + ty + "*)A.src[" + I(li) + "] + " +
                 chan_off(n.id, false, li, ch) + " + (long long)yr * A.src_rs[" + I(li) + "];");
            for (int k = 0; k < g.TX; ++k) {
                // VGPR sub-tiles load straight into their ring registers (no
                // copy, so the wait for the load falls at its first use);
                // LDS sub-tiles go through a temporary.
                std::vector<std::string> dst;
                std::string v;
                if (k >= SX) {
                    for (int e = 0; e < V; ++e) dst.push_back(reg(n.id, slot, ch, k - SX, e));
                } else {
                    v = fresh("ld");
                    line(ct + " " + v + "[" + I(V) + "];");
                    for (int e = 0; e < V; ++e) dst.push_back(v + "[" + I(e) + "]");
                }
                std::string xb = "x0 + " + I(n.skew) + " + " + I(k * SUB) + " + lane * " + I(V);
                line("{ const int xb = " + xb + ";");
                if (!border) {
                    std::string ld0 = g.NT ? "__builtin_nontemporal_load(rp + xb)" : "rp[xb]";
                    if (V == 1) line("  " + dst[0] + " = (" + ct + ")" + ld0 + ";");
                    else {
                        std::string vt = gvec(ty, V);
                        if (g.NT)
                            line("  const " + vt + " q = __builtin_nontemporal_load((const " + vt + "*)(rp + xb));");
                        else
                            line("  const " + vt + " q = *(const " + vt + "*)(rp + xb);");
                        for (int e = 0; e < V; ++e) line("  " + dst[e] + " = (" + ct + ")q[" + I(e) + "];");
                    }
                } else {
                    for (int e = 0; e < V; ++e)
                        line("  " + dst[e] + " = (" + ct + ")rp[wt_clampi(xb + " + I(e) + ", 0, W - 1)];");
                }
                line("}");
                if (k < SX) emit_lds_store(n, slot, ch, k, v);
            }
            if (n.ghl > 0) emit_ghost_load(li, n, true, slot, ch, ty, ct);
            if (n.ghr > 0) emit_ghost_load(li, n, false, slot, ch, ty, ct);
            ind.resize(ind.size() - 4);
            line("}");
        }
        if (SX > 0) line("wt_wave_sync();");
    }

    // Ghost columns of a loaded row.  Every lane loads (lanes outside the
    // ghost lanes repeat the nearest ghost lane's address, so the load stays
    // within one or two cache lines and needs no branch); interior waves read
    // in-bounds columns, border waves clamp each column like the main load.
    // (Range-checked buffer loads with only the ghost lanes in range measured
    // slower on gfx950 than these replicated-address loads.)
    void emit_ghost_load(int li, const NodeGeom& n, bool left, int slot, int ch, const std::string& ty,
                         const std::string& ct) {
        (void)li;
        const int nl = left ? ghost_lanes_l(n) : ghost_lanes_r(n);
        std::string xg;
        if (nl == 1)  // one lane, placed where the one-lane shift reads it
            xg = left ? "x0 + " + I(n.skew) + " - " + I(V) : "x0 + " + I(n.skew) + " + " + I(g.TX * SUB);
        else
            xg = left ? "x0 + " + I(n.skew) + " - (64 - max(lane, " + I(64 - nl) + ")) * " + I(V)
                      : "x0 + " + I(n.skew) + " + " + I(g.TX * SUB) + " + min(lane, " + I(nl - 1) + ") * " + I(V);
        line("{ const int xg = " + xg + ";  // ghost columns " + std::string(left ? "left" : "right"));
        std::vector<std::string> dst;
        for (int e = 0; e < V; ++e) dst.push_back(ghost(n.id, left, slot, ch, e));
        if (!border) {
            if (V == 1) line("  " + dst[0] + " = (" + ct + ")rp[xg];");
            else {
                std::string vt = gvec(ty, V);
                line("  const " + vt + " q = *(const " + vt + "*)(rp + xg);");
                for (int e = 0; e < V; ++e) line("  " + dst[e] + " = (" + ct + ")q[" + I(e) + "];");
            }
        } else {
            for (int e = 0; e < V; ++e)
                line("  " + dst[e] + " = (" + ct + ")rp[wt_clampi(xg + " + I(e) + ", 0, W - 1)];");
        }
        line("}");
    }

    void emit_lds_store(const NodeGeom& n, int slot, int ch, int k, const std::string& arr) {
        std::string j = I(k * SUB) + " + lane * " + I(V);
        std::string base = "&" + lidx(n.id, slot, ch, j);
        if (n.half) {
            if (V == 1) line(base.substr(1) + " = (_Float16)" + arr + "[0];");
            else {
                std::string vt = V == 4 ? "wt_h4" : "wt_h2";
                std::string init;
                for (int e = 0; e < V; ++e) init += (e ? ", " : "") + std::string("(_Float16)") + arr + "[" + I(e) + "]";
                line("*(" + vt + "*)(" + base + ") = " + vt + "{" + init + "};");
            }
        } else {
            if (V == 1) line(base.substr(1) + " = " + arr + "[0];");
            else {
                std::string vt = vec(ctype(n.id), V);
                std::string init;
                for (int e = 0; e < V; ++e) init += (e ? ", " : "") + arr + "[" + I(e) + "]";
                line("*(" + vt + "*)(" + base + ") = " + vt + "{" + init + "};");
            }
        }
    }

    // ----------------------------------------------------------- stores --
    // Live-out row stored with buffer stores: rows and columns outside the
    // tile's output range get an offset past the buffer's end, which the
    // hardware discards, so no branch (and no conservative s_waitcnt at a
    // control-flow merge) surrounds the store.
    void emit_store(int oi, const NodeGeom& n, int ch, int k, const std::string& arr, const std::string& R) {
        std::string rsrc = "S" + I(oi) + "_" + I(ch);
        const std::string aux = g.NT ? "WT_CPOL_NT" : "0";
        int esz = msize(n);
        line("{ const int jb = " + I(k * SUB) + " + lane * " + I(V) + ";");
        line("  const int xp = x0 + " + I(n.skew) + " + jb;");
        line("  const bool ok = " + R + " >= y0 && " + R + " < kend && " + R + " < H && jb >= " + I(geo.S0) +
             " && jb < " + I(geo.S0 + geo.X) + ";");
        line("  const int ob = (int)(((long long)" + R + " * A.dst_rs[" + I(oi) + "] + xp) * " + I(esz) + ");");
        if (isint(n.id)) {
            // integer live-out: values are already saturated to the type
            const std::string mt = mtype(n);
            if (!border) {
                line("  const int off = ok ? ob : WT_OOB;");
                std::string v;
                if (V == 1) v = "(" + mt + ")" + arr + "[0]";
                else {
                    std::string vals;
                    for (int e = 0; e < V; ++e) vals += (e ? ", " : "") + std::string("(") + mt + ")" + arr + "[" + I(e) + "]";
                    v = vec(mt, V) + "{" + vals + "}";
                }
                line("  " + store_fn(V * esz) + "(__builtin_bit_cast(" + store_ty(V * esz) + ", " + v + "), " + rsrc +
                     ", off, 0, " + aux + ");");
            } else {
                for (int e = 0; e < V; ++e) {
                    line("  { const int off = (ok && xp + " + I(e) + " >= 0 && xp + " + I(e) + " < W) ? ob + " +
                         I(e * esz) + " : WT_OOB;");
                    line("    " + store_fn(esz) + "(__builtin_bit_cast(" + store_ty(esz) + ", (" + mt + ")" + arr + "[" +
                         I(e) + "]), " + rsrc + ", off, 0, " + aux + "); }");
                }
            }
        } else if (!border) {
            line("  const int off = ok ? ob : WT_OOB;");
            if (n.mem_half) {
                std::string vals;
                for (int e = 0; e < V; ++e) vals += (e ? ", " : "") + std::string("(_Float16)") + arr + "[" + I(e) + "]";
                if (V == 1) line("  __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, (_Float16)" + arr + "[0]), " + rsrc + ", off, 0, " + aux + ");");
                else if (V == 2) line("  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, wt_h2{" + vals + "}), " + rsrc + ", off, 0, " + aux + ");");
                else line("  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(wt_u2, wt_h4{" + vals + "}), " + rsrc + ", off, 0, " + aux + ");");
            } else {
                std::string vals;
                for (int e = 0; e < V; ++e) vals += (e ? ", " : "") + arr + "[" + I(e) + "]";
                if (V == 1) line("  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, " + arr + "[0]), " + rsrc + ", off, 0, " + aux + ");");
                else if (V == 2) line("  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(wt_u2, wt_f2{" + vals + "}), " + rsrc + ", off, 0, " + aux + ");");
                else line("  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(wt_u4, wt_f4{" + vals + "}), " + rsrc + ", off, 0, " + aux + ");");
            }
        } else {
            for (int e = 0; e < V; ++e) {
                line("  { const int off = (ok && xp + " + I(e) + " >= 0 && xp + " + I(e) + " < W) ? ob + " + I(e * esz) +
                     " : WT_OOB;");
                if (n.mem_half)
                    line("    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, (_Float16)" + arr + "[" +
                         I(e) + "]), " + rsrc + ", off, 0, " + aux + "); }");
                else
                    line("    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, " + arr + "[" + I(e) +
                         "]), " + rsrc + ", off, 0, " + aux + "); }");
            }
        }
        line("}");
    }

    // Element size in memory of decimated output k (a down2 of a member).
    int dec_size(size_t k) const {
        int d = geo.dec[k].first;
        return P.nodes[d].is_int() ? dtype_size(P.nodes[d].dtype) : (dec_half(k) ? 2 : 4);
    }
    bool dec_half(size_t k) const {
        int d = geo.dec[k].first;
        return g.fp16 && P.half_storable(d) && !P.is_output(d);
    }
    // Decimated store of a member row (down2 fused into its producer): on
    // even rows, the elements at even x go to (x/2, r/2) of the down2 node;
    // every other element's offset is past the buffer, so the hardware drops
    // it (no branch).
    void emit_dec_store(size_t k, const NodeGeom& n, int ch, int kk, const std::string& arr, const std::string& R) {
        int oi = (int)(geo.liveouts.size() + k);
        std::string rsrc = "S" + I(oi) + "_" + I(ch);
        const std::string aux = g.NT ? "WT_CPOL_NT" : "0";
        int esz = dec_size(k);
        int d = geo.dec[k].first;
        std::string mt = P.nodes[d].is_int() ? dtype_ctype(P.nodes[d].dtype) : (dec_half(k) ? "_Float16" : "float");
        line("{ const int jb = " + I(kk * SUB) + " + lane * " + I(V) + ";");
        line("  const int xp = x0 + " + I(n.skew) + " + jb;");
        line("  const bool okd = (" + R + " & 1) == 0 && " + R + " >= y0 && " + R + " < kend && " + R +
             " < H && jb >= " + I(geo.S0) + " && jb < " + I(geo.S0 + geo.X) + ";");
        line("  const long long rb = (long long)(" + R + " >> 1) * A.dst_rs[" + I(oi) + "];");
        for (int e = 0; e < V; ++e) {
            std::string x = "(xp + " + I(e) + ")";
            line("  { const int off = (okd && (" + x + " & 1) == 0 && " + x + " >= 0 && " + x + " < W) ? (int)((rb + (" + x +
                 " >> 1)) * " + I(esz) + ") : WT_OOB;");
            line("    " + store_fn(esz) + "(__builtin_bit_cast(" + store_ty(esz) + ", (" + mt + ")" + arr + "[" + I(e) +
                 "]), " + rsrc + ", off, 0, " + aux + "); }");
        }
        line("}");
    }

    // ------------------------------------------------------- histograms --
    // Each wave counts into bins of its own in LDS (hb: every histogram of
    // the group, R copies of its bins for all channel slots, one after
    // another); the tile's counts, summed over the copies, are added to the
    // device-wide output once, at its end.
    int hist_words(size_t k) const { return P.nodes[geo.hist[k].first].bins * G(geo.hist[k].second).nch; }
    // words of histogram k's copies in the wave's LDS bins
    int hist_span(size_t k) const { return (hist_words(k) + 1) * hist_replicas(hist_words(k)); }
    int hist_off(size_t k) const {
        int o = 0;
        for (size_t i = 0; i < k; ++i) o += (hist_span(i) + 3) / 4 * 4;
        return o;
    }
    int hist_oi(size_t k) const { return (int)(geo.liveouts.size() + geo.dec.size() + k); }
    // Counts the values of member n at row R that belong to this tile's
    // output range and to the image, into the lane's copy of the bins.
    void emit_hist(size_t k, const NodeGeom& n, int ch, int kk, const std::string& arr, const std::string& R) {
        const Node& h = P.nodes[geo.hist[k].first];
        const int rep = hist_replicas(hist_words(k));
        const std::string lo = flit((double)(float)h.hlo), sc = flit((double)(float)(h.bins / (h.hhi - h.hlo)));
        const std::string base = "hb + " + I(hist_off(k) + ch * h.bins) + " + (lane & " + I(rep - 1) + ") * " +
                                 I(hist_words(k) + 1);
        line("{ const int jb = " + I(kk * SUB) + " + lane * " + I(V) + ";");
        line("  const int xp = x0 + " + I(n.skew) + " + jb;");
        line("  const bool okh = " + R + " >= y0 && " + R + " < kend && " + R + " < H && jb >= " + I(geo.S0) +
             " && jb < " + I(geo.S0 + geo.X) + ";");
        for (int e = 0; e < V; ++e) {
            // the value as the group holds it (FP16 rows are rounded)
            std::string v = arr + "[" + I(e) + "]";
            if (isint(n.id)) v = "(float)" + v;
            else if (n.half) v = "(float)(_Float16)" + v;
            line("  if (okh && xp + " + I(e) + " >= 0 && xp + " + I(e) + " < W) wt_count_lds(" + base +
                 " + wt_hist_bin(" + v + ", " + lo + ", " + sc + ", " + I(h.bins) + "), 1u);");
        }
        line("}");
    }
    // ----------------------------------------------------- equalize tables --
    // A histogram an equalize member reads is loaded whole at the start of
    // each tile and turned into cumulative counts in the wave's LDS: each
    // lane sums a run of consecutive bins, the lanes' totals are added up
    // for the lanes above them, and rn<k>_<slot> = 1 / total (0 for an empty
    // histogram).
    int table_index(int h) const {
        for (size_t i = 0; i < geo.tables.size(); ++i)
            if (geo.tables[i] == h) return (int)i;
        fail(WT_E_INTERNAL, "equalize table not in the group");
        return -1;
    }
    int table_off(size_t k) const {
        int o = 0;
        for (size_t i = 0; i < k; ++i) {
            const Node& h = P.nodes[geo.tables[i]];
            o += (h.bins * (geo.chan_parallel ? 1 : h.channels) + 3) / 4 * 4;
        }
        return o;
    }
    void emit_tables() {
        if (geo.tables.empty()) return;
        const std::string scr = "(tb + " + I(table_off(geo.tables.size())) + ")";
        line("wt_wave_sync();  // a previous tile of this wave may still be reading the tables");
        for (size_t k = 0; k < geo.tables.size(); ++k) {
            const Node& h = P.nodes[geo.tables[k]];
            const int si = (int)geo.loaded.size() + (int)k, nch = geo.chan_parallel ? 1 : h.channels;
            const int cnk = (h.bins + 63) / 64;
            line("unsigned int* ht" + I((int)k) + " = tb + " + I(table_off(k)) + ";");
            for (int ch = 0; ch < nch; ++ch) {
                std::string coff = geo.chan_parallel ? (h.channels == 1 ? "0" : "(long long)cp * A.src_cs[" + I(si) + "]")
                                                     : "(long long)" + I(ch) + " * A.src_cs[" + I(si) + "]";
                const std::string T = "ht" + I((int)k) + " + " + I(ch * h.bins);
                line("float rn" + I((int)k) + "_" + I(ch) + ";");
                line("{ const unsigned int* cnt = (const unsigned int*)A.src[" + I(si) + "] + " + coff + ";");
                line("  unsigned int* T = " + T + ";");
                line("  unsigned int run = 0u;");
                line("  for (int i = 0; i < " + I(cnk) + "; ++i) { const int b = lane * " + I(cnk) +
                     " + i; if (b < " + I(h.bins) + ") { run += cnt[b]; T[b] = run; } }");
                line("  " + scr + "[lane] = run;");
                line("  wt_wave_sync();");
                line("  unsigned int below = 0u;");
                line("  for (int j = 0; j < lane; ++j) below += " + scr + "[j];");
                line("  for (int i = 0; i < " + I(cnk) + "; ++i) { const int b = lane * " + I(cnk) +
                     " + i; if (b < " + I(h.bins) + ") T[b] += below; }");
                line("  wt_wave_sync();");
                line("  const unsigned int tot = T[" + I(h.bins - 1) + "];");
                line("  rn" + I((int)k) + "_" + I(ch) + " = tot ? 1.0f / (float)tot : 0.0f; }");
            }
        }
    }
    void emit_hist_clear() {
        if (geo.hist.empty()) return;
        line("wt_wave_sync();");
        line("for (int i = lane; i < " + I(hist_off(geo.hist.size())) + "; i += 64) hb[i] = 0u;");
        line("wt_wave_sync();");
    }
    void emit_hist_flush() {
        if (geo.hist.empty()) return;
        line("wt_wave_sync();");
        for (size_t k = 0; k < geo.hist.size(); ++k) {
            const Node& h = P.nodes[geo.hist[k].first];
            const int oi = hist_oi(k), rep = hist_replicas(hist_words(k)), stride = hist_words(k) + 1;
            for (int ch = 0; ch < G(geo.hist[k].second).nch; ++ch) {
                line("for (int i = lane; i < " + I(h.bins) + "; i += 64) {");
                line("    const unsigned int* q = hb + " + I(hist_off(k) + ch * h.bins) + " + i;");
                std::string sum = "q[0]";
                for (int r = 1; r < rep; ++r) sum += " + q[" + I(r * stride) + "]";
                line("    const unsigned int c = " + sum + ";");
                line("    if (c) wt_count_global((unsigned int*)A.dst[" + I(oi) + "] + " +
                     chan_off(geo.hist[k].second, true, oi, ch) + " + i, c);");
                line("}");
            }
        }
    }

    // ----------------------------------------------------- clamp fix-ups --
    // Positions of a stage row outside [0, W) take the value at x = 0 / W-1
    // (per-stage clamp to edge); only border waves execute this.
    void emit_fix_x(const NodeGeom& n, int slot) {
        line("{  // clamp node " + I(n.id) + " at the image's left/right edge");
        ind += "    ";
        line("const int j0 = -x0 - " + I(n.skew) + ";");
        line("const int jw = W - 1 - x0 - " + I(n.skew) + ";");
        for (int ch = 0; ch < n.nch; ++ch) {
            std::string e0 = fresh("edge"), ew = fresh("edge");
            line(ctype(n.id) + " " + e0 + " = 0, " + ew + " = 0;");
            for (int pass = 0; pass < 2; ++pass) {
                std::string j = pass ? "jw" : "j0", dst = pass ? ew : e0;
                line("if (" + j + " >= 0 && " + j + " < " + I(N) + ") {");
                line("  const int fk = " + j + " / " + I(SUB) + ", ft = (" + j + " % " + I(SUB) + ") / " + I(V) +
                     ", fe = " + j + " % " + I(V) + ";");
                if (SX > 0) line("  if (fk < " + I(SX) + ") " + dst + " = " + lread(n.id, slot, ch, j) + ";");
                for (int k = SX; k < g.TX; ++k)
                    for (int e = 0; e < V; ++e)
                        line("  if (fk == " + I(k) + " && fe == " + I(e) + ") " + dst + " = wt_readlane(" +
                             reg(n.id, slot, ch, k - SX, e) + ", ft);");
                line("}");
            }
            for (int k = 0; k < g.TX; ++k)
                for (int e = 0; e < V; ++e) {
                    std::string pos = "(x0 + " + I(n.skew) + " + " + I(k * SUB) + " + lane * " + I(V) + " + " + I(e) + ")";
                    if (k >= SX && packed(n.id)) {
                        std::string r = reg(n.id, slot, ch, k - SX, e);
                        line(preg(n.id, slot, ch, k - SX, e) + "[" + I(e % 2) + "] = (_Float16)(" + pos + " < 0 ? " +
                             e0 + " : (" + pos + " >= W ? " + ew + " : " + r + "));");
                    } else if (k >= SX) {
                        std::string r = reg(n.id, slot, ch, k - SX, e);
                        line(r + " = " + pos + " < 0 ? " + e0 + " : (" + pos + " >= W ? " + ew + " : " + r + ");");
                    } else {
                        std::string l = lidx(n.id, slot, ch, I(k * SUB) + " + lane * " + I(V) + " + " + I(e));
                        line("if (" + pos + " < 0) " + l + " = " + e0 + "; else if (" + pos + " >= W) " + l +
                             " = " + ew + ";");
                    }
                }
        }
        if (SX > 0) line("wt_wave_sync();");
        ind.resize(ind.size() - 4);
        line("}");
    }

    void copy_row(const NodeGeom& n, int from, int to) {
        for (int ch = 0; ch < n.nch; ++ch) {
            for (int kr = 0; kr < RX; ++kr)
                for (int e = 0; e < V; ++e) {
                    if (packed(n.id)) {
                        if (e % 2 == 0) line(preg(n.id, to, ch, kr, e) + " = " + preg(n.id, from, ch, kr, e) + ";");
                    } else {
                        line(reg(n.id, to, ch, kr, e) + " = " + reg(n.id, from, ch, kr, e) + ";");
                    }
                }
            for (int k = 0; k < SX; ++k)
                for (int e = 0; e < V; ++e) {
                    std::string j = I(k * SUB) + " + lane * " + I(V) + " + " + I(e);
                    line(lidx(n.id, to, ch, j) + " = " + lidx(n.id, from, ch, j) + ";");
                }
        }
    }

    // ----------------------------------------------------- folded up2 --
    // u = up2(down2(P)) computed from P's rows (P is a member whose down2
    // this group writes decimated).  Row r of u blends the even rows of P
    // around it: r even -> (P(r-2) + 6 P(r) + P(r+2)) / 8, r odd ->
    // (P(r-1) + P(r+1)) / 2; the same in x on the blended row.  A tap past
    // the last even row (column) of P -- 2*ceil(H/2)-2 -- takes the even row
    // (column) the coarse clamp selects: the centre tap for even points, the
    // lower tap for odd ones.  Taps before row (column) 0 read P's clamped
    // rows, which equal row (column) 0, as the coarse clamp at 0 does.
    void fold_weights(const NodeGeom& n, const std::string& R) {
        if (kpar >= 0)  // this step's row parity is known here
            line("const bool fo" + I(n.id) + " = " + ((kpar + n.lead) & 1 ? "true" : "false") + ";");
        else
            line("const bool fo" + I(n.id) + " = (" + R + " & 1) != 0;");
        line("const bool fc" + I(n.id) + " = " + R + " + 2 - (" + R + " & 1) > ((H + 1) >> 1) * 2 - 2;");
    }
    std::vector<std::vector<std::string>> fold_vertical(const NodeGeom& n, int ch, int ph) {
        const int src = P.fold_source(n.id);
        const int chp = src_chan(G(src), ch, -1);
        const std::string fo = "fo" + I(n.id), fc = "fc" + I(n.id);
        // blended at the producer's own slots (its skew relative to u)
        const int sk = G(src).skew - n.skew;
        std::vector<std::vector<std::string>> q(g.TX, std::vector<std::string>(V));
        for (int k = 0; k < g.TX; ++k)
            for (int e = 0; e < V; ++e) {
                std::string m2 = read(n.id, src, chp, k, e, sk, -2, ph), m1 = read(n.id, src, chp, k, e, sk, -1, ph),
                            c0 = read(n.id, src, chp, k, e, sk, 0, ph), p1 = read(n.id, src, chp, k, e, sk, 1, ph),
                            p2 = read(n.id, src, chp, k, e, sk, 2, ph);
                q[k][e] = memoize("(" + fo + " ? fmaf(0.5f, " + fc + " ? " + m1 + " : " + p1 + ", 0.5f * " + m1 +
                                  ") : fmaf(0.125f, " + fc + " ? " + c0 + " : " + p2 + ", fmaf(0.75f, " + c0 +
                                  ", 0.125f * " + m2 + ")))");
            }
        return q;
    }
    // Value of the blended row at element e + dx of sub-tile k: own lane,
    // or a neighbouring lane through a DPP shift (lanes past the tile's edge
    // belong to the overlap and take any value).
    std::string fold_read(const std::vector<std::vector<std::string>>& q, int k, int e, int dx) {
        int qq = e + dx;
        if (qq >= 0 && qq < V) return q[k][qq];
        if (qq < 0) {
            int d = (-qq + V - 1) / V, ep = qq + d * V;
            const std::string& cur = q[k][ep];
            const std::string& prv = k > 0 ? q[k - 1][ep] : cur;
            if (d == 1) return memoize(k > 0 ? "wt_shift1(" + cur + ", " + prv + ")" : "wt_mov_shr1(" + cur + ")");
            if (d == 2) return memoize("wt_shift2(" + cur + ", " + prv + ")");
            return memoize("wt_shiftd(" + cur + ", " + prv + ", " + I(d) + ", lane)");
        }
        int d = qq / V, ep = qq - d * V;
        const std::string& cur = q[k][ep];
        const std::string& nxt = k + 1 < g.TX ? q[k + 1][ep] : cur;
        if (d == 1) return memoize(k + 1 < g.TX ? "wt_shift1n(" + cur + ", " + nxt + ")" : "wt_mov_shl1(" + cur + ")");
        if (d == 2) return memoize("wt_shift2n(" + cur + ", " + nxt + ")");
        return memoize("wt_shiftdn(" + cur + ", " + nxt + ", " + I(d) + ", lane)");
    }
    std::string fold_horizontal(const NodeGeom& n, const std::vector<std::vector<std::string>>& q, int k, int e) {
        std::string x = memoize("(x0 + " + I(n.skew) + " + " + I(k * SUB) + " + lane * " + I(V) + " + " + I(e) + ")");
        const int sk = G(P.fold_source(n.id)).skew - n.skew;
        std::string m2 = fold_read(q, k, e, -2 - sk), m1 = fold_read(q, k, e, -1 - sk), c0 = fold_read(q, k, e, -sk),
                    p1 = fold_read(q, k, e, 1 - sk), p2 = fold_read(q, k, e, 2 - sk);
        // interior waves: every tap of a valid slot lies inside the image,
        // so the right-edge clamp never applies there
        std::string hi = border ? memoize("(" + x + " + 2 - (" + x + " & 1) > ((W + 1) >> 1) * 2 - 2)") : "false";
        return "((" + x + " & 1) ? fmaf(0.5f, " + hi + " ? " + m1 + " : " + p1 + ", 0.5f * " + m1 +
               ") : fmaf(0.125f, " + hi + " ? " + c0 + " : " + p2 + ", fmaf(0.75f, " + c0 + ", 0.125f * " + m2 + ")))";
    }

    // ----------------------------------------------------------- member --
    void emit_member(const NodeGeom& n, int ph, bool stores) {
        int slot = pmod(ph, n.win);
        if (n.even_rows && kpar >= 0 && ((kpar + n.lead) & 1)) {
            line("// stage " + I(n.id) + ": row kk + " + I(n.lead) + " is odd and never used");
            return;
        }
        line("// stage " + I(n.id) + ": row r = kk + " + I(n.lead));
        std::string R = "r" + I(n.id);
        line("const int " + R + " = kk + " + I(n.lead) + ";");
        int oi = -1;
        for (size_t i = 0; i < geo.liveouts.size(); ++i)
            if (geo.liveouts[i] == n.id) oi = (int)i;
        const bool folded = P.nodes[n.id].kind == Kind::Up2;
        if (folded) fold_weights(n, R);
        for (int ch = 0; ch < n.nch; ++ch) {
            std::vector<std::vector<std::string>> qv;
            if (folded) qv = fold_vertical(n, ch, ph);
            for (int k = 0; k < g.TX; ++k) {
                std::string arr = fresh("v");
                line(ctype(n.id) + " " + arr + "[" + I(V) + "];");
                for (int e = 0; e < V; ++e)
                    line(arr + "[" + I(e) + "] = " + (folded ? fold_horizontal(n, qv, k, e) : value(n.id, ch, k, e, ph)) + ";");
                if (n.consumed) {
                    if (k >= SX && packed(n.id)) {
                        for (int e = 0; e < V; e += 2)
                            line(preg(n.id, slot, ch, k - SX, e) + " = wt_h2{(_Float16)" + arr + "[" + I(e) +
                                 "], (_Float16)" + arr + "[" + I(e + 1) + "]};");
                    } else if (k >= SX) {
                        for (int e = 0; e < V; ++e)
                            line(reg(n.id, slot, ch, k - SX, e) + " = " + (n.half ? "wt_h(" + arr + "[" + I(e) + "])"
                                                                                  : arr + "[" + I(e) + "]") + ";");
                    } else {
                        emit_lds_store(n, slot, ch, k, arr);
                    }
                }
                if (oi >= 0 && stores) emit_store(oi, n, ch, k, arr, R);
                for (size_t d = 0; d < geo.dec.size(); ++d)
                    if (stores && geo.dec[d].second == n.id) emit_dec_store(d, n, ch, k, arr, R);
                for (size_t h = 0; h < geo.hist.size(); ++h)
                    if (stores && geo.hist[h].second == n.id) emit_hist(h, n, ch, k, arr, R);
            }
        }
        if (n.consumed && SX > 0) line("wt_wave_sync();");
        if (border && n.consumed && n.fix_x) emit_fix_x(n, slot);
        if (n.consumed && n.fix_top && n.win > 1) {
            line("if (" + R + " == 0) {  // rows above the image repeat row 0");
            ind += "    ";
            for (int s = 1; s < n.win; ++s) copy_row(n, slot, pmod(slot - s, n.win));
            if (SX > 0) line("wt_wave_sync();");
            ind.resize(ind.size() - 4);
            line("}");
        }
        if (n.consumed && n.fix_bot) {
            line("if (" + R + " >= H) {  // rows below the image repeat row H-1");
            ind += "    ";
            copy_row(n, pmod(slot - 1, n.win), slot);
            if (SX > 0) line("wt_wave_sync();");
            ind.resize(ind.size() - 4);
            line("}");
        }
    }

    bool border = false;

    // The whole streamed loop, for interior waves (vector loads and stores,
    // no clamping) or for border waves (clamped loads, masked stores, x
    // fix-ups).  Every path through one body issues the same memory
    // instructions, so the compiler's wait counts stay exact.
    // One streamed step: loads, then every member in topological order.
    // `pro` >= 0 marks prologue step `pro` (only nodes whose rows are already
    // needed are computed; stores only of rows inside the tile); `q` >= 0 is the output-row index of an
    // epilogue step (loads past the tile's last needed row are skipped).
    // Parity of the current step's kk when the generator knows it (tiles
    // start on even rows and the unrolled period is even), else -1.
    int kpar = -1;

    void emit_step(int ph, const std::string& kk, int pro, int q, int par = -1) {
        memo.clear();
        kpar = g.TY % 2 == 0 ? par : -1;
        line("{ const int kk = " + kk + ";");
        ind += "    ";
        // The group's last stage is followed by no sync, and it may read a
        // loaded node's LDS sub-tile across lanes; the loads below overwrite
        // such a sub-tile's oldest ring slot, so the previous step's reads
        // must be ordered before them.
        bool lds_loads = false;
        for (auto& n : geo.nodes) lds_loads |= !n.member && has_lds(n);
        if (lds_loads) line("wt_wave_sync();");
        int li = 0;
        for (auto& n : geo.nodes) {
            if (n.member) continue;
            bool on = (pro < 0 || n.first_step <= pro) && (q < 0 || q <= g.TY - 1 - g.PF);
            if (on) emit_load(li, n, ph);
            ++li;
        }
        // a consumed live-out leads the group's last stage, so its first
        // rows of the tile (row offset pro - D + lead >= 0) come out of the
        // warm-up steps and are stored there
        for (auto& n : geo.nodes)
            if (n.member && (pro < 0 || n.first_step <= pro)) emit_member(n, ph, pro < 0 || pro - geo.D + n.lead >= 0);
        ind.resize(ind.size() - 4);
        line("}");
    }

    // The whole streamed tile, for interior waves (vector loads and stores,
    // no clamping) or for border waves (clamped loads, masked stores, x
    // fix-ups).  Every path through one body issues the same memory
    // instructions, so the compiler's wait counts stay exact.
    void body(bool b) {
        border = b;
        ind += "    ";
        for (auto& n : geo.nodes) {
            if (packed(n.id))
                line("wt_h2 w" + I(n.id) + "[" + I(n.win) + "][" + I(n.nch) + "][" + I(RX) + "][" + I(V / 2) + "] = {};");
            else if (has_regs(n))
                line(ctype(n.id) + " w" + I(n.id) + "[" + I(n.win) + "][" + I(n.nch) + "][" + I(RX) + "][" + I(V) + "] = {};");
            if (n.ghl > 0)
                line(ctype(n.id) + " g" + I(n.id) + "l[" + I(n.win) + "][" + I(n.nch) + "][" + I(V) + "] = {};");
            if (n.ghr > 0)
                line(ctype(n.id) + " g" + I(n.id) + "r[" + I(n.win) + "][" + I(n.nch) + "][" + I(V) + "] = {};");
        }
        prime_coarse_rings();
        for (int s = 0; s < geo.D; ++s) emit_step(s % geo.U, "y0 - " + I(geo.D - s), s, -1, (geo.D - s) & 1);
        if (geo.NMAIN > 0) {
            line("for (int it = 0; it < " + I(geo.NMAIN) + "; ++it) {");
            ind += "    ";
            line("const int kb = y0 + it * " + I(geo.U) + ";");
            for (int j = 0; j < geo.U; ++j)
                emit_step((geo.D + j) % geo.U, "kb + " + I(j), -1, -1, geo.U % 2 == 0 ? j & 1 : -1);
            ind.resize(ind.size() - 4);
            line("}");
        }
        for (int j = 0; j < geo.E; ++j) {
            int qrow = geo.NMAIN * geo.U + j;
            emit_step((geo.D + j) % geo.U, "y0 + " + I(qrow), -1, qrow, qrow & 1);
        }
        ind.resize(ind.size() - 4);
    }

    int amax_ = 0, amin_ = 0;

    void header() {
        amax_ = 0;
        amin_ = 1 << 30;
        for (auto& n : geo.nodes) {
            amax_ = std::max(amax_, n.skew);
            amin_ = std::min(amin_, n.skew);
        }
        o << "// group: " << describe_group(g) << "\n";
        o << "// N=" << N << " X=" << geo.X << " S0=" << geo.S0 << " base=" << geo.base << " D=" << geo.D << " U=" << geo.U
          << " NMAIN=" << geo.NMAIN << " E=" << geo.E
          << " lds/wave=" << geo.lds_bytes << " chan_parallel=" << geo.chan_parallel << "\n";
        for (auto& n : geo.nodes)
            o << "//   node " << n.id << (n.member ? " member" : " loaded") << (n.liveout ? " liveout" : "")
              << " skew=" << n.skew << " lead=" << n.lead << " win=" << n.win << " nch=" << n.nch
              << " first=" << n.first_step << " vlo=" << n.vlo << " vhi=" << n.vhi << (n.half ? " fp16" : "")
              << (n.mem_half ? " mem-fp16" : "") << "\n";
    }

    // Index of this wave among all waves of the launch (wave-uniform, in an
    // SGPR).  Workgroups are dispatched round-robin over the 8 XCDs; with
    // XCD=1 each XCD gets a contiguous range of tiles so vertically adjacent
    // tiles (which share halo rows) run on one XCD and meet in its L2.
    void wave_index(const std::string& var) {
        if (g.XCD) {
            line("const int nb = gridDim.x, b = blockIdx.x;");
            line("const int xq = nb / WT_NXCD, xr = nb % WT_NXCD, xi = b % WT_NXCD;");
            line("const int lb = xi * xq + min(xi, xr) + b / WT_NXCD;");
            line("const int " + var + " = __builtin_amdgcn_readfirstlane(lb * " + I(g.WPB) + " + (threadIdx.x >> 6));");
        } else {
            line("const int " + var + " = __builtin_amdgcn_readfirstlane(blockIdx.x * " + I(g.WPB) +
                 " + (threadIdx.x >> 6));");
        }
    }

    void lds_decl() {
        if (geo.lds_bytes <= 0) return;
        line("__shared__ __attribute__((aligned(16))) char wt_lds[" + I(geo.lds_bytes_per_wg) + "];");
        line("char* lds = wt_lds + (threadIdx.x >> 6) * " + I(geo.lds_bytes) + ";");
        lds_ptrs();
    }

    // The nodes' LDS sub-tiles (and histogram bins, tables) in the wave's
    // LDS `lds`.
    void lds_ptrs() {
        if (geo.lds_bytes <= 0) return;
        if (!geo.hist.empty()) line("unsigned int* hb = (unsigned int*)(lds + " + I(geo.hist_lds_off) + ");");
        if (!geo.tables.empty()) line("unsigned int* tb = (unsigned int*)(lds + " + I(geo.table_lds_off) + ");");
        for (auto& n : geo.nodes)
            if (has_lds(n))
                line(std::string(n.half ? "_Float16" : ctype(n.id)) + "* L" + I(n.id) + " = (" +
                     (n.half ? "_Float16" : ctype(n.id)) + "*)(lds + " + I(n.lds_off) + ");");
    }

    // One wave tile `wid` of the image described by `A`.
    void tile() {
        if (g.ORD == 1) {  // horizontally adjacent tiles on consecutive waves
            line("const int tx = wid % A.tiles_x;");
            line("const int rr = wid / A.tiles_x;");
            line("const int ty = rr % A.tiles_y;");
            line("const int cp = rr / A.tiles_y;");
        } else {
            line("const int ty = wid % A.tiles_y;");
            line("const int rr = wid / A.tiles_y;");
            line("const int tx = rr % A.tiles_x;");
            line("const int cp = rr / A.tiles_x;");
        }
        line("(void)cp;");
        line("const int W = A.W, H = A.H;");
        line("const int x0 = tx * " + I(geo.X) + " + (" + I(geo.base) + ");");
        line("const int y0 = ty * " + I(g.TY) + ";");
        line("const int kend = y0 + " + I(g.TY) + ";");
        int gml = 0, gmr = 0;  // ghost columns read past the slots
        for (auto& n : geo.nodes) {
            gml = std::max(gml, ghost_lanes_l(n) * V);
            gmr = std::max(gmr, ghost_lanes_r(n) * V);
        }
        line("const bool bx = (x0 + " + I(amin_ - gml) + " < 0) || (x0 + " + I(amax_ + gmr) + " + " + I(N) + " > W);");
        // buffer resources for the live-outs, one per channel plane
        for (size_t oi = 0; oi < geo.liveouts.size(); ++oi) {
            const NodeGeom& n = G(geo.liveouts[oi]);
            std::string ty = mtype(n);
            for (int ch = 0; ch < n.nch; ++ch)
                line("const __amdgpu_buffer_rsrc_t S" + I((int)oi) + "_" + I(ch) +
                     " = __builtin_amdgcn_make_buffer_rsrc((" + ty + "*)A.dst[" + I((int)oi) + "] + " +
                     chan_off(n.id, true, (int)oi, ch) + ", 0, (int)((long long)H * A.dst_rs[" + I((int)oi) +
                     "] * " + I(msize(n)) + "), WT_RSRC_W3);");
        }
        for (size_t k = 0; k < geo.dec.size(); ++k) {
            int oi = (int)(geo.liveouts.size() + k);
            const NodeGeom& src = G(geo.dec[k].second);
            for (int ch = 0; ch < src.nch; ++ch)
                line("const __amdgpu_buffer_rsrc_t S" + I(oi) + "_" + I(ch) +
                     " = __builtin_amdgcn_make_buffer_rsrc((char*)A.dst[" + I(oi) + "] + " +
                     I(dec_size(k)) + " * (" + chan_off(src.id, true, oi, ch) + "), 0, (int)((long long)((H + 1) >> 1) * A.dst_rs[" +
                     I(oi) + "] * " + I(dec_size(k)) + "), WT_RSRC_W3);");
        }
        emit_hist_clear();
        emit_tables();
        line("if (!bx) {");
        body(false);
        line("} else {");
        body(true);
        line("}");
        emit_hist_flush();
    }

    // Single-image kernel: one wave per tile.
    std::string kernel(const std::string& kname) {
        header();
        o << "extern \"C\" __global__ void __launch_bounds__(" << 64 * g.WPB << ") " << kname
          << "(const WtArgs A) {\n";
        line("const int lane = threadIdx.x & 63;");
        wave_index("wid");
        line("if (wid >= A.nwaves) return;");
        lds_decl();
        tile();
        o << "}\n";
        return o.str();
    }

    // Batched kernel: the launch's waves loop over the tiles of all images
    // with the launch's stride (one pass per wave when the grid has a
    // workgroup per work unit); image i owns tiles start[i] .. start[i+1]-1
    // and its arguments are AB[i].
    std::string batch_kernel(const std::string& kname) {
        o << "extern \"C\" __global__ void __launch_bounds__(" << 64 * g.WPB << ") " << kname
          << "_batch(const WtArgs* __restrict__ AB, const int* __restrict__ start, const int nimg, const int total) {\n";
        line("const int lane = threadIdx.x & 63;");
        wave_index("w0");
        line("const int wstride = gridDim.x * " + I(g.WPB) + ";");
        lds_decl();
        line("for (int t = w0; t < total; t += wstride) {");
        ind += "    ";
        line("int lo = 0, hi = nimg;");
        line("while (hi - lo > 1) { const int mid = (lo + hi) >> 1; if (start[mid] <= t) lo = mid; else hi = mid; }");
        line("const int img = __builtin_amdgcn_readfirstlane(lo);");
        // a private copy: the compiler keeps the fields it uses in registers
        // instead of reloading them after every store
        line("const WtArgs A = AB[img];");
        line("const int wid = t - start[img];");
        line("{");
        tile();
        line("}");
        ind.resize(ind.size() - 4);
        line("}");
        o << "}\n";
        return o.str();
    }

    // Wave tile `wid` of the image `A` as a device function of the
    // whole-pipeline kernel, with the wave's LDS at `lds`.
    std::string tile_function(const std::string& fname) {
        o << "WT_DEV void " << fname << "(const WtArgs& A, const int wid, const int lane, char* lds) {\n";
        line("(void)lds;");
        lds_ptrs();
        tile();
        o << "}\n";
        return o.str();
    }
};

}  // namespace

namespace {

// The paper's one-overlapped-tile-per-thread-block execution (Section 3,
// Fig. 3), kept as the ablation baseline of OTPW: a workgroup computes one
// BX x BY output tile; every stage is evaluated over its whole (halo-grown)
// region into LDS by all threads, with a workgroup barrier between stages;
// loaded nodes are staged into LDS first; live-outs are written at the end.
struct BlockGen {
    const Pipeline& P;
    const GroupSched& g;
    const GroupGeom& geo;
    std::ostringstream o;
    int BX, BY, T;
    struct Region { int x0 = 0, x1 = 0, y0 = 0, y1 = 0, off = 0; };
    std::map<int, Region> reg;  // node id -> region relative to the tile origin
    int lds_elems = 0;

    BlockGen(const Pipeline& p, const GroupSched& gs, const GroupGeom& ge)
        : P(p), g(gs), geo(ge), BX(block_tile_w(gs)), BY(gs.TY), T(64 * gs.WPB) {
        std::set<int> mem(g.nodes.begin(), g.nodes.end());
        for (int m : g.nodes)
            if (P.nodes[m].kind == Kind::Up2)
                fail(WT_E_UNSUPPORTED, "one-tile-per-workgroup groups do not fold up2 stages");
        auto cons = P.consumers();
        for (int lo : geo.outs) reg[lo] = {0, BX, 0, BY, 0};
        std::vector<int> order;
        for (auto& ng : geo.nodes) order.push_back(ng.id);
        std::sort(order.rbegin(), order.rend());
        for (int id : order) {
            Region r;
            bool any = reg.count(id) > 0;
            if (any) r = reg[id];
            for (int c : cons[id]) {
                if (!mem.count(c)) continue;
                const Region& rc = reg.at(c);
                for (const Tap& t : P.taps(c, id)) {
                    Region q{rc.x0 + t.dx, rc.x1 + t.dx, rc.y0 + t.dy, rc.y1 + t.dy, 0};
                    if (!any) r = q;
                    r.x0 = std::min(r.x0, q.x0);
                    r.x1 = std::max(r.x1, q.x1);
                    r.y0 = std::min(r.y0, q.y0);
                    r.y1 = std::max(r.y1, q.y1);
                    any = true;
                }
            }
            reg[id] = r;
        }
        for (auto& ng : geo.nodes) {
            Region& r = reg[ng.id];
            r.off = lds_elems;
            lds_elems += (r.x1 - r.x0) * (r.y1 - r.y0) * ng.nch;
        }
        // a workgroup may hold up to 160 KiB of LDS on gfx950
        if ((long long)lds_elems * 4 > 160 * 1024)
            fail(WT_E_UNSUPPORTED, "one-tile-per-workgroup group needs more than 160 KiB of LDS");
    }
    const NodeGeom& G(int id) const { return geo.nodes.at(geo.index.at(id)); }
    static std::string I(long long v) { return std::to_string(v); }
    std::string ct(int id) const { return P.nodes[id].is_int() ? "int" : "float"; }
    std::string arr(int id) const { return "L" + I(id); }
    int RW(int id) const { return reg.at(id).x1 - reg.at(id).x0; }
    int RH(int id) const { return reg.at(id).y1 - reg.at(id).y0; }
    int chan(int p, int ch_c, int explicit_ch) const {
        if (explicit_ch >= 0) return explicit_ch;
        return G(p).nch == 1 ? 0 : ch_c;
    }
    // value of producer p (channel slot chp) at global (gx + dx, gy + dy),
    // clamped to the image (per-stage clamp to edge)
    bool fast = false;  // interior tile: every region lies inside the image
    std::string rd(int c, int p, int chp, int dx, int dy) {
        const Region& r = reg.at(p);
        if (fast) {  // no clamps: the element's own offset plus a constant
            const Region& rc = reg.at(c);
            std::string v = arr(p) + "[" + I((long long)chp * RW(p) * RH(p)) + " + (iy + (" + I(rc.y0 + dy - r.y0) +
                            ")) * " + I(RW(p)) + " + ix + (" + I(rc.x0 + dx - r.x0) + ")]";
            return (!P.nodes[c].is_int() && P.nodes[p].is_int()) ? "(float)" + v : v;
        }
        std::string x = "(wt_clampi(gx + (" + I(dx) + "), 0, W - 1) - ox - (" + I(r.x0) + "))";
        std::string y = "(wt_clampi(gy + (" + I(dy) + "), 0, H - 1) - oy - (" + I(r.y0) + "))";
        std::string v = arr(p) + "[" + I((long long)chp * RW(p) * RH(p)) + " + wt_clampi(" + y + ", 0, " + I(RH(p) - 1) +
                        ") * " + I(RW(p)) + " + wt_clampi(" + x + ", 0, " + I(RW(p) - 1) + ")]";
        return (!P.nodes[c].is_int() && P.nodes[p].is_int()) ? "(float)" + v : v;
    }
    std::string expr(const Expr& e, int c, int ch) {
        const bool in = P.nodes[c].is_int();
        auto K = [&](int i) { return expr(e.kids[i], c, ch); };
        char b[64];
        switch (e.op) {
            case Expr::Const:
                if (in) return "(" + I((long long)e.value) + ")";
                std::snprintf(b, sizeof b, "(%.9ef)", (double)(float)e.value);
                return b;
            case Expr::Src: {
                int p = P.nodes[c].srcs[e.src];
                return rd(c, p, chan(p, ch, e.chan), 0, 0);
            }
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
    std::string value(int c, int ch) {
        const Node& n = P.nodes[c];
        std::string sat;
        if (n.is_int() && n.dtype != WT_I32) {
            auto r = dtype_range(n.dtype);
            sat = ", " + I(r.first) + ", " + I(r.second) + ")";
        }
        if (n.kind == Kind::Pointwise) {
            std::string v = expr(n.expr, c, ch);
            return sat.empty() ? v : "wt_sat(" + v + sat;
        }
        int p = n.srcs[0];
        int chp = chan(p, ch, -1);
        std::string acc;
        if (n.is_int()) {
            for (int j = 0; j < n.kh; ++j)
                for (int i = 0; i < n.kw; ++i) {
                    long long w = n.iweights[(size_t)j * n.kw + i];
                    if (!w) continue;
                    std::string t = "(" + I(w) + ") * " + rd(c, p, chp, i - n.ax, j - n.ay);
                    acc = acc.empty() ? t : acc + " + " + t;
                }
            if (acc.empty()) acc = "0";
            std::string q = n.divisor > 1 ? "wt_rdiv(" + acc + ", " + I(n.divisor) + ")" : "(" + acc + ")";
            return sat.empty() ? q : "wt_sat(" + q + sat;
        }
        for (const Tap& t : P.taps(c, p)) {
            char w[64];
            std::snprintf(w, sizeof w, "(%.9ef)", (double)(float)t.w);
            std::string r = rd(c, p, chp, t.dx, t.dy);
            acc = acc.empty() ? std::string(w) + " * " + r : "fmaf(" + std::string(w) + ", " + r + ", " + acc + ")";
        }
        return acc.empty() ? "0.0f" : acc;
    }
    std::string chan_off(int id, bool dst, int slot, int ch) {
        std::string cs = std::string(dst ? "A.dst_cs[" : "A.src_cs[") + I(slot) + "]";
        if (geo.chan_parallel) return P.nodes[id].channels == 1 ? "0" : "(long long)cp * " + cs;
        return "(long long)" + I(ch) + " * " + cs;
    }
    std::string mtype(int id, bool half) const {
        return P.nodes[id].is_int() ? dtype_ctype(P.nodes[id].dtype) : (half ? "_Float16" : "float");
    }
    // body for tile index t of the image described by A
    void tile_body() {
        o << "    const int ty = t % A.tiles_y, rr = t / A.tiles_y, tx = rr % A.tiles_x, cp = rr / A.tiles_x;\n";
        o << "    (void)cp;\n";
        o << "    const int W = A.W, H = A.H;\n";
        o << "    const int ox = tx * " << BX << ", oy = ty * " << BY << ";\n";
        int x0 = 0, x1 = BX, y0 = 0, y1 = BY;
        for (auto& kv : reg) {
            x0 = std::min(x0, kv.second.x0);
            x1 = std::max(x1, kv.second.x1);
            y0 = std::min(y0, kv.second.y0);
            y1 = std::max(y1, kv.second.y1);
        }
        // tiles whose halo-grown regions lie inside the image read without
        // clamps (the workgroup takes one branch, so its barriers match)
        o << "    const bool fin = ox + (" << x0 << ") >= 0 && ox + " << x1 << " <= W && oy + (" << y0 << ") >= 0 && oy + "
          << y1 << " <= H;\n";
        o << "    if (fin) {\n";
        stages(true);
        o << "    } else {\n";
        stages(false);
        o << "    }\n";
        stores();
    }
    void stages(bool f) {
        fast = f;
        // stage the loaded nodes
        for (size_t li = 0; li < geo.loaded.size(); ++li) {
            const NodeGeom& n = G(geo.loaded[li]);
            const Region& r = reg.at(n.id);
            std::string ty = mtype(n.id, n.mem_half);
            for (int ch = 0; ch < n.nch; ++ch) {
                o << "    { const " << ty << "* s = (const " << ty << "*)A.src[" << li << "] + " << chan_off(n.id, false, (int)li, ch)
                  << ";\n";
                o << "      for (int i = threadIdx.x; i < " << RW(n.id) * RH(n.id) << "; i += " << T << ") {\n";
                if (fast) {
                    o << "        const int gx = ox + (" << r.x0 << ") + i % " << RW(n.id) << ";\n";
                    o << "        const int gy = oy + (" << r.y0 << ") + i / " << RW(n.id) << ";\n";
                } else {
                    o << "        const int gx = wt_clampi(ox + (" << r.x0 << ") + i % " << RW(n.id) << ", 0, W - 1);\n";
                    o << "        const int gy = wt_clampi(oy + (" << r.y0 << ") + i / " << RW(n.id) << ", 0, H - 1);\n";
                }
                o << "        " << arr(n.id) << "[" << (long long)ch * RW(n.id) * RH(n.id) << " + i] = (" << ct(n.id)
                  << ")s[(long long)gy * A.src_rs[" << li << "] + gx];\n";
                o << "      } }\n";
            }
        }
        o << "    __syncthreads();\n";
        for (int m : g.nodes) {
            const NodeGeom& n = G(m);
            const Region& r = reg.at(m);
            for (int ch = 0; ch < n.nch; ++ch) {
                o << "    for (int i = threadIdx.x; i < " << RW(m) * RH(m) << "; i += " << T << ") {  // stage " << m << "\n";
                if (fast)
                    o << "      const int ix = i % " << RW(m) << ", iy = i / " << RW(m) << ";\n";
                else
                    o << "      const int gx = ox + (" << r.x0 << ") + i % " << RW(m) << ", gy = oy + (" << r.y0
                      << ") + i / " << RW(m) << ";\n";
                o << "      " << arr(m) << "[" << (long long)ch * RW(m) * RH(m) << " + i] = " << value(m, ch) << ";\n";
                o << "    }\n";
            }
            o << "    __syncthreads();\n";
        }
    }
    void stores() {
        for (size_t oi = 0; oi < geo.liveouts.size(); ++oi) {
            int id = geo.liveouts[oi];
            const NodeGeom& n = G(id);
            const Region& r = reg.at(id);
            std::string ty = mtype(id, n.mem_half);
            for (int ch = 0; ch < n.nch; ++ch) {
                o << "    { " << ty << "* d = (" << ty << "*)A.dst[" << oi << "] + " << chan_off(id, true, (int)oi, ch) << ";\n";
                o << "      for (int i = threadIdx.x; i < " << BX * BY << "; i += " << T << ") {\n";
                o << "        const int gx = ox + i % " << BX << ", gy = oy + i / " << BX << ";\n";
                o << "        if (gx < W && gy < H) d[(long long)gy * A.dst_rs[" << oi << "] + gx] = (" << ty << ")"
                  << arr(id) << "[" << (long long)ch * RW(id) * RH(id) << " + (i / " << BX << " - (" << r.y0 << ")) * "
                  << RW(id) << " + i % " << BX << " - (" << r.x0 << ")];\n";
                o << "      } }\n";
            }
        }
    }
    void lds_decl() {
        o << "    __shared__ float wt_lds[" << std::max(1, lds_elems) << "];\n";
        for (auto& ng : geo.nodes)
            o << "    " << ct(ng.id) << "* " << arr(ng.id) << " = (" << ct(ng.id) << "*)(wt_lds + " << reg.at(ng.id).off
              << ");\n";
    }
    std::string single(const std::string& kname) {
        o.str("");
        o << "extern \"C\" __global__ void __launch_bounds__(" << T << ") " << kname << "(const WtArgs A) {\n";
        lds_decl();
        o << "    const int t = blockIdx.x;\n";
        tile_body();
        o << "}\n";
        return o.str();
    }
    std::string batch(const std::string& kname) {
        o.str("");
        o << "extern \"C\" __global__ void __launch_bounds__(" << T << ") " << kname
          << "_batch(const WtArgs* __restrict__ AB, const int* __restrict__ start, const int nimg, const int total) {\n";
        lds_decl();
        o << "  for (int tt = blockIdx.x; tt < total; tt += gridDim.x) {\n";
        o << "    int lo = 0, hi = nimg;\n";
        o << "    while (hi - lo > 1) { const int mid = (lo + hi) >> 1; if (start[mid] <= tt) lo = mid; else hi = mid; }\n";
        o << "    const WtArgs A = AB[lo];\n";
        o << "    const int t = tt - start[lo];\n";
        o << "    __syncthreads();\n";
        tile_body();
        o << "  }\n";
        o << "}\n";
        return o.str();
    }
};

}  // namespace

int block_tile_w(const GroupSched& g) { return 64 * g.V * g.TX; }

GroupSources generate_group_source(const Pipeline& p, const GroupSched& g, const GroupGeom& geo,
                                   const std::string& kname) {
    if ((int)(geo.loaded.size() + geo.tables.size()) > 16 ||
        (int)(geo.liveouts.size() + geo.dec.size() + geo.hist.size()) > 16)
        fail(WT_E_UNSUPPORTED, "group has more than 16 inputs or live-outs");
    if (g.BLK) {
        if (!geo.dec.empty() || !g.exp.empty()) fail(WT_E_UNSUPPORTED, "fused resampling in a one-tile-per-workgroup group");
        if (!geo.hist.empty() || !geo.tables.empty())
            fail(WT_E_UNSUPPORTED, "histogram or equalize stage in a one-tile-per-workgroup group");
        BlockGen b(p, g, geo);
        std::string single = b.single(kname);
        std::string batch = b.batch(kname);
        return GroupSources{device_prelude(), "", single, batch};
    }
    Gen gen(p, g, geo);
    std::string single = gen.kernel(kname);
    Gen gb(p, g, geo);
    gb.header();
    gb.o.str("");
    std::string batch = gb.batch_kernel(kname);
    return GroupSources{device_prelude(), "", single, batch};
}

// The whole group sequence of a batch in one persistent launch.  A chunk is
// a run of consecutive wave tiles of one group and one image; chunks are
// numbered group by group (all chunks of group g before those of g + 1) and
// handed out in that order by an atomic ticket, one chunk per wave at a
// time.  Before its chunk a wave waits until every producer group of its
// group has completed all its tiles of the same image (the per-image
// completion counters; images of a batch are independent), and after it
// adds its tile count to its own group's counter.  A wave waits only for
// chunks with smaller tickets, which waves already running hold, so the
// smallest unfinished chunk can always proceed and the ordering cannot
// deadlock at any grid size (the argument; the lane emulator checks it with
// several waves at once); every wait is also bounded in time (after
// `limit` ticks of the constant-rate clock the status word is set and all
// waits end, so every wave still reaches the end of the queue).
std::string generate_whole_source(const Pipeline& p, const std::vector<const GroupSched*>& gs,
                                  const std::vector<const GroupGeom*>& geos, const std::string& kname, int wpb,
                                  int& lds_per_wave) {
    if (gs.empty() || gs.size() > 64) fail(WT_E_UNSUPPORTED, "whole-pipeline launch needs 1 to 64 groups");
    if (wpb < 1 || wpb > 16) fail(WT_E_INVALID, "whole-pipeline launch: 1 to 16 waves per workgroup");
    lds_per_wave = 0;
    for (size_t k = 0; k < gs.size(); ++k) {
        if (gs[k]->BLK) fail(WT_E_UNSUPPORTED, "whole-pipeline launch of a one-tile-per-workgroup group");
        if (!geos[k]->hist.empty() || !geos[k]->tables.empty())
            fail(WT_E_UNSUPPORTED, "whole-pipeline launch of a histogram or equalize stage");
        if ((int)(geos[k]->loaded.size()) > 16 || (int)(geos[k]->liveouts.size() + geos[k]->dec.size()) > 16)
            fail(WT_E_UNSUPPORTED, "group has more than 16 inputs or live-outs");
        lds_per_wave = std::max(lds_per_wave, (geos[k]->lds_bytes + 15) / 16 * 16);
    }
    if ((long long)lds_per_wave * wpb > 160 * 1024)
        fail(WT_E_UNSUPPORTED, "whole-pipeline launch needs more than 160 KiB of LDS per workgroup");
    std::ostringstream o;
    o << device_prelude() << "\n";
    o << "struct WtWhole {\n"
         "    const WtArgs* AB;                 // [group][image] kernel arguments\n"
         "    const int* start;                 // [group][image + 1] tile prefix sums\n"
         "    const wt_i4* chunks;              // group, image, first tile, tiles\n"
         "    const unsigned long long* deps;   // [group] producer groups (bit mask)\n"
         "    int* done;                        // [group][image] completed tiles\n"
         "    int* next;                        // ticket counter\n"
         "    int* status;                      // non-zero once a wait gave up\n"
         "    long long limit;                  // longest wait, clock ticks\n"
         "    int nchunks, nimg;\n"
         "};\n";
    for (size_t k = 0; k < gs.size(); ++k) {
        Gen gen(p, *gs[k], *geos[k]);
        gen.header();
        o << gen.o.str();
        gen.o.str("");
        o << gen.tile_function(kname + "_g" + std::to_string(k));
    }
    o << "WT_DEV void " << kname << "_wait(const WtWhole& P, unsigned long long dm, const int img) {\n"
         "    const unsigned long long t0 = wall_clock64();\n"
         "    for (; dm; dm &= dm - 1) {\n"
         "        const int q = __builtin_ctzll(dm);\n"
         "        const int need = P.start[q * (P.nimg + 1) + img + 1] - P.start[q * (P.nimg + 1) + img];\n"
         "        while (__hip_atomic_load(P.done + q * P.nimg + img, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {\n"
         "            if (__hip_atomic_load(P.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;\n"
         "            if ((long long)(wall_clock64() - t0) > P.limit) {\n"
         "                __hip_atomic_store(P.status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);\n"
         "                return;\n"
         "            }\n"
         "            __builtin_amdgcn_s_sleep(2);\n"
         "        }\n"
         "    }\n"
         "}\n";
    o << "extern \"C\" __global__ void __launch_bounds__(" << 64 * wpb << ") " << kname << "(const WtWhole P) {\n";
    o << "    const int lane = threadIdx.x & 63;\n";
    if (lds_per_wave > 0) {
        o << "    __shared__ __attribute__((aligned(16))) char wt_lds[" << lds_per_wave * wpb << "];\n";
        o << "    char* lds = wt_lds + (threadIdx.x >> 6) * " << lds_per_wave << ";\n";
    } else {
        o << "    char* lds = nullptr;\n";
    }
    o << "    for (;;) {\n"
         "        int c = 0;\n"
         "        if (lane == 0) c = __hip_atomic_fetch_add(P.next, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);\n"
         "        c = __builtin_amdgcn_readfirstlane(c);\n"
         "        if (c >= P.nchunks) break;\n"
         "        const wt_i4 ch = P.chunks[c];\n"
         "        const int g = __builtin_amdgcn_readfirstlane(ch.x), img = __builtin_amdgcn_readfirstlane(ch.y);\n"
         "        const int t0 = __builtin_amdgcn_readfirstlane(ch.z), nt = __builtin_amdgcn_readfirstlane(ch.w);\n"
         "        const unsigned long long dm = P.deps[g];\n"
         "        if (dm) {\n"
         "            if (lane == 0) " << kname << "_wait(P, dm, img);\n"
         "            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, \"agent\");\n"
         "        }\n"
         "        wt_wave_sync();  // the previous chunk's LDS reads before this chunk's stores\n"
         "        switch (g) {\n";
    // a private copy of the arguments per tile, as in the batched kernels:
    // the fields the group uses are loaded into registers at each tile
    // rather than held across the chunk's tiles
    for (size_t k = 0; k < gs.size(); ++k)
        o << "        case " << k << ":\n"
          << "            for (int t = t0; t < t0 + nt; ++t) {\n"
          << "                const WtArgs A = P.AB[g * P.nimg + img];\n"
          << "                " << kname << "_g" << k << "(A, t, lane, lds);\n"
          << "            }\n"
          << "            break;\n";
    o << "        default: break;\n"
         "        }\n"
         "        __builtin_amdgcn_fence(__ATOMIC_RELEASE, \"agent\");\n"
         "        if (lane == 0) __hip_atomic_fetch_add(P.done + g * P.nimg + img, nt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);\n"
         "    }\n"
         "}\n";
    return o.str();
}

// 2x resampling kernels (not fused: a scaled dependence ends a group in this
// implementation).  down2: a thread per output pixel, 64 x 4 per 256-thread
// workgroup.  up2: a thread per coarse pixel (i, j) producing the output quad
// (2i..2i+1, 2j..2j+1) from the clamped 3 x 3 coarse neighbourhood -- the
// separable expansion in x (even (P(i-1) + 6 P(i) + P(i+1)) / 8, odd
// (P(i) + P(i+1)) / 2) on three coarse rows, then the same in y -- 128 x 8
// outputs per workgroup.  The single-image kernel runs a
// (tiles_x, tiles_y, channels) grid; the batched kernel loops its workgroups
// over the blocks of all images.
void resample_block(const Pipeline& p, const GroupSched& g, int& bw, int& bh) {
    const Kind k = p.nodes[g.nodes[0]].kind;
    bw = k == Kind::Up2 ? 128 : 64;
    bh = k == Kind::Up2 ? 8 : k == Kind::Hist ? 64 : 4;
}

// A histogram of a stage held in memory (its source not computed by a fused
// group): a workgroup counts a 64 x 64 block of one channel into LDS bins
// (each thread 16 rows of one column), then adds its non-zero bins to the
// output.  Same launch shape as the resampling kernels.
GroupSources generate_hist_source(const Pipeline& p, const GroupSched& g, const std::string& kname, bool src_half) {
    const Node& n = p.nodes[g.nodes[0]];
    const Node& sn = p.nodes[n.srcs[0]];
    const std::string st = sn.is_int() ? dtype_ctype(sn.dtype) : src_half ? "_Float16" : "float";
    const std::string lo = flit((double)(float)n.hlo), sc = flit((double)(float)(n.bins / (n.hhi - n.hlo)));
    std::ostringstream o;
    o << "static __device__ __forceinline__ void " << kname << "_body(const WtArgs& A, int bxi, int byi, int c) {\n";
    o << "    __shared__ unsigned int hb[" << n.bins << "];\n";
    o << "    __syncthreads();\n";
    o << "    for (int i = threadIdx.x; i < " << n.bins << "; i += 256) hb[i] = 0u;\n";
    o << "    __syncthreads();\n";
    o << "    const " << st << "* s = (const " << st << "*)A.src[0] + (long long)c * A.src_cs[0];\n";
    o << "    const int x = bxi * 64 + (threadIdx.x & 63);\n";
    o << "    if (x < A.W)\n";
    o << "        for (int r = 0; r < 16; ++r) {\n";
    o << "            const int y = byi * 64 + (threadIdx.x >> 6) + 4 * r;\n";
    o << "            if (y < A.H) wt_count_lds(hb + wt_hist_bin((float)s[(long long)y * A.src_rs[0] + x], " << lo << ", "
      << sc << ", " << n.bins << "), 1u);\n";
    o << "        }\n";
    o << "    __syncthreads();\n";
    o << "    unsigned int* d = (unsigned int*)A.dst[0] + (long long)c * A.dst_cs[0];\n";
    o << "    for (int i = threadIdx.x; i < " << n.bins << "; i += 256) if (hb[i]) wt_count_global(d + i, hb[i]);\n";
    o << "}\n";
    const std::string body = o.str();
    o.str("");
    o << "extern \"C\" __global__ void __launch_bounds__(256) " << kname << "(const WtArgs A) {\n";
    o << "    " << kname << "_body(A, blockIdx.x, blockIdx.y, blockIdx.z);\n";
    o << "}\n";
    const std::string single = o.str();
    o.str("");
    o << "extern \"C\" __global__ void __launch_bounds__(256) " << kname
      << "_batch(const WtArgs* __restrict__ AB, const int* __restrict__ start, const int nimg, const int total) {\n";
    o << "    for (int t = blockIdx.x; t < total; t += gridDim.x) {\n";
    o << "        int lo = 0, hi = nimg;\n";
    o << "        while (hi - lo > 1) { const int mid = (lo + hi) >> 1; if (start[mid] <= t) lo = mid; else hi = mid; }\n";
    o << "        const WtArgs A = AB[lo];\n";
    o << "        const int l = t - start[lo];\n";
    o << "        const int r = l / A.tiles_x;\n";
    o << "        " << kname << "_body(A, l % A.tiles_x, r % A.tiles_y, r / A.tiles_y);\n";
    o << "    }\n";
    o << "}\n";
    return GroupSources{device_prelude(), body, single, o.str()};
}

GroupSources generate_resample_source(const Pipeline& p, const GroupSched& g, const std::string& kname,
                                      bool src_half, bool dst_half) {
    const Node& n = p.nodes[g.nodes[0]];
    const Node& sn = p.nodes[n.srcs[0]];
    const std::string st = sn.is_int() ? dtype_ctype(sn.dtype) : src_half ? "_Float16" : "float";
    const std::string dt = n.is_int() ? dtype_ctype(n.dtype) : dst_half ? "_Float16" : "float";
    std::ostringstream o;
    o << "static __device__ __forceinline__ void " << kname << "_body(const WtArgs& A, int bxi, int byi, int c) {\n";
    o << "    const " << st << "* s = (const " << st << "*)A.src[0] + (long long)c * A.src_cs[0];\n";
    o << "    " << dt << "* d = (" << dt << "*)A.dst[0] + (long long)c * A.dst_cs[0];\n";
    o << "    const long long rs = A.src_rs[0], ds = A.dst_rs[0];\n";
    if (n.kind == Kind::Down2) {
        o << "    const int x = bxi * 64 + (threadIdx.x & 63);\n";
        o << "    const int y = byi * 4 + (threadIdx.x >> 6);\n";
        o << "    if (x >= A.W || y >= A.H) return;\n";
        o << "    d[(long long)y * ds + x] = (" << dt << ")(" << (n.is_int() ? "int" : "float")
          << ")s[(long long)(2 * y) * rs + 2 * x];\n";
    } else {
        o << "    const int i = bxi * 64 + (threadIdx.x & 63);\n";
        o << "    const int j = byi * 4 + (threadIdx.x >> 6);\n";
        o << "    const int x = 2 * i, y = 2 * j;\n";
        o << "    if (x >= A.W || y >= A.H) return;\n";
        o << "    const int Ws = A.Ws, Hs = A.Hs;\n";
        o << "    const int xm = wt_clampi(i - 1, 0, Ws - 1), x0 = min(i, Ws - 1), xp = min(i + 1, Ws - 1);\n";
        o << "    float he[3], ho[3];\n";
        o << "    for (int b = 0; b < 3; ++b) {\n";
        o << "        const " << st << "* row = s + (long long)wt_clampi(j - 1 + b, 0, Hs - 1) * rs;\n";
        o << "        const float pm = (float)row[xm], p0 = (float)row[x0], pp = (float)row[xp];\n";
        o << "        he[b] = fmaf(0.125f, pp, fmaf(0.75f, p0, 0.125f * pm));\n";
        o << "        ho[b] = fmaf(0.5f, pp, 0.5f * p0);\n";
        o << "    }\n";
        o << "    " << dt << "* r0 = d + (long long)y * ds;\n";
        o << "    r0[x] = (" << dt << ")fmaf(0.125f, he[2], fmaf(0.75f, he[1], 0.125f * he[0]));\n";
        o << "    if (x + 1 < A.W) r0[x + 1] = (" << dt << ")fmaf(0.125f, ho[2], fmaf(0.75f, ho[1], 0.125f * ho[0]));\n";
        o << "    if (y + 1 < A.H) {\n";
        o << "        " << dt << "* r1 = r0 + ds;\n";
        o << "        r1[x] = (" << dt << ")fmaf(0.5f, he[2], 0.5f * he[1]);\n";
        o << "        if (x + 1 < A.W) r1[x + 1] = (" << dt << ")fmaf(0.5f, ho[2], 0.5f * ho[1]);\n";
        o << "    }\n";
    }
    o << "}\n";
    const std::string body = o.str();
    o.str("");
    o << "extern \"C\" __global__ void __launch_bounds__(256) " << kname << "(const WtArgs A) {\n";
    o << "    " << kname << "_body(A, blockIdx.x, blockIdx.y, blockIdx.z);\n";
    o << "}\n";
    const std::string single = o.str();
    o.str("");
    o << "extern \"C\" __global__ void __launch_bounds__(256) " << kname
      << "_batch(const WtArgs* __restrict__ AB, const int* __restrict__ start, const int nimg, const int total) {\n";
    o << "    for (int t = blockIdx.x; t < total; t += gridDim.x) {\n";
    o << "        int lo = 0, hi = nimg;\n";
    o << "        while (hi - lo > 1) { const int mid = (lo + hi) >> 1; if (start[mid] <= t) lo = mid; else hi = mid; }\n";
    o << "        const WtArgs A = AB[lo];\n";
    o << "        const int l = t - start[lo];\n";
    o << "        const int r = l / A.tiles_x;\n";
    o << "        " << kname << "_body(A, l % A.tiles_x, r % A.tiles_y, r / A.tiles_y);\n";
    o << "    }\n";
    o << "}\n";
    return GroupSources{device_prelude(), body, single, o.str()};
}

}  // namespace wt
