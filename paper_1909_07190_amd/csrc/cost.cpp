// Analytical cost model (the paper, Section 6 and Algorithm 2), with the
// machine model of Table 1 rewritten for gfx950.
//
// alg2() evaluates Algorithm 2's seven terms from the quantities the
// algorithm reads (scratchpad per thread block, registers per thread, warps
// per block, transactions, memory and compute time, overlap, block count),
// so the same code scores the paper's worked examples with the GTX 1080Ti
// table and gfx950 wave-tile schedules with the gfx950 table.
//
// Readings of garbled or undefined parts of Algorithm 2:
//  * the shared-memory split uses the pre-split footprint for both the LDS
//    part and the register tile (the listing rescales before it splits);
//  * transactions are the distinct txSz-aligned segments one wave's input
//    footprint touches, times the number of waves, normalised by the
//    compulsory count (the listing adds a raw count to fractions);
//  * per-wave bandwidth is HBM bandwidth divided by the CUs and then by the
//    waves resident on a CU (the text's description of the per-warp share);
//  * extra blocks = ceil(blocks / CUs) mod blocks resident per CU;
//  * on gfx950 register occupancy is waves/SIMD = min(8, 512 / alloc8(vgpr)),
//    times 4 SIMDs, instead of registers-per-SM / registers-per-thread.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <set>

#include "wt_cost.h"

namespace wt {

Machine machine_gtx1080ti() {
    Machine m;
    m.name = "GTX 1080Ti";
    m.ncu = 28;
    m.wave = 32;
    m.simd_per_cu = 4;
    m.max_waves_per_cu = 64;
    m.max_wg_per_cu = 16;
    m.lds_per_cu = 96 * 1024;
    m.max_lds_per_wg = 48 * 1024;
    m.regs_per_cu = 65536;
    m.max_regs_per_lane = 256;
    m.amd_vgpr_alloc = false;
    m.hbm_bw = 484e9;
    m.cores_per_cu = 128;
    return m;
}

Machine machine_gfx950() { return Machine{}; }

// Section 4: warp sizes from the thread-block size.
void warp_sizes(const int B[3], int ws, int W[3]) {
    W[0] = std::min(B[0], ws);
    W[1] = std::min(B[1], std::max(1, ws / W[0]));
    W[2] = std::min(B[2], std::max(1, ws / (W[0] * W[1])));
}

// Section 4: scratchpad of one stage for one thread block,
// prod_i ceil(B_i / W_i) * (T_i * W_i + O_i), in elements.
long long scratchpad_elems(const int T[3], const int B[3], const int W[3], const int O[3]) {
    long long e = 1;
    for (int i = 0; i < 3; ++i) e *= (long long)((B[i] + W[i] - 1) / W[i]) * (T[i] * W[i] + O[i]);
    return e;
}

int waves_per_cu_by_regs(const Machine& m, double regs_per_lane) {
    if (regs_per_lane <= 0) regs_per_lane = 1;
    if (m.amd_vgpr_alloc) {
        int alloc = (int)std::ceil(regs_per_lane / m.vgpr_granule) * m.vgpr_granule;
        int per_simd = std::min(m.max_waves_per_simd, m.vgpr_per_simd_lane / std::max(alloc, 1));
        return per_simd * m.simd_per_cu;
    }
    double max_th = std::min((double)m.regs_per_cu / regs_per_lane, (double)m.max_waves_per_cu * m.wave);
    return (int)(max_th / m.wave);
}

Alg2Out alg2(const Alg2In& in, const Machine& m, const double w[7]) {
    Alg2Out o;
    if (in.smem_per_wg > m.max_lds_per_wg || in.regs_per_lane > m.max_regs_per_lane) {
        o.feasible = false;
        o.score = INFINITY;
        return o;
    }
    int max_wg = in.smem_per_wg > 0 ? (int)std::floor(m.lds_per_cu / in.smem_per_wg) : m.max_wg_per_cu;
    max_wg = std::min(max_wg, m.max_wg_per_cu);
    if (max_wg < 1) {
        o.feasible = false;
        o.score = INFINITY;
        return o;
    }
    o.max_wg_per_cu = max_wg;
    o.shmem_occ = std::min(max_wg * in.waves_per_wg, m.max_waves_per_cu);
    o.reg_occ = std::min(waves_per_cu_by_regs(m, in.regs_per_lane), m.max_waves_per_cu);
    // whole workgroups only
    int waves = std::min(o.shmem_occ, o.reg_occ);
    waves = waves / in.waves_per_wg * in.waves_per_wg;
    o.occupancy = (double)waves / m.max_waves_per_cu;
    if (waves < in.waves_per_wg) {
        o.feasible = false;
        o.score = INFINITY;
        return o;
    }
    double resident = std::max(1, waves);
    double wave_bw = m.hbm_bw / m.ncu / resident;
    double mem_time = in.mem_bytes_per_wave / wave_bw;
    o.mem_over_compute = in.compute_time_per_wave > 0 ? mem_time / in.compute_time_per_wave : 0.0;
    double smem_cu = in.smem_per_wg * std::min(max_wg, waves / in.waves_per_wg);
    o.unalloc_smem = 1.0 - smem_cu / m.lds_per_cu;
    double reg_file = m.amd_vgpr_alloc ? (double)m.vgpr_per_simd_lane * m.simd_per_cu * m.wave : (double)m.regs_per_cu;
    o.unused_reg = 1.0 - in.regs_per_lane * m.max_waves_per_cu * m.wave * o.occupancy / reg_file;
    long long wg_per_cu = (in.total_wg + m.ncu - 1) / m.ncu;
    int wg_resident = std::max(1, waves / in.waves_per_wg);
    o.extra_wg = (double)(wg_per_cu % wg_resident);
    double tx_norm = in.compulsory_tx > 0 ? in.total_tx / in.compulsory_tx : in.total_tx;
    o.terms[0] = tx_norm;
    o.terms[1] = 1.0 - o.occupancy;
    o.terms[2] = o.mem_over_compute;
    o.terms[3] = o.unalloc_smem;
    o.terms[4] = o.unused_reg;
    o.terms[5] = in.frac_overlap;
    o.terms[6] = o.extra_wg;
    o.score = 0;
    for (int i = 0; i < 7; ++i) o.score += w[i] * o.terms[i];
    o.feasible = true;
    return o;
}

// --------------------------------------------------------------------------
// gfx950 adapter: quantities of a wave-tile schedule
// --------------------------------------------------------------------------

// VALU operations to produce one point of a stage (the stage-body cost the
// per-stage pre-profiling measures; this is the fallback estimate).
static int expr_ops(const Expr& e) {
    int n = (e.op == Expr::Const || e.op == Expr::Src) ? 0 : 1;
    if (e.op == Expr::Select) n = 2;
    if (e.op == Expr::Div || e.op == Expr::Sqrt) n = 10;
    for (const Expr& k : e.kids) n += expr_ops(k);
    return n;
}

StageProfile estimate_stage(const Pipeline& p, int id, const Machine& m) {
    const Node& n = p.nodes[id];
    StageProfile s;
    if (lookup_profile(p, id, s)) return s;  // measured by pre-profiling
    int ops = 1;
    if (n.kind == Kind::Stencil) {
        int taps = 0, dx = 0;
        for (double w : n.weights) taps += (w != 0.0);
        for (int i = 0; i < n.kw; ++i) dx += (i != n.ax);
        ops = taps + (dx ? 2 : 0);
    } else if (n.kind == Kind::Pointwise) {
        ops = std::max(1, expr_ops(n.expr));
    } else if (n.kind == Kind::Equalize) {
        ops = 8;  // the bin, an LDS read of its cumulative count, a scale
    } else {
        ops = 12;
    }
    s.valu_ops = ops;
    // one wave instruction issues every 4 cycles on a 16-lane SIMD
    s.ns_per_point = ops * 4.0 / m.clock_hz * 1e9;
    s.vgprs = 2 + ops / 4;
    s.measured = false;
    return s;
}

GroupCost group_cost(const Pipeline& p, const GroupSched& g, const GroupGeom& geo, const Machine& m,
                     int W, int H, const std::map<int, StageProfile>& prof, int tx_size, const double w[7], int batch) {
    GroupCost c;
    batch = std::max(1, batch);
    int lw = W, lh = H;
    for (int i = 0; i < p.nodes[g.nodes[0]].level; ++i) {
        lw = (lw + 1) / 2;
        lh = (lh + 1) / 2;
    }
    int amin = 1 << 30, amax = 0;
    for (int lo : geo.outs) {
        amin = std::min(amin, geo.nodes[geo.index.at(lo)].skew);
        amax = std::max(amax, geo.nodes[geo.index.at(lo)].skew);
    }
    long long tiles_x = (lw - (amin - amax) + geo.X - 1) / geo.X;
    long long tiles_y = (lh + g.TY - 1) / g.TY;
    long long nwaves = tiles_x * tiles_y * (geo.chan_parallel ? geo.C : 1) * batch;
    c.nwaves = nwaves;
    long long total_wg = (nwaves + g.WPB - 1) / g.WPB;
    int steps = geo.D + g.TY;

    // registers: ring windows plus per-stage working registers
    double regs = 12;  // addresses, loop counters, lane id
    double lds = 0;
    double compute_ns = 0, valu_ops = 0;
    double load_bytes = 0, store_bytes = 0, tx = 0, tx_comp = 0, comp_bytes = 0;
    double computed = 0, useful = 0;
    for (const NodeGeom& n : geo.nodes) {
        int RX = g.TX - g.SX;
        bool stored = !n.member || n.consumed;
        // FP16 register rows with an even number of elements per lane pack
        // two values per VGPR
        double per = n.half && n.member && g.V % 2 == 0 ? 0.5 : 1.0;
        if (stored) regs += (double)n.win * n.nch * RX * g.V * per;
        if (!n.member) {
            const Node& nd = p.nodes[n.id];
            int esz = p.nodes[n.id].is_int() ? dtype_size(p.nodes[n.id].dtype) : (n.mem_half ? 2 : 4);
            int rows = std::max(0, steps - g.PF - n.first_step);
            // an expanded up2 reads its coarse source: half the columns, and
            // each coarse row serves two fine rows
            double row_bytes = (double)geo.N * esz * (n.expand_src >= 0 ? 0.25 : 1.0);
            load_bytes += rows * row_bytes * n.nch;
            int segs = (int)std::ceil(row_bytes / tx_size) + 1;
            tx += (double)rows * segs * n.nch;
            int ch = geo.chan_parallel ? 1 : nd.channels;
            comp_bytes += (double)lw * lh * esz * (geo.chan_parallel ? nd.channels : ch) *
                          (n.expand_src >= 0 ? 0.25 : 1.0);
            continue;
        }
        auto it = prof.find(n.id);
        StageProfile sp = it != prof.end() ? it->second : estimate_stage(p, n.id, m);
        regs += sp.vgprs;
        int active = steps - n.first_step;
        double pts = (double)active * g.TX * g.V * n.nch;  // per lane
        compute_ns += sp.ns_per_point * pts;
        valu_ops += sp.valu_ops * pts;
        computed += (double)active * geo.N * n.nch;
        c.code_ops += (double)sp.valu_ops * n.nch * g.TX * g.V;
        useful += (double)g.TY * geo.X * n.nch;
        if (n.liveout) {
            int esz = p.nodes[n.id].is_int() ? dtype_size(p.nodes[n.id].dtype) : (n.mem_half ? 2 : 4);
            store_bytes += (double)g.TY * geo.X * esz * n.nch;
            int ch = geo.chan_parallel ? 1 : p.nodes[n.id].channels;
            comp_bytes += (double)lw * lh * esz * (geo.chan_parallel ? p.nodes[n.id].channels : ch);
        }
    }
    for (auto& ds : geo.dec) {  // decimated outputs: a quarter of the member's points
        const NodeGeom& n = geo.nodes[geo.index.at(ds.second)];
        int esz = p.nodes[ds.first].is_int() ? dtype_size(p.nodes[ds.first].dtype) : (n.mem_half ? 2 : 4);
        store_bytes += (double)g.TY * geo.X * esz * n.nch / 4.0;
        comp_bytes += (double)lw * lh * esz * p.nodes[ds.first].channels / 4.0;
    }
    comp_bytes *= batch;
    lds = geo.lds_bytes_per_wg;
    tx_comp = 0;
    for (int l : geo.loaded) {
        const NodeGeom& n = geo.nodes[geo.index.at(l)];
        int esz = p.nodes[l].is_int() ? dtype_size(p.nodes[l].dtype) : (n.mem_half ? 2 : 4);
        tx_comp += std::ceil((double)lw * lh * esz * p.nodes[l].channels / tx_size) * batch;
    }

    Alg2In in;
    in.smem_per_wg = lds;
    in.regs_per_lane = regs;
    in.waves_per_wg = g.WPB;
    in.total_wg = total_wg;
    in.total_tx = tx * nwaves;
    in.compulsory_tx = std::max(1.0, tx_comp);
    in.mem_bytes_per_wave = load_bytes + store_bytes;
    in.compute_time_per_wave = compute_ns * 1e-9;
    in.frac_overlap = useful > 0 ? computed / useful - 1.0 : 0.0;
    c.alg2 = alg2(in, m, w);
    c.code_ops *= geo.D + geo.U + geo.E;
    if (c.code_ops > m.max_code_ops) c.alg2.feasible = false;
    c.regs_est = regs;
    c.lds_per_wg = lds;
    c.requested_bytes = (load_bytes + store_bytes) * nwaves;
    c.compulsory_bytes = comp_bytes;
    c.valu_ops = valu_ops * nwaves;
    if (!c.alg2.feasible) {
        c.pred_us = INFINITY;
        c.cal_us = INFINITY;
        return c;
    }
    // Predicted time (the additive quantity the fusion search sums): HBM
    // time for the compulsory bytes plus a share of the redundant halo
    // traffic, derated when too few bytes are in flight; VALU time at the
    // SIMD issue rate; and the launch overhead.  The partly filled last
    // round of waves is not modelled here (Algorithm 2's extra-blocks term
    // describes it, and the gfx950 refit gives that term weight 0).
    double hbm_bytes = comp_bytes + 0.5 * std::max(0.0, c.requested_bytes - comp_bytes);
    double resident_waves = std::min<double>(nwaves, c.alg2.occupancy * m.max_waves_per_cu * m.ncu);
    double row_in_flight = 0;
    for (int l : geo.loaded) {
        const NodeGeom& n = geo.nodes[geo.index.at(l)];
        row_in_flight += (double)geo.N * (p.nodes[l].is_int() ? dtype_size(p.nodes[l].dtype) : (n.mem_half ? 2 : 4)) * n.nch;
    }
    double inflight = resident_waves * row_in_flight * (g.PF + 1);
    double need = m.hbm_bw * m.mem_latency_s;
    double eff = std::min(1.0, inflight / need) * m.hbm_efficiency;
    double t_mem = hbm_bytes / (m.hbm_bw * std::max(eff, 0.02));
    double t_alu = c.valu_ops * 64 / (m.ncu * m.simd_per_cu * 16.0 * m.clock_hz);
    c.pred_us = std::max(t_mem, t_alu) * 1e6 + m.launch_us;
    c.cal_us = calibrated_us(c.pred_us, c.alg2.terms, active_fit());
    return c;
}

double calibrated_us(double pred_us, const double terms[7], const AnalyticFit& f) {
    if (!(pred_us > 0) || !std::isfinite(pred_us)) return INFINITY;
    double z = f.c0 + f.c1 * std::log(pred_us);
    for (int k = 0; k < 7; ++k) z += f.w[k] * terms[k];
    return std::exp(z);
}

double resample_pred_us(const Pipeline& p, int id, const Machine& m, int W, int H, bool half_in, bool half_out) {
    const Node& n = p.nodes[id];
    int lw = W, lh = H;
    for (int i = 0; i < n.level; ++i) {
        lw = (lw + 1) / 2;
        lh = (lh + 1) / 2;
    }
    int sw = W, sh = H;
    for (int i = 0; i < p.nodes[n.srcs[0]].level; ++i) {
        sw = (sw + 1) / 2;
        sh = (sh + 1) / 2;
    }
    double in_b = (double)n.channels * (n.kind == Kind::Down2 ? (double)lw * lh : (double)sw * sh) * (half_in ? 2 : 4);
    double out_b = (double)n.channels * (n.kind == Kind::Hist ? (double)n.bins : (double)lw * lh) * (half_out ? 2 : 4);
    return (in_b + out_b) / (m.hbm_bw * m.hbm_efficiency) * 1e6 + m.launch_us;
}

}  // namespace wt

namespace wt {

std::vector<double> group_features(const Pipeline& p, const GroupSched& g, const GroupGeom& geo,
                                   const GroupCost& c, int W, int H, int tx_size) {
    std::vector<double> f;
    f.reserve(kNumFeatures);
    // structural (12)
    int nst = 0, npw = 0, ndn = 0, nup = 0, taps = 0, hx_max = 0, hx_sum = 0, hy_max = 0, hy_sum = 0;
    for (int id : g.nodes) {
        const Node& n = p.nodes[id];
        if (n.kind == Kind::Stencil) {
            ++nst;
            for (double w : n.weights) taps += (w != 0.0);
            int hx = std::max(n.ax, n.kw - 1 - n.ax), hy = std::max(n.ay, n.kh - 1 - n.ay);
            hx_max = std::max(hx_max, hx);
            hy_max = std::max(hy_max, hy);
            hx_sum += hx;
            hy_sum += hy;
        } else if (n.kind == Kind::Pointwise || n.kind == Kind::Equalize) {
            ++npw;
        } else if (n.kind == Kind::Down2) {
            ++ndn;
        } else if (n.kind == Kind::Up2) {
            // a folded up2 runs as a separable 5-tap stencil pair on the
            // stage it folds (half its taps weigh zero at each point)
            ++nst;
            taps += 10;
            hx_max = std::max(hx_max, 2);
            hy_max = std::max(hy_max, 2);
            hx_sum += 2;
            hy_sum += 2;
        }
    }
    f.push_back(g.nodes.size());
    f.push_back(nst);
    f.push_back(npw);
    f.push_back(ndn);
    f.push_back(nup);
    f.push_back(geo.loaded.size());
    f.push_back(geo.liveouts.size());
    f.push_back(taps);
    f.push_back(hx_max);
    f.push_back(hx_sum);
    f.push_back(hy_max);
    f.push_back(hy_sum);
    // schedule (10)
    f.push_back(g.V);
    f.push_back(g.TX);
    f.push_back(g.SX);
    f.push_back(g.TY);
    f.push_back(g.WPB);
    f.push_back(g.PF);
    f.push_back(g.TX > 0 ? (double)(g.TX - g.SX) / g.TX : 0.0);
    f.push_back(g.fp16 ? 1 : 0);
    f.push_back(tx_size);
    f.push_back(std::log2(std::max<long long>(1, c.nwaves)));
    // analytical model (12)
    const Alg2Out& a = c.alg2;
    f.push_back(c.lds_per_wg / 1024.0);
    f.push_back(c.regs_est);
    f.push_back(a.shmem_occ);
    f.push_back(a.reg_occ);
    f.push_back(a.occupancy);
    f.push_back(a.terms[0]);
    f.push_back(a.terms[2]);
    f.push_back(a.terms[3]);
    f.push_back(a.terms[4]);
    f.push_back(a.terms[5]);
    f.push_back(a.terms[6]);
    f.push_back(a.score);
    // workload (6)
    f.push_back(std::log2(std::max(1, W)));
    f.push_back(std::log2(std::max(1, H)));
    f.push_back(std::log2(std::max(1.0, c.compulsory_bytes)));
    f.push_back(std::log2(std::max(1.0, c.valu_ops)));
    f.push_back(c.compulsory_bytes > 0 ? c.valu_ops / c.compulsory_bytes : 0.0);
    f.push_back(c.compulsory_bytes > 0 ? c.requested_bytes / c.compulsory_bytes : 1.0);
    return f;
}

}  // namespace wt
