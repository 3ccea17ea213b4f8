// Internal types of the wavetile library (host side).
#pragma once

#include <cstdint>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/wt.h"

namespace wt {

struct Mlp;

// Error carried across internal layers; converted to wt_status at the C ABI.
struct Error : std::runtime_error {
    wt_status status;
    Error(wt_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};
[[noreturn]] void fail(wt_status s, const std::string& msg);

// ---------------------------------------------------------------- IR -----

// Pointwise expression tree.
struct Expr {
    enum Op { Const, Src, Neg, Add, Sub, Mul, Div, Lt, Le, Gt, Ge,
              Abs, Min, Max, Select, Sqrt, Floor };
    Op op = Const;
    double value = 0.0;  // Const
    int src = -1;        // Src: index into the stage's source list
    int chan = -1;       // Src: explicit channel, or -1 for "same channel"
    std::vector<Expr> kids;
};
Expr parse_expr(const std::string& text, int nsrc);
// max |value| over all points, given bounds on each source's magnitude.
double expr_bound(const Expr& e, const std::vector<double>& src_bounds);
bool expr_has_explicit_channel(const Expr& e);
int expr_max_channel(const Expr& e, int src);

enum class Kind { Input, Stencil, Pointwise, Down2, Up2, Hist, Equalize };

// Element types (wt_dtype): integer stages compute exactly in 32-bit
// integers and saturate to their type's range.
bool is_int_dtype(int dt);
int dtype_size(int dt);                        // bytes per element in memory
std::pair<long long, long long> dtype_range(int dt);
const char* dtype_ctype(int dt);               // C type of one element
// Interval [lo, hi] of an expression over sources in the given intervals,
// and the largest magnitude any subexpression can take.
struct Interval { double lo, hi; };
Interval expr_range(const Expr& e, const std::vector<Interval>& srcs, double* max_abs);

struct Tap { int dx, dy; double w; };

struct Node {
    Kind kind = Kind::Input;
    int id = -1;
    int channels = 1;
    int level = 0;               // pyramid level (0 = input resolution)
    std::vector<int> srcs;
    // stencil
    int kw = 1, kh = 1, ax = 0, ay = 0;
    std::vector<double> weights;
    double scale = 1.0;
    // pointwise
    std::string expr_text;
    Expr expr;
    double bound = 1.0;          // magnitude bound (float inputs: 1, or as declared)
    // element type; integer stencils use integer weights and a divisor
    int dtype = WT_F32;
    std::vector<long long> iweights;
    long long divisor = 1;
    double rlo = 0, rhi = 0;     // integer stages: value interval (after saturation)
    // histogram (a reduction): per channel, `bins` int32 counts of the
    // source's values over [hlo, hhi); its image is bins x 1
    int bins = 0;
    double hlo = 0, hhi = 1;
    bool is_int() const { return is_int_dtype(dtype); }
};

struct Pipeline {
    std::vector<Node> nodes;
    std::vector<int> inputs;     // node ids of inputs, creation order
    std::vector<int> outputs;    // node ids of outputs, wt_output order
    // consumers[n] = node ids reading n
    std::vector<std::vector<int>> consumers() const;
    // Constant-offset taps of consumer c on producer p (empty if c does not
    // read p, or reads it through a resampling dependence).  A foldable up2
    // (below) has the 5x5 footprint {-2..2}^2 on the stage it folds (weight
    // 0 in the list: its weights depend on the parity of the point).
    std::vector<Tap> taps(int c, int p) const;
    // The stage P an up2 node u folds, or -1.  u = up2(down2(P)) with P a
    // float stencil or pointwise stage is, at P's level, a constant-offset
    // dependence on P (the paper's alignment and scaling, Section 5): the
    // 2x expansion of P's even samples reads P at offsets -2..2 in x and y,
    // with weights set by the parity of the point.  A fused group that holds
    // P and writes the down2 decimated may then compute u from P's rows.
    int fold_source(int u) const;
    bool is_output(int n) const;
    // FP16 storage (the plan's FP16-intermediate option) is allowed for
    // float stages whose magnitude bound fits FP16's finite range; every
    // other stage keeps its own element type.
    bool half_storable(int n) const;
};

// ---------------------------------------------------------- schedule -----

// One fused group and its tile configuration (the paper's tile sizes, thread
// block size and register fraction, Algorithm 2's arguments).
struct GroupSched {
    std::vector<int> nodes;  // member stage ids, topological order
    int V = 4;               // contiguous elements per lane along x
    int TX = 1;              // sub-tiles along x, each 64*V columns
    int SX = 0;              // leading sub-tiles kept in LDS (TX-SX in VGPRs)
    int TY = 16;             // output rows per wave tile
    int WPB = 1;             // waves per workgroup
    bool fp16 = false;       // intermediates stored as FP16
    int PF = 1;              // rows of input loaded ahead of their first use
    int XCD = 0;             // 1: remap workgroups so each XCD gets adjacent tiles
    int ORD = 0;             // tile order of the wave index: 0 rows of tiles fastest
                             // (vertical neighbours adjacent), 1 columns fastest
    int NT = 0;              // 1: non-temporal loads and stores
    int align = 0;           // 0: centred (reads from both neighbours);
                             // 1: the paper's right-hyperplane skew (reads from the left only)
    std::vector<int> dec;    // down2 stages this group writes directly: the even
                             // rows and columns of a member, stored decimated
    std::vector<int> exp;    // up2 stages this group reads by expanding their
                             // coarse source on the fly (never materialised)
    std::vector<int> hst;    // histogram stages this group accumulates from a
                             // member's values as it computes them
    int BLK = 0;             // 1: one tile per workgroup, stages in LDS with
                             // workgroup barriers between them (the paper's
                             // OTPTB baseline); tile (64*V*TX) x TY
    int GH = 0;              // 1: loaded rows carry ghost columns (the halo
                             // their direct consumers read past the tile's
                             // slots) in the edge lanes of two extra
                             // registers, so those consumers are valid on every
                             // slot and tiles start on 64*V*TX-column
                             // boundaries (requires SX=0, align=0)
};
int block_tile_w(const GroupSched& g);  // output columns of a BLK tile
bool is_resample_group(const Pipeline& p, const GroupSched& g);
// a lone histogram stage (its source read from memory)
bool is_hist_group(const Pipeline& p, const GroupSched& g);
// Copies of a wave's histogram bins for `words` = bins x channel slots (lane
// t counts into copy t mod R, each copy `words + 1` words long so that one
// bin's copies fall in different LDS banks): up to 8, within 16 KiB, so that
// neighbouring lanes counting into one bin do not serialise on one address.
inline int hist_replicas(int words) {
    int r = 1;
    while (r < 8 && (words + 1) * r * 2 <= 4096) r *= 2;
    return r;
}

struct Schedule { std::vector<GroupSched> groups; };

std::string describe_group(const GroupSched& g);
// `partial`: the text may name a subset of the stages (measurement).
Schedule parse_schedule(const std::string& text, const Pipeline& p, bool partial = false);

// Geometry of a stencil/pointwise group (Section 4's warp-overlapped tile with
// Section 5's skewed sub-tiles); see geometry.cpp.
struct NodeGeom {
    int id;
    bool member;        // computed in the group (else loaded from memory)
    bool liveout;       // stored to memory
    bool out = false;   // needed over the tile's output range (live-out or decimated)
    int expand_src = -1; // loaded up2 node computed from this coarse node on the fly
    int skew;           // x alignment a_n: slot j <-> x = x0 - skew + j
    int lead;           // at step k the node holds row k + lead
    int win;            // rows kept (ring size)
    int nch;            // storage channels held by one wave
    bool fix_top, fix_bot, fix_x;  // clamp fix-ups needed (see codegen)
    int vlo;            // first valid slot
    int vhi;            // invalid slots at the right end of a row
    int first_step;     // first step (0 = tile start) at which its row is needed
    bool consumed;      // read by another member of the group
    bool even_rows = false;  // only its even rows are used (by decimated
                             // stores and folded up2s): odd rows may be skipped
    int lds_off;        // byte offset of its LDS ring within the wave's LDS
    bool half;          // in-group storage is FP16
    bool mem_half;      // its memory buffer holds FP16 (set by the runtime)
    int ghl = 0, ghr = 0;  // ghost columns loaded left / right of the slots (GH=1)
};
struct GroupGeom {
    std::vector<NodeGeom> nodes;    // loaded nodes first, then members (topo)
    std::map<int, int> index;       // node id -> position in `nodes`
    bool chan_parallel = true;      // one channel per wave
    int C = 1;                      // channel count when chan_parallel
    int N = 0;                      // slots per row = TX*64*V
    int X = 0;                      // output columns per tile
    int S0 = 0;                     // first stored slot
    int base = 0;                   // x0 of tile 0
    int D = 0;                      // warm-up steps before the first output row
    int U = 1;                      // steps per unrolled loop body
    int NMAIN = 0;                  // full U-step periods of the main loop
    int E = 0;                      // epilogue steps (TY = NMAIN*U + E)
    int lds_bytes = 0;              // LDS bytes per wave
    int lds_bytes_per_wg = 0;
    std::vector<int> loaded, liveouts;
    std::vector<std::pair<int, int>> dec;  // (down2 node, member it decimates)
    std::vector<int> outs;          // nodes needed over the tile's output range:
                                    // live-outs, decimated members and the
                                    // sources of accumulated histograms
    std::vector<std::pair<int, int>> hist;  // (histogram node, member it counts)
    int hist_lds_off = 0;           // the wave's histogram bins in its LDS
    std::vector<int> tables;        // histograms read whole by equalize members
                                    // (after `loaded` in the source slots)
    int table_lds_off = 0;          // their cumulative counts in the wave's LDS
};
GroupGeom group_geometry(const Pipeline& p, const GroupSched& g);

// ---------------------------------------------------------- machine ------
// The paper's Table 1 parameters, for gfx950 (MI355X) by default.
struct Machine {
    std::string name = "gfx950";
    int ncu = 256;                 // compute units (NSMs)
    int simd_per_cu = 4;
    int wave = 64;                 // WarpSize
    int vgpr_per_simd_lane = 512;  // VGPR file per lane per SIMD
    int vgpr_granule = 8;          // allocation granule
    int max_waves_per_simd = 8;
    int max_waves_per_cu = 32;     // MaxWarpPerSM
    int max_wg_per_cu = 32;        // MaxTbPerSM
    int lds_per_cu = 160 * 1024;   // ShMemPerSM
    int max_lds_per_wg = 160 * 1024;  // MaxShMemPerTb
    int regs_per_cu = 131072;      // RegPerSM (4 SIMDs x 512 VGPRs x 64 lanes)
    int max_regs_per_lane = 256;   // MaxRegPerThread (architectural VGPRs)
    bool amd_vgpr_alloc = true;    // occupancy from per-SIMD VGPR allocation
    int cores_per_cu = 64;         // 4 SIMDs x 16 lanes
    double hbm_bw = 8.0e12;        // GlMemBW, bytes / s
    double clock_hz = 2.4e9;
    int tx_sizes[2] = {64, 128};   // GlMemTxSize candidates, bytes
    double mem_latency_s = 2.0e-6; // loaded HBM latency (bytes in flight needed)
    double hbm_efficiency = 0.75;  // achievable fraction of peak for streaming
    double launch_us = 2.0;        // per-kernel launch and drain
    int max_vgpr_per_wave = 256;   // architectural VGPRs addressable by a wave
    // Straight-line code bound: estimated VALU operations emitted per kernel
    // body (prologue + unrolled main loop + epilogue, every member, every
    // element a lane owns).  Beyond it the kernel no longer fits the
    // instruction cache and takes tens of seconds to compile.
    double max_code_ops = 12000;
};
Machine machine_from_device(int device);  // falls back to the constant table

// ------------------------------------------------------------- codegen ---
// A group's kernels: the single-image kernel `kname` and the batched
// kernel `kname_batch` (its waves loop over the tiles of all images with the
// launch's stride, so any grid size covers them), each after the shared
// device prelude.
// They are compiled as separate modules (the batched one on first use).
struct GroupSources {
    std::string prelude, common, single, batch;  // common: helpers both kernels call
    std::string full() const { return prelude + "\n" + common + single + "\n" + batch; }
    std::string single_module() const { return prelude + "\n" + common + single; }
    std::string batch_module() const { return prelude + "\n" + common + batch; }
};
GroupSources generate_group_source(const Pipeline& p, const GroupSched& g,
                                   const GroupGeom& geo, const std::string& kname);
GroupSources generate_resample_source(const Pipeline& p, const GroupSched& g,
                                      const std::string& kname, bool src_half, bool dst_half);
// A lone histogram stage: counts its source read from memory.
// The batch's whole group sequence as one persistent kernel `kname`
// (wave-tiled fused groups only; `wpb` waves per workgroup); sets
// `lds_per_wave` to the LDS each wave holds.
std::string generate_whole_source(const Pipeline& p, const std::vector<const GroupSched*>& gs,
                                  const std::vector<const GroupGeom*>& geos, const std::string& kname, int wpb,
                                  int& lds_per_wave);
GroupSources generate_hist_source(const Pipeline& p, const GroupSched& g, const std::string& kname, bool src_half);
// Output pixels one 256-thread workgroup of a resampling kernel covers:
// down2 64 x 4 (a pixel per thread), up2 128 x 8 (a 2x2 quad per thread);
// source pixels of a lone histogram's workgroup: 64 x 64.
void resample_block(const Pipeline& p, const GroupSched& g, int& bw, int& bh);
std::string device_prelude();

// ----------------------------------------------------------- scheduler ---
struct SchedRequest {
    int mode = WT_SCHED_ANALYTIC;
    bool fp16 = false;
    int W = 0, H = 0;
    std::string fixed;
    std::string model_path;
    int max_group = 12;               // bound on stages per fused group
    bool any_width = false;           // caller images of any width / stride
    int batch = 1;                    // images per batched run (analytical cost only)
    bool fold = true;                 // the search may fold up2 stages into groups
    const double* weights = nullptr;  // Algorithm 2 weights (default: refitted table)
    Mlp* model = nullptr;             // learned cost model (WT_SCHED_MLP)
};
Schedule make_schedule(const Pipeline& p, const Machine& m, const SchedRequest& r);
Schedule schedule_unfused(const Pipeline& p, bool fp16);
int max_vector_width(const Pipeline& p, const GroupSched& g, int W, int H, bool any_width = false);
void fusion_costs(const Pipeline& p, const Machine& m, const SchedRequest& r, double* dp, double* brute);

// ----------------------------------------------------------------- jit ---
std::vector<char> compile_hip(const std::string& src, const std::string& name,
                              const std::string& cache_dir);

}  // namespace wt
