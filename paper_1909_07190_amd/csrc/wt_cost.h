// Analytical cost model (Algorithm 2) and the gfx950 schedule adapter.
#pragma once
#include <map>
#include <memory>

#include "wt_internal.h"

namespace wt {

// Quantities Algorithm 2 reads.
struct Alg2In {
    double smem_per_wg = 0;          // scratchpad bytes per thread block (after the hybrid split)
    double regs_per_lane = 0;        // register tile + per-stage register usage
    int waves_per_wg = 1;
    long long total_wg = 1;
    double total_tx = 0;             // global-memory transactions of the whole launch
    double compulsory_tx = 1;        // transactions for the group's inputs read once
    double mem_bytes_per_wave = 0;   // bytes one wave moves
    double compute_time_per_wave = 0;  // seconds: sum of TimePerIter x points per lane
    double frac_overlap = 0;         // redundant / useful computations
};
struct Alg2Out {
    bool feasible = false;
    int max_wg_per_cu = 0;
    int shmem_occ = 0, reg_occ = 0;  // waves per CU allowed by LDS / registers
    double occupancy = 0;
    double mem_over_compute = 0, unalloc_smem = 0, unused_reg = 0, extra_wg = 0;
    double terms[7] = {0, 0, 0, 0, 0, 0, 0};
    double score = 0;
};
Alg2Out alg2(const Alg2In& in, const Machine& m, const double w[7]);

Machine machine_gtx1080ti();
Machine machine_gfx950();
void warp_sizes(const int B[3], int ws, int W[3]);
long long scratchpad_elems(const int T[3], const int B[3], const int W[3], const int O[3]);
int waves_per_cu_by_regs(const Machine& m, double regs_per_lane);

// Per-stage pre-profiling result (Section 6): time per iteration and
// register usage of one stage's body.
struct StageProfile {
    double ns_per_point = 0;
    int vgprs = 0;
    int valu_ops = 0;
    bool measured = false;
};
StageProfile estimate_stage(const Pipeline& p, int id, const Machine& m);
// The measured profile of a stage, if pre-profiling has timed its signature.
bool lookup_profile(const Pipeline& p, int id, StageProfile& out);

struct GroupCost {
    Alg2Out alg2;
    double pred_us = 0;          // predicted kernel time
    double regs_est = 0, lds_per_wg = 0;
    double requested_bytes = 0, compulsory_bytes = 0, valu_ops = 0;
    long long nwaves = 0;
    double code_ops = 0;         // straight-line VALU operations per kernel body
    double cal_us = 0;           // calibrated time (active_fit())
};
// `batch`: images of this size run together (one launch per group over
// all of them), which multiplies the waves and the compulsory traffic.
GroupCost group_cost(const Pipeline& p, const GroupSched& g, const GroupGeom& geo, const Machine& m, int W,
                     int H, const std::map<int, StageProfile>& prof, int tx_size, const double w[7], int batch = 1);
// One scored configuration of a group.
struct ScoredConfig {
    GroupSched g;
    GroupCost cost;
    int tx_size = 128;
    std::shared_ptr<const GroupGeom> geo;  // geometry of (V, TX, SX, PF)
};
// Every feasible configuration of the group `nodes` (writing the down2
// stages `dec` decimated) over the search grid.
std::vector<ScoredConfig> score_configs(const Pipeline& p, const Machine& m, const SchedRequest& r,
                                        const std::vector<int>& nodes, const std::vector<int>& dec = {});
// Algorithm 2's weights as the paper's Table 3 gives them for the V100 (the
// score keeps the paper's form; it is also one of the learned model's
// features).
extern const double kGfx950Weights[7];
// The analytical model refitted on gfx950 measurements: calibrated time
// exp(c0 + c1 log(pred_us) + sum_k w_k term_k), the quantity the analytical
// scheduler minimises within a group and sums across groups.
struct AnalyticFit {
    double c0, c1, w[7];
};
extern const AnalyticFit kGfx950Fit;
// The fit in use: kGfx950Fit, or nine numbers "c0,c1,w0,...,w6" from
// $WT_ANALYTIC_FIT (read once; for evaluating refits without a rebuild).
const AnalyticFit& active_fit();
double calibrated_us(double pred_us, const double terms[7], const AnalyticFit& f);

// 40 features of a (group, configuration) for the learned cost model:
// 12 structural, 10 schedule, 12 analytical-model terms, 6 workload.
constexpr int kNumFeatures = 40;
std::vector<double> group_features(const Pipeline& p, const GroupSched& g, const GroupGeom& geo,
                                   const GroupCost& c, int W, int H, int tx_size);

double resample_pred_us(const Pipeline& p, int id, const Machine& m, int W, int H, bool half_in, bool half_out);

}  // namespace wt
