// Plan objects shared by the runtime and the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "wt_internal.h"
#include "wt_cost.h"

namespace wt {

// Host mirror of the device-side WtArgs (device/wt_device.h); field order and
// sizes must match.
struct WtArgsHost {
    const void* src[16];
    void* dst[16];
    long long src_rs[16];
    long long src_cs[16];
    long long dst_rs[16];
    long long dst_cs[16];
    int W, H;
    int Ws, Hs;
    int tiles_x, tiles_y;
    int nwaves;
    int pad;
};
static_assert(sizeof(WtArgsHost) == 16 * 8 * 6 + 8 * 4, "WtArgs layout");

struct Buf {
    void* ptr = nullptr;
    int64_t rs = 0, cs = 0;
    bool half = false;
};

struct GroupRt {
    GroupSched g;
    GroupGeom geo;
    bool resample = false;
    std::string src, kname;            // src: both kernels (for inspection)
    std::string src_single, src_batch; // the two compiled modules
    hipModule_t mod = nullptr, mod_batch = nullptr;
    hipFunction_t fn = nullptr;        // single image, one wave (or block) per tile
    hipFunction_t fn_batch = nullptr;  // all images of a batch
    int W = 0, H = 0, Ws = 0, Hs = 0;
    int tiles_x = 0, tiles_y = 0, nwaves = 0;
    std::vector<int> loaded, liveouts;
    std::vector<bool> mem_half_in, mem_half_out;
};

// State of the last batch shape run through a plan (see batch.cpp).
struct BatchState {
    std::vector<std::pair<int, int>> sizes;
    void* arena = nullptr;
    size_t arena_bytes = 0;
    std::vector<std::map<int, Buf>> offs;  // per image: intermediates' offsets in the arena
    std::vector<std::map<int, Buf>> bufs;  // per image: intermediates in the arena
    std::vector<std::array<int, 3>> tiles; // [group][img]: tiles_x, tiles_y, work items
    std::vector<int> total, grid, per_cu;  // per group
    void* dargs = nullptr;                 // device argument table
    size_t args_bytes = 0, dargs_bytes = 0;
    std::vector<char> host;                // host copy of the table
    std::vector<char> uploaded;            // the table as last copied to the device
    // whole-pipeline launch (WT_PLAN_BATCH_WHOLE): chunk table and producer
    // masks at whole_off in the table, completion counters (zeroed by a
    // kernel before every launch) at ctr_off
    size_t whole_off = 0, ctr_off = 0;
    int nchunks = 0, ctr_words = 0, whole_grid = 0;
    bool whole_ran = false;                        // a whole-pipeline launch was issued
    std::vector<int> chunk_tab;                    // 4 ints per chunk
    std::vector<unsigned long long> dep_tab;       // per group
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool owned = true;                     // arena and table allocated for this state
    ~BatchState();
};

struct Plan {
    Pipeline p;
    Schedule sched;
    std::vector<GroupRt> groups;
    std::map<int, Buf> bufs;  // intermediates materialised between groups
    Machine machine;
    int W = 0, H = 0;
    int device = 0;
    bool no_device = false;
    bool no_compile = false;
    bool fp16 = false;
    bool any_width = false;
    bool batch_resident = false;  // WT_PLAN_BATCH_RESIDENT
    bool batch_whole = false;     // WT_PLAN_BATCH_WHOLE
    // the whole-pipeline kernel of the current groups (loaded on first use)
    std::string whole_src, whole_kname;
    hipModule_t whole_mod = nullptr;
    hipFunction_t whole_fn = nullptr;
    int whole_wpb = 2;
    hipStream_t setup_stream = nullptr;  // caller's stream for planning-time measurements
    std::string cache_dir;
    std::unique_ptr<BatchState> batch;
    std::unique_ptr<BatchState> batch_static;  // layout of the last run in the fixed workspace
    ~Plan();
};

struct ImgRef {
    const void* ptr;
    int64_t rs, cs;
};

void hip_check(hipError_t e, const char* what);

// Owned HIP stream and event pair, released on every exit path.
// A stream for the library's own measurements: the caller's when given
// (not destroyed), else one created and destroyed here.
struct OwnedStream {
    hipStream_t s = nullptr;
    bool owned = false;
    explicit OwnedStream(hipStream_t ext = nullptr) : s(ext) {
        if (!s) {
            hip_check(hipStreamCreate(&s), "hipStreamCreate");
            owned = true;
        }
    }
    ~OwnedStream() {
        if (s && owned) hipStreamDestroy(s);
    }
    OwnedStream(const OwnedStream&) = delete;
    OwnedStream& operator=(const OwnedStream&) = delete;
};
struct OwnedEvents {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    OwnedEvents() {
        hip_check(hipEventCreate(&e0), "hipEventCreate");
        if (hipEventCreate(&e1) != hipSuccess) {
            hipEventDestroy(e0);
            e0 = nullptr;
            hip_check(hipErrorOutOfMemory, "hipEventCreate");
        }
    }
    ~OwnedEvents() {
        if (e0) hipEventDestroy(e0);
        if (e1) hipEventDestroy(e1);
    }
    OwnedEvents(const OwnedEvents&) = delete;
    OwnedEvents& operator=(const OwnedEvents&) = delete;
};
// Bytes per element of node `id`'s images in memory (`half`: FP16 storage of
// a float intermediate).
inline int node_esize(const Pipeline& p, int id, bool half) {
    return p.nodes[id].is_int() ? dtype_size(p.nodes[id].dtype) : (half ? 2 : 4);
}
std::pair<int, int> level_dims(int W, int H, int level);
// a node's image size for a W x H pipeline: its level's, or bins x 1 for a
// histogram
std::pair<int, int> node_dims(const Pipeline& p, int id, int W, int H);
// Clears histogram outputs (int32 counts) before the group that accumulates
// them: `planes` planes of n counts, cs elements apart; the batched form
// takes output `d` of each of the nimg entries of a device argument table.
hipError_t zero_hist(void* base, long long cs, int n, int planes, hipStream_t s);
hipError_t zero_hist_batch(const void* table, int nimg, int d, int n, int planes, hipStream_t s);
void prepare_group(const Plan& plan, GroupRt& gr, int gi);
// With `failed`, a group that does not compile is marked there (and left
// unloaded) instead of failing the call.
void compile_groups(const Plan& plan, std::vector<GroupRt*>& grs, bool batch = false,
                    std::vector<bool>* failed = nullptr);
void unload_group(GroupRt& gr);
// Releases the plan's whole-pipeline kernel (its groups changed or the plan ends).
void unload_whole(Plan& plan);
// Validates a caller image against node `n` at W x H (null data, size,
// channels, element type, strides); returns its dense-resolved strides.
ImgRef check_image(const wt_image& im, const Node& n, int W, int H, const std::string& tag);
// Refuses live-out planes whose byte offsets would not fit the 32-bit
// offsets of buffer stores.
void check_store_planes(const Plan& plan, const GroupRt& gr, const WtArgsHost& a, int H);
void launch_group(const Plan& plan, const GroupRt& gr, const std::map<int, ImgRef>& mem, hipStream_t st);
void fill_args(const Plan& plan, const GroupRt& gr, const std::map<int, ImgRef>& mem, WtArgsHost& a,
               const std::string& tag);
int resident_blocks_per_cu(const Plan& plan, hipFunction_t fn, int threads);
// count < 0: every group, replayed from the batch shape's graph; otherwise
// groups [first, first + count), launched directly on the stream.
void run_plan_batch(Plan& plan, int nimg, const wt_image* in, const wt_image* out, void* stream, int first = 0,
                    int count = -1);
// The same batch with its intermediates and argument table in the library's
// fixed workspace, every group launched directly: no device allocation.
void run_plan_batch_static(Plan& plan, int nimg, const wt_image* in, const wt_image* out, void* stream);
// Times each group's configuration and its neighbours on this batch itself
// (the batched kernels over the caller's images), keeps the fastest per
// group, rebuilds the plan and runs the batch once more.
void tune_plan_batch(Plan& plan, int nimg, const wt_image* in, const wt_image* out, void* stream);
std::vector<GroupSched> config_neighbours(const GroupSched& best, int vmax);
// Compiles and loads the batched kernels of the groups that lack them.
void load_batch_kernels(const Plan& plan, std::vector<GroupRt>& groups);
// Chunk table (group, image, first tile, tiles per chunk) and per-group
// producer masks of the whole-pipeline launch for images of `sizes` with `rw`
// waves resident (no device needed).
void whole_tables(const Plan& plan, const std::vector<std::pair<int, int>>& sizes, long long rw,
                  std::vector<int>& chunk_tab, std::vector<unsigned long long>& dep_tab);
// Source of the whole-pipeline kernel of the plan's groups (named `kname`).
std::string whole_kernel_source(const Plan& plan, std::string& kname);
// WT_E_INTERNAL when the last whole-pipeline launch of the plan's batch gave
// up waiting for a producer (after synchronising `stream`).
void check_batch_status(Plan& plan, void* stream);
// The fixed workspace (scratch.hip): `device`'s copy, device current.
void* static_scratch(int device, hipError_t* err);
// Measures candidate configurations of every fused group and keeps the
// fastest; candidates ranked by the learned model when `model_path` is set.
// With `batch` > 1 the candidates are timed on an image as tall as up to
// `batch` images of the plan's size, the wave count of a batched launch.
// Returns the measured time of the chosen plan per image (the sum over its
// groups, in microseconds).  `memo` (optional) keeps each tuned group's
// choice and time by its stages, for tuning other groupings of the plan.
using TuneMemo = std::map<std::string, std::pair<GroupSched, double>>;
double autotune_plan(Plan& plan, int topk, const std::string& model_path = "", int batch = 1,
                     TuneMemo* memo = nullptr);
// Autotune schedule cache (see wt.h): key of a plan, lookup and store.
std::string schedule_text(const Schedule& s);
std::string tune_key(const Plan& plan, const wt_sched_opts& opts);
bool tune_cache_lookup(const std::string& dir, const std::string& key, std::string& text);
void tune_cache_store(const std::string& dir, const std::string& key, const std::string& text);
// Times every stage body of plan.p not yet profiled (needs a device).
void preprofile(const Plan& plan);
bool preprofile_enabled();
// Profile of stage `id` as the cost model sees it; `measure` runs the
// pre-profiling on the device first, otherwise only compiles its kernels.
StageProfile stage_profile(const Pipeline& p, int id, int W, int H, bool measure);
void measure_groups(const Pipeline& p, int W, int H, bool fp16, const std::vector<std::string>& descs, int reps,
                    const std::string& tag, double* out_us);
std::unique_ptr<Plan> create_plan(const Pipeline& p, const wt_sched_opts* o, int W, int H, void* stream);
// WT_VERBOSE is set: planning steps that measure report progress on stderr.
bool verbose();
void build_groups(Plan& plan);
void run_plan(Plan& plan, const wt_image* in, int nin, const wt_image* out, int nout, void* stream);
std::string describe_plan(const Plan& plan);

}  // namespace wt
