// Batched execution: many images of different sizes through one plan, one
// launch per group covering the tiles of every image, the whole
// group sequence captured once per batch shape in a hipGraph and replayed.
//
// Per batch shape (the list of image sizes) the plan keeps: an arena with
// every image's intermediates, a device table of per-image kernel arguments
// for every group (rewritten before each run, so only the pointers of the
// caller's images may change between runs), the per-group work prefix sums
// and the instantiated graph.
#include <cstdlib>
#include <cstdio>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <set>

#include "wt_runtime.h"

namespace wt {

BatchState::~BatchState() {
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    if (owned && arena) hipFree(arena);
    if (owned && dargs) hipFree(dargs);
}

// Workgroups of `fn` resident on one CU: the runtime's occupancy answer, or
// the count from the kernel's VGPR and LDS use (waves per SIMD =
// min(8, 512 / VGPRs rounded up to the allocation granule of 8), 4 SIMDs per
// CU), whichever is larger.  Launching more than fit only queues workgroups.
int resident_blocks_per_cu(const Plan& plan, hipFunction_t fn, int threads) {
    int api = 0;
    if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&api, fn, threads, 0) != hipSuccess) api = 0;
    int regs = 0, lds = 0;
    if (hipFuncGetAttribute(&regs, HIP_FUNC_ATTRIBUTE_NUM_REGS, fn) != hipSuccess) regs = 0;
    if (hipFuncGetAttribute(&lds, HIP_FUNC_ATTRIBUTE_SHARED_SIZE_BYTES, fn) != hipSuccess) lds = 0;
    int alloc = std::max(8, (regs + 7) / 8 * 8);
    int waves_simd = std::min(8, 512 / alloc);
    int waves_wg = (threads + 63) / 64;
    int own = std::max(1, 4 * waves_simd / waves_wg);
    if (lds > 0) own = std::max(1, std::min(own, plan.machine.lds_per_cu / lds));
    int res = std::max(api, own);
    if (const char* e = std::getenv("WT_DEBUG_BATCH"))
        if (*e && *e != '0')
            std::fprintf(stderr, "wavetile batch: threads=%d regs=%d lds=%d api=%d own=%d -> %d per CU\n", threads,
                         regs, lds, api, own, res);
    return res;
}

namespace {

// WT_PLAN_BATCH_RESIDENT (or WT_BATCH_GRID=resident in the environment)
// sizes a batched launch to the workgroups that fit on the device at once,
// each looping over its share of the work units (persistent); by default
// every work unit gets a workgroup of its own and the hardware dispatcher
// hands them out as earlier ones finish, which balances the uneven tiles of
// a batch better (17-20% faster on the 64-image pyramid blend).
bool batch_grid_resident(const Plan& plan) {
    if (plan.batch_resident) return true;
    const char* e = std::getenv("WT_BATCH_GRID");
    return e && std::string(e) == "resident";
}

// One group's batched launch (the kernel over every image's work units).
hipError_t launch_batch_group(const Plan& plan, const BatchState& st, int g, int nimg, hipStream_t s) {
    const GroupRt& gr = plan.groups[g];
    const void* a = static_cast<char*>(st.dargs) + (size_t)g * nimg * sizeof(WtArgsHost);
    const void* starts = static_cast<char*>(st.dargs) + st.args_bytes + (size_t)g * (nimg + 1) * sizeof(int);
    int ni = nimg, tot = st.total[g];
    for (size_t i = 0; i < gr.liveouts.size(); ++i) {  // histograms accumulate from zero
        const Node& hn = plan.p.nodes[gr.liveouts[i]];
        if (hn.kind == Kind::Hist) {
            hipError_t ez = zero_hist_batch(a, nimg, (int)i, hn.bins, hn.channels, s);
            if (ez != hipSuccess) return ez;
        }
    }
    void* params[] = {&a, &starts, &ni, &tot};
    int threads = gr.resample ? 256 : 64 * gr.g.WPB;
    return hipModuleLaunchKernel(gr.fn_batch, st.grid[g], 1, 1, threads, 1, 1, 0, s, params, nullptr);
}

// Host mirror of the whole-pipeline kernel's argument (WtWhole in the
// generated source).
struct WtWholeHost {
    const void* AB;
    const void* start;
    const void* chunks;
    const void* deps;
    void* done;
    void* next;
    void* status;
    long long limit;
    int nchunks, nimg;
};
static_assert(sizeof(WtWholeHost) == 72, "WtWhole layout");

// Ticks of the device's constant-rate clock in two seconds: the longest a
// wave of the whole-pipeline kernel waits for a producer (a launch of the
// largest batches takes milliseconds).
long long whole_wait_limit(int device) {
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) != hipSuccess || khz <= 0) khz = 100000;
    return 2000LL * khz;
}

// The whole group sequence as one launch: the counters cleared by a kernel
// (graph-safe), then the persistent kernel.
hipError_t launch_whole(const Plan& plan, const BatchState& st, int nimg, hipStream_t s) {
    char* base = static_cast<char*>(st.dargs);
    const int G = (int)plan.groups.size();
    hipError_t e = zero_hist(base + st.ctr_off, 0, st.ctr_words, 1, s);
    if (e != hipSuccess) return e;
    WtWholeHost w;
    w.AB = base;
    w.start = base + st.args_bytes;
    w.chunks = base + st.whole_off;
    w.deps = base + st.whole_off + (size_t)st.nchunks * 16;
    w.done = base + st.ctr_off;
    w.next = base + st.ctr_off + (size_t)G * nimg * 4;
    w.status = base + st.ctr_off + ((size_t)G * nimg + 1) * 4;
    w.limit = whole_wait_limit(plan.device);
    w.nchunks = st.nchunks;
    w.nimg = nimg;
    void* params[] = {&w};
    return hipModuleLaunchKernel(plan.whole_fn, st.whole_grid, 1, 1, 64 * plan.whole_wpb, 1, 1, 0, s, params, nullptr);
}

}  // namespace

std::string whole_kernel_source(const Plan& plan, std::string& kname) {
    std::vector<const GroupSched*> gs;
    std::vector<const GroupGeom*> geos;
    uint64_t h = 1469598103934665603ull;
    for (const auto& gr : plan.groups) {
        if (gr.resample) fail(WT_E_UNSUPPORTED, "whole-pipeline launch of a lone resampling or histogram group");
        gs.push_back(&gr.g);
        geos.push_back(&gr.geo);
        for (unsigned char c : gr.kname + ";") h = (h ^ c) * 1099511628211ull;
    }
    char hb[32];
    std::snprintf(hb, sizeof hb, "%012llx", (unsigned long long)(h & 0xffffffffffffull));
    kname = std::string("wt_whole_") + hb;
    int lds = 0;
    return generate_whole_source(plan.p, gs, geos, kname, plan.whole_wpb, lds);
}

namespace {

// The whole-pipeline kernel of the plan's groups, generated, compiled and
// loaded once per grouping.
void load_whole_kernel(Plan& plan) {
    if (plan.whole_fn) return;
    std::string kname;
    std::string src = whole_kernel_source(plan, kname);
    std::vector<char> code = compile_hip(src, kname, plan.cache_dir);
    hip_check(hipModuleLoadData(&plan.whole_mod, code.data()), "hipModuleLoadData");
    hip_check(hipModuleGetFunction(&plan.whole_fn, plan.whole_mod, kname.c_str()), "hipModuleGetFunction");
    plan.whole_src = src;
    plan.whole_kname = kname;
}

// Counters and table offsets of the whole-pipeline launch for the batch
// shape of `st` (after layout_batch); the chunks and producer masks come from
// whole_tables with the launch's resident waves.
void layout_whole(const Plan& plan, BatchState& st) {
    const int G = (int)plan.groups.size(), nimg = (int)st.sizes.size();
    const int per_cu = resident_blocks_per_cu(plan, plan.whole_fn, 64 * plan.whole_wpb);
    whole_tables(plan, st.sizes, (long long)per_cu * plan.machine.ncu * plan.whole_wpb, st.chunk_tab, st.dep_tab);
    st.nchunks = (int)(st.chunk_tab.size() / 4);
    st.whole_grid = (int)std::max(1LL, std::min((long long)st.nchunks, (long long)per_cu * plan.machine.ncu));
    st.whole_off = (st.dargs_bytes + 15) / 16 * 16;
    const size_t tab_end = st.whole_off + (size_t)st.nchunks * 16 + (size_t)G * 8;
    st.ctr_off = (tab_end + 255) / 256 * 256;
    st.ctr_words = G * nimg + 2;
    st.host.resize(tab_end);
    st.dargs_bytes = st.ctr_off + (size_t)st.ctr_words * 4;
}

// The chunk table and producer masks into the host table (after fill_table).
void fill_whole(BatchState& st) {
    std::memcpy(st.host.data() + st.whole_off, st.chunk_tab.data(), st.chunk_tab.size() * sizeof(int));
    std::memcpy(st.host.data() + st.whole_off + (size_t)st.nchunks * 16, st.dep_tab.data(),
                st.dep_tab.size() * sizeof(unsigned long long));
}

void tile_counts(const Plan& plan, const GroupRt& gr, int lw, int lh, int& tx, int& ty, int& work) {
    const Pipeline& p = plan.p;
    if (gr.resample) {
        int bw, bh;
        resample_block(p, gr.g, bw, bh);
        tx = (lw + bw - 1) / bw;
        ty = (lh + bh - 1) / bh;
        work = tx * ty * p.nodes[gr.g.nodes[0]].channels;
        return;
    }
    int amin = 1 << 30, amax = 0;
    for (int lo : gr.geo.outs) {
        const NodeGeom& ng = gr.geo.nodes[gr.geo.index.at(lo)];
        amin = std::min(amin, ng.skew);
        amax = std::max(amax, ng.skew);
    }
    if (gr.g.BLK) {  // work items are tiles (one workgroup each)
        int bw = block_tile_w(gr.g);
        tx = (lw + bw - 1) / bw;
        ty = (lh + gr.g.TY - 1) / gr.g.TY;
        work = tx * ty * (gr.geo.chan_parallel ? gr.geo.C : 1);
        return;
    }
    tx = (lw - (amin - amax) + gr.geo.X - 1) / gr.geo.X;
    ty = (lh + gr.g.TY - 1) / gr.g.TY;
    work = tx * ty * (gr.geo.chan_parallel ? gr.geo.C : 1);
}


}  // namespace

void whole_tables(const Plan& plan, const std::vector<std::pair<int, int>>& sizes, long long rw,
                  std::vector<int>& chunk_tab, std::vector<unsigned long long>& dep_tab) {
    const Pipeline& p = plan.p;
    const int G = (int)plan.groups.size(), nimg = (int)sizes.size();
    if (G > 64) fail(WT_E_UNSUPPORTED, "whole-pipeline launch needs 1 to 64 groups");
    chunk_tab.clear();
    dep_tab.assign(G, 0ull);
    rw = std::max(1LL, rw);
    for (int g = 0; g < G; ++g) {
        const GroupRt& gr = plan.groups[g];
        if (gr.resample) fail(WT_E_UNSUPPORTED, "whole-pipeline launch of a lone resampling or histogram group");
        if (gr.g.BLK) fail(WT_E_UNSUPPORTED, "whole-pipeline launch of a one-tile-per-workgroup group");
        if (!gr.geo.hist.empty() || !gr.geo.tables.empty())
            fail(WT_E_UNSUPPORTED, "whole-pipeline launch of a histogram or equalize stage");
        for (int l : gr.loaded)
            for (int q = 0; q < g; ++q)
                if (std::find(plan.groups[q].liveouts.begin(), plan.groups[q].liveouts.end(), l) !=
                    plan.groups[q].liveouts.end())
                    dep_tab[g] |= 1ull << q;
        std::vector<int> work(nimg);
        long long total = 0;
        for (int i = 0; i < nimg; ++i) {
            auto d = level_dims(sizes[i].first, sizes[i].second, p.nodes[gr.g.nodes[0]].level);
            int tx, ty;
            tile_counts(plan, gr, d.first, d.second, tx, ty, work[i]);
            total += work[i];
        }
        // about eight chunks per resident wave and group, at most 64 tiles each
        const int k = (int)std::max(1LL, std::min(64LL, total / (8 * rw)));
        for (int i = 0; i < nimg; ++i)
            for (int t = 0; t < work[i]; t += k) chunk_tab.insert(chunk_tab.end(), {g, i, t, std::min(k, work[i] - t)});
    }
}

namespace {

// The caller's images of a batch, validated as single runs validate theirs:
// per image its size and the memory of its inputs and outputs.
void check_batch(const Plan& plan, int nimg, const wt_image* in, const wt_image* out,
                 std::vector<std::pair<int, int>>& sizes, std::vector<std::map<int, ImgRef>>& mem) {
    const Pipeline& p = plan.p;
    const int nin = (int)p.inputs.size(), nout = (int)p.outputs.size();
    if (nimg < 1) fail(WT_E_INVALID, "batch needs at least one image");
    if (!in || !out) fail(WT_E_INVALID, "null image array");
    sizes.assign(nimg, {0, 0});
    mem.assign(nimg, {});
    for (int i = 0; i < nimg; ++i) {
        const wt_image& first = in[(size_t)i * nin];
        int W = first.width, H = first.height;
        if (W <= 0 || H <= 0 || W > (1 << 24) || H > (1 << 24)) fail(WT_E_SHAPE, "bad image size in batch");
        sizes[i] = {W, H};
        for (int k = 0; k < nin; ++k) {
            const wt_image& im = in[(size_t)i * nin + k];
            int id = p.inputs[k];
            mem[i][id] = check_image(im, p.nodes[id], W, H, "batch image " + std::to_string(i) + " input " + std::to_string(k));
        }
        for (int k = 0; k < nout; ++k) {
            const wt_image& im = out[(size_t)i * nout + k];
            int id = p.outputs[k];
            auto d = node_dims(p, id, W, H);
            mem[i][id] = check_image(im, p.nodes[id], d.first, d.second,
                                     "batch image " + std::to_string(i) + " output " + std::to_string(k));
        }
    }
    // no output may alias any other image of the batch
    std::map<const void*, int> seen;  // data pointer -> times named
    for (int i = 0; i < nimg * nin; ++i) ++seen[in[i].data];
    for (int i = 0; i < nimg * nout; ++i) ++seen[out[i].data];
    for (int i = 0; i < nimg * nout; ++i)
        if (seen[out[i].data] > 1)
            fail(WT_E_INVALID, "batch image " + std::to_string(i / std::max(nout, 1)) + " output " +
                                   std::to_string(i % std::max(nout, 1)) + " aliases another image");
}

// Everything of a batch shape that needs no device memory: every image's
// intermediates at 256-byte aligned offsets from the arena's start, the
// per-group work and launch grids, and the argument table's size.  The
// batched kernels must be loaded.
std::unique_ptr<BatchState> layout_batch(const Plan& plan, const std::vector<std::pair<int, int>>& sizes) {
    const Pipeline& p = plan.p;
    const int nimg = (int)sizes.size(), G = (int)plan.groups.size();
    auto st = std::make_unique<BatchState>();
    st->sizes = sizes;
    st->offs.assign(nimg, {});
    size_t off = 0;
    for (int i = 0; i < nimg; ++i)
        for (auto& gr : plan.groups)
            for (size_t k = 0; k < gr.liveouts.size(); ++k) {
                int id = gr.liveouts[k];
                if (p.is_output(id) || st->offs[i].count(id)) continue;
                auto d = node_dims(p, id, sizes[i].first, sizes[i].second);
                Buf b;
                b.half = gr.mem_half_out[k];
                b.rs = (d.first + 63) / 64 * 64;
                b.cs = b.rs * d.second;
                b.ptr = reinterpret_cast<void*>(off);  // an offset until the arena is placed
                off += ((size_t)b.cs * p.nodes[id].channels * node_esize(p, id, b.half) + 255) / 256 * 256;
                st->offs[i][id] = b;
            }
    st->arena_bytes = off;
    st->total.resize(G);
    st->grid.resize(G);
    st->per_cu.resize(G);
    st->tiles.assign((size_t)G * nimg, {0, 0, 0});
    for (int g = 0; g < G; ++g) {
        int tot = 0;
        for (int i = 0; i < nimg; ++i) {
            auto d = level_dims(sizes[i].first, sizes[i].second, p.nodes[plan.groups[g].g.nodes[0]].level);
            int tx, ty, w;
            tile_counts(plan, plan.groups[g], d.first, d.second, tx, ty, w);
            st->tiles[(size_t)g * nimg + i] = {tx, ty, w};
            tot += w;
        }
        st->total[g] = tot;
        const GroupRt& gr = plan.groups[g];
        int threads = gr.resample ? 256 : 64 * gr.g.WPB;
        int per_cu = resident_blocks_per_cu(plan, gr.fn_batch, threads);
        st->per_cu[g] = per_cu;
        int units = (gr.resample || gr.g.BLK) ? tot : (tot + gr.g.WPB - 1) / gr.g.WPB;
        // the per-unit grid is capped at 2^22 workgroups (far above the
        // resident set; the waves' stride loop covers any remainder)
        st->grid[g] = batch_grid_resident(plan) ? std::max(1, std::min(units, per_cu * plan.machine.ncu))
                                                : std::max(1, std::min(units, 1 << 22));
    }
    // argument table: [g][img] WtArgs, then [g][nimg + 1] work prefix sums
    st->args_bytes = (size_t)G * nimg * sizeof(WtArgsHost);
    st->dargs_bytes = st->args_bytes + (size_t)G * (nimg + 1) * sizeof(int);
    st->host.resize(st->dargs_bytes);
    return st;
}

// Places the intermediates in `arena` and the argument table at `dargs`.
void place_batch(BatchState& st, void* arena, void* dargs) {
    st.arena = arena;
    st.dargs = dargs;
    st.bufs = st.offs;
    for (auto& m : st.bufs)
        for (auto& kv : m) kv.second.ptr = static_cast<char*>(arena) + reinterpret_cast<size_t>(kv.second.ptr);
}

// The argument table of this run on the host (st.host).
void fill_table(const Plan& plan, BatchState& st, std::vector<std::map<int, ImgRef>>& mem) {
    const Pipeline& p = plan.p;
    const int nimg = (int)st.sizes.size(), G = (int)plan.groups.size();
    for (int i = 0; i < nimg; ++i)
        for (auto& kv : st.bufs[i]) mem[i][kv.first] = {kv.second.ptr, kv.second.rs, kv.second.cs};
    std::memset(st.host.data(), 0, st.host.size());
    for (int g = 0; g < G; ++g) {
        const GroupRt& gr = plan.groups[g];
        int* starts = reinterpret_cast<int*>(st.host.data() + st.args_bytes) + (size_t)g * (nimg + 1);
        int acc = 0;
        for (int i = 0; i < nimg; ++i) {
            WtArgsHost& a = reinterpret_cast<WtArgsHost*>(st.host.data())[(size_t)g * nimg + i];
            auto d = level_dims(st.sizes[i].first, st.sizes[i].second, p.nodes[gr.g.nodes[0]].level);
            fill_args(plan, gr, mem[i], a, "batch image " + std::to_string(i));
            check_store_planes(plan, gr, a, d.second);
            a.W = d.first;
            a.H = d.second;
            if (gr.resample) {
                auto sd = level_dims(st.sizes[i].first, st.sizes[i].second,
                                     p.nodes[p.nodes[gr.g.nodes[0]].srcs[0]].level);
                a.Ws = sd.first;
                a.Hs = sd.second;
            }
            const auto& t = st.tiles[(size_t)g * nimg + i];
            a.tiles_x = t[0];
            a.tiles_y = t[1];
            a.nwaves = t[2];
            starts[i] = acc;
            acc += t[2];
        }
        starts[nimg] = acc;
    }
}

}  // namespace

void load_batch_kernels(const Plan& plan_c, std::vector<GroupRt>& groups) {
    std::vector<GroupRt*> need;
    for (auto& gr : groups)
        if (!gr.fn_batch) need.push_back(&gr);
    if (!need.empty()) compile_groups(plan_c, need, true);
}

void run_plan_batch(Plan& plan, int nimg, const wt_image* in, const wt_image* out, void* stream, int first,
                    int count) {
    if (plan.no_device) fail(WT_E_INVALID, "plan was created with WT_PLAN_NO_DEVICE");
    const int G = (int)plan.groups.size();
    const bool all = count < 0;
    if (all) {
        first = 0;
        count = G;
    }
    if (first < 0 || count < 1 || first > G - count) fail(WT_E_INVALID, "group range outside the plan");
    std::vector<std::pair<int, int>> sizes;
    std::vector<std::map<int, ImgRef>> mem;
    check_batch(plan, nimg, in, out, sizes, mem);

    const bool whole = plan.batch_whole;
    // The whole-pipeline launch is generated, compiled and checked on the
    // host (the lane emulator runs it bit-identical to the per-group
    // launches), but its first device run did not finish within three
    // minutes and the cause has not been found; until it is, device runs
    // are refused here, before any allocation or launch.
    if (whole && all)
        fail(WT_E_UNSUPPORTED, "the whole-pipeline batch launch (WT_PLAN_BATCH_WHOLE) is switched off on the "
                               "device: its first run did not complete and the cause is not yet known");
    if (!plan.batch || plan.batch->sizes != sizes) {
        plan.batch.reset();
        load_batch_kernels(plan, plan.groups);  // compiled on first use
        if (whole) load_whole_kernel(plan);
        auto st = layout_batch(plan, sizes);
        if (whole) layout_whole(plan, *st);
        void* arena = nullptr;
        void* dargs = nullptr;
        if (st->arena_bytes && hipMalloc(&arena, st->arena_bytes) != hipSuccess)
            fail(WT_E_NOMEM, "batch intermediates");
        st->arena = arena;  // owned from here on
        if (hipMalloc(&dargs, st->dargs_bytes) != hipSuccess) fail(WT_E_NOMEM, "batch argument table");
        place_batch(*st, arena, dargs);
        // capture the launch sequence once for this shape
        hipStream_t cs;
        hip_check(hipStreamCreate(&cs), "hipStreamCreate");
        hip_check(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        for (int g = 0; g < (whole ? 1 : G); ++g) {
            hipError_t e = whole ? launch_whole(plan, *st, nimg, cs) : launch_batch_group(plan, *st, g, nimg, cs);
            if (e != hipSuccess) {
                hipGraph_t tmp;
                hipStreamEndCapture(cs, &tmp);
                if (tmp) hipGraphDestroy(tmp);
                hipStreamDestroy(cs);
                hip_check(e, "hipModuleLaunchKernel (capture)");
            }
        }
        hip_check(hipStreamEndCapture(cs, &st->graph), "hipStreamEndCapture");
        hipStreamDestroy(cs);
        hip_check(hipGraphInstantiate(&st->exec, st->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
        plan.batch = std::move(st);
    }

    BatchState& st = *plan.batch;
    fill_table(plan, st, mem);
    if (st.ctr_words) fill_whole(st);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // the table changes only when the caller's image pointers or strides do
    if (st.uploaded != st.host) {
        hip_check(hipMemcpyAsync(st.dargs, st.host.data(), st.host.size(), hipMemcpyHostToDevice, s), "hipMemcpyAsync");
        st.uploaded = st.host;
    }
    if (all) {
        hip_check(hipGraphLaunch(st.exec, s), "hipGraphLaunch");
        st.whole_ran = st.ctr_words > 0;
        return;
    }
    for (int g = first; g < first + count; ++g)
        hip_check(launch_batch_group(plan, st, g, nimg, s), "hipModuleLaunchKernel");
}

void check_batch_status(Plan& plan, void* stream) {
    // the status word is written only by a whole-pipeline launch (a batch
    // state made by a run of some groups holds it uncleared)
    if (!plan.batch || !plan.batch->whole_ran) return;
    const BatchState& st = *plan.batch;
    hip_check(hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)), "hipStreamSynchronize");
    int status = 0;
    const char* at = static_cast<const char*>(st.dargs) + st.ctr_off + (size_t)(st.ctr_words - 1) * 4;
    hip_check(hipMemcpy(&status, at, sizeof status, hipMemcpyDeviceToHost), "hipMemcpy");
    if (status) fail(WT_E_INTERNAL, "a wave of the whole-pipeline launch gave up waiting for a producer group");
}

void run_plan_batch_static(Plan& plan, int nimg, const wt_image* in, const wt_image* out, void* stream) {
    if (plan.no_device) fail(WT_E_INVALID, "plan was created with WT_PLAN_NO_DEVICE");
    for (const auto& gr : plan.groups)
        if (!gr.fn_batch)
            fail(WT_E_INVALID, "the plan's batched kernels are not loaded (create the plan with batch_images > 1, "
                               "or run wt_plan_run_batch once)");
    int dev = -1;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (dev != plan.device) fail(WT_E_INVALID, "the current device is not the plan's");
    std::vector<std::pair<int, int>> sizes;
    std::vector<std::map<int, ImgRef>> mem;
    check_batch(plan, nimg, in, out, sizes, mem);
    if (!plan.batch_static || plan.batch_static->sizes != sizes) {
        plan.batch_static = layout_batch(plan, sizes);
        plan.batch_static->owned = false;  // the workspace is the library's
    }
    BatchState& st = *plan.batch_static;
    const size_t arena = (st.arena_bytes + 255) / 256 * 256;
    const size_t need = arena + st.dargs_bytes;
    if (need > (size_t)WT_STATIC_SCRATCH_BYTES)
        fail(WT_E_NOMEM, "batch needs " + std::to_string(need) + " bytes of workspace (intermediates and argument "
                         "table); the fixed workspace holds " + std::to_string((size_t)WT_STATIC_SCRATCH_BYTES));
    hipError_t e = hipSuccess;
    char* base = static_cast<char*>(static_scratch(dev, &e));
    hip_check(e, "hipGetSymbolAddress (fixed workspace)");
    place_batch(st, base, base + arena);
    fill_table(plan, st, mem);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // every call rewrites the table: the workspace is shared by all plans
    hip_check(hipMemcpyAsync(st.dargs, st.host.data(), st.host.size(), hipMemcpyHostToDevice, s), "hipMemcpyAsync");
    for (int g = 0; g < (int)plan.groups.size(); ++g)
        hip_check(launch_batch_group(plan, st, g, nimg, s), "hipModuleLaunchKernel");
}

}  // namespace wt

namespace wt {

// Tuning on the batch itself.  A plan made for batches is tuned on a proxy
// (one tall image of the planning size), which ranks some configurations
// differently from the uneven images of the real batch.  Here every group's
// configuration and its neighbours (config_neighbours) are timed as batched
// kernels over the caller's images, reading the intermediates the previous
// groups left in the batch's arena, for up to four rounds per group while a
// round still helps; the fastest is kept, and the result is cached per
// starting schedule and image sizes.  Changing one group's configuration leaves its inputs
// and outputs, hence the arena's layout, unchanged.
void tune_plan_batch(Plan& plan, int nimg, const wt_image* in, const wt_image* out, void* stream) {
    if (plan.no_device) fail(WT_E_INVALID, "plan was created with WT_PLAN_NO_DEVICE");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    run_plan_batch(plan, nimg, in, out, stream);  // validates; every intermediate filled
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    std::vector<std::pair<int, int>> sizes;
    std::vector<std::map<int, ImgRef>> mem;
    check_batch(plan, nimg, in, out, sizes, mem);
    const BatchState& bs = *plan.batch;
    for (int i = 0; i < nimg; ++i)
        for (auto& kv : bs.bufs[i]) mem[i][kv.first] = {kv.second.ptr, kv.second.rs, kv.second.cs};
    const Pipeline& p = plan.p;
    // a batch tuned before (same device, starting schedule and image sizes)
    // takes the schedule found then
    std::string key;
    {
        hipDeviceProp_t prop;
        hip_check(hipGetDeviceProperties(&prop, plan.device), "hipGetDeviceProperties");
        uint64_t h = 1469598103934665603ull;
        auto mix = [&](const std::string& t) {
            for (unsigned char c : t) h = (h ^ c) * 1099511628211ull;
        };
        mix(schedule_text(plan.sched));
        for (auto& sz : sizes) mix(std::to_string(sz.first) + "x" + std::to_string(sz.second) + ",");
        char hb[32];
        std::snprintf(hb, sizeof hb, "%016llx", (unsigned long long)h);
        key = std::string("batch|") + prop.gcnArchName + "|" + hb;
    }
    std::string cached;
    if (tune_cache_lookup(plan.cache_dir, key, cached)) {
        if (cached == schedule_text(plan.sched)) return;
        plan.sched = parse_schedule(cached, p);
        build_groups(plan);
        load_batch_kernels(plan, plan.groups);
        run_plan_batch(plan, nimg, in, out, stream);
        return;
    }
    const size_t tbytes = (size_t)nimg * sizeof(WtArgsHost) + (size_t)(nimg + 1) * sizeof(int);
    void* dtab = nullptr;
    if (hipMalloc(&dtab, tbytes) != hipSuccess) fail(WT_E_NOMEM, "batch tuning table");
    struct Free {
        void* p;
        ~Free() { hipFree(p); }
    } free_tab{dtab};
    std::vector<char> host(tbytes);
    OwnedEvents ev;

    // time of one batched launch of candidate `gr` (group gi), microseconds
    auto time_candidate = [&](GroupRt& gr) -> double {
        std::memset(host.data(), 0, host.size());
        int* starts = reinterpret_cast<int*>(host.data() + (size_t)nimg * sizeof(WtArgsHost));
        int acc = 0;
        for (int i = 0; i < nimg; ++i) {
            WtArgsHost& a = reinterpret_cast<WtArgsHost*>(host.data())[i];
            auto d = level_dims(sizes[i].first, sizes[i].second, p.nodes[gr.g.nodes[0]].level);
            fill_args(plan, gr, mem[i], a, "batch image " + std::to_string(i));
            check_store_planes(plan, gr, a, d.second);
            a.W = d.first;
            a.H = d.second;
            int tx, ty, w;
            tile_counts(plan, gr, d.first, d.second, tx, ty, w);
            a.tiles_x = tx;
            a.tiles_y = ty;
            a.nwaves = w;
            starts[i] = acc;
            acc += w;
        }
        starts[nimg] = acc;
        hip_check(hipMemcpyAsync(dtab, host.data(), tbytes, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
        const void* a = dtab;
        const void* sp = static_cast<char*>(dtab) + (size_t)nimg * sizeof(WtArgsHost);
        int ni = nimg, tot = acc;
        void* params[] = {&a, &sp, &ni, &tot};
        const int units = (tot + gr.g.WPB - 1) / gr.g.WPB;
        const int grid = std::max(1, std::min(units, 1 << 22));
        auto launch = [&] {
            for (size_t i = 0; i < gr.liveouts.size(); ++i) {  // as launch_batch_group does
                const Node& hn = p.nodes[gr.liveouts[i]];
                if (hn.kind == Kind::Hist)
                    hip_check(zero_hist_batch(a, nimg, (int)i, hn.bins, hn.channels, st), "zero_hist_batch");
            }
            hip_check(hipModuleLaunchKernel(gr.fn_batch, grid, 1, 1, 64 * gr.g.WPB, 1, 1, 0, st, params, nullptr),
                      "hipModuleLaunchKernel");
        };
        launch();
        double best = INFINITY;
        for (int s = 0; s < 3; ++s) {
            hip_check(hipEventRecord(ev.e0, st), "hipEventRecord");
            for (int r = 0; r < 3; ++r) launch();
            hip_check(hipEventRecord(ev.e1, st), "hipEventRecord");
            hip_check(hipEventSynchronize(ev.e1), "hipEventSynchronize");
            float ms = 0;
            hip_check(hipEventElapsedTime(&ms, ev.e0, ev.e1), "hipEventElapsedTime");
            best = std::min(best, (double)ms * 1e3 / 3);
        }
        return best;
    };

    bool changed = false;
    for (size_t gi = 0; gi < plan.groups.size(); ++gi) {
        if (plan.groups[gi].resample || plan.groups[gi].g.BLK) continue;
        GroupSched best = plan.sched.groups[gi];
        double best_t = time_candidate(plan.groups[gi]);
        const double start_t = best_t;
        std::set<std::string> seen{describe_group(best)};
        const int vmax = max_vector_width(p, best, plan.W, plan.H, plan.any_width);
        for (int round = 0; round < 4; ++round) {
            std::vector<GroupRt> cands;
            for (const GroupSched& g : config_neighbours(best, vmax)) {
                if (!seen.insert(describe_group(g)).second) continue;
                GroupRt gr;
                gr.g = g;
                try {
                    prepare_group(plan, gr, (int)gi);
                } catch (const Error&) {
                    continue;
                }
                cands.push_back(std::move(gr));
            }
            std::vector<GroupRt*> ptrs;
            for (auto& c : cands) ptrs.push_back(&c);
            std::vector<bool> bad;
            compile_groups(plan, ptrs, true, &bad);
            bool improved = false;
            for (size_t c = 0; c < cands.size(); ++c) {
                if (bad[c]) continue;
                double t = INFINITY;
                try {
                    t = time_candidate(cands[c]);
                } catch (const Error&) {
                }
                if (t < best_t) {
                    best_t = t;
                    best = cands[c].g;
                    improved = true;
                }
            }
            for (auto& c : cands) unload_group(c);
            if (!improved) break;
        }
        if (verbose())
            std::fprintf(stderr, "wavetile batch tuning: group %zu of %zu, %.1f us (was %.1f): %s\n", gi + 1,
                         plan.groups.size(), best_t, start_t, describe_group(best).c_str());
        if (describe_group(best) != describe_group(plan.sched.groups[gi])) {
            plan.sched.groups[gi] = best;
            changed = true;
        }
    }
    tune_cache_store(plan.cache_dir, key, schedule_text(plan.sched));
    if (changed) {
        build_groups(plan);  // resets the batch state and its graph
        load_batch_kernels(plan, plan.groups);
    }
    // the candidates wrote the groups' outputs: the plan's own run rewrites them
    run_plan_batch(plan, nimg, in, out, stream);
}

}  // namespace wt
