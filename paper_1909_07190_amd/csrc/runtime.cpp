// Plans and their execution: schedule -> generated kernels -> launches.
// The host side of the paper's compilation pipeline (Fig. 6: fusion, OTPW,
// hybrid tiling, code generation) plus the run-time launch of one kernel per
// fused group in topological order (Section 7's execution protocol).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <set>
#include <sstream>
#include <thread>

#include "wt_internal.h"
#include "wt_runtime.h"

namespace wt {

void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) fail(WT_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

std::pair<int, int> level_dims(int W, int H, int level) {
    for (int i = 0; i < level; ++i) {
        W = (W + 1) / 2;
        H = (H + 1) / 2;
    }
    return {W, H};
}

// A histogram is of use as an output or as the table of equalize stages.
static bool hist_is_read(const Pipeline& p, int h) {
    if (p.is_output(h)) return true;
    for (const Node& n : p.nodes)
        if (n.kind == Kind::Equalize && n.srcs[1] == h) return true;
    return false;
}

std::pair<int, int> node_dims(const Pipeline& p, int id, int W, int H) {
    const Node& n = p.nodes[id];
    if (n.kind == Kind::Hist) return {n.bins, 1};
    return level_dims(W, H, n.level);
}

namespace {

int64_t round_up64(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Content-addressed kernel names: the hash of the generated text (written
// with a placeholder name), so two kernels share a name only if their code
// is identical, and any change to the generator renames the kernel (profile
// figures keyed by name then no longer apply to it).
const char* const kNamePlaceholder = "wt_kernel_name_placeholder";

std::string kernel_name(const GroupSources& gs, const GroupSched& g, int gi) {
    uint64_t h = 1469598103934665603ull;
    for (const std::string* part : {&gs.prelude, &gs.common, &gs.single, &gs.batch})
        for (unsigned char c : *part) h = (h ^ c) * 1099511628211ull;
    char buf[64];
    std::snprintf(buf, sizeof buf, "wt_g%d_%s_%012llx", gi, g.nodes.size() > 1 ? "fused" : "stage",
                  (unsigned long long)(h & 0xffffffffffffull));
    return buf;
}

void name_sources(GroupRt& gr, GroupSources gs, int gi) {
    gr.kname = kernel_name(gs, gr.g, gi);
    for (std::string* part : {&gs.common, &gs.single, &gs.batch}) {
        std::string& t = *part;
        const std::string ph = kNamePlaceholder;
        for (size_t pos = 0; (pos = t.find(ph, pos)) != std::string::npos; pos += gr.kname.size())
            t.replace(pos, ph.size(), gr.kname);
    }
    gr.src = gs.full();
    gr.src_single = gs.single_module();
    gr.src_batch = gs.batch_module();
}

}  // namespace

Plan::~Plan() {
    batch.reset();
    unload_whole(*this);
    for (auto& g : groups) unload_group(g);
    for (auto& b : bufs)
        if (b.second.ptr) hipFree(b.second.ptr);
}

namespace {

// ---------------------------------------------------- autotune schedule cache
std::mutex g_tune_mu;
std::map<std::string, std::string> g_tune;  // key -> schedule text
std::set<std::string> g_tune_dirs;          // cache directories already read

uint64_t fnv1a64(const std::string& s) {
    uint64_t h = 1469598103934665603ull;
    for (unsigned char c : s) {
        h ^= c;
        h *= 1099511628211ull;
    }
    return h;
}

// Everything that defines what a pipeline computes, in node order.
std::string pipeline_signature(const Pipeline& p) {
    std::ostringstream os;
    os.precision(17);
    for (const Node& n : p.nodes) {
        os << (int)n.kind << ':' << n.channels << ':' << n.level << ':' << n.dtype << ':';
        for (int s : n.srcs) os << s << ',';
        os << ':' << n.kw << 'x' << n.kh << '@' << n.ax << ',' << n.ay << ':' << n.scale << ':' << n.divisor << ':'
           << n.expr_text << ':';
        for (double w : n.weights) os << w << ',';
        for (long long w : n.iweights) os << w << ',';
        os << ';';
    }
    os << "out:";
    for (int o : p.outputs) os << o << ',';
    return os.str();
}

std::string tune_file(const std::string& dir) { return dir + "/autotune.tsv"; }

}  // namespace

std::string schedule_text(const Schedule& s) {
    std::string t;
    for (size_t i = 0; i < s.groups.size(); ++i) t += (i ? ";" : "") + describe_group(s.groups[i]);
    return t;
}

std::string tune_key(const Plan& plan, const wt_sched_opts& opts) {
    hipDeviceProp_t prop;
    hip_check(hipGetDeviceProperties(&prop, plan.device), "hipGetDeviceProperties");
    std::ostringstream os;
    os << prop.gcnArchName << '|' << (plan.W + 255) / 256 << 'x' << (plan.H + 255) / 256 << 'm' << (plan.W & 3) << '|'
       << (plan.fp16 ? 1 : 0) << (plan.any_width ? 1 : 0) << 'b' << std::max(1, opts.batch_images) << '|'
       << opts.autotune_topk << '|'
       << (opts.model_path ? opts.model_path : "") << '|' << std::hex << fnv1a64(pipeline_signature(plan.p));
    std::string k = os.str();
    for (char& c : k)
        if (c == '\t' || c == '\n' || c == '\r') c = ' ';
    return k;
}

bool tune_cache_lookup(const std::string& dir, const std::string& key, std::string& text) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!dir.empty() && !g_tune_dirs.count(dir)) {
        g_tune_dirs.insert(dir);
        std::ifstream f(tune_file(dir));
        std::string line;
        while (std::getline(f, line)) {
            size_t tab = line.find('\t');
            if (tab != std::string::npos && tab + 1 < line.size()) g_tune[line.substr(0, tab)] = line.substr(tab + 1);
        }
    }
    auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    text = it->second;
    return true;
}

void tune_cache_store(const std::string& dir, const std::string& key, const std::string& text) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = text;
    if (dir.empty()) return;
    std::ofstream f(tune_file(dir), std::ios::app);
    if (f) f << key << '\t' << text << '\n';
}

// WT_VERBOSE set (and not "0"): planning reports its measured steps on stderr.
bool verbose() {
    static const bool v = [] {
        const char* e = std::getenv("WT_VERBOSE");
        return e && *e && std::string(e) != "0";
    }();
    return v;
}

namespace {

// Whether two schedules fuse the same stages the same way (configurations
// aside).
bool same_grouping(const Schedule& a, const Schedule& b) {
    auto key = [](const Schedule& s) {
        std::vector<std::string> k;
        for (const GroupSched& g : s.groups) {
            std::ostringstream os;
            for (int n : g.nodes) os << n << ',';
            os << '|';
            for (int n : g.dec) os << n << ',';
            os << '|';
            for (int n : g.exp) os << n << ',';
            os << '|';
            for (int n : g.hst) os << n << ',';
            k.push_back(os.str());
        }
        std::sort(k.begin(), k.end());
        return k;
    };
    return key(a) == key(b);
}

// The planning settings of `from` (pipeline, size, device, options).
void copy_settings(const Plan& from, Plan& to) {
    to.p = from.p;
    to.W = from.W;
    to.H = from.H;
    to.device = from.device;
    to.no_device = from.no_device;
    to.no_compile = from.no_compile;
    to.fp16 = from.fp16;
    to.any_width = from.any_width;
    to.batch_resident = from.batch_resident;
    to.batch_whole = from.batch_whole;
    to.setup_stream = from.setup_stream;
    to.cache_dir = from.cache_dir;
    to.machine = from.machine;
}

}  // namespace

std::unique_ptr<Plan> create_plan(const Pipeline& p, const wt_sched_opts* o, int W, int H, void* stream) {
    if (W <= 0 || H <= 0) fail(WT_E_SHAPE, "plan size must be positive");
    if (W > (1 << 24) || H > (1 << 24)) fail(WT_E_SHAPE, "plan size too large");
    if (p.outputs.empty()) fail(WT_E_INVALID, "pipeline has no outputs");
    auto plan = std::make_unique<Plan>();
    plan->p = p;
    plan->W = W;
    plan->H = H;
    wt_sched_opts def{};
    def.mode = WT_SCHED_ANALYTIC;
    const wt_sched_opts& opts = o ? *o : def;
    plan->no_device = (opts.flags & (WT_PLAN_NO_DEVICE | WT_PLAN_NO_COMPILE)) != 0;
    plan->no_compile = (opts.flags & WT_PLAN_NO_COMPILE) != 0;
    plan->fp16 = opts.fp16_intermediates != 0;
    plan->any_width = (opts.flags & WT_PLAN_ANY_WIDTH) != 0;
    plan->batch_resident = (opts.flags & WT_PLAN_BATCH_RESIDENT) != 0;
    plan->batch_whole = (opts.flags & WT_PLAN_BATCH_WHOLE) != 0;
    plan->setup_stream = reinterpret_cast<hipStream_t>(stream);
    const char* env_cache = std::getenv("WT_CACHE_DIR");
    plan->cache_dir = opts.cache_dir ? opts.cache_dir : (env_cache ? env_cache : "");
    if (!plan->no_device) hip_check(hipGetDevice(&plan->device), "hipGetDevice");
    plan->machine = plan->no_device ? Machine{} : machine_from_device(plan->device);

    SchedRequest req;
    req.mode = opts.mode;
    req.fp16 = plan->fp16;
    req.W = W;
    req.H = H;
    req.any_width = plan->any_width;
    req.batch = std::max(1, opts.batch_images);
    req.fold = (opts.flags & WT_PLAN_NO_FOLD) == 0;
    if (opts.fixed_schedule) req.fixed = opts.fixed_schedule;
    if (opts.model_path) req.model_path = opts.model_path;
    const bool tune = opts.mode == WT_SCHED_AUTOTUNE && !plan->no_device;
    std::string key;
    if (tune) {
        key = tune_key(*plan, opts);
        std::string text;
        if (!(opts.flags & WT_PLAN_RETUNE) && tune_cache_lookup(plan->cache_dir, key, text)) {
            req.mode = WT_SCHED_FIXED;
            req.fixed = text;
            plan->sched = make_schedule(p, plan->machine, req);
            build_groups(*plan);
            if (opts.batch_images > 1) load_batch_kernels(*plan, plan->groups);
            return plan;
        }
    }
    if (!plan->no_device && preprofile_enabled() &&
        (opts.mode == WT_SCHED_ANALYTIC || opts.mode == WT_SCHED_MLP || opts.mode == WT_SCHED_AUTOTUNE))
        preprofile(*plan);
    plan->sched = make_schedule(p, plan->machine, req);
    build_groups(*plan);
    if (tune) {
        const int topk = opts.autotune_topk > 0 ? opts.autotune_topk : 4;
        const std::string model = opts.model_path ? opts.model_path : "";
        TuneMemo memo;
        double t = autotune_plan(*plan, topk, model, req.batch, &memo);
        // Other groupings the search proposes are measured too, and the
        // fastest tuned plan is kept: the same search with up2 stages only
        // expanded (never folded into the group of the stage they
        // resample), and the analytical model's search for one image of
        // this size (the cost models rank folded groups differently; a
        // group tuned for one grouping is reused by the others).
        std::vector<SchedRequest> alts;
        SchedRequest nofold = req;
        nofold.fold = false;
        if (req.fold) alts.push_back(nofold);
        SchedRequest one = req;
        one.mode = WT_SCHED_ANALYTIC;
        one.model_path.clear();
        one.batch = 1;
        alts.push_back(one);
        std::vector<Schedule> seen = {plan->sched};
        for (const SchedRequest& ar : alts) {
            Schedule alt_sched = make_schedule(p, plan->machine, ar);
            bool dup = false;
            for (const Schedule& sc : seen) dup = dup || same_grouping(sc, alt_sched);
            if (dup) continue;
            seen.push_back(alt_sched);
            auto alt = std::make_unique<Plan>();
            copy_settings(*plan, *alt);
            alt->sched = alt_sched;
            build_groups(*alt);
            double t_alt = autotune_plan(*alt, topk, model, req.batch, &memo);
            if (verbose())
                std::fprintf(stderr, "wavetile autotune: another grouping (%s%s): %.1f us per image, against %.1f\n",
                             ar.mode == WT_SCHED_ANALYTIC && ar.batch == 1 ? "analytical, one image" : "search",
                             ar.fold ? "" : ", no folded up2s", t_alt, t);
            if (t_alt < t) {
                plan = std::move(alt);
                t = t_alt;
            }
        }
        tune_cache_store(plan->cache_dir, key, schedule_text(plan->sched));
    }
    // a plan made for batches loads its batched kernels now, so batched runs
    // (wt_plan_run_batch_static in particular) need no compilation
    if (!plan->no_device && opts.batch_images > 1) load_batch_kernels(*plan, plan->groups);
    return plan;
}

// Geometry, memory dtypes and generated source of group `gi` of a plan.
void prepare_group(const Plan& plan, GroupRt& gr, int gi) {
    const Pipeline& p = plan.p;
    gr.resample = is_resample_group(p, gr.g) || is_hist_group(p, gr.g);
    int lvl = p.nodes[gr.g.nodes[0]].level;
    auto d = level_dims(plan.W, plan.H, lvl);
    gr.W = d.first;
    gr.H = d.second;
    auto half_mem = [&](int id) {
        return plan.fp16 && p.half_storable(id) && !p.is_output(id);
    };
    gr.mem_half_in.clear();
    gr.mem_half_out.clear();
    if (gr.resample) {
        const Node& n = p.nodes[gr.g.nodes[0]];
        auto sd = level_dims(plan.W, plan.H, p.nodes[n.srcs[0]].level);
        gr.Ws = sd.first;
        gr.Hs = sd.second;
        gr.loaded = {n.srcs[0]};
        gr.liveouts = {n.id};
        if (n.kind == Kind::Hist) {
            if (!hist_is_read(p, n.id))
                fail(WT_E_INVALID, "histogram node " + std::to_string(n.id) + " is not an output and no stage reads it");
            name_sources(gr, generate_hist_source(p, gr.g, kNamePlaceholder, half_mem(n.srcs[0])), gi);
        } else {
            name_sources(gr, generate_resample_source(p, gr.g, kNamePlaceholder, half_mem(n.srcs[0]), half_mem(n.id)),
                         gi);
        }
        gr.mem_half_in = {half_mem(n.srcs[0])};
        gr.mem_half_out = {half_mem(n.id)};
        int bw, bh;
        resample_block(p, gr.g, bw, bh);
        gr.tiles_x = (gr.W + bw - 1) / bw;
        gr.tiles_y = (gr.H + bh - 1) / bh;
        gr.nwaves = gr.tiles_x * gr.tiles_y * n.channels;
        return;
    }
    gr.geo = group_geometry(p, gr.g);
    // an expanded up2 is read from its coarse source's buffer
    auto buffer_of = [&](int id) {
        const NodeGeom& ng = gr.geo.nodes[gr.geo.index.at(id)];
        return ng.expand_src >= 0 ? ng.expand_src : id;
    };
    for (auto& ng : gr.geo.nodes)
        ng.mem_half = (!ng.member || ng.liveout) && half_mem(ng.member ? ng.id : buffer_of(ng.id));
    for (int l : gr.geo.loaded) gr.mem_half_in.push_back(half_mem(buffer_of(l)));
    for (int l : gr.geo.liveouts) gr.mem_half_out.push_back(half_mem(l));
    gr.loaded.clear();
    for (int l : gr.geo.loaded) gr.loaded.push_back(buffer_of(l));
    for (int t : gr.geo.tables) {  // histograms read whole follow the loaded rows
        gr.loaded.push_back(t);
        gr.mem_half_in.push_back(false);
    }
    gr.liveouts = gr.geo.liveouts;
    for (auto& ds : gr.geo.dec) {  // decimated outputs follow the live-outs
        gr.liveouts.push_back(ds.first);
        gr.mem_half_out.push_back(half_mem(ds.first));
    }
    for (auto& hs : gr.geo.hist) {  // then accumulated histograms
        if (!hist_is_read(p, hs.first))
            fail(WT_E_INVALID, "histogram node " + std::to_string(hs.first) + " is not an output and no stage reads it");
        gr.liveouts.push_back(hs.first);
        gr.mem_half_out.push_back(false);
    }
    name_sources(gr, generate_group_source(p, gr.g, gr.geo, kNamePlaceholder), gi);
    int amin = 1 << 30, amax = 0;
    for (int lo : gr.geo.outs) {
        const NodeGeom& ng = gr.geo.nodes[gr.geo.index.at(lo)];
        amin = std::min(amin, ng.skew);
        amax = std::max(amax, ng.skew);
    }
    int start_min = amin - amax;  // leftmost stored x of tile 0
    int ch = gr.geo.chan_parallel ? gr.geo.C : 1;
    if (gr.g.BLK) {  // one tile per workgroup: nwaves counts every wave of every tile
        int bw = block_tile_w(gr.g);
        gr.tiles_x = (gr.W + bw - 1) / bw;
        gr.tiles_y = (gr.H + gr.g.TY - 1) / gr.g.TY;
        gr.nwaves = gr.tiles_x * gr.tiles_y * ch * gr.g.WPB;
        return;
    }
    gr.tiles_x = (gr.W - start_min + gr.geo.X - 1) / gr.geo.X;
    gr.tiles_y = (gr.H + gr.g.TY - 1) / gr.g.TY;
    gr.nwaves = gr.tiles_x * gr.tiles_y * ch;
    if (gr.geo.lds_bytes_per_wg > plan.machine.max_lds_per_wg)
        fail(WT_E_UNSUPPORTED, "group needs " + std::to_string(gr.geo.lds_bytes_per_wg) + " bytes of LDS per workgroup");
}

void unload_whole(Plan& plan) {
    if (plan.whole_mod) hipModuleUnload(plan.whole_mod);
    plan.whole_mod = nullptr;
    plan.whole_fn = nullptr;
    plan.whole_src.clear();
    plan.whole_kname.clear();
}

void unload_group(GroupRt& gr) {
    if (gr.mod) hipModuleUnload(gr.mod);
    if (gr.mod_batch) hipModuleUnload(gr.mod_batch);
    gr.mod = gr.mod_batch = nullptr;
    gr.fn = gr.fn_batch = nullptr;
}

// Compiles the groups' single-image modules (or, with `batch`, their batched
// modules) in parallel on host cores (hipRTC), then loads the code objects
// unless the plan has no device.
void compile_groups(const Plan& plan, std::vector<GroupRt*>& grs, bool batch, std::vector<bool>* failed) {
    std::vector<std::vector<char>> code(grs.size());
    std::vector<std::string> errs(grs.size());
    std::atomic<size_t> next{0};
    int nthr = std::max(1, std::min<int>((int)grs.size(), (int)std::thread::hardware_concurrency()));
    nthr = std::min(nthr, 16);
    std::vector<std::thread> pool;
    for (int t = 0; t < nthr; ++t)
        pool.emplace_back([&] {
            for (size_t i; (i = next++) < grs.size();) {
                try {
                    code[i] = compile_hip(batch ? grs[i]->src_batch : grs[i]->src_single,
                                          grs[i]->kname + (batch ? "_batch" : ""), plan.cache_dir);
                } catch (const std::exception& e) {
                    errs[i] = e.what();
                }
            }
        });
    for (auto& t : pool) t.join();
    if (failed) failed->assign(grs.size(), false);
    for (size_t i = 0; i < errs.size(); ++i)
        if (!errs[i].empty()) {
            if (!failed) fail(WT_E_COMPILE, errs[i]);
            (*failed)[i] = true;
        }
    if (plan.no_device) return;
    for (size_t i = 0; i < grs.size(); ++i) {
        if (failed && (*failed)[i]) continue;
        GroupRt& g = *grs[i];
        if (batch) {
            if (g.mod_batch) continue;
            hip_check(hipModuleLoadData(&g.mod_batch, code[i].data()), "hipModuleLoadData");
            hip_check(hipModuleGetFunction(&g.fn_batch, g.mod_batch, (g.kname + "_batch").c_str()),
                      "hipModuleGetFunction");
        } else {
            if (g.mod) continue;
            hip_check(hipModuleLoadData(&g.mod, code[i].data()), "hipModuleLoadData");
            hip_check(hipModuleGetFunction(&g.fn, g.mod, g.kname.c_str()), "hipModuleGetFunction");
        }
    }
}

// Geometry, code generation, compilation and module loading for every group
// of plan.sched, then device buffers for the intermediates.
void build_groups(Plan& plan) {
    const Pipeline& p = plan.p;
    plan.batch.reset();
    plan.batch_static.reset();  // its tile counts and grids follow the groups
    unload_whole(plan);
    for (auto& g : plan.groups) unload_group(g);
    plan.groups.clear();
    std::vector<bool> in_memory(p.nodes.size(), false);
    for (int i : p.inputs) in_memory[i] = true;
    for (size_t gi = 0; gi < plan.sched.groups.size(); ++gi) {
        GroupRt gr;
        gr.g = plan.sched.groups[gi];
        prepare_group(plan, gr, (int)gi);
        for (int l : gr.loaded)
            if (!in_memory[l]) fail(WT_E_INVALID, "schedule order: node " + std::to_string(l) + " used before produced");
        for (int l : gr.liveouts) in_memory[l] = true;
        plan.groups.push_back(std::move(gr));
    }
    for (int o : p.outputs)
        if (!in_memory[o]) fail(WT_E_INVALID, "schedule does not produce output node " + std::to_string(o));
    std::vector<GroupRt*> grs;
    for (auto& g : plan.groups) grs.push_back(&g);
    if (!plan.no_compile) compile_groups(plan, grs);
    if (plan.no_device) return;
    // device buffers for intermediates materialised between groups
    for (auto& gr : plan.groups) {
        for (size_t i = 0; i < gr.liveouts.size(); ++i) {
            int id = gr.liveouts[i];
            if (p.is_output(id) || plan.bufs.count(id)) continue;
            auto d = node_dims(p, id, plan.W, plan.H);
            Buf b;
            b.half = gr.mem_half_out[i];
            b.rs = round_up64(d.first, 64);
            b.cs = b.rs * d.second;
            size_t bytes = (size_t)b.cs * p.nodes[id].channels * node_esize(p, id, b.half);
            hipError_t e = hipMalloc(&b.ptr, std::max<size_t>(bytes, 256));
            if (e != hipSuccess) fail(WT_E_NOMEM, "hipMalloc of an intermediate buffer failed");
            plan.bufs[id] = b;
        }
    }
}

ImgRef check_image(const wt_image& im, const Node& n, int W, int H, const std::string& tag) {
    if (!im.data) fail(WT_E_INVALID, tag + ": null data");
    if (im.width != W || im.height != H)
        fail(WT_E_SHAPE, tag + ": size " + std::to_string(im.width) + "x" + std::to_string(im.height) +
                             " differs from the planned " + std::to_string(W) + "x" + std::to_string(H));
    if (im.channels != n.channels)
        fail(WT_E_SHAPE, tag + ": " + std::to_string(im.channels) + " channels, expected " +
                             std::to_string(n.channels));
    if (im.dtype != n.dtype)
        fail(WT_E_SHAPE, tag + ": element type " + std::to_string(im.dtype) + ", the node's is " +
                             std::to_string(n.dtype));
    ImgRef r;
    r.ptr = im.data;
    r.rs = im.row_stride ? im.row_stride : im.width;
    r.cs = im.chan_stride ? im.chan_stride : r.rs * im.height;
    if (r.rs < im.width) fail(WT_E_SHAPE, tag + ": row stride smaller than the width");
    if (im.channels > 1 && r.cs < r.rs * im.height)
        fail(WT_E_SHAPE, tag + ": channel stride smaller than a plane");
    return r;
}

void check_store_planes(const Plan& plan, const GroupRt& gr, const WtArgsHost& a, int H) {
    // stores address a plane with 32-bit byte offsets (buffer stores)
    for (size_t i = 0; i < gr.liveouts.size(); ++i)
        if (plan.p.nodes[gr.liveouts[i]].kind != Kind::Hist &&
            (double)a.dst_rs[i] * H * node_esize(plan.p, gr.liveouts[i], gr.mem_half_out[i]) >= 2147483647.0)
            fail(WT_E_UNSUPPORTED, "an output plane of 2 GiB or more");
}

namespace {

// Caller images: 32-bit elements need only their own alignment (vector
// accesses of them are 4-byte aligned); narrower integer elements are
// accessed in aligned vectors of V elements.
void check_align(const ImgRef& r, int V, int esize, const std::string& tag) {
    if (reinterpret_cast<uintptr_t>(r.ptr) % esize)
        fail(WT_E_SHAPE, tag + ": buffer not aligned to its element size");
    if (V == 1 || esize >= 4) return;
    if ((reinterpret_cast<uintptr_t>(r.ptr) % (esize * V)) || (r.rs % V) || (r.cs % V))
        fail(WT_E_SHAPE, tag + ": buffer or strides not aligned to " + std::to_string(V) +
                             " elements as the plan's vector width requires");
}
}  // namespace

void run_plan(Plan& plan, const wt_image* in, int nin, const wt_image* out, int nout, void* stream) {
    if (plan.no_device) fail(WT_E_INVALID, "plan was created with WT_PLAN_NO_DEVICE");
    const Pipeline& p = plan.p;
    if (nin != (int)p.inputs.size()) fail(WT_E_INVALID, "expected " + std::to_string(p.inputs.size()) + " inputs");
    if (nout != (int)p.outputs.size())
        fail(WT_E_INVALID, "expected " + std::to_string(p.outputs.size()) + " outputs");
    if ((!in && nin) || (!out && nout)) fail(WT_E_INVALID, "null image array");
    std::map<int, ImgRef> mem;
    for (int i = 0; i < nin; ++i)
        mem[p.inputs[i]] = check_image(in[i], p.nodes[p.inputs[i]], plan.W, plan.H, "input " + std::to_string(i));
    for (int i = 0; i < nout; ++i) {
        int id = p.outputs[i];
        auto d = node_dims(p, id, plan.W, plan.H);
        ImgRef r = check_image(out[i], p.nodes[id], d.first, d.second, "output " + std::to_string(i));
        for (auto& kv : mem)
            if (kv.second.ptr == r.ptr) fail(WT_E_INVALID, "output " + std::to_string(i) + " aliases another image");
        mem[id] = r;
    }
    for (auto& kv : plan.bufs) mem[kv.first] = {kv.second.ptr, kv.second.rs, kv.second.cs};

    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    for (auto& gr : plan.groups) launch_group(plan, gr, mem, st);
}

void fill_args(const Plan& plan, const GroupRt& gr, const std::map<int, ImgRef>& mem, WtArgsHost& a,
               const std::string& tag) {
    const Pipeline& p = plan.p;
    std::memset(&a, 0, sizeof a);
    for (size_t i = 0; i < gr.loaded.size(); ++i) {
        const ImgRef& r = mem.at(gr.loaded[i]);
        if (!gr.resample && p.nodes[gr.loaded[i]].kind == Kind::Input)
            check_align(r, gr.g.V, node_esize(p, gr.loaded[i], false), tag + " input node " + std::to_string(gr.loaded[i]));
        a.src[i] = r.ptr;
        a.src_rs[i] = r.rs;
        a.src_cs[i] = r.cs;
    }
    for (size_t i = 0; i < gr.liveouts.size(); ++i) {
        const ImgRef& r = mem.at(gr.liveouts[i]);
        bool decimated = std::find(gr.g.dec.begin(), gr.g.dec.end(), gr.liveouts[i]) != gr.g.dec.end();
        if (!gr.resample && !decimated && p.is_output(gr.liveouts[i]) && p.nodes[gr.liveouts[i]].kind != Kind::Hist)
            check_align(r, gr.g.V, node_esize(p, gr.liveouts[i], false), tag + " output node " + std::to_string(gr.liveouts[i]));
        a.dst[i] = const_cast<void*>(r.ptr);
        a.dst_rs[i] = r.rs;
        a.dst_cs[i] = r.cs;
    }
}

void launch_group(const Plan& plan, const GroupRt& gr, const std::map<int, ImgRef>& mem, hipStream_t st) {
    const Pipeline& p = plan.p;
    WtArgsHost a;
    fill_args(plan, gr, mem, a, "");
    check_store_planes(plan, gr, a, gr.H);
    a.W = gr.W;
    a.H = gr.H;
    a.Ws = gr.Ws;
    a.Hs = gr.Hs;
    a.tiles_x = gr.tiles_x;
    a.tiles_y = gr.tiles_y;
    a.nwaves = gr.nwaves;
    for (size_t i = 0; i < gr.liveouts.size(); ++i) {  // histograms accumulate from zero
        const Node& hn = p.nodes[gr.liveouts[i]];
        if (hn.kind == Kind::Hist) hip_check(zero_hist(a.dst[i], a.dst_cs[i], hn.bins, hn.channels, st), "zero_hist");
    }
    void* params[] = {&a};
    hipError_t e;
    if (gr.resample) {
        int C = p.nodes[gr.g.nodes[0]].channels;
        e = hipModuleLaunchKernel(gr.fn, gr.tiles_x, gr.tiles_y, C, 256, 1, 1, 0, st, params, nullptr);
    } else {
        int grid = (gr.nwaves + gr.g.WPB - 1) / gr.g.WPB;
        e = hipModuleLaunchKernel(gr.fn, grid, 1, 1, 64 * gr.g.WPB, 1, 1, 0, st, params, nullptr);
    }
    hip_check(e, "hipModuleLaunchKernel");
}

std::string describe_plan(const Plan& plan) {
    std::ostringstream os;
    for (size_t i = 0; i < plan.sched.groups.size(); ++i) {
        os << "g" << i << " " << describe_group(plan.sched.groups[i]);
        if (plan.batch && i < plan.batch->grid.size())
            os << " batch_grid=" << plan.batch->grid[i] << " batch_wg_per_cu=" << plan.batch->per_cu[i]
               << " batch_work=" << plan.batch->total[i];
        os << "\n";
    }
    return os.str();
}

Machine machine_from_device(int device) {
    Machine m;
    hipDeviceProp_t pr;
    if (hipGetDeviceProperties(&pr, device) != hipSuccess) return m;
    if (pr.multiProcessorCount > 0) m.ncu = pr.multiProcessorCount;
    if (pr.warpSize > 0) m.wave = pr.warpSize;
    if (pr.maxSharedMemoryPerMultiProcessor > 0) m.lds_per_cu = (int)pr.maxSharedMemoryPerMultiProcessor;
    if (pr.sharedMemPerBlock > 0) m.max_lds_per_wg = (int)pr.sharedMemPerBlock;
    if (pr.clockRate > 0) m.clock_hz = pr.clockRate * 1e3;
    m.name = pr.gcnArchName;
    return m;
}

}  // namespace wt
