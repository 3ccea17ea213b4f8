// The C ABI (include/wt.h): argument checking, error translation and the
// pipeline builder.  No exception crosses this boundary.
#include <cmath>
#include <functional>
#include <cstring>
#include <string>

#include "wt_cost.h"
#include "wt_internal.h"
#include "wt_mlp.h"
#include "wt_runtime.h"

struct wt_pipeline {
    wt::Pipeline p;
};
struct wt_plan {
    std::unique_ptr<wt::Plan> impl;
};
struct wt_mlp {
    std::unique_ptr<wt::Mlp> impl;
};

namespace {
thread_local std::string g_err;

template <class F>
wt_status guard(F&& f) {
    try {
        f();
        return WT_OK;
    } catch (const wt::Error& e) {
        g_err = e.what();
        return e.status;
    } catch (const std::bad_alloc&) {
        g_err = "out of host memory";
        return WT_E_NOMEM;
    } catch (const std::exception& e) {
        g_err = e.what();
        return WT_E_INTERNAL;
    }
}

wt::Node& new_node(wt_pipeline* p, wt::Kind k) {
    p->p.nodes.emplace_back();
    wt::Node& n = p->p.nodes.back();
    n.kind = k;
    n.id = (int)p->p.nodes.size() - 1;
    return n;
}

void check_src(const wt_pipeline* p, int src) {
    if (src < 0 || src >= (int)p->p.nodes.size()) wt::fail(WT_E_INVALID, "unknown source node " + std::to_string(src));
    if (p->p.nodes[src].kind == wt::Kind::Hist) wt::fail(WT_E_UNSUPPORTED, "a histogram cannot be read by a stage");
}
}  // namespace

extern "C" {

const char* wt_last_error(void) { return g_err.c_str(); }

wt_status wt_pipeline_create(wt_pipeline** out) {
    return guard([&] {
        if (!out) wt::fail(WT_E_INVALID, "null output pointer");
        *out = new wt_pipeline();
    });
}

void wt_pipeline_destroy(wt_pipeline* p) { delete p; }

wt_status wt_input_typed(wt_pipeline* p, int channels, int dtype, int* id) {
    return guard([&] {
        if (!p || !id) wt::fail(WT_E_INVALID, "null argument");
        if (channels < 1 || channels > 16) wt::fail(WT_E_INVALID, "channels must be in 1..16");
        if (dtype != WT_F32 && !wt::is_int_dtype(dtype)) wt::fail(WT_E_UNSUPPORTED, "input element type");
        wt::Node& n = new_node(p, wt::Kind::Input);
        n.channels = channels;
        n.dtype = dtype;
        n.bound = 1.0;
        if (n.is_int()) {
            auto r = wt::dtype_range(dtype);
            n.rlo = (double)r.first;
            n.rhi = (double)r.second;
            n.bound = std::max(std::fabs(n.rlo), std::fabs(n.rhi));
        }
        p->p.inputs.push_back(n.id);
        *id = n.id;
    });
}

wt_status wt_input(wt_pipeline* p, int channels, int* id) { return wt_input_typed(p, channels, WT_F32, id); }

wt_status wt_input_bound(wt_pipeline* p, int id, double max_abs) {
    return guard([&] {
        if (!p) wt::fail(WT_E_INVALID, "null pipeline");
        if (id < 0 || id >= (int)p->p.nodes.size() || p->p.nodes[id].kind != wt::Kind::Input)
            wt::fail(WT_E_INVALID, "node " + std::to_string(id) + " is not an input");
        wt::Node& n = p->p.nodes[id];
        if (n.is_int()) wt::fail(WT_E_INVALID, "integer inputs carry their type's range");
        if (!(max_abs > 0.0) || !std::isfinite(max_abs)) wt::fail(WT_E_INVALID, "bound must be positive and finite");
        for (const wt::Node& m : p->p.nodes)
            for (int s : m.srcs)
                if (s == id) wt::fail(WT_E_INVALID, "declare an input's bound before a stage reads it");
        n.bound = max_abs;
    });
}

namespace {
// Integer values are exact in 32-bit registers below this magnitude.
constexpr double kInt32Max = 2147483647.0;

bool expr_is_integer(const wt::Expr& e) {
    switch (e.op) {
        case wt::Expr::Div: case wt::Expr::Sqrt: case wt::Expr::Floor: return false;
        case wt::Expr::Const:
            if (e.value != std::floor(e.value) || std::fabs(e.value) > 16777216.0) return false;
            break;
        default: break;
    }
    for (const auto& k : e.kids)
        if (!expr_is_integer(k)) return false;
    return true;
}
}  // namespace

wt_status wt_stencil_int(wt_pipeline* p, int src, int kw, int kh, int ax, int ay, const int32_t* weights,
                         int32_t divisor, int out, int* id) {
    return guard([&] {
        if (!p || !id || !weights) wt::fail(WT_E_INVALID, "null argument");
        check_src(p, src);
        if (kw < 1 || kw > 15 || kh < 1 || kh > 15) wt::fail(WT_E_INVALID, "stencil sides must be in 1..15");
        if (ax < 0 || ax >= kw || ay < 0 || ay >= kh) wt::fail(WT_E_INVALID, "stencil anchor outside the kernel");
        if (!wt::is_int_dtype(out)) wt::fail(WT_E_INVALID, "integer stencils produce an integer type");
        if (divisor < 1 || divisor > (1 << 24)) wt::fail(WT_E_INVALID, "divisor must be in 1..2^24");
        const wt::Node s = p->p.nodes[src];
        if (!s.is_int()) wt::fail(WT_E_UNSUPPORTED, "integer stencils read integer stages");
        double lo = 0, hi = 0, wsum = 0;
        for (int i = 0; i < kw * kh; ++i) {
            if (weights[i] < -32767 || weights[i] > 32767) wt::fail(WT_E_INVALID, "|weight| must be <= 32767");
            double w = weights[i];
            lo += std::min(w * s.rlo, w * s.rhi);
            hi += std::max(w * s.rlo, w * s.rhi);
            wsum += std::fabs(w);
        }
        (void)wsum;
        double half = (double)(divisor / 2);
        if (std::max(std::fabs(lo), std::fabs(hi)) + half > kInt32Max)
            wt::fail(WT_E_UNSUPPORTED, "integer stencil sums may leave the 32-bit range");
        wt::Node& n = new_node(p, wt::Kind::Stencil);
        n.srcs = {src};
        n.channels = s.channels;
        n.level = s.level;
        n.kw = kw;
        n.kh = kh;
        n.ax = ax;
        n.ay = ay;
        n.dtype = out;
        n.iweights.assign(weights, weights + kw * kh);
        n.weights.assign(weights, weights + kw * kh);
        n.divisor = divisor;
        n.scale = 1.0 / divisor;
        auto r = wt::dtype_range(out);
        n.rlo = std::max((double)r.first, std::floor((lo + half) / divisor));
        n.rhi = std::min((double)r.second, std::floor((hi + half) / divisor));
        if (n.rlo > n.rhi) n.rlo = n.rhi = std::min(std::max(0.0, (double)r.first), (double)r.second);
        n.bound = std::max(std::fabs(n.rlo), std::fabs(n.rhi));
        *id = n.id;
    });
}

wt_status wt_stencil(wt_pipeline* p, int src, int kw, int kh, int ax, int ay, const double* weights,
                     double scale, int* id) {
    return guard([&] {
        if (!p || !id || !weights) wt::fail(WT_E_INVALID, "null argument");
        check_src(p, src);
        if (kw < 1 || kw > 15 || kh < 1 || kh > 15) wt::fail(WT_E_INVALID, "stencil sides must be in 1..15");
        if (ax < 0 || ax >= kw || ay < 0 || ay >= kh) wt::fail(WT_E_INVALID, "stencil anchor outside the kernel");
        if (!std::isfinite(scale)) wt::fail(WT_E_INVALID, "non-finite scale");
        double absum = 0.0;
        for (int i = 0; i < kw * kh; ++i) {
            if (!std::isfinite(weights[i])) wt::fail(WT_E_INVALID, "non-finite weight");
            absum += std::fabs(weights[i]);
        }
        const wt::Node s = p->p.nodes[src];
        wt::Node& n = new_node(p, wt::Kind::Stencil);
        n.srcs = {src};
        n.channels = s.channels;
        n.level = s.level;
        n.kw = kw;
        n.kh = kh;
        n.ax = ax;
        n.ay = ay;
        n.weights.assign(weights, weights + kw * kh);
        n.scale = scale;
        n.bound = absum * std::fabs(scale) * s.bound;
        *id = n.id;
    });
}

wt_status wt_pointwise(wt_pipeline* p, const int* srcs, int nsrc, const char* expr, int out_channels, int* id) {
    return wt_pointwise_typed(p, srcs, nsrc, expr, out_channels, WT_F32, id);
}

wt_status wt_pointwise_typed(wt_pipeline* p, const int* srcs, int nsrc, const char* expr, int out_channels, int out,
                             int* id) {
    return guard([&] {
        if (out != WT_F32 && !wt::is_int_dtype(out)) wt::fail(WT_E_UNSUPPORTED, "pointwise element type");
        if (!p || !id || !srcs || !expr) wt::fail(WT_E_INVALID, "null argument");
        if (nsrc < 1 || nsrc > 8) wt::fail(WT_E_INVALID, "pointwise stages take 1..8 sources");
        if (out_channels < 1 || out_channels > 16) wt::fail(WT_E_INVALID, "channels must be in 1..16");
        std::vector<double> bounds;
        int level = -1;
        for (int i = 0; i < nsrc; ++i) {
            check_src(p, srcs[i]);
            const wt::Node& s = p->p.nodes[srcs[i]];
            if (level >= 0 && s.level != level) wt::fail(WT_E_INVALID, "pointwise sources on different levels");
            level = s.level;
            bounds.push_back(s.bound);
        }
        wt::Expr e = wt::parse_expr(expr, nsrc);
        for (int i = 0; i < nsrc; ++i) {
            const wt::Node& s = p->p.nodes[srcs[i]];
            if (wt::expr_max_channel(e, i) >= s.channels)
                wt::fail(WT_E_INVALID, "channel subscript beyond source " + std::to_string(i) + "'s channels");
        }
        // implicit (same-channel) references need 1 or out_channels channels
        std::function<void(const wt::Expr&)> chk = [&](const wt::Expr& x) {
            if (x.op == wt::Expr::Src && x.chan < 0) {
                int c = p->p.nodes[srcs[x.src]].channels;
                if (c != 1 && c != out_channels)
                    wt::fail(WT_E_INVALID, "source s" + std::to_string(x.src) + " has " + std::to_string(c) +
                                               " channels; use s" + std::to_string(x.src) + "[k]");
            }
            for (const auto& k : x.kids) chk(k);
        };
        chk(e);
        double rlo = 0, rhi = 0;
        if (wt::is_int_dtype(out)) {
            std::vector<wt::Interval> iv;
            for (int i = 0; i < nsrc; ++i) {
                const wt::Node& s = p->p.nodes[srcs[i]];
                if (!s.is_int()) wt::fail(WT_E_UNSUPPORTED, "integer pointwise stages read integer stages only");
                iv.push_back({s.rlo, s.rhi});
            }
            if (!expr_is_integer(e))
                wt::fail(WT_E_UNSUPPORTED, "integer expressions take integer constants and no /, sqrt or floor");
            double mx = 0;
            wt::Interval r = wt::expr_range(e, iv, &mx);
            if (!(mx <= kInt32Max)) wt::fail(WT_E_UNSUPPORTED, "integer expression may leave the 32-bit range");
            auto tr = wt::dtype_range(out);
            rlo = std::max((double)tr.first, r.lo);
            rhi = std::min((double)tr.second, r.hi);
            if (rlo > rhi) rlo = rhi = std::min(std::max(r.lo, (double)tr.first), (double)tr.second);
        }
        wt::Node& n = new_node(p, wt::Kind::Pointwise);
        n.srcs.assign(srcs, srcs + nsrc);
        n.channels = out_channels;
        n.level = level;
        n.expr_text = expr;
        n.expr = std::move(e);
        n.dtype = out;
        n.bound = wt::expr_bound(n.expr, bounds);
        if (n.is_int()) {
            n.rlo = rlo;
            n.rhi = rhi;
            n.bound = std::max(std::fabs(rlo), std::fabs(rhi));
        }
        *id = n.id;
    });
}

wt_status wt_resample(wt_pipeline* p, int src, int kind, int* id) {
    return guard([&] {
        if (!p || !id) wt::fail(WT_E_INVALID, "null argument");
        check_src(p, src);
        if (kind != WT_DOWN2 && kind != WT_UP2) wt::fail(WT_E_INVALID, "unknown resample kind");
        const wt::Node s = p->p.nodes[src];
        if (kind == WT_UP2 && s.level < 1) wt::fail(WT_E_INVALID, "up2 of a full-resolution node");
        if (kind == WT_DOWN2 && s.level >= 24) wt::fail(WT_E_INVALID, "too many decimations");
        if (kind == WT_UP2 && s.is_int()) wt::fail(WT_E_UNSUPPORTED, "up2 of an integer stage");
        wt::Node& n = new_node(p, kind == WT_DOWN2 ? wt::Kind::Down2 : wt::Kind::Up2);
        n.srcs = {src};
        n.channels = s.channels;
        n.level = s.level + (kind == WT_DOWN2 ? 1 : -1);
        n.bound = s.bound;
        n.dtype = s.dtype;
        n.rlo = s.rlo;
        n.rhi = s.rhi;
        *id = n.id;
    });
}

wt_status wt_histogram(wt_pipeline* p, int src, int bins, double lo, double hi, int* id) {
    return guard([&] {
        if (!p || !id) wt::fail(WT_E_INVALID, "null argument");
        check_src(p, src);
        if (bins < 1 || bins > 4096) wt::fail(WT_E_INVALID, "histogram bins must be in 1..4096");
        if (!std::isfinite(lo) || !std::isfinite(hi) || !(lo < hi)) wt::fail(WT_E_INVALID, "histogram needs lo < hi");
        const wt::Node s = p->p.nodes[src];
        wt::Node& n = new_node(p, wt::Kind::Hist);
        n.srcs = {src};
        n.channels = s.channels;
        n.level = s.level;
        n.dtype = WT_I32;
        n.bins = bins;
        n.hlo = lo;
        n.hhi = hi;
        n.bound = 2147483647.0;
        n.rlo = 0;
        n.rhi = 2147483647.0;
        *id = n.id;
    });
}

wt_status wt_equalize(wt_pipeline* p, int src, int hist, int* id) {
    return guard([&] {
        if (!p || !id) wt::fail(WT_E_INVALID, "null argument");
        check_src(p, src);
        if (hist < 0 || hist >= (int)p->p.nodes.size() || p->p.nodes[hist].kind != wt::Kind::Hist)
            wt::fail(WT_E_INVALID, "equalize needs a histogram node");
        const wt::Node s = p->p.nodes[src];
        if (s.channels != p->p.nodes[hist].channels) wt::fail(WT_E_INVALID, "equalize: channel counts differ");
        wt::Node& n = new_node(p, wt::Kind::Equalize);
        n.srcs = {src, hist};
        n.channels = s.channels;
        n.level = s.level;
        n.dtype = WT_F32;
        n.bound = 1.0;
        *id = n.id;
    });
}

wt_status wt_output(wt_pipeline* p, int id) {
    return guard([&] {
        if (!p) wt::fail(WT_E_INVALID, "null pipeline");
        if (id < 0 || id >= (int)p->p.nodes.size()) wt::fail(WT_E_INVALID, "unknown node " + std::to_string(id));
        if (p->p.nodes[id].kind == wt::Kind::Input) wt::fail(WT_E_INVALID, "an input cannot be an output");
        if (p->p.is_output(id)) wt::fail(WT_E_INVALID, "node already marked as output");
        p->p.outputs.push_back(id);
    });
}

wt_status wt_plan_create(const wt_pipeline* p, const wt_sched_opts* opts, int width, int height, void* stream,
                         wt_plan** out) {
    return guard([&] {
        if (!p || !out) wt::fail(WT_E_INVALID, "null argument");
        *out = nullptr;
        auto impl = wt::create_plan(p->p, opts, width, height, stream);
        *out = new wt_plan{std::move(impl)};
    });
}

wt_status wt_plan_run(wt_plan* plan, const wt_image* in, int nin, const wt_image* out, int nout, void* stream) {
    return guard([&] {
        if (!plan) wt::fail(WT_E_INVALID, "null plan");
        wt::run_plan(*plan->impl, in, nin, out, nout, stream);
    });
}

wt_status wt_plan_run_batch(wt_plan* plan, int nimg, const wt_image* in, const wt_image* out, void* stream) {
    return guard([&] {
        if (!plan) wt::fail(WT_E_INVALID, "null plan");
        wt::run_plan_batch(*plan->impl, nimg, in, out, stream);
    });
}

wt_status wt_plan_run_batch_static(wt_plan* plan, int nimg, const wt_image* in, const wt_image* out, void* stream) {
    return guard([&] {
        if (!plan) wt::fail(WT_E_INVALID, "null plan");
        wt::run_plan_batch_static(*plan->impl, nimg, in, out, stream);
    });
}

wt_status wt_plan_batch_check(wt_plan* plan, void* stream) {
    return guard([&] {
        if (!plan) wt::fail(WT_E_INVALID, "null plan");
        wt::check_batch_status(*plan->impl, stream);
    });
}

wt_status wt_plan_whole_tables(const wt_plan* plan, int nimg, const int* wh, int resident_waves, int* chunks,
                               int max_chunks, int* nchunks, unsigned long long* deps) {
    return guard([&] {
        if (!plan || !wh || !nchunks) wt::fail(WT_E_INVALID, "null argument");
        if (nimg < 1 || resident_waves < 1 || max_chunks < 0) wt::fail(WT_E_INVALID, "bad count");
        std::vector<std::pair<int, int>> sizes(nimg);
        for (int i = 0; i < nimg; ++i) {
            if (wh[2 * i] < 1 || wh[2 * i + 1] < 1 || wh[2 * i] > (1 << 24) || wh[2 * i + 1] > (1 << 24))
                wt::fail(WT_E_SHAPE, "bad image size");
            sizes[i] = {wh[2 * i], wh[2 * i + 1]};
        }
        std::vector<int> tab;
        std::vector<unsigned long long> dep;
        wt::whole_tables(*plan->impl, sizes, resident_waves, tab, dep);
        *nchunks = (int)(tab.size() / 4);
        if (chunks) {
            if (*nchunks > max_chunks) wt::fail(WT_E_INVALID, "chunk buffer too small");
            std::memcpy(chunks, tab.data(), tab.size() * sizeof(int));
        }
        if (deps) std::memcpy(deps, dep.data(), dep.size() * sizeof(unsigned long long));
    });
}

wt_status wt_plan_tune_batch(wt_plan* plan, int nimg, const wt_image* in, const wt_image* out, void* stream) {
    return guard([&] {
        if (!plan) wt::fail(WT_E_INVALID, "null plan");
        wt::tune_plan_batch(*plan->impl, nimg, in, out, stream);
    });
}

wt_status wt_plan_run_batch_groups(wt_plan* plan, int first, int count, int nimg, const wt_image* in,
                                   const wt_image* out, void* stream) {
    return guard([&] {
        if (!plan) wt::fail(WT_E_INVALID, "null plan");
        if (count < 1) wt::fail(WT_E_INVALID, "count must be at least 1");
        wt::run_plan_batch(*plan->impl, nimg, in, out, stream, first, count);
    });
}

static wt_status copy_out(const std::string& s, char* buf, size_t len, size_t* needed) {
    if (needed) *needed = s.size() + 1;
    if (buf && len) {
        size_t n = std::min(len - 1, s.size());
        std::memcpy(buf, s.data(), n);
        buf[n] = '\0';
    }
    return WT_OK;
}

wt_status wt_plan_describe(const wt_plan* plan, char* buf, size_t len, size_t* needed) {
    wt_status st = guard([&] {
        if (!plan) wt::fail(WT_E_INVALID, "null plan");
    });
    if (st != WT_OK) return st;
    return copy_out(wt::describe_plan(*plan->impl), buf, len, needed);
}

wt_status wt_plan_source(const wt_plan* plan, int group, char* buf, size_t len, size_t* needed) {
    std::string whole;
    wt_status st = guard([&] {
        if (!plan) wt::fail(WT_E_INVALID, "null plan");
        if (group == -1) {
            std::string kname;
            whole = wt::whole_kernel_source(*plan->impl, kname);
        } else if (group < 0 || group >= (int)plan->impl->groups.size()) {
            wt::fail(WT_E_INVALID, "group out of range");
        }
    });
    if (st != WT_OK) return st;
    return copy_out(group == -1 ? whole : plan->impl->groups[group].src, buf, len, needed);
}

wt_status wt_plan_group_info(const wt_plan* plan, int group, wt_group_info* out) {
    return guard([&] {
        if (!plan || !out) wt::fail(WT_E_INVALID, "null argument");
        if (group < 0 || group >= (int)plan->impl->groups.size()) wt::fail(WT_E_INVALID, "group out of range");
        const wt::GroupRt& g = plan->impl->groups[group];
        std::memset(out, 0, sizeof *out);
        out->resample = g.resample;
        out->waves_per_group = g.g.WPB;
        out->nwaves = g.nwaves;
        out->tiles_x = g.tiles_x;
        out->tiles_y = g.tiles_y;
        out->width = g.W;
        out->height = g.H;
        out->src_width = g.Ws;
        out->src_height = g.Hs;
        out->channels = plan->impl->p.nodes[g.g.nodes[0]].channels;
        out->nloaded = (int)g.loaded.size();
        out->nliveouts = (int)g.liveouts.size();
        for (size_t i = 0; i < g.loaded.size(); ++i) {
            out->loaded[i] = g.loaded[i];
            out->loaded_half[i] = g.mem_half_in[i];
            out->loaded_dtype[i] = g.mem_half_in[i] ? WT_F16 : plan->impl->p.nodes[g.loaded[i]].dtype;
        }
        for (size_t i = 0; i < g.liveouts.size(); ++i) {
            out->liveouts[i] = g.liveouts[i];
            out->liveout_half[i] = g.mem_half_out[i];
            out->liveout_dtype[i] = g.mem_half_out[i] ? WT_F16 : plan->impl->p.nodes[g.liveouts[i]].dtype;
        }
    });
}

wt_status wt_fusion_costs(const wt_pipeline* p, int width, int height, int fp16, int max_group, double* dp_us,
                          double* exhaustive_us) {
    return guard([&] {
        if (!p || !dp_us || !exhaustive_us) wt::fail(WT_E_INVALID, "null argument");
        wt::SchedRequest r;
        r.W = width;
        r.H = height;
        r.fp16 = fp16 != 0;
        r.max_group = max_group;
        wt::fusion_costs(p->p, wt::Machine{}, r, dp_us, exhaustive_us);
    });
}

wt_status wt_measure_groups(const wt_pipeline* p, int width, int height, int fp16, int n,
                            const char* const* groups, int reps, const char* tag, double* times_us) {
    return guard([&] {
        if (!p || (n > 0 && (!groups || !times_us))) wt::fail(WT_E_INVALID, "null argument");
        if (n < 0 || reps < 0 || reps > 100000) wt::fail(WT_E_INVALID, "bad count");
        if (width <= 0 || height <= 0 || width > (1 << 16) || height > (1 << 16))
            wt::fail(WT_E_SHAPE, "bad measurement size");
        std::vector<std::string> d;
        for (int i = 0; i < n; ++i) {
            if (!groups[i]) wt::fail(WT_E_INVALID, "null group text");
            d.emplace_back(groups[i]);
        }
        wt::measure_groups(p->p, width, height, fp16 != 0, d, reps, tag ? tag : "", times_us);
    });
}

wt_status wt_stage_profile(const wt_pipeline* p, int node, int width, int height, int measure,
                           double* ns_per_point, int* vgprs, int* measured) {
    return guard([&] {
        if (!p || !ns_per_point || !vgprs || !measured) wt::fail(WT_E_INVALID, "null argument");
        check_src(p, node);
        const wt::Node& n = p->p.nodes[node];
        if (n.kind != wt::Kind::Stencil && n.kind != wt::Kind::Pointwise)
            wt::fail(WT_E_INVALID, "only stencil and pointwise stages are profiled");
        if (width <= 0 || height <= 0) wt::fail(WT_E_SHAPE, "bad size");
        wt::StageProfile sp = wt::stage_profile(p->p, node, width, height, measure != 0);
        *ns_per_point = sp.ns_per_point;
        *vgprs = sp.vgprs;
        *measured = sp.measured ? 1 : 0;
    });
}

wt_status wt_alg2_eval(int machine, const double* in, const double* w, double* out) {
    return guard([&] {
        if (!in || !out) wt::fail(WT_E_INVALID, "null argument");
        if (machine != 0 && machine != 1) wt::fail(WT_E_INVALID, "machine must be 0 or 1");
        wt::Machine m = machine ? wt::machine_gtx1080ti() : wt::machine_gfx950();
        wt::Alg2In a;
        a.smem_per_wg = in[0];
        a.regs_per_lane = in[1];
        a.waves_per_wg = (int)in[2];
        a.total_wg = (long long)in[3];
        a.total_tx = in[4];
        a.compulsory_tx = in[5];
        a.mem_bytes_per_wave = in[6];
        a.compute_time_per_wave = in[7];
        a.frac_overlap = in[8];
        if (a.waves_per_wg < 1 || a.total_wg < 1) wt::fail(WT_E_INVALID, "bad block counts");
        wt::Alg2Out o = wt::alg2(a, m, w ? w : wt::kGfx950Weights);
        out[0] = o.feasible ? 1 : 0;
        out[1] = o.score;
        out[2] = o.occupancy;
        out[3] = o.shmem_occ;
        out[4] = o.reg_occ;
        for (int k = 0; k < 7; ++k) out[5 + k] = o.terms[k];
    });
}

wt_status wt_otpw_geometry(const int* block, int ws, const int* tile, const int* overlap, int* warp,
                           int64_t* scratch_elems) {
    return guard([&] {
        if (!block || !tile || !overlap || !warp || !scratch_elems) wt::fail(WT_E_INVALID, "null argument");
        if (ws < 1) wt::fail(WT_E_INVALID, "bad warp size");
        for (int i = 0; i < 3; ++i)
            if (block[i] < 1 || tile[i] < 1 || overlap[i] < 0) wt::fail(WT_E_INVALID, "bad sizes");
        wt::warp_sizes(block, ws, warp);
        *scratch_elems = wt::scratchpad_elems(tile, block, warp, overlap);
    });
}

wt_status wt_stream_copy(const void* src, void* dst, size_t bytes, void* stream) {
    return guard([&] {
        if (bytes == 0) return;
        if (!src || !dst) wt::fail(WT_E_INVALID, "null pointer");
        if (((uintptr_t)src | (uintptr_t)dst) % 16) wt::fail(WT_E_INVALID, "pointers must be 16-byte aligned");
        const uintptr_t a = (uintptr_t)src, b = (uintptr_t)dst;
        if (a < b + bytes && b < a + bytes) wt::fail(WT_E_INVALID, "source and destination overlap");
        hipError_t e = wt::stream_copy(src, dst, bytes, (hipStream_t)stream);
        if (e != hipSuccess) wt::fail(WT_E_HIP, std::string("stream copy: ") + hipGetErrorString(e));
    });
}

wt_status wt_mlp_create(const int* dims, int nlayers, uint64_t seed, wt_mlp** out) {
    return guard([&] {
        if (!dims || !out || nlayers < 2 || nlayers > 16) wt::fail(WT_E_INVALID, "bad mlp arguments");
        *out = new wt_mlp{std::make_unique<wt::Mlp>(std::vector<int>(dims, dims + nlayers), seed)};
    });
}
void wt_mlp_destroy(wt_mlp* m) { delete m; }
size_t wt_mlp_num_params(const wt_mlp* m) { return m ? m->impl->nparams : 0; }
wt_status wt_mlp_get_params(const wt_mlp* m, float* params, size_t n) {
    return guard([&] {
        if (!m || !params || n != m->impl->nparams) wt::fail(WT_E_INVALID, "bad parameter buffer");
        std::memcpy(params, m->impl->host.data(), n * sizeof(float));
    });
}
wt_status wt_mlp_set_params(wt_mlp* m, const float* params, size_t n) {
    return guard([&] {
        if (!m || !params || n != m->impl->nparams) wt::fail(WT_E_INVALID, "bad parameter buffer");
        std::memcpy(m->impl->host.data(), params, n * sizeof(float));
        m->impl->upload_params();
    });
}
wt_status wt_mlp_forward(wt_mlp* m, const float* x, int batch, float* y) {
    return guard([&] {
        if (!m || !x || !y || batch < 1) wt::fail(WT_E_INVALID, "bad forward arguments");
        m->impl->forward(x, batch, y);
    });
}
wt_status wt_mlp_forward_backward(wt_mlp* m, const float* x, const float* t, int batch, float* loss, float* grads) {
    return guard([&] {
        if (!m || !x || !t || !loss || batch < 1) wt::fail(WT_E_INVALID, "bad backward arguments");
        *loss = m->impl->forward_backward(x, t, batch, grads);
    });
}
wt_status wt_mlp_adam_step(wt_mlp* m, const float* grads, float lr) {
    return guard([&] {
        if (!m || !grads) wt::fail(WT_E_INVALID, "bad adam arguments");
        m->impl->adam_from_host(grads, lr);
    });
}
wt_status wt_mlp_train(wt_mlp* m, const float* x, const float* t, int n, int epochs, int batch, float lr,
                       uint64_t seed, float* final_loss) {
    return guard([&] {
        if (!m || !x || !t || n < 2 || epochs < 1 || batch < 1) wt::fail(WT_E_INVALID, "bad training arguments");
        float l = m->impl->train(x, t, n, epochs, batch, lr, seed);
        if (final_loss) *final_loss = l;
    });
}
wt_status wt_model_train(const char* measure_db, const char* out_model, void* stream) {
    return guard([&] {
        if (!measure_db || !out_model) wt::fail(WT_E_INVALID, "null path");
        wt::train_model_from_db(measure_db, out_model, reinterpret_cast<hipStream_t>(stream));
    });
}

wt_status wt_model_rows(const char* measure_db, int* rows) {
    return guard([&] {
        if (!measure_db || !rows) wt::fail(WT_E_INVALID, "null argument");
        std::vector<float> x, t;
        *rows = wt::read_measure_db(measure_db, x, t);
    });
}

wt_status wt_mlp_predict(wt_mlp* m, const float* x, int n, float* y) {
    return guard([&] {
        if (!m || !x || !y || n < 1) wt::fail(WT_E_INVALID, "bad predict arguments");
        m->impl->predict(x, n, y);
    });
}
wt_status wt_mlp_save(const wt_mlp* m, const char* path) {
    return guard([&] {
        if (!m || !path) wt::fail(WT_E_INVALID, "null argument");
        m->impl->save(path);
    });
}
wt_status wt_mlp_load(const char* path, wt_mlp** out) {
    return guard([&] {
        if (!path || !out) wt::fail(WT_E_INVALID, "null argument");
        *out = new wt_mlp{wt::Mlp::load(path)};
    });
}

wt_status wt_group_features(const wt_pipeline* p, const int* nodes, int nnodes, int width, int height, int fp16,
                            float* features, int max_rows, int* rows, char* text, size_t text_len) {
    return guard([&] {
        if (!p || !nodes || nnodes < 1 || !rows) wt::fail(WT_E_INVALID, "null argument");
        wt::SchedRequest r;
        r.W = width;
        r.H = height;
        r.fp16 = fp16 != 0;
        std::vector<int> ns, dec;
        for (int i = 0; i < nnodes; ++i) {
            if (nodes[i] < 0 || nodes[i] >= (int)p->p.nodes.size()) wt::fail(WT_E_INVALID, "node out of range");
            (p->p.nodes[nodes[i]].kind == wt::Kind::Down2 ? dec : ns).push_back(nodes[i]);
        }
        std::sort(ns.begin(), ns.end());
        std::sort(dec.begin(), dec.end());
        if (ns.empty()) wt::fail(WT_E_INVALID, "group without a fusable stage");
        auto cfgs = wt::score_configs(p->p, wt::Machine{}, r, ns, dec);
        std::string all;
        int n = 0;
        for (const auto& c : cfgs) {
            if (n >= max_rows) break;
            wt::GroupGeom geo = wt::group_geometry(p->p, c.g);
            std::vector<double> f = wt::group_features(p->p, c.g, geo, c.cost, width, height, c.tx_size);
            if (features)
                for (int k = 0; k < wt::kNumFeatures; ++k) features[(size_t)n * wt::kNumFeatures + k] = (float)f[k];
            all += (n ? ";" : "") + wt::describe_group(c.g);
            ++n;
        }
        *rows = n;
        if (text && text_len) {
            size_t k = std::min(text_len - 1, all.size());
            std::memcpy(text, all.data(), k);
            text[k] = '\0';
        }
    });
}

int wt_plan_num_groups(const wt_plan* plan) { return plan ? (int)plan->impl->groups.size() : 0; }

void wt_plan_destroy(wt_plan* plan) { delete plan; }

}  // extern "C"
