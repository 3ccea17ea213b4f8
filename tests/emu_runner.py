"""Runs a plan's generated kernels on the CPU with the lane emulator
(tests/emu/wt_emu.h): the exact HIP source the library compiles for gfx950,
built for the host with clang, one wavefront at a time as 64 threads."""
import ctypes
import hashlib
import os
import subprocess

import numpy as np

import oracle
import paper_1909_07190_amd as wt

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(os.path.dirname(HERE), "_build", "emu")
CLANG = "/opt/rocm/llvm/bin/clang++"


GroupInfo = wt.GroupInfo


class Args(ctypes.Structure):
    _fields_ = [("src", ctypes.c_void_p * 16), ("dst", ctypes.c_void_p * 16),
                ("src_rs", ctypes.c_int64 * 16), ("src_cs", ctypes.c_int64 * 16),
                ("dst_rs", ctypes.c_int64 * 16), ("dst_cs", ctypes.c_int64 * 16)] + \
               [(n, ctypes.c_int32) for n in ("W", "H", "Ws", "Hs", "tiles_x", "tiles_y", "nwaves", "pad")]



RUNNER = r"""
extern "C" int wt_emu_run(const WtArgs* a, int nwaves, int wpb) {
    std::barrier<> bar(64);
    wt_emu_bar = &bar;
    std::vector<std::thread> th;
    int nblocks = (nwaves + wpb - 1) / wpb;
    for (int l = 0; l < 64; ++l)
        th.emplace_back([&, l] {
            wt_emu_lane = l;
            for (int b = 0; b < nblocks; ++b)
                for (int w = 0; w < wpb; ++w) {
                    blockIdx.x = b; threadIdx.x = w * 64 + l; gridDim.x = nblocks;
                    bar.arrive_and_wait();
                    WT_EMU_KERNEL(*a);
                    bar.arrive_and_wait();
                }
        });
    for (auto& t : th) t.join();
    return 0;
}
// one-tile-per-workgroup kernels: all waves of a workgroup run together
// (their __syncthreads is a barrier over 64 * wpb threads; they use no lane
// exchanges)
extern "C" int wt_emu_run_wg(const WtArgs* a, int nblocks, int wpb) {
    std::barrier<> bar(64 * wpb);
    wt_emu_bar = &bar;
    std::vector<std::thread> th;
    for (int t = 0; t < 64 * wpb; ++t)
        th.emplace_back([&, t] {
            wt_emu_lane = t & 63;
            for (int b = 0; b < nblocks; ++b) {
                blockIdx.x = b; threadIdx.x = t; gridDim.x = nblocks;
                bar.arrive_and_wait();
                WT_EMU_KERNEL(*a);
                bar.arrive_and_wait();
            }
        });
    for (auto& t : th) t.join();
    return 0;
}
extern "C" int wt_emu_run_wg_batch(const WtArgs* ab, const int* start, int nimg, int total, int nblocks, int wpb) {
    std::barrier<> bar(64 * wpb);
    wt_emu_bar = &bar;
    std::vector<std::thread> th;
    for (int t = 0; t < 64 * wpb; ++t)
        th.emplace_back([&, t] {
            wt_emu_lane = t & 63;
            for (int b = 0; b < nblocks; ++b) {
                blockIdx.x = b; threadIdx.x = t; gridDim.x = nblocks;
                bar.arrive_and_wait();
                WT_EMU_KERNEL_BATCH(ab, start, nimg, total);
                bar.arrive_and_wait();
            }
        });
    for (auto& t : th) t.join();
    return 0;
}
extern "C" int wt_emu_run_batch(const WtArgs* ab, const int* start, int nimg, int total, int nblocks, int wpb) {
    std::barrier<> bar(64);
    wt_emu_bar = &bar;
    std::vector<std::thread> th;
    for (int l = 0; l < 64; ++l)
        th.emplace_back([&, l] {
            wt_emu_lane = l;
            for (int b = 0; b < nblocks; ++b)
                for (int w = 0; w < wpb; ++w) {
                    blockIdx.x = b; threadIdx.x = w * 64 + l; gridDim.x = nblocks;
                    bar.arrive_and_wait();
                    WT_EMU_KERNEL_BATCH(ab, start, nimg, total);
                    bar.arrive_and_wait();
                }
        });
    for (auto& t : th) t.join();
    return 0;
}
extern "C" int wt_emu_run_grid_batch(const WtArgs* ab, const int* start, int nimg, int total, int nblocks) {
    for (int b = 0; b < nblocks; ++b)
        for (int t = 0; t < 256; ++t) {
            blockIdx.x = b; threadIdx.x = t; gridDim.x = nblocks;
            WT_EMU_KERNEL_BATCH(ab, start, nimg, total);
        }
    return 0;
}
// lone-histogram kernels: a 3-D grid of workgroups whose threads meet at
// __syncthreads (nthr threads started together, one workgroup at a time)
extern "C" int wt_emu_run_grid_wg(const WtArgs* a, int gx, int gy, int gz, int nthr) {
    std::barrier<> bar(nthr);
    wt_emu_bar = &bar;
    std::vector<std::thread> th;
    for (int t = 0; t < nthr; ++t)
        th.emplace_back([&, t] {
            wt_emu_lane = t & 63;
            for (int z = 0; z < gz; ++z) for (int y = 0; y < gy; ++y) for (int x = 0; x < gx; ++x) {
                blockIdx.x = x; blockIdx.y = y; blockIdx.z = z; threadIdx.x = t;
                gridDim.x = gx; gridDim.y = gy; gridDim.z = gz;
                bar.arrive_and_wait();
                WT_EMU_KERNEL(*a);
                bar.arrive_and_wait();
            }
        });
    for (auto& t : th) t.join();
    return 0;
}
extern "C" int wt_emu_run_grid(const WtArgs* a, int gx, int gy, int gz, int nthr) {
    for (int z = 0; z < gz; ++z) for (int y = 0; y < gy; ++y) for (int x = 0; x < gx; ++x)
        for (int t = 0; t < nthr; ++t) {
            blockIdx.x = x; blockIdx.y = y; blockIdx.z = z; threadIdx.x = t;
            gridDim.x = gx; gridDim.y = gy; gridDim.z = gz;
            WT_EMU_KERNEL(*a);
        }
    return 0;
}
"""


def _text_hash(text):
    """Cache key of an emulator build: its source and the emulation header it
    includes (a changed header rebuilds every kernel)."""
    with open(os.path.join(HERE, "emu", "wt_emu.h"), "rb") as f:
        return hashlib.sha1(text.encode() + f.read()).hexdigest()[:16]


def _compile(src, kname):
    os.makedirs(CACHE, exist_ok=True)
    text = '#include "wt_emu.h"\n' + src + f"\n#define WT_EMU_KERNEL {kname}\n#define WT_EMU_KERNEL_BATCH {kname}_batch\n" + RUNNER
    h = _text_hash(text)
    so = os.path.join(CACHE, f"{kname}_{h}.so")
    if not os.path.exists(so):
        cpp = so[:-3] + ".cpp"
        open(cpp, "w").write(text)
        subprocess.run([CLANG, "-std=c++20", "-O1", "-shared", "-fPIC", "-pthread", "-w",
                        f"-I{os.path.join(HERE, 'emu')}", cpp, "-o", so + ".tmp"], check=True)
        os.replace(so + ".tmp", so)
    lib = ctypes.CDLL(so)
    lib.wt_emu_run.argtypes = [ctypes.POINTER(Args), ctypes.c_int, ctypes.c_int]
    lib.wt_emu_run_grid.argtypes = [ctypes.POINTER(Args)] + [ctypes.c_int] * 4
    lib.wt_emu_run_grid_wg.argtypes = [ctypes.POINTER(Args)] + [ctypes.c_int] * 4
    lib.wt_emu_run_batch.argtypes = [ctypes.c_void_p, ctypes.c_void_p] + [ctypes.c_int] * 4
    lib.wt_emu_run_grid_batch.argtypes = [ctypes.c_void_p, ctypes.c_void_p] + [ctypes.c_int] * 3
    lib.wt_emu_run_wg.argtypes = [ctypes.POINTER(Args), ctypes.c_int, ctypes.c_int]
    lib.wt_emu_run_wg_batch.argtypes = [ctypes.c_void_p, ctypes.c_void_p] + [ctypes.c_int] * 4
    return lib


def _is_blk(plan, g):
    """Whether group g runs one tile per workgroup (BLK=1 in its schedule)."""
    return "BLK=1" in plan.describe().splitlines()[g].split()


def _meta(spec):
    lv, ch = {}, {}
    names = []
    for i in spec["inputs"]:
        lv[i["name"]], ch[i["name"]] = 0, i["channels"]
        names.append(i["name"])
    for st in spec["stages"]:
        n = st["name"]
        names.append(n)
        if st["kind"] == "pointwise":
            lv[n], ch[n] = lv[st["srcs"][0]], st["channels"]
        else:
            d = {"down2": 1, "up2": -1}.get(st["kind"], 0)
            lv[n], ch[n] = lv[st["src"]] + d, ch[st["src"]]
    return names, lv, ch


NP_DTYPE = {0: np.float32, 1: np.float16, 2: np.uint8, 3: np.uint16, 4: np.int16, 5: np.int32}
SPEC_NP = {"f32": np.float32, "u8": np.uint8, "u16": np.uint16, "i16": np.int16, "i32": np.int32}


def _blank(shape, code):
    t = NP_DTYPE[code]
    if np.issubdtype(t, np.floating):
        return np.full(shape, np.nan, dtype=t)
    return np.full(shape, 0x5A, dtype=t)  # a value kernels must overwrite


def _result(b):
    return b.astype(np.int64) if np.issubdtype(b.dtype, np.integer) else b.astype(np.float32)


def _check_caller_alignment(plan, g, gi, caller, width):
    """The device runtime refuses caller images whose rows are not aligned to
    a group's vector width (its intermediates are padded); the emulator runs
    the same code on the host, so it refuses such images too instead of
    taking a misaligned vector access."""
    if gi.resample:
        return
    toks = plan.describe().splitlines()[g].split()
    v = int(next(t for t in toks if t.startswith("V=")).split("=")[1])
    nodes = list(gi.loaded[:gi.nloaded]) + list(gi.liveouts[:gi.nliveouts])
    narrow = {2, 3, 4}  # u8, u16, i16 element codes
    dts = {gi.loaded[i]: gi.loaded_dtype[i] for i in range(gi.nloaded)}
    dts.update({gi.liveouts[i]: gi.liveout_dtype[i] for i in range(gi.nliveouts)})
    if v > 1 and width % v and any(n in caller and dts.get(n) in narrow for n in nodes):
        raise ValueError(f"group {g}: image rows of width {width} not aligned to V={v}")


def emulate(spec, inputs, **plan_kw):
    """Runs `spec` through the generated kernels on the CPU; returns the outputs."""
    names, lv, ch = _meta(spec)
    first = inputs[spec["inputs"][0]["name"]]
    h, w = first.shape[-2:]
    plan = wt.from_spec(spec).plan(w, h, no_device=True, **plan_kw)
    bufs = {}  # node id -> array

    hists = {st["name"]: st for st in spec["stages"] if st["kind"] == "hist"}

    def buf(node_id, code):
        if node_id not in bufs:
            nm = names[node_id]
            if nm in hists:  # counts start at zero (the runtime clears them before the group)
                bufs[node_id] = np.zeros((ch[nm], 1, hists[nm]["bins"]), dtype=NP_DTYPE[code])
            else:
                bw, bh = oracle.level_size(w, h, lv[nm])
                bufs[node_id] = _blank((ch[nm], bh, bw), code)
        return bufs[node_id]

    import concurrent.futures as cf
    srcs = [plan.source(g) for g in range(plan.num_groups)]
    knames = [s[s.index("void __launch_bounds__"):].split("(")[1].split(")")[1].strip() for s in srcs]
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 4)) as ex:
        libs = list(ex.map(lambda a: _compile(*a), zip(srcs, knames)))
    for i, inp in enumerate(spec["inputs"]):
        t = SPEC_NP[inp.get("dtype", "f32")]
        bufs[i] = np.ascontiguousarray(inputs[inp["name"]]).astype(t).reshape(ch[inp["name"]], h, w)
    caller = set(range(len(spec["inputs"]))) | {names.index(o) for o in spec["outputs"]}
    for g in range(plan.num_groups):
        gi = GroupInfo()
        wt._check(wt.lib.wt_plan_group_info(plan._h, g, ctypes.byref(gi)))
        _check_caller_alignment(plan, g, gi, caller, w)
        lib = libs[g]
        a = Args()
        for i in range(gi.nloaded):
            b = buf(gi.loaded[i], gi.loaded_dtype[i])
            a.src[i] = b.ctypes.data
            a.src_rs[i], a.src_cs[i] = b.shape[2], b.shape[1] * b.shape[2]
        for i in range(gi.nliveouts):
            b = buf(gi.liveouts[i], gi.liveout_dtype[i])
            a.dst[i] = b.ctypes.data
            a.dst_rs[i], a.dst_cs[i] = b.shape[2], b.shape[1] * b.shape[2]
        a.W, a.H, a.Ws, a.Hs = gi.width, gi.height, gi.src_width, gi.src_height
        a.tiles_x, a.tiles_y, a.nwaves = gi.tiles_x, gi.tiles_y, gi.nwaves
        if gi.resample and names[gi.liveouts[0]] in hists:
            lib.wt_emu_run_grid_wg(ctypes.byref(a), gi.tiles_x, gi.tiles_y, gi.channels, 256)
        elif gi.resample:
            lib.wt_emu_run_grid(ctypes.byref(a), gi.tiles_x, gi.tiles_y, gi.channels, 256)
        elif _is_blk(plan, g):
            lib.wt_emu_run_wg(ctypes.byref(a), gi.nwaves // gi.waves_per_group, gi.waves_per_group)
        else:
            lib.wt_emu_run(ctypes.byref(a), gi.nwaves, gi.waves_per_group)
    plan.emu_buffers = bufs  # node id -> array, for diagnosis
    return {o: _result(bufs[names.index(o)]) for o in spec["outputs"]}, plan


def emulate_batch(spec, images, nblocks=3, **plan_kw):
    """Runs a batch of images (list of input dicts, sizes may differ) through
    the persistent batch kernels on the CPU, `nblocks` workgroups per launch
    so the grid-stride loop runs; per-image arguments come from one plan per
    image size (no device).  Returns one output dict per image."""
    names, lv, ch = _meta(spec)
    hists = {st["name"]: st for st in spec["stages"] if st["kind"] == "hist"}
    plans, bufs_all = _batch_inputs(spec, images, plan_kw, names, ch)
    ngroups = plans[0].num_groups
    for g in range(ngroups):
        src = plans[0].source(g)
        kname = src[src.index("void __launch_bounds__"):].split("(")[1].split(")")[1].strip()
        lib = _compile(src, kname)
        arr, start, total, resample, wpb, gi = _group_tables(plans, bufs_all, g, names, lv, ch, hists)
        if resample and names[gi.liveouts[0]] in hists:  # 256 threads meeting at __syncthreads
            lib.wt_emu_run_wg_batch(ctypes.addressof(arr), ctypes.addressof(start), len(images), total, nblocks, 4)
        elif resample:
            lib.wt_emu_run_grid_batch(ctypes.addressof(arr), ctypes.addressof(start), len(images), total, nblocks)
        elif _is_blk(plans[0], g):
            lib.wt_emu_run_wg_batch(ctypes.addressof(arr), ctypes.addressof(start), len(images), total, nblocks, wpb)
        else:
            lib.wt_emu_run_batch(ctypes.addressof(arr), ctypes.addressof(start), len(images), total, nblocks, wpb)
    emulate_batch.buffers = bufs_all  # every image's node buffers, for diagnosis
    return [{o: _result(b[names.index(o)]) for o in spec["outputs"]} for (_, _, b) in bufs_all]


def _group_tables(plans, bufs_all, g, names, lv, ch, hists):
    """Group g's per-image argument table and work prefix sums for a batch
    (one plan per image size; missing intermediates are created in each
    image's buffers)."""
    nimg = len(plans)
    arr = (Args * nimg)()
    start = (ctypes.c_int * (nimg + 1))()
    total = 0
    resample = False
    wpb = 1
    gi = None
    for k, plan in enumerate(plans):
        gi = GroupInfo()
        wt._check(wt.lib.wt_plan_group_info(plan._h, g, ctypes.byref(gi)))
        resample = bool(gi.resample)
        wpb = gi.waves_per_group
        w, h, bufs = bufs_all[k]

        def buf(node_id, code):
            if node_id not in bufs:
                nm = names[node_id]
                if nm in hists:  # counts start at zero
                    bufs[node_id] = np.zeros((ch[nm], 1, hists[nm]["bins"]), dtype=NP_DTYPE[code])
                else:
                    bw, bh = oracle.level_size(w, h, lv[nm])
                    bufs[node_id] = _blank((ch[nm], bh, bw), code)
            return bufs[node_id]

        a = arr[k]
        for i in range(gi.nloaded):
            b = buf(gi.loaded[i], gi.loaded_dtype[i])
            a.src[i] = b.ctypes.data
            a.src_rs[i], a.src_cs[i] = b.shape[2], b.shape[1] * b.shape[2]
        for i in range(gi.nliveouts):
            b = buf(gi.liveouts[i], gi.liveout_dtype[i])
            a.dst[i] = b.ctypes.data
            a.dst_rs[i], a.dst_cs[i] = b.shape[2], b.shape[1] * b.shape[2]
        a.W, a.H, a.Ws, a.Hs = gi.width, gi.height, gi.src_width, gi.src_height
        a.tiles_x, a.tiles_y = gi.tiles_x, gi.tiles_y
        if gi.resample:
            work = gi.tiles_x * gi.tiles_y * gi.channels
        elif _is_blk(plan, g):
            work = gi.nwaves // gi.waves_per_group  # one workgroup per tile
        else:
            work = gi.nwaves
        a.nwaves = gi.nwaves
        start[k] = total
        total += work
    start[nimg] = total
    return arr, start, total, resample, wpb, gi


def _batch_inputs(spec, images, plan_kw, names, ch):
    plans, bufs_all = [], []
    for inputs in images:
        first = inputs[spec["inputs"][0]["name"]]
        h, w = first.shape[-2:]
        if not plans:
            plans.append(wt.from_spec(spec).plan(w, h, no_device=True, **plan_kw))
        else:  # a batch shares one schedule: replay the first plan's
            kw = dict(plan_kw, mode="fixed", fixed=plans[0].describe())
            plans.append(wt.from_spec(spec).plan(w, h, no_device=True, **kw))
        bufs = {}
        for i, inp in enumerate(spec["inputs"]):
            t = SPEC_NP[inp.get("dtype", "f32")]
            bufs[i] = np.ascontiguousarray(inputs[inp["name"]]).astype(t).reshape(ch[inp["name"]], h, w)
        bufs_all.append((w, h, bufs))
    return plans, bufs_all


class Whole(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("AB", "start", "chunks", "deps", "done", "next", "status")] + \
               [("limit", ctypes.c_int64), ("nchunks", ctypes.c_int32), ("nimg", ctypes.c_int32)]


WHOLE_RUNNER = r"""
extern "C" int wt_emu_run_whole(const WtWhole* p, int nwaves) {
    std::barrier<> bar(64);
    wt_emu_bar = &bar;
    std::vector<std::thread> th;
    for (int l = 0; l < 64; ++l)
        th.emplace_back([&, l] {
            wt_emu_lane = l;
            for (int w = 0; w < nwaves; ++w) {
                blockIdx.x = w; threadIdx.x = l; gridDim.x = nwaves;
                bar.arrive_and_wait();
                WT_EMU_KERNEL(*p);
                bar.arrive_and_wait();
            }
        });
    for (auto& t : th) t.join();
    return 0;
}
// `nwaves` waves at once, 64 lane threads each with the wave's own barrier
// and exchange buffer; wave w uses LDS slot w (the kernel's LDS array is
// widened to 16 slots for this runner).
extern "C" int wt_emu_run_whole_concurrent(const WtWhole* p, int nwaves) {
    std::vector<std::barrier<>*> bars;
    std::vector<std::vector<uint32_t>> xs(nwaves, std::vector<uint32_t>(64));
    for (int w = 0; w < nwaves; ++w) bars.push_back(new std::barrier<>(64));
    std::vector<std::thread> th;
    for (int w = 0; w < nwaves; ++w)
        for (int l = 0; l < 64; ++l)
            th.emplace_back([&, w, l] {
                wt_emu_lane = l;
                wt_emu_wave_bar = bars[w];
                wt_emu_wave_x = xs[w].data();
                blockIdx.x = 0; threadIdx.x = w * 64 + l; gridDim.x = 1;
                WT_EMU_KERNEL(*p);
            });
    for (auto& t : th) t.join();
    for (auto* b : bars) delete b;
    return 0;
}
"""


def emulate_whole(spec, images, chunk=3, concurrent=0, limit_s=60, resident_waves=None, **plan_kw):
    """Runs a batch through the whole-pipeline kernel (every group in one
    launch, chunks of `chunk` tiles handed out by the ticket counter) on the
    CPU.  By default one wave at a time: the first wave takes every chunk in
    ticket order, so each wait finds its producers complete.  With
    `concurrent` = n, n waves run at once and take chunks as they free up,
    so waits on producers still in progress really block.  Returns one
    output dict per image, the final counters (done per group and image,
    the ticket, the status word) and the producer masks.  With
    `resident_waves`, the chunk table and producer masks are the library's
    own (wt_plan_whole_tables for that many resident waves), checked here
    against the masks and per-image tile counts derived from the plans."""
    names, lv, ch = _meta(spec)
    hists = {st["name"]: st for st in spec["stages"] if st["kind"] == "hist"}
    plans, bufs_all = _batch_inputs(spec, images, plan_kw, names, ch)
    nimg, ngroups = len(images), plans[0].num_groups
    ab = (Args * (ngroups * nimg))()
    starts = (ctypes.c_int * (ngroups * (nimg + 1)))()
    chunks, deps, liveouts = [], [], []
    for g in range(ngroups):
        arr, start, total, resample, wpb, gi = _group_tables(plans, bufs_all, g, names, lv, ch, hists)
        for k in range(nimg):
            ctypes.memmove(ctypes.addressof(ab) + (g * nimg + k) * ctypes.sizeof(Args), ctypes.addressof(arr[k]),
                           ctypes.sizeof(Args))
            starts[g * (nimg + 1) + k] = start[k]
        starts[g * (nimg + 1) + nimg] = start[nimg]
        loaded = set(gi.loaded[:gi.nloaded])
        deps.append(sum(1 << q for q in range(g) if loaded & liveouts[q]))
        liveouts.append(set(gi.liveouts[:gi.nliveouts]))
        for k in range(nimg):
            n = start[k + 1] - start[k]
            chunks += [(g, k, t, min(chunk, n - t)) for t in range(0, n, chunk)]
    if resident_waves:
        sizes = [(w, h) for (w, h, _) in bufs_all]
        tab, lib_deps = plans[0].whole_tables(sizes, resident_waves)
        assert lib_deps == deps, (lib_deps, deps)
        for g in range(ngroups):
            for k in range(nimg):
                rows = tab[(tab[:, 0] == g) & (tab[:, 1] == k)]
                n = starts[g * (nimg + 1) + k + 1] - starts[g * (nimg + 1) + k]
                assert rows[:, 3].sum() == n and (len(rows) == 0 or rows[0, 2] == 0), (g, k)
                assert np.array_equal(rows[1:, 2], (rows[:, 2] + rows[:, 3])[:-1]), (g, k)  # contiguous
        assert np.all(np.diff(tab[:, 0]) >= 0)  # group by group
        chunks = [tuple(r) for r in tab.tolist()]
    src = plans[0].source(-1)
    kname = src[src.index("void __launch_bounds__"):].split("(")[1].split(")")[1].strip()
    if concurrent:  # one LDS slot per emulated wave
        import re
        src = re.sub(r"char wt_lds\[(\d+)\];", lambda m: f"char wt_lds[{int(m.group(1)) * 16}];", src)
        assert concurrent <= 16
    os.makedirs(CACHE, exist_ok=True)
    text = '#include "wt_emu.h"\n' + src + f"\n#define WT_EMU_KERNEL {kname}\n" + WHOLE_RUNNER
    h = _text_hash(text)
    so = os.path.join(CACHE, f"{kname}_{h}.so")
    if not os.path.exists(so):
        cpp = so[:-3] + ".cpp"
        open(cpp, "w").write(text)
        subprocess.run([CLANG, "-std=c++20", "-O1", "-shared", "-fPIC", "-pthread", "-w",
                        f"-I{os.path.join(HERE, 'emu')}", cpp, "-o", so + ".tmp"], check=True)
        os.replace(so + ".tmp", so)
    lib = ctypes.CDLL(so)
    lib.wt_emu_run_whole.argtypes = [ctypes.POINTER(Whole), ctypes.c_int]
    lib.wt_emu_run_whole_concurrent.argtypes = [ctypes.POINTER(Whole), ctypes.c_int]
    ctab = np.ascontiguousarray(np.array(chunks, dtype=np.int32).reshape(-1, 4))
    dtab = np.array(deps, dtype=np.uint64)
    ctr = np.zeros(ngroups * nimg + 2, dtype=np.int32)
    wh = Whole(ctypes.addressof(ab), ctypes.addressof(starts), ctab.ctypes.data, dtab.ctypes.data,
               ctr.ctypes.data, ctr[ngroups * nimg:].ctypes.data, ctr[ngroups * nimg + 1:].ctypes.data,
               int(limit_s * 10 ** 8), len(chunks), nimg)
    if concurrent:
        lib.wt_emu_run_whole_concurrent(ctypes.byref(wh), concurrent)
    else:
        lib.wt_emu_run_whole(ctypes.byref(wh), 2)
    outs = [{o: _result(b[names.index(o)]) for o in spec["outputs"]} for (_, _, b) in bufs_all]
    emulate_whole.buffers = bufs_all  # every image's node buffers, for diagnosis
    return outs, ctr, deps
