/*
 * wavetile -- fused wave-tiled stencil pipelines for MI355X (gfx950).
 *
 * C ABI of the library.  No C++ types cross this boundary; every call returns
 * a wt_status and, on failure, leaves a message retrievable with
 * wt_last_error() (thread-local, valid until the next failing call on the
 * same thread).  No call throws.
 *
 * The operation (the paper, Sections 2.2-2.3 and Fig. 2): an image-processing
 * pipeline is a DAG of stages; each stage is a function over an integer
 * domain whose value at a point is an expression of producer values at
 * constant offsets (dependence vectors).  The library evaluates the pipeline
 * by fusing stages into groups executed as overlapped tiles, one tile per
 * 64-lane wavefront (Section 4), storing each tile partly in VGPRs and partly
 * in LDS (hybrid tiling, Section 5 and Algorithm 1), with fusion and tile
 * sizes chosen by a cost model (Section 6 and Algorithm 2).
 *
 * Boundary reading used throughout (the paper uses interior-only domains):
 * every stage's domain is its full image size, and a producer read outside
 * the producer's domain takes the value at the nearest domain point (clamp
 * to edge, applied per stage).
 *
 * Images are planar (channel-major), row-major, with strides in ELEMENTS.
 * Pixel buffers are device memory owned by the caller; the library never
 * frees or retains them beyond a call.
 */
#ifndef WAVETILE_WT_H
#define WAVETILE_WT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    WT_OK = 0,
    WT_E_INVALID = -1,     /* bad argument or malformed pipeline             */
    WT_E_UNSUPPORTED = -2, /* valid request the library does not handle      */
    WT_E_SHAPE = -3,       /* image size / channels / alignment mismatch     */
    WT_E_NOMEM = -4,       /* device or host allocation failed               */
    WT_E_COMPILE = -5,     /* run-time compilation of a kernel failed        */
    WT_E_HIP = -6,         /* a HIP runtime call failed (incl. async faults) */
    WT_E_INTERNAL = -7
} wt_status;

/* Element types.  WT_F32 images feed float stages; the integer types carry
 * integer stages (exact integer arithmetic, saturated to the type's range).
 * WT_F16 describes FP16 intermediates only (never a caller image). */
typedef enum { WT_F32 = 0, WT_F16 = 1, WT_U8 = 2, WT_U16 = 3, WT_I16 = 4, WT_I32 = 5 } wt_dtype;

typedef enum { WT_DOWN2 = 0, WT_UP2 = 1 } wt_resample_kind;

typedef struct {
    void* data;          /* device pointer to channel 0, row 0, column 0        */
    int32_t width;
    int32_t height;
    int32_t channels;
    int32_t dtype;       /* wt_dtype                                            */
    int64_t row_stride;  /* elements between rows; 0 means width                */
    int64_t chan_stride; /* elements between channel planes; 0 = height*row_stride */
} wt_image;

typedef struct wt_pipeline wt_pipeline; /* opaque */
typedef struct wt_plan wt_plan;         /* opaque */

/* ---------------------------------------------------------------------- */
/* Pipeline construction.  Node ids are dense, in creation order; inputs and  */
/* stages share one id space.  A pipeline is immutable once a plan uses it.   */
/* ---------------------------------------------------------------------- */

wt_status wt_pipeline_create(wt_pipeline** out);
void wt_pipeline_destroy(wt_pipeline* p);

/* An input image with `channels` planes (WT_F32 elements). */
wt_status wt_input(wt_pipeline* p, int channels, int* id);

/* Declares |value| <= max_abs for every element of float input `id` (the
 * default is 1).  The builders propagate these magnitude bounds through
 * every stage (sum of |weights| times the source's bound for stencils,
 * interval arithmetic on expressions), and FP16 intermediates are used only
 * for stages whose bound fits FP16's finite range (|v| <= 65504): other
 * stages keep FP32 storage.  Must be called before any stage reads `id`
 * (WT_E_INVALID otherwise, and for integer inputs or a bound that is not
 * positive and finite). */
wt_status wt_input_bound(wt_pipeline* p, int id, double max_abs);

/* An input image of element type `dtype` (WT_F32, WT_U8, WT_U16, WT_I16 or
 * WT_I32).  Integer inputs make integer stages possible downstream; float
 * stages reading them see the values converted to FP32. */
wt_status wt_input_typed(wt_pipeline* p, int channels, int dtype, int* id);

/* Stencil stage, per channel (the paper's Stencil / Correlate stages, Fig. 2):
 *   S_c(x,y) = scale * sum_{j<kh, i<kw} weights[j*kw+i] * P_c(x+i-ax, y+j-ay)
 * with clamp-to-edge producer reads.  `weights` (kh*kw values, row-major) is
 * copied.  Kernel sides 1..15. */
wt_status wt_stencil(wt_pipeline* p, int src, int kw, int kh, int ax, int ay,
                     const double* weights, double scale, int* id);

/* Integer stencil stage of type `out` (WT_U8, WT_U16, WT_I16, WT_I32) on an
 * integer source, per channel:
 *   acc = sum_{j<kh, i<kw} weights[j*kw+i] * P_c(x+i-ax, y+j-ay)   (exact)
 *   S_c(x,y) = saturate_out(floor((acc + floor(divisor/2)) / divisor))
 * i.e. division rounding halves up (for divisor 2^s: (acc + 2^(s-1)) >> s).
 * Clamp-to-edge reads as for wt_stencil.  |weights| <= 32767,
 * 1 <= divisor <= 2^24; a pipeline whose sums could leave the 32-bit range
 * is refused with WT_E_UNSUPPORTED (GPU arithmetic is 32-bit and exact). */
wt_status wt_stencil_int(wt_pipeline* p, int src, int kw, int kh, int ax, int ay,
                         const int32_t* weights, int32_t divisor, int out, int* id);

/* Pointwise stage (the paper's Function with a Case expression, Fig. 2).
 * `expr` is infix over s0..s{nsrc-1} (source i at the same channel; a
 * one-channel source broadcasts) and s<i>[k] (channel k of source i), with
 * numbers, unary -, + - * /, one comparison (< <= > >=) inside
 * select(cond, a, b), and abs, min, max, sqrt, floor.  All sources must lie
 * on the same pyramid level.  Output has `out_channels` planes. */
wt_status wt_pointwise(wt_pipeline* p, const int* srcs, int nsrc,
                       const char* expr, int out_channels, int* id);

/* Pointwise stage of element type `out`.  WT_F32 is wt_pointwise.  An
 * integer `out` needs integer sources and an integer expression (integer
 * constants; no /, sqrt or floor), evaluated exactly and saturated to the
 * type's range; expressions whose intermediate values could leave the
 * 32-bit range are refused with WT_E_UNSUPPORTED. */
wt_status wt_pointwise_typed(wt_pipeline* p, const int* srcs, int nsrc, const char* expr,
                             int out_channels, int out, int* id);

/* 2x resampling (scaled dependences, Section 5's alignment and scaling);
 * the result has the source's element type (WT_UP2 of an integer stage is
 * refused: the expansion would need a rounding rule):
 *   WT_DOWN2: D(x,y) = P(2x,2y), domain ceil(W/2) x ceil(H/2);
 *   WT_UP2:   separable binomial expansion, even 2i -> (P(i-1)+6P(i)+P(i+1))/8,
 *             odd 2i+1 -> (P(i)+P(i+1))/2, to the next finer level's domain. */
wt_status wt_resample(wt_pipeline* p, int src, int kind, int* id);

/* Histogram of a stage (a reduction; the paper's Section 7 names such
 * scatter/reduction stages, as in the bilateral grid, as what its fusion
 * does not cover).  Per channel, `bins` int32 counts: a value v of `src`
 * (converted to FP32) falls in bin floor((v - lo) * (bins / (hi - lo))),
 * computed in FP32 and clamped to 0..bins-1 (values outside [lo, hi) count
 * in the end bins; NaN counts in bin 0).  Its image is bins x 1 (WT_I32,
 * the source's channels) and must be a pipeline output or read by
 * wt_equalize stages; no other stage may read it.  A group that computes `src` accumulates the histogram as it goes, so
 * `src` itself need not be stored; with FP16 intermediates the value
 * counted is the FP16-rounded one the plan keeps.  The plan clears the
 * counts before accumulating (every run starts from zero).  bins in
 * 1..4096, lo < hi, both finite; WT_E_INVALID otherwise. */
wt_status wt_histogram(wt_pipeline* p, int src, int bins, double lo, double hi, int* id);

/* Histogram equalisation, a stage that reads a reduction: per channel, the
 * value v of `src` maps to C(b) / N, where b is v's bin in histogram `hist`
 * (the bin rule of wt_histogram, with hist's bins, lo and hi), C(b) the
 * count of bins 0..b and N the total count; C(b) converted to FP32 times
 * 1/N rounded to FP32 (0 when N = 0).  `hist` must count a stage with
 * src's channels; it is computed by an earlier kernel than the one that
 * reads it (the counts must be complete), and its counts need not be an
 * output.  The result is FP32 in [0, 1] at src's level.  WT_E_INVALID for a
 * `hist` that is not a histogram or a channel mismatch. */
wt_status wt_equalize(wt_pipeline* p, int src, int hist, int* id);

/* Marks a node as a pipeline output (outputs are numbered in call order). */
wt_status wt_output(wt_pipeline* p, int id);

/* ---------------------------------------------------------------------- */
/* Planning                                                                  */
/* ---------------------------------------------------------------------- */

typedef enum {
    WT_SCHED_UNFUSED = 0,  /* one kernel per stage, intermediates in HBM      */
    WT_SCHED_ANALYTIC = 1, /* DP fusion with the analytical cost (Alg. 2)      */
    WT_SCHED_MLP = 2,      /* DP fusion ranked by the learned cost model       */
    WT_SCHED_AUTOTUNE = 3, /* top-k candidates (analytic or learned), measured */
    WT_SCHED_FIXED = 4     /* schedule text in `fixed_schedule`                */
} wt_sched_mode;

enum {
    WT_PLAN_NO_DEVICE = 1, /* generate and compile code only; run() refused   */
    WT_PLAN_ANY_WIDTH = 2, /* caller images of 8- or 16-bit integer
                              elements may have any width and stride: groups
                              touching them use one element per lane (32-bit
                              elements allow any width and stride in every
                              plan) */
    WT_PLAN_NO_COMPILE = 4, /* schedule and generate code only (implies
                               WT_PLAN_NO_DEVICE); wt_plan_source still works */
    WT_PLAN_RETUNE = 8,     /* WT_SCHED_AUTOTUNE: measure again even when the
                               schedule cache holds a result (and replace it) */
    WT_PLAN_BATCH_RESIDENT = 16, /* wt_plan_run_batch launches only the
                               workgroups resident at once, each looping over
                               its share of the work units (persistent); by
                               default every work unit gets a workgroup */
    WT_PLAN_NO_FOLD = 32,   /* the fusion search keeps every up2 out of the
                               groups (read by expansion in its consumers'
                               groups) instead of folding an up2 of a
                               decimated stage into that stage's group */
    WT_PLAN_BATCH_WHOLE = 64 /* wt_plan_run_batch runs the whole group
                               sequence as one persistent launch (see
                               wt_plan_run_batch) */
};

/* WT_SCHED_AUTOTUNE results are cached, keyed by the device architecture,
 * a hash of the pipeline's definition, the size bucket (width and height in
 * units of 256, and width mod 4), the FP16 and any-width choices, the
 * candidate count and the model path: in process memory and, when a cache
 * directory is set, as lines of <cache_dir>/autotune.tsv ("key<TAB>schedule
 * text"), read on first use.  A hit builds the cached schedule without
 * measuring anything. */

typedef struct {
    int32_t mode;               /* wt_sched_mode                               */
    int32_t fp16_intermediates; /* store fused/materialised intermediates FP16
                                   (stages whose magnitude bound exceeds
                                   65504 keep FP32; see wt_input_bound)     */
    int32_t flags;              /* WT_PLAN_* bits                              */
    int32_t autotune_topk;      /* candidates measured in WT_SCHED_AUTOTUNE per
                                   ranking (0: 4)                             */
    const char* fixed_schedule; /* WT_SCHED_FIXED (see wt_plan_describe)       */
    const char* model_path;     /* WT_SCHED_MLP weights file; with WT_SCHED_
                                   AUTOTUNE, the learned model ranks candidates */
    const char* cache_dir;      /* code-object cache; NULL = $WT_CACHE_DIR or none */
    int32_t batch_images;       /* images per batched run (0 or 1: single): the
                                   analytical cost counts waves and traffic of
                                   that many images of this size, so tile
                                   shapes suit the batched launch;
                                   WT_SCHED_AUTOTUNE times its candidates on
                                   an image as tall as up to that many (its
                                   buffers within 4 GiB of scratch) */
} wt_sched_opts;

/* Plans `p` for width x height inputs (the paper, Section 6 and Fig. 6): the
 * fusion of stages into groups (DP-Fusion driven by the GPU cost function),
 * per group the argmin of Algorithm 2 over tile sizes, workgroup size,
 * register fraction and transaction size (or the learned model's, or the
 * autotuner's measured choice), then code generation (Section 4's one
 * overlapped tile per wavefront, Section 5's hybrid VGPR/LDS tiling,
 * Algorithm 1) and compilation for the current device.  `opts` may be NULL
 * (analytic mode, FP32).  Measurements made while planning (Section 6's
 * pre-profiling, WT_SCHED_AUTOTUNE's timings) run on `hip_stream` (a
 * hipStream_t) when it is not NULL, else on a stream the library creates and
 * destroys; the call returns when they are done.  Allocates device buffers
 * for intermediates materialised between groups; *out is owned by the
 * caller (wt_plan_destroy).  WT_E_SHAPE for sizes outside 1..2^24,
 * WT_E_INVALID for a malformed schedule text, WT_E_UNSUPPORTED when no
 * feasible schedule exists, WT_E_COMPILE / WT_E_HIP on device failures. */
wt_status wt_plan_create(const wt_pipeline* p, const wt_sched_opts* opts,
                         int width, int height, void* hip_stream, wt_plan** out);

/* Runs the plan asynchronously on `hip_stream` (a hipStream_t; NULL = the
 * default stream): one launch per group, in the order the fusion search
 * chose.  The outputs equal the plain stage-by-stage evaluation of the
 * pipeline up to floating-point rounding (Section 2.2: overlapped tiles
 * recompute their halos and change no values).  in[i] is input i (creation
 * order), out[i] output i, device buffers owned by the caller; sizes must
 * equal the planned ones (WT_E_SHAPE otherwise, and for a channel count,
 * element type or stride the node does not allow).  Outputs must not alias
 * any other image (WT_E_INVALID).  Kernel faults surface at the caller's
 * next synchronisation. */
wt_status wt_plan_run(wt_plan* plan, const wt_image* in, int nin,
                      const wt_image* out, int nout, void* hip_stream);

/* Runs the plan over a batch of `nimg` image sets of possibly different
 * sizes (the paper runs one image per launch sequence, Section 7; batching
 * is this library's addition, each image's result being the one
 * wt_plan_run computes): in[i*nin + k] is input k of image i,
 * out[i*nout + k] output k; the image checks of wt_plan_run apply to every
 * image, and no output may alias any image of the batch.
 * Every group runs as one launch over the tiles of all images (one
 * workgroup per work unit; with WT_PLAN_BATCH_RESIDENT or the environment
 * variable WT_BATCH_GRID=resident, only the workgroups that fit on the
 * device at once, each looping over its share); the group sequence is
 * captured in a
 * hipGraph on the first run of a batch shape (the list of sizes) and
 * replayed while the shape is unchanged (only image pointers may change).
 * Intermediates live in a plan-owned arena sized for the shape.  Images of
 * 8- or 16-bit integer elements must satisfy the plan's vector-width
 * alignment (plan with WT_PLAN_ANY_WIDTH for arbitrary widths).
 * With WT_PLAN_BATCH_WHOLE the graph holds a single persistent launch of one
 * kernel that contains every group (the paper's fusion taken across the
 * groups a kernel boundary would separate, Sections 4 and 5, with the
 * ordering of the kernel boundaries kept by device-side counters): waves take
 * chunks of consecutive tiles of one group and one image in group order
 * from an atomic ticket and start a chunk once every producer group has
 * finished that image.  Plans whose groups are all wave-tiled fused groups
 * only (WT_E_UNSUPPORTED for lone resampling, histogram, equalize or
 * one-tile-per-workgroup groups, and beyond 64 groups); outputs equal the
 * per-group launches' bit for bit (on the host's lane emulation).  Every
 * wait is bounded (two seconds); wt_plan_batch_check reports a launch that
 * gave up.  Switched off for now: with WT_PLAN_BATCH_WHOLE this call
 * returns WT_E_UNSUPPORTED before any launch (its first device run did not
 * complete and the cause is not yet known); wt_plan_source(plan, -1, ...)
 * still returns the kernel.
 * Asynchronous on `hip_stream`. */
wt_status wt_plan_run_batch(wt_plan* plan, int nimg, const wt_image* in,
                            const wt_image* out, void* hip_stream);

/* Synchronises `hip_stream` and returns WT_E_INTERNAL if a wave of the
 * plan's last whole-pipeline batch launch (WT_PLAN_BATCH_WHOLE) gave up
 * waiting for a producer group (its outputs are then not valid); WT_OK
 * otherwise, and for plans without such a launch.  A library addition: the
 * paper launches one kernel per fused group (Section 7), where the kernel
 * boundary itself orders producers before consumers; this call reports
 * whether the device-side ordering that replaces those boundaries held. */
wt_status wt_plan_batch_check(wt_plan* plan, void* hip_stream);

/* Bytes of device memory in the library's fixed workspace: one copy on each
 * GPU that wt_plan_run_batch_static runs on, held until the process ends. */
#define WT_STATIC_SCRATCH_BYTES (256u * 1024u * 1024u)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * batch of wt_plan_run_batch, same arguments, same kernels and launch
 * grids and bit-identical outputs, with every intermediate and the
 * per-image argument table in the library's fixed workspace
 * (WT_STATIC_SCRATCH_BYTES) instead of plan-owned device memory.  Calls no
 * device allocator and captures no graph: every group is launched directly
 * on `hip_stream`, after an asynchronous copy of the argument table from
 * host memory the plan owns (reused by the plan's next call).  Every call
 * on one GPU, from any plan, shares that GPU's workspace: calls that
 * overlap on one GPU (different streams, or threads) race, while calls in
 * order on one stream are safe (nothing in the workspace needs to start
 * at zero: each group writes the intermediates it produces before any
 * later group reads them).  Needs the plan's batched kernels loaded
 * (planned with batch_images > 1, or after a wt_plan_run_batch) and the
 * plan's device current (WT_E_INVALID otherwise); WT_E_NOMEM, before any
 * launch, when the batch's intermediates and table exceed the workspace;
 * the image checks of wt_plan_run_batch apply. */
wt_status wt_plan_run_batch_static(wt_plan* plan, int nimg, const wt_image* in,
                                   const wt_image* out, void* hip_stream);

/* Runs only groups first .. first+count-1 of the batched plan over the same
 * arguments as wt_plan_run_batch, with the same kernels and launch grids,
 * launched directly on `hip_stream` (not from the graph), in group order.
 * The groups read the intermediates their producer groups wrote in the
 * batch's arena by the last run of the same batch shape, so a complete
 * wt_plan_run_batch must precede it for results to be meaningful.  Meant for
 * per-kernel measurement (timing one group's launch with events) and for
 * callers interleaving other work between groups.  WT_E_INVALID for a
 * range outside 0 .. wt_plan_num_groups(plan); the image checks of
 * wt_plan_run_batch apply. */
wt_status wt_plan_run_batch_groups(wt_plan* plan, int first, int count, int nimg, const wt_image* in,
                                   const wt_image* out, void* hip_stream);

/* The plan's schedule (the paper's fusion groups, Section 6, and each
 * group's tile configuration, Algorithm 2's arguments) as text: one line per
 * group,
 *   "g<i> nodes=<id,id,...> V=<v> TX=<t> SX=<s> TY=<rows> WPB=<w> PF=<p>
 *    fp16=<0|1> align=<0|1> XCD=<0|1> NT=<0|1> [ORD=1] [BLK=1] [GH=1]
 *    [dec=<id,...>] [exp=<id,...>]"
 * V: columns per lane (1, 2, 4); TX: sub-tiles of 64*V columns, the first
 * SX in LDS; TY: output rows per wave tile; WPB: waves per workgroup; PF:
 * rows loaded ahead; align=1: the paper's right-hyperplane skew; XCD=1:
 * adjacent tiles on one XCD; NT: nontemporal memory access; ORD=1: tiles
 * ordered along x; BLK=1: one tile per workgroup with barriers between
 * stages (the paper's baseline); GH=1: loaded rows carry ghost columns;
 * dec: down2 stages written decimated by this group; exp: up2 stages read
 * by expansion.  Batched plans append batch_* launch figures.
 * The same text (lines or ';'-separated) is accepted by WT_SCHED_FIXED;
 * omitted keys take their defaults.
 * Writes at most `len` bytes including the terminator; *needed gets the full
 * size. */
wt_status wt_plan_describe(const wt_plan* plan, char* buf, size_t len, size_t* needed);

/* Tunes a plan on a batch itself (the autotuner's measurement, Section 6's
 * protocol, on the caller's images instead of a proxy image): runs the
 * batch once, then for every group times its configuration and each
 * neighbouring one (V, TX, TY, WPB, PF one step away) as batched kernels
 * over these images, for up to four rounds, keeps the fastest, rebuilds the
 * plan and runs the batch again, so `out` holds the pipeline's result.  The
 * result is cached (in memory and in the plan's cache directory) per
 * device, starting schedule and image sizes, and reused without timing.
 * Arguments and errors as wt_plan_run_batch; it allocates a small table
 * and compiles candidates (seconds). */
wt_status wt_plan_tune_batch(wt_plan* plan, int nimg, const wt_image* in, const wt_image* out, void* stream);

/* Test hook of WT_PLAN_BATCH_WHOLE's host logic (any plan, no device
 * needed): for a batch of `nimg` images of sizes wh[2i] x wh[2i+1] and
 * `resident_waves` waves resident at once, the chunk table the launch would
 * hand out, 4 ints per chunk (group, image, first tile, tiles; group by
 * group, images in order; a group's chunk holds about 1/(8 resident_waves)
 * of its tiles, 1 to 64) into `chunks` (NULL: count only; WT_E_INVALID if
 * more than `max_chunks`), their number into `nchunks`, and into `deps` (NULL,
 * or one entry per group) each group's producer groups as a bit mask.
 * WT_E_UNSUPPORTED as the launch itself refuses; WT_E_SHAPE for sizes
 * outside 1..2^24. */
wt_status wt_plan_whole_tables(const wt_plan* plan, int nimg, const int* wh, int resident_waves, int* chunks,
                               int max_chunks, int* nchunks, unsigned long long* deps);

/* HIP source generated for group `group`; group -1: the whole-pipeline
 * kernel of WT_PLAN_BATCH_WHOLE (generated on each call, for any plan;
 * WT_E_UNSUPPORTED where that launch is refused). */
wt_status wt_plan_source(const wt_plan* plan, int group, char* buf, size_t len,
                         size_t* needed);

/* Number of kernel launches per run. */
int wt_plan_num_groups(const wt_plan* plan);

/* Launch description of group `group`, for tools and tests that execute
 * the generated source themselves (e.g. a host emulator).  Buffers follow
 * the group's loaded/live-out order; *_half flags mark FP16 buffers and
 * *_dtype give every buffer's element type. */
typedef struct {
    int32_t resample;         /* 1: 2x resampling kernel (grid tiles_x x tiles_y x channels, 256 threads) */
    int32_t waves_per_group;  /* fused kernels: waves per workgroup                                  */
    int32_t nwaves;           /* fused kernels: wave tiles in the launch                             */
    int32_t tiles_x, tiles_y;
    int32_t width, height;    /* domain of the group's stages                                        */
    int32_t src_width, src_height; /* resampling: source domain                                      */
    int32_t channels;         /* resampling: channel planes                                          */
    int32_t nloaded, nliveouts;
    int32_t loaded[16], liveouts[16];
    int32_t loaded_half[16], liveout_half[16];
    int32_t loaded_dtype[16], liveout_dtype[16]; /* wt_dtype of each buffer  */
} wt_group_info;
wt_status wt_plan_group_info(const wt_plan* plan, int group, wt_group_info* out);

/* Test hook for the fusion search (Section 6, DP-Fusion with Algorithm 2):
 * minimum total predicted time (microseconds, gfx950 machine model) found by
 * the dynamic program, and by exhaustive enumeration of every partition into
 * ready, connected, single-level groups of at most `max_group` stages under
 * the same group costs (+inf when the pipeline has more than 10 stages). */
wt_status wt_fusion_costs(const wt_pipeline* p, int width, int height, int fp16, int max_group,
                          double* dp_us, double* exhaustive_us);

/* Test hooks for the model's formulas (Section 4, Algorithm 2, Table 1).
 * wt_alg2_eval evaluates Algorithm 2 for one configuration given the
 * quantities it reads, on machine table `machine` (0: gfx950, 1: GTX 1080Ti),
 * with weights w[7] (NULL: Table 3's V100 row).
 *   in[9]  = {scratchpad bytes per block, registers per thread, warps per
 *             block, blocks, transactions, compulsory transactions, bytes per
 *             warp, compute seconds per warp, redundant / useful points}
 *   out[12] = {feasible, score, occupancy, scratchpad-limited warps per SM,
 *              register-limited warps per SM, terms[0..6]}
 * wt_otpw_geometry gives Section 4's warp sizes for block[3] and warp size
 * `ws`, and the scratchpad elements of one block for tile[3] and overlap[3]:
 * prod_i ceil(block_i / warp_i) * (tile_i * warp_i + overlap_i). */
wt_status wt_alg2_eval(int machine, const double* in, const double* w, double* out);

/* Achievable-bandwidth reference (not a pipeline operation): copies `bytes`
 * bytes from `src` to `dst`, both device pointers owned by the caller,
 * 16-byte aligned and not overlapping, asynchronously on `stream` (a
 * hipStream_t; NULL = the null stream), one 16-byte element per thread with
 * nontemporal loads and stores.  WT_E_INVALID for null or misaligned
 * pointers or overlapping ranges; WT_E_HIP when the launch fails. */
wt_status wt_stream_copy(const void* src, void* dst, size_t bytes, void* stream);
wt_status wt_otpw_geometry(const int* block, int ws, const int* tile, const int* overlap, int* warp,
                           int64_t* scratch_elems);

/* ---------------------------------------------------------------------- */
/* Learned cost model: a fully connected ReLU network over the 40 model      */
/* features of a (group, configuration), predicting log kernel time; trained */
/* on the device (forward, backward, MSE and Adam kernels).  Host pointers;  */
/* the library copies to and from the device.  Parameters are laid out layer */
/* by layer: W_l (dims[l] x dims[l+1], row-major) then b_l.                  */
/* ---------------------------------------------------------------------- */
typedef struct wt_mlp wt_mlp;
wt_status wt_mlp_create(const int* dims, int nlayers, uint64_t seed, wt_mlp** out);
void wt_mlp_destroy(wt_mlp* m);
size_t wt_mlp_num_params(const wt_mlp* m);
wt_status wt_mlp_get_params(const wt_mlp* m, float* params, size_t n);
wt_status wt_mlp_set_params(wt_mlp* m, const float* params, size_t n);
/* Raw network output for `batch` rows of x (no normalisation). */
wt_status wt_mlp_forward(wt_mlp* m, const float* x, int batch, float* y);
/* MSE of the raw output against t and its gradient w.r.t. every parameter. */
wt_status wt_mlp_forward_backward(wt_mlp* m, const float* x, const float* t, int batch,
                                  float* loss, float* grads);
/* One Adam step (lr, beta1 0.9, beta2 0.999, eps 1e-8) with given gradients. */
wt_status wt_mlp_adam_step(wt_mlp* m, const float* grads, float lr);
/* Trains on n samples (features z-scored and target standardised on this
 * set, stored in the model); returns the last epoch's mean loss. */
wt_status wt_mlp_train(wt_mlp* m, const float* x, const float* t, int n, int epochs, int batch,
                       float lr, uint64_t seed, float* final_loss);
/* Trains the learned cost model from a measurement database and saves it
 * (the network this library adds to the paper's analytical model of
 * Section 6, used by WT_SCHED_MLP and to rank WT_SCHED_AUTOTUNE's
 * candidates).  `measure_db` is a JSON-lines file as wt_measure_groups and
 * the autotuner append (WT_MEASURE_DB): per line a configuration, its
 * measured_us, the analytical model's pred_us and terms, and its 40
 * features.  Usable lines (positive finite time, all quantities finite) are
 * the training set: the target is log(measured_us), features and target
 * are standardised on it, and a 40-128-128-128-1 ReLU network is trained
 * for 200 epochs of Adam (batch 256, lr 1e-3, seed 1) on the device with the
 * library's kernels, on `hip_stream` (a hipStream_t; NULL: a stream of the
 * model's own).  Held-out evaluation is the caller's: pass a file holding
 * the training pipelines' lines only.  Synchronous.  The model is written
 * to `out_model` (wt_mlp_save's format).  WT_E_INVALID for an unreadable
 * file, a line without measured_us or fewer than two usable lines. */
wt_status wt_model_train(const char* measure_db, const char* out_model, void* hip_stream);
/* Number of usable lines (as wt_model_train counts them) in a measurement
 * database; reads the file only. */
wt_status wt_model_rows(const char* measure_db, int* rows);
/* Prediction in target units for n feature rows (stored normalisation). */
wt_status wt_mlp_predict(wt_mlp* m, const float* x, int n, float* y);
wt_status wt_mlp_save(const wt_mlp* m, const char* path);
wt_status wt_mlp_load(const char* path, wt_mlp** out);
/* Features of every configuration the search grid holds for `nodes` of a
 * pipeline planned at width x height (row-major, 40 per configuration), with
 * each configuration's schedule text (';'-separated) -- the learned model's
 * inputs as the scheduler sees them.  down2 stages among `nodes` are written
 * decimated by the group (the source must be a member), and an up2 of such
 * a down2 is folded into it. */
wt_status wt_group_features(const wt_pipeline* p, const int* nodes, int nnodes, int width, int height,
                            int fp16, float* features, int max_rows, int* rows, char* text,
                            size_t text_len);

/* Measures candidate groups of a pipeline on the current device, for the
 * learned model's training data (the paper times whole schedules; this times
 * single groups).  groups[i] is one group's schedule text ("nodes=... V=...
 * TX=... SX=... TY=... WPB=... PF=...", as in wt_plan_describe), timed on
 * zero-filled scratch images of every node at width x height: 3 samples of
 * `reps` back-to-back launches, minimum of the sample means, in
 * microseconds, into times_us[i] (host array of n doubles; +inf when the
 * group cannot be built for this pipeline).  When $WT_MEASURE_DB names a
 * file, one JSON line per fused group is appended (tagged `tag`) with its
 * 40 model features.  Synchronous; allocates and frees its scratch.
 * reps == 0 compiles the groups into the code cache only (no device is
 * touched; times_us[i] = 0 for buildable groups). */
wt_status wt_measure_groups(const wt_pipeline* p, int width, int height, int fp16, int n,
                            const char* const* groups, int reps, const char* tag,
                            double* times_us);

/* Pre-profiling of stage `node` (the paper, Section 6): the time of one
 * evaluation of its body by a single lane with operands in LDS (microbench-
 * mark over many iterations, less the bare loop), and the VGPRs of its body
 * (its unfused kernel's allocation less input rings and addressing), as the
 * analytical model uses them.  measure = 1 times it on the current device
 * (results are cached per stage signature for the process); measure = 0 only
 * compiles the microbenchmarks and returns the static estimate.  *measured
 * tells which. */
wt_status wt_stage_profile(const wt_pipeline* p, int node, int width, int height, int measure,
                           double* ns_per_point, int* vgprs, int* measured);

/* Destroys the plan; its stream must have drained. */
void wt_plan_destroy(wt_plan* plan);

const char* wt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* WAVETILE_WT_H */
