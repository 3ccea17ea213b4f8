// Device primitives for generated wave-tile kernels (gfx950, wave64).
//
// Prepended to every generated kernel source.  Hand-written; the code
// generator only composes calls to these.  Lane exchange follows the four
// producer-load types of hybrid tiling (the paper, Section 5, Fig. 4 and
// Fig. 7): (1) own VGPR, (2) LDS, (3) another lane of the same register
// sub-tile, (4) another lane of the previous register sub-tile.  Types 3 and
// 4 for a one-lane shift use DPP wavefront shifts (one VALU op each); longer
// shifts use ds_bpermute_b32 through the LDS crossbar (no LDS allocation).

typedef float wt_f2 __attribute__((ext_vector_type(2)));
typedef float wt_f4 __attribute__((ext_vector_type(4)));
typedef _Float16 wt_h2 __attribute__((ext_vector_type(2)));
typedef _Float16 wt_h4 __attribute__((ext_vector_type(4)));
typedef unsigned int wt_u2 __attribute__((ext_vector_type(2)));
typedef unsigned int wt_u4 __attribute__((ext_vector_type(4)));

// Buffer resource word 3 for raw (untyped, stride 0) buffers on GFX9/CDNA,
// and an offset past any buffer this library describes (<= 2 GiB): stores
// at WT_OOB are discarded by the hardware range check.
#define WT_RSRC_W3 0x00020000
#define WT_OOB 0x7FFFFFFF
// Cache-policy operand of buffer stores: the non-temporal (streaming) bit.
#define WT_CPOL_NT 2
// Accelerator complex dies; workgroups are dispatched to them round-robin.
#define WT_NXCD 8

#define WT_DEV static __device__ __forceinline__

// DPP controls of the GFX9/CDNA encoding: whole-wavefront shift / rotate by
// one lane toward higher (SHR, ROR) or lower (SHL, ROL) lane numbers.
#define WT_DPP_WAVE_SHL1 0x130
#define WT_DPP_WAVE_ROL1 0x134
#define WT_DPP_WAVE_SHR1 0x138
#define WT_DPP_WAVE_ROR1 0x13C

#define WT_MAXIO 16

struct WtArgs {
    const void* src[WT_MAXIO];   // loaded nodes: channel 0, row 0, column 0
    void* dst[WT_MAXIO];         // live-outs
    long long src_rs[WT_MAXIO];  // row strides (elements)
    long long src_cs[WT_MAXIO];  // channel strides (elements)
    long long dst_rs[WT_MAXIO];
    long long dst_cs[WT_MAXIO];
    int W, H;                    // domain of the group's stages
    int Ws, Hs;                  // source domain (resampling kernels)
    int tiles_x, tiles_y;        // wave tiles per channel plane
    int nwaves;                  // tiles_x * tiles_y * parallel channels
    int pad;
};

WT_DEV float wt_as_f(int v) { return __builtin_bit_cast(float, v); }
WT_DEV int wt_as_i(float v) { return __builtin_bit_cast(int, v); }

// Lane t receives cur from lane t-1; lane 0 keeps `old0` (its own value of
// the second operand).  bound_ctrl off: the invalid source lane keeps old.
WT_DEV float wt_shr1(float cur, float old0) {
    return wt_as_f(__builtin_amdgcn_update_dpp(wt_as_i(old0), wt_as_i(cur),
                                               WT_DPP_WAVE_SHR1, 0xF, 0xF, false));
}

// Lane t receives v from lane (t-1) mod 64.
WT_DEV float wt_ror1(float v) {
    return wt_as_f(__builtin_amdgcn_mov_dpp(wt_as_i(v), WT_DPP_WAVE_ROR1, 0xF, 0xF, false));
}

// Types 3 + 4 for a one-lane shift: lanes 1..63 read `cur` of lane t-1 (same
// sub-tile); lane 0 reads `prev` of lane 63 (previous sub-tile).
WT_DEV float wt_shift1(float cur, float prev) { return wt_shr1(cur, wt_ror1(prev)); }

// Mirror images for reads to the right: lane t receives cur from lane t+1;
// lane 63 keeps `old63`.
WT_DEV float wt_shl1(float cur, float old63) {
    return wt_as_f(__builtin_amdgcn_update_dpp(wt_as_i(old63), wt_as_i(cur),
                                               WT_DPP_WAVE_SHL1, 0xF, 0xF, false));
}
WT_DEV float wt_rol1(float v) {
    return wt_as_f(__builtin_amdgcn_mov_dpp(wt_as_i(v), WT_DPP_WAVE_ROL1, 0xF, 0xF, false));
}
// Lanes 0..62 read cur of lane t+1; lane 63 reads `next` of lane 0 (next sub-tile).
WT_DEV float wt_shift1n(float cur, float next) { return wt_shl1(cur, wt_rol1(next)); }
// Lanes t < 64-d read cur of lane t+d; lanes t >= 64-d read next of lane t+d-64.
WT_DEV float wt_shiftdn(float cur, float next, int d, int lane) {
    int a = ((lane + d) & 63) << 2;
    float c = wt_as_f(__builtin_amdgcn_ds_bpermute(a, wt_as_i(cur)));
    float n = wt_as_f(__builtin_amdgcn_ds_bpermute(a, wt_as_i(next)));
    return lane < 64 - d ? c : n;
}

// Two-lane shifts composed from one-lane DPP shifts (no LDS crossbar):
// lanes 2..63 read cur of lane t-2, lanes 0..1 read prev of lanes 62..63.
WT_DEV float wt_shift2(float cur, float prev) {
    return wt_shift1(wt_shift1(cur, prev), wt_shift1(prev, prev));
}
// Mirror image: lanes 0..61 read cur of lane t+2, lanes 62..63 next of lanes 0..1.
WT_DEV float wt_shift2n(float cur, float next) {
    return wt_shift1n(wt_shift1n(cur, next), wt_shift1n(next, next));
}

// Types 3 + 4 for a d-lane shift, 1 <= d <= 63: lanes t >= d read cur of lane
// t-d, lanes t < d read prev of lane 64+t-d.
WT_DEV float wt_shiftd(float cur, float prev, int d, int lane) {
    int a = ((lane - d) & 63) << 2;
    float c = wt_as_f(__builtin_amdgcn_ds_bpermute(a, wt_as_i(cur)));
    float p = wt_as_f(__builtin_amdgcn_ds_bpermute(a, wt_as_i(prev)));
    return lane >= d ? c : p;
}

// As wt_shiftd, with lanes t < d taking `prev_here`, a value each such lane
// already holds (read from the LDS sub-tile: load type 2).
WT_DEV float wt_shiftd_l(float cur, float prev_here, int d, int lane) {
    float c = wt_as_f(__builtin_amdgcn_ds_bpermute(((lane - d) & 63) << 2, wt_as_i(cur)));
    return lane >= d ? c : prev_here;
}

// Value of v in lane `src` (wave-uniform), broadcast.
WT_DEV float wt_readlane(float v, int src) {
    return wt_as_f(__builtin_amdgcn_readlane(wt_as_i(v), src));
}

// Orders this wave's LDS accesses across lanes: the hardware executes one
// wave's LDS instructions in order, so only compiler reordering has to be
// prevented (the wave-level synchronisation of Section 4; no s_barrier).
WT_DEV void wt_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// FP16 storage of an FP32 value (round to nearest even), read back as FP32.
WT_DEV float wt_h(float v) { return (float)(_Float16)v; }

WT_DEV int wt_clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }
