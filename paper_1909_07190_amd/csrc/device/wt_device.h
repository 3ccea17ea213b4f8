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
typedef int wt_i2 __attribute__((ext_vector_type(2)));
typedef int wt_i4 __attribute__((ext_vector_type(4)));
typedef unsigned char wt_b2 __attribute__((ext_vector_type(2)));
typedef unsigned char wt_b4 __attribute__((ext_vector_type(4)));
typedef unsigned short wt_us2 __attribute__((ext_vector_type(2)));
typedef unsigned short wt_us4 __attribute__((ext_vector_type(4)));
typedef short wt_s2 __attribute__((ext_vector_type(2)));
typedef short wt_s4 __attribute__((ext_vector_type(4)));
// The same vectors of 32-bit elements with 4-byte alignment: global loads
// of rows that start at any element (the caller's images of any width and
// row stride).  gfx950 executes them as single dwordx2 / dwordx4 loads (the
// memory system runs in unaligned-access mode under ROCm).
typedef float wt_f2d __attribute__((ext_vector_type(2), aligned(4)));
typedef float wt_f4d __attribute__((ext_vector_type(4), aligned(4)));
typedef int wt_i2d __attribute__((ext_vector_type(2), aligned(4)));
typedef int wt_i4d __attribute__((ext_vector_type(4), aligned(4)));

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

// Lane exchanges move 32-bit values: FP32 stage values or the exact 32-bit
// integers of integer stages (T = float or int).
template <typename T> WT_DEV int wt_bits(T v) { return __builtin_bit_cast(int, v); }
template <typename T> WT_DEV T wt_unbits(int v) { return __builtin_bit_cast(T, v); }

// Lane t receives cur from lane t-1; lane 0 keeps `old0` (its own value of
// the second operand).  bound_ctrl off: the invalid source lane keeps old.
template <typename T> WT_DEV T wt_shr1(T cur, T old0) {
    return wt_unbits<T>(__builtin_amdgcn_update_dpp(wt_bits(old0), wt_bits(cur),
                                                     WT_DPP_WAVE_SHR1, 0xF, 0xF, false));
}

// Lane t receives v from lane (t-1) mod 64.
template <typename T> WT_DEV T wt_ror1(T v) {
    return wt_unbits<T>(__builtin_amdgcn_mov_dpp(wt_bits(v), WT_DPP_WAVE_ROR1, 0xF, 0xF, false));
}

// Types 3 + 4 for a one-lane shift: lanes 1..63 read `cur` of lane t-1 (same
// sub-tile); lane 0 reads `prev` of lane 63 (previous sub-tile).
template <typename T> WT_DEV T wt_shift1(T cur, T prev) { return wt_shr1(cur, wt_ror1(prev)); }

// Mirror images for reads to the right: lane t receives cur from lane t+1;
// lane 63 keeps `old63`.
template <typename T> WT_DEV T wt_shl1(T cur, T old63) {
    return wt_unbits<T>(__builtin_amdgcn_update_dpp(wt_bits(old63), wt_bits(cur),
                                                     WT_DPP_WAVE_SHL1, 0xF, 0xF, false));
}
template <typename T> WT_DEV T wt_rol1(T v) {
    return wt_unbits<T>(__builtin_amdgcn_mov_dpp(wt_bits(v), WT_DPP_WAVE_ROL1, 0xF, 0xF, false));
}
// One-lane shifts where the lane past the end may take any value (it lies in
// the tile's overlap): bound_ctrl on, a single DPP move.
template <typename T> WT_DEV T wt_mov_shr1(T v) {
    return wt_unbits<T>(__builtin_amdgcn_mov_dpp(wt_bits(v), WT_DPP_WAVE_SHR1, 0xF, 0xF, true));
}
template <typename T> WT_DEV T wt_mov_shl1(T v) {
    return wt_unbits<T>(__builtin_amdgcn_mov_dpp(wt_bits(v), WT_DPP_WAVE_SHL1, 0xF, 0xF, true));
}
// Value of v in lane (byte address addr) / 4, through the LDS crossbar.
template <typename T> WT_DEV T wt_bperm(int addr, T v) {
    return wt_unbits<T>(__builtin_amdgcn_ds_bpermute(addr, wt_bits(v)));
}
// Lanes 0..62 read cur of lane t+1; lane 63 reads `next` of lane 0 (next sub-tile).
template <typename T> WT_DEV T wt_shift1n(T cur, T next) { return wt_shl1(cur, wt_rol1(next)); }
// Lanes t < 64-d read cur of lane t+d; lanes t >= 64-d read next of lane t+d-64.
template <typename T> WT_DEV T wt_shiftdn(T cur, T next, int d, int lane) {
    int a = ((lane + d) & 63) << 2;
    T c = wt_bperm(a, cur);
    T n = wt_bperm(a, next);
    return lane < 64 - d ? c : n;
}

// Two-lane shifts composed from one-lane DPP shifts (no LDS crossbar):
// lanes 2..63 read cur of lane t-2, lanes 0..1 read prev of lanes 62..63.
template <typename T> WT_DEV T wt_shift2(T cur, T prev) {
    return wt_shift1(wt_shift1(cur, prev), wt_shift1(prev, prev));
}
// Mirror image: lanes 0..61 read cur of lane t+2, lanes 62..63 next of lanes 0..1.
template <typename T> WT_DEV T wt_shift2n(T cur, T next) {
    return wt_shift1n(wt_shift1n(cur, next), wt_shift1n(next, next));
}

// Types 3 + 4 for a d-lane shift, 1 <= d <= 63: lanes t >= d read cur of lane
// t-d, lanes t < d read prev of lane 64+t-d.
template <typename T> WT_DEV T wt_shiftd(T cur, T prev, int d, int lane) {
    int a = ((lane - d) & 63) << 2;
    T c = wt_bperm(a, cur);
    T p = wt_bperm(a, prev);
    return lane >= d ? c : p;
}

// As wt_shiftd, with lanes t < d taking `prev_here`, a value each such lane
// already holds (read from the LDS sub-tile: load type 2).
template <typename T> WT_DEV T wt_shiftd_l(T cur, T prev_here, int d, int lane) {
    T c = wt_bperm(((lane - d) & 63) << 2, cur);
    return lane >= d ? c : prev_here;
}

// Value of v in lane `src` (wave-uniform), broadcast.
template <typename T> WT_DEV T wt_readlane(T v, int src) {
    return wt_unbits<T>(__builtin_amdgcn_readlane(wt_bits(v), src));
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

// Histogram bin of value v: floor((v - lo) * scale) in FP32, clamped to
// 0..nb-1 (NaN and values below lo count in bin 0, values at or past the
// top in bin nb-1).
WT_DEV int wt_hist_bin(float v, float lo, float scale, int nb) {
    const float t = (v - lo) * scale;
    return !(t >= 0.0f) ? 0 : (t >= (float)nb ? nb - 1 : (int)t);
}
// Counter increments: a wave's own LDS bins, and the device-wide output
WT_DEV void wt_count_lds(unsigned int* p, unsigned int v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
WT_DEV void wt_count_global(unsigned int* p, unsigned int v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Integer stage arithmetic (exact in 32 bits: the library bounds every sum).
// Quotient rounded half up: floor((a + d/2) / d) for d >= 1.
WT_DEV int wt_rdiv(int a, int d) {
    int n = a + (d >> 1);
    int q = n / d;
    return (n % d != 0 && n < 0) ? q - 1 : q;
}
// Same for d = 2^s, s >= 1: arithmetic shift floors.
WT_DEV int wt_rshift(int a, int s) { return (a + (1 << (s - 1))) >> s; }
WT_DEV int wt_sat(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }
WT_DEV int wt_abs(int v) { return v < 0 ? -v : v; }
WT_DEV float wt_abs(float v) { return fabsf(v); }
WT_DEV int wt_min(int a, int b) { return a < b ? a : b; }
WT_DEV float wt_min(float a, float b) { return fminf(a, b); }
WT_DEV int wt_max(int a, int b) { return a > b ? a : b; }
WT_DEV float wt_max(float a, float b) { return fmaxf(a, b); }
