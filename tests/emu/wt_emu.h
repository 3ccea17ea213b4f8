// Host emulation of generated wave-tile kernels (test infrastructure).
//
// A wavefront is run as 64 std::threads, one per lane.  Every cross-lane
// operation the generated code uses (DPP wavefront shifts and rotates,
// ds_bpermute, readlane, readfirstlane) and the wave-level synchronisation
// become barrier-synchronised exchanges, so the kernel source produced by the
// code generator runs unchanged on the CPU.  Buffer stores apply the
// hardware's range check (out-of-range offsets are discarded).  DPP
// semantics follow the GFX9/CDNA ISA: wave_shr:1 moves lane i-1 to lane i,
// wave_ror:1 rotates (lane 0 receives lane 63), wave_shl:1 / wave_rol:1 are
// the mirror images; a lane whose source is invalid keeps `old` unless
// bound_ctrl is set, in which case it receives 0.
#pragma once
#include <algorithm>
#include <atomic>
#include <barrier>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

struct wt_emu_dim3 { unsigned x = 0, y = 0, z = 0; };
static thread_local wt_emu_dim3 threadIdx, blockIdx, gridDim;
static thread_local int wt_emu_lane = 0;
static std::barrier<>* wt_emu_bar = nullptr;
static uint32_t wt_emu_x[64];
// Several waves running at once: each lane thread names its own wave's
// barrier and exchange buffer (otherwise the shared ones above serve).
static thread_local std::barrier<>* wt_emu_wave_bar = nullptr;
static thread_local uint32_t* wt_emu_wave_x = nullptr;

static inline void wt_emu_sync() { (wt_emu_wave_bar ? wt_emu_wave_bar : wt_emu_bar)->arrive_and_wait(); }

static inline uint32_t wt_emu_xchg(uint32_t v, int src) {
    uint32_t* x = wt_emu_wave_x ? wt_emu_wave_x : wt_emu_x;
    x[wt_emu_lane] = v;
    wt_emu_sync();
    uint32_t r = x[src & 63];
    wt_emu_sync();
    return r;
}

static inline int wt_emu_dpp(int old, int src, int ctrl, bool bound_ctrl) {
    int l = wt_emu_lane, s = -1;
    switch (ctrl) {
        case 0x138: s = l - 1; break;           // wave_shr:1
        case 0x13C: s = (l + 63) & 63; break;   // wave_ror:1
        case 0x130: s = l + 1; break;           // wave_shl:1
        case 0x134: s = (l + 1) & 63; break;    // wave_rol:1
        default: std::abort();
    }
    uint32_t r = wt_emu_xchg((uint32_t)src, s < 0 || s > 63 ? l : s);
    if (s < 0 || s > 63) return bound_ctrl ? 0 : old;
    return (int)r;
}

#define __builtin_amdgcn_update_dpp(old, src, ctrl, rm, bm, bc) wt_emu_dpp((old), (src), (ctrl), (bc))
#define __builtin_amdgcn_mov_dpp(src, ctrl, rm, bm, bc) wt_emu_dpp(0x7fc00000, (src), (ctrl), (bc))
#define __builtin_amdgcn_ds_bpermute(addr, v) ((int)wt_emu_xchg((uint32_t)(v), ((addr) >> 2) & 63))
#define __builtin_amdgcn_readlane(v, l) ((int)wt_emu_xchg((uint32_t)(v), (l)))
#define __builtin_amdgcn_readfirstlane(v) ((int)wt_emu_xchg((uint32_t)(v), 0))
#define __builtin_amdgcn_wave_barrier() wt_emu_sync()
// a barrier over the threads the runner started together: one wave, or a
// whole workgroup for one-tile-per-workgroup kernels
#define __syncthreads() wt_emu_sync()
// A wavefront executes in lockstep, so every lane's earlier stores precede
// an agent-scope fence the whole wave executes; the lane threads meet at it.
// (Wave-scope fences only order the compiler's view: nothing to do here.)
static inline void wt_emu_fence(const char* scope) {
    if (scope[0] == 'a') {
        std::atomic_thread_fence(std::memory_order_seq_cst);
        wt_emu_sync();
        std::atomic_thread_fence(std::memory_order_seq_cst);
    }
}
#define __builtin_amdgcn_fence(a, b) wt_emu_fence(b)
// atomics: the lanes are threads
#define __hip_atomic_fetch_add(p, v, order, scope) __atomic_fetch_add((p), (v), __ATOMIC_RELAXED)
#define __hip_atomic_load(p, order, scope) __atomic_load_n((p), __ATOMIC_SEQ_CST)
#define __hip_atomic_store(p, v, order, scope) __atomic_store_n((p), (v), __ATOMIC_SEQ_CST)
#define __builtin_amdgcn_s_sleep(n) std::this_thread::yield()
static inline unsigned long long wall_clock64() {
    return (unsigned long long)std::chrono::steady_clock::now().time_since_epoch().count() / 10;
}
#ifndef __HIP_MEMORY_SCOPE_WAVEFRONT
#define __HIP_MEMORY_SCOPE_WAVEFRONT 0
#define __HIP_MEMORY_SCOPE_WORKGROUP 0
#define __HIP_MEMORY_SCOPE_AGENT 0
#endif

struct wt_emu_rsrc { char* base; uint32_t num; };
#define __amdgpu_buffer_rsrc_t wt_emu_rsrc
static inline wt_emu_rsrc wt_emu_make_rsrc(const void* p, int, int num, int) {
    return {(char*)p, (uint32_t)num};
}
#define __builtin_amdgcn_make_buffer_rsrc(p, s, n, f) wt_emu_make_rsrc((p), (s), (n), (f))
template <class T>
static inline void wt_emu_bstore(T v, wt_emu_rsrc r, int off) {
    if ((uint64_t)(uint32_t)off + sizeof(T) <= r.num) std::memcpy(r.base + (uint32_t)off, &v, sizeof(T));
}
#define __builtin_amdgcn_raw_buffer_store_b8(v, r, o, so, aux) wt_emu_bstore((v), (r), (o))
#define __builtin_amdgcn_raw_buffer_store_b16(v, r, o, so, aux) wt_emu_bstore((v), (r), (o))
#define __builtin_amdgcn_raw_buffer_store_b32(v, r, o, so, aux) wt_emu_bstore((v), (r), (o))
#define __builtin_amdgcn_raw_buffer_store_b64(v, r, o, so, aux) wt_emu_bstore((v), (r), (o))
#define __builtin_amdgcn_raw_buffer_store_b128(v, r, o, so, aux) wt_emu_bstore((v), (r), (o))
// buffer loads: offsets past num_records read 0 (the hardware range check)
template <class T>
static inline T wt_emu_bload(wt_emu_rsrc r, int off) {
    T v{};
    if ((uint64_t)(uint32_t)off + sizeof(T) <= r.num) std::memcpy(&v, r.base + (uint32_t)off, sizeof(T));
    return v;
}
#define __builtin_amdgcn_raw_buffer_load_b8(r, o, so, aux) wt_emu_bload<unsigned char>((r), (o))
#define __builtin_amdgcn_raw_buffer_load_b16(r, o, so, aux) wt_emu_bload<unsigned short>((r), (o))
#define __builtin_amdgcn_raw_buffer_load_b32(r, o, so, aux) wt_emu_bload<unsigned int>((r), (o))
#define __builtin_amdgcn_raw_buffer_load_b64(r, o, so, aux) wt_emu_bload<wt_u2>((r), (o))
#define __builtin_amdgcn_raw_buffer_load_b128(r, o, so, aux) wt_emu_bload<wt_u4>((r), (o))

#define __global__
#define __device__
#define __forceinline__ inline
#define __launch_bounds__(n)
#define __shared__ static
using std::max;
using std::min;
