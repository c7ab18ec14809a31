// Device-side building blocks shared by the engine's kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gputx.h"

#define GTX_BLOCK 256          // threads per workgroup for every kernel
#define GTX_WAVES (GTX_BLOCK / 64)
#define GTX_MAX_OPS 16         // basic operations of one transaction after dedupe
#define GTX_MAX_APPEND 4       // append-only tables per context
#define GTX_MAX_PARAMS 34      // widest signature (new-order)
#define GTX_MAX_RESULTS 16
#define GTX_ROLES GPUTX_MAX_ROLES

// Per-bulk device state, inside the workspace.  The first kernel of a bulk
// clears it.
struct GtxState {
    int32_t error;        // bulk error (GPUTX_E_*), 0 = none
    int32_t unsorted;     // timestamps not ascending in input order
    int32_t chosen;       // strategy that runs
    int32_t run_part;     // 1 when PART runs (gates its sort)
    int64_t m;            // basic operations emitted
    int64_t app_total[GTX_MAX_APPEND];
    int64_t w0, depth, cross, waves;
    int64_t committed, aborted, invalid;
    int64_t part_keys;    // distinct partition ids (PART sort domain, incl. sentinel)
    int32_t type_count[GPUTX_MAX_TYPES];
    uint32_t done_ctr[4]; // last-block tickets
    uint32_t ticket;      // TPL window ticket
    uint32_t bar_count;   // grid barrier arrivals
    uint32_t bar_gen;     // grid barrier generation
    int32_t kset_fill[3][GPUTX_MAX_TYPES];  // K-SET frontier fill per type (rotating)
    int32_t dup_adj;      // two adjacent input timestamps are equal
    uint32_t narrow_gen;  // K-SET: bumped when workgroup 0 leaves narrow mode
    int32_t narrow_done;  // K-SET: narrow mode ran the last wave
    int64_t narrow_k;     // K-SET: next wave after narrow mode
    int64_t narrow_prog;  // K-SET: waves finished in narrow mode (watchdog progress)
    int32_t n_heads;      // PART: non-empty partitions
    int32_t pad;
    int64_t scan_chunks;  // PART: chunks run in the scan form
};

namespace gtx {

__device__ __forceinline__ int lane_id() { return __lane_id(); }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }
__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

// ---- memory model helpers (agent scope = the whole GPU, all 8 XCDs) -------
template <class T>
__device__ __forceinline__ T ld_relaxed(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void st_relaxed(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void fence_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
__device__ __forceinline__ void fence_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void fence_acq_rel() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent"); }

__device__ __forceinline__ uint64_t now_ticks() { return wall_clock64(); }

// ---- wave-level scans (64 lanes) ------------------------------------------
__device__ __forceinline__ int wave_incl_sum(int v) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int u = __shfl_up(v, d);
        if (lane_id() >= d) v += u;
    }
    return v;
}
__device__ __forceinline__ int wave_incl_max(int v) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int u = __shfl_up(v, d);
        if (lane_id() >= d) v = max(v, u);
    }
    return v;
}
__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = max(v, __shfl_xor(v, d));
    return v;
}
__device__ __forceinline__ long long wave_sum64(long long v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    return v;
}

// Block-wide exclusive sum over GTX_BLOCK threads; returns the block total in *total.
__device__ __forceinline__ int block_excl_sum(int v, int* total, int* lds /* >= GTX_WAVES+1 */) {
    int inc = wave_incl_sum(v);
    if (lane_id() == 63) lds[wave_id()] = inc;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < GTX_WAVES; ++w) {
        int s = lds[w];
        if (w < wave_id()) base += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return base + inc - v;
}

// Match-any over an 8-bit value: mask of lanes in this wave holding the same value.
__device__ __forceinline__ uint64_t match_u8(uint32_t v, uint64_t active) {
    uint64_t m = active;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        uint64_t bal = __ballot((v >> b) & 1u);
        m &= ((v >> b) & 1u) ? bal : ~bal;
    }
    return m;
}

}  // namespace gtx
