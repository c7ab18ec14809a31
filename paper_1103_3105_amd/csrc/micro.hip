// Branch-divergence micro benchmark (Section 6.2, Appendix D, Figures 3
// and 12).
//
// A bulk of independent transactions, each of one of T types, each reading
// one tuple, computing on it and writing the result back.  The types are the
// T cases of one switch, so a wave64 whose lanes hold k distinct types runs k
// case bodies one after another.  Grouping the bulk by type (a radix
// partition of the transaction order on the type id) removes that
// divergence at the cost of the partitioning passes; partitioning into p
// groups (the top log2 p bits of the type id, one bit per pass) trades the
// two, and a calibration picks p (Appendix D).
//
// The paper's per-type computation calls a transcendental function 100 x
// times; here each case runs 100 x rounds of an integer mixing step with
// constants of its own (exact, so results are compared bit for bit):
//     v <- (v xor (v >> 29)) * M_k + (k + 1),   M_k = 0x9E3779B97F4A7C15 + 2k.
//
//   k_micro_split_count / k_micro_split_scan / k_micro_split_scatter
//              one stable 1-bit partition pass of the transaction order
//   k_micro_exec  the combined kernel: one lane per transaction of the
//              (grouped) order, switch on its type
#include <hip/hip_runtime.h>

#include <algorithm>

#include "runtime.h"

namespace gtx {

constexpr int kMicroMaxTypes = 32;
constexpr int kMicroTile = 1024;  // transactions per partition-pass workgroup (4 per thread)

template <int K>
__device__ __forceinline__ uint64_t micro_body(uint64_t v, int rounds) {
    constexpr uint64_t M = 0x9E3779B97F4A7C15ull + 2ull * K;
    for (int r = 0; r < rounds; ++r) v = (v ^ (v >> 29)) * M + (uint64_t)(K + 1);
    return v;
}

__global__ __launch_bounds__(256) void k_micro_exec(const int32_t* __restrict__ type, const int32_t* __restrict__ order,
                                                    int64_t* tuples, int64_t n, int rounds) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int32_t t = order ? order[i] : (int32_t)i;
    const int ty = type[t];
    uint64_t v = (uint64_t)tuples[t];
    switch (ty) {
#define GTX_MICRO_CASE(K) \
    case K:               \
        v = micro_body<K>(v, rounds); \
        break;
        GTX_MICRO_CASE(0) GTX_MICRO_CASE(1) GTX_MICRO_CASE(2) GTX_MICRO_CASE(3)
        GTX_MICRO_CASE(4) GTX_MICRO_CASE(5) GTX_MICRO_CASE(6) GTX_MICRO_CASE(7)
        GTX_MICRO_CASE(8) GTX_MICRO_CASE(9) GTX_MICRO_CASE(10) GTX_MICRO_CASE(11)
        GTX_MICRO_CASE(12) GTX_MICRO_CASE(13) GTX_MICRO_CASE(14) GTX_MICRO_CASE(15)
        GTX_MICRO_CASE(16) GTX_MICRO_CASE(17) GTX_MICRO_CASE(18) GTX_MICRO_CASE(19)
        GTX_MICRO_CASE(20) GTX_MICRO_CASE(21) GTX_MICRO_CASE(22) GTX_MICRO_CASE(23)
        GTX_MICRO_CASE(24) GTX_MICRO_CASE(25) GTX_MICRO_CASE(26) GTX_MICRO_CASE(27)
        GTX_MICRO_CASE(28) GTX_MICRO_CASE(29) GTX_MICRO_CASE(30) GTX_MICRO_CASE(31)
#undef GTX_MICRO_CASE
        default:
            return;  // no such type: the tuple is left as it is
    }
    tuples[t] = (int64_t)v;
}

// One stable split of `in` (transaction indices) on bit `bit` of the type:
// zeros first, in order, then ones.  Pass 1: per-tile count of zeros.
__global__ __launch_bounds__(256) void k_micro_split_count(const int32_t* __restrict__ type,
                                                           const int32_t* __restrict__ in, int64_t n, int bit,
                                                           int32_t* tile_zeros) {
    __shared__ int part[GTX_WAVES];
    const int64_t base = (int64_t)blockIdx.x * kMicroTile;
    int z = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t i = base + k * 256 + threadIdx.x;
        if (i < n) z += ((type[in ? in[i] : (int32_t)i] >> bit) & 1) == 0;
    }
    z = wave_sum(z);
    if (lane_id() == 0) part[wave_id()] = z;
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int w = 0; w < GTX_WAVES; ++w) s += part[w];
        tile_zeros[blockIdx.x] = s;
    }
}

// Pass 2 (one workgroup): exclusive scan of the tile counts in place; the
// total number of zeros goes to tile_zeros[n_tiles].
__global__ __launch_bounds__(256) void k_micro_split_scan(int32_t* tile_zeros, int n_tiles) {
    __shared__ int lds[GTX_WAVES + 1];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int c0 = 0; c0 < n_tiles; c0 += 256) {
        const int i = c0 + threadIdx.x;
        const int v = i < n_tiles ? tile_zeros[i] : 0;
        int tot;
        const int ex = block_excl_sum(v, &tot, lds);
        if (i < n_tiles) tile_zeros[i] = carry + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) tile_zeros[n_tiles] = carry;
}

// Pass 3: scatter, keeping the order within zeros and within ones.
__global__ __launch_bounds__(256) void k_micro_split_scatter(const int32_t* __restrict__ type,
                                                             const int32_t* __restrict__ in, int64_t n, int bit,
                                                             const int32_t* __restrict__ tile_zeros, int n_tiles,
                                                             int32_t* __restrict__ out) {
    __shared__ int lds[GTX_WAVES + 1];
    const int64_t base = (int64_t)blockIdx.x * kMicroTile;
    const int zeros_before = tile_zeros[blockIdx.x];
    const int zeros_total = tile_zeros[n_tiles];
    int seen_zero = 0;  // zeros in earlier sub-rounds of this tile
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t i = base + k * 256 + threadIdx.x;
        int32_t t = 0;
        int z = 0;
        if (i < n) {
            t = in ? in[i] : (int32_t)i;
            z = ((type[t] >> bit) & 1) == 0;
        }
        int tot;
        const int ex = block_excl_sum(z, &tot, lds);
        if (i < n) {
            const int64_t zpos = zeros_before + seen_zero + ex;                // zeros before me
            const int64_t dst = z ? zpos : zeros_total + (i - zpos);          // ones keep their order
            out[dst] = t;
        }
        seen_zero += tot;
    }
}

}  // namespace gtx

using namespace gtx;

extern "C" size_t gputx_micro_workspace_size(int64_t n) {
    if (n < 0) return 0;
    const int64_t tiles = (n + kMicroTile - 1) / kMicroTile;
    return 2 * (((size_t)std::max<int64_t>(n, 1) * 4 + 255) & ~size_t(255)) + (size_t)(tiles + 1) * 4 + 256;
}

extern "C" int gputx_micro_run(int64_t n, const int32_t* type, int64_t* tuples, int32_t n_types, int32_t x,
                               int32_t groups, void* workspace, size_t ws_bytes, int32_t phase,
                               gputx_stream_t stream) {
    if (n < 0 || n > ((int64_t)1 << 31) - 1 || n_types < 1 || n_types > kMicroMaxTypes || x < 0 || x > 1000 ||
        groups < 1 || groups > n_types || (groups & (groups - 1)) || phase < 0 || phase > 2)
        return gtx_set_err(nullptr, GPUTX_E_ARG, "bad micro benchmark argument");
    if (n > 0 && (!type || !tuples)) return gtx_set_err(nullptr, GPUTX_E_ARG, "null array");
    if (n == 0) return GPUTX_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int tbits = 0;
    while ((1 << tbits) < n_types) ++tbits;
    int gbits = 0;
    while ((1 << gbits) < groups) ++gbits;
    const int32_t* order = nullptr;
    if (gbits > 0) {
        if (!workspace || ws_bytes < gputx_micro_workspace_size(n) || (uintptr_t)workspace % 256)
            return gtx_set_err(nullptr, GPUTX_E_CAPACITY, "micro workspace too small or misaligned");
        const size_t arr = ((size_t)n * 4 + 255) & ~size_t(255);
        int32_t* buf[2] = {reinterpret_cast<int32_t*>(workspace),
                           reinterpret_cast<int32_t*>((char*)workspace + arr)};
        int32_t* tiles = reinterpret_cast<int32_t*>((char*)workspace + 2 * arr);
        const int n_tiles = (int)((n + kMicroTile - 1) / kMicroTile);
        // LSD over the top gbits bits of the type id: afterwards the order is
        // grouped by those bits (2^gbits groups), stable within each group
        const int32_t* in = nullptr;
        for (int b = 0; b < gbits; ++b) {
            const int bit = tbits - gbits + b;
            int32_t* out = buf[b & 1];
            if (phase != 2) {
                hipLaunchKernelGGL(k_micro_split_count, dim3(n_tiles), dim3(256), 0, s, type, in, n, bit, tiles);
                hipLaunchKernelGGL(k_micro_split_scan, dim3(1), dim3(256), 0, s, tiles, n_tiles);
                hipLaunchKernelGGL(k_micro_split_scatter, dim3(n_tiles), dim3(256), 0, s, type, in, n, bit, tiles,
                                   n_tiles, out);
            }
            in = out;
        }
        order = in;
    }
    if (phase != 1) {
        const int rounds = 100 * x;
        hipLaunchKernelGGL(k_micro_exec, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, type, order, tuples, n,
                           rounds);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return gtx_set_err(nullptr, GPUTX_E_HIP, "micro launch: %s", hipGetErrorString(e));
    return GPUTX_OK;
}
