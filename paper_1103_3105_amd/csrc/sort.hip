// Stable LSD radix sort of (key, value) pairs, 8-bit digits, for gfx950.
//
// Section 4.2 groups the basic operations "firstly on v and then on id" with
// a sort primitive; the paper reuses an existing GPU sort.  Here the pairs
// are emitted in timestamp order, so a *stable* sort on the item key alone
// yields (item, timestamp) order.  The same sort orders timestamps (64-bit
// keys) and groups transactions by partition for PART (Section 5.2).
//
// One pass per digit, one kernel per pass (reduce-free "onesweep" design):
//  * a histogram kernel counts every pass's digits once up front and turns
//    them into global exclusive digit offsets (last-block pattern);
//  * each pass kernel takes a tile of 8192 32-bit or 4096 64-bit keys (dynamic
//    tile id, so every earlier tile is already running), ranks keys within each
//    wave64 by an 8-ballot match on the digit, combines the waves through LDS, publishes
//    its per-digit count and resolves its global offset by decoupled
//    look-back over earlier tiles (flag and count share one 32-bit word, so
//    no fence is needed), then scatters through LDS so that each digit's run
//    is written contiguously.
#include "sort.h"

namespace gtx {

constexpr int kItems = 16;
constexpr int kHistLoads = 8;
// Workgroup of a pass: 8 waves for 32-bit keys (8192-key tiles, so half as
// many tiles walk the look-back chain), 4 for 64-bit keys (LDS for 4096).
template <class K>
constexpr int sort_block() { return sizeof(K) == 4 ? 512 : 256; }
template <class K>
constexpr int sort_tile() { return sort_block<K>() * kItems; }
constexpr int kTileMin = 256 * kItems;  // sizes the look-back words for either key width
constexpr uint32_t kAgg = 1u << 30;
constexpr uint32_t kPrefix = 2u << 30;
constexpr uint32_t kCountMask = (1u << 30) - 1u;

template <class K>
__device__ __forceinline__ uint32_t digit_of(K k, int pass) {
    return (uint32_t)(k >> (8 * pass)) & 0xffu;
}

__device__ __forceinline__ bool sort_gated(const int32_t* gate, const GtxState* st) {
    if (st && ld_relaxed(&st->error) != 0) return true;
    return gate && ld_relaxed(gate) == 0;
}

__global__ __launch_bounds__(GTX_BLOCK) void k_sort_init(uint32_t* status, int64_t n_status,
                                                         uint32_t* hist, uint32_t* ctrl,
                                                         const int32_t* gate, const GtxState* st) {
    if (sort_gated(gate, st)) return;
    int64_t tid = (int64_t)blockIdx.x * GTX_BLOCK + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * GTX_BLOCK;
    for (int64_t i = tid; i < n_status; i += stride) status[i] = 0;
    if (blockIdx.x == 0) {
        for (int i = threadIdx.x; i < 8 * 256; i += GTX_BLOCK) hist[i] = 0;
        if (threadIdx.x < 16) ctrl[threadIdx.x] = 0;
    }
}

template <class K>
__global__ __launch_bounds__(GTX_BLOCK) void k_sort_hist(const K* keys, const int64_t* count_dev,
                                                         int64_t count_cap, int npass,
                                                         uint32_t* hist, uint32_t* ctrl,
                                                         const int32_t* gate, const GtxState* st) {
    if (sort_gated(gate, st)) return;
    __shared__ uint32_t h[8][256];
    __shared__ uint32_t is_last;
    for (int i = threadIdx.x; i < 8 * 256; i += GTX_BLOCK) (&h[0][0])[i] = 0;
    __syncthreads();
    int64_t count = count_dev ? *count_dev : count_cap;
    // kHistLoads keys per thread in flight at once: one load per loop trip
    // left the kernel waiting on memory latency every trip
    const int64_t step = (int64_t)gridDim.x * GTX_BLOCK * kHistLoads;
    for (int64_t i0 = (int64_t)blockIdx.x * GTX_BLOCK * kHistLoads + threadIdx.x; i0 < count; i0 += step) {
        K k[kHistLoads];
#pragma unroll
        for (int j = 0; j < kHistLoads; ++j) {
            const int64_t i = i0 + (int64_t)j * GTX_BLOCK;
            k[j] = i < count ? keys[i] : (K)0;
        }
#pragma unroll
        for (int j = 0; j < kHistLoads; ++j)
            if (i0 + (int64_t)j * GTX_BLOCK < count)
                for (int p = 0; p < npass; ++p) atomicAdd(&h[p][digit_of(k[j], p)], 1u);
    }
    __syncthreads();
    for (int p = 0; p < npass; ++p) {
        uint32_t c = h[p][threadIdx.x];
        if (c) atomicAdd(&hist[p * 256 + threadIdx.x], c);
    }
    // the last block to finish turns counts into exclusive offsets
    __syncthreads();
    if (threadIdx.x == 0) {
        fence_release();
        uint32_t t = atomicAdd(&ctrl[8], 1u);
        is_last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (!is_last) return;
    fence_acquire();
    __shared__ int scratch[GTX_WAVES + 1];
    for (int p = 0; p < npass; ++p) {
        int c = (int)ld_relaxed(&hist[p * 256 + threadIdx.x]);
        int tot;
        int ex = block_excl_sum(c, &tot, scratch);
        hist[p * 256 + threadIdx.x] = (uint32_t)ex;
    }
}

// Exclusive sum over the threads of a B-thread workgroup.
template <int B>
__device__ __forceinline__ int sort_block_excl_sum(int v, int* lds /* >= B / 64 */) {
    int inc = wave_incl_sum(v);
    if (lane_id() == 63) lds[wave_id()] = inc;
    __syncthreads();
    int base = 0;
#pragma unroll
    for (int w = 0; w < B / 64; ++w)
        if (w < wave_id()) base += lds[w];
    __syncthreads();
    return base + inc - v;
}

template <class K>
__global__ __launch_bounds__(sort_block<K>()) void k_sort_pass(const K* __restrict__ kin,
                                                         const uint32_t* __restrict__ vin,
                                                         K* __restrict__ kout, uint32_t* __restrict__ vout,
                                                         const int64_t* count_dev, int64_t count_cap,
                                                         int pass, const uint32_t* hist,
                                                         uint32_t* status, int64_t max_tiles,
                                                         uint32_t* ctrl, const int32_t* gate,
                                                         GtxState* st, uint64_t spin_ticks,
                                                         uint32_t* __restrict__ inv) {
    constexpr int B = sort_block<K>();
    constexpr int kW = B / 64;
    constexpr int kTile = sort_tile<K>();
    __shared__ uint32_t tile_s;
    __shared__ uint32_t wcnt[kW][256];
    __shared__ uint32_t dstart[256];
    __shared__ int64_t gbase[256];
    __shared__ K skeys[kTile];
    __shared__ uint32_t svals[kTile];
    __shared__ int scratch[kW + 1];

    // The tile ticket, the gate words, the key count and this digit's global
    // offset are independent loads: issue them together, then wait once.
    if (threadIdx.x == 0) {
        const uint32_t ticket = atomicAdd(&ctrl[pass], 1u);
        tile_s = sort_gated(gate, st) ? 0xffffffffu : ticket;
    }
    const int64_t count = count_dev ? *count_dev : count_cap;
    const int d = threadIdx.x;
    const bool digit = d < 256;
    const uint32_t goff = digit ? hist[pass * 256 + d] : 0u;
    for (int i = threadIdx.x; i < kW * 256; i += B) (&wcnt[0][0])[i] = 0;
    __syncthreads();
    if (tile_s == 0xffffffffu) return;
    const int64_t tile = tile_s;
    const int64_t base = tile * kTile;
    if (base >= count) return;

    const int w = wave_id();
    const int lane = lane_id();
    K k[kItems];
    uint32_t v[kItems];
    uint32_t rk[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        int64_t idx = base + (int64_t)w * 64 * kItems + j * 64 + lane;
        bool ok = idx < count;
        k[j] = ok ? kin[idx] : (K)0;
        v[j] = ok ? vin[idx] : 0u;
        uint64_t active = __ballot(ok);
        uint32_t d = digit_of(k[j], pass);
        uint64_t peers = match_u8(d, active);
        uint32_t pre = 0;
        if (ok) pre = wcnt[w][d];
        int leader = peers ? __ffsll((unsigned long long)peers) - 1 : -1;
        if (ok && lane == leader) wcnt[w][d] = pre + (uint32_t)__popcll(peers);
        rk[j] = pre + (uint32_t)__popcll(peers & lanemask_lt());
    }
    __syncthreads();

    // per digit (threads 0..255): exclusive offsets over waves, block total,
    // block-local start
    uint32_t tot = 0;
    if (digit) {
#pragma unroll
        for (int ww = 0; ww < kW; ++ww) {
            uint32_t c = wcnt[ww][d];
            wcnt[ww][d] = tot;
            tot += c;
        }
    }
    const int ds = sort_block_excl_sum<B>(digit ? (int)tot : 0, scratch);
    if (digit) dstart[d] = (uint32_t)ds;

    // decoupled look-back for digit d
    uint32_t* my = status + ((int64_t)pass * max_tiles + tile) * 256 + d;
    uint32_t excl = 0;
    if (!digit) {
    } else if (tile == 0) {
        st_relaxed(my, kPrefix | tot);
    } else {
        st_relaxed(my, kAgg | tot);
        // walk back over up to kLook predecessors per round trip: their
        // status words are loaded together, then taken nearest first until a
        // prefix (done) or a tile that has not published yet (wait for it)
        constexpr int kLook = 4;
        int64_t t = tile - 1;
        uint64_t t0 = 0;
        const uint32_t* col = status + (int64_t)pass * max_tiles * 256 + d;
        bool done = false;
        while (!done) {
            uint32_t w[kLook];
#pragma unroll
            for (int j = 0; j < kLook; ++j) w[j] = t - j >= 0 ? ld_relaxed(col + (t - j) * 256) : kPrefix;
            int took = 0;
            bool stalled = false;
#pragma unroll
            for (int j = 0; j < kLook; ++j) {
                if (done || stalled) continue;
                if (w[j] & kPrefix) {
                    excl += w[j] & kCountMask;
                    done = true;
                } else if (w[j] & kAgg) {
                    excl += w[j] & kCountMask;
                    ++took;
                } else {
                    stalled = true;
                }
            }
            t -= took;
            if (done) break;
            if (stalled) {
                if (t0 == 0) t0 = now_ticks();
                else if (now_ticks() - t0 > spin_ticks) {
                    atomicCAS(&st->error, 0, GPUTX_E_DEADLOCK);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            } else {
                t0 = 0;  // progress: restart the watchdog
            }
        }
        st_relaxed(my, kPrefix | (excl + tot));
    }
    if (digit) gbase[d] = (int64_t)goff + excl - dstart[d];
    __syncthreads();

#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        int64_t idx = base + (int64_t)w * 64 * kItems + j * 64 + lane;
        if (idx < count) {
            uint32_t dg = digit_of(k[j], pass);
            uint32_t pos = dstart[dg] + wcnt[w][dg] + rk[j];
            skeys[pos] = k[j];
            svals[pos] = v[j];
        }
    }
    __syncthreads();
    int64_t n_here = count - base < kTile ? count - base : kTile;
    for (int i = threadIdx.x; i < n_here; i += B) {
        K kk = skeys[i];
        int64_t out = gbase[digit_of(kk, pass)] + i;
        const uint32_t vv = svals[i];
        kout[out] = kk;
        vout[out] = vv;
        if (inv) inv[vv] = (uint32_t)out;
    }
}

int64_t sort_tiles(int64_t cap) { return (cap + kTileMin - 1) / kTileMin; }

size_t sort_status_words(int64_t cap, int npass) { return (size_t)sort_tiles(cap) * 256 * npass; }

template <class K>
static void sort_impl(const SortPlan& p, hipStream_t s) {
    const int64_t tiles = (p.cap + sort_tile<K>() - 1) / sort_tile<K>();
    if (tiles == 0 || p.npass == 0) return;
    int64_t n_status = tiles * 256 * p.npass;
    int init_blocks = (int)std::min<int64_t>(1024, (n_status + GTX_BLOCK * 16 - 1) / (GTX_BLOCK * 16));
    if (init_blocks < 1) init_blocks = 1;
    hipLaunchKernelGGL(k_sort_init, dim3(init_blocks), dim3(GTX_BLOCK), 0, s, p.status, n_status,
                       p.hist, p.ctrl, p.gate, p.st);
    int hist_blocks = (int)std::min<int64_t>(512, (p.cap + GTX_BLOCK * kHistLoads - 1) / (GTX_BLOCK * kHistLoads));
    if (hist_blocks < 1) hist_blocks = 1;
    hipLaunchKernelGGL(k_sort_hist<K>, dim3(hist_blocks), dim3(GTX_BLOCK), 0, s,
                       (const K*)p.keys[0], p.count_dev, p.cap, p.npass, p.hist, p.ctrl, p.gate, p.st);
    for (int pass = 0; pass < p.npass; ++pass) {
        int src = pass & 1;
        hipLaunchKernelGGL(k_sort_pass<K>, dim3((unsigned)tiles), dim3(sort_block<K>()), 0, s,
                           (const K*)p.keys[src], (const uint32_t*)p.vals[src], (K*)p.keys[src ^ 1],
                           p.vals[src ^ 1], p.count_dev, p.cap, pass, p.hist, p.status, tiles,
                           p.ctrl, p.gate, p.st, p.spin_ticks, pass == p.npass - 1 ? p.inv : nullptr);
    }
}

void sort_pairs(const SortPlan& p, hipStream_t s) {
    if (p.key_bytes == 8) sort_impl<uint64_t>(p, s);
    else sort_impl<uint32_t>(p, s);
}

}  // namespace gtx
