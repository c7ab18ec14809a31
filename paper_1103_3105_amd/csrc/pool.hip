// K-SET over a standing transaction pool (Section 5.3, incremental k-set).
//
// Transactions are added to a pool in timestamp order, bulk by bulk.  The
// pool keeps the basic operations of every pending transaction in one array
// sorted by (item, timestamp) -- Section 4.2's grouping, held across bulks.
// Adding a bulk sorts only the new operations and merges them into that
// array; a step then takes the pool's 0-set (transactions none of whose
// operations has a conflicting predecessor still pending), runs it without
// locks, and removes its operations.  After the 0-set leaves, the 1-set is
// the new 0-set (Section 5.3), so repeated steps run the pool in an order
// equivalent to the serial timestamp order (Definition 1), however the
// additions interleave with the steps.
//
// Layout (device, allocated at creation): a ring of `cap` transaction slots
// (slot = sequence number mod cap) holding each pending transaction's type,
// parameters, timestamp, append rows and, once it ran, its status and
// results; the sorted operations (item key, slot << 1 | write) in two
// buffers of cap * max_ops.  Adding a bulk runs the one-bulk front end
// (validation, count scans, operation emission, item-key sort) on the
// bulk alone in the pool's own workspace, then:
//   k_pool_check   the bulk follows the pool in timestamp order; its appends fit
//   k_pool_ingest  copy the bulk into its slots in timestamp order, with the
//                  rows its appends take (reserved now: they depend on the
//                  signature alone); invalid transactions are done at once
//   k_pool_merge   merge the bulk's sorted operations into the pool's (the
//                  bulk's come after the pool's within an item: they are
//                  later in timestamp order); each element finds its place
//                  by binary search in the other array
// A step:
//   k_pool_scan_*  for every operation: is it first in its item's group, or
//                  a read with only reads before it?  (segmented scan of
//                  "a write came before", three phases); transactions with an
//                  operation that is not are blocked
//   k_pool_exec    run every pending, unblocked transaction (the 0-set)
//   k_pool_compact drop the operations of transactions that ran
//   k_pool_tail    advance the done prefix of the sequence
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "runtime.h"

namespace gtx {

struct PoolDev {
    int32_t error;       // sticky: a bulk error, nothing runs after it
    int32_t pad;
    int64_t m;           // operations in the sorted array
    int64_t head;        // next sequence number
    int64_t tail;        // every transaction before it has run
    int64_t waves;       // steps that ran at least one transaction
    int64_t committed, aborted, invalid, executed;
    int64_t last_width;  // transactions the last step ran
    int64_t last_ts;     // timestamp of the last transaction added
    unsigned long long min_pending;  // smallest sequence number still pending after a step
};

struct PoolArgs {
    PoolDev* pd;
    int64_t cap;         // ring slots (power of two)
    int32_t n_params;
    int32_t width;
    int32_t max_ops;
    int32_t cur;         // which op buffer holds the sorted operations
    const DevType* types;
    int64_t* rowcount;
    int32_t n_app;
    // ring
    int32_t* type;       // [cap]
    int64_t* params;     // [n_params][cap]
    int64_t* ts;         // [cap]
    int64_t* app;        // [2][cap] rows of the transaction's appends
    int32_t* state;      // [cap] 0 pending, 1 done
    int32_t* blocked;    // [cap]
    int32_t* status;     // [cap]
    int64_t* results;    // [cap][width]
    // sorted operations, two buffers
    uint32_t* key[2];
    uint32_t* val[2];
    // scan scratch
    int32_t* tile_or;    // [tiles]: tile has a group start, "write after the last start"
    int32_t* tile_carry; // [tiles]
    int32_t* keep;       // [cap * max_ops + 1] compaction offsets
};

constexpr int kPoolTile = GTX_BLOCK * 4;

__device__ __forceinline__ bool pool_failed(const PoolArgs& P) { return ld_relaxed(&P.pd->error) != 0; }

// ---- adding a bulk --------------------------------------------------------
// a: the one-bulk front end's arguments over the added bulk (serial position
// p of the bulk becomes sequence number head + p).
__global__ __launch_bounds__(GTX_BLOCK) void k_pool_ingest(BulkArgs a, PoolArgs P) {
    if (pool_failed(P) || ld_relaxed(&a.ws.st->error) != 0) return;
    const int64_t head = P.pd->head;
    int inv = 0;
    for (int64_t p = (int64_t)blockIdx.x * GTX_BLOCK + threadIdx.x; p < a.n; p += (int64_t)gridDim.x * GTX_BLOCK) {
        const int64_t slot = (head + p) & (P.cap - 1);
        const int64_t i = a.ws.st->unsorted ? (int64_t)a.ws.tsv[0][p] : p;
        const int32_t t = a.ws.tty[p];
        P.type[slot] = t;
        for (int q = 0; q < P.n_params; ++q)
            P.params[(int64_t)q * P.cap + slot] = q < a.n_params ? a.params[(int64_t)q * a.n + i] : 0;
        P.ts[slot] = a.ts[i];
        int64_t app0 = 0, app1 = 0;
        if (t >= 0) {
            const DevType& T = a.types[t];
            if (T.app_idx[0] >= 0) app0 = a.rowcount[T.app_idx[0]] + a.ws.cnt[(int64_t)(1 + T.app_idx[0]) * a.n + p];
            if (T.app_idx[1] >= 0) app1 = a.rowcount[T.app_idx[1]] + a.ws.cnt[(int64_t)(1 + T.app_idx[1]) * a.n + p];
        }
        P.app[slot] = app0;
        P.app[P.cap + slot] = app1;
        P.state[slot] = t < 0;  // invalid: done already, no effect
        P.blocked[slot] = 0;
        if (t < 0) {
            ++inv;
            P.status[slot] = GPUTX_INVALID;
            for (int r = 0; r < P.width; ++r) P.results[slot * P.width + r] = 0;
        }
    }
    inv = wave_sum(inv);
    if (lane_id() == 0 && inv) atomicAdd((unsigned long long*)&P.pd->invalid, (unsigned long long)inv);
}

// Before the ingest: the bulk must come after everything in the pool in
// timestamp order, and its appends must fit; otherwise it is a bulk error
// and nothing of it enters the pool.
__global__ void k_pool_check(BulkArgs a, PoolArgs P) {
    if (threadIdx.x != 0 || pool_failed(P) || a.ws.st->error) return;
    const int64_t i0 = a.ws.st->unsorted ? (int64_t)a.ws.tsv[0][0] : 0;
    if (P.pd->head > 0 && a.ts[i0] <= P.pd->last_ts) {
        a.ws.st->error = GPUTX_E_UNSORTED;
        return;
    }
    for (int k = 0; k < a.n_app; ++k)
        if (a.ws.st->app_total[k] > 0 && a.rowcount[k] + a.ws.st->app_total[k] > a.capacity[k]) {
            a.ws.st->error = GPUTX_E_CAPACITY;
            return;
        }
}

// After the ingest: reserve the append rows and advance the sequence.
__global__ void k_pool_commit_add(BulkArgs a, PoolArgs P) {
    if (threadIdx.x != 0 || pool_failed(P)) return;
    const int err = a.ws.st->error;
    if (err) {
        P.pd->error = err;
        return;
    }
    for (int k = 0; k < a.n_app; ++k) a.rowcount[k] += a.ws.st->app_total[k];
    const int64_t il = a.ws.st->unsorted ? (int64_t)a.ws.tsv[0][a.n - 1] : a.n - 1;
    P.pd->last_ts = a.ts[il];
    P.pd->head += a.n;
}

__device__ __forceinline__ int64_t lower_bound_key(const uint32_t* k, int64_t n, uint32_t v) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (k[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}
__device__ __forceinline__ int64_t upper_bound_key(const uint32_t* k, int64_t n, uint32_t v) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (k[mid] <= v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Merge the pool's sorted operations (buffer P.cur) with the bulk's (sorted
// by item key in serial order) into buffer 1 - P.cur.  Ties: the pool's first.
__global__ __launch_bounds__(GTX_BLOCK) void k_pool_merge(BulkArgs a, PoolArgs P) {
    if (pool_failed(P) || ld_relaxed(&a.ws.st->error) != 0) return;
    const int64_t m0 = P.pd->m;
    const int64_t m1 = a.ws.st->m;
    const uint32_t* ok = P.key[P.cur];
    const uint32_t* ov = P.val[P.cur];
    uint32_t* nk = P.key[1 - P.cur];
    uint32_t* nv = P.val[1 - P.cur];
    const uint32_t* bk = a.ws.pk[a.key_passes & 1];
    const uint32_t* bv = a.ws.pv[a.key_passes & 1];
    const int64_t head = P.pd->head;
    const int64_t total = m0 + m1;
    for (int64_t e = (int64_t)blockIdx.x * GTX_BLOCK + threadIdx.x; e < total; e += (int64_t)gridDim.x * GTX_BLOCK) {
        if (e < m0) {
            const uint32_t k = ok[e];
            const int64_t d = e + lower_bound_key(bk, m1, k);
            nk[d] = k;
            nv[d] = ov[e];
        } else {
            const int64_t j = e - m0;
            const uint32_t k = bk[j];
            const uint32_t v = bv[j];
            const int64_t d = j + upper_bound_key(ok, m0, k);
            // the bulk's operation index -> its transaction's slot
            const int64_t p = a.ws.op_txn[v >> 1];
            const uint32_t slot = (uint32_t)((head + p) & (P.cap - 1));
            nk[d] = k;
            nv[d] = (slot << 1) | (v & 1u);
        }
    }
}

__global__ void k_pool_merge_done(BulkArgs a, PoolArgs P) {
    if (threadIdx.x != 0 || pool_failed(P) || a.ws.st->error) return;
    P.pd->m += a.ws.st->m;
}

// ---- one step: the pool's 0-set --------------------------------------------
// An operation is free when it starts its item's group, or it is a read and
// no write comes before it in the group.  Segmented OR-scan of "is a write"
// over each item's group: tile aggregate = (a group starts in the tile, OR
// of writes after the tile's last group start).
__global__ __launch_bounds__(GTX_BLOCK) void k_pool_scan_up(PoolArgs P) {
    if (pool_failed(P)) return;
    const int64_t m = P.pd->m;
    const int64_t base = (int64_t)blockIdx.x * kPoolTile;
    if (base >= m) return;
    const uint32_t* k = P.key[P.cur];
    const uint32_t* v = P.val[P.cur];
    __shared__ int s_start, s_last;  // any start; last start position within the tile
    __shared__ int s_or;
    if (threadIdx.x == 0) {
        s_start = 0;
        s_last = -1;
        s_or = 0;
    }
    __syncthreads();
    int mylast = -1;
    for (int j = threadIdx.x; j < kPoolTile; j += GTX_BLOCK) {
        const int64_t i = base + j;
        if (i < m && (i == 0 || k[i - 1] != k[i])) mylast = max(mylast, j);
    }
    if (mylast >= 0) {
        atomicMax(&s_last, mylast);
        s_start = 1;
    }
    __syncthreads();
    const int last = s_last;
    int w = 0;
    for (int j = threadIdx.x; j < kPoolTile; j += GTX_BLOCK) {
        const int64_t i = base + j;
        if (i < m && j >= max(last, 0) && (v[i] & 1u)) w = 1;
    }
    if (w) s_or = 1;
    __syncthreads();
    if (threadIdx.x == 0) P.tile_or[blockIdx.x] = (s_start << 1) | s_or;
}

// Tile carries: for each tile, was there a write in the group that reaches
// into it from before?  One workgroup scans the tile aggregates with the
// operator (s1, o1) then (s2, o2) = (s1 | s2, s2 ? o2 : o1 | o2), in chunks
// of GTX_BLOCK tiles.
__global__ __launch_bounds__(GTX_BLOCK) void k_pool_scan_mid(PoolArgs P) {
    if (pool_failed(P)) return;
    const int64_t m = P.pd->m;
    const int64_t tiles = (m + kPoolTile - 1) / kPoolTile;
    __shared__ int ws_s[GTX_WAVES], ws_o[GTX_WAVES];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < tiles; c0 += GTX_BLOCK) {
        const int64_t t = c0 + threadIdx.x;
        const int agg = t < tiles ? P.tile_or[t] : 0;
        int ss = (agg >> 1) & 1, oo = agg & 1;
        // inclusive scan in the wave
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int s2 = __shfl_up(ss, d), o2 = __shfl_up(oo, d);
            if (lane_id() >= d) {
                oo = ss ? oo : (oo | o2);
                ss = ss | s2;
            }
        }
        if (lane_id() == 63) {
            ws_s[wave_id()] = ss;
            ws_o[wave_id()] = oo;
        }
        __syncthreads();
        // prefix of the earlier waves, with the chunk's carry in front
        int ps = 0, po = carry;
        for (int w = 0; w < wave_id(); ++w) {
            po = ws_s[w] ? ws_o[w] : (po | ws_o[w]);
            ps = ps | ws_s[w];
        }
        // inclusive value of this tile with everything before it
        const int inc_o = ss ? oo : (po | oo);
        // exclusive: the inclusive value of the tile before
        int ex = __shfl_up(inc_o, 1);
        if (lane_id() == 0) ex = po;
        if (t < tiles) P.tile_carry[t] = ex;
        __syncthreads();
        if (threadIdx.x == GTX_BLOCK - 1) carry = inc_o;
        __syncthreads();
    }
}

// Block-wide inclusive max over GTX_BLOCK threads.
__device__ __forceinline__ int block_incl_max(int v, int* lds /* >= GTX_WAVES */) {
    const int w = wave_incl_max(v);
    if (lane_id() == 63) lds[wave_id()] = w;
    __syncthreads();
    int before = -1;
#pragma unroll
    for (int k = 0; k < GTX_WAVES; ++k)
        if (k < wave_id()) before = max(before, lds[k]);
    __syncthreads();
    return max(before, w);
}

// Mark the transactions of operations that are not free.  Per pass of
// GTX_BLOCK operations: the position of the last group start at or before
// each operation and of the last write before it (block max scans); a write
// lies between the group's start and the operation exactly when the second
// is not below the first.  A group that started in an earlier pass takes the
// carry of the passes before.
__global__ __launch_bounds__(GTX_BLOCK) void k_pool_scan_down(PoolArgs P) {
    if (pool_failed(P)) return;
    const int64_t m = P.pd->m;
    const int64_t base = (int64_t)blockIdx.x * kPoolTile;
    if (base >= m) return;
    const uint32_t* k = P.key[P.cur];
    const uint32_t* v = P.val[P.cur];
    __shared__ int lds[GTX_WAVES];
    __shared__ int last_s, last_w;
    int carry = P.tile_carry[blockIdx.x];
    for (int pass = 0; pass < kPoolTile / GTX_BLOCK; ++pass) {
        const int64_t i = base + (int64_t)pass * GTX_BLOCK + threadIdx.x;
        const bool in = i < m;
        const uint32_t vi = in ? v[i] : 0u;
        const bool start = in && (i == 0 || k[i - 1] != k[i]);
        const bool w = in && (vi & 1u);
        const int ls = block_incl_max(start ? (int)threadIdx.x : -1, lds);  // last start at or before
        const int lw = block_incl_max(w ? (int)threadIdx.x : -1, lds);      // last write at or before
        if (threadIdx.x == GTX_BLOCK - 1) {
            last_s = ls;
            last_w = lw;
        }
        __syncthreads();
        if (in && !start) {
            // a write that does not start its group waits; a read waits when a
            // write lies between its group's start and itself (for a read,
            // the last write at or before it is strictly before it)
            const bool blocked = w || (ls >= 0 ? lw >= ls : (carry || lw >= 0));
            if (blocked) P.blocked[vi >> 1] = 1;
        }
        // carry into the next pass
        carry = last_s >= 0 ? (last_w >= last_s) : (carry || last_w >= 0);
        __syncthreads();
    }
}

__global__ __launch_bounds__(GTX_BLOCK) void k_pool_unblock(PoolArgs P) {
    if (pool_failed(P)) return;
    const int64_t tail = P.pd->tail, head = P.pd->head;
    for (int64_t s = tail + (int64_t)blockIdx.x * GTX_BLOCK + threadIdx.x; s < head;
         s += (int64_t)gridDim.x * GTX_BLOCK)
        P.blocked[s & (P.cap - 1)] = 0;
}

// Run the 0-set: every pending transaction whose operations are all free.
__global__ __launch_bounds__(GTX_BLOCK) void k_pool_exec(PoolArgs P) {
    if (pool_failed(P)) return;
    const int64_t tail = P.pd->tail, head = P.pd->head;
    int c = 0, ab = 0, ran = 0;
    unsigned long long lo = ~0ull;  // smallest blocked sequence number seen
    for (int64_t s = tail + (int64_t)blockIdx.x * GTX_BLOCK + threadIdx.x; s < head;
         s += (int64_t)gridDim.x * GTX_BLOCK) {
        const int64_t slot = s & (P.cap - 1);
        if (P.state[slot] != 0) continue;
        if (P.blocked[slot]) {
            lo = min(lo, (unsigned long long)s);
            continue;
        }
        const int32_t t = P.type[slot];
        const DevType& T = P.types[t];
        int64_t prm[GTX_MAX_PARAMS];
#pragma unroll
        for (int q = 0; q < GTX_MAX_PARAMS; ++q) prm[q] = q < P.n_params ? P.params[(int64_t)q * P.cap + slot] : 0;
        int64_t res[GTX_MAX_RESULTS];
        const int32_t st = txn_exec(T, prm, P.ts[slot], P.app[slot], P.app[P.cap + slot], res);
        P.status[slot] = st;
        for (int r = 0; r < P.width; ++r) P.results[slot * P.width + r] = r < GTX_MAX_RESULTS ? res[r] : 0;
        P.state[slot] = 1;
        c += st == GPUTX_COMMIT;
        ab += st == GPUTX_ABORT;
        ++ran;
    }
    c = wave_sum(c);
    ab = wave_sum(ab);
    ran = wave_sum(ran);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const unsigned long long o = __shfl_xor(lo, d);
        lo = o < lo ? o : lo;
    }
    if (lane_id() == 0) {
        if (lo != ~0ull) atomicMin(&P.pd->min_pending, lo);
        if (c) atomicAdd((unsigned long long*)&P.pd->committed, (unsigned long long)c);
        if (ab) atomicAdd((unsigned long long*)&P.pd->aborted, (unsigned long long)ab);
        if (ran) atomicAdd((unsigned long long*)&P.pd->last_width, (unsigned long long)ran);
    }
}

// Compaction of the sorted operations: keep those of pending transactions.
__global__ __launch_bounds__(GTX_BLOCK) void k_pool_keep(PoolArgs P) {
    if (pool_failed(P)) return;
    const int64_t m = P.pd->m;
    const uint32_t* v = P.val[P.cur];
    __shared__ int lds[GTX_WAVES + 1];
    const int64_t base = (int64_t)blockIdx.x * kPoolTile;
    int cnt = 0;
#pragma unroll
    for (int j = 0; j < kPoolTile / GTX_BLOCK; ++j) {
        const int64_t i = base + j * GTX_BLOCK + threadIdx.x;
        if (i < m) cnt += P.state[v[i] >> 1] == 0;
    }
    int tot;
    block_excl_sum(cnt, &tot, lds);
    if (threadIdx.x == 0) P.tile_or[blockIdx.x] = tot;
}

__global__ __launch_bounds__(GTX_BLOCK) void k_pool_keep_scan(PoolArgs P) {
    if (pool_failed(P)) return;
    const int64_t m = P.pd->m;
    const int64_t tiles = (m + kPoolTile - 1) / kPoolTile;
    __shared__ int lds[GTX_WAVES + 1];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < tiles; c0 += GTX_BLOCK) {
        const int64_t t = c0 + threadIdx.x;
        const int v = t < tiles ? P.tile_or[t] : 0;
        int tot;
        const int ex = block_excl_sum(v, &tot, lds);
        if (t < tiles) P.tile_carry[t] = carry + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) P.keep[0] = carry;  // operations kept
}

__global__ __launch_bounds__(GTX_BLOCK) void k_pool_compact(PoolArgs P) {
    if (pool_failed(P)) return;
    const int64_t m = P.pd->m;
    const uint32_t* k = P.key[P.cur];
    const uint32_t* v = P.val[P.cur];
    uint32_t* nk = P.key[1 - P.cur];
    uint32_t* nv = P.val[1 - P.cur];
    __shared__ int lds[GTX_WAVES + 1];
    const int64_t base = (int64_t)blockIdx.x * kPoolTile;
    int run = base < m ? P.tile_carry[blockIdx.x] : 0;
#pragma unroll
    for (int j = 0; j < kPoolTile / GTX_BLOCK; ++j) {
        const int64_t i = base + j * GTX_BLOCK + threadIdx.x;
        const int keep = i < m && P.state[v[i] >> 1] == 0;
        int tot;
        const int ex = block_excl_sum(keep, &tot, lds);
        if (keep) {
            nk[run + ex] = k[i];
            nv[run + ex] = v[i];
        }
        run += tot;
    }
}

__global__ void k_pool_tail(PoolArgs P) {
    if (threadIdx.x != 0 || pool_failed(P)) return;
    P.pd->tail = (int64_t)P.pd->min_pending;  // every transaction below it has run
    P.pd->m = P.keep[0];
    if (P.pd->last_width > 0) P.pd->waves += 1;
    P.pd->executed += P.pd->last_width;
}

__global__ void k_pool_step_begin(PoolArgs P) {
    if (threadIdx.x == 0) {
        P.pd->last_width = 0;
        P.pd->min_pending = (unsigned long long)P.pd->head;
    }
}

}  // namespace gtx

using namespace gtx;

struct gputx_pool_t {
    gputx_handle h = nullptr;
    PoolArgs P{};
    PoolDev* pd = nullptr;
    char* mem = nullptr;     // the ring and the operation arrays
    void* ws = nullptr;      // front-end workspace for one added bulk
    size_t ws_bytes = 0;
    int64_t max_add = 0;
    int64_t head = 0;        // host copy of the sequence counter
    int64_t fetched = 0;     // results handed back (their slots are free)
    gputx_bulk_stats* stats = nullptr;
    int32_t* dummy_status = nullptr;
    int64_t* dummy_results = nullptr;
};

extern "C" int gputx_pool_create(gputx_handle h, int64_t capacity, int32_t n_params, int32_t width,
                                 int32_t max_ops, int64_t max_add, gputx_pool* out) {
    if (!h || !out || capacity < 1 || capacity > ((int64_t)1 << 26) || n_params < 1 || n_params > GTX_MAX_PARAMS ||
        width < 1 || max_ops < 0 || max_add < 1)
        return gtx_set_err(h, GPUTX_E_ARG, "bad pool arguments");
    *out = nullptr;
    HIP_OK(h, hipSetDevice(h->device));
    int64_t cap = 1;
    while (cap < capacity) cap <<= 1;
    const int mo = max_ops > 0 ? std::min(max_ops, h->max_ops) : h->max_ops;
    const int64_t mcap = cap * mo;
    const int64_t tiles = (mcap + kPoolTile - 1) / kPoolTile + 1;
    auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += up(std::max<size_t>(bytes, 1));
        return o;
    };
    const size_t o_pd = take(sizeof(PoolDev));
    const size_t o_type = take(cap * 4), o_params = take(cap * 8 * n_params), o_ts = take(cap * 8),
                 o_app = take(2 * cap * 8), o_state = take(cap * 4), o_blocked = take(cap * 4),
                 o_status = take(cap * 4), o_results = take(cap * 8 * width), o_k0 = take(mcap * 4),
                 o_k1 = take(mcap * 4), o_v0 = take(mcap * 4), o_v1 = take(mcap * 4), o_tor = take(tiles * 4),
                 o_tc = take(tiles * 4), o_keep = take(8), o_stats = take(sizeof(gputx_bulk_stats)),
                 o_dst = take(max_add * 4), o_dres = take(max_add * 8);
    gputx_pool_t* Q = new gputx_pool_t();
    Q->h = h;
    hipError_t e = hipMalloc(&Q->mem, off);
    if (e == hipSuccess) e = hipMemset(Q->mem, 0, off);
    Q->ws_bytes = gputx_workspace_size_ops(h, max_add, max_ops);
    if (e == hipSuccess) e = hipMalloc(&Q->ws, Q->ws_bytes);
    if (e != hipSuccess) {
        if (Q->mem) (void)hipFree(Q->mem);
        if (Q->ws) (void)hipFree(Q->ws);
        delete Q;
        return gtx_set_err(h, GPUTX_E_HIP, "pool allocation: %s", hipGetErrorString(e));
    }
    char* m = Q->mem;
    PoolArgs& P = Q->P;
    Q->pd = reinterpret_cast<PoolDev*>(m + o_pd);
    P.pd = Q->pd;
    P.cap = cap;
    P.n_params = n_params;
    P.width = width;
    P.max_ops = mo;
    P.cur = 0;
    P.types = h->d_types;
    P.rowcount = h->d_rowcount;
    P.n_app = h->n_app;
    P.type = reinterpret_cast<int32_t*>(m + o_type);
    P.params = reinterpret_cast<int64_t*>(m + o_params);
    P.ts = reinterpret_cast<int64_t*>(m + o_ts);
    P.app = reinterpret_cast<int64_t*>(m + o_app);
    P.state = reinterpret_cast<int32_t*>(m + o_state);
    P.blocked = reinterpret_cast<int32_t*>(m + o_blocked);
    P.status = reinterpret_cast<int32_t*>(m + o_status);
    P.results = reinterpret_cast<int64_t*>(m + o_results);
    P.key[0] = reinterpret_cast<uint32_t*>(m + o_k0);
    P.key[1] = reinterpret_cast<uint32_t*>(m + o_k1);
    P.val[0] = reinterpret_cast<uint32_t*>(m + o_v0);
    P.val[1] = reinterpret_cast<uint32_t*>(m + o_v1);
    P.tile_or = reinterpret_cast<int32_t*>(m + o_tor);
    P.tile_carry = reinterpret_cast<int32_t*>(m + o_tc);
    P.keep = reinterpret_cast<int32_t*>(m + o_keep);
    Q->stats = reinterpret_cast<gputx_bulk_stats*>(m + o_stats);
    Q->dummy_status = reinterpret_cast<int32_t*>(m + o_dst);
    Q->dummy_results = reinterpret_cast<int64_t*>(m + o_dres);
    Q->max_add = max_add;
    *out = Q;
    return GPUTX_OK;
}

extern "C" int gputx_pool_destroy(gputx_pool Q) {
    if (!Q) return GPUTX_E_ARG;
    (void)hipSetDevice(Q->h->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(Q->mem);
    (void)hipFree(Q->ws);
    delete Q;
    return GPUTX_OK;
}

extern "C" int gputx_pool_add(gputx_pool Q, const gputx_bulk* b, gputx_stream_t stream) {
    if (!Q || !b) return gtx_set_err(nullptr, GPUTX_E_ARG, "null argument");
    gputx_handle h = Q->h;
    if (b->n < 0 || b->n > Q->max_add) return gtx_set_err(h, GPUTX_E_ARG, "bulk of %lld > max_add", (long long)b->n);
    if (b->n == 0) return GPUTX_OK;
    if (Q->head + b->n - Q->fetched > Q->P.cap)
        return gtx_set_err(h, GPUTX_E_CAPACITY, "pool full: fetch results first");
    HIP_OK(h, hipSetDevice(h->device));
    BulkArgs a;
    gputx_bulk bb = *b;
    if (bb.max_ops == 0) bb.max_ops = Q->P.max_ops;
    // the bulk's own width: results are not written by the front end
    int rc = gtx_make_args(h, &bb, GPUTX_KSET, Q->ws, Q->ws_bytes, Q->dummy_status, Q->dummy_results, 1, Q->stats,
                           gtx_grid_for(h, 1), &a);
    if (rc) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    PhaseMarks none;
    a.part_early = 0;
    (void)launch_front(a, s, none);
    const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((b->n + GTX_BLOCK - 1) / GTX_BLOCK, 4096));
    PoolArgs P = Q->P;
    hipLaunchKernelGGL(k_pool_check, dim3(1), dim3(64), 0, s, a, P);
    hipLaunchKernelGGL(k_pool_ingest, dim3(nb), dim3(GTX_BLOCK), 0, s, a, P);
    const int64_t mtot = (int64_t)Q->P.cap * Q->P.max_ops;
    const unsigned nbm = (unsigned)std::max<int64_t>(1, std::min<int64_t>((mtot + GTX_BLOCK - 1) / GTX_BLOCK, 8192));
    hipLaunchKernelGGL(k_pool_merge, dim3(nbm), dim3(GTX_BLOCK), 0, s, a, P);
    hipLaunchKernelGGL(k_pool_merge_done, dim3(1), dim3(64), 0, s, a, P);
    hipLaunchKernelGGL(k_pool_commit_add, dim3(1), dim3(64), 0, s, a, P);
    Q->P.cur = 1 - Q->P.cur;
    Q->head += b->n;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return gtx_set_err(h, GPUTX_E_HIP, "pool add: %s", hipGetErrorString(e));
    return GPUTX_OK;
}

extern "C" int gputx_pool_step(gputx_pool Q, int32_t waves, gputx_stream_t stream) {
    if (!Q || waves < 1) return gtx_set_err(Q ? Q->h : nullptr, GPUTX_E_ARG, "bad step");
    gputx_handle h = Q->h;
    HIP_OK(h, hipSetDevice(h->device));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    const int64_t mtot = (int64_t)Q->P.cap * Q->P.max_ops;
    const unsigned tiles = (unsigned)((mtot + kPoolTile - 1) / kPoolTile);
    const unsigned nbs = (unsigned)std::max<int64_t>(1, std::min<int64_t>((Q->P.cap + GTX_BLOCK - 1) / GTX_BLOCK, 4096));
    for (int w = 0; w < waves; ++w) {
        PoolArgs P = Q->P;
        hipLaunchKernelGGL(k_pool_step_begin, dim3(1), dim3(64), 0, s, P);
        hipLaunchKernelGGL(k_pool_unblock, dim3(nbs), dim3(GTX_BLOCK), 0, s, P);
        hipLaunchKernelGGL(k_pool_scan_up, dim3(tiles), dim3(GTX_BLOCK), 0, s, P);
        hipLaunchKernelGGL(k_pool_scan_mid, dim3(1), dim3(GTX_BLOCK), 0, s, P);
        hipLaunchKernelGGL(k_pool_scan_down, dim3(tiles), dim3(GTX_BLOCK), 0, s, P);
        hipLaunchKernelGGL(k_pool_exec, dim3(nbs), dim3(GTX_BLOCK), 0, s, P);
        hipLaunchKernelGGL(k_pool_keep, dim3(tiles), dim3(GTX_BLOCK), 0, s, P);
        hipLaunchKernelGGL(k_pool_keep_scan, dim3(1), dim3(GTX_BLOCK), 0, s, P);
        hipLaunchKernelGGL(k_pool_compact, dim3(tiles), dim3(GTX_BLOCK), 0, s, P);
        hipLaunchKernelGGL(k_pool_tail, dim3(1), dim3(64), 0, s, P);
        Q->P.cur = 1 - Q->P.cur;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return gtx_set_err(h, GPUTX_E_HIP, "pool step: %s", hipGetErrorString(e));
    return GPUTX_OK;
}

extern "C" int gputx_pool_state(gputx_pool Q, gputx_pool_stats* out, gputx_stream_t stream) {
    if (!Q || !out) return gtx_set_err(nullptr, GPUTX_E_ARG, "null argument");
    gputx_handle h = Q->h;
    HIP_OK(h, hipSetDevice(h->device));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    PoolDev d{};
    HIP_OK(h, hipMemcpyAsync(&d, Q->pd, sizeof d, hipMemcpyDeviceToHost, s));
    HIP_OK(h, hipStreamSynchronize(s));
    out->error = d.error;
    out->reserved = 0;
    out->added = d.head;
    out->done_prefix = d.tail;
    out->pending_ops = d.m;
    out->waves = d.waves;
    out->executed = d.executed;
    out->committed = d.committed;
    out->aborted = d.aborted;
    out->invalid = d.invalid;
    out->last_width = d.last_width;
    out->fetched = Q->fetched;
    return GPUTX_OK;
}

extern "C" int gputx_pool_results(gputx_pool Q, int64_t n, int32_t* status, int64_t* results,
                                  gputx_stream_t stream) {
    if (!Q || n < 0 || (n > 0 && (!status || !results))) return gtx_set_err(nullptr, GPUTX_E_ARG, "bad arguments");
    gputx_handle h = Q->h;
    gputx_pool_stats st;
    int rc = gputx_pool_state(Q, &st, stream);
    if (rc) return rc;
    if (Q->fetched + n > st.done_prefix)
        return gtx_set_err(h, GPUTX_E_STATE, "only %lld transactions have run in sequence",
                           (long long)(st.done_prefix - Q->fetched));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t cap = Q->P.cap, W = Q->P.width;
    int64_t done = 0;
    while (done < n) {  // the ring may wrap: at most two pieces
        const int64_t slot = (Q->fetched + done) & (cap - 1);
        const int64_t c = std::min(n - done, cap - slot);
        HIP_OK(h, hipMemcpyAsync(status + done, Q->P.status + slot, c * 4, hipMemcpyDefault, s));
        HIP_OK(h, hipMemcpyAsync(results + done * W, Q->P.results + slot * W, c * 8 * W, hipMemcpyDefault, s));
        done += c;
    }
    HIP_OK(h, hipStreamSynchronize(s));
    Q->fetched += n;
    return GPUTX_OK;
}
