// Bulk generation: everything before a strategy runs (Sections 4.2 and 5).
//
//   k_reset        clear the bulk state
//   k_order_check  are the timestamps (transaction ids, Section 3.2) ascending?
//   [ts sort]      stable radix sort of the timestamps when they are not
//   k_ts_check     duplicate / unsorted timestamps are bulk errors
//   k_prepare      per serial position: type, validity, op and append counts
//   scan (3)       exclusive scans of the counts; append capacity check
//   k_emit         basic operations (item key, op index << 1 | write) in
//                  serial order; cross-partition count c; PART partition keys
//   [side stream]  one-bulk calls where PART may run: PART's partition sort,
//                  heads and records from here on, beside the next three steps
//   [op sort]      stable radix sort on the item key: Section 4.2 step 1
//   rank (3)       steps 2-3: group boundaries and per-op rank (three-phase
//                  segmented scan over the sorted operations); lock targets,
//                  successor ranges and in-edges come from a second downsweep
//                  launched with the executors, only when TPL or K-SET runs
//   k_features     steps 4-5 without a second sort: per-transaction max rank
//                  over its contiguous op range; w0, depth; Algorithm 1 picks
//                  the strategy
#include "engine.h"

namespace gtx {

__device__ __forceinline__ bool bulk_failed(const GtxState* st) { return ld_relaxed(&st->error) != 0; }
__device__ __forceinline__ void set_error(GtxState* st, int code) { atomicCAS(&st->error, 0, code); }
__device__ __forceinline__ int64_t gid() { return (int64_t)blockIdx.x * GTX_BLOCK + threadIdx.x; }
__device__ __forceinline__ int64_t input_index(const BulkArgs& a, int64_t p) {
    return a.ws.st->unsorted ? (int64_t)a.ws.tsv[0][p] : p;
}

__global__ __launch_bounds__(GTX_BLOCK) void k_reset(GtxState* st) {
    int* w = reinterpret_cast<int*>(st);
    for (int i = threadIdx.x; i < (int)(sizeof(GtxState) / 4); i += GTX_BLOCK) w[i] = 0;
}

__global__ __launch_bounds__(GTX_BLOCK) void k_order_check(BulkArgs a) {
    int64_t i = gid();
    bool uns = false, dup = false;
    if (i < a.n) {
        int64_t t = a.ts[i];
        if (i > 0) {
            int64_t prev = a.ts[i - 1];
            uns = t < prev;
            dup = t == prev;
        }
        if (!a.ts_sorted) {
            a.ws.tsk[0][i] = (uint64_t)t ^ 0x8000000000000000ull;  // order-preserving
            a.ws.tsv[0][i] = (uint32_t)i;
        }
    }
    if (__any(uns) && lane_id() == 0) atomicOr(&a.ws.st->unsorted, 1);
    if (__any(dup) && lane_id() == 0) atomicOr(&a.ws.st->dup_adj, 1);
}

__global__ __launch_bounds__(GTX_BLOCK) void k_ts_check(BulkArgs a) {
    GtxState* st = a.ws.st;
    const int uns = st->unsorted;
    int64_t i = gid();
    if (uns && !a.ts_sorted && i >= 1 && i < a.n && a.ws.tsk[0][i] == a.ws.tsk[0][i - 1])
        set_error(st, GPUTX_E_DUP_TS);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (a.ts_sorted && uns) set_error(st, GPUTX_E_UNSORTED);
        else if (!uns && st->dup_adj) set_error(st, GPUTX_E_DUP_TS);
    }
}

__global__ __launch_bounds__(GTX_BLOCK) void k_prepare(BulkArgs a) {
    GtxState* st = a.ws.st;
    if (bulk_failed(st)) return;
    __shared__ int tcount[GPUTX_MAX_TYPES];
    if (threadIdx.x < GPUTX_MAX_TYPES) tcount[threadIdx.x] = 0;
    __syncthreads();
    int ninv = 0;
    for (int64_t p = gid(); p < a.n; p += (int64_t)gridDim.x * GTX_BLOCK) {
        const int64_t i = input_index(a, p);
        const int32_t t = a.type[i];
        bool valid = false;
        int nops = 0, a0 = 0, a1 = 0, ai0 = -1, ai1 = -1;
        if (t >= 0 && t < GPUTX_MAX_TYPES && ((a.type_mask >> t) & 1u) && a.types[t].proc != 0) {
            const DevType& T = a.types[t];
            int64_t prm[GTX_MAX_PARAMS];
            load_params(a.params, a.n, min(a.n_params, T.n_params), i, prm);
            valid = txn_valid(T, prm);
            if (valid) {
                OpList L;
                txn_ops(T, prm, L);
                nops = L.n;
                txn_appends(T, prm, &a0, &a1);
                ai0 = T.app_idx[0];
                ai1 = T.app_idx[1];
            }
        }
        a.ws.tty[p] = valid ? t : -1;
        a.ws.cnt[p] = nops;
        for (int k = 0; k < a.n_app; ++k)
            a.ws.cnt[(int64_t)(1 + k) * a.n + p] = (k == ai0 ? a0 : 0) + (k == ai1 ? a1 : 0);
        if (valid) {
            atomicAdd(&tcount[t], 1);
        } else {
            ++ninv;
            a.status[i] = GPUTX_INVALID;
            for (int r = 0; r < a.width; ++r) a.results[i * a.width + r] = 0;
        }
    }
    ninv = wave_sum(ninv);
    if (lane_id() == 0 && ninv) atomicAdd((unsigned long long*)&st->invalid, (unsigned long long)ninv);
    __syncthreads();
    // per-block type counts; the scan's single workgroup adds them up
    if (threadIdx.x < GPUTX_MAX_TYPES) a.ws.tcnt_tmp[blockIdx.x * GPUTX_MAX_TYPES + threadIdx.x] = tcount[threadIdx.x];
}

// ---- exclusive scans of the per-position counts --------------------------
__global__ __launch_bounds__(GTX_BLOCK) void k_scan_up(BulkArgs a, int K, int nb) {
    if (bulk_failed(a.ws.st)) return;
    __shared__ int lds[GTX_WAVES + 1];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    for (int k = 0; k < K; ++k) {
        const int32_t* c = a.ws.cnt + (int64_t)k * a.n;
        int s = 0;
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) {
            int64_t idx = base + j * GTX_BLOCK + threadIdx.x;
            if (idx < a.n) s += c[idx];
        }
        int tot;
        block_excl_sum(s, &tot, lds);
        if (threadIdx.x == 0) a.ws.scan_tmp[k * nb + blockIdx.x] = tot;
    }
}

// Block k < K scans row k of the per-block sums; block K adds up the
// per-block type counts.  The rows are independent, so they run side by side.
__global__ __launch_bounds__(GTX_BLOCK) void k_scan_mid(BulkArgs a, int K, int nb) {
    GtxState* st = a.ws.st;
    if (bulk_failed(st)) return;
    __shared__ int lds[GTX_WAVES + 1];
    const int k = blockIdx.x;
    if (k < K) {
        int64_t running = 0;
        for (int c0 = 0; c0 < nb; c0 += GTX_BLOCK) {
            int idx = c0 + threadIdx.x;
            int v = idx < nb ? a.ws.scan_tmp[k * nb + idx] : 0;
            int tot;
            int ex = block_excl_sum(v, &tot, lds);
            if (idx < nb) a.ws.scan_tmp[k * nb + idx] = (int)running + ex;
            running += tot;
        }
        if (threadIdx.x == 0) {
            if (k == 0) {
                st->m = running;
                // (append capacity depends on the tables' row counts, so it is
                // checked at the start of execution, not here)
                if (running > a.mcap) set_error(st, GPUTX_E_CAPACITY);
            } else {
                st->app_total[k - 1] = running;
            }
        }
        return;
    }
    // type counts: 16 threads per type, each over a stride of the blocks
    __shared__ int part[GTX_BLOCK];
    const int nblk = (int)std::min<int64_t>(kPrepBlocks, (a.n + GTX_BLOCK - 1) / GTX_BLOCK);
    const int ty = threadIdx.x % GPUTX_MAX_TYPES, lane16 = threadIdx.x / GPUTX_MAX_TYPES;
    constexpr int kStride = GTX_BLOCK / GPUTX_MAX_TYPES;
    int c = 0;
#pragma unroll 8
    for (int b = lane16; b < nblk; b += kStride) c += a.ws.tcnt_tmp[b * GPUTX_MAX_TYPES + ty];
    part[threadIdx.x] = c;
    __syncthreads();
    if (threadIdx.x < GPUTX_MAX_TYPES) {
        int tot = 0;
        for (int j = 0; j < kStride; ++j) tot += part[j * GPUTX_MAX_TYPES + threadIdx.x];
        st->type_count[threadIdx.x] = tot;
    }
}

__global__ __launch_bounds__(GTX_BLOCK) void k_scan_down(BulkArgs a, int K, int nb) {
    if (bulk_failed(a.ws.st)) return;
    __shared__ int lds[GTX_WAVES + 1];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    for (int k = 0; k < K; ++k) {
        int32_t* c = a.ws.cnt + (int64_t)k * a.n;
        int v[kScanItems];
        int s = 0;
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) {
            int64_t idx = base + j;
            v[j] = idx < a.n ? c[idx] : 0;
            s += v[j];
        }
        int tot;
        int run = block_excl_sum(s, &tot, lds) + a.ws.scan_tmp[k * nb + blockIdx.x];
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) {
            int64_t idx = base + j;
            if (idx < a.n) c[idx] = run;
            run += v[j];
        }
    }
}

// ---- basic operations in serial order -----------------------------------
__global__ __launch_bounds__(GTX_BLOCK) void k_emit(BulkArgs a) {
    GtxState* st = a.ws.st;
    if (bulk_failed(st)) return;
    const int64_t p = gid();
    bool cross = false;
    if (p < a.n) {
        uint32_t qkey = (uint32_t)a.n_parts;  // sentinel partition: not executed by PART
        const int32_t t = a.ws.tty[p];
        if (t >= 0) {
            const DevType& T = a.types[t];
            int64_t prm[GTX_MAX_PARAMS];
            load_params(a.params, a.n, min(a.n_params, T.n_params), input_index(a, p), prm);
            OpList L;
            txn_ops(T, prm, L);
            const int64_t off = a.ws.cnt[p];
            int64_t pid0 = L.pid[0];
            cross = pid0 < 0;
#pragma unroll
            for (int j = 0; j < GTX_MAX_OPS; ++j) {
                if (j < L.n) {
                    a.ws.pk[0][off + j] = L.key[j];
                    a.ws.pv[0][off + j] = (uint32_t)((off + j) << 1) | L.w[j];
                    a.ws.op_txn[off + j] = (int32_t)p;
                    cross = cross || L.pid[j] != pid0;
                }
            }
            if (!cross) qkey = (uint32_t)pid0;
        }
        a.ws.qk[0][p] = qkey;
        a.ws.qv[0][p] = (uint32_t)p;
    }
    int nc = wave_sum(cross ? 1 : 0);
    if (lane_id() == 0 && nc) atomicAdd((unsigned long long*)&st->cross, (unsigned long long)nc);
}

// ---- ranking scan over the (item, serial position)-sorted operations -----
__device__ __forceinline__ RankAgg agg_identity() {
    RankAgg r;
    r.segf = 0; r.segs = 0; r.gs = -1; r.A = 0; r.g = 0; r.B = INT32_MAX;
    return r;
}
// a precedes b
__device__ __forceinline__ RankAgg agg_combine(const RankAgg& a, const RankAgg& b) {
    RankAgg r;
    r.segf = a.segf | b.segf;
    r.segs = b.segf ? b.segs : a.segs + b.segs;
    r.gs = max(a.gs, b.gs);
    r.A = max(a.A, b.A);
    r.g = a.g + b.g;
    r.B = min(a.B, b.B);
    return r;
}
// Element i: a group starts where the item key changes; the paper's rank
// grows by one unless both this op and the previous one read (Section 4.2).
__device__ __forceinline__ RankAgg agg_element(int32_t i, bool start, bool w, bool wprev) {
    RankAgg r;
    r.segf = start;
    r.segs = start ? 0 : ((w || wprev) ? 1 : 0);
    r.gs = start ? i : -1;
    r.A = w ? i + 1 : 0;
    r.g = start ? 1 : 0;
    r.B = (w || start) ? i : INT32_MAX;
    return r;
}

__device__ __forceinline__ RankAgg shfl_up_agg(const RankAgg& v, int d) {
    RankAgg r;
    r.segf = __shfl_up(v.segf, d); r.segs = __shfl_up(v.segs, d); r.gs = __shfl_up(v.gs, d);
    r.A = __shfl_up(v.A, d); r.g = __shfl_up(v.g, d); r.B = __shfl_up(v.B, d);
    return r;
}

// Block exclusive scan (forward fields) of one aggregate per thread.
__device__ RankAgg block_excl_agg(RankAgg v, RankAgg* lds /* GTX_WAVES */) {
    RankAgg inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        RankAgg u = shfl_up_agg(inc, d);
        if (lane_id() >= d) inc = agg_combine(u, inc);
    }
    RankAgg ex = shfl_up_agg(inc, 1);
    if (lane_id() == 0) ex = agg_identity();
    if (lane_id() == 63) lds[wave_id()] = inc;
    __syncthreads();
    RankAgg pre = agg_identity();
    for (int w = 0; w < wave_id(); ++w) pre = agg_combine(pre, lds[w]);
    __syncthreads();
    return agg_combine(pre, ex);
}
// Block exclusive suffix minimum of one value per thread.
__device__ int block_excl_suffix_min(int v, int* lds /* GTX_WAVES */) {
    int inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int u = __shfl_down(inc, d);
        if (lane_id() + d < 64) inc = min(inc, u);
    }
    int ex = __shfl_down(inc, 1);
    if (lane_id() == 63) ex = INT32_MAX;
    if (lane_id() == 0) lds[wave_id()] = inc;
    __syncthreads();
    int suf = INT32_MAX;
    for (int w = wave_id() + 1; w < GTX_WAVES; ++w) suf = min(suf, lds[w]);
    __syncthreads();
    return min(suf, ex);
}

struct RankIn {
    const uint32_t* key;
    const uint32_t* val;
};
__device__ __forceinline__ RankIn rank_input(const BulkArgs& a) {
    int src = a.key_passes & 1;
    RankIn r;
    r.key = a.ws.pk[src];
    r.val = a.ws.pv[src];
    return r;
}

__global__ __launch_bounds__(GTX_BLOCK) void k_rank_up(BulkArgs a) {
    const GtxState* st = a.ws.st;
    if (bulk_failed(st)) return;
    __shared__ RankAgg lds[GTX_WAVES];
    const int32_t m = (int32_t)st->m;
    const int64_t base = (int64_t)blockIdx.x * kRankTile;
    if (base >= m) return;
    RankIn in = rank_input(a);
    RankAgg t = agg_identity();
    const int64_t i0 = base + (int64_t)threadIdx.x * kRankItems;
    uint32_t kprev = i0 > 0 && i0 <= m ? in.key[i0 - 1] : 0u;
    bool wprev = i0 > 0 && i0 <= m ? (in.val[i0 - 1] & 1u) : false;
#pragma unroll
    for (int j = 0; j < kRankItems; ++j) {
        int64_t i = i0 + j;
        if (i < m) {
            uint32_t k = in.key[i];
            bool w = in.val[i] & 1u;
            bool start = (i == 0) || k != kprev;
            t = agg_combine(t, agg_element((int32_t)i, start, w, wprev));
            kprev = k;
            wprev = w;
        }
    }
    RankAgg ex = block_excl_agg(t, lds);
    int bmin = block_excl_suffix_min(t.B, (int*)lds);
    RankAgg* out = &a.ws.rank_tmp[blockIdx.x];
    if (threadIdx.x == GTX_BLOCK - 1) {  // forward fields: prefix of the last thread + its own
        RankAgg tot = agg_combine(ex, t);
        out->segf = tot.segf;
        out->segs = tot.segs;
        out->gs = tot.gs;
        out->A = tot.A;
        out->g = tot.g;
    }
    if (threadIdx.x == 0) out->B = min(bmin, t.B);  // suffix after thread 0 + its own
}

// One workgroup: carries between tiles (forward prefix; suffix minimum of B).
__global__ __launch_bounds__(GTX_BLOCK) void k_rank_mid(BulkArgs a, int nb_cap) {
    const GtxState* st = a.ws.st;
    if (bulk_failed(st)) return;
    __shared__ RankAgg lds[GTX_WAVES];
    const int32_t m = (int32_t)st->m;
    const int nb = (int)((m + kRankTile - 1) / kRankTile);
    const int per = (nb + GTX_BLOCK - 1) / GTX_BLOCK;
    const int b0 = threadIdx.x * per;
    RankAgg t = agg_identity();
    for (int b = b0; b < b0 + per && b < nb; ++b) t = agg_combine(t, a.ws.rank_tmp[b]);
    RankAgg pre = block_excl_agg(t, lds);
    int suf = block_excl_suffix_min(t.B, (int*)lds);
    // forward carries in order; B suffix carries walking backwards
    RankAgg run = pre;
    for (int b = b0; b < b0 + per && b < nb; ++b) {
        RankAgg cur = a.ws.rank_tmp[b];
        RankAgg out = run;
        a.ws.rank_tmp[nb_cap + b] = out;
        run = agg_combine(run, cur);
    }
    int rb = suf;
    for (int b = min(b0 + per, nb) - 1; b >= b0; --b) {
        int cb = a.ws.rank_tmp[b].B;
        a.ws.rank_tmp[nb_cap + b].B = rb;
        rb = min(rb, cb);
    }
}

// Downsweep of the ranking scan.  The front end (kFull = false) keeps only
// each operation's rank, all that the features need; the lock and k-set
// executors' wait targets, groups and successor ranges (kFull = true) are
// written by a second downsweep over the same sorted pairs and carries, only
// when one of those executors was chosen.
template <bool kFull>
__global__ __launch_bounds__(GTX_BLOCK) void k_rank_down(BulkArgs a, int nb_cap) {
    const GtxState* st = a.ws.st;
    if (bulk_failed(st)) return;
    if (kFull && st->chosen != GPUTX_TPL && st->chosen != GPUTX_KSET) return;
    __shared__ RankAgg lds[GTX_WAVES];
    const int32_t m = (int32_t)st->m;
    const int64_t base = (int64_t)blockIdx.x * kRankTile;
    if (base >= m) return;
    RankIn in = rank_input(a);
    const RankAgg carry = a.ws.rank_tmp[nb_cap + blockIdx.x];
    const int64_t i0 = base + (int64_t)threadIdx.x * kRankItems;

    uint32_t key[kRankItems];
    uint32_t val[kRankItems];
    RankAgg el[kRankItems];
    RankAgg t = agg_identity();
    uint32_t kprev = i0 > 0 && i0 <= m ? in.key[i0 - 1] : 0u;
    bool wprev = i0 > 0 && i0 <= m ? (in.val[i0 - 1] & 1u) : false;
#pragma unroll
    for (int j = 0; j < kRankItems; ++j) {
        int64_t i = i0 + j;
        key[j] = i < m ? in.key[i] : 0u;
        val[j] = i < m ? in.val[i] : 0u;
        bool w = val[j] & 1u;
        bool start = (i == 0) || key[j] != kprev;
        el[j] = i < m ? agg_element((int32_t)i, start, w, wprev) : agg_identity();
        t = agg_combine(t, el[j]);
        kprev = key[j];
        wprev = w;
    }
    RankAgg pre = agg_combine(carry, block_excl_agg(t, lds));
    int bsuf = min(carry.B, block_excl_suffix_min(t.B, (int*)lds));
    // exclusive suffix minimum of B per element
    int bex[kRankItems];
    {
        int run = bsuf;
#pragma unroll
        for (int j = kRankItems - 1; j >= 0; --j) {
            bex[j] = run;
            run = min(run, el[j].B);
        }
    }
    // element after this thread's last (for write successors)
    const int64_t ilast = i0 + kRankItems;
    uint32_t knext_tail = ilast < m ? in.key[ilast] : 0u;
    bool wnext_tail = ilast < m ? (in.val[ilast] & 1u) : false;

    RankAgg cur = pre;
#pragma unroll
    for (int j = 0; j < kRankItems; ++j) {
        const int64_t i = i0 + j;
        if (i >= m) break;
        const int32_t Aex = cur.A;  // last write before i, + 1
        cur = agg_combine(cur, el[j]);
        const int32_t gs = cur.gs;
        const int32_t g = cur.g - 1;
        const int32_t rank = cur.segs;
        const bool w = val[j] & 1u;
        const int32_t o = (int32_t)(val[j] >> 1);
        const int32_t rs = max(gs, Aex);  // start of the read run that ends at i
        const int32_t rel = (int32_t)i - gs;
        // lock target: completed ops of the group this op waits for
        const int32_t tgt = w ? rel : rs - gs;
        int32_t slo = 0, shi = 0, in_c = 0;
        const int32_t Bx = bex[j];
        if (w) {
            uint32_t kn = (j + 1 < kRankItems) ? key[j + 1] : knext_tail;
            bool wn = (j + 1 < kRankItems) ? (val[j + 1] & 1u) : wnext_tail;
            if (i + 1 < m && kn == key[j]) {
                slo = (int32_t)i + 1;
                shi = wn ? (int32_t)i + 2 : min(Bx, m);  // run may reach the end
            }
            in_c = (i == gs) ? 0 : (rs == i ? 1 : (int32_t)i - rs);
        } else {
            if (Bx < m && in.key[Bx] == key[j]) {
                slo = Bx;
                shi = Bx + 1;
            }
            in_c = Aex > gs ? 1 : 0;
        }
        if (!kFull) {
            a.ws.op_rank[o] = rank;
            continue;
        }
        OpInfo inf;
        inf.grp = g;
        inf.tgt = tgt;
        inf.slo = slo;
        inf.shi = shi;
        inf.rank = rank;
        inf.in = in_c;
        inf.s0 = -1;    // filled by kset_succ when K-SET runs
        inf.s0ty = -1;
        a.ws.op_info[o] = inf;
        if (i == gs) a.ws.grp_cnt[g] = 0;
    }
}

// ---- features and Algorithm 1 --------------------------------------------
__global__ __launch_bounds__(GTX_BLOCK) void k_features(BulkArgs a) {
    GtxState* st = a.ws.st;
    if (bulk_failed(st)) return;
    __shared__ uint32_t is_last;
    __shared__ int red[2][GTX_WAVES];
    int zero = 0, dmax = 0;
    for (int64_t p = gid(); p < a.n; p += (int64_t)gridDim.x * GTX_BLOCK) {
        int mr = 0;
        // Section 4.2 steps 4-5: a transaction's k-set rank is the maximum
        // rank of its operations (reduced over its contiguous op range); the
        // first four ranks are loaded together
        const int32_t ty = a.ws.tty[p];
        const int64_t o0 = a.ws.cnt[p];
        const int64_t o1 = p + 1 < a.n ? (int64_t)a.ws.cnt[p + 1] : st->m;
        if (ty >= 0) {
            int32_t r[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) r[k] = o0 + k < o1 ? a.ws.op_rank[o0 + k] : 0;
            mr = max(max(r[0], r[1]), max(r[2], r[3]));
            for (int64_t o = o0 + 4; o < o1; ++o) mr = max(mr, a.ws.op_rank[o]);
            zero += mr == 0;
            dmax = max(dmax, mr);
        }
        a.ws.maxrank[p] = mr;
    }
    int z = wave_sum(zero);
    int d = wave_max(dmax);
    if (lane_id() == 0) {
        red[0][wave_id()] = z;
        red[1][wave_id()] = d;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int zz = 0, dd = 0;
        for (int w = 0; w < GTX_WAVES; ++w) {
            zz += red[0][w];
            dd = max(dd, red[1][w]);
        }
        if (zz) atomicAdd((unsigned long long*)&st->w0, (unsigned long long)zz);
        if (dd) atomicMax((unsigned long long*)&st->depth, (unsigned long long)dd);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        fence_release();
        is_last = atomicAdd(&st->done_ctr[0], 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!is_last || threadIdx.x != 0) return;
    fence_acquire();
    const int64_t w0 = ld_relaxed(&st->w0), depth = ld_relaxed(&st->depth);
    const int64_t cross = ld_relaxed(&st->cross);
    int chosen = a.strategy;
    if (chosen == GPUTX_AUTO) {  // Algorithm 1 (Appendix D)
        if (w0 >= a.w0_bar) chosen = GPUTX_KSET;
        else if (cross <= a.c_bar || depth >= a.d_bar) chosen = GPUTX_PART;
        else chosen = GPUTX_TPL;
    }
    // Section 5.2: cross-partition transactions run under TPL
    if (chosen == GPUTX_PART && cross > 0) chosen = GPUTX_TPL;
    st->chosen = chosen;
    st->run_part = chosen == GPUTX_PART;
}

// ---- host side ------------------------------------------------------------
static unsigned blocks_for(int64_t n, int64_t per) { return (unsigned)std::max<int64_t>(1, (n + per - 1) / per); }

hipError_t launch_front(const BulkArgs& a, hipStream_t s, const PhaseMarks& pm, const SideLane* side) {
    pm.mark(PH_START, s);
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(GTX_BLOCK), 0, s, a.ws.st);
    hipLaunchKernelGGL(k_order_check, dim3(blocks_for(a.n, GTX_BLOCK)), dim3(GTX_BLOCK), 0, s, a);
    if (!a.ts_sorted) {
        SortPlan sp{};
        sp.key_bytes = 8;
        sp.keys[0] = a.ws.tsk[0]; sp.keys[1] = a.ws.tsk[1];
        sp.vals[0] = a.ws.tsv[0]; sp.vals[1] = a.ws.tsv[1];
        sp.hist = a.ws.sort_hist; sp.status = a.ws.sort_status; sp.ctrl = a.ws.sort_ctrl;
        sp.cap = a.n; sp.count_dev = nullptr; sp.npass = 8;
        sp.gate = &a.ws.st->unsorted; sp.st = a.ws.st; sp.spin_ticks = a.spin_ticks;
        sort_pairs(sp, s);  // 8 passes: result back in buffer 0
    }
    hipLaunchKernelGGL(k_ts_check, dim3(blocks_for(a.n, GTX_BLOCK)), dim3(GTX_BLOCK), 0, s, a);
    pm.mark(PH_ORDER, s);
    hipLaunchKernelGGL(k_prepare, dim3(std::min<unsigned>(kPrepBlocks, blocks_for(a.n, GTX_BLOCK))), dim3(GTX_BLOCK), 0, s, a);
    const int K = 1 + a.n_app;
    const int nb = (int)blocks_for(a.n, kScanTile);
    hipLaunchKernelGGL(k_scan_up, dim3(nb), dim3(GTX_BLOCK), 0, s, a, K, nb);
    hipLaunchKernelGGL(k_scan_mid, dim3(K + 1), dim3(GTX_BLOCK), 0, s, a, K, nb);
    hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(GTX_BLOCK), 0, s, a, K, nb);
    pm.mark(PH_PREPARE, s);
    hipLaunchKernelGGL(k_emit, dim3(blocks_for(a.n, GTX_BLOCK)), dim3(GTX_BLOCK), 0, s, a);
    pm.mark(PH_EMIT, s);
    // PART's partition ids are known once the operations are emitted: with a
    // side lane, its sort, heads and records run beside the item-key sort and
    // the ranking
    const bool early = side && a.part_early;
    hipError_t e = hipSuccess;
    if (early) {
        e = hipEventRecord(side->fork, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(side->s, side->fork, 0);
        if (e != hipSuccess) return e;
        launch_part_sort(a, side->s);
    }
    {
        SortPlan sp{};
        sp.key_bytes = 4;
        sp.keys[0] = a.ws.pk[0]; sp.keys[1] = a.ws.pk[1];
        sp.vals[0] = a.ws.pv[0]; sp.vals[1] = a.ws.pv[1];
        sp.hist = a.ws.sort_hist; sp.status = a.ws.sort_status; sp.ctrl = a.ws.sort_ctrl;
        sp.cap = a.mcap; sp.count_dev = &a.ws.st->m; sp.npass = a.key_passes;
        sp.gate = nullptr; sp.st = a.ws.st; sp.spin_ticks = a.spin_ticks;
        sort_pairs(sp, s);
    }
    pm.mark(PH_OPSORT, s);
    if (early) {
        // PART's records are written beside the ranking rather than beside
        // the item-key sort: both move much of the bulk through HBM, and the
        // sort's last pass ran twice as long with the gather beside it
        e = hipEventRecord(side->sorted, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(side->s, side->sorted, 0);
        if (e != hipSuccess) return e;
        launch_part_gather(a, side->s);
        e = hipEventRecord(side->join, side->s);
        if (e != hipSuccess) return e;
    }
    const int nbr = (int)blocks_for(a.mcap, kRankTile);
    hipLaunchKernelGGL(k_rank_up, dim3(nbr), dim3(GTX_BLOCK), 0, s, a);
    hipLaunchKernelGGL(k_rank_mid, dim3(1), dim3(GTX_BLOCK), 0, s, a, nbr);
    hipLaunchKernelGGL(k_rank_down<false>, dim3(nbr), dim3(GTX_BLOCK), 0, s, a, nbr);
    pm.mark(PH_RANK, s);
    // each workgroup ends with three atomics on the same words, which the
    // device serialises: a small grid (256 workgroups: 23 us at 2^20 against
    // 31 us with 1024 and 89 us with 4096) beats one transaction per thread
    hipLaunchKernelGGL(k_features, dim3(std::min<unsigned>(256, blocks_for(a.n, GTX_BLOCK))), dim3(GTX_BLOCK), 0, s, a);
    pm.mark(PH_FEATURES, s);
    if (early) e = hipStreamWaitEvent(s, side->join, 0);
    return e;
}

// Bulk generation without the timestamp constraint (Appendix G): no
// timestamp order, no operation sort, no ranking -- validation, the count
// scans (append slots in input order) and the basic operations only.
void launch_front_relaxed(const BulkArgs& a, hipStream_t s, const PhaseMarks& pm) {
    pm.mark(PH_START, s);
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(GTX_BLOCK), 0, s, a.ws.st);
    pm.mark(PH_ORDER, s);
    hipLaunchKernelGGL(k_prepare, dim3(std::min<unsigned>(kPrepBlocks, blocks_for(a.n, GTX_BLOCK))), dim3(GTX_BLOCK), 0, s, a);
    const int K = 1 + a.n_app;
    const int nb = (int)blocks_for(a.n, kScanTile);
    hipLaunchKernelGGL(k_scan_up, dim3(nb), dim3(GTX_BLOCK), 0, s, a, K, nb);
    hipLaunchKernelGGL(k_scan_mid, dim3(K + 1), dim3(GTX_BLOCK), 0, s, a, K, nb);
    hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(GTX_BLOCK), 0, s, a, K, nb);
    pm.mark(PH_PREPARE, s);
    hipLaunchKernelGGL(k_emit, dim3(blocks_for(a.n, GTX_BLOCK)), dim3(GTX_BLOCK), 0, s, a);
    pm.mark(PH_EMIT, s);
    pm.mark(PH_OPSORT, s);
    pm.mark(PH_RANK, s);
}

void launch_rank_full(const BulkArgs& a, hipStream_t s) {
    const int nbr = (int)blocks_for(a.mcap, kRankTile);
    hipLaunchKernelGGL(k_rank_down<true>, dim3(nbr), dim3(GTX_BLOCK), 0, s, a, nbr);
}

}  // namespace gtx
