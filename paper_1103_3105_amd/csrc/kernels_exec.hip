// Bulk execution strategies (Section 5) and the batched update.
//
//   k_kset     K-SET (Section 5.3): take the 0-set, run it without locks,
//              remove it; the 1-set becomes the new 0-set.  Kahn frontier over
//              the operation successor ranges, so wave k is exactly the k-set
//              (Properties 1-2).  Persistent grid, one grid barrier per wave;
//              the next frontier is built into per-type regions, so every
//              wave64 runs a single procedure (Section 5.4 grouping for free).
//   k_tpl      TPL (Section 5.1, Appendix C): counter-based locks.  Each
//              operation waits until its item's completion counter reaches its
//              target, the transaction runs, every counter is incremented.
//              Workgroups claim 256-transaction windows in timestamp order
//              and group each window by type.
//   k_part_gather PART: every transaction's record (input index, type,
//              parameters) at its partition-sorted position, so that a
//              partition's records lie together, and its appended rows; in
//              the one-bulk call it runs ahead of the choice on a second stream.
//   k_part_pipe PART (Section 5.2), few long partitions: one workgroup per
//              partition; staging waves put each chunk's cells in an LDS
//              table while the serial wave runs the previous chunk against
//              it, in timestamp order (one transaction at a time, or a
//              window of 64 as a scan over each cell's updates when the
//              procedure's effect on each cell is a map of the cell alone).
//              k_part_wave is the one-wave form (stage, then run).
//   k_part     PART, many small partitions: one lane per partition runs its
//              transactions one after another.
//   k_finalize batched update (Section 3.2): advance append-table row counts;
//              publish statistics.
#include "engine.h"

namespace gtx {

__device__ __forceinline__ bool failed(const GtxState* st) { return ld_relaxed(&st->error) != 0; }
__device__ __forceinline__ void fail(GtxState* st, int code) { atomicCAS(&st->error, 0, code); }

__device__ __forceinline__ int64_t in_index(const BulkArgs& a, int64_t p) {
    return a.ws.st->unsorted ? (int64_t)a.ws.tsv[0][p] : p;
}

// One transaction's signature, loaded and ready to run.
struct TxnIn {
    int64_t i;     // input index (status / results slot)
    int64_t ts;
    int64_t app0;  // rows its appends occupy
    int64_t app1;
    int32_t t;     // registered type
    int32_t np;    // parameters loaded
    int64_t prm[GTX_MAX_PARAMS];
};

// The type descriptors do not change while a kernel runs.  One that is the
// same for the whole wave is read through the constant address space, so
// the compiler can use scalar loads: their completion is counted apart from
// the vector memory operations, and waiting for a descriptor field then does
// not also wait for reads and stores in flight (the staging lanes' records
// read a step ahead, the serial waves' outcomes of the chunk before).
#define GTX_CONST __attribute__((address_space(4)))
__device__ __forceinline__ DevType dev_type_uniform(const DevType* types, int t) {
#if defined(__HIP_DEVICE_COMPILE__)
    return ((const GTX_CONST DevType*)(uintptr_t)types)[__builtin_amdgcn_readfirstlane(t)];
#else
    return types[t];  // the host pass only parses device functions
#endif
}

__device__ __forceinline__ void load_txn(const BulkArgs& a, const DevType& T, int64_t p, int32_t t, TxnIn& x) {
    x.t = t;
    x.i = in_index(a, p);
    x.np = min(a.n_params, T.n_params);
    load_params(a.params, a.n, x.np, x.i, x.prm);
    x.ts = a.ts[x.i];
    x.app0 = T.app_idx[0] >= 0 ? a.rowcount[T.app_idx[0]] + a.ws.cnt[(int64_t)(1 + T.app_idx[0]) * a.n + p] : 0;
    x.app1 = T.app_idx[1] >= 0 ? a.rowcount[T.app_idx[1]] + a.ws.cnt[(int64_t)(1 + T.app_idx[1]) * a.n + p] : 0;
}
__device__ __forceinline__ void load_txn(const BulkArgs& a, int64_t p, int32_t t, TxnIn& x) {
    load_txn(a, a.types[t], p, t, x);
}

__device__ __forceinline__ int64_t rl64(int64_t v, int k) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, k);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), k);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Lane k's signature, broadcast to the whole wave (uniform values).
__device__ __forceinline__ void bcast_txn(const TxnIn& x, int k, TxnIn& y) {
    y.t = __builtin_amdgcn_readlane(x.t, k);
    y.np = __builtin_amdgcn_readlane(x.np, k);
    y.i = rl64(x.i, k);
    y.ts = rl64(x.ts, k);
    y.app0 = rl64(x.app0, k);
    y.app1 = rl64(x.app1, k);
#pragma unroll
    for (int q = 0; q < GTX_MAX_PARAMS; ++q) y.prm[q] = q < y.np ? rl64(x.prm[q], k) : 0;
}

__device__ __forceinline__ int32_t exec_txn(const BulkArgs& a, const TxnIn& x) {
    int64_t res[GTX_MAX_RESULTS];
    const int32_t s = txn_exec(a.types[x.t], x.prm, x.ts, x.app0, x.app1, res);
    a.status[x.i] = s;
    int64_t* out = a.results + x.i * a.width;
#pragma unroll
    for (int r = 0; r < GTX_MAX_RESULTS; ++r)
        if (r < a.width) out[r] = res[r];
    for (int r = GTX_MAX_RESULTS; r < a.width; ++r) out[r] = 0;
    return s;
}

// exec_txn with the cells accessed coherently across the device (CoherentAcc).
// tu >= 0: every active lane's transaction has type tu.  For the narrow
// procedures of fixed columns its descriptor is then read through scalar
// loads (dev_type_uniform), one copy per procedure; the others (and mixed
// waves) keep the per-lane read, which keeps this hot loop's code small.
__device__ __forceinline__ int32_t exec_txn_coherent(const BulkArgs& a, const TxnIn& x, int32_t tu = -1) {
    int64_t res[GTX_MAX_RESULTS];
    CoherentAcc acc;
    int32_t s;
    const int pu = tu >= 0 ? dev_type_uniform(a.types, tu).proc : 0;
    switch (pu) {
#define GTX_TPL_CASE(P)                                                              \
    case P: {                                                                        \
        const DevType T = dev_type_uniform(a.types, tu);                             \
        s = txn_exec_p<P>(acc, T, x.prm, x.ts, x.app0, x.app1, res);                 \
        break;                                                                       \
    }
        GTX_TPL_CASE(GPUTX_DEBIT_CREDIT)
        GTX_TPL_CASE(GPUTX_PAYMENT)
        GTX_TPL_CASE(GPUTX_ORDER_STATUS)
#undef GTX_TPL_CASE
    default:
        s = txn_exec_any(acc, a.types[x.t], x.prm, x.ts, x.app0, x.app1, res);
    }
    a.status[x.i] = s;
    int64_t* out = a.results + x.i * a.width;
#pragma unroll
    for (int r = 0; r < GTX_MAX_RESULTS; ++r)
        if (r < a.width) out[r] = res[r];
    for (int r = GTX_MAX_RESULTS; r < a.width; ++r) out[r] = 0;
    return s;
}

// exec_txn for a chunk whose transactions all run procedure P: the type
// descriptor is read once per chunk by the caller.
template <int P>
__device__ __forceinline__ int32_t exec_txn_p(const BulkArgs& a, const DevType& T, const TxnIn& x) {
    int64_t res[GTX_MAX_RESULTS];
    DirectAcc acc;
    const int32_t s = txn_exec_p<P>(acc, T, x.prm, x.ts, x.app0, x.app1, res);
    a.status[x.i] = s;
    int64_t* out = a.results + x.i * a.width;
#pragma unroll
    for (int r = 0; r < GTX_MAX_RESULTS; ++r)
        if (r < a.width) out[r] = res[r];
    for (int r = GTX_MAX_RESULTS; r < a.width; ++r) out[r] = 0;
    return s;
}

// Run the transaction at serial position p (type t >= 0); returns its status.
__device__ int32_t run_at(const BulkArgs& a, int64_t p, int32_t t) {
    TxnIn x;
    load_txn(a, p, t, x);
    return exec_txn(a, x);
}

// run_at without the transaction's appends (written beforehand).
__device__ int32_t run_at_noapp(const BulkArgs& a, int64_t p, int32_t t) {
    TxnIn x;
    load_txn(a, p, t, x);
    int64_t res[GTX_MAX_RESULTS];
    NoAppendAcc acc;
    const int32_t s = txn_exec_any(acc, a.types[x.t], x.prm, x.ts, x.app0, x.app1, res);
    a.status[x.i] = s;
    int64_t* out = a.results + x.i * a.width;
#pragma unroll
    for (int r = 0; r < GTX_MAX_RESULTS; ++r)
        if (r < a.width) out[r] = res[r];
    for (int r = GTX_MAX_RESULTS; r < a.width; ++r) out[r] = 0;
    return s;
}

__device__ __forceinline__ void count_status(GtxState* st, bool ran, int32_t s) {
    int c = wave_sum(ran && s == GPUTX_COMMIT ? 1 : 0);
    int ab = wave_sum(ran && s == GPUTX_ABORT ? 1 : 0);
    if (lane_id() == 0) {
        if (c) atomicAdd((unsigned long long*)&st->committed, (unsigned long long)c);
        if (ab) atomicAdd((unsigned long long*)&st->aborted, (unsigned long long)ab);
    }
}

__device__ __forceinline__ void add_counts(GtxState* st, int64_t committed, int64_t aborted) {
    long long c = wave_sum64(committed), ab = wave_sum64(aborted);
    if (lane_id() == 0) {
        if (c) atomicAdd((unsigned long long*)&st->committed, (unsigned long long)c);
        if (ab) atomicAdd((unsigned long long*)&st->aborted, (unsigned long long)ab);
    }
}

__device__ __forceinline__ int64_t op_begin(const BulkArgs& a, int64_t p) { return a.ws.cnt[p]; }
__device__ __forceinline__ int64_t op_end(const BulkArgs& a, int64_t p) {
    return p + 1 < a.n ? (int64_t)a.ws.cnt[p + 1] : a.ws.st->m;
}

// Software grid barrier for a persistent, fully resident grid.  Returns false
// when the bulk failed (watchdog or error elsewhere): the caller then exits.
__device__ bool grid_barrier(GtxState* st, uint64_t spin_ticks) {
    __shared__ int ok_s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        const uint32_t gen = ld_relaxed(&st->bar_gen);
        fence_release();
        const uint32_t arrived = atomicAdd(&st->bar_count, 1u);
        if (arrived == gridDim.x - 1) {
            st_relaxed(&st->bar_count, 0u);
            __hip_atomic_store(&st->bar_gen, gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            uint64_t t0 = now_ticks();
            while (ld_relaxed(&st->bar_gen) == gen) {
                if (failed(st)) { ok = 0; break; }
                if (now_ticks() - t0 > spin_ticks) { fail(st, GPUTX_E_DEADLOCK); ok = 0; break; }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        fence_acquire();
        ok_s = ok && !failed(st);
    }
    __syncthreads();
    return ok_s;
}

// ---------------------------------------------------------------------------
// K-SET

__device__ __forceinline__ void kset_push(const BulkArgs& a, int32_t* fill, int32_t* front,
                                          const int* reg_off, int32_t q) {
    const int32_t t = a.ws.tty[q];
    const int slot = atomicAdd(&fill[t], 1);
    front[reg_off[t] + slot] = q;
}

// Run chunk c of the frontier (type regions cut in 64-transaction chunks) and
// release its successors into the next frontier.
//
// Each step of a wave is a chain of dependent memory round trips, which the
// chunk keeps short: the first successors come from the transaction's
// 32-byte record (one load, where the operation range and then the
// operation records were two dependent ones), and their in-degree
// decrements are all issued together, before the procedure's loads, so
// their round trips overlap one another and the procedure's (the next wave
// starts only after this wave's barrier, so the order inside the wave is
// free).
// (Loading the named successors' signatures ahead, toward the cache, measured
// slower: each extra wave-wide load of 64 scattered lines costs issue time on
// a path this short.)  Status counts accumulate in the caller's registers.
__device__ __forceinline__ void kset_chunk(const BulkArgs& a, int c, const int* cpre, const int* cnt,
                                           const int* reg_off, const int32_t* F, int32_t* fill_next,
                                           int32_t* F_next, int64_t& committed, int64_t& aborted) {
    int t = 0;
    while (cpre[t + 1] <= c) ++t;  // wave-uniform: this chunk's type
    const int idx = (c - cpre[t]) * 64 + lane_id();
    const bool live = idx < cnt[t];
    if (!live) return;
    const int32_t q = F[reg_off[t] + idx];
    // the first successors in one load (the operation records only when the
    // transaction has more operations or read runs)
    const KsetRec R = a.ws.ksrec[q];
    TxnIn x;
    {  // the chunk's type is the wave's: its descriptor through scalar loads
        const DevType Tl = dev_type_uniform(a.types, t);
        load_txn(a, Tl, q, t, x);
    }
    // the first operations' in-degree decrements, all in flight together
    int32_t left[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) left[k] = R.s0[k] >= 0 ? atomicSub(&a.ws.indeg[R.s0[k]], 1) : 0;
    // run this transaction, dispatched once on the chunk's procedure with a
    // scalar-loaded descriptor per case (waiting for it then waits for none
    // of the in-degree atomics in flight; only the procedures that pick a
    // column at run time keep their copy in private memory)
    int32_t s;
    switch (dev_type_uniform(a.types, t).proc) {
#define GTX_KSET_CASE(P)                                       \
    case P: {                                                  \
        const DevType T = dev_type_uniform(a.types, t);        \
        s = exec_txn_p<P>(a, T, x);                            \
        break;                                                 \
    }
        GTX_KSET_CASE(GPUTX_DEBIT_CREDIT)
        GTX_KSET_CASE(GPUTX_NEW_ORDER)
        GTX_KSET_CASE(GPUTX_NEW_ORDER_RB)
        GTX_KSET_CASE(GPUTX_PAYMENT)
        GTX_KSET_CASE(GPUTX_ORDER_STATUS)
        GTX_KSET_CASE(GPUTX_GET_SUB)
        GTX_KSET_CASE(GPUTX_GET_CF)
        GTX_KSET_CASE(GPUTX_UPD_SUB_FIELD)
        GTX_KSET_CASE(GPUTX_UPD_LOC)
        GTX_KSET_CASE(GPUTX_INS_CF)
        GTX_KSET_CASE(GPUTX_DEL_CF)
#undef GTX_KSET_CASE
    default:
        s = exec_txn(a, x);
    }
    committed += s == GPUTX_COMMIT;
    aborted += s == GPUTX_ABORT;
    // successors that became ready join the next frontier
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (left[k] == 1) {
            const int ty = R.s0ty[k] & 0xffff;
            const int slot = atomicAdd(&fill_next[ty], 1);
            F_next[reg_off[ty] + slot] = R.s0[k];
        }
    }
    if (R.s0ty[3] >> 16) {
        // operations past the fourth, and the rest of every read run
        const int64_t o0 = op_begin(a, q);
        const int64_t o1 = op_end(a, q);
        for (int64_t o = o0; o < o1; ++o) {
            const OpInfo inf = a.ws.op_info[o];
            if (o - o0 >= 4 && inf.slo < inf.shi && atomicSub(&a.ws.indeg[inf.s0], 1) == 1) {
                const int slot = atomicAdd(&fill_next[inf.s0ty], 1);
                F_next[reg_off[inf.s0ty] + slot] = inf.s0;
            }
            for (int32_t j = inf.slo + 1; j < inf.shi; ++j) {  // rest of a read run
                const int32_t q2 = a.ws.srt_txn[j];
                if (atomicSub(&a.ws.indeg[q2], 1) == 1) kset_push(a, fill_next, F_next, reg_off, q2);
            }
        }
    }
}

// Only when K-SET runs: each transaction's in-degree, the in-edges its
// operations contribute (Section 4.2's dependency graph) ...
// (The three passes run on K-SET's own persistent grid, before its first
// wave, with grid barriers between them, so a bulk that runs another
// executor pays one gated launch for all of K-SET.)
__device__ __forceinline__ void kset_indeg(const BulkArgs& a, int64_t gt, int64_t gs) {
    const GtxState* st = a.ws.st;
    for (int64_t p = gt; p < a.n; p += gs) {
        int in = 0;
        bool more = false;  // operations past the fourth, or read runs to walk
        if (a.ws.tty[p] >= 0) {
            const int64_t o0 = a.ws.cnt[p];
            const int64_t o1 = p + 1 < a.n ? (int64_t)a.ws.cnt[p + 1] : st->m;
            more = o1 - o0 > 4;
            for (int64_t o = o0; o < o1; ++o) {
                const OpInfo inf = a.ws.op_info[o];
                in += inf.in;
                more = more || inf.shi - inf.slo > 1;
            }
        }
        a.ws.indeg[p] = in;
        KsetRec r;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            r.s0[k] = -1;
            r.s0ty[k] = 0;
        }
        r.s0ty[3] = more ? 1 << 16 : 0;  // bit 16 of the fourth type word: more
        a.ws.ksrec[p] = r;
    }
}

// ... the transaction of each operation in item-sorted
// order (the read runs K-SET releases) ...
__device__ __forceinline__ void kset_sorted_txn(const BulkArgs& a, int64_t gt, int64_t gs) {
    const int64_t m = a.ws.st->m;
    const uint32_t* val = a.ws.pv[a.key_passes & 1];
    for (int64_t i = gt; i < m; i += gs) a.ws.srt_txn[i] = a.ws.op_txn[val[i] >> 1];
}

// ... and each operation's first successor transaction and its type, so a
// wave releases successors without gathers on its own path.
__device__ __forceinline__ void kset_succ(const BulkArgs& a, int64_t gt, int64_t gs) {
    const int64_t m = a.ws.st->m;
    for (int64_t o = gt; o < m; o += gs) {
        OpInfo& inf = a.ws.op_info[o];
        const int32_t slo = inf.slo, shi = inf.shi;
        if (slo < shi) {
            const int32_t q = a.ws.srt_txn[slo];
            const int32_t qt = a.ws.tty[q];
            inf.s0 = q;
            inf.s0ty = qt;
            // the transaction's record holds its first four operations' ones
            const int32_t p = a.ws.op_txn[o];
            const int64_t k = o - (int64_t)a.ws.cnt[p];
            if (k < 4) {
                a.ws.ksrec[p].s0[k] = q;
                if (k < 3) a.ws.ksrec[p].s0ty[k] = qt;
                else a.ws.ksrec[p].s0ty[3] = (a.ws.ksrec[p].s0ty[3] & (1 << 16)) | qt;
            }
        }
    }
}

__device__ __forceinline__ int chunk_prefix(const int* cnt, int* cpre) {
    int c = 0;
    for (int t = 0; t < GPUTX_MAX_TYPES; ++t) {
        cpre[t] = c;
        c += (cnt[t] + 63) / 64;
    }
    cpre[GPUTX_MAX_TYPES] = c;
    return c;
}

// Wave-wide inclusive scans through DPP (GFX9 controls: shift right within
// 16-lane rows, then the broadcasts of lanes 15 and 31 that carry the scan
// across rows).  All 64 lanes must be active.
constexpr int kDppRowShr = 0x110, kDppBcast15 = 0x142, kDppBcast31 = 0x143;
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_add_step(int v) {
    return v + __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xf, false);
}
__device__ __forceinline__ int wave_incl_sum_dpp(int v) {
    v = dpp_add_step<kDppRowShr + 1, 0xf>(v);
    v = dpp_add_step<kDppRowShr + 2, 0xf>(v);
    v = dpp_add_step<kDppRowShr + 4, 0xf>(v);
    v = dpp_add_step<kDppRowShr + 8, 0xf>(v);
    v = dpp_add_step<kDppBcast15, 0xa>(v);
    return dpp_add_step<kDppBcast31, 0xc>(v);
}
// Wave 0 of a workgroup, after a narrow wave: the next frontier's per-type
// counts (fill, which is cleared for the wave after), their total and the
// chunk prefix.
__device__ __forceinline__ void kset_level_counts(int* fill, int* wcnt, int* cpre, int* total) {
    const int l = lane_id();
    const int v = l < GPUTX_MAX_TYPES ? fill[l] : 0;
    if (l < GPUTX_MAX_TYPES) fill[l] = 0;
    const int ch = (v + 63) / 64;
    const int inc = wave_incl_sum_dpp(ch);  // DPP: no LDS round trip on the wave's path
    const int tot = __builtin_amdgcn_readlane(wave_incl_sum_dpp(v), 63);
    if (l < GPUTX_MAX_TYPES) {
        wcnt[l] = v;
        cpre[l] = inc - ch;
    }
    if (l == GPUTX_MAX_TYPES - 1) cpre[GPUTX_MAX_TYPES] = inc;
    if (l == 0) *total = tot;
}

__global__ __launch_bounds__(GTX_BLOCK) void k_kset(BulkArgs a) {
    GtxState* st = a.ws.st;
    if (failed(st) || st->chosen != GPUTX_KSET) return;
    int64_t committed = 0, aborted = 0;
    __shared__ int reg_off[GPUTX_MAX_TYPES];
    __shared__ int wcnt[GPUTX_MAX_TYPES];
    __shared__ int lfill[GPUTX_MAX_TYPES];
    __shared__ int cpre[GPUTX_MAX_TYPES + 1];
    __shared__ int64_t k_s;
    __shared__ int done_s, total_s, failed_s;
    if (threadIdx.x == 0) {
        int o = 0;
        for (int t = 0; t < GPUTX_MAX_TYPES; ++t) {
            reg_off[t] = o;
            o += st->type_count[t];
        }
    }
    __syncthreads();
    // in-degrees and sorted transactions, then first successors (which read
    // the sorted transactions of the whole grid)
    const int64_t gt = (int64_t)blockIdx.x * GTX_BLOCK + threadIdx.x, gs = (int64_t)gridDim.x * GTX_BLOCK;
    kset_indeg(a, gt, gs);
    kset_sorted_txn(a, gt, gs);
    if (!grid_barrier(st, a.spin_ticks)) return;
    kset_succ(a, gt, gs);
    // wave 0: every valid transaction without predecessors
    for (int64_t p = (int64_t)blockIdx.x * GTX_BLOCK + threadIdx.x; p < a.n;
         p += (int64_t)gridDim.x * GTX_BLOCK) {
        if (a.ws.tty[p] >= 0 && a.ws.indeg[p] == 0) kset_push(a, st->kset_fill[0], a.ws.front[0], reg_off, (int32_t)p);
    }
    const int gwaves = gridDim.x * GTX_WAVES;
    const int gw = blockIdx.x * GTX_WAVES + wave_id();
    int64_t k = 0;
    uint32_t nphase = 0;  // narrow phases completed
    bool finished = false;
    while (!finished && grid_barrier(st, a.spin_ticks)) {
        if (threadIdx.x < GPUTX_MAX_TYPES) {
            wcnt[threadIdx.x] = ld_relaxed(&st->kset_fill[k % 3][threadIdx.x]);
            if (blockIdx.x == 0) st_relaxed(&st->kset_fill[(k + 2) % 3][threadIdx.x], 0);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int tot = 0;
            for (int t = 0; t < GPUTX_MAX_TYPES; ++t) tot += wcnt[t];
            total_s = tot;
            chunk_prefix(wcnt, cpre);
        }
        __syncthreads();
        if (total_s == 0) break;  // every transaction has run
        if (total_s <= a.kset_narrow) {
            // narrow waves: workgroup 0 runs them alone with workgroup barriers
            if (blockIdx.x == 0) {
                int64_t kk = k;
                if (threadIdx.x < GPUTX_MAX_TYPES) lfill[threadIdx.x] = 0;
                __syncthreads();
                while (true) {
                    const int32_t* F = a.ws.front[kk & 1];
                    int32_t* Fn = a.ws.front[(kk + 1) & 1];
                    for (int c = wave_id(); c < cpre[GPUTX_MAX_TYPES]; c += GTX_WAVES)
                        kset_chunk(a, c, cpre, wcnt, reg_off, F, lfill, Fn, committed, aborted);
                    __syncthreads();
                    ++kk;
                    if (wave_id() == 0) {
                        kset_level_counts(lfill, wcnt, cpre, &total_s);
                        if (lane_id() == 0) {
                            if ((kk & 63) == 0) st_relaxed(&st->narrow_prog, kk);
                            // one read for the workgroup: every thread must take the same exit
                            failed_s = failed(st);
                        }
                    }
                    __syncthreads();
                    if (total_s == 0 || total_s > a.kset_narrow || failed_s) break;
                }
                if (threadIdx.x < GPUTX_MAX_TYPES) {
                    st_relaxed(&st->kset_fill[kk % 3][threadIdx.x], wcnt[threadIdx.x]);
                    st_relaxed(&st->kset_fill[(kk + 1) % 3][threadIdx.x], 0);
                }
                __syncthreads();
                if (threadIdx.x == 0) {
                    st->narrow_k = kk;
                    st->narrow_done = total_s == 0;
                    fence_release();
                    __hip_atomic_fetch_add(&st->narrow_gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                    k_s = kk;
                    done_s = total_s == 0;
                }
                __syncthreads();
            } else {
                if (threadIdx.x == 0) {
                    // wait for workgroup 0; the watchdog restarts whenever it makes progress
                    // narrow phases happen at the same waves in every workgroup,
                    // so the generation to wait for is known locally
                    uint64_t t0 = now_ticks();
                    int64_t prog = ld_relaxed(&st->narrow_prog);
                    while (ld_relaxed(&st->narrow_gen) < nphase + 1) {
                        if (failed(st)) break;
                        const int64_t pr = ld_relaxed(&st->narrow_prog);
                        if (pr != prog) { prog = pr; t0 = now_ticks(); }
                        else if (now_ticks() - t0 > a.spin_ticks) { fail(st, GPUTX_E_DEADLOCK); break; }
                        __builtin_amdgcn_s_sleep(2);
                    }
                    fence_acquire();
                    k_s = st->narrow_k;
                    done_s = st->narrow_done || failed(st);
                }
                __syncthreads();
            }
            k = k_s;
            finished = done_s;
            ++nphase;
            continue;
        }
        const int32_t* F = a.ws.front[k & 1];
        int32_t* Fn = a.ws.front[(k + 1) & 1];
        for (int c = gw; c < cpre[GPUTX_MAX_TYPES]; c += gwaves)
            kset_chunk(a, c, cpre, wcnt, reg_off, F, st->kset_fill[(k + 1) % 3], Fn, committed, aborted);
        ++k;
    }
    add_counts(st, committed, aborted);
    if (blockIdx.x == 0 && threadIdx.x == 0) st->waves = k;
}

// ---------------------------------------------------------------------------
// TPL with counter-based locks

// TPL's poll back-off: naps of kTplNap x 64 cycles (about 0.25 us), at most
// kTplMaxNaps between two polls.
constexpr int kTplNap = 10;
constexpr int kTplMaxNaps = 8;

__device__ __forceinline__ int wave_min_int(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off));
    return v;
}

// One window of transactions, at most one per lane (type t < 0: none): each
// waits until every lock counter of its operations reaches its target, runs,
// and increments the counters.  A lane that becomes ready runs with the
// wave's other ready lanes; the wave loops until all have run.
__device__ __forceinline__ void tpl_window(const BulkArgs& a, int64_t p, int32_t t, bool& ran, int32_t& s) {
    GtxState* st = a.ws.st;
    bool done = t < 0;
    int64_t o0 = 0, o1 = 0;
    TxnIn x;
    if (!done) {
        o0 = op_begin(a, p);
        o1 = op_end(a, p);
        load_txn(a, p, t, x);  // signatures are immutable: load before waiting
    }
    // lock groups and targets of the first ops, kept in registers while waiting
    constexpr int kPre = 4;
    int32_t pg[kPre], pt[kPre];
#pragma unroll
    for (int k = 0; k < kPre; ++k) {
        pg[k] = 0;
        pt[k] = 0;
        if (!done && o0 + k < o1) {
            const OpInfo inf = a.ws.op_info[o0 + k];
            pg[k] = inf.grp;
            pt[k] = inf.tgt;
        }
    }
    uint64_t t0 = 0;
    while (__any(!done)) {
        // how many more releases this lane's farthest counter still needs
        int lack = 0;
        if (!done) {
#pragma unroll
            for (int k = 0; k < kPre; ++k)
                if (o0 + k < o1) lack = max(lack, pt[k] - ld_relaxed(&a.ws.grp_cnt[pg[k]]));
            for (int64_t o = o0 + kPre; o < o1; ++o) {
                const OpInfo inf = a.ws.op_info[o];
                lack = max(lack, inf.tgt - ld_relaxed(&a.ws.grp_cnt[inf.grp]));
            }
        }
        const bool ready = !done && lack <= 0;
        if (__any(ready)) {
            // The cells go through coherent loads and stores (CoherentAcc):
            // a lane loads its cells only after it has seen its counters at
            // their targets, and moves the counters only after its stores
            // have completed, so the hand-off needs no cache-wide write-back
            // or invalidation (which would cost every other wave on the XCD
            // its cached signatures and operation records too).
            __asm__ volatile("" ::: "memory");
            // the ready lanes' type, when they share one
            const int32_t tr = __builtin_amdgcn_readfirstlane(ready ? t : INT32_MAX);
            const int32_t tu = __ballot(ready && t != tr) == 0 ? tr : -1;
            if (ready) {
                s = exec_txn_coherent(a, x, tu);
                ran = true;
            }
            __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
            if (ready) {
#pragma unroll
                for (int k = 0; k < kPre; ++k)
                    if (o0 + k < o1) atomicAdd(&a.ws.grp_cnt[pg[k]], 1);
                for (int64_t o = o0 + kPre; o < o1; ++o) atomicAdd(&a.ws.grp_cnt[a.ws.op_info[o].grp], 1);
                done = true;
            }
            t0 = 0;
        } else {
            if (t0 == 0) t0 = now_ticks();
            else if (now_ticks() - t0 > a.spin_ticks) {
                fail(st, GPUTX_E_DEADLOCK);
                break;
            }
            if (failed(st)) break;
            // proportional back-off: every release the nearest waiting lane
            // still needs takes at least one lock hand-off (about a
            // microsecond), so the wave polls again after a nap per missing
            // release; only the transactions next in line poll at full rate,
            // which keeps the polls off the hot counters' lines
            const int naps = min(wave_min_int(done ? INT32_MAX : lack) - 1, kTplMaxNaps);
            __builtin_amdgcn_s_sleep(1);
            for (int z = 0; z < naps; ++z) __builtin_amdgcn_s_sleep(kTplNap);
        }
    }
}

__global__ __launch_bounds__(GTX_BLOCK) void k_tpl(BulkArgs a) {
    GtxState* st = a.ws.st;
    if (failed(st) || st->chosen != GPUTX_TPL) return;
    __shared__ int win_s;
    __shared__ int32_t slot_pos[GTX_BLOCK];
    __shared__ int tcnt[GTX_WAVES][GPUTX_MAX_TYPES + 1];
    __shared__ int toff[GTX_WAVES][GPUTX_MAX_TYPES + 1];
    const int lane = lane_id();
    const int w = wave_id();
    // window width: the option, or (0) from the bulk's average parallelism
    // n / (d + 1) -- enough transactions in flight for about four times the
    // transactions one dependent step can run, over the grid's waves
    int L = a.tpl_lanes;
    if (L == 0) {
        const int64_t par = a.n / (st->depth + 1);
        const int64_t want = (4 * par + (int64_t)gridDim.x * GTX_WAVES - 1) / ((int64_t)gridDim.x * GTX_WAVES);
        L = 1;
        while (L < 64 && L < want) L <<= 1;
    }
    if (L < 64) {
        // narrow windows: each wave claims L transactions of its own and the
        // other lanes idle, so a transaction that becomes ready waits for
        // fewer other critical sections to finish first (deep chains are
        // bound by the dependent step, not by the work); the status counts
        // are flushed once at the end
        int64_t committed = 0, aborted = 0;
        while (true) {
            uint32_t win = 0;
            if (lane == 0) win = atomicAdd(&st->ticket, 1u);
            win = __shfl(win, 0);
            const int64_t base = (int64_t)win * L;
            if (base >= a.n || failed(st)) break;
            const int64_t p = base + lane;
            const int32_t t = lane < L && p < a.n ? a.ws.tty[p] : -1;
            bool ran = false;
            int32_t s = 0;
            tpl_window(a, p, t, ran, s);
            committed += ran && s == GPUTX_COMMIT;
            aborted += ran && s == GPUTX_ABORT;
        }
        add_counts(st, committed, aborted);
        return;
    }
    while (true) {
        if (threadIdx.x == 0) win_s = (int)atomicAdd(&st->ticket, 1u);
        __syncthreads();
        const int64_t base = (int64_t)win_s * GTX_BLOCK;
        if (base >= a.n || failed(st)) break;
        int64_t p = base + threadIdx.x;
        int32_t t = p < a.n ? a.ws.tty[p] : -1;
        if (a.group_by_type) {
            // stable counting sort of the window by type, so each wave64 runs
            // (mostly) one procedure (Section 5.4); invalid transactions last
            int rank = 0;
            for (int ty = -1; ty < GPUTX_MAX_TYPES; ++ty) {
                const uint64_t bm = __ballot(t == ty);
                if (lane == 0) tcnt[w][ty + 1] = __popcll(bm);
                if (t == ty) rank = __popcll(bm & lanemask_lt());
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                int o = 0;
                for (int ty = 1; ty <= GPUTX_MAX_TYPES; ++ty)
                    for (int ww = 0; ww < GTX_WAVES; ++ww) {
                        toff[ww][ty] = o;
                        o += tcnt[ww][ty];
                    }
                for (int ww = 0; ww < GTX_WAVES; ++ww) {
                    toff[ww][0] = o;
                    o += tcnt[ww][0];
                }
            }
            __syncthreads();
            slot_pos[toff[w][t + 1] + rank] = (int32_t)p;
            __syncthreads();
            p = slot_pos[threadIdx.x];
            t = p < a.n ? a.ws.tty[p] : -1;
        }
        bool ran = false;
        int32_t s = 0;
        tpl_window(a, p, t, ran, s);
        count_status(st, ran, s);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Without the timestamp constraint (Appendix G): serializability only.
//
// TPL takes basic 0/1 spin locks (Figure 10): a transaction acquires the
// locks of all its items with compare-and-swap, in ascending lock order, and
// gives back what it holds when one is taken, so no lane ever waits while
// holding a lock (a wave64 cannot wait on one of its own lanes).  Locks are
// 64-bit words in a table of power-of-two size indexed by a hash of the
// item key; items sharing a word only lock more coarsely.  A word holds a
// logical clock besides the held bit: the holder takes 1 + the largest clock
// of its words as its key and releases every word with that clock, so two
// conflicting transactions get keys in the order they ran, and sorting by
// key gives a serial order the execution is equivalent to.
//
// PART groups transactions by partition with per-partition counters
// instead of a sort: each transaction takes its position in its partition
// from its partition's counter, a prefix sum over the counters gives the
// groups' starts, and a scatter places it.  Partitions are then executed by
// the PART kernels, in that (arbitrary) order inside each partition; the
// grouped position is the serial key.

__device__ __forceinline__ uint32_t lock_hash(uint32_t key) {
    uint32_t h = key * 0x9E3779B1u;
    return h ^ (h >> 15);
}

__global__ void k_relaxed_choose(BulkArgs a) {
    GtxState* st = a.ws.st;
    if (threadIdx.x != 0 || st->error) return;
    // Section 5.2: transactions that span partitions go to the lock executor
    const int chosen = (a.strategy == GPUTX_PART && st->cross == 0) ? GPUTX_PART : GPUTX_TPL;
    st->chosen = chosen;
    st->run_part = chosen == GPUTX_PART;
}

__global__ __launch_bounds__(GTX_BLOCK) void k_lock_clear(BulkArgs a, uint64_t* locks, int64_t n_locks) {
    const GtxState* st = a.ws.st;
    if (ld_relaxed(&st->error) != 0 || st->chosen != GPUTX_TPL) return;
    for (int64_t i = (int64_t)blockIdx.x * GTX_BLOCK + threadIdx.x; i < n_locks; i += (int64_t)gridDim.x * GTX_BLOCK)
        locks[i] = 0;
}

__global__ __launch_bounds__(GTX_BLOCK) void k_tpl_relaxed(BulkArgs a, uint64_t* locks, uint32_t lock_mask,
                                                           int64_t* serial_key) {
    GtxState* st = a.ws.st;
    if (failed(st) || st->chosen != GPUTX_TPL) return;
    const int64_t stride = (int64_t)gridDim.x * GTX_BLOCK;
    for (int64_t base = (int64_t)blockIdx.x * GTX_BLOCK + wave_id() * 64; base < a.n; base += stride) {
        const int64_t p = base + lane_id();
        const int32_t t = p < a.n ? a.ws.tty[p] : -1;
        bool done = t < 0;
        if (p < a.n && done) serial_key[p] = -1;  // invalid: never runs
        // the transaction's lock words, ascending and distinct
        uint32_t slot[GTX_MAX_OPS];
#pragma unroll
        for (int j = 0; j < GTX_MAX_OPS; ++j) slot[j] = 0xffffffffu;
        int nk = 0;
        TxnIn x;
        if (!done) {
            load_txn(a, p, t, x);
            const int64_t o0 = op_begin(a, p), o1 = op_end(a, p);
            for (int64_t o = o0; o < o1; ++o) {
                const uint32_t v = lock_hash(a.ws.pk[0][o]) & lock_mask;
                bool dup = false;
#pragma unroll
                for (int j = 0; j < GTX_MAX_OPS; ++j) dup = dup || (j < nk && slot[j] == v);
                if (dup) continue;
#pragma unroll
                for (int j = 0; j < GTX_MAX_OPS; ++j)
                    if (j == nk) slot[j] = v;
                ++nk;
            }
            // ascending (unused entries hold the largest value and stay last)
#pragma unroll
            for (int i = 0; i < GTX_MAX_OPS - 1; ++i)
#pragma unroll
                for (int j = 0; j < GTX_MAX_OPS - 1 - i; ++j) {
                    const uint32_t lo = min(slot[j], slot[j + 1]), hi = max(slot[j], slot[j + 1]);
                    slot[j] = lo;
                    slot[j + 1] = hi;
                }
        }
        uint64_t held[GTX_MAX_OPS];
        uint64_t t0 = 0;
        while (__any(!done)) {
            bool got = false;
            if (!done) {
                got = true;
                int taken = 0;
#pragma unroll
                for (int j = 0; j < GTX_MAX_OPS; ++j) {
                    if (j < nk && got) {
                        const uint64_t cur = ld_relaxed(&locks[slot[j]]);
                        if ((cur & 1ull) ||
                            atomicCAS((unsigned long long*)&locks[slot[j]], (unsigned long long)cur,
                                      (unsigned long long)(cur | 1ull)) != cur) {
                            got = false;
                        } else {
                            held[j] = cur;
                            taken = j + 1;
                        }
                    }
                }
                if (!got) {  // give back what was taken, unchanged
#pragma unroll
                    for (int j = 0; j < GTX_MAX_OPS; ++j)
                        if (j < taken) st_relaxed(&locks[slot[j]], held[j]);
                }
            }
            if (__any(got)) {
                fence_acquire();  // see the writes of the previous holders
                int32_t s = 0;
                if (got) s = exec_txn(a, x);
                fence_release();  // publish this transaction's writes before unlocking
                if (got) {
                    uint64_t c = 0;
#pragma unroll
                    for (int j = 0; j < GTX_MAX_OPS; ++j)
                        if (j < nk) c = max(c, held[j] >> 1);
                    c += 1;
#pragma unroll
                    for (int j = 0; j < GTX_MAX_OPS; ++j)
                        if (j < nk) st_relaxed(&locks[slot[j]], c << 1);
                    serial_key[x.i] = (int64_t)c;
                    done = true;
                }
                count_status(st, got, s);
                t0 = 0;
            } else {
                if (t0 == 0) t0 = now_ticks();
                else if (now_ticks() - t0 > a.spin_ticks) {
                    fail(st, GPUTX_E_DEADLOCK);
                    break;
                }
                if (failed(st)) break;
                __builtin_amdgcn_s_sleep(1);
            }
        }
        if (failed(st)) break;
    }
}

// ---- PART grouping by per-partition counters ------------------------------
constexpr int kGroupTile = 1024;       // transactions per counting workgroup
constexpr int kGroupLdsBins = 4096;    // partitions counted in LDS first

// Each transaction's position within its partition (kept in tsv[0]); the
// counters end up holding the partition sizes.
__global__ __launch_bounds__(GTX_BLOCK) void k_pgroup_count(BulkArgs a, int32_t* counter) {
    GtxState* st = a.ws.st;
    if (ld_relaxed(&st->error) != 0 || !st->run_part) return;
    __shared__ int hist[kGroupLdsBins];
    __shared__ int base[kGroupLdsBins];
    const int64_t bins = a.n_parts + 1;  // the last bin: transactions PART does not run
    const bool lds = bins <= kGroupLdsBins;
    if (lds) {
        for (int b = threadIdx.x; b < bins; b += GTX_BLOCK) hist[b] = 0;
        __syncthreads();
    }
    const int64_t t0 = (int64_t)blockIdx.x * kGroupTile;
    int local[kGroupTile / GTX_BLOCK];
    uint32_t pid[kGroupTile / GTX_BLOCK];
#pragma unroll
    for (int k = 0; k < kGroupTile / GTX_BLOCK; ++k) {
        const int64_t p = t0 + k * GTX_BLOCK + threadIdx.x;
        pid[k] = p < a.n ? a.ws.qk[0][p] : 0;
        local[k] = 0;
        if (p < a.n) local[k] = lds ? atomicAdd(&hist[pid[k]], 1) : atomicAdd(&counter[pid[k]], 1);
    }
    if (!lds) {
#pragma unroll
        for (int k = 0; k < kGroupTile / GTX_BLOCK; ++k) {
            const int64_t p = t0 + k * GTX_BLOCK + threadIdx.x;
            if (p < a.n) a.ws.tsv[0][p] = (uint32_t)local[k];
        }
        return;
    }
    __syncthreads();
    for (int b = threadIdx.x; b < bins; b += GTX_BLOCK)
        base[b] = hist[b] ? atomicAdd(&counter[b], hist[b]) : 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kGroupTile / GTX_BLOCK; ++k) {
        const int64_t p = t0 + k * GTX_BLOCK + threadIdx.x;
        if (p < a.n) a.ws.tsv[0][p] = (uint32_t)(base[pid[k]] + local[k]);
    }
}

__global__ __launch_bounds__(GTX_BLOCK) void k_pgroup_clear(BulkArgs a, int32_t* counter) {
    const GtxState* st = a.ws.st;
    if (ld_relaxed(&st->error) != 0 || !st->run_part) return;
    for (int64_t b = (int64_t)blockIdx.x * GTX_BLOCK + threadIdx.x; b <= a.n_parts; b += (int64_t)gridDim.x * GTX_BLOCK)
        counter[b] = 0;
}

// One workgroup: exclusive scan of the counters in place (group starts).
__global__ __launch_bounds__(GTX_BLOCK) void k_pgroup_scan(BulkArgs a, int32_t* counter) {
    const GtxState* st = a.ws.st;
    if (ld_relaxed(&st->error) != 0 || !st->run_part) return;
    __shared__ int lds[GTX_WAVES + 1];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int64_t bins = a.n_parts + 1;
    for (int64_t c0 = 0; c0 < bins; c0 += GTX_BLOCK) {
        const int64_t b = c0 + threadIdx.x;
        const int v = b < bins ? counter[b] : 0;
        int tot;
        const int ex = block_excl_sum(v, &tot, lds);
        if (b < bins) counter[b] = carry + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry += tot;
        __syncthreads();
    }
}

// Place every transaction in its group: the grouped arrays are the ones the
// partition sort would have produced (partition ids and serial positions).
__global__ __launch_bounds__(GTX_BLOCK) void k_pgroup_scatter(BulkArgs a, const int32_t* start, int64_t* serial_key) {
    const GtxState* st = a.ws.st;
    if (ld_relaxed(&st->error) != 0 || !st->run_part) return;
    const int fb = a.part_passes & 1;
    for (int64_t p = (int64_t)blockIdx.x * GTX_BLOCK + threadIdx.x; p < a.n; p += (int64_t)gridDim.x * GTX_BLOCK) {
        const uint32_t pid = a.ws.qk[0][p];
        const int64_t dst = (int64_t)start[pid] + a.ws.tsv[0][p];
        a.ws.qk[fb][dst] = pid;
        a.ws.qv[fb][dst] = (uint32_t)p;
        a.ws.qinv[p] = (uint32_t)dst;
        serial_key[p] = a.ws.tty[p] >= 0 ? dst : -1;
    }
}

// ---------------------------------------------------------------------------
// PART

// ---- PART partitions ------------------------------------------------------
// After the partition sort, the non-empty partitions are listed in order:
// heads[b] is the first sorted position of the b-th one and heads[b + 1] its
// end (heads[n_heads] is where the transactions PART does not run begin).
constexpr int kHeadItems = 8;
constexpr int kHeadTile = GTX_BLOCK * kHeadItems;

__device__ __forceinline__ bool part_head(const uint32_t* key, int64_t i, uint32_t sentinel) {
    const uint32_t k = key[i];
    return k < sentinel && (i == 0 || key[i - 1] != k);
}

__global__ __launch_bounds__(GTX_BLOCK) void k_heads_up(BulkArgs a) {
    const GtxState* st = a.ws.st;
    if (!(a.part_early || st->run_part) || ld_relaxed(&st->error) != 0) return;
    __shared__ int lds[GTX_WAVES + 1];
    const uint32_t* key = a.ws.qk[a.part_passes & 1];
    const int64_t i0 = (int64_t)blockIdx.x * kHeadTile + (int64_t)threadIdx.x * kHeadItems;
    int c = 0;
#pragma unroll
    for (int j = 0; j < kHeadItems; ++j)
        if (i0 + j < a.n) c += part_head(key, i0 + j, (uint32_t)a.n_parts);
    int tot;
    (void)block_excl_sum(c, &tot, lds);
    if (threadIdx.x == 0) a.ws.heads_tmp[blockIdx.x] = tot;
}

__global__ __launch_bounds__(GTX_BLOCK) void k_heads_mid(BulkArgs a, int nb) {
    GtxState* st = a.ws.st;
    if (!(a.part_early || st->run_part) || ld_relaxed(&st->error) != 0) return;
    __shared__ int lds[GTX_WAVES + 1];
    int carry = 0;
    for (int b0 = 0; b0 < nb; b0 += GTX_BLOCK) {
        const int b = b0 + (int)threadIdx.x;
        const int v = b < nb ? a.ws.heads_tmp[b] : 0;
        int tot;
        const int ex = block_excl_sum(v, &tot, lds);
        if (b < nb) a.ws.heads_tmp[b] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        st->n_heads = carry;
        a.ws.heads[carry] = (int32_t)a.n;  // no transaction outside PART
    }
}

__global__ __launch_bounds__(GTX_BLOCK) void k_heads_down(BulkArgs a) {
    const GtxState* st = a.ws.st;
    if (!(a.part_early || st->run_part) || ld_relaxed(&st->error) != 0) return;
    __shared__ int lds[GTX_WAVES + 1];
    const uint32_t* key = a.ws.qk[a.part_passes & 1];
    const uint32_t sentinel = (uint32_t)a.n_parts;
    const int64_t i0 = (int64_t)blockIdx.x * kHeadTile + (int64_t)threadIdx.x * kHeadItems;
    bool h[kHeadItems];
    int c = 0;
#pragma unroll
    for (int j = 0; j < kHeadItems; ++j) {
        const int64_t i = i0 + j;
        h[j] = i < a.n && part_head(key, i, sentinel);
        c += h[j];
        // first transaction PART does not run: the end of the last partition
        if (i < a.n && key[i] == sentinel && (i == 0 || key[i - 1] != sentinel))
            a.ws.heads[st->n_heads] = (int32_t)i;
    }
    int tot;
    int at = a.ws.heads_tmp[blockIdx.x] + block_excl_sum(c, &tot, lds);
#pragma unroll
    for (int j = 0; j < kHeadItems; ++j)
        if (h[j]) a.ws.heads[at++] = (int32_t)(i0 + j);
}

// One lane per short partition (fewer than a.long_part transactions): its
// transactions run one after another, in place.
// Before PART runs: each transaction's record (input index, type and
// parameters, at its partition-grouped position) and its appended rows (they
// depend on the signature alone).  The bulk is walked in serial order, so
// the signatures are read and the appended rows written contiguously; each
// record goes to its grouped position (qinv), so a partition's records lie
// together and a partition kernel reads them contiguously.  Under PART no
// transaction crosses partitions (Algorithm 1 falls back to TPL otherwise),
// so every valid transaction is PART's.
__global__ __launch_bounds__(GTX_BLOCK) void k_part_gather(BulkArgs a) {
    const GtxState* st = a.ws.st;
    // ahead of the choice too: the records are workspace, and the appended
    // rows (a function of the signatures alone) are the ones any executor writes
    if (failed(st) || !(a.part_early || st->chosen == GPUTX_PART)) return;
    // Ahead of the choice it may also run before the execution gate's capacity
    // check: a bulk whose appends overflow a table writes nothing (the gate
    // then fails it).
    for (int k = 0; k < a.n_app; ++k)
        if (st->app_total[k] > 0 && a.rowcount[k] + st->app_total[k] > a.capacity[k]) return;
    for (int64_t q = (int64_t)blockIdx.x * GTX_BLOCK + threadIdx.x; q < a.n;
         q += (int64_t)gridDim.x * GTX_BLOCK) {
        const int32_t t = a.ws.tty[q];
        if (t < 0) continue;
        // the appended rows of the transaction at serial position q
        TxnIn y;
        load_txn(a, q, t, y);
        AppendOnlyAcc ap;
        int64_t unused[GTX_MAX_RESULTS];
        (void)txn_exec_any(ap, a.types[t], y.prm, y.ts, y.app0, y.app1, unused);
        // its record, at its grouped position
        int64_t* r = a.ws.rec + (int64_t)a.ws.qinv[q] * a.rec_words;
        r[0] = (int64_t)(((uint64_t)(uint32_t)t << 32) | (uint32_t)y.i);
#pragma unroll
        for (int k = 0; k < GTX_MAX_PARAMS; ++k)
            if (k < a.prm_rows) r[1 + k] = y.prm[k];
    }
}

__global__ __launch_bounds__(GTX_BLOCK) void k_part(BulkArgs a) {
    GtxState* st = a.ws.st;
    if (failed(st) || st->chosen != GPUTX_PART) return;
    const int nh = st->n_heads;
    const uint32_t* pos = a.ws.qv[a.part_passes & 1];
    int64_t committed = 0, aborted = 0;
    for (int64_t b = (int64_t)blockIdx.x * GTX_BLOCK + threadIdx.x; b < nh;
         b += (int64_t)gridDim.x * GTX_BLOCK) {
        const int64_t lo = a.ws.heads[b], end = a.ws.heads[b + 1];
        if (end - lo >= a.long_part) continue;  // a workgroup runs it
        for (int64_t i = lo; i < end; ++i) {
            const int32_t p = (int32_t)pos[i];
            const int32_t s = run_at_noapp(a, p, a.ws.tty[p]);
            committed += s == GPUTX_COMMIT;
            aborted += s == GPUTX_ABORT;
        }
    }
    add_counts(st, committed, aborted);
}

// Signatures of one PART chunk of cw transactions staged in LDS.  Parameters,
// cell addresses and results are stored one row per transaction (odd
// strides, part_ps/css/rs); the parameter and address arrays have
// kChunkSpare spare rows so reading up to three transactions ahead needs no
// bound.
constexpr int kChunkSpare = 4;
struct PartChunk {
    int64_t* res;   // [cw][rs] results
    int64_t* prm;   // [cw + kChunkSpare][ps] parameters
    int64_t* idx;   // [cw] input index (status / results slot)
    int32_t* t;     // [cw] type
    int32_t* proc;  // [cw] procedure (bits 0-15) and cell class (bits 16-31)
    int32_t* st;    // [cw] status
    uint32_t* cs;   // [cw + kChunkSpare][css] LDS address of each of the transaction's staged cells
    int cw, ps, css, rs;
};
// Odd row strides (in elements): the staging lanes write one row each, and
// an odd stride spreads consecutive lanes over the LDS banks.
__host__ __device__ inline int part_ps(int prm_rows) { return prm_rows | 1; }
__host__ __device__ inline int part_css(int cells) { return cells | 1; }
__host__ __device__ inline int part_rs(int res_rows) { return res_rows | 1; }

// The chunk's table cells, staged in LDS: an open-addressing hash table keyed
// by cell address (bit 1: 64-bit cell, bit 0: written; key 0 = empty slot),
// plus the list of claimed slots.  Under PART a cell belongs to exactly one
// partition, so the wave may hold it in LDS while the chunk runs and write it
// back afterwards: no other wave reads or writes it meanwhile.
#define GTX_LDS __attribute__((address_space(3)))
struct __attribute__((aligned(16))) CellSlot {
    uint64_t key;
    int64_t val;
};
struct CellTab {
    GTX_LDS CellSlot* slot;  // [1 << bits], then one sink slot outside the table
    GTX_LDS int32_t* list;   // claimed slots
    GTX_LDS int32_t* nlist;  // [4]: the count, then two flags of the pipelined form
    GTX_LDS uint8_t* tag;    // [serial waves][tstride]: group_ordinal's scratch per wave
    int bits, tstride;
};
// LDS address of a slot's value (16-byte slots: bit 3 is set), and of the
// sink slot's key (bit 3 clear), which stands for an ordinal no cell backs.
__device__ __forceinline__ uint32_t lds_addr(GTX_LDS const void* p) { return (uint32_t)(uintptr_t)p; }

__device__ __forceinline__ uint32_t cell_val_addr(const CellTab& t, uint32_t h) { return lds_addr(&t.slot[h].val); }
__device__ __forceinline__ uint32_t cell_sink_addr(const CellTab& t) { return lds_addr(&t.slot[1u << t.bits].key); }
template <class V>
__device__ __forceinline__ uint64_t cell_key(GTX_GLOBAL V* p) {
    return (uint64_t)p | (sizeof(V) == 8 ? 2u : 0u);
}
__device__ __forceinline__ uint32_t cell_hash(uint64_t key, int bits) {
    return ((uint32_t)(key >> 2) * 0x9E3779B1u) >> (32 - bits);
}

// Fetch side: each lane claims the cells of its transaction and records,
// per cell ordinal, the LDS address of the cell's staged value.  A probe
// reads the slot's key first: a cell staged already (the common case for
// hot cells) costs no atomic, and an empty slot is taken with a CAS.  A cell
// the procedure may write is marked written (bit 0), so it is stored back
// when the table is flushed.  The first claimant of a cell (won, one bit per
// ordinal) lists the slot and loads the cell's value afterwards
// (part_claim_wave, claim_values_issue): all of a transaction's claims go first,
// so its loads are in flight together.  With NV > 0 (procedures of at most NV
// cells, their ordinals known at compile time) each cell's value is loaded
// before its claim instead, into a register, and the won ones are stored
// after the last claim (store_won): the loads then overlap the claims.
// CAS_FIRST: procedures whose cells are mostly new to the table (a
// new-order's stock rows) try the CAS at once, one LDS round trip per probe
// instead of a read and then the CAS.
template <int NV, bool CAS_FIRST = false>
struct CellClaim {
    CellTab tab;
    uint32_t* cs;  // the transaction's row of cell addresses
    uint32_t won;
    int64_t v[NV > 0 ? NV : 1];
    uint32_t at[NV > 0 ? NV : 1];
    template <class V>
    __device__ __forceinline__ void cell(int ord, GTX_GLOBAL V* p, bool w) {
        if constexpr (NV > 0) v[ord] = (int64_t)*p;  // kept only if this lane wins the cell
        const uint64_t key = cell_key(p);
        const uint64_t want = key | (w ? 1u : 0u);
        const uint32_t mask = (1u << tab.bits) - 1;
        uint32_t h = cell_hash(key, tab.bits);
        uint32_t got = cell_sink_addr(tab);  // no free slot: the serial side reports the miss
        for (uint32_t probe = 0; probe <= mask; ++probe, h = (h + 1) & mask) {
            uint64_t cur = 0;
            if constexpr (!CAS_FIRST)
                cur = __hip_atomic_load(&tab.slot[h].key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (cur == 0) {  // on failure the CAS leaves the slot's key in cur
                __hip_atomic_compare_exchange_strong(&tab.slot[h].key, &cur, want, __ATOMIC_RELAXED,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (cur == 0) {
                    got = cell_val_addr(tab, h);
                    won |= 1u << ord;
                    if constexpr (NV > 0) at[ord] = got;
                    break;
                }
            }
            if ((cur & ~(uint64_t)1) == key) {  // staged already
                if (w && !(cur & 1))
                    __hip_atomic_fetch_or(&tab.slot[h].key, (uint64_t)1, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_WORKGROUP);
                got = cell_val_addr(tab, h);
                break;
            }
        }
        cs[ord] = got;
    }
    __device__ __forceinline__ void store_won() const {
#pragma unroll
        for (int r = 0; r < NV; ++r)
            if ((won >> r) & 1u) *(GTX_LDS int64_t*)(uintptr_t)at[r] = v[r];
    }
};
// The won cells' values, four loads in flight at a time; the slot's key holds
// the cell's global address and width.  claim_values_issue loads those of
// ordinals 0-3 into registers (and handles any further ordinals itself);
// claim_values_finish stores them, so other work can cover the loads.
struct ValLoads {
    int64_t v[4];
};
__device__ __forceinline__ int64_t cell_value_of(const uint32_t at_lds) {
    const uint64_t key = *(GTX_LDS const uint64_t*)(uintptr_t)(at_lds - 8);
    const uint64_t at = key & ~(uint64_t)3;
    return (key & 2) ? *(GTX_GLOBAL const int64_t*)at : (int64_t)*(GTX_GLOBAL const int32_t*)at;
}
__device__ __forceinline__ void claim_values_issue(const uint32_t* cs, uint32_t won, ValLoads& L) {
    for (int r0 = 4; won >> r0; r0 += 4) {
        int64_t v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if ((won >> (r0 + q)) & 1u) v[q] = cell_value_of(cs[r0 + q]);
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if ((won >> (r0 + q)) & 1u) *(GTX_LDS int64_t*)(uintptr_t)cs[r0 + q] = v[q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if ((won >> q) & 1u) L.v[q] = cell_value_of(cs[q]);
}
__device__ __forceinline__ void claim_values_finish(const uint32_t* cs, uint32_t won, const ValLoads& L) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if ((won >> q) & 1u) *(GTX_LDS int64_t*)(uintptr_t)cs[q] = L.v[q];
}

// Serial side: the procedures' accessor over the staged cells.  The fetch
// lanes resolved every cell ordinal of the transaction to the LDS address
// of its staged value, so a reference is one LDS read and a write one LDS
// store: no address or hash arithmetic on the serial path, and no global
// access (no store can then alias the type descriptor, whose fields stay in
// registers).  An ordinal the cell list did not name points at the sink
// slot; its bit 3 is clear, which the AND of all addresses in *seen shows,
// and the bulk fails with GPUTX_E_INTERNAL.
struct LdsAcc {
    const uint32_t* ids;  // LDS address per cell ordinal (registers)
    uint32_t* seen;
    template <class V>
    struct Ref {
        GTX_LDS int64_t* s;
        int64_t v;
        __device__ __forceinline__ V get() const { return (V)v; }
        __device__ __forceinline__ void set(V x) { *s = (int64_t)x; v = (int64_t)x; }
    };
    template <class V>
    __device__ __forceinline__ Ref<V> ref(int ord, GTX_GLOBAL V*) {
        const uint32_t at = ids[ord];
        *seen &= at;
        Ref<V> r;
        r.s = (GTX_LDS int64_t*)(uintptr_t)at;
        r.v = *r.s;
        return r;
    }
    template <class V>
    __device__ __forceinline__ V ld(int ord, GTX_GLOBAL V* p) { return ref(ord, p).get(); }
    template <class V>
    __device__ __forceinline__ void st(int ord, GTX_GLOBAL V* p, V v) { ref(ord, p).set(v); }
    template <class V>
    __device__ __forceinline__ void app(GTX_GLOBAL V*, V) {}  // written by k_part_gather
};

// Serial accessor over registers: the running transaction's cell values were
// read one transaction ahead; a write goes to the staged cell and to the
// register (so a later reference of the same transaction sees it).
struct RegAcc {
    const uint32_t* ids;  // LDS address of each cell ordinal's staged value
    int64_t* vals;        // the values, read ahead
    template <class V>
    struct Ref {
        GTX_LDS int64_t* s;
        int64_t* v;
        __device__ __forceinline__ V get() const { return (V)*v; }
        __device__ __forceinline__ void set(V x) {
            *s = (int64_t)x;
            *v = (int64_t)x;
        }
    };
    template <class V>
    __device__ __forceinline__ Ref<V> ref(int ord, GTX_GLOBAL V*) {
        return Ref<V>{(GTX_LDS int64_t*)(uintptr_t)ids[ord], &vals[ord]};
    }
    template <class V>
    __device__ __forceinline__ V ld(int ord, GTX_GLOBAL V* p) { return ref(ord, p).get(); }
    template <class V>
    __device__ __forceinline__ void st(int ord, GTX_GLOBAL V* p, V v) { ref(ord, p).set(v); }
    template <class V>
    __device__ __forceinline__ void app(GTX_GLOBAL V*, V) {}  // written by k_part_gather
};

// Cell addresses, parameters and cell values of one transaction, in registers.
template <int NP, int NC>
struct SerialRegs {
    uint32_t ids[NC];
    int64_t prm[NP];
    int64_t val[NC];
};

// One step of the forwarding pipeline.  X holds transaction k (addresses,
// parameters, values), Y transaction k + 1 (addresses and parameters), and
// Z is free.  The step starts loading the addresses and parameters of
// k + 2 into Z and the values of k + 1 into Y (before k writes), runs k,
// then forwards k's final value wherever k + 1 names the same cell at the
// same ordinal.  Every load has a whole step to arrive.
template <int P, int NP, int NC, int NR>
__device__ __forceinline__ void serial_fwd_step(const DevType& T, const PartChunk& c, int k, int cnt,
                                                SerialRegs<NP, NC>& X, SerialRegs<NP, NC>& Y,
                                                SerialRegs<NP, NC>& Z, int64_t& committed,
                                                int64_t& aborted) {
    (void)cnt;  // rows past the chunk hold table addresses (part_init_rows)
#pragma unroll
    for (int r = 0; r < NC; ++r) Z.ids[r] = c.cs[(k + 2) * c.css + r];
#pragma unroll
    for (int r = 0; r < NP; ++r) Z.prm[r] = c.prm[(k + 2) * c.ps + r];
#pragma unroll
    for (int r = 0; r < NC; ++r) Y.val[r] = *(GTX_LDS const int64_t*)(uintptr_t)Y.ids[r];
    int64_t prm[GTX_MAX_PARAMS];
#pragma unroll
    for (int r = 0; r < GTX_MAX_PARAMS; ++r) prm[r] = r < NP ? X.prm[r] : 0;
    RegAcc acc{X.ids, X.val};
    int64_t res[GTX_MAX_RESULTS];
    const int32_t s = txn_exec_p<P>(acc, T, prm, 0, 0, 0, res);  // appends: k_part_gather
    if (s != GPUTX_COMMIT) c.st[k] = s;  // staged as COMMIT
#pragma unroll
    for (int r = 0; r < NR; ++r) c.res[k * c.rs + r] = res[r];
    committed += s == GPUTX_COMMIT;
    aborted += s == GPUTX_ABORT;
#pragma unroll
    for (int r = 0; r < NC; ++r)
        if (Y.ids[r] == X.ids[r]) Y.val[r] = X.val[r];
}

// One transaction k of procedure P against the staged cells (LdsAcc, which
// checks that every cell ordinal P names was staged); returns its status.
template <int P>
__device__ __forceinline__ int32_t serial_one(const DevType& T, const PartChunk& c, int k, uint32_t* seen) {
    constexpr int NP = proc_params(P);
    constexpr int NR = proc_results(P);
    constexpr int NC = proc_cells(P);
    int64_t prm[GTX_MAX_PARAMS];
    uint32_t ids[NC];
#pragma unroll
    for (int r = 0; r < GTX_MAX_PARAMS; ++r) prm[r] = r < NP ? c.prm[k * c.ps + r] : 0;
#pragma unroll
    for (int r = 0; r < NC; ++r) ids[r] = c.cs[k * c.css + r];
    LdsAcc acc{ids, seen};
    int64_t res[GTX_MAX_RESULTS];
    const int32_t s = txn_exec_p<P>(acc, T, prm, 0, 0, 0, res);  // appends: k_part_gather
    if (s != GPUTX_COMMIT) c.st[k] = s;  // staged as COMMIT
#pragma unroll
    for (int r = 0; r < NR; ++r) c.res[k * c.rs + r] = res[r];
    return s;
}

// The serial waves of a workgroup: this one's index and their number, and
// its scratch for grouping (group_ordinal).
struct SerialWave {
    int ws, nsw;
    GTX_LDS uint8_t* tag;  // [512 + tag bytes]: 64 group masks, then a tag byte per slot
};

// The order-entry procedures name distinct cells within one transaction
// (payment: a warehouse, a district and a customer row; a new-order: its
// items, checked for repeats here).  Their transactions then run one after
// another with the whole wave on each, lane r updating the cell of ordinal r
// -- the partition's order is kept, only one transaction's cells are worked
// on side by side.  A transaction's signature is first read into registers,
// one parameter and one cell ordinal per lane (wave_fetch).  LDS operations
// of one wave complete in issue order, so a transaction's read of its cells
// sees every earlier transaction's writes.  The forms return the
// transaction's status, the same on every lane, and write what serial_one
// writes.
struct WaveTxn {
    int64_t a;    // new-order: lane's item; payment: the amount
    int32_t n;    // new-order: item count (1..15 in a valid one)
    int32_t b;    // new-order: lane's quantity (1..1000 in a valid one)
    uint32_t at;  // LDS address of the lane's cell ordinal
};
__device__ __forceinline__ void wave_fetch(const PartChunk& c, int k, int32_t pc, WaveTxn& x) {
    const int lane = lane_id();
    switch (pc & 0xffff) {
    case GPUTX_NEW_ORDER:
    case GPUTX_NEW_ORDER_RB: {  // 34 parameter rows and 15 ordinals exist
        const int j = min(lane, 14);
        x.n = (int32_t)c.prm[k * c.ps + 3];
        x.a = c.prm[k * c.ps + 4 + j];
        x.b = (int32_t)c.prm[k * c.ps + 19 + j];
        x.at = c.cs[k * c.css + j];
        break;
    }
    case GPUTX_PAYMENT:
        x.a = c.prm[k * c.ps + 3];
        x.at = c.cs[k * c.css + min(lane, 2)];
        break;
    case GPUTX_ORDER_STATUS:
        x.at = c.cs[k * c.css];
        break;
    default:
        break;
    }
}

template <int Q>  // GPUTX_NEW_ORDER or GPUTX_NEW_ORDER_RB
__device__ __forceinline__ int32_t wave_new_order(const DevType& T, const PartChunk& c, int k, const WaveTxn& x,
                                                  uint32_t* seen) {
    const int lane = lane_id();
    const int64_t nk = x.n;
    const bool live = lane < nk;
    const int64_t item = live ? x.a : -1;
    const int64_t q = live ? x.b : 0;
    // a rollback new-order stops at its first unused item
    const bool unused = Q == GPUTX_NEW_ORDER_RB && live && item == T.dims[3];
    const uint64_t ub = __ballot(unused);
    const int stop = ub ? __ffsll((unsigned long long)ub) - 1 : 64;
    const bool mine = live && lane < stop;
    const uint32_t at = mine ? x.at : 0xffffffffu;
    GTX_LDS int64_t* cell = (GTX_LDS int64_t*)(uintptr_t)at;
    // the undo log entry for the item; read before the repeat check (a
    // transaction with a repeat reruns on one lane below)
    const int64_t old = mine ? *cell : 0;
    bool dup = false;
#pragma unroll
    for (int r = 1; r < 15; ++r) {
        const uint32_t o = __shfl(at, (lane + r) & 63);
        dup = dup || (mine && o == at);
    }
    if (__any(dup)) {  // an item named twice: the updates must follow each other
        int32_t s = 0;
        if (lane == 0) s = serial_one<Q>(T, c, k, seen);
        return __shfl(s, 0);
    }
    if (mine) *seen &= at;
    int32_t nv = 0;
    if (mine) {
        int64_t s = (int64_t)(int32_t)old - q;
        if (s < 10) s += 91;
        nv = to_i32(s);
        *cell = (int64_t)nv;
    }
    if (stop < 64) {  // roll back from the undo log: no effect, results 0
        if (mine) *cell = old;
        if (lane < proc_results(Q)) c.res[k * c.rs + lane] = 0;
        if (lane == 0) c.st[k] = GPUTX_ABORT;
        return GPUTX_ABORT;
    }
    // result 0: the item count; result 1 + r: item r's new quantity
    if (lane < 15) c.res[k * c.rs + 1 + lane] = live ? (int64_t)nv : 0;
    else if (lane == 15) c.res[k * c.rs] = nk;
    return GPUTX_COMMIT;
}

// Up to four consecutive new-orders of one type at once, sixteen lanes each
// (lane 16 g + j: item j of the g-th, transaction kg), when no two of their
// items are the same cell and none rolls back: each lane stores its lane
// number in its cell's tag byte and reads it back, and one that reads another
// lane's number shares its cell with that lane (the same transaction or
// another of the group).  Disjoint new-orders commute, so running them
// side by side leaves what running them in turn leaves.  Returns false,
// having changed nothing, when the group must run one at a time.
template <int Q>  // GPUTX_NEW_ORDER or GPUTX_NEW_ORDER_RB
__device__ __forceinline__ bool wave_new_order_group(const DevType& T, const PartChunk& c, const CellTab& tab,
                                                     const SerialWave& sw, int k0, int k1, int k2, int k3, int G,
                                                     uint32_t* seen) {
    const int lane = lane_id();
    const int g = lane >> 4, j = lane & 15;
    const int k = g == 0 ? k0 : g == 1 ? k1 : g == 2 ? k2 : k3;
    const bool grp = g < G;
    int32_t nk = 0, q = 0;
    int64_t item = -1;
    uint32_t at = 0;
    if (grp) {  // 34 parameter rows and 15 ordinals exist
        const int jj = min(j, 14);
        nk = (int32_t)c.prm[k * c.ps + 3];
        item = c.prm[k * c.ps + 4 + jj];
        q = (int32_t)c.prm[k * c.ps + 19 + jj];
        at = c.cs[k * c.css + jj];
    }
    const bool live = grp && j < nk;
    const bool unused = Q == GPUTX_NEW_ORDER_RB && live && item == T.dims[3];
    volatile GTX_LDS uint8_t* tag = sw.tag + 512;
    const uint32_t h = (at - lds_addr(tab.slot)) >> 4;
    if (live) tag[h] = (uint8_t)lane;
    bool clash = false;
    int64_t old = 0;
    if (live) {  // LDS operations of a wave complete in order
        clash = tag[h] != (uint8_t)lane;
        old = *(GTX_LDS const int64_t*)(uintptr_t)at;
    }
    if (__any(clash || unused)) return false;
    int32_t nv = 0;
    if (live) {
        *seen &= at;
        int64_t s = (int64_t)(int32_t)old - q;
        if (s < 10) s += 91;
        nv = to_i32(s);
        *(GTX_LDS int64_t*)(uintptr_t)at = (int64_t)nv;
    }
    // result 0: the item count; result 1 + r: item r's new quantity
    if (grp) {
        if (j < 15) c.res[k * c.rs + 1 + j] = live ? (int64_t)nv : 0;
        else c.res[k * c.rs] = nk;
    }
    return true;
}

// Up to four consecutive subscriber reads at once, sixteen lanes each (lane
// 16 g + j reads field j of the g-th, transaction kg): reads with no write
// between them see the same values in any order.
__device__ __forceinline__ void wave_get_sub_group(const PartChunk& c, int k0, int k1, int k2, int k3, int G,
                                                   uint32_t* seen) {
    constexpr int NF = proc_cells(GPUTX_GET_SUB);
    const int lane = lane_id();
    const int g = lane >> 4, j = lane & 15;
    const int k = g == 0 ? k0 : g == 1 ? k1 : g == 2 ? k2 : k3;
    if (g < G && j < NF) {
        const uint32_t at = c.cs[k * c.css + j];
        *seen &= at;
        c.res[k * c.rs + j] = *(GTX_LDS const int64_t*)(uintptr_t)at;
    }
}

__device__ __forceinline__ int32_t wave_payment(const PartChunk& c, int k, const WaveTxn& x, uint32_t* seen) {
    const int lane = lane_id();
    if (lane < 3) {
        *seen &= x.at;
        GTX_LDS int64_t* cell = (GTX_LDS int64_t*)(uintptr_t)x.at;
        const int64_t nv = wrap_add(*cell, x.a);
        *cell = nv;
        c.res[k * c.rs + lane] = nv;
    }
    return GPUTX_COMMIT;
}

__device__ __forceinline__ int32_t wave_order_status(const PartChunk& c, int k, const WaveTxn& x, uint32_t* seen) {
    if (lane_id() == 0) {
        *seen &= x.at;
        c.res[k * c.rs] = *(GTX_LDS const int64_t*)(uintptr_t)x.at;
    }
    return GPUTX_COMMIT;
}

// Maps v -> a ? v + b : b (wrapping add; a is 0 or 1).  A lane composes its
// map after the one it receives; lanes without a source receive the
// identity (1, 0).
template <int CTRL, int ROWS>
__device__ __forceinline__ void dpp_affine_step(int& a, int64_t& b) {
    const uint64_t ub = (uint64_t)b;
    const int pa = __builtin_amdgcn_update_dpp(1, a, CTRL, ROWS, 0xf, false);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)ub, CTRL, ROWS, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(ub >> 32), CTRL, ROWS, 0xf, false);
    const int64_t pb = (int64_t)(((uint64_t)hi << 32) | lo);
    b = a ? wrap_add(pb, b) : b;
    a &= pa;
}
__device__ __forceinline__ void wave_affine_scan(int& a, int64_t& b) {
    dpp_affine_step<kDppRowShr + 1, 0xf>(a, b);
    dpp_affine_step<kDppRowShr + 2, 0xf>(a, b);
    dpp_affine_step<kDppRowShr + 4, 0xf>(a, b);
    dpp_affine_step<kDppRowShr + 8, 0xf>(a, b);
    dpp_affine_step<kDppBcast15, 0xa>(a, b);
    dpp_affine_step<kDppBcast31, 0xc>(a, b);
}

__device__ __forceinline__ int64_t wave_shr1(int64_t v) {  // lane i gets lane i - 1's v, lane 0 gets 0
    constexpr int kDppWaveShr1 = 0x138;
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, kDppWaveShr1, 0xf, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), kDppWaveShr1, 0xf, 0xf, false);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}


// Sort a window's lanes (transactions k0 .. k0+n-1, lane j holding k0 + j,
// naming the cell at LDS address id) into groups naming the same cell,
// stably: every lane stores its lane number in the tag byte of its cell's
// slot, and the value it reads back (one of the group's lanes, the same for
// the whole group) names the group; each lane ORs its bit into that lane's
// group mask, then reads the mask, and the groups are laid out in the order
// of those lanes.  Returns the lane's sorted slot, and whether it starts or
// ends its group.  Lanes that are not live are groups of their own.  Needs
// all 64 lanes of the wave.
__device__ __forceinline__ int group_ordinal(const CellTab& tab, GTX_LDS uint8_t* mine, uint32_t id, bool live,
                                             bool& head, bool& last) {
    const int j = lane_id();
    GTX_LDS uint64_t* gmask = (GTX_LDS uint64_t*)mine;
    // volatile: the read must see whichever lane's store landed, not this lane's
    volatile GTX_LDS uint8_t* tag = mine + 512;
    const uint32_t h = (id - lds_addr(tab.slot)) >> 4;  // the sink is slot 1 << bits
    gmask[j] = 0;
    int rep = j;
    if (live) {
        tag[h] = (uint8_t)j;
        rep = tag[h];
    }
    __hip_atomic_fetch_or(&gmask[rep], 1ull << j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    const uint64_t eq = __hip_atomic_load(&gmask[rep], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    const int rank = __popcll(eq & lanemask_lt());
    const int size = __popcll(eq);
    const int own = rep == j ? size : 0;
    head = rank == 0;
    last = rank == size - 1;
    return __shfl(wave_incl_sum_dpp(own) - own, rep) + rank;
}
// Lane to (push): the value lands in lane `to` (a permutation of the wave).
__device__ __forceinline__ uint32_t push32(int to, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_ds_permute(to * 4, (int)v);
}
__device__ __forceinline__ int64_t push64(int to, int64_t v) {
    const uint64_t u = (uint64_t)v;
    return (int64_t)(((uint64_t)push32(to, (uint32_t)(u >> 32)) << 32) | push32(to, (uint32_t)u));
}

// Cellwise procedures (proc_cellwise) run a window of up to 64 transactions
// at a time, one cell ordinal after the other; cells of different ordinals
// are different columns, so ordinals do not interact and the serial waves
// share them out (ordinal r goes to serial wave r mod nsw).  A transaction's
// effect on its cell is the map v -> a ? v + b : b (cell_affine), and such
// maps compose into maps of the same form, so the value a transaction sees
// -- the maps of the earlier transactions on the same cell applied in order
// to the staged value -- is a prefix composition.  group_ordinal sorts the
// window's transactions into groups naming the same cell, each contiguous
// and in timestamp order; lane s takes the transaction at sorted slot s.  The
// group's first map is replaced by the constant it yields from the staged
// value, so one scan over the wave gives every lane the value after its
// transaction without anything crossing a group boundary, and the lane
// before it holds the value before.  The last lane of each group writes the
// cell.  The result equals running the window's transactions one after
// another.  Read-only procedures see the staged values and need no grouping.
// Each lane stores its transaction's result of ordinal r straight to the
// results array (ordinal r yields result column r, or column 0 for
// single-cell procedures).
template <int P>
__device__ __forceinline__ void lanes_window(const BulkArgs& a, const PartChunk& c, const CellTab& tab,
                                             const SerialWave& sw, int k0, int n) {
    constexpr int NP = proc_params(P);
    constexpr int NC = proc_cells(P);
    constexpr bool kW = proc_cell_writes(P);
    const int s = lane_id();
    const bool live = s < n;
#pragma unroll
    for (int r = 0; r < NC; ++r) {
        if (r % sw.nsw != sw.ws) continue;
        // this lane's transaction in window order
        const int kj = k0 + s;  // < cw: every row read exists
        uint32_t id = c.cs[kj * c.css + r];
        int64_t p[NP];
#pragma unroll
        for (int q = 0; q < NP; ++q) p[q] = c.prm[kj * c.ps + q];
        int64_t init = *(GTX_LDS const int64_t*)(uintptr_t)id;
        int64_t idx = c.idx[kj];
        int64_t old = init;
        bool last = true;
        if constexpr (kW) {
            // take the transaction at this lane's sorted slot instead
            bool hd, ls;
            const int to = group_ordinal(tab, sw.tag, id, live, hd, ls);
            const uint32_t fl = push32(to, (hd ? 1u : 0u) | (ls ? 2u : 0u));
            id = push32(to, id);
#pragma unroll
            for (int q = 0; q < NP; ++q) p[q] = push64(to, p[q]);
            init = push64(to, init);
            idx = push64(to, idx);
            const bool head = fl & 1u;
            last = fl & 2u;
            bool fa;
            int64_t fb;
            cell_affine<P>(r, p, fa, fb);
            int a = fa;
            int64_t b = fb;
            if (head) {
                b = a ? wrap_add(init, b) : b;
                a = 0;
            }
            wave_affine_scan(a, b);
            const int64_t before = wave_shr1(b);
            old = head ? init : before;
        }
        int64_t nv, res;
        bool w;
        int at;
        cell_apply<P>(r, old, p, nv, w, at, res);
        if (live) {  // sorted slots below n hold the live transactions
            if (at >= 0 && at < a.width) a.results[idx * a.width + at] = res;
            if (w && last) *(GTX_LDS int64_t*)(uintptr_t)id = nv;
        }
    }
}

// Cellwise procedures of at most three cells, which a mixed window takes.
__device__ __forceinline__ bool mixed_window_proc(int pc) {
    return pc == GPUTX_DEBIT_CREDIT || pc == GPUTX_PAYMENT || pc == GPUTX_ORDER_STATUS || pc == GPUTX_GET_CF ||
           pc == GPUTX_UPD_SUB_FIELD || pc == GPUTX_UPD_LOC;
}
__device__ __forceinline__ void mixed_cell_map(int pc, int r, const int64_t* p, int64_t old, bool& fa, int64_t& fb,
                                               int64_t& nv, bool& w, int& res_at, int64_t& res, bool apply) {
    switch (pc) {
#define GTX_MIXED(P)                                          \
    case P:                                                   \
        if (apply)                                            \
            cell_apply<P>(r, old, p, nv, w, res_at, res);     \
        else                                                  \
            cell_affine<P>(r, p, fa, fb);                     \
        break;
        GTX_MIXED(GPUTX_DEBIT_CREDIT)
        GTX_MIXED(GPUTX_PAYMENT)
        GTX_MIXED(GPUTX_ORDER_STATUS)
        GTX_MIXED(GPUTX_GET_CF)
        GTX_MIXED(GPUTX_UPD_SUB_FIELD)
        GTX_MIXED(GPUTX_UPD_LOC)
#undef GTX_MIXED
    default:
        break;
    }
}

// A run of G (2..21) transactions of one serial wave's list, all of
// cellwise procedures of at most three cells (mixed_window_proc), as one
// window: lane 3 t + r takes cell ordinal r of the run's t-th transaction
// (b0 + the t-th set bit of run).  A transaction names each of its cells
// once, so lanes in transaction order give each cell's accesses in
// timestamp order, and grouping the lanes by cell and scanning the groups'
// maps gives every access the value before it, as in the window form of one
// procedure (lanes_window) -- whatever the procedures and ordinals that meet
// on a cell.  The last access of each group stores the cell, also when it
// only reads it.  Results go to the chunk's rows; every such procedure
// commits.
__device__ __forceinline__ void mixed_window(const PartChunk& c, const CellTab& tab, const SerialWave& sw, int b0,
                                             int32_t pw, uint64_t run, int G, uint32_t* seen) {
    const int lane = lane_id();
    const int t = lane / 3, r = lane - 3 * t;
    int pos = 0;
    uint64_t mm = run;
    for (int q = 0; q < G; ++q) {
        const int j = __ffsll((unsigned long long)mm) - 1;
        mm &= mm - 1;
        if (t == q) pos = j;
    }
    const int pc = __shfl(pw, pos) & 0xffff;
    const int k = b0 + pos;
    const bool act = t < G && r < proc_cells(pc);
    uint32_t id = 0;
    int64_t p[4] = {0, 0, 0, 0};
    int64_t init = 0;
    if (act) {
        id = c.cs[k * c.css + r];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (q < c.ps) p[q] = c.prm[k * c.ps + q];
        init = *(GTX_LDS const int64_t*)(uintptr_t)id;
        *seen &= id;
    }
    if (!__any(act && proc_cell_writes(pc))) {  // reads only: every access sees the staged value
        if (act) {
            bool fa, w;
            int64_t fb, nv, res;
            int at = -1;
            mixed_cell_map(pc, r, p, init, fa, fb, nv, w, at, res, true);
            if (at >= 0 && at < c.rs) c.res[k * c.rs + at] = res;
        }
        return;
    }
    bool hd, ls;
    const int to = group_ordinal(tab, sw.tag, id, act, hd, ls);
    // each lane takes the access at its sorted slot
    const uint32_t fl = push32(to, (act ? 1u : 0u) | (hd ? 2u : 0u) | (ls ? 4u : 0u) | ((uint32_t)r << 3) |
                                       ((uint32_t)pc << 8));
    id = push32(to, id);
    init = push64(to, init);
#pragma unroll
    for (int q = 0; q < 4; ++q) p[q] = push64(to, p[q]);
    const int kk = (int)push32(to, (uint32_t)k);
    const bool live = fl & 1u, head = fl & 2u, last = fl & 4u;
    const int rr = (fl >> 3) & 3, pcx = (int)(fl >> 8);
    bool fa = false;
    int64_t fb = 0, nv = 0, res = 0;
    bool w = false;
    int at = -1;
    if (live) mixed_cell_map(pcx, rr, p, 0, fa, fb, nv, w, at, res, false);
    int A = fa;
    int64_t B = fb;
    if (head) {
        B = A ? wrap_add(init, B) : B;
        A = 0;
    }
    wave_affine_scan(A, B);
    const int64_t before = wave_shr1(B);
    const int64_t old = head ? init : before;
    if (live) {
        mixed_cell_map(pcx, rr, p, old, fa, fb, nv, w, at, res, true);
        if (at >= 0 && at < c.rs) c.res[kk * c.rs + at] = res;
        // the group's last access leaves the cell's final value, whether or
        // not its own procedure writes (a read after writes must not drop
        // them)
        if (last) *(GTX_LDS int64_t*)(uintptr_t)id = w ? nv : old;
    }
}

// The chunk's cnt transactions run in order against the staged cells: as
// windows (cellwise procedures, all serial waves; outcomes go straight to
// the status and results arrays, and part_serial returns true), or on lane 0
// of the first serial wave (statuses and results go to the chunk's LDS rows,
// which the caller writes out).  P != 0: all run procedure P with descriptor
// T; P == 0: mixed types.  The LDS parameter rows past a transaction's own
// are zero, so they are read without a bound.
//
// Narrow procedures whose cell ordinals cannot alias across transactions
// (proc_typed_cells) run as a forwarding pipeline (serial_fwd_step), which
// keeps the LDS latency off the dependence chain.  Every procedure also runs
// through the generic path, which checks that each ordinal it names was
// staged, whenever a chunk mixes types.
template <int P, int MC>
__device__ __forceinline__ bool part_serial(const BulkArgs& a, const DevType& T, const PartChunk& c,
                                            const CellTab& tab, const SerialWave& sw, int cnt,
                                            int64_t& committed, int64_t& aborted) {
    constexpr int NP = proc_params(P);  // parameters the procedure can read
    constexpr int NR = proc_results(P); // results it can write (P == 0: up to res_rows)
    constexpr int NC = proc_cells(P);   // cells it can name
    constexpr bool ahead = P != 0 && NP <= 8 && NC <= 4 && proc_typed_cells(P);
    if constexpr (P != 0 && proc_cellwise(P) && proc_typed_cells(P) && NP <= 8) {
      if (a.part_scan) {
        for (int k0 = 0; k0 < cnt; k0 += 64) lanes_window<P>(a, c, tab, sw, k0, min(64, cnt - k0));
        if (sw.ws == 0) {  // every cellwise procedure commits; the other result columns are zero
            if (lane_id() == 0) {
                committed += cnt;
                atomicAdd((unsigned long long*)&a.ws.st->scan_chunks, 1ull);
            }
            constexpr int NR = proc_results(P);
            for (int r = lane_id(); r < cnt; r += 64) {
                const int64_t i = c.idx[r];
                a.status[i] = GPUTX_COMMIT;
                for (int q = NR; q < a.width; ++q) a.results[i * a.width + q] = 0;
            }
        }
        return true;
      }
    }
    if constexpr (P == 0 || P == GPUTX_NEW_ORDER || P == GPUTX_NEW_ORDER_RB) {
        // one serial wave per cell class, which lists its own transactions of
        // each 64 with one ballot.  With the scan form, several transactions
        // at once where that leaves the serial result: runs of cellwise ones
        // as a window, up to four disjoint new-orders or four subscriber
        // reads; otherwise one at a time, the order-entry procedures with
        // the whole wave, others on lane 0.
        if constexpr (P != 0)
            if (T.cell_class % sw.nsw != sw.ws) return false;
        const int lane = lane_id();
        uint32_t seen = ~0u;
        int n_commit = 0, n_abort = 0;
        bool multi = false;  // some transactions ran side by side (the scan form)
        for (int b0 = 0; b0 < cnt; b0 += 64) {
            const int r = b0 + lane;
            int32_t pw = 0, tw = 0;
            if (r < cnt) {
                pw = P != 0 ? (P | (T.cell_class << 16)) : c.proc[r];
                if constexpr (P == 0) tw = c.t[r];
            }
            uint64_t m = __ballot(r < cnt && (pw >> 16) % sw.nsw == sw.ws);
            while (m) {
                const int j = __ffsll((unsigned long long)m) - 1;
                const int k = b0 + j;
                const int32_t pc = __builtin_amdgcn_readlane(pw, j);
                const int32_t tk = P != 0 ? 0 : __builtin_amdgcn_readlane(tw, j);
                DevType Tm;
                if constexpr (P == 0) Tm = dev_type_uniform(a.types, tk);
                const DevType& Tk = P != 0 ? T : Tm;
                const int pq = pc & 0xffff;
                if (a.part_scan && mixed_window_proc(pq)) {
                    // this one and the cellwise ones right after it, up to 21
                    uint64_t run = 0, mm = m;
                    int G = 0;
                    while (mm && G < 21) {
                        const int jn = __ffsll((unsigned long long)mm) - 1;
                        if (!mixed_window_proc(__builtin_amdgcn_readlane(pw, jn) & 0xffff)) break;
                        run |= 1ull << jn;
                        mm &= mm - 1;
                        ++G;
                    }
                    if (G >= 8) {  // shorter runs are faster one at a time
                        mixed_window(c, tab, sw, b0, pw, run, G, &seen);
                        multi = true;
                        n_commit += G;
                        m = mm;
                        continue;
                    }
                }
                if (a.part_scan && pq == GPUTX_GET_SUB && proc_cells(GPUTX_GET_SUB) <= MC) {
                    // this one and up to three more reads of the subscriber row that follow it
                    int k1 = k, k2 = k, k3 = k, G = 1;
                    uint64_t mm = m & (m - 1);
#pragma unroll
                    for (int e = 1; e < 4; ++e) {
                        if (!mm) break;
                        const int jn = __ffsll((unsigned long long)mm) - 1;
                        if ((__builtin_amdgcn_readlane(pw, jn) & 0xffff) != GPUTX_GET_SUB) break;
                        if (e == 1) k1 = b0 + jn;
                        if (e == 2) k2 = b0 + jn;
                        if (e == 3) k3 = b0 + jn;
                        G = e + 1;
                        mm &= mm - 1;
                    }
                    wave_get_sub_group(c, k, k1, k2, k3, G, &seen);
                    multi = multi || G > 1;
                    n_commit += G;
                    m = mm;
                    continue;
                }
                constexpr bool kNewOrder = MC >= proc_cells(GPUTX_NEW_ORDER);
                if (kNewOrder && a.part_scan && (pq == GPUTX_NEW_ORDER || pq == GPUTX_NEW_ORDER_RB)) {
                    // this one and up to three more of its type that follow it
                    int k1 = k, k2 = k, k3 = k, G = 1;
                    uint64_t mm = m & (m - 1);
#pragma unroll
                    for (int e = 1; e < 4; ++e) {
                        if (!mm) break;
                        const int jn = __ffsll((unsigned long long)mm) - 1;
                        if (__builtin_amdgcn_readlane(pw, jn) != pc ||
                            (P == 0 && __builtin_amdgcn_readlane(tw, jn) != tk))
                            break;
                        if (e == 1) k1 = b0 + jn;
                        if (e == 2) k2 = b0 + jn;
                        if (e == 3) k3 = b0 + jn;
                        G = e + 1;
                        mm &= mm - 1;
                    }
                    const bool done =
                        pq == GPUTX_NEW_ORDER
                            ? wave_new_order_group<GPUTX_NEW_ORDER>(Tk, c, tab, sw, k, k1, k2, k3, G, &seen)
                            : wave_new_order_group<GPUTX_NEW_ORDER_RB>(Tk, c, tab, sw, k, k1, k2, k3, G, &seen);
                    if (done) {
                        multi = multi || G > 1;
                        n_commit += G;
                        m = mm;
                        continue;
                    }
                }
                m &= m - 1;
                WaveTxn x;
                wave_fetch(c, k, pc, x);
                int32_t s = GPUTX_INVALID;
                switch (kNewOrder ? pq : (pq == GPUTX_NEW_ORDER || pq == GPUTX_NEW_ORDER_RB) ? -1 : pq) {
                case GPUTX_NEW_ORDER:
                    if constexpr (kNewOrder) s = wave_new_order<GPUTX_NEW_ORDER>(Tk, c, k, x, &seen);
                    break;
                case GPUTX_NEW_ORDER_RB:
                    if constexpr (kNewOrder) s = wave_new_order<GPUTX_NEW_ORDER_RB>(Tk, c, k, x, &seen);
                    break;
                case GPUTX_PAYMENT: s = wave_payment(c, k, x, &seen); break;
                case GPUTX_ORDER_STATUS: s = wave_order_status(c, k, x, &seen); break;
                default: {
                    int32_t s0 = 0;
                    if (lane == 0) {
                        switch (pq) {
#define GTX_ONE(Q)                                                    \
    case Q:                                                           \
        if constexpr (proc_cells(Q) <= MC)                            \
            s0 = serial_one<Q>(Tk, c, k, &seen);                      \
        else                                                          \
            seen = 0;                                                 \
        break;
                            GTX_ONE(GPUTX_DEBIT_CREDIT)
                            GTX_ONE(GPUTX_GET_SUB)
                            GTX_ONE(GPUTX_GET_CF)
                            GTX_ONE(GPUTX_UPD_SUB_FIELD)
                            GTX_ONE(GPUTX_UPD_LOC)
                            GTX_ONE(GPUTX_INS_CF)
                            GTX_ONE(GPUTX_DEL_CF)
#undef GTX_ONE
                        default:
                            s0 = GPUTX_INVALID;
                            seen = 0;  // a staged transaction of no known procedure
                        }
                    }
                    s = __shfl(s0, 0);
                }
                }
                n_commit += s == GPUTX_COMMIT;
                n_abort += s == GPUTX_ABORT;
            }
        }
        if (lane == 0) {
            committed += n_commit;
            aborted += n_abort;
            if (multi) atomicAdd((unsigned long long*)&a.ws.st->scan_chunks, 1ull);
        }
        if (__any(!(seen & 8u))) {
            if (lane == 0) fail(a.ws.st, GPUTX_E_INTERNAL);
        }
        return false;
    }
    // lane 0 of one serial wave per cell class: classes never share a cell
    if (lane_id() != 0) return false;
    if constexpr (P != 0)
        if (T.cell_class % sw.nsw != sw.ws) return false;
    uint32_t seen = ~0u;
    if constexpr (ahead) {
        SerialRegs<NP, NC> A, B;  // transactions 0 and 1 (row 1 exists even if cnt == 1)
#pragma unroll
        for (int r = 0; r < NC; ++r) {
            A.ids[r] = c.cs[r];
            B.ids[r] = c.cs[c.css + r];
        }
#pragma unroll
        for (int r = 0; r < NP; ++r) {
            A.prm[r] = c.prm[r];
            B.prm[r] = c.prm[c.ps + r];
        }
#pragma unroll
        for (int r = 0; r < NC; ++r) A.val[r] = *(GTX_LDS const int64_t*)(uintptr_t)A.ids[r];
        SerialRegs<NP, NC> C;
        int k = 0;
        for (; k + 2 < cnt; k += 3) {  // three steps with rotated register sets: no moves
            serial_fwd_step<P, NP, NC, NR>(T, c, k, cnt, A, B, C, committed, aborted);
            serial_fwd_step<P, NP, NC, NR>(T, c, k + 1, cnt, B, C, A, committed, aborted);
            serial_fwd_step<P, NP, NC, NR>(T, c, k + 2, cnt, C, A, B, committed, aborted);
        }
        if (k < cnt) serial_fwd_step<P, NP, NC, NR>(T, c, k, cnt, A, B, C, committed, aborted);
        if (k + 1 < cnt) serial_fwd_step<P, NP, NC, NR>(T, c, k + 1, cnt, B, C, A, committed, aborted);
    } else if constexpr (P != 0) {
        int n_commit = 0, n_abort = 0;
        for (int k = 0; k < cnt; ++k) {
            const int32_t s = serial_one<P>(T, c, k, &seen);
            n_commit += s == GPUTX_COMMIT;
            n_abort += s == GPUTX_ABORT;
        }
        committed += n_commit;
        aborted += n_abort;
    }
    if (!(seen & 8u)) fail(a.ws.st, GPUTX_E_INTERNAL);
    return false;
}


__host__ __device__ inline size_t part_chunk_bytes(const BulkArgs& a, int cw) {
    return (size_t)8 * part_rs(a.res_rows) * cw + (size_t)8 * part_ps(a.prm_rows) * (cw + kChunkSpare) +
           (size_t)8 * cw + (size_t)4 * 3 * cw + (size_t)4 * part_css(a.cells_max) * (cw + kChunkSpare);
}
// Per serial wave: 64 group masks (8 bytes each), then a tag byte per slot.
__host__ __device__ inline int part_tstride(int bits) { return 512 + (1 << bits) + 16; }
size_t part_wave_lds(const BulkArgs& a) {
    return part_chunk_bytes(a, 64) + ((size_t)sizeof(CellSlot) << a.cell_bits) + sizeof(CellSlot) +
           (size_t)4 * (64 * a.cells_max + 4) + part_tstride(a.cell_bits);
}
// Serial waves of the pipelined form: cellwise procedures share their cell
// ordinals among them (debit-credit and payment have three).
constexpr int kPipeSerial = 3;
// The most cells per transaction the pipelined form of width cw is built
// for: the wide forms' cell tables could not hold more than this many per
// transaction below their fill limit anyway, so the procedures with more
// (new-order, and the full subscriber read at width 256) are left out of
// them, which keeps their registers for the procedures that do run there.
constexpr int kAllCells = proc_cells(0);  // the most any procedure names
__host__ __device__ constexpr int part_pipe_cells(int cw) { return cw >= 256 ? 8 : cw >= 128 ? 14 : kAllCells; }
// The pipelined form's table holds at most half of its slots: it
// is flushed before a chunk could take it past that.
__host__ __device__ inline int part_pipe_fill(int cap) { return cap / 2; }
size_t part_pipe_lds(const BulkArgs& a, int cw) {
    return 2 * part_chunk_bytes(a, cw) + ((size_t)sizeof(CellSlot) << a.pipe_bits) + sizeof(CellSlot) +
           (size_t)4 * (part_pipe_fill(1 << a.pipe_bits) + 4) + (size_t)kPipeSerial * part_tstride(a.pipe_bits);
}
// Dynamic LDS a PART workgroup may use: the device's opt-in per-workgroup
// limit (160 KB on gfx950), or the default 64 KB if raising it fails.
static size_t g_part_lds_limit = 64 * 1024;
// The pipelined form of width cw runs when its LDS fits, one chunk's cells
// fit in half the table (so that several chunks fit below the fill limit),
// and no registered procedure of the bulk names more cells than the form's
// instance is built for.
static bool part_pipe_fits(const BulkArgs& a, int cw) {
    return a.part_pipeline && part_pipe_lds(a, cw) <= g_part_lds_limit &&
           (int64_t(1) << a.pipe_bits) >= int64_t(2) * cw * a.cells_max && a.cells_max <= part_pipe_cells(cw);
}

__device__ __forceinline__ PartChunk part_chunk_at(unsigned char* base, const BulkArgs& a, int cw) {
    PartChunk c;
    c.cw = cw;
    c.ps = part_ps(a.prm_rows);
    c.css = part_css(a.cells_max);
    c.rs = part_rs(a.res_rows);
    c.res = reinterpret_cast<int64_t*>(base);
    c.prm = c.res + cw * c.rs;
    c.idx = c.prm + (cw + kChunkSpare) * c.ps;
    c.t = reinterpret_cast<int32_t*>(c.idx + cw);
    c.proc = c.t + cw;
    c.st = c.proc + cw;
    c.cs = reinterpret_cast<uint32_t*>(c.st + cw);
    return c;
}

// A staging lane's transaction as read a step before its cells are claimed,
// from its record (k_part_gather): serial position p, type, input index and
// first kStagePrm parameters (wider signatures read the rest when claimed).
// Timestamps and append rows serve only the appends, which k_part_gather
// wrote.
constexpr int kStagePrm = 8;
struct StagedTxn {
    int64_t i;
    int32_t p, t;
    int64_t prm[kStagePrm];
};
__device__ __forceinline__ void stage_load(const BulkArgs& a, int32_t p, StagedTxn& x) {
    const int64_t* r = a.ws.rec + (int64_t)p * a.rec_words;
    const uint64_t w0 = (uint64_t)r[0];
    x.p = p;
    x.t = (int32_t)(w0 >> 32);
    x.i = (int64_t)(uint32_t)w0;
#pragma unroll
    for (int k = 0; k < kStagePrm; ++k) x.prm[k] = k < a.prm_rows ? r[1 + k] : 0;
}

// One lane per transaction of a chunk (the lane's row): write its signature
// into the chunk buffer and stage its cells in the table (its appended rows
// were written by k_part_gather).  The cells are claimed first, then the won
// cells' values are read together.
// P != 0: every transaction of the wave has type tu, of procedure P; its
// descriptor is then read through the scalar cache, and only P's parameters
// and cell ordinals are handled.
template <int P>
__device__ __forceinline__ uint32_t part_claim(const BulkArgs& a, const PartChunk& c, const CellTab& tab,
                                               const StagedTxn& s, int lane, int32_t tu, uint32_t& pending) {
    // values loaded during the claims for procedures of a few cells
    constexpr int NV = (P != 0 && proc_cells(P) <= 4) ? proc_cells(P) : 0;
    constexpr int NP = P != 0 ? proc_params(P) : GTX_MAX_PARAMS;
    const int32_t t = P != 0 ? tu : s.t;
    DevType Tu;
    if constexpr (P != 0) Tu = dev_type_uniform(a.types, tu);
    const DevType& T = P != 0 ? Tu : a.types[t];
    TxnIn x;
    x.t = t;
    x.i = s.i;
    x.ts = 0;
    x.np = min(a.n_params, T.n_params);
#pragma unroll
    for (int k = 0; k < GTX_MAX_PARAMS; ++k)
        x.prm[k] = (k >= NP || k >= x.np) ? 0
                 : k < kStagePrm ? s.prm[k] : a.ws.rec[(int64_t)s.p * a.rec_words + 1 + k];
    const int ncs = P != 0 ? proc_cells(P) : c.css;  // ordinals the serial side can read
    for (int r = 0; r < ncs; ++r) c.cs[lane * c.css + r] = cell_sink_addr(tab);
    CellClaim<NV, P == GPUTX_NEW_ORDER || P == GPUTX_NEW_ORDER_RB> claim;
    claim.tab = tab;
    claim.cs = c.cs + lane * c.css;
    claim.won = 0;
    txn_cells<P>(T, x.prm, claim);
    if constexpr (NV > 0) claim.store_won();
    pending = NV > 0 ? 0u : claim.won;
    x.app0 = 0;
    x.app1 = 0;
    const int rows = P != 0 ? NP : a.prm_rows;  // P's serial code reads only its own
#pragma unroll
    for (int k = 0; k < GTX_MAX_PARAMS; ++k)
        if (k < rows) c.prm[lane * c.ps + k] = x.prm[k];
#pragma unroll
    for (int r = 0; r < GTX_MAX_RESULTS; ++r)
        if (r < a.res_rows) c.res[lane * c.rs + r] = 0;
    c.idx[lane] = x.i;
    c.t[lane] = t;
    c.proc[lane] = T.proc | (T.cell_class << 16);
    c.st[lane] = GPUTX_COMMIT;
    return claim.won;
}

// A transaction of a procedure this kernel instance was built without (it
// names more cells than the instance's chunk width allows; the host never
// sends one): its row gets the sink slot and no procedure, which the serial
// side reports, and the bulk fails.
__device__ __forceinline__ void part_claim_none(const BulkArgs& a, const PartChunk& c, const CellTab& tab,
                                                const StagedTxn& x, int lane) {
    for (int r = 0; r < c.css; ++r) c.cs[lane * c.css + r] = cell_sink_addr(tab);
    c.idx[lane] = x.i;
    c.t[lane] = x.t;
    c.proc[lane] = 0xffff;
    c.st[lane] = GPUTX_INVALID;
    fail(a.ws.st, GPUTX_E_INTERNAL);
}

// The live lanes (c0 + lane < end) claim their transactions, read earlier
// into x, and the wave lists the slots it won.  Returns the lane's won cells
// whose values are still to be loaded.  Needs the whole wave.  MC: the most
// cells per transaction of the procedures compiled in.
template <int MC>
__device__ __forceinline__ uint32_t part_claim_wave(const BulkArgs& a, const PartChunk& c, const CellTab& tab,
                                                    const StagedTxn& x, int64_t c0, int64_t end, int lane,
                                                    int& list0, int& nlisted) {
    const bool live = c0 + lane < end;
    uint32_t won = 0, pending = 0;
    // one pass per type present, its lanes specialised on its procedure with
    // the type's descriptor read once for the wave (the passes run one after
    // another, as divergent lanes would)
    uint64_t left = __ballot(live);
    while (left) {
        const int32_t t0 = __builtin_amdgcn_readlane(x.t, __ffsll((unsigned long long)left) - 1);
        const bool mine = live && x.t == t0;
        left &= ~__ballot(mine);
        if (mine) {
            switch (dev_type_uniform(a.types, t0).proc) {
#define GTX_CLAIM_CASE(P)                                         \
    case P:                                                       \
        if constexpr (proc_cells(P) <= MC)                        \
            won = part_claim<P>(a, c, tab, x, lane, t0, pending); \
        else                                                      \
            part_claim_none(a, c, tab, x, lane);                  \
        break;
                GTX_CLAIM_CASE(GPUTX_DEBIT_CREDIT)
                GTX_CLAIM_CASE(GPUTX_NEW_ORDER)
                GTX_CLAIM_CASE(GPUTX_NEW_ORDER_RB)
                GTX_CLAIM_CASE(GPUTX_PAYMENT)
                GTX_CLAIM_CASE(GPUTX_ORDER_STATUS)
                GTX_CLAIM_CASE(GPUTX_GET_SUB)
                GTX_CLAIM_CASE(GPUTX_GET_CF)
                GTX_CLAIM_CASE(GPUTX_UPD_SUB_FIELD)
                GTX_CLAIM_CASE(GPUTX_UPD_LOC)
                GTX_CLAIM_CASE(GPUTX_INS_CF)
                GTX_CLAIM_CASE(GPUTX_DEL_CF)
#undef GTX_CLAIM_CASE
            default:
                if constexpr (MC >= kAllCells)
                    won = part_claim<0>(a, c, tab, x, lane, 0, pending);
                else
                    part_claim_none(a, c, tab, x, lane);
            }
        }
    }
    // list the won slots: one counter update for the whole wave
    const int nw = __popc(won);
    const int incl = wave_incl_sum_dpp(nw);
    const int total = __builtin_amdgcn_readlane(incl, 63);
    list0 = 0;
    nlisted = total;
    if (total == 0) return pending;
    int e0 = 0;
    if (lane % 64 == 63) e0 = __hip_atomic_fetch_add(tab.nlist, total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    list0 = __builtin_amdgcn_readlane(e0, 63);
    int e = list0 + incl - nw;
    const uint32_t* row = c.cs + lane * c.css;
    const uint32_t base = lds_addr(tab.slot);
    for (uint32_t m = won; m; m &= m - 1) tab.list[e++] = (int32_t)((row[__ffs(m) - 1] - base) >> 4);
    return pending;
}

// The values of the cells a wave won (list entries list0 .. list0 + n - 1),
// spread over its lanes with up to eight loads in flight per lane.  None of
// these cells was in the table before this chunk's claims, so no serial
// wave works on them yet, and a value already loaded during the claims is
// loaded again unchanged (the tables change only at flushes).
__device__ __forceinline__ void list_values_load(const CellTab& tab, int list0, int n) {
    const int lane = lane_id();  // the wave's own lanes (not the chunk's rows)
    for (int b = 0; b < n; b += 8 * 64) {
        int32_t h[8];
        int64_t v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = b + q * 64 + lane;
            h[q] = e < n ? tab.list[list0 + e] : -1;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (h[q] >= 0) v[q] = cell_value_of(cell_val_addr(tab, (uint32_t)h[q]));
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (h[q] >= 0) tab.slot[h[q]].val = v[q];
    }
}

// Stage a chunk whose transactions were read already (x): claim the cells,
// then load the won ones (lane by lane when only procedures of a few cells
// left values to load, else spread over the wave).  Needs the whole wave.
template <int MC>
__device__ __forceinline__ void part_stage_read(const BulkArgs& a, const PartChunk& c, const CellTab& tab,
                                                const StagedTxn& x, int64_t c0, int64_t end, int lane) {
    int list0, nlisted;
    const uint32_t pending = part_claim_wave<MC>(a, c, tab, x, c0, end, lane, list0, nlisted);
    if (__any(pending >> 4)) {
        list_values_load(tab, list0, nlisted);
        return;
    }
    const uint32_t* row = c.cs + lane * c.css;
    ValLoads vl;
    claim_values_issue(row, pending, vl);
    claim_values_finish(row, pending, vl);
}
// Read and stage the chunk starting at c0 in one go (no read-ahead).
__device__ __forceinline__ void part_stage(const BulkArgs& a, const PartChunk& c, const CellTab& tab,
                                           int64_t c0, int64_t end, int lane) {
    StagedTxn x;
    x.t = 0;
    if (c0 + lane < end) stage_load(a, (int32_t)(c0 + lane), x);
    part_stage_read<kAllCells>(a, c, tab, x, c0, end, lane);
}

// A serial wave writes the statuses and results of the chunk's transactions
// it ran: those of its cell classes (it reads no global memory, so the stores
// never hold it up).
__device__ __forceinline__ void part_writeout_own(const BulkArgs& a, const PartChunk& c, int cnt, int lane,
                                                  const SerialWave& sw) {
    for (int r = lane; r < cnt; r += 64) {
        if ((c.proc[r] >> 16) % sw.nsw != sw.ws) continue;
        const int64_t i = c.idx[r];
        a.status[i] = c.st[r];
        int64_t* out = a.results + i * a.width;
#pragma unroll
        for (int q = 0; q < GTX_MAX_RESULTS; ++q)
            if (q < a.width) out[q] = q < a.res_rows ? c.res[r * c.rs + q] : 0;
        for (int q = GTX_MAX_RESULTS; q < a.width; ++q) out[q] = 0;
    }
}

// The owning lanes write the chunk's statuses and results.
__device__ __forceinline__ void part_writeout(const BulkArgs& a, const PartChunk& c, int64_t c0,
                                              int64_t end, int lane) {
    if (c0 + lane >= end) return;
    const int64_t i = c.idx[lane];
    a.status[i] = c.st[lane];
    int64_t* out = a.results + i * a.width;
#pragma unroll
    for (int r = 0; r < GTX_MAX_RESULTS; ++r)
        if (r < a.width) out[r] = r < a.res_rows ? c.res[lane * c.rs + r] : 0;
    for (int r = GTX_MAX_RESULTS; r < a.width; ++r) out[r] = 0;
}

// Written cells back to the tables; the listed slots are emptied.  The
// caller resets the list count after a barrier.
__device__ __forceinline__ void part_flush(const CellTab& tab, int tid, int nthreads) {
    const int ncl = *tab.nlist;
    for (int e = tid; e < ncl; e += nthreads) {
        const int32_t h = tab.list[e];
        const uint64_t sk = tab.slot[h].key;
        const int64_t sv = tab.slot[h].val;
        if (sk & 1) {
            const uint64_t addr = sk & ~(uint64_t)3;
            if (sk & 2) *(GTX_GLOBAL int64_t*)addr = sv;
            else *(GTX_GLOBAL int32_t*)addr = (int32_t)sv;
        }
        tab.slot[h].key = 0;
    }
}

// The serial waves run the chunk, specialised on its procedure when every
// transaction of the chunk has the same type.  Returns true when the
// outcomes went straight to the status and results arrays (window form);
// otherwise they are in the chunk's rows.
template <int MC>
__device__ __forceinline__ bool part_run_chunk(const BulkArgs& a, const PartChunk& c, const CellTab& tab,
                                               const SerialWave& sw, int cnt, int lane, int64_t& committed,
                                               int64_t& aborted) {
    const int t0 = __builtin_amdgcn_readfirstlane(c.t[0]);
    bool differ = false;
    for (int e = lane; e < cnt; e += 64) differ = differ || c.t[e] != t0;
    const bool uniform = __ballot(differ) == 0;
    const DevType T0 = dev_type_uniform(a.types, t0);
    const int proc = uniform ? T0.proc : 0;
    switch (proc) {
#define GTX_PART_CASE(P)                                                              \
    case P:                                                                           \
        if constexpr (proc_cells(P) <= MC)                                            \
            return part_serial<P, MC>(a, T0, c, tab, sw, cnt, committed, aborted);       \
        else                                                                          \
            return part_serial<0, MC>(a, T0, c, tab, sw, cnt, committed, aborted);
        GTX_PART_CASE(GPUTX_DEBIT_CREDIT)
        GTX_PART_CASE(GPUTX_NEW_ORDER)
        GTX_PART_CASE(GPUTX_NEW_ORDER_RB)
        GTX_PART_CASE(GPUTX_PAYMENT)
        GTX_PART_CASE(GPUTX_ORDER_STATUS)
        GTX_PART_CASE(GPUTX_GET_SUB)
        GTX_PART_CASE(GPUTX_GET_CF)
        GTX_PART_CASE(GPUTX_UPD_SUB_FIELD)
        GTX_PART_CASE(GPUTX_UPD_LOC)
        GTX_PART_CASE(GPUTX_INS_CF)
        GTX_PART_CASE(GPUTX_DEL_CF)
#undef GTX_PART_CASE
    default:
        return part_serial<0, MC>(a, T0, c, tab, sw, cnt, committed, aborted);
    }
}

// Every row of a chunk's address array starts at the sink slot, so reads
// ahead past the chunk's last transaction always find an address inside the
// table.
__device__ __forceinline__ void part_init_rows(const PartChunk& c, const CellTab& tab, int tid, int nthreads) {
    for (int e = tid; e < (c.cw + kChunkSpare) * c.css; e += nthreads) c.cs[e] = cell_sink_addr(tab);
}

__device__ __forceinline__ CellTab part_table_at(unsigned char* base, int bits, int list_cap) {
    CellTab tab;
    tab.bits = bits;
    tab.slot = (GTX_LDS CellSlot*)base;
    tab.list = (GTX_LDS int32_t*)(tab.slot + (1 << bits) + 1);
    tab.nlist = tab.list + list_cap;
    tab.tag = (GTX_LDS uint8_t*)(tab.nlist + 4);
    tab.tstride = part_tstride(bits);
    return tab;
}

// One wave per long partition (Section 5.2).  For each chunk of 64 of the
// partition's transactions the lanes read the records into LDS and stage
// every cell the chunk may use in the LDS cell table; the wave then runs the
// 64 in order against the table (part_run_chunk); finally the lanes write
// statuses and results if the chunk's form left them in LDS, and the cells
// that were written.  Workgroups take long partitions in turn.
__global__ __launch_bounds__(64) void k_part_wave(BulkArgs a) {
    GtxState* st = a.ws.st;
    if (failed(st) || st->chosen != GPUTX_PART || (int)blockIdx.x >= st->n_heads) return;
    extern __shared__ __attribute__((aligned(16))) unsigned char part_lds[];
    const int lane = lane_id();
    const PartChunk c = part_chunk_at(part_lds, a, 64);
    const CellTab tab = part_table_at(part_lds + part_chunk_bytes(a, 64), a.cell_bits, 64 * a.cells_max);
    for (int s = lane; s < (1 << a.cell_bits); s += 64) tab.slot[s].key = 0;
    part_init_rows(c, tab, lane, 64);
    if (lane == 0) *tab.nlist = 0;
    __syncthreads();

    const int nh = st->n_heads;
    const SerialWave sw{0, 1, tab.tag};
    int64_t committed = 0, aborted = 0;
    for (int b = blockIdx.x; b < nh; b += gridDim.x) {
        const int64_t lo = a.ws.heads[b], end = a.ws.heads[b + 1];
        if (end - lo < a.long_part) continue;  // a lane of k_part runs it
        for (int64_t c0 = lo; c0 < end; c0 += 64) {
            part_stage(a, c, tab, c0, end, lane);
            __syncthreads();
            const bool written =
                part_run_chunk<kAllCells>(a, c, tab, sw, (int)min<int64_t>(64, end - c0), lane, committed, aborted);
            __syncthreads();
            if (!written) part_writeout(a, c, c0, end, lane);
            part_flush(tab, lane, 64);
            __syncthreads();
            if (lane == 0) *tab.nlist = 0;
            __syncthreads();
        }
    }
    add_counts(st, committed, aborted);
}

// Pipelined PART: one workgroup per long partition at a time.  The
// kPipeSerial serial waves run chunk k (CW transactions) in timestamp order
// (the window form shares the cell ordinals among them; otherwise lane 0 of
// the first runs the chunk) and write out its outcomes, while the CW / 64
// staging waves, one lane per transaction, stage chunk k+1 in the other
// buffer.  The cell table persists across chunks (a cell chunk k+1
// shares with chunk k is found staged, with chunk k's writes applied by the
// time chunk k+1 runs); it is flushed and emptied when a further chunk might
// fill it past part_pipe_fill, and at the end of each partition, at points
// where no wave probes it, so linear probing never sees a deleted slot.
template <int CW>
__global__ __launch_bounds__(64 * kPipeSerial + CW) void k_part_pipe(BulkArgs a) {
    constexpr int cw = CW;
    constexpr int MC = part_pipe_cells(CW);
    constexpr int nser = 64 * kPipeSerial;
    constexpr int nthr = nser + cw;
    GtxState* st = a.ws.st;
    extern __shared__ __attribute__((aligned(16))) unsigned char part_lds[];
    const int tid = threadIdx.x;
    const bool serial = __builtin_amdgcn_readfirstlane(tid) < nser;
    const int lane = tid & 63;
    const int sl = tid - nser;  // staging lane: the transaction's column in the chunk
    const size_t cb = part_chunk_bytes(a, cw);
    auto buf = [&](int64_t k) { return part_chunk_at(part_lds + (k & 1) * cb, a, cw); };
    const int cap = 1 << a.pipe_bits;
    const CellTab tab = part_table_at(part_lds + 2 * cb, a.pipe_bits, part_pipe_fill(cap));
    GTX_LDS int32_t* flag = tab.nlist + 1;  // [2] flush before the next chunk: the step's stamp
    // one decision for the whole workgroup (another workgroup may fail the
    // bulk meanwhile; all waves must still meet at every barrier)
    if (tid == 0) flag[0] = !failed(st) && st->chosen == GPUTX_PART && (int)blockIdx.x < st->n_heads;
    __syncthreads();
    if (!flag[0]) return;
    for (int s = tid; s < cap; s += nthr) tab.slot[s].key = 0;
    part_init_rows(buf(0), tab, tid, nthr);
    part_init_rows(buf(1), tab, tid, nthr);
    if (tid == 0) *tab.nlist = 0;

    if (tid == 0) flag[0] = flag[1] = -1;  // every wave read the decision above

    const int nh = st->n_heads;
    const int ws = __builtin_amdgcn_readfirstlane(tid >> 6);
    const SerialWave sw{ws, kPipeSerial, tab.tag + (serial ? ws : 0) * tab.tstride};
    int64_t committed = 0, aborted = 0;
    int32_t steps = 0;  // chunks run so far, the same count in every wave
    __syncthreads();
    for (int b = blockIdx.x; b < nh; b += gridDim.x) {
        const int64_t lo = a.ws.heads[b], end = a.ws.heads[b + 1];
        if (end - lo < a.long_part) continue;  // a lane of k_part runs it
        const int64_t nch = (end - lo + cw - 1) / cw;
        // A staging wave that finds the table too full to stage chunk k + 1
        // asks for a flush: it stamps flag[k & 1] with the step's number
        // before the barrier that ends the step.  Then every wave writes back
        // and empties the table, and the staging waves stage chunk k + 1
        // (again, for any that staged it already).  The stamp needs no reset,
        // and every wave reads the same value: the slot is written again only
        // two barriers later.  The serial and the staging waves run loops of
        // their own (so that neither holds the other's registers), which
        // meet the same barriers in the same order.
        auto flush_step = [&](int64_t k, auto&& restage) {
            if (flag[k & 1] == steps) {  // same value in every wave
                part_flush(tab, tid, nthr);
                __syncthreads();
                if (tid == 0) *tab.nlist = 0;
                __syncthreads();
                restage();
                __syncthreads();
            }
        };
        if (serial) {
            __syncthreads();  // chunk 0 staged
            for (int64_t k = 0; k < nch; ++k) {
                const int cnt = (int)min<int64_t>(cw, end - lo - cw * k);
                if (!part_run_chunk<MC>(a, buf(k), tab, sw, cnt, lane, committed, aborted))
                    part_writeout_own(a, buf(k), cnt, lane, sw);
                __syncthreads();
                flush_step(k, [] {});
                ++steps;
            }
        } else {
            // A staging lane reads its transaction's record for chunk k + 2
            // (the records lie in partition order) while it claims the cells
            // of chunk k + 1, so a step's global reads do not wait on one
            // another.  xn: the next chunk to claim.
            StagedTxn xn;
            xn.t = 0;
            {
                const int64_t j0 = lo + sl, j1 = j0 + cw;
                StagedTxn x0;
                x0.t = 0;
                if (j0 < end) stage_load(a, (int32_t)j0, x0);
                if (j1 < end) stage_load(a, (int32_t)j1, xn);
                part_stage_read<MC>(a, buf(0), tab, x0, lo, end, sl);
            }
            __syncthreads();  // chunk 0 staged
            for (int64_t k = 0; k < nch; ++k) {
                const int64_t c0 = lo + cw * k;
                StagedTxn xa = xn;
                bool flush = false;
                if (k + 1 < nch) {
                    flush = *tab.nlist + cw * a.cells_max > part_pipe_fill(cap);
                    const int64_t j2 = c0 + 2 * cw + sl;
                    if (j2 < end) stage_load(a, (int32_t)j2, xa);
                    if (!flush) part_stage_read<MC>(a, buf(k + 1), tab, xn, c0 + cw, end, sl);
                }
                if (flush && lane == 0) flag[k & 1] = steps;
                __syncthreads();
                flush_step(k, [&] { part_stage_read<MC>(a, buf(k + 1), tab, xn, c0 + cw, end, sl); });
                ++steps;
                xn = xa;
            }
        }
        // every staged cell; the table is empty after
        part_flush(tab, tid, nthr);
        __syncthreads();
        if (tid == 0) *tab.nlist = 0;
        __syncthreads();
    }
    add_counts(st, committed, aborted);
}

// ---------------------------------------------------------------------------

__global__ void k_finalize(BulkArgs a) {
    GtxState* st = a.ws.st;
    if (threadIdx.x != 0) return;
    gputx_bulk_stats* o = a.stats;
    const int err = st->error;
    if (!err) {
        // only the tables this bulk appends to: bulks on other streams of a
        // batch may be updating the others' counts meanwhile
        for (int k = 0; k < a.n_app; ++k)
            if (st->app_total[k] != 0) a.rowcount[k] += st->app_total[k];
    }
    int64_t app = 0;
    for (int k = 0; k < a.n_app; ++k) app += st->app_total[k];
    o->error = err;
    o->chosen = st->chosen;
    o->n_ops = st->m;
    o->w0 = st->w0;
    o->depth = st->depth;
    o->cross = st->cross;
    o->waves = st->waves;
    o->committed = st->committed;
    o->aborted = st->aborted;
    o->invalid = st->invalid;
    o->appended = err ? 0 : app;
    o->part_scan = st->scan_chunks;
    for (int k = 0; k < 6; ++k) o->reserved[k] = 0;
}

// ---------------------------------------------------------------------------

// First kernel of the execution phase: the batched update must fit the
// append tables (their row counts are final once the previous bulk on the
// same tables has finished).  Nothing runs after a failure.
__global__ void k_exec_gate(BulkArgs a) {
    GtxState* st = a.ws.st;
    if (threadIdx.x != 0 || st->error) return;
    for (int k = 0; k < a.n_app; ++k)
        if (st->app_total[k] > 0 && a.rowcount[k] + st->app_total[k] > a.capacity[k])
            st->error = GPUTX_E_CAPACITY;
}

__global__ void k_reset_state(GtxState* st) {
    int* w = reinterpret_cast<int*>(st);
    for (int i = threadIdx.x; i < (int)(sizeof(GtxState) / 4); i += blockDim.x) w[i] = 0;
}

void launch_empty(const BulkArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_state, dim3(1), dim3(64), 0, s, a.ws.st);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, s, a);
}


void exec_init_attributes(int dev) {
    static bool done = false;
    if (done) return;
    done = true;
    int optin = 0;
    if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess || optin <= 0)
        optin = 64 * 1024;
    const int want = std::min(optin, kPartLdsMax);
    if (hipFuncSetAttribute((const void*)k_part_wave, hipFuncAttributeMaxDynamicSharedMemorySize, want) ==
            hipSuccess &&
        hipFuncSetAttribute((const void*)k_part_pipe<256>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            want) == hipSuccess &&
        hipFuncSetAttribute((const void*)k_part_pipe<128>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            want) == hipSuccess &&
        hipFuncSetAttribute((const void*)k_part_pipe<64>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            want) == hipSuccess)
        g_part_lds_limit = (size_t)want;
    (void)hipGetLastError();
}

int exec_resident_blocks_per_cu() {
    static int cached = -1;
    if (cached >= 0) return cached;
    int b1 = 0, b2 = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b1, k_kset, GTX_BLOCK, 0) != hipSuccess) b1 = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b2, k_tpl, GTX_BLOCK, 0) != hipSuccess) b2 = 1;
    cached = std::max(1, std::min(b1, b2));
    return cached;
}

void launch_part_gather(const BulkArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_part_gather, dim3((unsigned)std::min<int64_t>((a.n + GTX_BLOCK - 1) / GTX_BLOCK, 4096)),
                       dim3(GTX_BLOCK), 0, s, a);
}

static void launch_part_heads(const BulkArgs& a, hipStream_t s) {
    const unsigned nbh = (unsigned)std::max<int64_t>(1, (a.n + kHeadTile - 1) / kHeadTile);
    hipLaunchKernelGGL(k_heads_up, dim3(nbh), dim3(GTX_BLOCK), 0, s, a);
    hipLaunchKernelGGL(k_heads_mid, dim3(1), dim3(GTX_BLOCK), 0, s, a, (int)nbh);
    hipLaunchKernelGGL(k_heads_down, dim3(nbh), dim3(GTX_BLOCK), 0, s, a);
}

void launch_part_sort(const BulkArgs& a, hipStream_t s) {
    SortPlan sp{};
    sp.key_bytes = 4;
    sp.keys[0] = a.ws.qk[0]; sp.keys[1] = a.ws.qk[1];
    sp.vals[0] = a.ws.qv[0]; sp.vals[1] = a.ws.qv[1];
    sp.hist = a.ws.psort_hist; sp.status = a.ws.psort_status; sp.ctrl = a.ws.psort_ctrl;
    sp.cap = a.n; sp.count_dev = nullptr; sp.npass = a.part_passes;
    sp.gate = a.part_early ? nullptr : &a.ws.st->run_part;
    sp.st = a.ws.st; sp.spin_ticks = a.spin_ticks;
    sp.inv = a.ws.qinv;  // the records' grouped positions, for k_part_gather
    sort_pairs(sp, s);
    launch_part_heads(a, s);
}

// The partition kernels over the grouped transactions: long partitions get a
// workgroup each with the LDS cell table (chunks of 256 transactions staged
// by four waves where the LDS fits, else 128 or 64, e.g. for new-order's
// wide signature); short ones a lane each.
static void launch_part_kernels(const BulkArgs& a, hipStream_t s) {
    BulkArgs b = a;
    const bool pipe256 = part_pipe_fits(a, 256);
    const bool pipe128 = !pipe256 && part_pipe_fits(a, 128);
    const bool pipe64 = !pipe256 && !pipe128 && part_pipe_fits(a, 64);
    const bool wave = !pipe256 && !pipe128 && !pipe64 && part_wave_lds(a) <= g_part_lds_limit;
    b.long_part = (pipe256 || pipe128 || pipe64 || wave) ? kLongPart : INT32_MAX;
    const unsigned groups = (unsigned)std::min<int64_t>(a.n / kLongPart + 1, 2048);
    if (pipe256)
        hipLaunchKernelGGL(k_part_pipe<256>, dim3(groups), dim3(64 * kPipeSerial + 256), part_pipe_lds(a, 256), s, b);
    else if (pipe128)
        hipLaunchKernelGGL(k_part_pipe<128>, dim3(groups), dim3(64 * kPipeSerial + 128), part_pipe_lds(a, 128), s, b);
    else if (pipe64)
        hipLaunchKernelGGL(k_part_pipe<64>, dim3(groups), dim3(64 * kPipeSerial + 64), part_pipe_lds(a, 64), s, b);
    else if (wave)
        hipLaunchKernelGGL(k_part_wave, dim3(groups), dim3(64), part_wave_lds(a), s, b);
    const unsigned lanes = (unsigned)std::max<int64_t>(
        1, std::min<int64_t>((std::min<int64_t>(a.n, a.n_parts) + GTX_BLOCK - 1) / GTX_BLOCK, 4096));
    hipLaunchKernelGGL(k_part, dim3(lanes), dim3(GTX_BLOCK), 0, s, b);
}

// serial keys of PART after the partition sort: each transaction's grouped position
__global__ __launch_bounds__(GTX_BLOCK) void k_pgroup_keys(BulkArgs a, int64_t* serial_key) {
    const GtxState* st = a.ws.st;
    if (ld_relaxed(&st->error) != 0 || !st->run_part) return;
    const int fb = a.part_passes & 1;
    for (int64_t d = (int64_t)blockIdx.x * GTX_BLOCK + threadIdx.x; d < a.n; d += (int64_t)gridDim.x * GTX_BLOCK) {
        const uint32_t p = a.ws.qv[fb][d];
        serial_key[p] = a.ws.tty[p] >= 0 ? d : -1;
    }
}

void launch_exec_relaxed(const BulkArgs& a, hipStream_t s, const PhaseMarks& pm, int64_t* serial_key) {
    hipLaunchKernelGGL(k_relaxed_choose, dim3(1), dim3(64), 0, s, a);
    pm.mark(PH_FEATURES, s);
    hipLaunchKernelGGL(k_exec_gate, dim3(1), dim3(64), 0, s, a);
    const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((a.n + GTX_BLOCK - 1) / GTX_BLOCK, 4096));
    if (a.strategy == GPUTX_PART) {
        int32_t* counter = a.ws.grp_cnt;  // [mcap] ints, free without the op sort
        if (a.n_parts + 1 <= a.mcap) {
            hipLaunchKernelGGL(k_pgroup_clear, dim3(nb), dim3(GTX_BLOCK), 0, s, a, counter);
            hipLaunchKernelGGL(k_pgroup_count, dim3((unsigned)((a.n + kGroupTile - 1) / kGroupTile)), dim3(GTX_BLOCK),
                               0, s, a, counter);
            hipLaunchKernelGGL(k_pgroup_scan, dim3(1), dim3(GTX_BLOCK), 0, s, a, counter);
            hipLaunchKernelGGL(k_pgroup_scatter, dim3(nb), dim3(GTX_BLOCK), 0, s, a, (const int32_t*)counter,
                               serial_key);
            launch_part_heads(a, s);
        } else {
            // more partitions than the counters' room in the workspace: group
            // with the partition sort instead
            BulkArgs b = a;
            b.part_early = 0;
            launch_part_sort(b, s);
            hipLaunchKernelGGL(k_pgroup_keys, dim3(nb), dim3(GTX_BLOCK), 0, s, a, serial_key);
        }
        pm.mark(PH_PARTSORT, s);
        launch_part_gather(a, s);
        pm.mark(PH_PARTGATHER, s);
        launch_part_kernels(a, s);
    } else {
        pm.mark(PH_PARTSORT, s);
        pm.mark(PH_PARTGATHER, s);
    }
    pm.mark(PH_PART, s);
    // lock words in the op-record region (unused without the op sort)
    int64_t n_locks = 4;
    while (n_locks * 2 <= a.mcap * (int64_t)(sizeof(OpInfo) / sizeof(uint64_t)) && n_locks < ((int64_t)1 << 22))
        n_locks *= 2;
    uint64_t* locks = reinterpret_cast<uint64_t*>(a.ws.op_info);
    hipLaunchKernelGGL(k_lock_clear, dim3(nb), dim3(GTX_BLOCK), 0, s, a, locks, n_locks);
    hipLaunchKernelGGL(k_tpl_relaxed, dim3(a.grid_blocks), dim3(GTX_BLOCK), 0, s, a, locks, (uint32_t)(n_locks - 1),
                       serial_key);
    pm.mark(PH_TPL, s);
    pm.mark(PH_KSET, s);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, s, a);
    pm.mark(PH_FINAL, s);
}

void launch_exec(const BulkArgs& a, hipStream_t s, const PhaseMarks& pm) {
    hipLaunchKernelGGL(k_exec_gate, dim3(1), dim3(64), 0, s, a);
    // PART: group transactions by partition (stable, so timestamp order is
    // kept inside each partition); only when PART was chosen
    const bool part = a.strategy == GPUTX_AUTO || a.strategy == GPUTX_PART;
    if (part && !a.part_early) launch_part_sort(a, s);
    pm.mark(PH_PARTSORT, s);
    if (part) {
        if (!a.part_early) launch_part_gather(a, s);
        pm.mark(PH_PARTGATHER, s);
        launch_part_kernels(a, s);
    } else {
        pm.mark(PH_PARTGATHER, s);
    }
    pm.mark(PH_PART, s);
    launch_rank_full(a, s);  // wait targets, groups, successors: TPL or K-SET chosen
    if (a.strategy == GPUTX_AUTO || a.strategy == GPUTX_TPL || a.strategy == GPUTX_PART)
        hipLaunchKernelGGL(k_tpl, dim3(a.grid_blocks), dim3(GTX_BLOCK), 0, s, a);
    pm.mark(PH_TPL, s);
    // Algorithm 1 picks K-SET only when the 0-set holds at least w0_bar
    // transactions, which a bulk of fewer cannot reach
    if (a.strategy == GPUTX_KSET || (a.strategy == GPUTX_AUTO && a.n >= a.w0_bar)) {
        hipLaunchKernelGGL(k_kset, dim3(a.grid_blocks), dim3(GTX_BLOCK), 0, s, a);
    }
    pm.mark(PH_KSET, s);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, s, a);
    pm.mark(PH_FINAL, s);
}

}  // namespace gtx
