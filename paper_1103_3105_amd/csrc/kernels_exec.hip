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
//   k_part     PART (Section 5.2): one lane per partition; binary search of
//              the partition's range in the partition-sorted transactions,
//              then its transactions run one after another.
//   k_finalize batched update (Section 3.2): advance append-table row counts;
//              publish statistics.
#include "engine.h"

namespace gtx {

__device__ __forceinline__ bool failed(const GtxState* st) { return ld_relaxed(&st->error) != 0; }
__device__ __forceinline__ void fail(GtxState* st, int code) { atomicCAS(&st->error, 0, code); }

__device__ __forceinline__ int64_t in_index(const BulkArgs& a, int64_t p) {
    return a.ws.st->unsorted ? (int64_t)a.ws.tsv[0][p] : p;
}

// Run the transaction at serial position p (type t >= 0); returns its status.
__device__ int32_t run_at(const BulkArgs& a, int64_t p, int32_t t) {
    const DevType& T = a.types[t];
    const int64_t i = in_index(a, p);
    int64_t prm[GTX_MAX_PARAMS];
    load_params(a.params, a.n, min(a.n_params, T.n_params), i, prm);
    int64_t app0 = 0, app1 = 0;
    if (T.app_idx[0] >= 0)
        app0 = a.rowcount[T.app_idx[0]] + a.ws.cnt[(int64_t)(1 + T.app_idx[0]) * a.n + p];
    if (T.app_idx[1] >= 0)
        app1 = a.rowcount[T.app_idx[1]] + a.ws.cnt[(int64_t)(1 + T.app_idx[1]) * a.n + p];
    int64_t res[GTX_MAX_RESULTS];
    const int32_t s = txn_exec(T, prm, a.ts[i], app0, app1, res);
    a.status[i] = s;
    int64_t* out = a.results + i * a.width;
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

__device__ __forceinline__ void kset_push(const BulkArgs& a, int next, const int* reg_off, int32_t q) {
    GtxState* st = a.ws.st;
    const int32_t t = a.ws.tty[q];
    const int slot = atomicAdd(&st->kset_fill[next % 3][t], 1);
    a.ws.front[next & 1][reg_off[t] + slot] = q;
}

__global__ __launch_bounds__(GTX_BLOCK) void k_kset(BulkArgs a) {
    GtxState* st = a.ws.st;
    if (failed(st) || st->chosen != GPUTX_KSET) return;
    __shared__ int reg_off[GPUTX_MAX_TYPES];
    __shared__ int wcnt[GPUTX_MAX_TYPES];
    __shared__ int cpre[GPUTX_MAX_TYPES + 1];
    if (threadIdx.x == 0) {
        int o = 0;
        for (int t = 0; t < GPUTX_MAX_TYPES; ++t) {
            reg_off[t] = o;
            o += st->type_count[t];
        }
    }
    __syncthreads();
    // wave 0: every valid transaction without predecessors
    for (int64_t p = (int64_t)blockIdx.x * GTX_BLOCK + threadIdx.x; p < a.n;
         p += (int64_t)gridDim.x * GTX_BLOCK) {
        if (a.ws.tty[p] >= 0 && a.ws.indeg[p] == 0) kset_push(a, 0, reg_off, (int32_t)p);
    }
    const int gwaves = gridDim.x * GTX_WAVES;
    const int gw = blockIdx.x * GTX_WAVES + wave_id();
    int64_t k = 0;
    while (grid_barrier(st, a.spin_ticks)) {
        const int cur = (int)(k % 3);
        if (threadIdx.x < GPUTX_MAX_TYPES) {
            wcnt[threadIdx.x] = ld_relaxed(&st->kset_fill[cur][threadIdx.x]);
            if (blockIdx.x == 0) st_relaxed(&st->kset_fill[(k + 2) % 3][threadIdx.x], 0);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int c = 0;
            for (int t = 0; t < GPUTX_MAX_TYPES; ++t) {
                cpre[t] = c;
                c += (wcnt[t] + 63) / 64;
            }
            cpre[GPUTX_MAX_TYPES] = c;
        }
        __syncthreads();
        const int nchunks = cpre[GPUTX_MAX_TYPES];
        if (nchunks == 0) break;  // every transaction has run
        const int32_t* F = a.ws.front[k & 1];
        for (int c = gw; c < nchunks; c += gwaves) {
            int t = 0;
            while (cpre[t + 1] <= c) ++t;  // wave-uniform: this chunk's type
            const int idx = (c - cpre[t]) * 64 + lane_id();
            const bool live = idx < wcnt[t];
            int32_t s = 0;
            int32_t q = 0;
            if (live) {
                q = F[reg_off[t] + idx];
                s = run_at(a, q, t);
            }
            count_status(st, live, s);
            if (live) {
                const int64_t o1 = op_end(a, q);
                for (int64_t o = op_begin(a, q); o < o1; ++o) {
                    const int32_t hi = a.ws.op_shi[o];
                    for (int32_t j = a.ws.op_slo[o]; j < hi; ++j) {
                        const int32_t q2 = a.ws.srt_txn[j];
                        if (atomicSub(&a.ws.indeg[q2], 1) == 1) kset_push(a, (int)(k + 1), reg_off, q2);
                    }
                }
            }
        }
        ++k;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) st->waves = k;
}

// ---------------------------------------------------------------------------
// TPL with counter-based locks

__global__ __launch_bounds__(GTX_BLOCK) void k_tpl(BulkArgs a) {
    GtxState* st = a.ws.st;
    if (failed(st) || st->chosen != GPUTX_TPL) return;
    __shared__ int win_s;
    __shared__ int32_t slot_pos[GTX_BLOCK];
    __shared__ int tcnt[GTX_WAVES][GPUTX_MAX_TYPES + 1];
    __shared__ int toff[GTX_WAVES][GPUTX_MAX_TYPES + 1];
    const int lane = lane_id();
    const int w = wave_id();
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
        bool done = t < 0;
        int64_t o0 = 0, o1 = 0;
        if (!done) {
            o0 = op_begin(a, p);
            o1 = op_end(a, p);
        }
        uint64_t t0 = 0;
        int32_t s = 0;
        bool ran = false;
        while (__any(!done)) {
            bool ready = false;
            if (!done) {
                ready = true;
                for (int64_t o = o0; o < o1; ++o)
                    ready = ready && ld_relaxed(&a.ws.grp_cnt[a.ws.op_grp[o]]) >= a.ws.op_tgt[o];
            }
            if (__any(ready)) {
                fence_acquire();  // see every write released by the predecessors
                if (ready) {
                    s = run_at(a, p, t);
                    ran = true;
                }
                fence_release();  // publish this transaction's writes
                if (ready) {
                    for (int64_t o = o0; o < o1; ++o) atomicAdd(&a.ws.grp_cnt[a.ws.op_grp[o]], 1);
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
                __builtin_amdgcn_s_sleep(1);
            }
        }
        count_status(st, ran, s);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// PART

__global__ __launch_bounds__(GTX_BLOCK) void k_part(BulkArgs a, int lane_stride) {
    GtxState* st = a.ws.st;
    if (failed(st) || st->chosen != GPUTX_PART) return;
    const int64_t g = (int64_t)blockIdx.x * GTX_BLOCK + threadIdx.x;
    const bool mine = (g % lane_stride) == 0;
    const int64_t q = g / lane_stride;
    const int src = a.part_passes & 1;
    const uint32_t* key = a.ws.qk[src];
    const uint32_t* pos = a.ws.qv[src];
    int32_t s = 0;
    int64_t committed = 0, aborted = 0;
    if (mine && q < a.n_parts) {
        // the partition's range in the partition-sorted bulk, by binary search
        int64_t lo = 0, hi = a.n;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (key[mid] < (uint32_t)q) lo = mid + 1;
            else hi = mid;
        }
        int64_t end = lo, hi2 = a.n;
        while (end < hi2) {
            int64_t mid = (end + hi2) >> 1;
            if (key[mid] <= (uint32_t)q) end = mid + 1;
            else hi2 = mid;
        }
        for (int64_t i = lo; i < end; ++i) {
            const int32_t p = (int32_t)pos[i];
            s = run_at(a, p, a.ws.tty[p]);
            committed += s == GPUTX_COMMIT;
            aborted += s == GPUTX_ABORT;
        }
    }
    long long c = wave_sum64(committed), ab = wave_sum64(aborted);
    if (lane_id() == 0) {
        if (c) atomicAdd((unsigned long long*)&st->committed, (unsigned long long)c);
        if (ab) atomicAdd((unsigned long long*)&st->aborted, (unsigned long long)ab);
    }
}

// ---------------------------------------------------------------------------

__global__ void k_finalize(BulkArgs a) {
    GtxState* st = a.ws.st;
    if (threadIdx.x != 0) return;
    gputx_bulk_stats* o = a.stats;
    const int err = st->error;
    if (!err) {
        for (int k = 0; k < a.n_app; ++k) a.rowcount[k] += st->app_total[k];
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
    for (int k = 0; k < 7; ++k) o->reserved[k] = 0;
}

// ---------------------------------------------------------------------------

__global__ void k_reset_state(GtxState* st) {
    int* w = reinterpret_cast<int*>(st);
    for (int i = threadIdx.x; i < (int)(sizeof(GtxState) / 4); i += blockDim.x) w[i] = 0;
}

void launch_empty(const BulkArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_state, dim3(1), dim3(64), 0, s, a.ws.st);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, s, a);
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

void launch_exec(const BulkArgs& a, hipStream_t s) {
    // PART: group transactions by partition (stable, so timestamp order is
    // kept inside each partition); only when PART was chosen
    if (a.strategy == GPUTX_AUTO || a.strategy == GPUTX_PART) {
        SortPlan sp{};
        sp.key_bytes = 4;
        sp.keys[0] = a.ws.qk[0]; sp.keys[1] = a.ws.qk[1];
        sp.vals[0] = a.ws.qv[0]; sp.vals[1] = a.ws.qv[1];
        sp.hist = a.ws.sort_hist; sp.status = a.ws.sort_status; sp.ctrl = a.ws.sort_ctrl;
        sp.cap = a.n; sp.count_dev = nullptr; sp.npass = a.part_passes;
        sp.gate = &a.ws.st->run_part; sp.st = a.ws.st; sp.spin_ticks = a.spin_ticks;
        sort_pairs(sp, s);
        const int stride = a.n_parts <= 4096 ? 64 : 1;
        const int64_t threads = a.n_parts * stride;
        const unsigned blocks = (unsigned)std::max<int64_t>(1, (threads + GTX_BLOCK - 1) / GTX_BLOCK);
        hipLaunchKernelGGL(k_part, dim3(blocks), dim3(GTX_BLOCK), 0, s, a, stride);
    }
    if (a.strategy == GPUTX_AUTO || a.strategy == GPUTX_TPL || a.strategy == GPUTX_PART)
        hipLaunchKernelGGL(k_tpl, dim3(a.grid_blocks), dim3(GTX_BLOCK), 0, s, a);
    if (a.strategy == GPUTX_AUTO || a.strategy == GPUTX_KSET)
        hipLaunchKernelGGL(k_kset, dim3(a.grid_blocks), dim3(GTX_BLOCK), 0, s, a);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, s, a);
}

}  // namespace gtx
