// Served form: continuous batching (Sections 3.2, 6.3).
//
// Section 3.2's pipeline: transactions enter a transaction pool, a bulk is
// formed from the pool at every interval t and runs on the GPU, and the
// results land in a result pool.  A server (gputx_serve_open) owns both pools
// in host memory and two native threads, one that cuts and issues bulks and
// one that retires them:
//   * gputx_serve_submit copies signatures into the transaction pool and
//     hands out tickets (consecutive sequence numbers);
//   * every interval the issuing thread cuts everything submitted so far (up
//     to the largest bulk) and issues it on a free slot;
//   * the retiring thread copies a finished bulk's statuses and results into
//     the result pool, where gputx_serve_poll picks them up in ticket order;
//   * gputx_serve_close waits for everything submitted, then frees the slots.
// gputx_serve replays an arrival trace through the same server: a driver
// loop submits each transaction once its arrival time has passed and polls
// the results.
//
// MI355X mapping:
//  * K slots, each with its own device bulk arrays, workspace and outputs, and
//    pre-instantiated HIP graphs (bulk generation and execution separately)
//    for a ladder of bulk sizes (four per octave, multiples of 256); a bulk is
//    padded to its size class with invalid transactions (no effect, outputs
//    ignored), at most a fifth more work.
//  * A bulk's upload and its results' return are copy kernels between device
//    memory and mapped pinned host buffers, on the bulk's own streams.
//  * Bulk generation of a bulk runs on its slot's stream and overlaps the
//    execution of earlier bulks; executions are ordered on one stream, so the
//    database sees the bulks in ticket order.
//  * Admission: the number of slots is capped by an HBM byte budget; a cut
//    waits for a free slot, and everything submitted meanwhile joins it.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "runtime.h"

using namespace gtx;
using Clock = std::chrono::steady_clock;

namespace {

constexpr int64_t kMinBucket = 256;

struct Slot {
    char* dev = nullptr;             // device buffer (bulk arrays, workspace, outputs, stats)
    char* stage = nullptr;           // pinned host staging of the bulk arrays
    char* out_h = nullptr;           // pinned host copy of statuses, results and stats
    char* stage_d = nullptr;         // the same two host buffers as the device addresses them
    char* out_d = nullptr;
    hipStream_t fs = nullptr;
    hipEvent_t ready = nullptr, done = nullptr;
    hipEvent_t t_up = nullptr, t_exec = nullptr;  // upload start, execution start (timed, with ready and done)
    std::vector<hipGraphExec_t> front, exec;
    std::vector<hipGraph_t> graphs;
    int64_t first = 0, count = 0, cut_ns = 0, issued_ns = 0, pad = 0;
};

struct BucketLayout {
    int64_t n;
    size_t off_type, off_params, off_ts, bytes;  // packed bulk arrays of this size
};

inline size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

// Byte copy between device memory and mapped pinned host memory, as a kernel
// on the bulk's own stream: a bulk's upload and its results' return then
// take exactly the transfer time, where an asynchronous DMA copy of the same
// buffers now and then held the server thread and the stream for several
// milliseconds.  Sizes and offsets are multiples of 4 bytes; 16-byte moves
// where both sides allow.
__global__ __launch_bounds__(256) void k_serve_copy(char* __restrict__ dst, const char* __restrict__ src,
                                                    int64_t bytes) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x, nt = (int64_t)gridDim.x * 256;
    if ((((uintptr_t)dst | (uintptr_t)src) & 15) == 0) {
        const int64_t n16 = bytes / 16;
        for (int64_t i = t; i < n16; i += nt)
            reinterpret_cast<uint4*>(dst)[i] = reinterpret_cast<const uint4*>(src)[i];
        for (int64_t i = n16 * 4 + t; i < bytes / 4; i += nt)
            reinterpret_cast<uint32_t*>(dst)[i] = reinterpret_cast<const uint32_t*>(src)[i];
    } else {
        for (int64_t i = t; i < bytes / 4; i += nt)
            reinterpret_cast<uint32_t*>(dst)[i] = reinterpret_cast<const uint32_t*>(src)[i];
    }
}

inline hipError_t serve_copy(char* dst, const char* src, int64_t bytes, hipStream_t s) {
    if (bytes <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<int64_t>(512, (bytes / 16 + 255) / 256 + 1);
    hipLaunchKernelGGL(k_serve_copy, dim3(blocks), dim3(256), 0, s, dst, src, bytes);
    return hipGetLastError();
}

BucketLayout layout_for(int64_t n, int np) {
    BucketLayout L;
    L.n = n;
    L.off_type = 0;
    L.off_params = up256((size_t)n * 4);
    L.off_ts = L.off_params + up256((size_t)n * 8 * np);
    L.bytes = L.off_ts + up256((size_t)n * 8);
    return L;
}

// Size classes: four per octave from 256 up, rounded up to multiples of 256,
// the last one covering `maxb`.
std::vector<int64_t> size_ladder(int64_t maxb) {
    std::vector<int64_t> v;
    for (int64_t oct = kMinBucket; v.empty() || v.back() < maxb; oct <<= 1)
        for (int q = 0; q < 4 && (v.empty() || v.back() < maxb); ++q) {
            int64_t s = (oct * (4 + q) / 4 + 255) / 256 * 256;
            if (v.empty() || s > v.back()) v.push_back(std::min(s, std::max(maxb, kMinBucket)));
        }
    return v;
}

inline int64_t since(Clock::time_point t0) {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - t0).count();
}

}  // namespace

struct gputx_server_t {
    gputx_handle h = nullptr;
    gputx_serve_opts o{};
    int np = 0, W = 0;
    int64_t cap = 0;  // pool capacity in transactions (both pools)
    // transaction pool and result pool: rings indexed by ticket % cap
    std::vector<int32_t> p_type;
    std::vector<int64_t> p_params;  // [np][cap]
    std::vector<int64_t> p_ts, p_arrival;
    std::vector<int32_t> r_status;
    std::vector<int64_t> r_results;  // [cap][W]
    std::vector<int64_t> r_done;
    std::atomic<int64_t> submitted{0};  // tickets handed out
    std::atomic<int64_t> answered{0};   // tickets whose results are in the result pool
    std::atomic<int64_t> polled{0};     // tickets handed back by poll (ring entries free)
    int64_t last_ts = INT64_MIN;        // submit side: ids must ascend
    bool any_ts = false;
    // device side (server thread only once running)
    std::vector<Slot> slots;
    hipStream_t es = nullptr;
    std::vector<int64_t> sizes;
    int64_t maxb = 0;
    size_t off_ws = 0, off_status = 0, off_results = 0, off_stats = 0, slot_bytes = 0, ws_bytes = 0;
    Clock::time_point t0;
    std::thread worker;   // cuts and issues bulks
    std::thread retirer;  // waits for bulks in issue order and fills the result pool
    // slots in flight: busy flags, and a ring of slot ids in issue order
    // (written by the issuing thread, consumed by the retiring one)
    std::unique_ptr<std::atomic<int>[]> busy;
    std::vector<int> ring;
    std::atomic<int64_t> pushed{0}, popped{0};
    std::atomic<bool> issue_done{false};
    std::atomic<bool> stop{false};
    std::atomic<int> err{0};
    std::mutex err_mu;
    std::string err_msg;
    std::mutex log_mu;
    std::vector<gputx_serve_bulk> log;
    gputx_serve_report rep{};
    int64_t last_done = 0;

    void set_error(int code, const std::string& msg) {
        std::lock_guard<std::mutex> lk(err_mu);
        if (!err.load()) {
            err_msg = msg;
            err.store(code);
        }
    }
    void release() {
        for (auto& s : slots) {
            for (auto g : s.front) (void)hipGraphExecDestroy(g);
            for (auto g : s.exec) (void)hipGraphExecDestroy(g);
            for (auto g : s.graphs) (void)hipGraphDestroy(g);
            if (s.ready) (void)hipEventDestroy(s.ready);
            if (s.done) (void)hipEventDestroy(s.done);
            if (s.t_up) (void)hipEventDestroy(s.t_up);
            if (s.t_exec) (void)hipEventDestroy(s.t_exec);
            if (s.fs) (void)hipStreamDestroy(s.fs);
            if (s.dev) (void)hipFree(s.dev);
            if (s.stage) (void)hipHostFree(s.stage);
            if (s.out_h) (void)hipHostFree(s.out_h);
        }
        slots.clear();
        if (es) (void)hipStreamDestroy(es);
        es = nullptr;
    }
    void run();
    void retire_loop();
    int retire_one(int si);
    bool issue(int si, int64_t first, int64_t cnt, int64_t now);
};

// Copy finished bulk si into the result pool (ticket order) and log it.
// Returns 1 when retired, 0 while it is still running, -1 on an error.
int gputx_server_t::retire_one(int si) {
    Slot& s = slots[si];
    // polled rather than waited on: a blocking wait inside the runtime held
    // up the issuing thread's launches meanwhile
    const hipError_t q = hipEventQuery(s.done);
    if (q == hipErrorNotReady) return 0;
    if (q != hipSuccess) {
        set_error(GPUTX_E_HIP, std::string("bulk completion: ") + hipGetErrorString(q));
        return -1;
    }
    const int64_t t = since(t0);
    last_done = t;
    const int32_t* st = reinterpret_cast<const int32_t*>(s.out_h);
    const int64_t* rs = reinterpret_cast<const int64_t*>(s.out_h + up256((size_t)maxb * 4));
    const gputx_bulk_stats* bs =
        reinterpret_cast<const gputx_bulk_stats*>(s.out_h + up256((size_t)maxb * 4) + up256((size_t)maxb * 8 * W));
    // the ring may wrap inside the bulk: copy in at most two pieces
    auto put = [&](int64_t k, int64_t j, int64_t m) {
        if (bs->error) std::fill(&r_status[k], &r_status[k] + m, (int32_t)GPUTX_INVALID);
        else std::memcpy(&r_status[k], st + j, sizeof(int32_t) * m);
        std::memcpy(&r_results[(size_t)k * W], rs + (size_t)j * W, sizeof(int64_t) * W * m);
        std::fill(&r_done[k], &r_done[k] + m, t);
    };
    const int64_t k0 = s.first % cap, c0 = std::min(s.count, cap - k0);
    put(k0, 0, c0);
    if (s.count > c0) put(0, c0, s.count - c0);
    {
        std::lock_guard<std::mutex> lk(log_mu);
        gputx_serve_bulk r{};
        r.first = s.first;
        r.count = s.count;
        r.cut_ns = s.cut_ns;
        r.issued_ns = s.issued_ns;
        r.done_ns = t;
        float f_ms = 0.f, x_ms = 0.f;
        if (hipEventElapsedTime(&f_ms, s.t_up, s.ready) != hipSuccess) f_ms = -1.f;
        if (hipEventElapsedTime(&x_ms, s.t_exec, s.done) != hipSuccess) x_ms = -1.f;
        r.front_us = (int32_t)(f_ms * 1000.f);
        r.exec_us = (int32_t)(x_ms * 1000.f);
        r.error = bs->error;
        r.slot = si;
        log.push_back(r);
        rep.committed += bs->committed;
        rep.aborted += bs->aborted;
        rep.invalid += bs->invalid - s.pad;  // padding is not part of the pool
    }
    if (bs->error)
        set_error(bs->error, "bulk at ticket " + std::to_string(s.first) + " failed on the device");
    answered.store(s.first + s.count, std::memory_order_release);
    busy[si].store(0, std::memory_order_release);
    return 1;
}

// The retiring thread: bulks complete in issue order (their executions share
// one stream), so it waits for the oldest in flight, copies its results out
// and frees its slot -- off the issuing thread, whose cuts it would
// otherwise hold up by the copy of a large bulk's results.
void gputx_server_t::retire_loop() {
    (void)hipSetDevice(h->device);
    while (true) {
        const int64_t p = popped.load(std::memory_order_relaxed);
        if (p < pushed.load(std::memory_order_acquire)) {
            const int r = retire_one(ring[p % ring.size()]);
            if (r < 0) break;
            if (r > 0) popped.store(p + 1, std::memory_order_release);
            else std::this_thread::yield();
        } else if (issue_done.load(std::memory_order_acquire)) {
            if (popped.load() == pushed.load()) break;
        } else {
            std::this_thread::yield();
        }
    }
}

// Pack tickets [first, first + cnt) from the pool into slot si and launch it.
bool gputx_server_t::issue(int si, int64_t first, int64_t cnt, int64_t now) {
    Slot& s = slots[si];
    int bi = 0;
    while (sizes[bi] < cnt) ++bi;
    const BucketLayout L = layout_for(sizes[bi], np);
    int32_t* st = reinterpret_cast<int32_t*>(s.stage + L.off_type);
    int64_t* sp = reinterpret_cast<int64_t*>(s.stage + L.off_params);
    int64_t* sts = reinterpret_cast<int64_t*>(s.stage + L.off_ts);
    // the ring may wrap inside the bulk: copy in at most two pieces
    const int64_t k0 = first % cap;
    const int64_t c0 = std::min(cnt, cap - k0), c1 = cnt - c0;
    std::memcpy(st, &p_type[k0], c0 * 4);
    if (c1) std::memcpy(st + c0, &p_type[0], c1 * 4);
    std::fill(st + cnt, st + L.n, -1);  // padding: invalid transactions
    for (int k = 0; k < np; ++k) {
        int64_t* dst = sp + (int64_t)k * L.n;
        const int64_t* src = &p_params[(size_t)k * cap];
        std::memcpy(dst, src + k0, c0 * 8);
        if (c1) std::memcpy(dst + c0, src, c1 * 8);
        std::fill(dst + cnt, dst + L.n, 0);
    }
    std::memcpy(sts, &p_ts[k0], c0 * 8);
    if (c1) std::memcpy(sts + c0, &p_ts[0], c1 * 8);
    const int64_t tlast = sts[cnt - 1];
    for (int64_t j = cnt; j < L.n; ++j) sts[j] = tlast + 1 + (j - cnt);
    s.first = first;
    s.count = cnt;
    s.pad = L.n - cnt;
    s.cut_ns = now;
    const size_t o_res = up256((size_t)maxb * 4), o_stats = o_res + up256((size_t)maxb * 8 * W);
    hipError_t e = hipEventRecord(s.t_up, s.fs);
    if (e == hipSuccess) e = serve_copy(s.dev, s.stage_d, (int64_t)L.bytes, s.fs);
    if (e == hipSuccess) e = hipGraphLaunch(s.front[bi], s.fs);
    if (e == hipSuccess) e = hipEventRecord(s.ready, s.fs);
    if (e == hipSuccess) e = hipStreamWaitEvent(es, s.ready, 0);
    if (e == hipSuccess) e = hipEventRecord(s.t_exec, es);
    if (e == hipSuccess) e = hipGraphLaunch(s.exec[bi], es);
    if (e == hipSuccess) e = serve_copy(s.out_d, s.dev + off_status, cnt * 4, es);
    if (e == hipSuccess) e = serve_copy(s.out_d + o_res, s.dev + off_results, cnt * 8 * W, es);
    if (e == hipSuccess) e = serve_copy(s.out_d + o_stats, s.dev + off_stats, (int64_t)sizeof(gputx_bulk_stats), es);
    if (e == hipSuccess) e = hipEventRecord(s.done, es);
    if (e != hipSuccess) {
        set_error(GPUTX_E_HIP, std::string("issuing a bulk failed: ") + hipGetErrorString(e));
        return false;
    }
    s.issued_ns = since(t0);
    return true;
}

// The issuing thread: every interval, cut what the pool holds into a bulk.
void gputx_server_t::run() {
    (void)hipSetDevice(h->device);
    const int64_t D = o.deadline_ns;
    int64_t issued = 0, deadline = D;
    int next_slot = 0;
    const int nslots = (int)slots.size();
    while (!err.load(std::memory_order_relaxed)) {
        const int64_t sub = submitted.load(std::memory_order_acquire);
        const bool stopping = stop.load(std::memory_order_acquire);
        if (stopping && issued == sub) break;
        const int64_t now = since(t0);
        if (issued < sub && (now >= deadline || stopping)) {
            if (busy[next_slot].load(std::memory_order_acquire)) {  // admission: wait for a slot
                std::this_thread::yield();
                continue;
            }
            const int64_t cnt = std::min(sub - issued, maxb);
            busy[next_slot].store(1, std::memory_order_relaxed);
            if (!issue(next_slot, issued, cnt, now)) {
                busy[next_slot].store(0, std::memory_order_relaxed);
                break;
            }
            ring[pushed.load(std::memory_order_relaxed) % nslots] = next_slot;
            pushed.fetch_add(1, std::memory_order_release);
            next_slot = (next_slot + 1) % nslots;
            issued += cnt;
            if (issued == sub) deadline = (now / D) * D + D;
        } else {
            if (now >= deadline) deadline = (now / D) * D + D;
            std::this_thread::yield();
        }
    }
    issue_done.store(true, std::memory_order_release);
}

extern "C" int gputx_serve_open(gputx_handle h, const gputx_serve_opts* o, int32_t n_params,
                                int64_t pool_capacity, gputx_server* out) {
    if (!h || !o || !out) return gtx_set_err(h, GPUTX_E_ARG, "null argument");
    *out = nullptr;
    if (o->deadline_ns <= 0 || o->slots < 1 || o->max_bulk < 1 || o->width < 1 || n_params < 1 ||
        n_params > GTX_MAX_PARAMS || o->strategy < GPUTX_AUTO || o->strategy > GPUTX_KSET || o->max_ops < 0 ||
        pool_capacity < 1 || pool_capacity > ((int64_t)1 << 32))
        return gtx_set_err(h, GPUTX_E_ARG, "bad serving options");
    HIP_OK(h, hipSetDevice(h->device));
    gputx_server_t* S = new gputx_server_t();
    S->h = h;
    S->o = *o;
    S->np = n_params;
    S->W = o->width;
    S->cap = pool_capacity;
    S->maxb = std::max<int64_t>(kMinBucket, (o->max_bulk + 255) / 256 * 256);
    S->sizes = size_ladder(S->maxb);
    S->maxb = S->sizes.back();
    const int np = n_params, W = o->width;
    const BucketLayout big = layout_for(S->maxb, np);
    S->ws_bytes = gputx_workspace_size_ops(h, S->maxb, o->max_ops);
    S->off_ws = up256(big.bytes);
    S->off_status = S->off_ws + up256(S->ws_bytes);
    S->off_results = S->off_status + up256((size_t)S->maxb * 4);
    S->off_stats = S->off_results + up256((size_t)S->maxb * 8 * W);
    S->slot_bytes = S->off_stats + up256(sizeof(gputx_bulk_stats));
    int nslots = o->slots;
    if (o->hbm_budget > 0) nslots = (int)std::min<int64_t>(nslots, o->hbm_budget / (int64_t)S->slot_bytes);
    if (nslots < 1) {
        const size_t sb = S->slot_bytes;
        delete S;
        return gtx_set_err(h, GPUTX_E_CAPACITY, "HBM budget below one slot (%zu bytes)", sb);
    }
    try {
        S->p_type.assign((size_t)S->cap, -1);
        S->p_params.assign((size_t)S->cap * np, 0);
        S->p_ts.assign((size_t)S->cap, 0);
        S->p_arrival.assign((size_t)S->cap, 0);
        S->r_status.assign((size_t)S->cap, 0);
        S->r_results.assign((size_t)S->cap * W, 0);
        S->r_done.assign((size_t)S->cap, 0);
    } catch (...) {
        delete S;
        return gtx_set_err(h, GPUTX_E_CAPACITY, "pool of %lld transactions does not fit in host memory",
                           (long long)pool_capacity);
    }
    S->slots.resize(nslots);
    S->busy.reset(new std::atomic<int>[nslots]);
    for (int i = 0; i < nslots; ++i) S->busy[i].store(0);
    S->ring.assign(nslots, 0);
#define OPEN_OK(call)                                                                             \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess) {                                                                   \
            const int rc_ = gtx_set_err(h, GPUTX_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
            S->release();                                                                         \
            delete S;                                                                             \
            return rc_;                                                                           \
        }                                                                                         \
    } while (0)
    OPEN_OK(hipStreamCreateWithFlags(&S->es, hipStreamNonBlocking));
    const int grid = gtx_grid_for(h, 1);
    const size_t out_bytes = up256((size_t)S->maxb * 4) + up256((size_t)S->maxb * 8 * W) +
                             up256(sizeof(gputx_bulk_stats));
    for (auto& s : S->slots) {
        OPEN_OK(hipMalloc(&s.dev, S->slot_bytes));
        OPEN_OK(hipHostMalloc(&s.stage, big.bytes, hipHostMallocMapped));
        OPEN_OK(hipHostMalloc(&s.out_h, out_bytes, hipHostMallocMapped));
        OPEN_OK(hipHostGetDevicePointer(reinterpret_cast<void**>(&s.stage_d), s.stage, 0));
        OPEN_OK(hipHostGetDevicePointer(reinterpret_cast<void**>(&s.out_d), s.out_h, 0));
        OPEN_OK(hipStreamCreateWithFlags(&s.fs, hipStreamNonBlocking));
        OPEN_OK(hipEventCreate(&s.ready));
        OPEN_OK(hipEventCreate(&s.done));
        OPEN_OK(hipEventCreate(&s.t_up));
        OPEN_OK(hipEventCreate(&s.t_exec));
        for (int64_t n : S->sizes) {
            const BucketLayout L = layout_for(n, np);
            gputx_bulk b{};
            b.n = n;
            b.type = reinterpret_cast<const int32_t*>(s.dev + L.off_type);
            b.params = reinterpret_cast<const int64_t*>(s.dev + L.off_params);
            b.n_params = np;
            b.ts = reinterpret_cast<const int64_t*>(s.dev + L.off_ts);
            b.ts_sorted = 1;
            b.max_ops = o->max_ops;
            BulkArgs a;
            int rc = gtx_make_args(h, &b, o->strategy, s.dev + S->off_ws, S->ws_bytes,
                                   reinterpret_cast<int32_t*>(s.dev + S->off_status),
                                   reinterpret_cast<int64_t*>(s.dev + S->off_results), W,
                                   reinterpret_cast<gputx_bulk_stats*>(s.dev + S->off_stats), grid, &a);
            if (rc) {
                S->release();
                delete S;
                return rc;
            }
            PhaseMarks none;
            hipGraph_t gf = nullptr, ge = nullptr;
            hipGraphExec_t xf = nullptr, xe = nullptr;
            OPEN_OK(hipStreamBeginCapture(s.fs, hipStreamCaptureModeThreadLocal));
            (void)launch_front(a, s.fs, none);
            OPEN_OK(hipStreamEndCapture(s.fs, &gf));
            s.graphs.push_back(gf);
            OPEN_OK(hipGraphInstantiate(&xf, gf, nullptr, nullptr, 0));
            s.front.push_back(xf);
            // upload now, so that the first bulk of this size class on this
            // slot does not pay for it while serving
            OPEN_OK(hipGraphUpload(xf, s.fs));
            OPEN_OK(hipStreamBeginCapture(S->es, hipStreamCaptureModeThreadLocal));
            launch_exec(a, S->es, none);
            OPEN_OK(hipStreamEndCapture(S->es, &ge));
            s.graphs.push_back(ge);
            OPEN_OK(hipGraphInstantiate(&xe, ge, nullptr, nullptr, 0));
            s.exec.push_back(xe);
            OPEN_OK(hipGraphUpload(xe, S->es));
        }
    }
    OPEN_OK(hipDeviceSynchronize());
#undef OPEN_OK
    S->t0 = Clock::now();
    try {
        S->retirer = std::thread([S] { S->retire_loop(); });
    } catch (...) {
        S->release();
        delete S;
        return gtx_set_err(h, GPUTX_E_STATE, "could not start the server threads");
    }
    try {
        S->worker = std::thread([S] { S->run(); });
    } catch (...) {
        S->issue_done.store(true);
        S->retirer.join();
        S->release();
        delete S;
        return gtx_set_err(h, GPUTX_E_STATE, "could not start the server threads");
    }
    *out = S;
    return GPUTX_OK;
}

extern "C" int gputx_serve_submit(gputx_server S, int64_t n, const int32_t* type, const int64_t* params,
                                  int64_t ld, const int64_t* ts, int64_t* first_ticket) {
    if (!S) return gtx_set_err(nullptr, GPUTX_E_ARG, "null server");
    if (n < 0 || (n > 0 && (!type || !params || !ts)) || ld < n)
        return gtx_set_err(S->h, GPUTX_E_ARG, "bad submission");
    if (S->stop.load()) return gtx_set_err(S->h, GPUTX_E_STATE, "server is closing");
    for (int64_t i = 0; i < n; ++i) {
        const int64_t prev = i ? ts[i - 1] : S->last_ts;
        if ((i || S->any_ts) && ts[i] <= prev)
            return gtx_set_err(S->h, GPUTX_E_ARG, "ids must ascend across submissions (at %lld)", (long long)i);
    }
    const int64_t sub = S->submitted.load(std::memory_order_relaxed);
    if (sub + n - S->polled.load(std::memory_order_acquire) > S->cap)
        return gtx_set_err(S->h, GPUTX_E_CAPACITY, "pool full: poll results first");
    const int64_t now = since(S->t0);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t k = (sub + i) % S->cap;
        S->p_type[k] = type[i];
        for (int q = 0; q < S->np; ++q) S->p_params[(size_t)q * S->cap + k] = params[(int64_t)q * ld + i];
        S->p_ts[k] = ts[i];
        S->p_arrival[k] = now;
    }
    if (n) {
        S->last_ts = ts[n - 1];
        S->any_ts = true;
    }
    if (first_ticket) *first_ticket = sub;
    S->submitted.store(sub + n, std::memory_order_release);
    return GPUTX_OK;
}

extern "C" int gputx_serve_poll(gputx_server S, int64_t max, int64_t* ticket, int32_t* status, int64_t* results,
                                int64_t* latency_ns, int64_t* n_out) {
    if (!S || !n_out || max < 0) return gtx_set_err(S ? S->h : nullptr, GPUTX_E_ARG, "bad poll");
    *n_out = 0;
    const int64_t done = S->answered.load(std::memory_order_acquire);
    const int64_t p0 = S->polled.load(std::memory_order_relaxed);
    const int64_t cnt = std::min(max, done - p0);
    for (int64_t j = 0; j < cnt; ++j) {
        const int64_t t = p0 + j, k = t % S->cap;
        if (ticket) ticket[j] = t;
        if (status) status[j] = S->r_status[k];
        if (results) std::memcpy(results + (size_t)j * S->W, &S->r_results[(size_t)k * S->W], sizeof(int64_t) * S->W);
        if (latency_ns) latency_ns[j] = S->r_done[k] - S->p_arrival[k];
    }
    S->polled.store(p0 + cnt, std::memory_order_release);
    *n_out = cnt;
    const int e = S->err.load();
    if (e) {
        std::lock_guard<std::mutex> lk(S->err_mu);
        return gtx_set_err(S->h, e, "%s", S->err_msg.c_str());
    }
    return GPUTX_OK;
}

// Server clock (ns since open) and the bulk log, for the trace driver.
static int64_t server_now(gputx_server S) { return since(S->t0); }

extern "C" int gputx_serve_close(gputx_server S, gputx_serve_report* report) {
    if (!S) return gtx_set_err(nullptr, GPUTX_E_ARG, "null server");
    S->stop.store(true, std::memory_order_release);
    if (S->worker.joinable()) S->worker.join();
    if (S->retirer.joinable()) S->retirer.join();
    // after an error bulks may still be in flight: drain before freeing
    (void)hipSetDevice(S->h->device);
    (void)hipStreamSynchronize(S->es);
    for (auto& sl : S->slots) (void)hipStreamSynchronize(sl.fs);
    {
        std::lock_guard<std::mutex> lk(S->log_mu);
        S->rep.n_bulks = (int64_t)S->log.size();
        S->rep.elapsed_ns = S->last_done;
        S->rep.slots_used = (int32_t)S->slots.size();
        S->rep.slot_bytes = (int64_t)S->slot_bytes;
    }
    int rc = GPUTX_OK;
    const int e = S->err.load();
    if (e) rc = gtx_set_err(S->h, e, "%s", S->err_msg.c_str());
    if (report) *report = S->rep;
    S->release();
    delete S;
    return rc;
}

extern "C" int gputx_serve(gputx_handle h, const gputx_trace* tr, const gputx_serve_opts* o,
                           int32_t* status_out, int64_t* results_out, gputx_serve_bulk* bulks,
                           int64_t bulk_capacity, gputx_serve_report* rep) {
    if (!h || !tr || !o || !rep || (tr->n > 0 && (!tr->arrival_ns || !tr->type || !tr->params ||
                                                   !tr->ts || !status_out || !results_out)))
        return gtx_set_err(h, GPUTX_E_ARG, "null argument");
    for (int64_t i = 1; i < tr->n; ++i)
        if (tr->arrival_ns[i] < tr->arrival_ns[i - 1] || tr->ts[i] <= tr->ts[i - 1])
            return gtx_set_err(h, GPUTX_E_ARG, "trace must be in arrival order with ascending ids");
    std::memset(rep, 0, sizeof *rep);
    const int64_t n = tr->n;
    gputx_server S = nullptr;
    int rc = gputx_serve_open(h, o, tr->n_params, std::max<int64_t>(n, 1), &S);
    if (rc) return rc;
    const int W = o->width;
    int64_t next = 0, got = 0;
    std::vector<int64_t> tk(4096);
    while (got < n) {
        const int64_t now = server_now(S);
        // release every transaction whose arrival time has passed
        const int64_t last = std::upper_bound(tr->arrival_ns + next, tr->arrival_ns + n, now) - tr->arrival_ns;
        if (last > next) {
            rc = gputx_serve_submit(S, last - next, tr->type + next, tr->params + next, n, tr->ts + next, nullptr);
            if (rc) break;
            next = last;
        }
        int64_t k = 0;
        rc = gputx_serve_poll(S, (int64_t)tk.size(), tk.data(), status_out + got, results_out + got * W, nullptr, &k);
        got += k;
        if (rc) break;
        if (!k && last == next) std::this_thread::yield();
    }
    {
        std::lock_guard<std::mutex> lk(S->log_mu);
        for (size_t b = 0; b < S->log.size() && (int64_t)b < bulk_capacity; ++b)
            if (bulks) bulks[b] = S->log[b];
    }
    const int rc2 = gputx_serve_close(S, rep);
    return rc ? rc : rc2;
}
