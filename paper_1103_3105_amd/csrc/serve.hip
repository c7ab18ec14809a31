// Served form: continuous batching over an arrival trace (Sections 3.2, 6.3).
//
// Transactions arrive into the transaction pool at their trace times; every
// bulk interval t (the paper's fixed interval, here `deadline_ns`) the loop
// cuts everything that has arrived into a bulk and issues it; results go back
// to the result pool (host memory) and each bulk's completion time is
// recorded, so the caller gets per-transaction commit latency.
//
// MI355X mapping:
//  * K slots, each with its own device bulk arrays, workspace and outputs, and
//    pre-instantiated HIP graphs (bulk generation and execution separately)
//    for power-of-two bulk sizes; a bulk is padded to its size class with
//    invalid transactions (no effect, outputs ignored).  Issuing a bulk costs
//    one host-to-device copy, two graph launches and two result copies.
//  * Bulk generation of a bulk runs on its slot's stream and overlaps the
//    execution of earlier bulks; executions are ordered on one stream, so the
//    database sees the bulks in arrival order.
//  * Admission: the number of slots is capped by an HBM byte budget; a cut
//    waits for a free slot, and everything that arrived meanwhile joins it.
#include <algorithm>
#include <chrono>
#include <cstring>
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
    gputx_bulk_stats* stats_h = nullptr;  // pinned
    hipStream_t fs = nullptr;
    hipEvent_t ready = nullptr, done = nullptr;
    std::vector<hipGraphExec_t> front, exec;
    std::vector<hipGraph_t> graphs;
    bool busy = false;
    int64_t first = 0, count = 0, cut_ns = 0, pad = 0;
};

struct BucketLayout {
    int64_t n;
    size_t off_type, off_params, off_ts, bytes;  // packed bulk arrays of this size
};

inline size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

BucketLayout layout_for(int64_t n, int np) {
    BucketLayout L;
    L.n = n;
    L.off_type = 0;
    L.off_params = up256((size_t)n * 4);
    L.off_ts = L.off_params + up256((size_t)n * 8 * np);
    L.bytes = L.off_ts + up256((size_t)n * 8);
    return L;
}

inline int64_t since(Clock::time_point t0) {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - t0).count();
}

}  // namespace

extern "C" int gputx_serve(gputx_handle h, const gputx_trace* tr, const gputx_serve_opts* o,
                           int32_t* status_out, int64_t* results_out, gputx_serve_bulk* bulks,
                           int64_t bulk_capacity, gputx_serve_report* rep) {
    if (!h || !tr || !o || !rep || (tr->n > 0 && (!tr->arrival_ns || !tr->type || !tr->params ||
                                                   !tr->ts || !status_out || !results_out)))
        return gtx_set_err(h, GPUTX_E_ARG, "null argument");
    if (o->deadline_ns <= 0 || o->slots < 1 || o->max_bulk < 1 || o->width < 1 || tr->n_params < 1 ||
        tr->n_params > GTX_MAX_PARAMS || o->strategy < GPUTX_AUTO || o->strategy > GPUTX_KSET)
        return gtx_set_err(h, GPUTX_E_ARG, "bad serving options");
    for (int64_t i = 1; i < tr->n; ++i)
        if (tr->arrival_ns[i] < tr->arrival_ns[i - 1] || tr->ts[i] <= tr->ts[i - 1])
            return gtx_set_err(h, GPUTX_E_ARG, "trace must be in arrival order with ascending ids");
    std::memset(rep, 0, sizeof *rep);
    HIP_OK(h, hipSetDevice(h->device));

    const int np = tr->n_params;
    const int W = o->width;
    int64_t maxb = kMinBucket;
    while (maxb < o->max_bulk) maxb <<= 1;
    std::vector<int64_t> sizes;
    for (int64_t b = kMinBucket; b <= maxb; b <<= 1) sizes.push_back(b);
    const BucketLayout big = layout_for(maxb, np);
    const size_t ws_bytes = gputx_workspace_size_ops(h, maxb, o->max_ops);
    const size_t off_ws = up256(big.bytes);
    const size_t off_status = off_ws + up256(ws_bytes);
    const size_t off_results = off_status + up256((size_t)maxb * 4);
    const size_t off_stats = off_results + up256((size_t)maxb * 8 * W);
    const size_t slot_bytes = off_stats + up256(sizeof(gputx_bulk_stats));
    rep->slot_bytes = (int64_t)slot_bytes;
    int nslots = o->slots;
    if (o->hbm_budget > 0) nslots = (int)std::min<int64_t>(nslots, o->hbm_budget / (int64_t)slot_bytes);
    if (nslots < 1) return gtx_set_err(h, GPUTX_E_CAPACITY, "HBM budget below one slot (%zu bytes)", slot_bytes);

    std::vector<Slot> slots(nslots);
    hipStream_t es = nullptr;
    int rc = GPUTX_OK;
    auto release = [&]() {
        for (auto& s : slots) {
            for (auto g : s.front) (void)hipGraphExecDestroy(g);
            for (auto g : s.exec) (void)hipGraphExecDestroy(g);
            for (auto g : s.graphs) (void)hipGraphDestroy(g);
            if (s.ready) (void)hipEventDestroy(s.ready);
            if (s.done) (void)hipEventDestroy(s.done);
            if (s.fs) (void)hipStreamDestroy(s.fs);
            if (s.dev) (void)hipFree(s.dev);
            if (s.stage) (void)hipHostFree(s.stage);
            if (s.stats_h) (void)hipHostFree(s.stats_h);
        }
        if (es) (void)hipStreamDestroy(es);
    };
#define SERVE_OK(call)                                                                        \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) {                                                               \
            rc = gtx_set_err(h, GPUTX_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
            release();                                                                        \
            return rc;                                                                        \
        }                                                                                     \
    } while (0)

    SERVE_OK(hipStreamCreateWithFlags(&es, hipStreamNonBlocking));
    const int grid = gtx_grid_for(h, 1);
    for (auto& s : slots) {
        SERVE_OK(hipMalloc(&s.dev, slot_bytes));
        SERVE_OK(hipHostMalloc(&s.stage, big.bytes, hipHostMallocDefault));
        SERVE_OK(hipHostMalloc(&s.stats_h, sizeof(gputx_bulk_stats), hipHostMallocDefault));
        SERVE_OK(hipStreamCreateWithFlags(&s.fs, hipStreamNonBlocking));
        SERVE_OK(hipEventCreateWithFlags(&s.ready, hipEventDisableTiming));
        SERVE_OK(hipEventCreateWithFlags(&s.done, hipEventDisableTiming));
        for (int64_t n : sizes) {
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
            rc = gtx_make_args(h, &b, o->strategy, s.dev + off_ws, ws_bytes,
                               reinterpret_cast<int32_t*>(s.dev + off_status),
                               reinterpret_cast<int64_t*>(s.dev + off_results), W,
                               reinterpret_cast<gputx_bulk_stats*>(s.dev + off_stats), grid, &a);
            if (rc) {
                release();
                return rc;
            }
            PhaseMarks none;
            hipGraph_t gf = nullptr, ge = nullptr;
            hipGraphExec_t xf = nullptr, xe = nullptr;
            SERVE_OK(hipStreamBeginCapture(s.fs, hipStreamCaptureModeThreadLocal));
            (void)launch_front(a, s.fs, none);
            SERVE_OK(hipStreamEndCapture(s.fs, &gf));
            s.graphs.push_back(gf);
            SERVE_OK(hipGraphInstantiate(&xf, gf, nullptr, nullptr, 0));
            s.front.push_back(xf);
            // upload now, so that the first bulk of this size class on this
            // slot does not pay for it in the middle of the trace
            SERVE_OK(hipGraphUpload(xf, s.fs));
            SERVE_OK(hipStreamBeginCapture(es, hipStreamCaptureModeThreadLocal));
            launch_exec(a, es, none);
            SERVE_OK(hipStreamEndCapture(es, &ge));
            s.graphs.push_back(ge);
            SERVE_OK(hipGraphInstantiate(&xe, ge, nullptr, nullptr, 0));
            s.exec.push_back(xe);
            SERVE_OK(hipGraphUpload(xe, es));
        }
    }
    SERVE_OK(hipDeviceSynchronize());

    const int64_t n = tr->n;
    const int64_t D = o->deadline_ns;
    std::vector<int> fifo;  // in-flight slots in issue order
    fifo.reserve(nslots);
    size_t head = 0;
    int64_t next_first = 0, deadline = D, nb = 0, last_done = 0;
    int next_slot = 0;
    const Clock::time_point t0 = Clock::now();

    auto retire = [&](bool block) -> int {
        while (head < fifo.size()) {
            Slot& s = slots[fifo[head]];
            hipError_t q = block ? hipEventSynchronize(s.done) : hipEventQuery(s.done);
            if (q == hipErrorNotReady) return GPUTX_OK;
            if (q != hipSuccess) return gtx_set_err(h, GPUTX_E_HIP, "bulk completion: %s", hipGetErrorString(q));
            const int64_t t = since(t0);
            last_done = t;
            if (nb < bulk_capacity && bulks) {
                gputx_serve_bulk& r = bulks[nb];
                r.first = s.first;
                r.count = s.count;
                r.cut_ns = s.cut_ns;
                r.done_ns = t;
                r.error = s.stats_h->error;
                r.slot = fifo[head];
            }
            ++nb;
            rep->committed += s.stats_h->committed;
            rep->aborted += s.stats_h->aborted;
            rep->invalid += s.stats_h->invalid - s.pad;  // padding is not part of the trace
            if (s.stats_h->error && !rc) rc = gtx_set_err(h, s.stats_h->error, "bulk at %lld failed on the device", (long long)s.first);
            s.busy = false;
            ++head;
            block = false;
        }
        return GPUTX_OK;
    };

    while (next_first < n || head < fifo.size()) {
        int r2 = retire(false);
        if (r2) {
            rc = r2;
            break;
        }
        const int64_t now = since(t0);
        if (next_first < n && now >= deadline) {
            Slot& s = slots[next_slot];
            if (s.busy) {  // admission: wait for the oldest bulk in flight
                std::this_thread::yield();
                continue;
            }
            const int64_t boundary = (now / D) * D;  // latest passed bulk interval
            const int64_t* last_p = std::lower_bound(tr->arrival_ns + next_first, tr->arrival_ns + n, boundary);
            const int64_t last = last_p - tr->arrival_ns;
            if (last == next_first) {
                deadline = boundary + D;
                continue;
            }
            const int64_t cnt = std::min<int64_t>(last - next_first, maxb);
            int bi = 0;
            while (sizes[bi] < cnt) ++bi;
            const BucketLayout L = layout_for(sizes[bi], np);
            // pack the bulk (param-major at its size class), padded with invalid
            // transactions whose ids follow the bulk's last id
            int32_t* st = reinterpret_cast<int32_t*>(s.stage + L.off_type);
            int64_t* sp = reinterpret_cast<int64_t*>(s.stage + L.off_params);
            int64_t* sts = reinterpret_cast<int64_t*>(s.stage + L.off_ts);
            std::memcpy(st, tr->type + next_first, cnt * 4);
            std::fill(st + cnt, st + L.n, -1);
            for (int k = 0; k < np; ++k) {
                std::memcpy(sp + (int64_t)k * L.n, tr->params + (int64_t)k * n + next_first, cnt * 8);
                std::fill(sp + (int64_t)k * L.n + cnt, sp + (int64_t)(k + 1) * L.n, 0);
            }
            std::memcpy(sts, tr->ts + next_first, cnt * 8);
            const int64_t tlast = tr->ts[next_first + cnt - 1];
            for (int64_t j = cnt; j < L.n; ++j) sts[j] = tlast + 1 + (j - cnt);
            s.first = next_first;
            s.count = cnt;
            s.pad = L.n - cnt;
            s.cut_ns = now;
            s.busy = true;
            hipError_t e = hipMemcpyAsync(s.dev, s.stage, L.bytes, hipMemcpyHostToDevice, s.fs);
            if (e == hipSuccess) e = hipGraphLaunch(s.front[bi], s.fs);
            if (e == hipSuccess) e = hipEventRecord(s.ready, s.fs);
            if (e == hipSuccess) e = hipStreamWaitEvent(es, s.ready, 0);
            if (e == hipSuccess) e = hipGraphLaunch(s.exec[bi], es);
            if (e == hipSuccess)
                e = hipMemcpyAsync(status_out + next_first, s.dev + off_status, cnt * 4, hipMemcpyDeviceToHost, es);
            if (e == hipSuccess)
                e = hipMemcpyAsync(results_out + next_first * W, s.dev + off_results, (size_t)cnt * 8 * W,
                                   hipMemcpyDeviceToHost, es);
            if (e == hipSuccess)
                e = hipMemcpyAsync(s.stats_h, s.dev + off_stats, sizeof(gputx_bulk_stats), hipMemcpyDeviceToHost, es);
            if (e == hipSuccess) e = hipEventRecord(s.done, es);
            if (e != hipSuccess) {
                rc = gtx_set_err(h, GPUTX_E_HIP, "issuing a bulk failed: %s", hipGetErrorString(e));
                break;
            }
            fifo.push_back(next_slot);
            next_slot = (next_slot + 1) % nslots;
            next_first += cnt;
            if (next_first == last) deadline = boundary + D;
        } else {
            std::this_thread::yield();
        }
    }
    (void)retire(true);
    (void)hipStreamSynchronize(es);
    rep->n_bulks = nb;
    rep->elapsed_ns = last_done;
    rep->slots_used = nslots;
    release();
#undef SERVE_OK
    return rc;
}
