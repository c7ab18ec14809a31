// Measurement probes: the ceilings the executors are judged against.
//
// Appendix D calibrates Algorithm 1 on the hardware at hand; these kernels
// measure the three quantities the engine's kernels are bound by on gfx950:
//
//   k_probe_handoff  one lock hand-off between two workgroups, with exactly
//                    the lock executor's sequence (relaxed spin on a counter,
//                    agent-scope acquire fence, a plain read-modify-write of
//                    a table cell, agent-scope release fence, atomic add).
//                    A chain of such hand-offs is the dependent step of TPL
//                    and of K-SET's cross-workgroup waves, so (depth + 1) x
//                    this latency bounds them from below.
//   k_probe_atomic   device atomic adds spread over n addresses (1, 64, 640:
//                    the hottest lock counters; millions: uniform random).
//   k_probe_gather   8-byte loads at uniform random rows of a table of a
//                    given size: a cache-resident size (the 256 MB Infinity
//                    Cache holds a 64 MB table) and an HBM-resident one.
//
// Random indices come from a counter-based mixer (SplitMix64's finaliser),
// so no index array adds traffic.  Every probe checks its own result.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "runtime.h"

namespace gtx {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Workgroup 0 and workgroup `partner` alternate turns; turn k belongs to
// player k % 2.  Consecutive workgroup ids are dispatched to different XCDs,
// so partner 1 sits on another XCD and partner 8 on the same one.
__global__ __launch_bounds__(64) void k_probe_handoff(int32_t* ctr, int64_t* cell, int32_t hops, int partner,
                                                      uint64_t spin_ticks, int32_t* err, uint64_t* elapsed) {
    int me;
    if (blockIdx.x == 0) me = 0;
    else if ((int)blockIdx.x == partner) me = 1;
    else return;
    if (threadIdx.x != 0) return;
    const uint64_t t0 = wall_clock64();
    for (int32_t k = me; k < hops; k += 2) {
        const uint64_t w0 = wall_clock64();
        while (ld_relaxed(ctr) < k) {
            if (ld_relaxed(err) != 0) return;
            if (wall_clock64() - w0 > spin_ticks) {
                atomicExch(err, 1);
                return;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        fence_acquire();   // see the partner's write of the cell
        *cell += 1;        // the critical section: a plain read-modify-write
        fence_release();   // publish it
        atomicAdd(ctr, 1); // hand the lock on
    }
    if (me == 0) elapsed[0] = wall_clock64() - t0;
}

__global__ __launch_bounds__(256) void k_probe_atomic(int32_t* ctr, uint64_t n_addr, int64_t per_thread) {
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t j = 0; j < per_thread; ++j) {
        const uint64_t a = n_addr == 1 ? 0 : mix64(g * (uint64_t)per_thread + (uint64_t)j) % n_addr;
        atomicAdd(&ctr[a], 1);
    }
}

__global__ __launch_bounds__(256) void k_probe_atomic_sum(const int32_t* ctr, uint64_t n_addr,
                                                          unsigned long long* total) {
    unsigned long long s = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_addr;
         i += (uint64_t)gridDim.x * blockDim.x)
        s += (unsigned long long)ctr[i];
    if (s) atomicAdd(total, s);
}

__global__ __launch_bounds__(256) void k_probe_gather(const int64_t* tbl, uint64_t mask, int64_t per_thread,
                                                      int64_t* out) {
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t acc = 0;
#pragma unroll 8
    for (int64_t j = 0; j < per_thread; ++j) acc += tbl[mix64(g * (uint64_t)per_thread + (uint64_t)j) & mask];
    out[g] = acc;
}

__global__ __launch_bounds__(256) void k_probe_fill(int64_t* tbl, uint64_t rows) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows;
         i += (uint64_t)gridDim.x * blockDim.x)
        tbl[i] = 1;
}

}  // namespace gtx

using namespace gtx;

namespace {
struct DevBuf {
    void* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};
struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};
}  // namespace

#define PROBE_OK(x)                                                                        \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess)                                                              \
            return gtx_set_err(nullptr, GPUTX_E_HIP, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

extern "C" int gputx_probe_handoff(int hip_device, int32_t hops, int32_t same_xcd, double* ns_per_hop) {
    if (!ns_per_hop || hops < 2 || hops > (1 << 24)) return gtx_set_err(nullptr, GPUTX_E_ARG, "bad probe argument");
    PROBE_OK(hipSetDevice(hip_device));
    int khz = 0;
    PROBE_OK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, hip_device));
    if (khz <= 0) khz = 100000;
    DevBuf buf;
    PROBE_OK(hipMalloc(&buf.p, 256));
    PROBE_OK(hipMemset(buf.p, 0, 256));
    char* base = (char*)buf.p;
    int32_t* ctr = (int32_t*)base;
    int32_t* err = (int32_t*)(base + 4);
    int64_t* cell = (int64_t*)(base + 128);  // its own cache line
    uint64_t* elapsed = (uint64_t*)(base + 64);
    const int partner = same_xcd ? 8 : 1;
    const uint64_t spin = (uint64_t)2000 * (uint64_t)khz;  // 2 s per turn at most
    hipLaunchKernelGGL(k_probe_handoff, dim3(partner + 1), dim3(64), 0, 0, ctr, cell, hops, partner, spin, err,
                       elapsed);
    PROBE_OK(hipGetLastError());
    PROBE_OK(hipDeviceSynchronize());
    int32_t e = 0;
    int64_t c = 0;
    uint64_t ticks = 0;
    PROBE_OK(hipMemcpy(&e, err, 4, hipMemcpyDeviceToHost));
    PROBE_OK(hipMemcpy(&c, cell, 8, hipMemcpyDeviceToHost));
    PROBE_OK(hipMemcpy(&ticks, elapsed, 8, hipMemcpyDeviceToHost));
    if (e) return gtx_set_err(nullptr, GPUTX_E_DEADLOCK, "hand-off probe: a turn waited more than 2 s");
    if (c != hops) return gtx_set_err(nullptr, GPUTX_E_INTERNAL, "hand-off probe: cell %lld != %d", (long long)c, hops);
    *ns_per_hop = (double)ticks * 1e6 / (double)khz / (double)hops;
    return GPUTX_OK;
}

extern "C" int gputx_probe_atomic_add(int hip_device, int64_t n_addr, int64_t n_updates, double* per_s) {
    if (!per_s || n_addr < 1 || n_addr > ((int64_t)1 << 30) || n_updates < 256 * 1024)
        return gtx_set_err(nullptr, GPUTX_E_ARG, "bad probe argument");
    PROBE_OK(hipSetDevice(hip_device));
    const int blocks = 1024;
    const int64_t threads = (int64_t)blocks * 256;
    const int64_t per_thread = std::max<int64_t>(1, n_updates / threads);
    const int64_t total = per_thread * threads;
    DevBuf ctr, sum;
    PROBE_OK(hipMalloc(&ctr.p, sizeof(int32_t) * (size_t)n_addr));
    PROBE_OK(hipMalloc(&sum.p, sizeof(unsigned long long)));
    Events ev;
    PROBE_OK(hipEventCreate(&ev.a));
    PROBE_OK(hipEventCreate(&ev.b));
    const int reps = 3;
    PROBE_OK(hipMemset(ctr.p, 0, sizeof(int32_t) * (size_t)n_addr));
    hipLaunchKernelGGL(k_probe_atomic, dim3(blocks), dim3(256), 0, 0, (int32_t*)ctr.p, (uint64_t)n_addr, per_thread);
    PROBE_OK(hipEventRecord(ev.a, 0));
    for (int r = 0; r < reps; ++r)
        hipLaunchKernelGGL(k_probe_atomic, dim3(blocks), dim3(256), 0, 0, (int32_t*)ctr.p, (uint64_t)n_addr,
                           per_thread);
    PROBE_OK(hipEventRecord(ev.b, 0));
    PROBE_OK(hipGetLastError());
    PROBE_OK(hipEventSynchronize(ev.b));
    float ms = 0;
    PROBE_OK(hipEventElapsedTime(&ms, ev.a, ev.b));
    PROBE_OK(hipMemset(sum.p, 0, sizeof(unsigned long long)));
    hipLaunchKernelGGL(k_probe_atomic_sum, dim3(256), dim3(256), 0, 0, (const int32_t*)ctr.p, (uint64_t)n_addr,
                       (unsigned long long*)sum.p);
    unsigned long long got = 0;
    PROBE_OK(hipMemcpy(&got, sum.p, sizeof got, hipMemcpyDeviceToHost));
    if (got != (unsigned long long)(total * (reps + 1)))
        return gtx_set_err(nullptr, GPUTX_E_INTERNAL, "atomic probe: %llu adds landed of %lld", got,
                           (long long)(total * (reps + 1)));
    *per_s = (double)total * reps / ((double)ms / 1e3);
    return GPUTX_OK;
}

extern "C" int gputx_probe_gather(int hip_device, int64_t table_bytes, int64_t n_gathers, double* gb_per_s) {
    if (!gb_per_s || table_bytes < 4096 || (table_bytes & (table_bytes - 1)) || n_gathers < 256 * 1024)
        return gtx_set_err(nullptr, GPUTX_E_ARG, "bad probe argument (table_bytes a power of two)");
    PROBE_OK(hipSetDevice(hip_device));
    const uint64_t rows = (uint64_t)table_bytes / 8;
    const int blocks = 2048;
    const int64_t threads = (int64_t)blocks * 256;
    const int64_t per_thread = std::max<int64_t>(1, n_gathers / threads);
    DevBuf tbl, out;
    PROBE_OK(hipMalloc(&tbl.p, (size_t)table_bytes));
    PROBE_OK(hipMalloc(&out.p, sizeof(int64_t) * (size_t)threads));
    hipLaunchKernelGGL(k_probe_fill, dim3(2048), dim3(256), 0, 0, (int64_t*)tbl.p, rows);
    Events ev;
    PROBE_OK(hipEventCreate(&ev.a));
    PROBE_OK(hipEventCreate(&ev.b));
    const int reps = 3;
    hipLaunchKernelGGL(k_probe_gather, dim3(blocks), dim3(256), 0, 0, (const int64_t*)tbl.p, rows - 1, per_thread,
                       (int64_t*)out.p);
    PROBE_OK(hipEventRecord(ev.a, 0));
    for (int r = 0; r < reps; ++r)
        hipLaunchKernelGGL(k_probe_gather, dim3(blocks), dim3(256), 0, 0, (const int64_t*)tbl.p, rows - 1,
                           per_thread, (int64_t*)out.p);
    PROBE_OK(hipEventRecord(ev.b, 0));
    PROBE_OK(hipGetLastError());
    PROBE_OK(hipEventSynchronize(ev.b));
    float ms = 0;
    PROBE_OK(hipEventElapsedTime(&ms, ev.a, ev.b));
    int64_t first = 0;
    PROBE_OK(hipMemcpy(&first, out.p, 8, hipMemcpyDeviceToHost));
    if (first != per_thread)  // every row holds 1
        return gtx_set_err(nullptr, GPUTX_E_INTERNAL, "gather probe: sum %lld != %lld", (long long)first,
                           (long long)per_thread);
    *gb_per_s = (double)per_thread * threads * 8 * reps / ((double)ms / 1e3) / 1e9;
    return GPUTX_OK;
}
