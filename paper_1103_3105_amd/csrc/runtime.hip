// Host runtime: the C ABI of include/gputx.h.
//
// A context holds the catalog (Appendix E: column metadata on the host,
// columns in device memory), the registered types resolved to device
// descriptors (Section 3.1), the device row counts of the append tables
// (Section 3.2 batched update) and the options of Algorithm 1.  A bulk runs
// as an asynchronous sequence of kernels on the caller's stream; every
// decision after the input arrives (timestamp order, strategy, wave count)
// is taken on the device, so no host round trip sits inside a bulk.
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "runtime.h"

using namespace gtx;

static thread_local std::string g_err;

int gtx_set_err(gputx_handle h, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (h) h->err = buf;
    else g_err = buf;
    return code;
}



static int bits_for(uint64_t v) {  // bits needed to represent v
    int b = 0;
    while (v) { ++b; v >>= 1; }
    return b;
}
static int passes_for(uint64_t maxkey) {
    int p = (bits_for(maxkey) + 7) / 8;
    return p < 1 ? 1 : p;
}

extern "C" int gputx_default_options(gputx_options* o) {
    if (!o) return GPUTX_E_ARG;
    // K-SET only for very wide 0-sets: on MI355X its per-wave barrier across 8
    // XCDs costs more than TPL's locks or PART's serial chains on every measured
    // workload (the autotuner fits all three thresholds to a workload mix)
    o->w0_bar = 1 << 20;
    o->c_bar = 0;
    o->d_bar = 1 << 30;
    o->part_size = 1;
    o->group_by_type = 1;
    o->kset_narrow = 256;
    o->spin_limit_ms = 5000;
    o->grid_blocks = 0;
    o->part_pipeline = 1;
    o->part_scan = 1;
    o->tpl_lanes = 0;
    return GPUTX_OK;
}

static int refresh_layout(gputx_handle h);

// ---- workspace for callers that cannot allocate ----------------------------
// gputx_execute_bulk_noalloc runs a bulk with its workspace in this array.
// In host code `scratch` names a host-side stand-in, not device memory: the
// device address of each GPU's copy is taken once per device when a context
// is created (with that device current) and only that address is used.
static __device__ __align__(256) unsigned char scratch[GPUTX_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64];

static int scratch_init(int dev) {
    if (dev < 0 || dev >= 64) return gtx_set_err(nullptr, GPUTX_E_ARG, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return GPUTX_OK;
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return gtx_set_err(nullptr, GPUTX_E_HIP, "scratch address on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
    return GPUTX_OK;
}

extern "C" int gputx_create(int dev, const gputx_options* opt, gputx_handle* out) {
    if (!out) return gtx_set_err(nullptr, GPUTX_E_ARG, "out is null");
    *out = nullptr;
    gputx_handle h = new gputx_ctx();
    h->device = dev;
    if (opt) h->opt = *opt;
    else gputx_default_options(&h->opt);
    hipError_t e = hipSetDevice(dev);
    int ncu = 0, khz = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    if (e == hipSuccess) e = hipMalloc(&h->d_types, sizeof(DevType) * GPUTX_MAX_TYPES);
    if (e == hipSuccess) e = hipMalloc(&h->d_rowcount, sizeof(int64_t) * GTX_MAX_APPEND);
    if (e == hipSuccess) e = hipMalloc(&h->d_capacity, sizeof(int64_t) * GTX_MAX_APPEND);
    if (e == hipSuccess) e = hipMemset(h->d_types, 0, sizeof(DevType) * GPUTX_MAX_TYPES);
    if (e == hipSuccess) e = hipMemset(h->d_rowcount, 0, sizeof(int64_t) * GTX_MAX_APPEND);
    if (e == hipSuccess) e = hipMemset(h->d_capacity, 0, sizeof(int64_t) * GTX_MAX_APPEND);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&h->side.s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->side.fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->side.join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->side.sorted, hipEventDisableTiming);
    if (e != hipSuccess) {
        int rc = gtx_set_err(nullptr, GPUTX_E_HIP, "device setup failed: %s", hipGetErrorString(e));
        if (h->d_types) (void)hipFree(h->d_types);
        if (h->d_rowcount) (void)hipFree(h->d_rowcount);
        if (h->d_capacity) (void)hipFree(h->d_capacity);
        if (h->side.join) (void)hipEventDestroy(h->side.join);
        if (h->side.sorted) (void)hipEventDestroy(h->side.sorted);
        if (h->side.fork) (void)hipEventDestroy(h->side.fork);
        if (h->side.s) (void)hipStreamDestroy(h->side.s);
        delete h;
        return rc;
    }
    h->ncu = ncu;
    h->wall_khz = khz > 0 ? (uint64_t)khz : 100000;
    exec_init_attributes(dev);
    const int src = scratch_init(dev);  // device current: this GPU's copy of the array
    if (src) {
        gputx_destroy(h);
        return src;
    }
    *out = h;
    return GPUTX_OK;
}

extern "C" int gputx_destroy(gputx_handle h) {
    if (!h) return GPUTX_E_ARG;
    (void)hipSetDevice(h->device);
    (void)hipFree(h->d_types);
    (void)hipFree(h->d_rowcount);
    (void)hipFree(h->d_capacity);
    (void)hipStreamSynchronize(h->side.s);
    (void)hipEventDestroy(h->side.join);
    (void)hipEventDestroy(h->side.fork);
    (void)hipEventDestroy(h->side.sorted);
    (void)hipStreamDestroy(h->side.s);
    if (h->ev) {
        for (int i = 0; i < gputx_ctx::kRing * PH_COUNT; ++i) (void)hipEventDestroy(h->ev[i]);
        delete[] h->ev;
    }
    delete h;
    return GPUTX_OK;
}

extern "C" int gputx_phase_timing(gputx_handle h, int enable) {
    if (!h) return gtx_set_err(h, GPUTX_E_ARG, "null handle");
    HIP_OK(h, hipSetDevice(h->device));
    if (enable && !h->ev) {
        h->ev = new hipEvent_t[gputx_ctx::kRing * PH_COUNT];
        for (int i = 0; i < gputx_ctx::kRing * PH_COUNT; ++i) HIP_OK(h, hipEventCreate(&h->ev[i]));
    }
    h->timing = enable != 0;
    h->ring_used = 0;
    return GPUTX_OK;
}

static const char* kPhaseNames[PH_COUNT - 1] = {"order", "prepare", "emit", "op_sort", "rank",
                                                "features", "part_sort", "part_gather", "part", "tpl",
                                                "kset", "finalize"};

extern "C" const char* gputx_phase_name(int i) {
    return (i >= 0 && i < PH_COUNT - 1) ? kPhaseNames[i] : nullptr;
}

extern "C" int gputx_phase_times(gputx_handle h, double* ms, int cap, int64_t* n_bulks) {
    if (!h || (cap > 0 && !ms)) return gtx_set_err(h, GPUTX_E_ARG, "bad arguments");
    HIP_OK(h, hipSetDevice(h->device));
    for (int i = 0; i < cap; ++i) ms[i] = 0;
    if (n_bulks) *n_bulks = h->ring_used;
    if (!h->ev || h->ring_used == 0) return PH_COUNT - 1;
    HIP_OK(h, hipEventSynchronize(h->ev[(h->ring_used - 1) * PH_COUNT + PH_FINAL]));
    for (int b = 0; b < h->ring_used; ++b) {
        for (int p = 1; p < PH_COUNT && p - 1 < cap; ++p) {
            float t = 0;
            HIP_OK(h, hipEventElapsedTime(&t, h->ev[b * PH_COUNT + p - 1], h->ev[b * PH_COUNT + p]));
            ms[p - 1] += t;
        }
    }
    return PH_COUNT - 1;
}

extern "C" int gputx_set_options(gputx_handle h, const gputx_options* opt) {
    if (!h || !opt) return gtx_set_err(h, GPUTX_E_ARG, "null argument");
    if (opt->part_size < 1 || opt->spin_limit_ms < 1 || opt->grid_blocks < 0 || opt->tpl_lanes < 0 ||
        opt->tpl_lanes > 64)
        return gtx_set_err(h, GPUTX_E_ARG, "bad option value");
    h->opt = *opt;
    return refresh_layout(h);
}

extern "C" int gputx_load_tables(gputx_handle h, const gputx_table_desc* t, int n) {
    if (!h || (n > 0 && !t) || n < 0) return gtx_set_err(h, GPUTX_E_ARG, "bad arguments");
    HIP_OK(h, hipSetDevice(h->device));
    for (int i = 0; i < n; ++i) {
        const gputx_table_desc& d = t[i];
        if (d.table_id < 0 || d.table_id >= GPUTX_MAX_TABLES)
            return gtx_set_err(h, GPUTX_E_ARG, "table_id %d out of range", d.table_id);
        if (h->tabs[d.table_id].present)
            return gtx_set_err(h, GPUTX_E_ARG, "table %d already loaded", d.table_id);
        if (d.n_cols < 1 || d.n_cols > GPUTX_MAX_COLS || d.n_rows < 0 || d.capacity < d.n_rows)
            return gtx_set_err(h, GPUTX_E_ARG, "table %d: bad shape", d.table_id);
        if (d.root_table_id >= GPUTX_MAX_TABLES || (d.root_table_id >= 0 && d.root_div < 1))
            return gtx_set_err(h, GPUTX_E_ARG, "table %d: bad root", d.table_id);
        for (int c = 0; c < d.n_cols; ++c) {
            if (d.col_dtype[c] != GPUTX_I32 && d.col_dtype[c] != GPUTX_I64)
                return gtx_set_err(h, GPUTX_E_ARG, "table %d col %d: bad dtype", d.table_id, c);
            if (!d.col_ptr[c] && d.capacity > 0)
                return gtx_set_err(h, GPUTX_E_ARG, "table %d col %d: null column", d.table_id, c);
        }
        if (d.append_only && h->n_app >= GTX_MAX_APPEND)
            return gtx_set_err(h, GPUTX_E_CAPACITY, "at most %d append-only tables", GTX_MAX_APPEND);
    }
    for (int i = 0; i < n; ++i) {
        const gputx_table_desc& d = t[i];
        auto& T = h->tabs[d.table_id];
        T.present = true;
        T.d = d;
        if (d.append_only) {
            T.app_idx = h->n_app;
            h->app_table[h->n_app] = d.table_id;
            int64_t rc = d.n_rows, cap = d.capacity;
            HIP_OK(h, hipMemcpy(h->d_rowcount + h->n_app, &rc, 8, hipMemcpyHostToDevice));
            HIP_OK(h, hipMemcpy(h->d_capacity + h->n_app, &cap, 8, hipMemcpyHostToDevice));
            h->n_app++;
        }
    }
    return refresh_layout(h);
}

// Item keys (Section 4.1 data items) are dense: table key base + row.
// Partition ids (Section 5.2) are dense per root table: base + root / size.
static int refresh_layout(gputx_handle h) {
    uint64_t base = 0;
    for (int i = 0; i < GPUTX_MAX_TABLES; ++i) {
        auto& T = h->tabs[i];
        if (!T.present || T.d.append_only) continue;
        T.key_base = (uint32_t)base;
        base += (uint64_t)T.d.n_rows;
    }
    if (base >= 0xffffffffull) return gtx_set_err(h, GPUTX_E_CAPACITY, "more than 2^32-1 data items");
    h->total_items = base;
    h->key_passes = passes_for(base ? base - 1 : 0);
    int64_t pb = 0;
    bool is_root[GPUTX_MAX_TABLES] = {};
    for (int i = 0; i < GPUTX_MAX_TABLES; ++i)
        if (h->tabs[i].present && h->tabs[i].d.root_table_id >= 0) is_root[h->tabs[i].d.root_table_id] = true;
    for (int i = 0; i < GPUTX_MAX_TABLES; ++i) {
        auto& T = h->tabs[i];
        T.part_base = -1;
        if (!T.present || !is_root[i]) continue;
        T.part_base = pb;
        pb += (T.d.n_rows + h->opt.part_size - 1) / h->opt.part_size;
    }
    if (pb >= 0xffffffffll) return gtx_set_err(h, GPUTX_E_CAPACITY, "too many partitions");
    h->n_parts = pb;
    h->part_passes = passes_for((uint64_t)pb);  // sentinel id = n_parts
    // re-resolve registered types (key bases or partition size may have moved)
    for (int t = 0; t < GPUTX_MAX_TYPES; ++t) {
        if (!h->type_present[t]) continue;
        int rc = gputx_register_types(h, &h->types[t], 1);
        if (rc) return rc;
    }
    return GPUTX_OK;
}

struct ProcSpec {
    int n_roles;
    int min_params;
    int max_results;
    int ops;
    // per role: expected dtypes (0 = unchecked), append flag
    int append[GTX_ROLES];
    int ncols[GTX_ROLES];
    int dtype[GTX_ROLES][16];
};

static bool proc_spec(int proc, ProcSpec* s) {
    std::memset(s, 0, sizeof *s);
    auto role = [&](int r, int app, std::initializer_list<int> dts) {
        s->append[r] = app;
        int c = 0;
        for (int d : dts) s->dtype[r][c++] = d;
        s->ncols[r] = c;
    };
    const int I = GPUTX_I32, L = GPUTX_I64;
    switch (proc) {
    case GPUTX_DEBIT_CREDIT:
        s->n_roles = 4; s->min_params = 4; s->max_results = 3; s->ops = 3;
        role(0, 0, {L}); role(1, 0, {L}); role(2, 0, {L}); role(3, 1, {L, L, L, L, L});
        return true;
    case GPUTX_NEW_ORDER:
    case GPUTX_NEW_ORDER_RB:
    case GPUTX_PAYMENT:
    case GPUTX_ORDER_STATUS: {
        const bool no = proc == GPUTX_NEW_ORDER || proc == GPUTX_NEW_ORDER_RB;
        s->n_roles = 6;
        s->min_params = no ? 34 : (proc == GPUTX_PAYMENT ? 4 : 3);
        s->max_results = no ? 16 : (proc == GPUTX_PAYMENT ? 3 : 1);
        s->ops = no ? 15 : (proc == GPUTX_PAYMENT ? 3 : 1);
        role(0, 0, {L}); role(1, 0, {L}); role(2, 0, {L}); role(3, 0, {I});
        role(4, 1, {L, L, L, L, L}); role(5, 1, {L, L, L, L, L});
        return true;
    }
    case GPUTX_GET_SUB:
    case GPUTX_GET_CF:
    case GPUTX_UPD_SUB_FIELD:
    case GPUTX_UPD_LOC:
    case GPUTX_INS_CF:
    case GPUTX_DEL_CF:
        s->n_roles = 2; s->ops = 1;
        s->min_params = (proc == GPUTX_GET_SUB) ? 1 : (proc == GPUTX_INS_CF ? 4 :
                        (proc == GPUTX_GET_CF || proc == GPUTX_DEL_CF) ? 2 : 3);
        s->max_results = proc == GPUTX_GET_SUB ? 14 : ((proc == GPUTX_GET_CF || proc == GPUTX_DEL_CF) ? 3 : 1);
        role(0, 0, {L, I, I, I, I, I, I, I, I, I, I, I, I, I, I});
        role(1, 0, {I, I, L});
        return true;
    }
    return false;
}

extern "C" int gputx_register_types(gputx_handle h, const gputx_type_desc* t, int n) {
    if (!h || (n > 0 && !t) || n < 0) return gtx_set_err(h, GPUTX_E_ARG, "bad arguments");
    HIP_OK(h, hipSetDevice(h->device));
    for (int i = 0; i < n; ++i) {
        const gputx_type_desc& d = t[i];
        if (d.type_id < 0 || d.type_id >= GPUTX_MAX_TYPES)
            return gtx_set_err(h, GPUTX_E_ARG, "type_id %d out of range", d.type_id);
        ProcSpec ps;
        if (!proc_spec(d.proc, &ps)) return gtx_set_err(h, GPUTX_E_TYPE, "type %d: unknown procedure %d", d.type_id, d.proc);
        if (d.n_params < ps.min_params || d.n_params > GTX_MAX_PARAMS)
            return gtx_set_err(h, GPUTX_E_TYPE, "type %d: n_params %d, procedure needs %d", d.type_id, d.n_params, ps.min_params);
        DevType D;
        std::memset(&D, 0, sizeof D);
        D.proc = d.proc;
        D.n_params = d.n_params;
        D.n_results = d.n_results;
        D.root_key = d.root_key ? 1 : 0;
        D.app_idx[0] = D.app_idx[1] = -1;
        D.part_size = h->opt.part_size;
        int app_slot = 0;
        for (int r = 0; r < ps.n_roles; ++r) {
            int tid = d.table_ids[r];
            if (tid < 0 || tid >= GPUTX_MAX_TABLES || !h->tabs[tid].present)
                return gtx_set_err(h, GPUTX_E_TYPE, "type %d role %d: table %d not loaded", d.type_id, r, tid);
            for (int r2 = 0; r2 < r; ++r2)
                if (d.table_ids[r2] == tid)
                    return gtx_set_err(h, GPUTX_E_TYPE, "type %d: table %d bound to two roles", d.type_id, tid);
            const auto& T = h->tabs[tid];
            if (!!T.d.append_only != !!ps.append[r])
                return gtx_set_err(h, GPUTX_E_TYPE, "type %d role %d: append-only mismatch", d.type_id, r);
            if (T.d.n_cols < ps.ncols[r])
                return gtx_set_err(h, GPUTX_E_TYPE, "type %d role %d: needs %d columns", d.type_id, r, ps.ncols[r]);
            for (int c = 0; c < ps.ncols[r]; ++c)
                if (T.d.col_dtype[c] != ps.dtype[r][c])
                    return gtx_set_err(h, GPUTX_E_TYPE, "type %d role %d col %d: wrong dtype", d.type_id, r, c);
            for (int c = 0; c < T.d.n_cols; ++c) D.col[r][c] = T.d.col_ptr[c];
            D.rows[r] = T.d.n_rows;
            D.key_base[r] = T.key_base;
            if (T.d.root_table_id >= 0) {
                const auto& R = h->tabs[T.d.root_table_id];
                if (!R.present) return gtx_set_err(h, GPUTX_E_TYPE, "table %d: root table %d not loaded", tid, T.d.root_table_id);
                D.root_div[r] = T.d.root_div;
                D.root_base[r] = R.key_base;
                D.part_base[r] = R.part_base;
            } else {
                D.root_div[r] = 1;
                D.root_base[r] = T.key_base;
                D.part_base[r] = -1;
                if (d.root_key && !ps.append[r])
                    return gtx_set_err(h, GPUTX_E_TYPE, "type %d: root-key mode but table %d has no root", d.type_id, tid);
            }
            if (ps.append[r]) {
                if (d.proc == GPUTX_DEBIT_CREDIT || d.proc == GPUTX_NEW_ORDER || d.proc == GPUTX_NEW_ORDER_RB)
                    D.app_idx[app_slot] = T.app_idx;
                ++app_slot;
            }
        }
        if (d.proc == GPUTX_NEW_ORDER || d.proc == GPUTX_NEW_ORDER_RB || d.proc == GPUTX_PAYMENT ||
            d.proc == GPUTX_ORDER_STATUS) {
            int64_t nw = D.rows[0], nd = D.rows[1];
            if (nw < 1 || nd < 1) return gtx_set_err(h, GPUTX_E_TYPE, "type %d: empty warehouse/district", d.type_id);
            D.dims[0] = nw;
            D.dims[1] = nd / nw;
            D.dims[2] = D.rows[2] / nd;
            D.dims[3] = D.rows[3] / nw;
        }
        HIP_OK(h, hipMemcpy(h->d_types + d.type_id, &D, sizeof D, hipMemcpyHostToDevice));
        h->types[d.type_id] = d;
        h->type_present[d.type_id] = true;
    }
    int mo = 1;
    for (int i = 0; i < GPUTX_MAX_TYPES; ++i) {
        if (!h->type_present[i]) continue;
        ProcSpec ps;
        proc_spec(h->types[i].proc, &ps);
        mo = std::max(mo, ps.ops);
    }
    h->max_ops = mo;
    // Cell classes: types whose procedures name rows of a common table are
    // joined, so types of different classes never name the same cell (PART
    // may run them side by side).
    int cls[GPUTX_MAX_TYPES];
    for (int i = 0; i < GPUTX_MAX_TYPES; ++i) cls[i] = i;
    auto find = [&](int x) {
        while (cls[x] != x) x = cls[x] = cls[cls[x]];
        return x;
    };
    auto tables_of = [&](int i, int64_t* ids) {
        const uint32_t roles = proc_cell_roles(h->types[i].proc);
        int k = 0;
        for (int r = 0; r < GTX_ROLES; ++r)
            if ((roles >> r) & 1u) ids[k++] = h->types[i].table_ids[r];
        return k;
    };
    for (int i = 0; i < GPUTX_MAX_TYPES; ++i) {
        if (!h->type_present[i]) continue;
        int64_t ti[GTX_ROLES];
        const int ni = tables_of(i, ti);
        for (int j = 0; j < i; ++j) {
            if (!h->type_present[j]) continue;
            int64_t tj[GTX_ROLES];
            const int nj = tables_of(j, tj);
            bool shared = false;
            for (int x = 0; x < ni && !shared; ++x)
                for (int y = 0; y < nj && !shared; ++y) shared = ti[x] == tj[y];
            if (shared) cls[find(i)] = find(j);
        }
    }
    int label[GPUTX_MAX_TYPES], nlabel = 0;
    for (int i = 0; i < GPUTX_MAX_TYPES; ++i) label[i] = -1;
    for (int i = 0; i < GPUTX_MAX_TYPES; ++i) {
        if (!h->type_present[i]) continue;
        const int root = find(i);
        if (label[root] < 0) label[root] = nlabel++;
        const int32_t c = label[root];
        HIP_OK(h, hipMemcpy((char*)(h->d_types + i) + offsetof(DevType, cell_class), &c, sizeof c,
                            hipMemcpyHostToDevice));
    }
    return GPUTX_OK;
}

// ---- workspace layout -----------------------------------------------------
struct Layout {
    size_t off = 0;
    char* base = nullptr;
    template <class T>
    T* take(int64_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += sizeof(T) * (size_t)std::max<int64_t>(count, 1);
        return p;
    }
};

static void plan_ws(const gputx_ctx* h, int64_t n, int max_ops, void* base, Ws* ws, size_t* bytes,
                    int64_t* mcap_out) {
    Layout L;
    L.base = (char*)base;
    const int64_t mcap = n * (max_ops > 0 ? std::min(max_ops, h->max_ops) : h->max_ops);
    Ws w{};
    w.st = L.take<GtxState>(1);
    w.tsk[0] = L.take<uint64_t>(n); w.tsk[1] = L.take<uint64_t>(n);
    w.tsv[0] = L.take<uint32_t>(n); w.tsv[1] = L.take<uint32_t>(n);
    w.tty = L.take<int32_t>(n);
    w.cnt = L.take<int32_t>(n * (1 + GTX_MAX_APPEND));
    w.maxrank = L.take<int32_t>(n);
    w.indeg = L.take<int32_t>(n);
    w.ksrec = L.take<KsetRec>(n);
    w.op_txn = L.take<int32_t>(mcap);
    w.pk[0] = L.take<uint32_t>(mcap); w.pk[1] = L.take<uint32_t>(mcap);
    w.pv[0] = L.take<uint32_t>(mcap); w.pv[1] = L.take<uint32_t>(mcap);
    w.op_rank = L.take<int32_t>(mcap);
    w.op_info = L.take<OpInfo>(mcap);
    w.srt_txn = L.take<int32_t>(mcap);
    w.grp_cnt = L.take<int32_t>(mcap);
    w.qk[0] = L.take<uint32_t>(n); w.qk[1] = L.take<uint32_t>(n);
    w.qv[0] = L.take<uint32_t>(n); w.qv[1] = L.take<uint32_t>(n);
    w.qinv = L.take<uint32_t>(n);
    w.heads = L.take<int32_t>(n + 1);
    w.heads_tmp = L.take<int32_t>(std::max<int64_t>(1, (n + 2047) / 2048));
    int prm_rows = 1;
    for (int i = 0; i < GPUTX_MAX_TYPES; ++i)
        if (h->type_present[i]) prm_rows = std::max(prm_rows, proc_params(h->types[i].proc));
    w.rec = L.take<int64_t>(n * part_rec_words(prm_rows));
    w.front[0] = L.take<int32_t>(n); w.front[1] = L.take<int32_t>(n);
    w.sort_hist = L.take<uint32_t>(8 * 256);
    size_t sw = std::max(sort_status_words(n, 8), sort_status_words(mcap, h->key_passes));
    w.sort_status = L.take<uint32_t>((int64_t)sw);
    w.sort_ctrl = L.take<uint32_t>(16);
    w.psort_hist = L.take<uint32_t>(8 * 256);
    w.psort_status = L.take<uint32_t>((int64_t)sort_status_words(n, h->part_passes));
    w.psort_ctrl = L.take<uint32_t>(16);
    const int64_t nb = std::max<int64_t>(1, (n + kScanTile - 1) / kScanTile);
    w.scan_tmp = L.take<int32_t>(nb * (1 + GTX_MAX_APPEND));
    w.tcnt_tmp = L.take<int32_t>(kPrepBlocks * GPUTX_MAX_TYPES);
    const int64_t nbr = std::max<int64_t>(1, (mcap + kRankTile - 1) / kRankTile);
    w.rank_tmp = L.take<RankAgg>(2 * nbr);
    *ws = w;
    *bytes = L.off + 256;
    *mcap_out = mcap;
}

extern "C" size_t gputx_workspace_size_ops(gputx_handle h, int64_t n, int32_t max_ops) {
    if (!h || n < 0 || max_ops < 0) return 0;
    Ws w;
    size_t b;
    int64_t mcap;
    plan_ws(h, n, max_ops, nullptr, &w, &b, &mcap);
    return b;
}

extern "C" size_t gputx_workspace_size(gputx_handle h, int64_t n) {
    return gputx_workspace_size_ops(h, n, 0);
}

// Validate one bulk's arguments and fill its kernel arguments.
int gtx_make_args(gputx_handle h, const gputx_bulk* b, int strategy, void* workspace, size_t ws_bytes,
                     int32_t* status_out, int64_t* results_out, int32_t width, gputx_bulk_stats* stats,
                     int grid_blocks, BulkArgs* out) {
    if (!b || !stats) return gtx_set_err(h, GPUTX_E_ARG, "null argument");
    if (strategy < GPUTX_AUTO || strategy > GPUTX_KSET) return gtx_set_err(h, GPUTX_E_ARG, "bad strategy %d", strategy);
    if (b->n < 0 || b->n > (int64_t)1 << 30) return gtx_set_err(h, GPUTX_E_ARG, "bulk size %lld", (long long)b->n);
    if (width < 1) return gtx_set_err(h, GPUTX_E_ARG, "width must be >= 1");
    if (b->n > 0 && (!b->type || !b->params || !b->ts || !status_out || !results_out || !workspace))
        return gtx_set_err(h, GPUTX_E_ARG, "null bulk or output pointer");
    if (b->n_params < 1 || b->n_params > GTX_MAX_PARAMS) return gtx_set_err(h, GPUTX_E_ARG, "n_params %d", b->n_params);
    bool any = false;
    for (int i = 0; i < GPUTX_MAX_TYPES; ++i) any = any || h->type_present[i];
    if (!any) return gtx_set_err(h, GPUTX_E_STATE, "no registered types");
    BulkArgs a{};
    size_t need;
    if (b->max_ops < 0) return gtx_set_err(h, GPUTX_E_ARG, "max_ops %d", b->max_ops);
    plan_ws(h, b->n, b->max_ops, workspace, &a.ws, &need, &a.mcap);
    if (ws_bytes < need) return gtx_set_err(h, GPUTX_E_CAPACITY, "workspace %zu < %zu bytes", ws_bytes, need);
    if ((uintptr_t)workspace % 256) return gtx_set_err(h, GPUTX_E_ARG, "workspace must be 256-byte aligned");
    if (a.mcap >= ((int64_t)1 << 31) - 2) return gtx_set_err(h, GPUTX_E_CAPACITY, "too many operations for one bulk");
    a.type = b->type;
    a.params = b->params;
    a.ts = b->ts;
    a.n = b->n;
    a.n_params = b->n_params;
    a.ts_sorted = b->ts_sorted ? 1 : 0;
    a.status = status_out;
    a.results = results_out;
    a.width = width;
    a.n_app = h->n_app;
    a.types = h->d_types;
    a.rowcount = h->d_rowcount;
    a.capacity = h->d_capacity;
    a.stats = stats;
    a.key_passes = h->key_passes;
    a.part_passes = h->part_passes;
    a.n_parts = h->n_parts;
    a.strategy = strategy;
    a.group_by_type = h->opt.group_by_type;
    a.w0_bar = h->opt.w0_bar;
    a.c_bar = h->opt.c_bar;
    a.d_bar = h->opt.d_bar;
    a.kset_narrow = h->opt.kset_narrow;
    a.part_pipeline = h->opt.part_pipeline;
    a.part_scan = h->opt.part_scan;
    a.tpl_lanes = h->opt.tpl_lanes;
    a.grid_blocks = grid_blocks;
    a.spin_ticks = (uint64_t)h->opt.spin_limit_ms * h->wall_khz;
    // PART cell table: at most half full when every lane of a chunk stages
    // the most cells any registered procedure lists
    uint32_t present = 0;
    for (int i = 0; i < GPUTX_MAX_TYPES; ++i)
        if (h->type_present[i]) present |= 1u << i;
    a.type_mask = (b->type_mask ? b->type_mask : present) & present;
    if (!a.type_mask) return gtx_set_err(h, GPUTX_E_ARG, "type_mask names no registered type");
    a.cells_max = 1;
    a.prm_rows = 1;
    a.res_rows = 1;
    for (int i = 0; i < GPUTX_MAX_TYPES; ++i) {
        if (!((a.type_mask >> i) & 1u)) continue;
        a.cells_max = std::max(a.cells_max, proc_cells(h->types[i].proc));
        a.prm_rows = std::max(a.prm_rows, proc_params(h->types[i].proc));
        a.res_rows = std::max(a.res_rows, proc_results(h->types[i].proc));
    }
    a.rec_words = part_rec_words(a.prm_rows);
    a.cell_bits = 1;
    while ((1 << a.cell_bits) < 2 * 64 * a.cells_max) ++a.cell_bits;
    // the pipelined form keeps cells across chunks: room for several chunks
    a.pipe_bits = a.cell_bits;
    while ((1 << a.pipe_bits) < 4 * 256 * a.cells_max && a.pipe_bits < 12) ++a.pipe_bits;
    // one chunk of the widest form that runs must fit in half the table;
    // launch_exec picks the widest form whose LDS fits
    while ((1 << a.pipe_bits) < 2 * 128 * a.cells_max) ++a.pipe_bits;
    *out = a;
    return GPUTX_OK;
}

// Most persistent-grid workgroups the device can hold at once.
static int resident_capacity(gputx_handle h) {
    return h->ncu * std::max(exec_resident_blocks_per_cu(), 1);
}

int gtx_grid_for(gputx_handle h, int lanes) {
    int cap = resident_capacity(h) / std::max(lanes, 1);
    int want = h->opt.grid_blocks > 0 ? h->opt.grid_blocks : h->ncu;
    return std::max(1, std::min(want, cap));
}

extern "C" int gputx_execute_bulk(gputx_handle h, const gputx_bulk* b, int strategy, void* workspace,
                                  size_t ws_bytes, int32_t* status_out, int64_t* results_out, int32_t width,
                                  gputx_bulk_stats* stats, gputx_stream_t stream) {
    if (!h) return gtx_set_err(h, GPUTX_E_ARG, "null handle");
    HIP_OK(h, hipSetDevice(h->device));
    BulkArgs a;
    int rc = gtx_make_args(h, b, strategy, workspace, ws_bytes, status_out, results_out, width, stats,
                       gtx_grid_for(h, 1), &a);
    if (rc) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    PhaseMarks pm;
    if (h->timing && h->ev && h->ring_used < gputx_ctx::kRing && b->n > 0)
        pm.ev = h->ev + (h->ring_used++) * PH_COUNT;
    if (b->n == 0) {
        launch_empty(a, s);
    } else {
        // PART's partition sort does not depend on the choice: when PART may
        // run, it overlaps the ranking on the context's second stream
        a.part_early = (strategy == GPUTX_AUTO || strategy == GPUTX_PART) ? 1 : 0;
        hipError_t fe = launch_front(a, s, pm, &h->side);
        if (fe != hipSuccess) return gtx_set_err(h, GPUTX_E_HIP, "stream fork failed: %s", hipGetErrorString(fe));
        launch_exec(a, s, pm);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return gtx_set_err(h, GPUTX_E_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    return GPUTX_OK;
}

extern "C" int gputx_execute_bulk_relaxed(gputx_handle h, const gputx_bulk* b, int strategy, void* workspace,
                                          size_t ws_bytes, int32_t* status_out, int64_t* results_out,
                                          int32_t width, int64_t* serial_key_out, gputx_bulk_stats* stats,
                                          gputx_stream_t stream) {
    if (!h) return gtx_set_err(h, GPUTX_E_ARG, "null handle");
    if (strategy != GPUTX_TPL && strategy != GPUTX_PART)
        return gtx_set_err(h, GPUTX_E_ARG, "relaxed execution runs GPUTX_TPL or GPUTX_PART, not %d", strategy);
    if (b && b->n > 0 && !serial_key_out) return gtx_set_err(h, GPUTX_E_ARG, "null serial_key_out");
    HIP_OK(h, hipSetDevice(h->device));
    BulkArgs a;
    int rc = gtx_make_args(h, b, strategy, workspace, ws_bytes, status_out, results_out, width, stats,
                           gtx_grid_for(h, 1), &a);
    if (rc) return rc;
    a.part_early = 0;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    PhaseMarks pm;
    if (h->timing && h->ev && h->ring_used < gputx_ctx::kRing && b->n > 0)
        pm.ev = h->ev + (h->ring_used++) * PH_COUNT;
    if (b->n == 0) {
        launch_empty(a, s);
    } else {
        launch_front_relaxed(a, s, pm);
        launch_exec_relaxed(a, s, pm, serial_key_out);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return gtx_set_err(h, GPUTX_E_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    return GPUTX_OK;
}

extern "C" int gputx_execute_bulk_noalloc(gputx_handle h, const gputx_bulk* b, int strategy,
                                          int32_t* status_out, int64_t* results_out, int32_t width,
                                          gputx_bulk_stats* stats, gputx_stream_t stream) {
    if (!h || !b) return gtx_set_err(h, GPUTX_E_ARG, "null argument");
    if (b->n < 0 || b->max_ops < 0) return gtx_set_err(h, GPUTX_E_ARG, "bad bulk");
    const size_t need = gputx_workspace_size_ops(h, b->n, b->max_ops);
    if (need > (size_t)GPUTX_SCRATCH_BYTES)
        return gtx_set_err(h, GPUTX_E_CAPACITY,
                           "bulk of %lld transactions needs %zu workspace bytes; the static workspace holds %zu",
                           (long long)b->n, need, (size_t)GPUTX_SCRATCH_BYTES);
    void* ws = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        ws = (h->device >= 0 && h->device < 64) ? g_scratch_ptr[h->device] : nullptr;
    }
    if (!ws) return gtx_set_err(h, GPUTX_E_STATE, "no static workspace address for device %d", h->device);
    return gputx_execute_bulk(h, b, strategy, ws, (size_t)GPUTX_SCRATCH_BYTES, status_out, results_out, width,
                              stats, stream);
}

// ---- batched form: many bulks in one HIP graph ------------------------------
struct gputx_batch_t {
    gputx_handle h = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int items = 0;
    int lanes = 0;
};

extern "C" int gputx_batch_create(gputx_handle h, const gputx_batch_item* items, int n, gputx_batch* out) {
    if (!h || !out || n < 0 || (n > 0 && !items)) return gtx_set_err(h, GPUTX_E_ARG, "bad arguments");
    *out = nullptr;
    HIP_OK(h, hipSetDevice(h->device));
    int lanes = 0;
    for (int k = 0; k < n; ++k) {
        if (items[k].lane < 0 || items[k].lane >= 64) return gtx_set_err(h, GPUTX_E_ARG, "lane %d out of range", items[k].lane);
        lanes = std::max(lanes, items[k].lane + 1);
    }
    const int grid = gtx_grid_for(h, lanes);
    const int cap = std::max(1, resident_capacity(h) / std::max(lanes, 1));  // every lane's grid resident
    std::vector<BulkArgs> args(n);
    for (int k = 0; k < n; ++k) {
        const gputx_batch_item& it = items[k];
        if (it.grid_blocks < 0 || it.kset_narrow < 0) return gtx_set_err(h, GPUTX_E_ARG, "item %d: bad launch shape", k);
        const int g = it.grid_blocks > 0 ? std::min(it.grid_blocks, cap) : grid;
        int rc = gtx_make_args(h, &it.bulk, it.strategy, it.workspace, it.ws_bytes, it.status_out,
                           it.results_out, it.width, it.stats, g, &args[k]);
        if (rc) return rc;
        if (it.kset_narrow > 0) args[k].kset_narrow = it.kset_narrow;
    }
    // Two streams per lane: bulk generation (front) and execution.  A lane's
    // executions stay in order; the front phase of a bulk only waits for the
    // previous front phase, so it overlaps the previous bulk's execution.
    std::vector<hipStream_t> fs(lanes), es(lanes);
    std::vector<hipEvent_t> evs;
    hipStream_t origin;
    auto mkev = [&]() {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return (hipEvent_t) nullptr;
        evs.push_back(e);
        return e;
    };
    auto cleanup = [&]() {
        for (auto e : evs) (void)hipEventDestroy(e);
        for (int l = 0; l < lanes; ++l) {
            if (fs[l]) (void)hipStreamDestroy(fs[l]);
            if (es[l]) (void)hipStreamDestroy(es[l]);
        }
        (void)hipStreamDestroy(origin);
    };
    HIP_OK(h, hipStreamCreateWithFlags(&origin, hipStreamNonBlocking));
    for (int l = 0; l < lanes; ++l) {
        fs[l] = es[l] = nullptr;
        if (hipStreamCreateWithFlags(&fs[l], hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&es[l], hipStreamNonBlocking) != hipSuccess) {
            cleanup();
            return gtx_set_err(h, GPUTX_E_HIP, "stream creation failed");
        }
    }
    (void)hipGetLastError();
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipEvent_t fork = mkev();
        e = hipEventRecord(fork, origin);
        for (int l = 0; l < lanes && e == hipSuccess; ++l) {
            e = hipStreamWaitEvent(fs[l], fork, 0);
            if (e == hipSuccess) e = hipStreamWaitEvent(es[l], fork, 0);
        }
        PhaseMarks none;
        for (int k = 0; k < n && e == hipSuccess; ++k) {
            const int l = items[k].lane;
            if (args[k].n == 0) {
                launch_empty(args[k], es[l]);
                continue;
            }
            (void)launch_front(args[k], fs[l], none);
            hipEvent_t ready = mkev();
            e = hipEventRecord(ready, fs[l]);
            if (e == hipSuccess) e = hipStreamWaitEvent(es[l], ready, 0);
            if (e == hipSuccess) launch_exec(args[k], es[l], none);
        }
        for (int l = 0; l < lanes && e == hipSuccess; ++l) {
            hipEvent_t j1 = mkev(), j2 = mkev();
            e = hipEventRecord(j1, fs[l]);
            if (e == hipSuccess) e = hipEventRecord(j2, es[l]);
            if (e == hipSuccess) e = hipStreamWaitEvent(origin, j1, 0);
            if (e == hipSuccess) e = hipStreamWaitEvent(origin, j2, 0);
        }
        if (e == hipSuccess) e = hipGetLastError();
        hipError_t e2 = hipStreamEndCapture(origin, &graph);
        if (e == hipSuccess) e = e2;
    }
    hipGraphExec_t ex = nullptr;
    if (e == hipSuccess) e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    cleanup();
    if (e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return gtx_set_err(h, GPUTX_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
    }
    gputx_batch b = new gputx_batch_t();
    b->h = h;
    b->graph = graph;
    b->exec = ex;
    b->items = n;
    b->lanes = lanes;
    *out = b;
    return GPUTX_OK;
}

extern "C" int gputx_batch_launch(gputx_batch b, gputx_stream_t stream) {
    if (!b) return gtx_set_err(nullptr, GPUTX_E_ARG, "null batch");
    HIP_OK(b->h, hipSetDevice(b->h->device));
    HIP_OK(b->h, hipGraphLaunch(b->exec, reinterpret_cast<hipStream_t>(stream)));
    return GPUTX_OK;
}

extern "C" int gputx_batch_destroy(gputx_batch b) {
    if (!b) return GPUTX_E_ARG;
    (void)hipSetDevice(b->h->device);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    delete b;
    return GPUTX_OK;
}

extern "C" int gputx_row_count(gputx_handle h, int32_t table_id, int64_t* out, gputx_stream_t stream) {
    if (!h || !out || table_id < 0 || table_id >= GPUTX_MAX_TABLES || !h->tabs[table_id].present)
        return gtx_set_err(h, GPUTX_E_ARG, "bad table");
    const auto& T = h->tabs[table_id];
    if (!T.d.append_only) {
        *out = T.d.n_rows;
        return GPUTX_OK;
    }
    HIP_OK(h, hipSetDevice(h->device));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIP_OK(h, hipMemcpyAsync(out, h->d_rowcount + T.app_idx, 8, hipMemcpyDeviceToHost, s));
    HIP_OK(h, hipStreamSynchronize(s));
    return GPUTX_OK;
}

extern "C" int gputx_set_row_count(gputx_handle h, int32_t table_id, int64_t n, gputx_stream_t stream) {
    if (!h || table_id < 0 || table_id >= GPUTX_MAX_TABLES || !h->tabs[table_id].present)
        return gtx_set_err(h, GPUTX_E_ARG, "bad table");
    const auto& T = h->tabs[table_id];
    if (!T.d.append_only || n < 0 || n > T.d.capacity)
        return gtx_set_err(h, GPUTX_E_ARG, "table %d: not append-only or %lld out of range", table_id, (long long)n);
    HIP_OK(h, hipSetDevice(h->device));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int64_t v = n;
    HIP_OK(h, hipMemcpyAsync(h->d_rowcount + T.app_idx, &v, 8, hipMemcpyHostToDevice, s));
    HIP_OK(h, hipStreamSynchronize(s));
    return GPUTX_OK;
}

extern "C" int gputx_read_table(gputx_handle h, int32_t table_id, int32_t col, int64_t row0, int64_t n,
                                void* host_dst, gputx_stream_t stream) {
    if (!h) return gtx_set_err(h, GPUTX_E_ARG, "null handle");
    if (table_id < 0 || table_id >= GPUTX_MAX_TABLES || !h->tabs[table_id].present)
        return gtx_set_err(h, GPUTX_E_ARG, "unknown table %d", table_id);
    const gputx_table_desc& d = h->tabs[table_id].d;
    if (col < 0 || col >= d.n_cols) return gtx_set_err(h, GPUTX_E_ARG, "table %d has no column %d", table_id, col);
    if (row0 < 0 || n < 0 || row0 + n > d.capacity || (n > 0 && !host_dst))
        return gtx_set_err(h, GPUTX_E_ARG, "rows [%lld, %lld) outside table %d's %lld rows", (long long)row0,
                           (long long)(row0 + n), table_id, (long long)d.capacity);
    if (n == 0) return GPUTX_OK;
    const size_t es = d.col_dtype[col] == GPUTX_I32 ? 4 : 8;
    HIP_OK(h, hipSetDevice(h->device));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIP_OK(h, hipMemcpyAsync(host_dst, (const char*)d.col_ptr[col] + (size_t)row0 * es, (size_t)n * es,
                             hipMemcpyDeviceToHost, s));
    HIP_OK(h, hipStreamSynchronize(s));
    return GPUTX_OK;
}

extern "C" const char* gputx_last_error(gputx_handle h) {
    if (!h) return g_err.c_str();
    return h->err.c_str();
}
