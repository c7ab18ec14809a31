// Compiled-in stored procedures and their basic operations.
//
// Section 3.2: every registered type is a device function and all of them
// form one kernel through a switch on the type.  Section 4.1: a transaction
// is a set of basic operations, each a read or a write of one data item;
// items here are table rows (a coarsening of the paper's field granularity
// that keeps every conflict, Appendix B), and a read-modify-write is one
// write.  Section 5.1: in root-key mode a type locks only the primary key of
// the root relation of its tree-shaped schema instead of every row.
#pragma once
#include "common.h"

namespace gtx {

// One registered type with its table bindings resolved (built on the host).
struct DevType {
    int32_t proc;       // GPUTX_* procedure, 0 = not registered
    int32_t n_params;
    int32_t n_results;
    int32_t root_key;
    int32_t app_idx[2];  // append-table index of the procedure's appends (-1: none)
    int32_t cell_class;  // types of different classes never name the same cell
    int32_t pad;
    int64_t dims[4];     // procedure dimensions (see type registration)
    int64_t rows[GTX_ROLES];        // rows of each bound (non-append) table
    int64_t root_div[GTX_ROLES];    // rows per root key
    int64_t part_base[GTX_ROLES];   // first global partition id of the role's root table
    int64_t part_size;              // root keys per partition
    uint32_t key_base[GTX_ROLES];   // first item key of the role's table
    uint32_t root_base[GTX_ROLES];  // first item key of the role's root table
    void* col[GTX_ROLES][GPUTX_MAX_COLS];
};

// Basic operations of one transaction: item key, write flag, partition id.
struct OpList {
    int n;
    uint32_t key[GTX_MAX_OPS];
    uint32_t w[GTX_MAX_OPS];
    int64_t pid[GTX_MAX_OPS];
};

__device__ __forceinline__ bool in_range(int64_t v, int64_t n) { return v >= 0 && v < n; }
__device__ __forceinline__ bool fits_i32(int64_t v) { return v >= INT32_MIN && v <= INT32_MAX; }
__device__ __forceinline__ int64_t wrap_add(int64_t a, int64_t b) {
    return (int64_t)((uint64_t)a + (uint64_t)b);
}
__device__ __forceinline__ int32_t to_i32(int64_t v) { return (int32_t)(uint32_t)(uint64_t)v; }

// Parameter validity; an invalid transaction has no effect (status INVALID).
__device__ inline bool txn_valid(const DevType& T, const int64_t* p) {
    switch (T.proc) {
    case GPUTX_DEBIT_CREDIT:
        return in_range(p[0], T.rows[0]) && in_range(p[1], T.rows[1]) && in_range(p[2], T.rows[2]);
    case GPUTX_NEW_ORDER:
    case GPUTX_NEW_ORDER_RB: {
        if (!(in_range(p[0], T.dims[0]) && in_range(p[1], T.dims[1]) && in_range(p[2], T.dims[2])))
            return false;
        int64_t k = p[3];
        if (k < 1 || k > 15) return false;
        // the rollback variant also takes the unused item id (== items per warehouse)
        const int64_t items = T.dims[3] + (T.proc == GPUTX_NEW_ORDER_RB ? 1 : 0);
        bool ok = true;
#pragma unroll
        for (int j = 0; j < 15; ++j)
            if (j < k) ok = ok && in_range(p[4 + j], items) && p[19 + j] >= 1 && p[19 + j] <= 1000;
        return ok;
    }
    case GPUTX_PAYMENT:
    case GPUTX_ORDER_STATUS:
        return in_range(p[0], T.dims[0]) && in_range(p[1], T.dims[1]) && in_range(p[2], T.dims[2]);
    case GPUTX_GET_SUB:
        return in_range(p[0], T.rows[0]);
    case GPUTX_GET_CF:
    case GPUTX_DEL_CF:
        return in_range(p[0], T.rows[0]) && in_range(p[1], 12);
    case GPUTX_UPD_SUB_FIELD:
        return in_range(p[0], T.rows[0]) && in_range(p[1], 4) && fits_i32(p[2]);
    case GPUTX_UPD_LOC:
        return in_range(p[0], T.rows[0]) && in_range(p[1], 10) && fits_i32(p[2]);
    case GPUTX_INS_CF:
        return in_range(p[0], T.rows[0]) && in_range(p[1], 12) && fits_i32(p[2]);
    }
    return false;
}

// A rollback new-order that names the unused item rolls back (and appends
// nothing); whether it does depends on its parameters alone.
__device__ __forceinline__ bool no_rb_rolls_back(const DevType& T, const int64_t* p) {
    bool rb = false;
#pragma unroll
    for (int j = 0; j < 15; ++j) rb = rb || (j < p[3] && p[4 + j] == T.dims[3]);
    return rb;
}

// Rows appended to the procedure's append tables (slot 0, slot 1).
__device__ __forceinline__ void txn_appends(const DevType& T, const int64_t* p, int* a0, int* a1) {
    *a0 = 0;
    *a1 = 0;
    if (T.proc == GPUTX_DEBIT_CREDIT) *a0 = 1;
    if (T.proc == GPUTX_NEW_ORDER) { *a0 = 1; *a1 = (int)p[3]; }
    if (T.proc == GPUTX_NEW_ORDER_RB && !no_rb_rolls_back(T, p)) { *a0 = 1; *a1 = (int)p[3]; }
}

__device__ __forceinline__ void op_add(OpList& L, const DevType& T, int role, int64_t row, bool w) {
    int64_t rk = row / T.root_div[role];
    uint32_t key = T.root_key ? T.root_base[role] + (uint32_t)rk : T.key_base[role] + (uint32_t)row;
    int64_t pid = T.part_base[role] < 0 ? -1 : T.part_base[role] + rk / T.part_size;
    // deduplicate: one operation per item, a write if any access writes
    bool found = false;
#pragma unroll
    for (int i = 0; i < GTX_MAX_OPS; ++i) {
        if (i < L.n && L.key[i] == key) {
            L.w[i] |= (uint32_t)w;
            found = true;
        }
    }
    if (found) return;
#pragma unroll
    for (int i = 0; i < GTX_MAX_OPS; ++i) {
        if (i == L.n) {
            L.key[i] = key;
            L.w[i] = (uint32_t)w;
            L.pid[i] = pid;
        }
    }
    L.n++;
}

// Basic operations of a valid transaction (Section 4.1), in procedure order.
__device__ inline void txn_ops(const DevType& T, const int64_t* p, OpList& L) {
    L.n = 0;
    switch (T.proc) {
    case GPUTX_DEBIT_CREDIT:
        op_add(L, T, 0, p[0], true);
        op_add(L, T, 1, p[1], true);
        op_add(L, T, 2, p[2], true);
        break;
    case GPUTX_NEW_ORDER:
    case GPUTX_NEW_ORDER_RB:  // the unused item has no row
#pragma unroll
        for (int j = 0; j < 15; ++j)
            if (j < p[3] && p[4 + j] < T.dims[3]) op_add(L, T, 3, p[0] * T.dims[3] + p[4 + j], true);
        break;
    case GPUTX_PAYMENT: {
        int64_t drow = p[0] * T.dims[1] + p[1];
        op_add(L, T, 0, p[0], true);
        op_add(L, T, 1, drow, true);
        op_add(L, T, 2, drow * T.dims[2] + p[2], true);
        break;
    }
    case GPUTX_ORDER_STATUS:
        op_add(L, T, 2, (p[0] * T.dims[1] + p[1]) * T.dims[2] + p[2], false);
        break;
    case GPUTX_GET_SUB:
        op_add(L, T, 0, p[0], false);
        break;
    case GPUTX_GET_CF:
        op_add(L, T, 1, p[0] * 12 + p[1], false);
        break;
    case GPUTX_UPD_SUB_FIELD:
    case GPUTX_UPD_LOC:
        op_add(L, T, 0, p[0], true);
        break;
    case GPUTX_INS_CF:
    case GPUTX_DEL_CF:
        op_add(L, T, 1, p[0] * 12 + p[1], true);
        break;
    }
}

// Parameters of transaction i (param-major bulk), zero past np.
__device__ __forceinline__ void load_params(const int64_t* __restrict__ params, int64_t n, int np,
                                            int64_t i, int64_t* p) {
#pragma unroll
    for (int k = 0; k < GTX_MAX_PARAMS; ++k) p[k] = (k < np) ? params[(int64_t)k * n + i] : 0;
}


// Table columns live in global memory: tag the pointers so that accesses
// compile to global_* rather than flat_* instructions.
#define GTX_GLOBAL __attribute__((address_space(1)))
template <class V>
__device__ __forceinline__ GTX_GLOBAL V* colp(const DevType& T, int role, int c) {
    return (GTX_GLOBAL V*)(T.col[role][c]);
}

// Every table cell (one column of one row, appended rows excluded) the
// transaction may read or write, passed as f.cell(ord, ptr, may_write) with
// the cell's value type.  ord numbers the procedure's cells; the procedure
// names each cell it touches by the same ordinal (acc.ref(ord, ptr) below).
// The set depends only on the parameters, and every cell lies in a row of
// the transaction's basic operations, so under PART (no cross-partition
// transaction) no two partitions share a cell.
// P != 0: the caller knows the procedure is P.
template <int P = 0, class F>
__device__ __forceinline__ void txn_cells(const DevType& T, const int64_t* p, F& f) {
    switch (P != 0 ? P : T.proc) {
    case GPUTX_DEBIT_CREDIT:
        f.cell(0, colp<int64_t>(T, 0, 0) + p[0], true);
        f.cell(1, colp<int64_t>(T, 1, 0) + p[1], true);
        f.cell(2, colp<int64_t>(T, 2, 0) + p[2], true);
        break;
    case GPUTX_NEW_ORDER:
    case GPUTX_NEW_ORDER_RB: {
        GTX_GLOBAL int32_t* S = colp<int32_t>(T, 3, 0) + p[0] * T.dims[3];
#pragma unroll
        for (int j = 0; j < 15; ++j)
            if (j < p[3] && p[4 + j] < T.dims[3]) f.cell(j, S + p[4 + j], true);
        break;
    }
    case GPUTX_PAYMENT: {
        int64_t drow = p[0] * T.dims[1] + p[1];
        f.cell(0, colp<int64_t>(T, 0, 0) + p[0], true);
        f.cell(1, colp<int64_t>(T, 1, 0) + drow, true);
        f.cell(2, colp<int64_t>(T, 2, 0) + (drow * T.dims[2] + p[2]), true);
        break;
    }
    case GPUTX_ORDER_STATUS:
        f.cell(0, colp<int64_t>(T, 2, 0) + ((p[0] * T.dims[1] + p[1]) * T.dims[2] + p[2]), false);
        break;
    case GPUTX_GET_SUB:
#pragma unroll
        for (int c = 0; c < 14; ++c) f.cell(c, colp<int32_t>(T, 0, 1 + c) + p[0], false);
        break;
    case GPUTX_UPD_SUB_FIELD:
    case GPUTX_UPD_LOC:
        f.cell(0, colp<int32_t>(T, 0, 1 + (int)p[1] + (T.proc == GPUTX_UPD_LOC ? 4 : 0)) + p[0], true);
        break;
    case GPUTX_GET_CF:
    case GPUTX_INS_CF:
    case GPUTX_DEL_CF: {
        const bool w = T.proc != GPUTX_GET_CF;
        int64_t slot = p[0] * 12 + p[1];
        f.cell(0, colp<int32_t>(T, 1, 0) + slot, w);
        f.cell(1, colp<int32_t>(T, 1, 1) + slot, w);
        f.cell(2, colp<int64_t>(T, 1, 2) + slot, w);
        break;
    }
    }
}

// Roles (bound tables) whose rows txn_cells names for procedure P.
__host__ __device__ constexpr uint32_t proc_cell_roles(int proc) {
    return (proc == GPUTX_DEBIT_CREDIT || proc == GPUTX_PAYMENT) ? 0x7u
         : (proc == GPUTX_NEW_ORDER || proc == GPUTX_NEW_ORDER_RB) ? 0x8u : proc == GPUTX_ORDER_STATUS ? 0x4u
         : (proc == GPUTX_GET_SUB || proc == GPUTX_UPD_SUB_FIELD || proc == GPUTX_UPD_LOC) ? 0x1u
         : (proc == GPUTX_GET_CF || proc == GPUTX_INS_CF || proc == GPUTX_DEL_CF) ? 0x2u : 0xffu;
}
// Most cells txn_cells lists for one transaction of procedure P (0: any).
__host__ __device__ constexpr int proc_cells(int proc) {
    return (proc == GPUTX_NEW_ORDER || proc == GPUTX_NEW_ORDER_RB) ? 15 : proc == GPUTX_GET_SUB ? 14
         : (proc == GPUTX_ORDER_STATUS || proc == GPUTX_UPD_SUB_FIELD || proc == GPUTX_UPD_LOC) ? 1
         : proc == 0 ? 15 : 3;
}

// Table-cell access used by the procedures.  acc.ref(ord, ptr) names one
// cell, ord being its ordinal in txn_cells (made after any earlier write to
// that cell by the same transaction); get/set read and write it; ld/st are
// one-shot forms; app writes a row appended to an append-only table.
// DirectAcc works on the columns in place.
struct DirectAcc {
    template <class V>
    struct Ref {
        GTX_GLOBAL V* p;
        __device__ __forceinline__ V get() const { return *p; }
        __device__ __forceinline__ void set(V v) const { *p = v; }
    };
    template <class V>
    __device__ __forceinline__ Ref<V> ref(int, GTX_GLOBAL V* p) { return Ref<V>{p}; }
    template <class V>
    __device__ __forceinline__ V ld(int, GTX_GLOBAL V* p) { return *p; }
    template <class V>
    __device__ __forceinline__ void st(int, GTX_GLOBAL V* p, V v) { *p = v; }
    template <class V>
    __device__ __forceinline__ void app(GTX_GLOBAL V* p, V v) { *p = v; }
};

// Table cells through agent-scope relaxed atomics, which the device keeps
// coherent across the XCDs' separate L2 caches load by load (they bypass the
// caches that are not coherent), so a hand-off needs neither a write-back nor
// an invalidation of a whole L2: the releasing side waits until its cell
// stores have completed, the acquiring side loads after it has seen the
// release.  Appended rows are plain stores: nothing reads them before the
// kernel ends.
struct CoherentAcc {
    template <class V>
    struct Ref {
        GTX_GLOBAL V* p;
        __device__ __forceinline__ V get() const {
            return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __device__ __forceinline__ void set(V v) const {
            __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    };
    template <class V>
    __device__ __forceinline__ Ref<V> ref(int, GTX_GLOBAL V* p) { return Ref<V>{p}; }
    template <class V>
    __device__ __forceinline__ V ld(int, GTX_GLOBAL V* p) {
        return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    template <class V>
    __device__ __forceinline__ void st(int, GTX_GLOBAL V* p, V v) {
        __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    template <class V>
    __device__ __forceinline__ void app(GTX_GLOBAL V* p, V v) { *p = v; }
};

// In every procedure below, whether and what a transaction appends depends
// only on its signature (appending procedures never abort, and appended
// values come from parameters and the timestamp).  So appends can be split
// from the rest of a transaction: AppendOnlyAcc performs only the appends
// (reads yield 0 and touch no memory), NoAppendAcc everything else.
struct AppendOnlyAcc {
    template <class V>
    struct Ref {
        __device__ __forceinline__ V get() const { return V(0); }
        __device__ __forceinline__ void set(V) const {}
    };
    template <class V>
    __device__ __forceinline__ Ref<V> ref(int, GTX_GLOBAL V*) { return Ref<V>{}; }
    template <class V>
    __device__ __forceinline__ V ld(int, GTX_GLOBAL V*) { return V(0); }
    template <class V>
    __device__ __forceinline__ void st(int, GTX_GLOBAL V*, V) {}
    template <class V>
    __device__ __forceinline__ void app(GTX_GLOBAL V* p, V v) { *p = v; }
};
struct NoAppendAcc : DirectAcc {
    template <class V>
    __device__ __forceinline__ void app(GTX_GLOBAL V*, V) {}
};

// Parameters procedure P reads (0: any procedure, the widest signature).
__host__ __device__ constexpr int proc_params(int proc) {
    return proc == GPUTX_DEBIT_CREDIT ? 4 : (proc == GPUTX_NEW_ORDER || proc == GPUTX_NEW_ORDER_RB) ? 34
         : proc == GPUTX_PAYMENT ? 4
         : proc == GPUTX_ORDER_STATUS ? 3 : proc == GPUTX_GET_SUB ? 1
         : (proc == GPUTX_GET_CF || proc == GPUTX_DEL_CF) ? 2
         : (proc == GPUTX_UPD_SUB_FIELD || proc == GPUTX_UPD_LOC) ? 3 : proc == GPUTX_INS_CF ? 4 : 34;
}
// Two transactions of procedure P can share a cell only at the same cell
// ordinal: each ordinal names one fixed column, or P has a single ordinal.
// Not so for new-order, whose item ordinals all name the stock column, nor
// for a mixed chunk (P == 0).
__host__ __device__ constexpr bool proc_typed_cells(int proc) {
    return proc != 0 && proc != GPUTX_NEW_ORDER && proc != GPUTX_NEW_ORDER_RB;
}
// Procedures whose effect on each of their cells depends only on that cell's
// old value and the parameters: no cell's value decides what happens to
// another, and each cell is named once.  Cell r's new value, whether it is
// written, and the result it yields can then be computed by lane r alone
// (cell_apply below restates these procedures of txn_exec_p per cell).
__host__ __device__ constexpr bool proc_cellwise(int proc) {
    return proc == GPUTX_DEBIT_CREDIT || proc == GPUTX_PAYMENT || proc == GPUTX_ORDER_STATUS ||
           proc == GPUTX_GET_SUB || proc == GPUTX_GET_CF || proc == GPUTX_UPD_SUB_FIELD ||
           proc == GPUTX_UPD_LOC;
}
// Cellwise procedures that write their cells.
__host__ __device__ constexpr bool proc_cell_writes(int proc) {
    return proc == GPUTX_DEBIT_CREDIT || proc == GPUTX_PAYMENT || proc == GPUTX_UPD_SUB_FIELD ||
           proc == GPUTX_UPD_LOC;
}
// Results procedure P can write (0: any procedure).
__host__ __device__ constexpr int proc_results(int proc) {
    return (proc == GPUTX_NEW_ORDER || proc == GPUTX_NEW_ORDER_RB) ? 16 : proc == GPUTX_GET_SUB ? 14
         : (proc == GPUTX_ORDER_STATUS || proc == GPUTX_UPD_SUB_FIELD || proc == GPUTX_UPD_LOC ||
            proc == GPUTX_INS_CF) ? 1
         : proc == 0 ? GTX_MAX_RESULTS : 3;
}
// Run one valid transaction of procedure P (one case of the switch of
// Section 3.2) through accessor acc.  app0/app1 are the rows its appends
// occupy.  Returns its status, fills res[0..15].
template <int P, class Acc>
__device__ __forceinline__ int32_t txn_exec_p(Acc& acc, const DevType& T, const int64_t* p, int64_t ts,
                                              int64_t app0, int64_t app1, int64_t* res) {
#pragma unroll
    for (int r = 0; r < GTX_MAX_RESULTS; ++r) res[r] = 0;
    switch (P) {
    case GPUTX_DEBIT_CREDIT: {
        auto A = acc.ref(0, colp<int64_t>(T, 0, 0) + p[0]);
        auto Tl = acc.ref(1, colp<int64_t>(T, 1, 0) + p[1]);
        auto B = acc.ref(2, colp<int64_t>(T, 2, 0) + p[2]);
        int64_t a = wrap_add(A.get(), p[3]);
        int64_t t = wrap_add(Tl.get(), p[3]);
        int64_t b = wrap_add(B.get(), p[3]);
        A.set(a);
        Tl.set(t);
        B.set(b);
        acc.app(colp<int64_t>(T, 3, 0) + app0, p[0]);
        acc.app(colp<int64_t>(T, 3, 1) + app0, p[1]);
        acc.app(colp<int64_t>(T, 3, 2) + app0, p[2]);
        acc.app(colp<int64_t>(T, 3, 3) + app0, p[3]);
        acc.app(colp<int64_t>(T, 3, 4) + app0, ts);
        res[0] = a;
        res[1] = t;
        res[2] = b;
        return GPUTX_COMMIT;
    }
    case GPUTX_NEW_ORDER: {
        int64_t k = p[3];
        res[0] = k;
#pragma unroll
        for (int j = 0; j < 15; ++j) {
            if (j < k) {
                auto S = acc.ref(j, colp<int32_t>(T, 3, 0) + (p[0] * T.dims[3] + p[4 + j]));
                int64_t s = (int64_t)S.get() - p[19 + j];
                if (s < 10) s += 91;
                int32_t s32 = to_i32(s);
                S.set(s32);
                res[1 + j] = s32;
                int64_t r = app1 + j;
                acc.app(colp<int64_t>(T, 5, 0) + r, ts);
                acc.app(colp<int64_t>(T, 5, 1) + r, (int64_t)j);
                acc.app(colp<int64_t>(T, 5, 2) + r, p[4 + j]);
                acc.app(colp<int64_t>(T, 5, 3) + r, p[19 + j]);
                acc.app(colp<int64_t>(T, 5, 4) + r, p[0]);
            }
        }
        acc.app(colp<int64_t>(T, 4, 0) + app0, ts);
        acc.app(colp<int64_t>(T, 4, 1) + app0, p[0]);
        acc.app(colp<int64_t>(T, 4, 2) + app0, p[1]);
        acc.app(colp<int64_t>(T, 4, 3) + app0, p[2]);
        acc.app(colp<int64_t>(T, 4, 4) + app0, k);
        return GPUTX_COMMIT;
    }
    case GPUTX_NEW_ORDER_RB: {
        // Not two-phase: each stock row is updated as its item is reached,
        // with the old value written to the transaction's undo log first; on
        // reaching the unused item the log is replayed backwards and the
        // transaction aborts.  Nothing else can see the rows meanwhile (the
        // executors hand a row on only after the transaction is over), so the
        // rollback touches this transaction alone.
        int64_t k = p[3];
        int32_t undo[15];
        GTX_GLOBAL int32_t* S0 = colp<int32_t>(T, 3, 0) + p[0] * T.dims[3];
#pragma unroll
        for (int j = 0; j < 15; ++j) {
            if (j < k) {
                if (p[4 + j] == T.dims[3]) {
#pragma unroll
                    for (int q = j - 1; q >= 0; --q) acc.ref(q, S0 + p[4 + q]).set(undo[q]);
#pragma unroll
                    for (int r = 0; r < GTX_MAX_RESULTS; ++r) res[r] = 0;
                    return GPUTX_ABORT;
                }
                auto S = acc.ref(j, S0 + p[4 + j]);
                const int32_t old = S.get();
                undo[j] = old;
                int64_t s = (int64_t)old - p[19 + j];
                if (s < 10) s += 91;
                int32_t s32 = to_i32(s);
                S.set(s32);
                res[1 + j] = s32;
            }
        }
        res[0] = k;
#pragma unroll
        for (int j = 0; j < 15; ++j) {
            if (j < k) {
                int64_t r = app1 + j;
                acc.app(colp<int64_t>(T, 5, 0) + r, ts);
                acc.app(colp<int64_t>(T, 5, 1) + r, (int64_t)j);
                acc.app(colp<int64_t>(T, 5, 2) + r, p[4 + j]);
                acc.app(colp<int64_t>(T, 5, 3) + r, p[19 + j]);
                acc.app(colp<int64_t>(T, 5, 4) + r, p[0]);
            }
        }
        acc.app(colp<int64_t>(T, 4, 0) + app0, ts);
        acc.app(colp<int64_t>(T, 4, 1) + app0, p[0]);
        acc.app(colp<int64_t>(T, 4, 2) + app0, p[1]);
        acc.app(colp<int64_t>(T, 4, 3) + app0, p[2]);
        acc.app(colp<int64_t>(T, 4, 4) + app0, k);
        return GPUTX_COMMIT;
    }
    case GPUTX_PAYMENT: {
        int64_t drow = p[0] * T.dims[1] + p[1];
        int64_t crow = drow * T.dims[2] + p[2];
        auto Wb = acc.ref(0, colp<int64_t>(T, 0, 0) + p[0]);
        auto Db = acc.ref(1, colp<int64_t>(T, 1, 0) + drow);
        auto Cb = acc.ref(2, colp<int64_t>(T, 2, 0) + crow);
        int64_t w = wrap_add(Wb.get(), p[3]);
        int64_t d = wrap_add(Db.get(), p[3]);
        int64_t c = wrap_add(Cb.get(), p[3]);
        Wb.set(w);
        Db.set(d);
        Cb.set(c);
        res[0] = w;
        res[1] = d;
        res[2] = c;
        return GPUTX_COMMIT;
    }
    case GPUTX_ORDER_STATUS: {
        int64_t crow = (p[0] * T.dims[1] + p[1]) * T.dims[2] + p[2];
        res[0] = acc.ld(0, colp<int64_t>(T, 2, 0) + crow);
        return GPUTX_COMMIT;
    }
    case GPUTX_GET_SUB: {
#pragma unroll
        for (int f = 0; f < 14; ++f) res[f] = acc.ld(f, colp<int32_t>(T, 0, 1 + f) + p[0]);
        return GPUTX_COMMIT;
    }
    case GPUTX_GET_CF: {
        int64_t slot = p[0] * 12 + p[1];
        res[0] = acc.ld(0, colp<int32_t>(T, 1, 0) + slot);
        res[1] = acc.ld(1, colp<int32_t>(T, 1, 1) + slot);
        res[2] = acc.ld(2, colp<int64_t>(T, 1, 2) + slot);
        return GPUTX_COMMIT;
    }
    case GPUTX_UPD_SUB_FIELD:
    case GPUTX_UPD_LOC: {
        int c = 1 + (int)p[1] + (P == GPUTX_UPD_LOC ? 4 : 0);
        auto F = acc.ref(0, colp<int32_t>(T, 0, c) + p[0]);
        res[0] = F.get();
        F.set(to_i32(p[2]));
        return GPUTX_COMMIT;
    }
    case GPUTX_INS_CF: {
        int64_t slot = p[0] * 12 + p[1];
        auto occ = acc.ref(0, colp<int32_t>(T, 1, 0) + slot);
        int32_t o = occ.get();
        res[0] = o;
        if (o) return GPUTX_ABORT;  // read phase decides; nothing written
        occ.set((int32_t)1);
        acc.st(1, colp<int32_t>(T, 1, 1) + slot, to_i32(p[2]));
        acc.st(2, colp<int64_t>(T, 1, 2) + slot, p[3]);
        return GPUTX_COMMIT;
    }
    case GPUTX_DEL_CF: {
        int64_t slot = p[0] * 12 + p[1];
        auto occ = acc.ref(0, colp<int32_t>(T, 1, 0) + slot);
        if (!occ.get()) return GPUTX_ABORT;
        auto num = acc.ref(1, colp<int32_t>(T, 1, 1) + slot);
        auto end = acc.ref(2, colp<int64_t>(T, 1, 2) + slot);
        res[0] = 1;
        res[1] = num.get();
        res[2] = end.get();
        occ.set((int32_t)0);
        num.set((int32_t)0);
        end.set((int64_t)0);
        return GPUTX_COMMIT;
    }
    }
    return GPUTX_INVALID;
}

// The same per-cell effect as a map of the cell's old value,
// v -> a ? v + b : b (wrapping add): cell_apply's new value for every old
// value.  Two such maps compose into one of the same form.
template <int P>
__device__ __forceinline__ void cell_affine(int r, const int64_t* p, bool& a, int64_t& b) {
    static_assert(proc_cellwise(P), "cell_affine: procedure is not cellwise");
    (void)r;
    switch (P) {
    case GPUTX_DEBIT_CREDIT:
    case GPUTX_PAYMENT:
        a = true;
        b = p[3];
        break;
    case GPUTX_ORDER_STATUS:
    case GPUTX_GET_SUB:
    case GPUTX_GET_CF:
        a = true;
        b = 0;
        break;
    case GPUTX_UPD_SUB_FIELD:
    case GPUTX_UPD_LOC:
        a = false;
        b = (int64_t)to_i32(p[2]);
        break;
    }
}

// Cell r of a cellwise procedure P (proc_cellwise), with old value old (an
// int32 cell sign-extended): its new value nv, whether it is written, and
// result res at index res_at (-1: none).  Every cellwise procedure commits.
template <int P>
__device__ __forceinline__ void cell_apply(int r, int64_t old, const int64_t* p, int64_t& nv, bool& w,
                                           int& res_at, int64_t& res) {
    static_assert(proc_cellwise(P), "cell_apply: procedure is not cellwise");
    switch (P) {
    case GPUTX_DEBIT_CREDIT:  // account, teller, branch balance += delta; results: the new balances
    case GPUTX_PAYMENT:       // warehouse, district, customer balance += h; results: the new balances
        nv = wrap_add(old, p[3]);
        w = true;
        res_at = r;
        res = nv;
        break;
    case GPUTX_ORDER_STATUS:  // read the customer balance
        nv = old;
        w = false;
        res_at = 0;
        res = old;
        break;
    case GPUTX_GET_SUB:  // read every field of the subscriber row
    case GPUTX_GET_CF:   // read the call-forwarding slot
        nv = old;
        w = false;
        res_at = r;
        res = old;
        break;
    case GPUTX_UPD_SUB_FIELD:  // result: the old field value; the field becomes p[2]
    case GPUTX_UPD_LOC:
        nv = (int64_t)to_i32(p[2]);
        w = true;
        res_at = 0;
        res = old;
        break;
    }
}

// The combined kernel's switch on the procedure (Section 3.2), any accessor.
template <class Acc>
__device__ __forceinline__ int32_t txn_exec_any(Acc& acc, const DevType& T, const int64_t* p, int64_t ts,
                                       int64_t app0, int64_t app1, int64_t* res) {
    switch (T.proc) {
    case GPUTX_DEBIT_CREDIT: return txn_exec_p<GPUTX_DEBIT_CREDIT>(acc, T, p, ts, app0, app1, res);
    case GPUTX_NEW_ORDER: return txn_exec_p<GPUTX_NEW_ORDER>(acc, T, p, ts, app0, app1, res);
    case GPUTX_NEW_ORDER_RB: return txn_exec_p<GPUTX_NEW_ORDER_RB>(acc, T, p, ts, app0, app1, res);
    case GPUTX_PAYMENT: return txn_exec_p<GPUTX_PAYMENT>(acc, T, p, ts, app0, app1, res);
    case GPUTX_ORDER_STATUS: return txn_exec_p<GPUTX_ORDER_STATUS>(acc, T, p, ts, app0, app1, res);
    case GPUTX_GET_SUB: return txn_exec_p<GPUTX_GET_SUB>(acc, T, p, ts, app0, app1, res);
    case GPUTX_GET_CF: return txn_exec_p<GPUTX_GET_CF>(acc, T, p, ts, app0, app1, res);
    case GPUTX_UPD_SUB_FIELD: return txn_exec_p<GPUTX_UPD_SUB_FIELD>(acc, T, p, ts, app0, app1, res);
    case GPUTX_UPD_LOC: return txn_exec_p<GPUTX_UPD_LOC>(acc, T, p, ts, app0, app1, res);
    case GPUTX_INS_CF: return txn_exec_p<GPUTX_INS_CF>(acc, T, p, ts, app0, app1, res);
    case GPUTX_DEL_CF: return txn_exec_p<GPUTX_DEL_CF>(acc, T, p, ts, app0, app1, res);
    }
    for (int r = 0; r < GTX_MAX_RESULTS; ++r) res[r] = 0;
    return GPUTX_INVALID;
}

__device__ inline int32_t txn_exec(const DevType& T, const int64_t* p, int64_t ts, int64_t app0,
                                   int64_t app1, int64_t* res) {
    DirectAcc acc;
    return txn_exec_any(acc, T, p, ts, app0, app1, res);
}


}  // namespace gtx
