/*
 * Serial oracle for bulk transaction execution.  TEST INFRASTRUCTURE ONLY:
 * tests, the smoke check and the benchmark's CPU baseline call it; the GPU
 * engine never does.  It shares no code with the engine.
 *
 * Definition 1 (Section 3.1): a bulk execution is correct iff the resulting
 * database equals executing the bulk's transactions one by one in increasing
 * timestamp order.  This file is that definition written out:
 *   1. timestamps must be unique (the id of a signature <id, type, params>
 *      is unique and serves as timestamp, Section 3.2) -> else ORC_E_DUP_TS;
 *   2. order the transactions by timestamp;
 *   3. run each one's stored procedure (Section 3.1) on the host tables;
 *   4. appended rows land in that order (insert buffer + batched update,
 *      Section 3.2);
 *   5. per-transaction status and results go to the caller's result arrays
 *      at the transaction's input index (result pool, Section 3.2).
 * Integer arithmetic wraps modulo 2^64 (done in uint64) so that no input is
 * undefined behaviour.  A transaction whose parameters name a row outside its
 * table, or whose type is unregistered, is INVALID and has no effect.
 * Two-phase transactions (Appendix D) may ABORT after their read phase and
 * then write nothing.
 */
#include "oracle.h"

#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t ts;
    int64_t idx;
} orc_key;

static int cmp_key(const void* a, const void* b) {
    const orc_key* x = (const orc_key*)a;
    const orc_key* y = (const orc_key*)b;
    if (x->ts != y->ts) return x->ts < y->ts ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

#define I64(t, c) ((int64_t*)(t)->col[(c)])
#define I32(t, c) ((int32_t*)(t)->col[(c)])

static int64_t wrap_add(int64_t a, int64_t b) { return (int64_t)((uint64_t)a + (uint64_t)b); }
static int32_t to_i32(int64_t v) { return (int32_t)(uint32_t)(uint64_t)v; }
static int in_range(int64_t v, int64_t n) { return v >= 0 && v < n; }
static int fits_i32(int64_t v) { return v >= INT32_MIN && v <= INT32_MAX; }

/* Order-entry dimensions derived from the table sizes. */
typedef struct { int64_t nw, dpw, cpd, ipw; } orc_odims;

static int order_dims(const orc_table* R, orc_odims* d) {
    const orc_table *w = &R[ORC_R_WAREHOUSE], *di = &R[ORC_R_DISTRICT],
                    *c = &R[ORC_R_CUSTOMER], *s = &R[ORC_R_STOCK];
    if (w->n_rows <= 0 || di->n_rows <= 0) return 0;
    d->nw = w->n_rows;
    d->dpw = di->n_rows / w->n_rows;
    d->cpd = c->n_rows / di->n_rows;
    d->ipw = s->n_rows / w->n_rows;
    return 1;
}

/* A new-order that is not two-phase (Appendix D) rolls back when one of its
 * items is the unused item id; a rolled-back transaction has no effect. */
static int names_unused_item(const int64_t* p, const orc_table* R) {
    orc_odims od = {0, 0, 0, 0};
    if (!order_dims(R, &od)) return 0;
    for (int64_t j = 0; j < p[3] && j < ORC_NO_MAX_ITEMS; ++j)
        if (p[4 + j] == od.ipw) return 1;   /* the unused item id */
    return 0;
}

/* Number of rows a valid transaction appends to history / orders / order_line. */
void orc_appends_of(int proc, const int64_t* p, const orc_table* R, int64_t* h, int64_t* o, int64_t* ol) {
    *h = *o = *ol = 0;
    if (proc == ORC_DEBIT_CREDIT) *h = 1;
    if (proc == ORC_NEW_ORDER) { *o = 1; *ol = p[3]; }
    if (proc == ORC_NEW_ORDER_RB && !names_unused_item(p, R)) { *o = 1; *ol = p[3]; }
}

/* Parameter validity (INVALID otherwise). */
int orc_is_valid(int proc, const int64_t* p, const orc_table* R) {
    orc_odims od = {0, 0, 0, 0};
    switch (proc) {
    case ORC_DEBIT_CREDIT:
        return in_range(p[0], R[ORC_R_ACCOUNT].n_rows) && in_range(p[1], R[ORC_R_TELLER].n_rows) &&
               in_range(p[2], R[ORC_R_BRANCH].n_rows);
    case ORC_NEW_ORDER:
    case ORC_NEW_ORDER_RB:
        if (!order_dims(R, &od)) return 0;
        if (!(in_range(p[0], od.nw) && in_range(p[1], od.dpw) && in_range(p[2], od.cpd))) return 0;
        if (p[3] < 1 || p[3] > ORC_NO_MAX_ITEMS) return 0;
        for (int64_t j = 0; j < p[3]; ++j) {
            /* the rollback variant also names the unused item id ipw */
            if (!in_range(p[4 + j], od.ipw + (proc == ORC_NEW_ORDER_RB))) return 0;
            if (p[4 + ORC_NO_MAX_ITEMS + j] < 1 || p[4 + ORC_NO_MAX_ITEMS + j] > 1000) return 0;
        }
        return 1;
    case ORC_PAYMENT:
    case ORC_ORDER_STATUS:
        if (!order_dims(R, &od)) return 0;
        return in_range(p[0], od.nw) && in_range(p[1], od.dpw) && in_range(p[2], od.cpd);
    case ORC_GET_SUB:
        return in_range(p[0], R[ORC_R_SUBSCRIBER].n_rows);
    case ORC_GET_CF:
    case ORC_DEL_CF:
        return in_range(p[0], R[ORC_R_SUBSCRIBER].n_rows) && in_range(p[1], ORC_CF_SLOTS);
    case ORC_UPD_SUB_FIELD:
        return in_range(p[0], R[ORC_R_SUBSCRIBER].n_rows) && in_range(p[1], ORC_SUB_FIELDS) &&
               fits_i32(p[2]);
    case ORC_UPD_LOC:
        return in_range(p[0], R[ORC_R_SUBSCRIBER].n_rows) && in_range(p[1], ORC_SUB_LOCS) &&
               fits_i32(p[2]);
    case ORC_INS_CF:
        return in_range(p[0], R[ORC_R_SUBSCRIBER].n_rows) && in_range(p[1], ORC_CF_SLOTS) &&
               fits_i32(p[2]);
    default:
        return 0;
    }
}

/* Run one valid transaction; returns its status, writes its results. */
int32_t orc_run_one(int proc, const int64_t* p, int64_t ts, orc_table* R, int64_t* res) {
    orc_odims od = {0, 0, 0, 0};
    switch (proc) {
    case ORC_DEBIT_CREDIT: {
        int64_t* A = I64(&R[ORC_R_ACCOUNT], 0);
        int64_t* T = I64(&R[ORC_R_TELLER], 0);
        int64_t* B = I64(&R[ORC_R_BRANCH], 0);
        A[p[0]] = wrap_add(A[p[0]], p[3]);
        T[p[1]] = wrap_add(T[p[1]], p[3]);
        B[p[2]] = wrap_add(B[p[2]], p[3]);
        orc_table* H = &R[ORC_R_HISTORY];
        int64_t r = H->n_rows++;
        I64(H, 0)[r] = p[0];
        I64(H, 1)[r] = p[1];
        I64(H, 2)[r] = p[2];
        I64(H, 3)[r] = p[3];
        I64(H, 4)[r] = ts;
        res[0] = A[p[0]];
        res[1] = T[p[1]];
        res[2] = B[p[2]];
        return ORC_COMMIT;
    }
    case ORC_NEW_ORDER_RB:
        /* rolls back when it names the unused item: no effect at all */
        if (names_unused_item(p, R)) return ORC_ABORT;
        /* otherwise exactly a new-order */
        __attribute__((fallthrough));
    case ORC_NEW_ORDER: {
        order_dims(R, &od);
        int32_t* S = I32(&R[ORC_R_STOCK], 0);
        int64_t k = p[3];
        res[0] = k;
        orc_table* O = &R[ORC_R_ORDERS];
        orc_table* L = &R[ORC_R_ORDER_LINE];
        for (int64_t j = 0; j < k; ++j) {
            int64_t item = p[4 + j], q = p[4 + ORC_NO_MAX_ITEMS + j];
            int64_t row = p[0] * od.ipw + item;
            int64_t s = (int64_t)S[row] - q;
            if (s < 10) s += 91;
            S[row] = to_i32(s);
            res[1 + j] = S[row];
            int64_t r = L->n_rows++;
            I64(L, 0)[r] = ts;
            I64(L, 1)[r] = j;
            I64(L, 2)[r] = item;
            I64(L, 3)[r] = q;
            I64(L, 4)[r] = p[0];
        }
        int64_t r = O->n_rows++;
        I64(O, 0)[r] = ts;
        I64(O, 1)[r] = p[0];
        I64(O, 2)[r] = p[1];
        I64(O, 3)[r] = p[2];
        I64(O, 4)[r] = k;
        return ORC_COMMIT;
    }
    case ORC_PAYMENT: {
        order_dims(R, &od);
        int64_t* Wb = I64(&R[ORC_R_WAREHOUSE], 0);
        int64_t* Db = I64(&R[ORC_R_DISTRICT], 0);
        int64_t* Cb = I64(&R[ORC_R_CUSTOMER], 0);
        int64_t drow = p[0] * od.dpw + p[1];
        int64_t crow = drow * od.cpd + p[2];
        Wb[p[0]] = wrap_add(Wb[p[0]], p[3]);
        Db[drow] = wrap_add(Db[drow], p[3]);
        Cb[crow] = wrap_add(Cb[crow], p[3]);
        res[0] = Wb[p[0]];
        res[1] = Db[drow];
        res[2] = Cb[crow];
        return ORC_COMMIT;
    }
    case ORC_ORDER_STATUS: {
        order_dims(R, &od);
        int64_t crow = (p[0] * od.dpw + p[1]) * od.cpd + p[2];
        res[0] = I64(&R[ORC_R_CUSTOMER], 0)[crow];
        return ORC_COMMIT;
    }
    case ORC_GET_SUB: {
        orc_table* S = &R[ORC_R_SUBSCRIBER];
        for (int f = 0; f < ORC_SUB_FIELDS + ORC_SUB_LOCS; ++f) res[f] = I32(S, 1 + f)[p[0]];
        return ORC_COMMIT;
    }
    case ORC_GET_CF: {
        orc_table* C = &R[ORC_R_CALL_FWD];
        int64_t slot = p[0] * ORC_CF_SLOTS + p[1];
        res[0] = I32(C, 0)[slot];
        res[1] = I32(C, 1)[slot];
        res[2] = I64(C, 2)[slot];
        return ORC_COMMIT;
    }
    case ORC_UPD_SUB_FIELD: {
        int32_t* F = I32(&R[ORC_R_SUBSCRIBER], 1 + p[1]);
        res[0] = F[p[0]];
        F[p[0]] = to_i32(p[2]);
        return ORC_COMMIT;
    }
    case ORC_UPD_LOC: {
        int32_t* F = I32(&R[ORC_R_SUBSCRIBER], 1 + ORC_SUB_FIELDS + p[1]);
        res[0] = F[p[0]];
        F[p[0]] = to_i32(p[2]);
        return ORC_COMMIT;
    }
    case ORC_INS_CF: {
        orc_table* C = &R[ORC_R_CALL_FWD];
        int64_t slot = p[0] * ORC_CF_SLOTS + p[1];
        res[0] = I32(C, 0)[slot];
        if (I32(C, 0)[slot]) return ORC_ABORT;     /* read phase decides */
        I32(C, 0)[slot] = 1;
        I32(C, 1)[slot] = to_i32(p[2]);
        I64(C, 2)[slot] = p[3];
        return ORC_COMMIT;
    }
    case ORC_DEL_CF: {
        orc_table* C = &R[ORC_R_CALL_FWD];
        int64_t slot = p[0] * ORC_CF_SLOTS + p[1];
        if (!I32(C, 0)[slot]) return ORC_ABORT;
        res[0] = 1;
        res[1] = I32(C, 1)[slot];
        res[2] = I64(C, 2)[slot];
        I32(C, 0)[slot] = 0;
        I32(C, 1)[slot] = 0;
        I64(C, 2)[slot] = 0;
        return ORC_COMMIT;
    }
    }
    return ORC_INVALID;
}

int orc_execute(int64_t n, const int32_t* type, const int64_t* params, int32_t n_params,
                const int64_t* ts, const int32_t* proc_of_type, int32_t n_types,
                orc_table* tables, int32_t* status, int64_t* results, int32_t width) {
    if (n < 0 || n_params < 1 || width < 1) return ORC_E_ARG;
    if (n == 0) return ORC_OK;
    orc_key* order = (orc_key*)malloc(sizeof(orc_key) * (size_t)n);
    int64_t* p = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_params > 64 ? n_params : 64));
    unsigned char* ok = (unsigned char*)malloc((size_t)n);
    if (!order || !p || !ok) { free(order); free(p); free(ok); return ORC_E_ARG; }
    for (int64_t i = 0; i < n; ++i) { order[i].ts = ts[i]; order[i].idx = i; }
    qsort(order, (size_t)n, sizeof(orc_key), cmp_key);
    for (int64_t i = 1; i < n; ++i)
        if (order[i].ts == order[i - 1].ts) { free(order); free(p); free(ok); return ORC_E_DUP_TS; }

    /* validity and append capacity, before any mutation */
    int64_t need_h = 0, need_o = 0, need_ol = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t t = type[i];
        int proc = (t >= 0 && t < n_types) ? proc_of_type[t] : 0;
        memset(p, 0, sizeof(int64_t) * 64);
        for (int32_t k = 0; k < n_params; ++k) p[k] = params[(int64_t)k * n + i];
        ok[i] = (unsigned char)(proc > 0 && orc_is_valid(proc, p, tables));
        if (ok[i]) {
            int64_t h, o, ol;
            orc_appends_of(proc, p, tables, &h, &o, &ol);
            need_h += h; need_o += o; need_ol += ol;
        }
    }
    if ((need_h && tables[ORC_R_HISTORY].n_rows + need_h > tables[ORC_R_HISTORY].capacity) ||
        (need_o && tables[ORC_R_ORDERS].n_rows + need_o > tables[ORC_R_ORDERS].capacity) ||
        (need_ol && tables[ORC_R_ORDER_LINE].n_rows + need_ol > tables[ORC_R_ORDER_LINE].capacity)) {
        free(order); free(p); free(ok);
        return ORC_E_CAPACITY;
    }

    for (int64_t s = 0; s < n; ++s) {
        int64_t i = order[s].idx;
        int64_t* res = results + i * (int64_t)width;
        for (int32_t w = 0; w < width; ++w) res[w] = 0;
        if (!ok[i]) { status[i] = ORC_INVALID; continue; }
        int proc = proc_of_type[type[i]];
        memset(p, 0, sizeof(int64_t) * 64);
        for (int32_t k = 0; k < n_params; ++k) p[k] = params[(int64_t)k * n + i];
        int64_t tmp[64];
        memset(tmp, 0, sizeof(tmp));
        status[i] = orc_run_one(proc, p, ts[i], tables, tmp);
        for (int32_t w = 0; w < width && w < 64; ++w) res[w] = tmp[w];
    }
    free(order); free(p); free(ok);
    return ORC_OK;
}
