/*
 * The paper's CPU counterpart, timed as a baseline beside the GPU engine.
 * TEST AND BENCHMARK INFRASTRUCTURE ONLY; the GPU engine never calls it.
 *
 * Section 6.3 compares GPUTx with an H-Store-like executor on the host's
 * cores: the database is split into partitions, every partition is served by
 * one worker that runs its transactions one after another, and a transaction
 * that spans partitions is run with the others held back.  Here:
 *   1. timestamps must be unique; transactions are taken in timestamp order
 *      (no sort when the input is already ascending);
 *   2. validity and the rows each valid transaction appends are settled
 *      first (each worker takes a contiguous share of timestamp order), and
 *      a timestamp-order scan gives every transaction the slots of its
 *      appended rows (so appends land exactly where the serial run puts
 *      them);
 *   3. transactions are routed: one whose rows all lie in partition p goes
 *      to worker p % n_threads, in timestamp order;
 *   4. the workers run their queues up to the next transaction that spans
 *      partitions, meet at a barrier, the first worker runs that one alone,
 *      and they meet again before going on.
 * Rows of different partitions are disjoint, so every worker's reads and
 * writes are its own between barriers and the outcome equals the serial
 * execution of Definition 1 (Section 3.1) exactly.
 */
#define _POSIX_C_SOURCE 200809L
#include "oracle.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t ts;
    int64_t idx;
} pt_key;

static int pt_cmp(const void* a, const void* b) {
    const pt_key* x = (const pt_key*)a;
    const pt_key* y = (const pt_key*)b;
    if (x->ts != y->ts) return x->ts < y->ts ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

typedef struct {
    int64_t n;
    const int32_t* type;
    const int64_t* params;
    int32_t n_params;
    const int64_t* ts;
    const int32_t* proc_of_type;
    int32_t n_types;
    const orc_table* tables;
    const int64_t* order;     /* serial position -> input index */
    const int64_t* part;
    unsigned char* ok;        /* valid transaction */
    int64_t* slot;            /* [3][n]: history, orders, order_line row of txn i */
    int64_t* chunk_sum;       /* [3][n_threads + 1]: appends per chunk, then offsets */
    int32_t n_threads;
    int32_t* status;
    int64_t* results;
    int32_t width;
    int capacity_error;
    pthread_barrier_t bar;
    pthread_mutex_t mu;       /* start gate: workers wait until every one exists */
    pthread_cond_t cv;
    int go, abort;
} pt_job;

typedef struct {
    pt_job* job;
    int32_t w;
} pt_arg;

static void load_params(const pt_job* J, int64_t i, int64_t* p) {
    int32_t k = 0;
    for (; k < J->n_params && k < 64; ++k) p[k] = J->params[(int64_t)k * J->n + i];
    for (; k < 40; ++k) p[k] = 0;
}

static int proc_of(const pt_job* J, int64_t i) {
    const int32_t t = J->type[i];
    return (t >= 0 && t < J->n_types) ? J->proc_of_type[t] : 0;
}

static void pt_run(const pt_job* J, orc_table* R, int64_t i) {
    int64_t* res = J->results + i * (int64_t)J->width;
    for (int32_t c = 0; c < J->width; ++c) res[c] = 0;
    if (!J->ok[i]) {
        J->status[i] = ORC_INVALID;
        return;
    }
    int64_t p[64];
    load_params(J, i, p);
    /* the appends of this transaction go to its pre-scanned slots */
    R[ORC_R_HISTORY].n_rows = J->slot[i];
    R[ORC_R_ORDERS].n_rows = J->slot[J->n + i];
    R[ORC_R_ORDER_LINE].n_rows = J->slot[2 * J->n + i];
    int64_t tmp[64];
    memset(tmp, 0, sizeof(int64_t) * 16);
    J->status[i] = orc_run_one(proc_of(J, i), p, J->ts[i], R, tmp);
    for (int32_t c = 0; c < J->width && c < 16; ++c) res[c] = tmp[c];
}

static void* pt_worker(void* arg) {
    pt_arg* A = (pt_arg*)arg;
    pt_job* J = A->job;
    pthread_mutex_lock(&J->mu);
    while (!J->go) pthread_cond_wait(&J->cv, &J->mu);
    const int abort = J->abort;
    pthread_mutex_unlock(&J->mu);
    if (abort) return NULL;
    const int64_t n = J->n, T = J->n_threads, w = A->w;
    /* validity and append counts of this worker's chunk of serial positions */
    const int64_t s0 = n * w / T, s1 = n * (w + 1) / T;
    int64_t sum[3] = {0, 0, 0};
    for (int64_t s = s0; s < s1; ++s) {
        const int64_t i = J->order[s];
        const int proc = proc_of(J, i);
        int64_t p[64];
        load_params(J, i, p);
        J->ok[i] = (unsigned char)(proc > 0 && orc_is_valid(proc, p, J->tables));
        int64_t h = 0, o = 0, l = 0;
        if (J->ok[i]) orc_appends_of(proc, p, J->tables, &h, &o, &l);
        J->slot[i] = h;
        J->slot[n + i] = o;
        J->slot[2 * n + i] = l;
        sum[0] += h; sum[1] += o; sum[2] += l;
    }
    for (int k = 0; k < 3; ++k) J->chunk_sum[k * (T + 1) + w + 1] = sum[k];
    pthread_barrier_wait(&J->bar);
    if (w == 0) {  /* chunk offsets; capacity */
        const int role[3] = {ORC_R_HISTORY, ORC_R_ORDERS, ORC_R_ORDER_LINE};
        for (int k = 0; k < 3; ++k) {
            int64_t* cs = J->chunk_sum + k * (T + 1);
            cs[0] = J->tables[role[k]].n_rows;
            for (int64_t c = 0; c < T; ++c) cs[c + 1] += cs[c];
            if (cs[T] > cs[0] && cs[T] > J->tables[role[k]].capacity) J->capacity_error = 1;
        }
    }
    pthread_barrier_wait(&J->bar);
    if (J->capacity_error) return NULL;
    for (int k = 0; k < 3; ++k) {  /* exclusive scan: the slot of each append */
        int64_t run = J->chunk_sum[k * (T + 1) + w];
        for (int64_t s = s0; s < s1; ++s) {
            int64_t* c = &J->slot[k * n + J->order[s]];
            const int64_t v = *c;
            *c = run;
            run += v;
        }
    }
    pthread_barrier_wait(&J->bar);
    /* this worker's partitions, in timestamp order; spanning txns alone */
    orc_table R[ORC_R_COUNT];
    memcpy(R, J->tables, sizeof R);  /* own descriptors: shared columns */
    for (int64_t s = 0; s < n; ++s) {
        const int64_t i = J->order[s];
        if (!J->ok[i]) {
            if (s % T == w) pt_run(J, R, i);
            continue;
        }
        const int64_t pid = J->part[i];
        if (pid >= 0) {
            if (pid % T == w) pt_run(J, R, i);
            continue;
        }
        pthread_barrier_wait(&J->bar);
        if (w == 0) pt_run(J, R, i);
        pthread_barrier_wait(&J->bar);
    }
    return NULL;
}

int orc_execute_partitioned(int64_t n, const int32_t* type, const int64_t* params, int32_t n_params,
                            const int64_t* ts, const int32_t* proc_of_type, int32_t n_types,
                            orc_table* tables, const int64_t* part, int32_t n_threads,
                            int32_t* status, int64_t* results, int32_t width) {
    if (n < 0 || n_params < 1 || width < 1 || n_threads < 1 || n_threads > 1024) return ORC_E_ARG;
    if (n == 0) return ORC_OK;
    int rc = ORC_OK;
    int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    unsigned char* ok = (unsigned char*)malloc((size_t)n);
    int64_t* slot = (int64_t*)malloc(sizeof(int64_t) * 3 * (size_t)n);
    int64_t* chunk_sum = (int64_t*)calloc(3 * ((size_t)n_threads + 1), sizeof(int64_t));
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)n_threads);
    pt_arg* args = (pt_arg*)malloc(sizeof(pt_arg) * (size_t)n_threads);
    if (!order || !ok || !slot || !chunk_sum || !th || !args) {
        rc = ORC_E_ARG;
        goto out;
    }

    /* timestamp order (no sort when the input is already ascending) */
    int asc = 1;
    for (int64_t i = 1; i < n && asc; ++i) asc = ts[i] > ts[i - 1];
    if (asc) {
        for (int64_t i = 0; i < n; ++i) order[i] = i;
    } else {
        pt_key* k = (pt_key*)malloc(sizeof(pt_key) * (size_t)n);
        if (!k) { rc = ORC_E_ARG; goto out; }
        for (int64_t i = 0; i < n; ++i) { k[i].ts = ts[i]; k[i].idx = i; }
        qsort(k, (size_t)n, sizeof(pt_key), pt_cmp);
        int dup = 0;
        for (int64_t i = 0; i < n; ++i) {
            order[i] = k[i].idx;
            if (i > 0 && k[i].ts == k[i - 1].ts) dup = 1;
        }
        free(k);
        if (dup) { rc = ORC_E_DUP_TS; goto out; }
    }

    pt_job J;
    J.n = n; J.type = type; J.params = params; J.n_params = n_params; J.ts = ts;
    J.proc_of_type = proc_of_type; J.n_types = n_types; J.tables = tables; J.order = order;
    J.part = part; J.ok = ok; J.slot = slot; J.chunk_sum = chunk_sum; J.n_threads = n_threads;
    J.status = status; J.results = results; J.width = width; J.capacity_error = 0;
    pthread_barrier_init(&J.bar, NULL, (unsigned)n_threads);
    pthread_mutex_init(&J.mu, NULL);
    pthread_cond_init(&J.cv, NULL);
    J.go = 0;
    J.abort = 0;
    int started = 0;
    for (int32_t w = 0; w < n_threads; ++w) {
        args[w].job = &J;
        args[w].w = w;
        if (pthread_create(&th[w], NULL, pt_worker, &args[w]) != 0) break;
        started++;
    }
    /* open the gate; if a worker could not be created, nobody starts (the
       barriers would never fill) and the call fails before any mutation */
    pthread_mutex_lock(&J.mu);
    J.go = 1;
    J.abort = started < n_threads;
    pthread_cond_broadcast(&J.cv);
    pthread_mutex_unlock(&J.mu);
    for (int32_t w = 0; w < started; ++w) pthread_join(th[w], NULL);
    pthread_barrier_destroy(&J.bar);
    pthread_mutex_destroy(&J.mu);
    pthread_cond_destroy(&J.cv);
    if (started < n_threads) {
        rc = ORC_E_ARG;
        goto out;
    }
    if (J.capacity_error) {
        rc = ORC_E_CAPACITY;
        goto out;
    }
    tables[ORC_R_HISTORY].n_rows = chunk_sum[0 * (n_threads + 1) + n_threads];
    tables[ORC_R_ORDERS].n_rows = chunk_sum[1 * (n_threads + 1) + n_threads];
    tables[ORC_R_ORDER_LINE].n_rows = chunk_sum[2 * (n_threads + 1) + n_threads];

out:
    free(order); free(ok); free(slot); free(chunk_sum); free(th); free(args);
    return rc;
}
