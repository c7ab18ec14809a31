/*
 * Serial oracle interface.  TEST INFRASTRUCTURE ONLY (tests, smoke check,
 * benchmark CPU baseline); the GPU engine never includes or links it.
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_E_ARG = -1, ORC_E_DUP_TS = -3, ORC_E_CAPACITY = -4 };
enum { ORC_COMMIT = 0, ORC_ABORT = 1, ORC_INVALID = 2 };

/* procedures (registered types map onto these) */
enum {
    ORC_DEBIT_CREDIT = 1, ORC_NEW_ORDER, ORC_PAYMENT, ORC_ORDER_STATUS,
    ORC_GET_SUB, ORC_GET_CF, ORC_UPD_SUB_FIELD, ORC_UPD_LOC, ORC_INS_CF, ORC_DEL_CF,
    ORC_NEW_ORDER_RB
};

/* table roles */
enum {
    ORC_R_ACCOUNT, ORC_R_TELLER, ORC_R_BRANCH, ORC_R_HISTORY,
    ORC_R_WAREHOUSE, ORC_R_DISTRICT, ORC_R_CUSTOMER, ORC_R_STOCK, ORC_R_ORDERS, ORC_R_ORDER_LINE,
    ORC_R_SUBSCRIBER, ORC_R_CALL_FWD, ORC_R_COUNT
};

#define ORC_NO_MAX_ITEMS 15
#define ORC_CF_SLOTS 12
#define ORC_SUB_FIELDS 4
#define ORC_SUB_LOCS 10

/* One table: host column pointers; for append tables n_rows is advanced. */
typedef struct {
    void* col[16];
    int64_t n_rows;
    int64_t capacity;
} orc_table;

/*
 * Execute a bulk serially in timestamp order.
 *   type[n], params[n_params][n] (param-major), ts[n]: the bulk, host memory.
 *   proc_of_type[t]: procedure of registered type t (0 = unregistered).
 *   tables[ORC_R_COUNT]: role-indexed tables, mutated in place.
 *   status[n], results[n][width]: per transaction, at its input index.
 * Returns ORC_OK, or ORC_E_DUP_TS / ORC_E_CAPACITY / ORC_E_ARG with no
 * table mutated.
 */
int orc_execute(int64_t n, const int32_t* type, const int64_t* params, int32_t n_params,
                const int64_t* ts, const int32_t* proc_of_type, int32_t n_types,
                orc_table* tables, int32_t* status, int64_t* results, int32_t width);

/*
 * The paper's CPU counterpart (Section 6.3): an H-Store-style partitioned
 * executor.  Each transaction is routed by its partition (part[i] >= 0: all
 * its rows lie in that partition; -1: it spans several).  Worker w of
 * n_threads owns the partitions p with p % n_threads == w and runs their
 * transactions one after another in timestamp order; a transaction that
 * spans partitions runs alone, after every earlier transaction and before
 * any later one (all workers wait at a barrier on each side).  Appended rows
 * take the slots a timestamp-order scan of the append counts gives them, so
 * the result equals orc_execute's exactly.  Same arguments and return codes
 * as orc_execute.
 */
int orc_execute_partitioned(int64_t n, const int32_t* type, const int64_t* params, int32_t n_params,
                            const int64_t* ts, const int32_t* proc_of_type, int32_t n_types,
                            orc_table* tables, const int64_t* part, int32_t n_threads,
                            int32_t* status, int64_t* results, int32_t width);

/* Pieces of the serial executor the partitioned one reuses (serial.c). */
int orc_is_valid(int proc, const int64_t* p, const orc_table* R);
void orc_appends_of(int proc, const int64_t* p, const orc_table* R, int64_t* h, int64_t* o, int64_t* ol);
int32_t orc_run_one(int proc, const int64_t* p, int64_t ts, orc_table* R, int64_t* res);

#ifdef __cplusplus
}
#endif
#endif
