/*
 * gputx.h -- C ABI of the MI355X bulk transaction engine.
 *
 * Model (He & Yu, "High-Throughput Transaction Executions on Graphics
 * Processors"):
 *  - Transactions are instances of pre-registered stored procedures,
 *    "Execute procedure_name(parameter list)" (Section 3.1); the procedures of
 *    all registered types form one combined kernel selected by a switch on the
 *    type (Section 3.2).
 *  - A transaction signature is <id, type, parameter values>; the unique id is
 *    its timestamp (Section 3.2).  A bulk is a set of such signatures that runs
 *    on the GPU as one task (Section 3.1).
 *  - Definition 1 (Section 3.1): the database after a bulk must equal the one
 *    obtained by running the bulk's transactions serially in increasing
 *    timestamp order.  Every strategy of gputx_execute_bulk meets it, and so do
 *    the per-transaction results.
 *  - Relations are stored column-wise in device memory, one array per
 *    fixed-length column (Section 3.2, Appendix E); inserts land in a buffer and
 *    are applied as a batched update after the bulk (Section 3.2).
 *
 * Conventions
 *  - Every call returns an int: GPUTX_OK (0) or a negative gputx error code.
 *    Nothing throws across the ABI.  gputx_last_error() gives a message.
 *  - "device" pointers are HIP device memory of the context's device; "host"
 *    pointers are ordinary host memory.  The caller owns every buffer it
 *    passes; the context borrows table columns for its lifetime and owns only
 *    its own small internal state.
 *  - Work is ordered on the hipStream_t the caller passes (0 = null stream).
 *    Calls on one context must not run concurrently from several host
 *    threads.
 */
#ifndef GPUTX_H
#define GPUTX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* gputx_stream_t; /* identical to hipStream_t */
typedef struct gputx_ctx* gputx_handle;

/* ---- status codes ------------------------------------------------------ */
enum {
    GPUTX_OK = 0,
    GPUTX_E_ARG = -1,       /* bad argument (null pointer, size, id)            */
    GPUTX_E_TYPE = -2,      /* unknown procedure or inconsistent type binding    */
    GPUTX_E_DUP_TS = -3,    /* two transactions of a bulk share a timestamp      */
    GPUTX_E_CAPACITY = -4,  /* an append table or the workspace is too small     */
    GPUTX_E_HIP = -5,       /* a HIP runtime call failed                         */
    GPUTX_E_STATE = -6,     /* call out of order (e.g. execute before load)      */
    GPUTX_E_DEADLOCK = -7,  /* a bounded device wait expired (watchdog)          */
    GPUTX_E_UNSORTED = -8,  /* bulk flagged ts_sorted but timestamps not ascending */
    GPUTX_E_INTERNAL = -9   /* an engine invariant failed on the device (a bug)  */
};

/* ---- execution strategies (Section 5) -------------------------------- */
enum {
    GPUTX_AUTO = 0, /* Algorithm 1 (Appendix D) picks one of the three below     */
    GPUTX_TPL = 1,  /* two-phase locking with counter-based locks (Section 5.1) */
    GPUTX_PART = 2, /* one thread per partition (Section 5.2)                   */
    GPUTX_KSET = 3  /* conflict-free k-set waves (Section 5.3)                  */
};

/* ---- per-transaction status ------------------------------------------ */
enum {
    GPUTX_COMMIT = 0,
    GPUTX_ABORT = 1,   /* two-phase transaction aborted in its read phase (Appendix D) */
    GPUTX_INVALID = 2  /* unregistered type or parameter outside its table: no effect   */
};

/* ---- compiled-in stored procedures ------------------------------------
 * Role bindings (gputx_type_desc.table_ids, in this order):
 *   bank procedures      : account, teller, branch, history
 *   order-entry procs    : warehouse, district, customer, stock, orders, order_line
 *   subscriber procs     : subscriber, call_fwd
 * Column 0 of account/teller/branch/warehouse/district/customer is the int64
 * balance; stock column 0 is the int32 quantity; subscriber columns are
 * id (int64), 4 int32 fields, 10 int32 locations; call_fwd columns are
 * occupied (int32), end (int32), number (int64); history, orders and
 * order_line have 5 int64 columns.
 * Parameters (param k of the signature):
 *   DEBIT_CREDIT (acct, teller, branch, delta) -> (acct', teller', branch')
 *       adds delta to the three balances, appends history (acct, teller,
 *       branch, delta, ts).
 *   NEW_ORDER (w, d, c, k, item[15], q[15]) -> (k, s_0..s_{k-1})
 *       for j < k: s = stock[w*ipw + item_j] - q_j, plus 91 if below 10;
 *       appends orders (ts, w, d, c, k) and k order lines (ts, j, item_j, q_j, w).
 *       Valid iff 1 <= k <= 15, items < ipw, 1 <= q_j <= 1000.
 *   PAYMENT (w, d, c, h) -> (warehouse', district', customer'), each += h.
 *   ORDER_STATUS (w, d, c) -> (customer balance).
 *   GET_SUB (sid) -> 14 int32 fields.            GET_CF (sid, slot) -> (occ, end, number).
 *   UPD_SUB_FIELD (sid, f < 4, v) / UPD_LOC (sid, l < 10, v) -> previous value.
 *   INS_CF (sid, slot, end, number): ABORT if occupied; -> (previous occupied).
 *   DEL_CF (sid, slot): ABORT if empty; -> (1, end, number) of the deleted row.
 *   NEW_ORDER_RB (same signature as NEW_ORDER): new-order that is NOT
 *       two-phase (Appendix D): an item id equal to ipw names an unused item;
 *       the procedure updates the stock of the items before it in order,
 *       meets the unused one, and rolls those updates back from its undo log:
 *       ABORT, no effect, results 0.  Otherwise as NEW_ORDER.  Items <= ipw.
 * Dimensions are derived from the bound tables: ipw = stock rows / warehouses,
 * dpw = districts / warehouses, cpd = customers / districts; a call_fwd slot is
 * sid * 12 + slot.  Arithmetic on int64 values wraps modulo 2^64.
 */
enum {
    GPUTX_DEBIT_CREDIT = 1,
    GPUTX_NEW_ORDER = 2,
    GPUTX_PAYMENT = 3,
    GPUTX_ORDER_STATUS = 4,
    GPUTX_GET_SUB = 5,
    GPUTX_GET_CF = 6,
    GPUTX_UPD_SUB_FIELD = 7,
    GPUTX_UPD_LOC = 8,
    GPUTX_INS_CF = 9,
    GPUTX_DEL_CF = 10,
    GPUTX_NEW_ORDER_RB = 11
};

enum { GPUTX_I32 = 1, GPUTX_I64 = 2 };

#define GPUTX_MAX_TYPES 16
#define GPUTX_MAX_TABLES 32
#define GPUTX_MAX_COLS 16
#define GPUTX_MAX_ROLES 8

/* Engine options; gputx_default_options fills every field. */
typedef struct {
    int64_t w0_bar;        /* Algorithm 1: K-SET when |0-set| >= w0_bar                  */
    int64_t c_bar;         /* Algorithm 1: PART when cross-partition txns <= c_bar ...  */
    int64_t d_bar;         /* ... or depth >= d_bar; TPL otherwise                      */
    int64_t part_size;     /* root keys per partition for PART and for c (Section 5.2)  */
    int32_t group_by_type; /* 1: group executing transactions by type (Section 5.4)     */
    int32_t kset_narrow;   /* K-SET waves of at most this many txns run in one workgroup */
    int32_t spin_limit_ms; /* watchdog on every device wait; expiry -> GPUTX_E_DEADLOCK  */
    int32_t grid_blocks;   /* persistent grid size (0: one workgroup per compute unit)  */
    int32_t part_pipeline; /* PART with a staging wave beside the serial one (1, default) */
    int32_t part_scan;     /* 1 (default): PART runs several transactions of a partition
                              at once where that leaves the serial result: procedures
                              whose effect on each cell is a map of that cell alone
                              (debit-credit, payment, order status, the subscriber reads
                              and field updates) as a scan of those maps per cell, up to
                              four new-orders with distinct items or four subscriber
                              reads side by side; reported as "PART-scan"
                              (stats.part_scan); 0: every partition runs its
                              transactions one after another (Section 5.2 as written)  */
    int32_t tpl_lanes;     /* TPL launch shape, 0..64: 64 runs windows of 256
                              transactions per workgroup, grouped by type (Section
                              5.4); 1..32 gives each wave its own window of tpl_lanes
                              transactions, one per lane, the other lanes idle, so a
                              transaction that becomes ready waits on fewer other
                              critical sections of its wave (deep dependency chains);
                              0 (default): chosen per bulk from its average
                              parallelism n / (d + 1) and the grid's waves          */
} gputx_options;

/* One relation.  Columns are device arrays of capacity rows, caller-owned,
 * borrowed for the context's lifetime (Appendix E column store). */
typedef struct {
    int32_t table_id;                 /* 0 .. GPUTX_MAX_TABLES-1, unique              */
    int32_t n_cols;                   /* 1 .. GPUTX_MAX_COLS                          */
    int64_t n_rows;                   /* rows present at load                         */
    int64_t capacity;                 /* rows the arrays hold (>= n_rows)             */
    int32_t append_only;              /* 1: only appended to, never read in a bulk    */
    int32_t root_table_id;            /* table holding this table's partition root, -1 none */
    int64_t root_div;                 /* rows of this table per root key (>= 1)       */
    int32_t col_dtype[GPUTX_MAX_COLS];/* GPUTX_I32 / GPUTX_I64                        */
    void* col_ptr[GPUTX_MAX_COLS];    /* device pointers                              */
} gputx_table_desc;

/* One registered transaction type (Section 3.1) with the DBA annotations of
 * Appendix E (partitioning through the tables' root keys; single-partition
 * flag is informational: the engine always counts cross-partition
 * transactions from their operations). */
typedef struct {
    int32_t type_id;                      /* 0 .. GPUTX_MAX_TYPES-1                 */
    int32_t proc;                         /* GPUTX_DEBIT_CREDIT ...                 */
    int32_t n_params;                     /* parameters the procedure reads         */
    int32_t n_results;                    /* result values it writes                */
    int32_t table_ids[GPUTX_MAX_ROLES];   /* role bindings, see above               */
    int32_t root_key;                     /* 1: lock only partition roots (Section 5.1) */
    int32_t single_partition;
} gputx_type_desc;

/* A bulk, structure-of-arrays in device memory (Section 3.2 signatures). */
typedef struct {
    int64_t n;              /* transactions                                         */
    const int32_t* type;    /* [n] device                                           */
    const int64_t* params;  /* [n_params][n] device, param-major                    */
    int32_t n_params;       /* >= every registered type's n_params it uses          */
    const int64_t* ts;      /* [n] device, unique                                   */
    int32_t ts_sorted;      /* 1: caller promises ascending ts (checked on device)  */
    int32_t max_ops;        /* most basic operations per txn, 0: the context's maximum
                               over registered types (checked on device)            */
    uint32_t type_mask;     /* registered types the bulk may hold (bit t: type t); 0:
                               all.  PART's per-chunk LDS rows are sized for these
                               types only (a context that registers order entry
                               and debit-credit runs debit-credit bulks with the
                               debit-credit layout); a transaction of a type outside
                               the mask is INVALID                                   */
    int32_t reserved;       /* 0                                                     */
} gputx_bulk;

/* Written by the device during gputx_execute_bulk; read it after the stream
 * has been synchronised. */
typedef struct {
    int32_t error;      /* 0 or a bulk error (DUP_TS, CAPACITY, UNSORTED, DEADLOCK) */
    int32_t chosen;     /* strategy that ran                                        */
    int64_t n_ops;      /* basic operations emitted (Section 4.1)                   */
    int64_t w0;         /* |0-set| (Appendix D)                                     */
    int64_t depth;      /* maximum operation rank (Section 4.2 step 5)              */
    int64_t cross;      /* cross-partition transactions c                           */
    int64_t waves;      /* K-SET waves executed (= true depth + 1)                  */
    int64_t committed;
    int64_t aborted;
    int64_t invalid;
    int64_t appended;   /* rows appended to append-only tables (batched update)   */
    int64_t part_scan;  /* PART ran: partition chunks (of a mixed chunk, each
                           serial wave's share) that ran transactions side by
                           side (gputx_options.part_scan); 0 = Section 5.2's
                           one-after-another run throughout                      */
    int64_t reserved[6];
} gputx_bulk_stats;

/* Fill *opt with defaults. */
int gputx_default_options(gputx_options* opt);

/* Create a context on HIP device hip_device; opt may be NULL (defaults). */
int gputx_create(int hip_device, const gputx_options* opt, gputx_handle* out);

/* Destroy a context (frees only its internal state). */
int gputx_destroy(gputx_handle h);

/* Replace the options of a context. */
int gputx_set_options(gputx_handle h, const gputx_options* opt);

/* Load (borrow) tables: the database is loaded once and stays resident
 * (Appendix E); load cost is not part of bulk execution.  May be called
 * again to add tables; row counts of append tables then live on the device
 * and advance with every bulk.  Errors: GPUTX_E_ARG. */
int gputx_load_tables(gputx_handle h, const gputx_table_desc* t, int n);

/* Register transaction types (Section 3.1: the combined kernel switches on
 * the type).  Tables must be loaded first.  Errors: GPUTX_E_TYPE for an
 * unknown procedure or a role bound to a missing or mis-typed table. */
int gputx_register_types(gputx_handle h, const gputx_type_desc* t, int n);

/* Workspace bytes gputx_execute_bulk needs for up to n_txns transactions
 * (max_ops per transaction = the context's maximum over registered types). */
size_t gputx_workspace_size(gputx_handle h, int64_t n_txns);

/* Same, for bulks whose gputx_bulk.max_ops is set to max_ops (> 0). */
size_t gputx_workspace_size_ops(gputx_handle h, int64_t n_txns, int32_t max_ops);

/* Execute one bulk (Section 5): order by timestamp, derive the basic
 * operations, group and rank them (Section 4.2), choose a strategy
 * (Algorithm 1, when strategy == GPUTX_AUTO) and run it, then apply the
 * batched appends.
 *   workspace: device, ws_bytes >= gputx_workspace_size(h, b->n).
 *   status_out: device int32[n]; results_out: device int64[n][width]; both
 *     indexed by the transaction's position in the bulk arrays.  Unused
 *     result entries are written 0.
 *   stats: device gputx_bulk_stats, overwritten.
 * Host-detectable errors return synchronously with nothing launched.  Device-
 * detected bulk errors (duplicate or unsorted timestamps, append overflow)
 * land in stats->error and leave every table unmodified. */
int gputx_execute_bulk(gputx_handle h, const gputx_bulk* b, int strategy, void* workspace,
                       size_t ws_bytes, int32_t* status_out, int64_t* results_out, int32_t width,
                       gputx_bulk_stats* stats, gputx_stream_t stream);

/* Execute one bulk without the timestamp constraint (Appendix G): the
 * result is serializable -- equal to running the bulk's transactions one by
 * one in SOME order -- but that order need not be the timestamp order, so
 * neither the timestamp sort nor the operation sort and ranking run.
 *   strategy GPUTX_TPL: basic 0/1 spin locks (Figure 10) taken with
 *     compare-and-swap on every item's lock word, all or none at a time;
 *   strategy GPUTX_PART: transactions grouped by partition with
 *     per-partition counters and a prefix sum instead of a sort, then each
 *     partition run one transaction after another; a bulk with
 *     cross-partition transactions runs under the TPL form (Section 5.2).
 *   serial_key_out: device int64[n]; after the bulk, ordering the committed
 *     and aborted transactions by this key (ties in any order: tied
 *     transactions do not conflict) gives a serial order equivalent to the
 *     execution; invalid transactions get -1.
 *   Timestamps are not checked and serve only as values (appended rows);
 *   appended rows take slots in input order.  Other arguments, workspace
 *   size, ordering and errors as gputx_execute_bulk; stats->w0, depth and
 *   waves are 0. */
int gputx_execute_bulk_relaxed(gputx_handle h, const gputx_bulk* b, int strategy, void* workspace,
                               size_t ws_bytes, int32_t* status_out, int64_t* results_out, int32_t width,
                               int64_t* serial_key_out, gputx_bulk_stats* stats, gputx_stream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * bulk execution as gputx_execute_bulk, with its workspace in a static
 * device array of GPUTX_SCRATCH_BYTES (64 MiB) that each GPU the library
 * runs on holds until the process ends.  The call allocates nothing; the
 * caller still passes the bulk and the outputs.
 *   Bulks whose workspace (gputx_workspace_size_ops(h, b->n, b->max_ops))
 *   exceeds GPUTX_SCRATCH_BYTES are rejected with GPUTX_E_CAPACITY before
 *   anything is launched (e.g. about 2^17 debit-credits fit).
 *   Every call on one GPU uses that GPU's one array: calls that overlap on
 *   one GPU (other streams, other contexts, other host threads) race and
 *   must be serialised by the caller.  Nothing needs to start at zero: each
 *   bulk clears the state it reads.
 * Other arguments, ordering and errors as gputx_execute_bulk. */
#define GPUTX_SCRATCH_BYTES ((size_t)64 << 20)
int gputx_execute_bulk_noalloc(gputx_handle h, const gputx_bulk* b, int strategy,
                               int32_t* status_out, int64_t* results_out, int32_t width,
                               gputx_bulk_stats* stats, gputx_stream_t stream);

/* ---- batched form: many bulks, one graph launch ------------------------
 * Each item is one bulk with its own workspace and outputs.  Items of one
 * lane share tables and run in item order (so the serial order across them is
 * the item order, then timestamps within a bulk); different lanes touch
 * disjoint tables and run concurrently.  Within a lane the bulk generation of
 * an item (timestamp order, operations, sort, ranks, Algorithm 1) overlaps the
 * execution of the previous item, since it reads no table.  Persistent grids
 * of concurrent lanes are sized so that all of them stay resident. */
typedef struct {
    gputx_bulk bulk;            /* device arrays, as for gputx_execute_bulk         */
    int32_t strategy;           /* GPUTX_AUTO .. GPUTX_KSET                         */
    int32_t lane;               /* 0 .. 63                                          */
    void* workspace;            /* device, >= gputx_workspace_size(h, bulk.n)       */
    size_t ws_bytes;
    int32_t* status_out;        /* device int32[n]                                  */
    int64_t* results_out;       /* device int64[n][width]                           */
    int32_t width;
    gputx_bulk_stats* stats;    /* device                                           */
    int32_t grid_blocks;        /* persistent grid of this bulk's lock / k-set executor
                                   (0: the context's; capped so that every lane's grid
                                   stays resident)                                  */
    int32_t kset_narrow;        /* K-SET narrow-wave width for this bulk (0: the
                                   context's)                                       */
} gputx_batch_item;

typedef struct gputx_batch_t* gputx_batch;

/* Capture every item into one HIP graph and instantiate it; nothing runs
 * yet.  Arguments are validated per item (same errors as gputx_execute_bulk).
 * The item array is not retained; the buffers it names must stay valid while
 * the batch exists. */
int gputx_batch_create(gputx_handle h, const gputx_batch_item* items, int n, gputx_batch* out);

/* Launch the whole batch on a stream (one graph launch).  Every launch runs
 * every item again against the current tables. */
int gputx_batch_launch(gputx_batch b, gputx_stream_t stream);

/* Free the graph. */
int gputx_batch_destroy(gputx_batch b);

/* ---- served form: continuous batching (Sections 3.2, 6.3) --------------
 * A server owns a transaction pool and a result pool in host memory and a
 * native thread.  Callers submit signatures into the transaction pool; at
 * every bulk interval (Section 6.3's fixed interval t) the thread cuts
 * everything submitted so far into a bulk (up to max_bulk transactions) and
 * issues it; finished bulks' statuses and results land in the result pool,
 * where gputx_serve_poll collects them in submission order.  Up to `slots`
 * bulks are in flight: the bulk generation of a new bulk overlaps the
 * execution of earlier ones, and executions keep submission order, so the
 * database sees the transactions in ticket order (ids must ascend).
 * Admission is bounded by an HBM budget: the slots it allows are allocated
 * at open; a cut waits for a free slot, and whatever arrives meanwhile joins
 * it.  Bulks are padded to a size class (four per octave) with invalid
 * transactions, which have no effect. */
typedef struct {
    int64_t deadline_ns;        /* bulk interval                                    */
    int32_t slots;              /* bulks in flight at most (>= 1)                   */
    int32_t strategy;           /* GPUTX_AUTO ..                                    */
    int64_t max_bulk;           /* largest bulk; a bigger backlog is cut in pieces  */
    int64_t hbm_budget;         /* device bytes the slots may use (0: no cap)       */
    int32_t width;              /* result values per transaction                    */
    int32_t max_ops;            /* per-transaction op bound (0: context maximum)    */
} gputx_serve_opts;

typedef struct {
    int64_t first;              /* first ticket of the bulk                         */
    int64_t count;
    int64_t cut_ns;             /* server clock when the bulk was cut               */
    int64_t issued_ns;          /* server clock when its copies and graphs were queued */
    int64_t done_ns;            /* server clock when its results were in host memory */
    int32_t error;              /* bulk error, 0 = none                             */
    int32_t slot;
    int32_t front_us;           /* device time: upload and bulk generation          */
    int32_t exec_us;            /* device time: execution start to results copied   */
} gputx_serve_bulk;

typedef struct {
    int64_t n_bulks;            /* bulks issued                                     */
    int64_t committed;
    int64_t aborted;
    int64_t invalid;
    int64_t elapsed_ns;         /* open .. last results back                        */
    int32_t slots_used;         /* slots the HBM budget allowed                     */
    int32_t reserved;
    int64_t slot_bytes;         /* device bytes one slot takes                      */
} gputx_serve_report;

typedef struct gputx_server_t* gputx_server;

/* Open a server on a context whose tables and types are loaded.  n_params:
 * parameters per submitted signature; pool_capacity: transactions the pools
 * hold (submitted but not yet polled).  Allocates the slots (device), their
 * graphs and pinned staging, then starts the server thread; the server
 * clock starts here.  Errors: GPUTX_E_ARG, GPUTX_E_CAPACITY (budget below
 * one slot, pool too large), GPUTX_E_HIP. */
int gputx_serve_open(gputx_handle h, const gputx_serve_opts* opts, int32_t n_params,
                     int64_t pool_capacity, gputx_server* out);

/* Put n signatures into the transaction pool (host arrays: type[n],
 * params[k * ld + i] for parameter k of transaction i, ts[n] ascending and
 * above every id submitted before).  They arrive now (server clock) and get
 * consecutive tickets starting at *first_ticket (may be NULL).  Nothing is
 * taken on error: GPUTX_E_ARG (ids out of order), GPUTX_E_CAPACITY (pool
 * full until results are polled), GPUTX_E_STATE (closing). */
int gputx_serve_submit(gputx_server s, int64_t n, const int32_t* type, const int64_t* params,
                       int64_t ld, const int64_t* ts, int64_t* first_ticket);

/* Take up to max finished transactions from the result pool, in ticket
 * order, without waiting: ticket[j], status[j], results[j * width ..],
 * latency_ns[j] (results in host memory minus arrival); any output pointer
 * may be NULL.  *n_out receives the count.  Returns a bulk error latched by
 * the server (its transactions then read GPUTX_INVALID), else GPUTX_OK. */
int gputx_serve_poll(gputx_server s, int64_t max, int64_t* ticket, int32_t* status, int64_t* results,
                     int64_t* latency_ns, int64_t* n_out);

/* Run every submitted transaction, stop the thread and free the server
 * (results not polled are dropped).  report may be NULL.  Returns the first
 * bulk error, if any. */
int gputx_serve_close(gputx_server s, gputx_serve_report* report);

/* Replay an arrival trace through a server: each transaction is submitted
 * once its arrival time (ns from open) has passed, and the results are
 * polled into status_out [n] / results_out [n][width] (host).  bulks[]
 * receives up to bulk_capacity per-bulk records in issue order (first =
 * trace index).  Per-transaction commit latency is done_ns of its bulk
 * minus its arrival time.  Errors: GPUTX_E_ARG (trace not in arrival order,
 * bad options), those of gputx_serve_open, a device bulk error code. */
typedef struct {
    int64_t n;                  /* transactions                                     */
    const int64_t* arrival_ns;  /* [n] host, non-decreasing, ns from the start      */
    const int32_t* type;        /* [n] host                                         */
    const int64_t* params;      /* [n_params][n] host, param-major                  */
    int32_t n_params;
    const int64_t* ts;          /* [n] host, ascending (ids in arrival order)       */
} gputx_trace;

int gputx_serve(gputx_handle h, const gputx_trace* trace, const gputx_serve_opts* opts,
                int32_t* status_out, int64_t* results_out, gputx_serve_bulk* bulks,
                int64_t bulk_capacity, gputx_serve_report* report);

/* Copy rows [row0, row0 + n) of column col of a loaded table into host_dst
 * (4-byte elements for GPUTX_I32 columns, 8-byte for GPUTX_I64), ordered on
 * the stream and synchronised: the database as the bulks left it (Section
 * 3.2's tables stay resident on the device).  Rows must lie within the
 * table's capacity.  Errors: GPUTX_E_ARG, GPUTX_E_HIP. */
int gputx_read_table(gputx_handle h, int32_t table_id, int32_t col, int64_t row0, int64_t n,
                     void* host_dst, gputx_stream_t stream);

/* Current row count of a table (append tables advance on the device);
 * synchronises the stream. */
int gputx_row_count(gputx_handle h, int32_t table_id, int64_t* out, gputx_stream_t stream);

/* Phase timing (Figure 5 / Figure 12 style breakdowns).  When enabled, every
 * gputx_execute_bulk records one HIP event on its stream at each phase
 * boundary (no synchronisation); up to 256 bulks are kept, counted from the
 * last enable.  Phases, in order: order (timestamp check/sort), prepare
 * (validation + scans), emit (basic operations), op_sort, rank, features
 * (+ Algorithm 1), part_sort, part, tpl, kset, finalize.  Phases that do not
 * run for a bulk take ~0 ms. */
int gputx_phase_timing(gputx_handle h, int enable);

/* Sum over the recorded bulks of each phase's duration in milliseconds:
 * ms[i] for phase i < cap; *n_bulks receives the number of bulks summed.
 * Synchronises with the last recorded event.  Returns the number of phases. */
int gputx_phase_times(gputx_handle h, double* ms, int cap, int64_t* n_bulks);

/* Name of phase i (static storage), or NULL past the last phase. */
const char* gputx_phase_name(int i);

/* Set the row count of an append-only table (0 <= n <= capacity), e.g. to
 * truncate it after its rows were archived; ordered on the stream and
 * synchronised.  Errors: GPUTX_E_ARG for a table that is not append-only. */
int gputx_set_row_count(gputx_handle h, int32_t table_id, int64_t n, gputx_stream_t stream);

/* ---- measurement probes ------------------------------------------------
 * The ceilings the executors are measured against, taken on the device at
 * hand (Appendix D calibrates Algorithm 1 on the machine it runs on).  Each
 * call allocates and frees its own device memory, synchronises the device
 * and checks its own result (GPUTX_E_INTERNAL if the check fails).  Errors
 * are reported through gputx_last_error(NULL).
 *
 * gputx_probe_handoff: mean latency of one lock hand-off between two
 *   workgroups (another XCD, or the same one when same_xcd != 0), each turn
 *   being the lock executor's own sequence: spin on a counter, acquire
 *   fence, read-modify-write of a cell, release fence, atomic add.  A chain
 *   of dependent transactions costs at least this per step, so
 *   (depth + 1) x ns_per_hop bounds TPL and K-SET from below.
 *   hops in [2, 2^24]; GPUTX_E_DEADLOCK if a turn waits more than 2 s.
 * gputx_probe_atomic_add: 32-bit device atomic adds per second over n_addr
 *   addresses (1, 64, 640: contended lock counters; large: uniform random),
 *   n_updates >= 2^18 in total.
 * gputx_probe_gather: gathered bytes per second (1e9) of 8-byte loads at
 *   uniform random rows of a table_bytes table (a power of two >= 4096):
 *   64 MiB stays in the Infinity Cache, 4 GiB does not.  n_gathers >= 2^18. */
int gputx_probe_handoff(int hip_device, int32_t hops, int32_t same_xcd, double* ns_per_hop);
int gputx_probe_atomic_add(int hip_device, int64_t n_addr, int64_t n_updates, double* updates_per_s);
int gputx_probe_gather(int hip_device, int64_t table_bytes, int64_t n_gathers, double* gb_per_s);

/* ---- K-SET over a standing pool (Section 5.3, incremental k-set) --------
 * A pool holds pending transactions across bulks.  gputx_pool_add puts a
 * bulk in (its basic operations are sorted and merged into the pool's
 * operations, sorted by item and timestamp); gputx_pool_step runs the pool's
 * 0-set -- every pending transaction none of whose operations has a
 * conflicting predecessor still pending -- without locks and removes it, as
 * many times as asked.  The 1-set then becomes the 0-set, so any
 * interleaving of adds and steps executes the transactions with the result
 * of running them serially in timestamp order (Definition 1): bulks must be
 * added in timestamp order (every id above those already added).  Results
 * stay in the pool until fetched, in sequence order.  A bulk error
 * (duplicate or out-of-order ids, append overflow) puts the pool in an error
 * state: nothing runs afterwards.  Appended rows are reserved when a bulk is
 * added (in timestamp order) and written when their transaction runs. */
typedef struct gputx_pool_t* gputx_pool;

typedef struct {
    int32_t error;        /* sticky bulk error, 0 = none                      */
    int32_t reserved;
    int64_t added;        /* transactions added (their sequence numbers 0..)  */
    int64_t done_prefix;  /* every transaction below this has run            */
    int64_t pending_ops;  /* operations of pending transactions              */
    int64_t waves;        /* steps that ran at least one transaction         */
    int64_t executed;     /* transactions run by steps                       */
    int64_t committed;
    int64_t aborted;
    int64_t invalid;      /* invalid transactions (done when added)          */
    int64_t last_width;   /* transactions the last step ran                  */
    int64_t fetched;      /* results handed back                             */
} gputx_pool_stats;

/* Create a pool for up to `capacity` transactions added and not yet fetched
 * (rounded up to a power of two), bulks of at most max_add transactions with
 * n_params parameters, results of `width` values, max_ops operations per
 * transaction (0: the context's maximum).  Allocates device memory. */
int gputx_pool_create(gputx_handle h, int64_t capacity, int32_t n_params, int32_t width, int32_t max_ops,
                      int64_t max_add, gputx_pool* out);
/* Add a bulk (device arrays as for gputx_execute_bulk); ordered on the
 * stream.  GPUTX_E_CAPACITY (host-side) when the pool lacks free slots. */
int gputx_pool_add(gputx_pool p, const gputx_bulk* b, gputx_stream_t stream);
/* Run `waves` successive 0-sets; ordered on the stream. */
int gputx_pool_step(gputx_pool p, int32_t waves, gputx_stream_t stream);
/* Counters of the pool (synchronises the stream). */
int gputx_pool_state(gputx_pool p, gputx_pool_stats* out, gputx_stream_t stream);
/* Copy the status and results of the next n transactions in sequence order
 * (all of them must have run: n <= done_prefix - fetched) into status[n],
 * results[n][width] (host or device); their slots become free.
 * GPUTX_E_STATE when fewer have run.  Synchronises the stream. */
int gputx_pool_results(gputx_pool p, int64_t n, int32_t* status, int64_t* results, gputx_stream_t stream);
/* Free the pool (synchronises the device). */
int gputx_pool_destroy(gputx_pool p);

/* ---- branch-divergence micro benchmark (Section 6.2, Figures 3 and 12) --
 * n independent transactions; transaction i has type type[i] in [0, n_types)
 * and reads tuples[i], runs its type's case of one switch -- 100 * x rounds
 * of v <- (v xor (v >> 29)) * M_k + (k + 1) with M_k = 0x9E3779B97F4A7C15 +
 * 2k (uint64 arithmetic) for type k -- and writes the result back.  With
 * groups > 1 the transaction order is first radix-partitioned on the top
 * log2(groups) bits of the type id, one stable 1-bit pass per bit (Appendix
 * D's grouping with a tunable number of partitions), so lanes of one wave
 * share fewer case bodies.  groups = 1 runs the bulk in input order.
 *   type, tuples: device arrays of n; n_types in [1, 32]; x in [0, 1000];
 *   groups a power of two <= n_types.
 *   workspace: device, 256-byte aligned, >= gputx_micro_workspace_size(n)
 *     (unused when groups == 1).
 *   phase: 0 both steps, 1 the grouping only, 2 the execution only (after a
 *     phase-1 call with the same arguments and workspace), for timing them
 *     apart.  After the grouping, the grouped order (int32 transaction
 *     indices, n of them) sits at byte 0 of the workspace when log2(groups)
 *     is odd and at byte round_up(4 n, 256) when it is even.
 * Ordered on the stream; errors GPUTX_E_ARG, GPUTX_E_CAPACITY, GPUTX_E_HIP
 * through gputx_last_error(NULL). */
size_t gputx_micro_workspace_size(int64_t n);
int gputx_micro_run(int64_t n, const int32_t* type, int64_t* tuples, int32_t n_types, int32_t x,
                    int32_t groups, void* workspace, size_t ws_bytes, int32_t phase,
                    gputx_stream_t stream);

/* Message of the last error on this context (static storage, never NULL). */
const char* gputx_last_error(gputx_handle h);

#ifdef __cplusplus
}
#endif
#endif /* GPUTX_H */
