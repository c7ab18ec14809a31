// Internal interface between the host runtime and the engine's kernels.
#pragma once
#include "procs.h"
#include "sort.h"

namespace gtx {

// Tile aggregate of the operation-ranking scan.
struct RankAgg {
    int32_t segf;  // a group starts inside the tile
    int32_t segs;  // rank increments after the last group start (or all)
    int32_t gs;    // last group-start position (inclusive max), -1 none
    int32_t A;     // max over writes of position + 1
    int32_t g;     // group starts
    int32_t B;     // min over writes and group starts of position (m: none)
};

// Everything later stages need about one basic operation, in op order
// (transaction-major), written with one 32-byte store by the ranking scan.
struct __attribute__((aligned(32))) OpInfo {
    int32_t grp;   // lock group (distinct item) of the op
    int32_t tgt;   // completed ops of the group the op waits for (TPL)
    int32_t slo;   // successor range in sorted order (K-SET)
    int32_t shi;
    int32_t rank;  // the paper's rank (Section 4.2 step 3)
    int32_t in;    // in-edges the op contributes to its transaction (K-SET)
    int32_t s0;    // transaction of the first successor op (-1: none)
    int32_t s0ty;  // its type
};

// K-SET's view of one transaction, written by its preparation passes: the
// first successor transaction of each of its first four operations (-1:
// none) and their types (low 16 bits), so a wave releases them with one
// load.  Bit 16 of s0ty[3]: the transaction has further operations or read
// runs, which the wave walks in the operation records.
struct __attribute__((aligned(32))) KsetRec {
    int32_t s0[4];
    int32_t s0ty[4];
};

// Device workspace of one bulk (carved from the caller's workspace).
struct Ws {
    GtxState* st;
    uint64_t* tsk[2];    // timestamp sort keys
    uint32_t* tsv[2];    // timestamp sort values: input index
    int32_t* tty;        // [n] type id at serial position, -1 invalid
    int32_t* cnt;        // [(1 + GTX_MAX_APPEND)][n]: op count then appends; scanned in place
    int32_t* maxrank;    // [n]
    int32_t* indeg;      // [n]
    KsetRec* ksrec;      // [n] K-SET: first successors per transaction
    int32_t* op_txn;     // [mcap] serial position of each operation
    uint32_t* pk[2];     // [mcap] operation sort: item key
    uint32_t* pv[2];     // [mcap] operation sort: op index << 1 | write
    int32_t* op_rank;    // [mcap] the paper's rank of each operation
    OpInfo* op_info;     // [mcap] written only when TPL or K-SET runs
    int32_t* srt_txn;    // [mcap] serial position of each sorted op
    int32_t* grp_cnt;    // [mcap] per-group completion counters
    uint32_t* qk[2];     // [n] PART sort: partition id
    uint32_t* qv[2];     // [n] PART sort: serial position
    uint32_t* qinv;      // [n] PART: partition-grouped position of each serial position
    int32_t* heads;      // [n + 1] PART: first sorted position of each non-empty partition
    int32_t* heads_tmp;  // [head blocks] PART: per-block head counts, then offsets
    // PART: one record per partition-sorted position (k_part_gather): input
    // index and type in the first word, then the parameters (zero past the
    // type's own)
    int64_t* rec;        // [n][rec_words]
    int32_t* front[2];   // [n] K-SET frontiers
    uint32_t* sort_hist; // [8][256]
    uint32_t* sort_status;
    uint32_t* sort_ctrl; // [16]
    // the partition sort's own histogram, look-back words and tile counters,
    // so that it can run beside the item-key sort
    uint32_t* psort_hist;   // [8][256]
    uint32_t* psort_status;
    uint32_t* psort_ctrl;   // [16]
    int32_t* scan_tmp;   // [(1 + GTX_MAX_APPEND)][scan blocks]
    int32_t* tcnt_tmp;   // [kPrepBlocks][GPUTX_MAX_TYPES] per-block type counts
    RankAgg* rank_tmp;   // [2][rank tiles]
};

// Words of a PART record: the index/type word, then prm_rows parameters
// (16-byte aligned records).
inline int part_rec_words(int prm_rows) { return (1 + prm_rows + 1) & ~1; }

struct BulkArgs {
    const int32_t* type;
    const int64_t* params;
    const int64_t* ts;
    int64_t n;
    int32_t n_params;
    int32_t ts_sorted;
    int32_t* status;
    int64_t* results;
    int32_t width;
    int32_t n_app;          // append tables in the context
    const DevType* types;   // [GPUTX_MAX_TYPES]
    int64_t* rowcount;      // [GTX_MAX_APPEND] device row counts of append tables
    const int64_t* capacity;// [GTX_MAX_APPEND]
    gputx_bulk_stats* stats;
    int64_t mcap;           // operation capacity of the workspace
    int32_t key_passes;     // digits of the item-key sort
    int32_t part_passes;    // digits of the partition sort
    int64_t n_parts;        // partitions (sentinel id = n_parts)
    int32_t strategy;       // requested (GPUTX_AUTO ...)
    int32_t group_by_type;
    int64_t w0_bar, c_bar, d_bar;
    int32_t kset_narrow;
    int32_t grid_blocks;    // persistent grid size
    uint64_t spin_ticks;    // watchdog
    int32_t cell_bits;      // PART cell table: 1 << cell_bits slots
    int32_t cells_max;      // most cells one registered type's transaction lists
    int32_t prm_rows;       // PART LDS parameter rows: widest registered procedure
    int32_t rec_words;      // PART record size in int64 words: 1 + prm_rows, rounded up to even
    int32_t pipe_bits;      // pipelined PART cell table: 1 << pipe_bits slots
    int32_t part_pipeline;  // 1: k_part_pipe where it fits, 0: k_part_wave
    int32_t part_scan;      // 1: cellwise procedures run as per-cell map scans
    int32_t tpl_lanes;      // TPL: transactions per wave window (64: workgroup windows, 0: from n / (d + 1))
    uint32_t type_mask;     // registered types the bulk may hold (others are INVALID)
    int32_t long_part;      // PART: partitions this long get a workgroup, shorter a lane
    int32_t res_rows;       // PART LDS result rows: most results of a registered procedure
    int32_t part_early;     // 1: PART's sort and records run before the choice, beside the ranking
    Ws ws;
};

constexpr int kPrepBlocks = 1024;
constexpr int kPartLdsMax = 160 * 1024;  // dynamic LDS cap of one PART workgroup (gfx950: 160 KB per CU)
constexpr int kLongPart = 32;            // PART: shortest partition given a workgroup
constexpr int kScanItems = 8;
constexpr int kScanTile = GTX_BLOCK * kScanItems;
constexpr int kRankItems = 8;
constexpr int kRankTile = GTX_BLOCK * kRankItems;

// Phase boundaries of one bulk; mark() records a timing event when enabled.
enum Phase { PH_START, PH_ORDER, PH_PREPARE, PH_EMIT, PH_OPSORT, PH_RANK, PH_FEATURES,
             PH_PARTSORT, PH_PARTGATHER, PH_PART, PH_TPL, PH_KSET, PH_FINAL, PH_COUNT };
struct PhaseMarks {
    hipEvent_t* ev = nullptr;  // PH_COUNT events of this bulk, or null
    void mark(int p, hipStream_t s) const {
        if (ev) (void)hipEventRecord(ev[p], s);
    }
};

// A second stream for work that may overlap the ranking: the fork event is
// recorded on the bulk's stream, the join event on this one.
struct SideLane {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    hipEvent_t sorted = nullptr;  // the bulk's stream passed the item-key sort
};

// bulk generation (kernels_front.hip); with a side lane and a.part_early set,
// PART's partition sort and records run on it from the emission on, and the
// bulk's stream waits for them after the features
hipError_t launch_front(const BulkArgs& a, hipStream_t s, const PhaseMarks& pm,
                        const SideLane* side = nullptr);
// bulk generation without the timestamp constraint (Appendix G): validation,
// count scans and basic operations only (kernels_front.hip)
void launch_front_relaxed(const BulkArgs& a, hipStream_t s, const PhaseMarks& pm);
// execution without the timestamp constraint (kernels_exec.hip): TPL with
// 0/1 spin locks, or PART grouped by per-partition counters; serial_key[i]
// receives a key whose order is a serial order the execution is equivalent to
void launch_exec_relaxed(const BulkArgs& a, hipStream_t s, const PhaseMarks& pm, int64_t* serial_key);
// the lock and k-set executors' per-operation records (kernels_front.hip),
// gated on the choice
void launch_rank_full(const BulkArgs& a, hipStream_t s);
// execution (kernels_exec.hip)
void launch_exec(const BulkArgs& a, hipStream_t s, const PhaseMarks& pm);
// PART's stable sort of transactions by partition and the partition heads
// (kernels_exec.hip), gated on the choice; with a.part_early set they run
// ungated
void launch_part_sort(const BulkArgs& a, hipStream_t s);
// PART's records and the bulk's appended rows (k_part_gather), after the
// partition sort on the same stream
void launch_part_gather(const BulkArgs& a, hipStream_t s);
// zero-transaction bulk: reset state and publish statistics
void launch_empty(const BulkArgs& a, hipStream_t s);
// workgroups of the persistent executors that fit on one compute unit
int exec_resident_blocks_per_cu();
// LDS bytes of one PART workgroup for these arguments (one wave; pipelined)
size_t part_wave_lds(const BulkArgs& a);
size_t part_pipe_lds(const BulkArgs& a, int cw);
// one-time kernel attributes (large dynamic LDS for PART)
void exec_init_attributes(int dev);

}  // namespace gtx
