// Host runtime internals shared by the C-ABI implementation files.
#pragma once
#include <string>

#include "engine.h"

struct gputx_ctx {
    int device = 0;
    int ncu = 0;
    uint64_t wall_khz = 0;
    gputx_options opt{};
    struct Tab {
        bool present = false;
        gputx_table_desc d{};
        int app_idx = -1;
        uint32_t key_base = 0;
        int64_t part_base = -1;  // for root tables: first global partition id
    } tabs[GPUTX_MAX_TABLES];
    int n_app = 0;
    int app_table[GTX_MAX_APPEND] = {-1, -1, -1, -1};
    uint64_t total_items = 0;
    int key_passes = 1;
    int64_t n_parts = 0;
    int part_passes = 1;
    bool type_present[GPUTX_MAX_TYPES] = {};
    gputx_type_desc types[GPUTX_MAX_TYPES]{};
    int max_ops = 1;
    gtx::DevType* d_types = nullptr;
    int64_t* d_rowcount = nullptr;
    int64_t* d_capacity = nullptr;
    std::string err;
    // phase timing ring
    static constexpr int kRing = 256;
    bool timing = false;
    hipEvent_t* ev = nullptr;  // kRing * PH_COUNT
    int ring_used = 0;
    // second stream of the one-bulk form (PART's partition sort beside the ranking)
    gtx::SideLane side{};
};


// Record an error message on h (or thread-locally when h is null); returns code.
int gtx_set_err(gputx_handle h, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));

// Validate one bulk's arguments and fill its kernel arguments.
int gtx_make_args(gputx_handle h, const gputx_bulk* b, int strategy, void* workspace, size_t ws_bytes,
                  int32_t* status_out, int64_t* results_out, int32_t width, gputx_bulk_stats* stats,
                  int grid_blocks, gtx::BulkArgs* out);

// Persistent-grid size when `lanes` executors may run at once.
int gtx_grid_for(gputx_handle h, int lanes);

#define HIP_OK(h, call)                                                                         \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return gtx_set_err((h), GPUTX_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)
