// Host interface of the stable LSD radix sort (sort.hip).
#pragma once
#include <algorithm>

#include "common.h"

namespace gtx {

struct SortPlan {
    int key_bytes;             // 4 (uint32 keys) or 8 (uint64 keys)
    void* keys[2];             // ping-pong key buffers; input in keys[0]
    uint32_t* vals[2];         // ping-pong values;     input in vals[0]
    uint32_t* hist;            // [8][256]
    uint32_t* status;          // sort_status_words(cap, npass) words
    uint32_t* ctrl;            // [16] tile tickets and a completion counter
    int64_t cap;               // most keys the buffers hold (grid size)
    const int64_t* count_dev;  // device key count, or nullptr: cap keys
    int npass;                 // digits sorted, low to high (1..8)
    const int32_t* gate;       // device flag: sort only when non-zero (nullptr: always)
    GtxState* st;              // bulk state: nothing runs after a bulk error
    uint64_t spin_ticks;       // look-back watchdog
    uint32_t* inv;             // optional [cap]: inv[value] = the pair's sorted position
                               // (values must be distinct and below cap)
};

int64_t sort_tiles(int64_t cap);
size_t sort_status_words(int64_t cap, int npass);

// Sort; the result is in keys[npass & 1] / vals[npass & 1].
void sort_pairs(const SortPlan& p, hipStream_t s);

}  // namespace gtx
