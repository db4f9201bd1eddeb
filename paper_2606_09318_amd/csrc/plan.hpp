// Host-side plan of one ranking call: recursion levels, ruler spacing per
// level and the workspace layout. Pure host code; no device is needed to
// build a plan, so workspace sizes can be queried anywhere.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "lr.h"

namespace lr {

constexpr uint32_t TILE = 4096;            // elements per compaction tile
constexpr uint32_t BASE_MAX_LIMIT = 16384; // one workgroup of 1024 lanes x 16 elements
constexpr size_t ALIGN = 256;

struct Plan {
    bool weighted = false;
    uint32_t levels = 0;                   // ruling-set levels before the base case
    uint32_t base_max = 0;
    uint64_t m[LR_MAX_LEVELS + 1] = {};
    uint32_t log2k[LR_MAX_LEVELS] = {};
    uint32_t lseed[LR_MAX_LEVELS] = {};
    uint32_t refill = 0;
    uint32_t ntiles[LR_MAX_LEVELS] = {};
    size_t rec_bytes = 0;                  // slot / record / result size (8 or 16)
    // workspace layout (byte offsets)
    size_t off_ctrl = 0;
    size_t off_slot[LR_MAX_LEVELS] = {};
    size_t off_eb[LR_MAX_LEVELS] = {};
    size_t off_tile[LR_MAX_LEVELS] = {};
    size_t off_batch_succ = 0, off_batch_desc = 0, off_batch_bases = 0;
    uint32_t batch_count = 0;
    size_t total = 0;
};

// Build the plan for n elements. batch_count > 0 adds the batch staging
// areas (concatenated successor array and request table).
lr_status make_plan(uint64_t n, bool weighted, const lr_opts* o, uint32_t batch_count, Plan* p);

// Base-case shared memory bytes for m elements.
inline size_t base_lds_bytes(uint64_t m, bool weighted) {
    return (size_t)m * (weighted ? 14 : 6) + 64;
}

}  // namespace lr
