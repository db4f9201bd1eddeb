// Host entry points into the kernel sequences (defined in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.hpp"
#include "plan.hpp"

namespace lr {

struct BatchDesc;
struct BatchHdr;

enum { EV_START, EV_DETECT, EV_HEADS, EV_CHASE0, EV_UPPER, EV_PART, EV_EXPAND, EV_COUNT };

struct RunArgs {
    const Plan* plan = nullptr;
    const Plan* lplan = nullptr;      // automatic contraction: the contracted path's plan (same workspace)
    const uint32_t* succ = nullptr;   // level-0 successor array (user's, or the batch concatenation)
    const void* weight = nullptr;
    int wt = 0;                       // 0: unit links, 1: int32, 2: int64
    uint32_t* rank = nullptr;
    uint32_t* root = nullptr;
    int64_t* sum = nullptr;
    // batch outputs (rank/root per request) instead of rank/root above
    const BatchDesc* desc = nullptr;
    const uint32_t* bases = nullptr;
    const uint32_t* boff = nullptr;   // batch: each request's first chunk (BATCH_CHUNK ids), count + 1 entries
    const BatchHdr* bhdr = nullptr;   // batch: the device table's header (request count, totals)
    uint32_t count = 0;               // batch: requests (with device-side sizes, the most a call takes)
    bool any_root = false;            // batch: some request wants roots
    bool dev_sizes = false;           // batch planned for a capacity: every level kernel reads the
                                      // actual sizes from Ctrl.dm (written by the table pass)
    char* ws = nullptr;
    hipStream_t stream = nullptr;
    bool validate = false;
    hipEvent_t* ev = nullptr;         // EV_COUNT events to record, or null
    void* rec = nullptr;              // weighted, internal callers: one (rank, root, sum) record per
                                      // element (Lay<true>::Res) instead of the separate arrays
    bool prologue = true;             // run validation and the head-sum pass (false: the caller did)
    Gate gate{};                      // device-side path selection (null: always run)
};

// Sparse ruling-set ranking over the whole plan. Enqueues only.
hipError_t run_srs(const RunArgs& a);

// Debug builds (LR_DEBUG_WRITES): set up and clear the write counters of a
// call before it, check them after it (Ctrl.err |= ERR_DEBUG_WRITES); no-ops
// in release builds.
hipError_t run_debug_begin(const RunArgs& a, const Plan& p);
hipError_t run_debug_check(const RunArgs& a, const Plan& p);

// Weighted ranking whose results land as one 16-byte (rank, root, sum)
// record per element at `rec` (the root field is not filled: NONE). Same
// arguments, workspace and checks as lr_prefix_sum otherwise, and one more
// weight type: wt = 3 for int8 weights.
lr_status prefix_sum_records(const uint32_t* succ, const void* weight, int wt, void* rec, uint64_t n, void* ws,
                             size_t ws_bytes, const lr_opts* opts, void* stream);

// Wyllie pointer doubling baseline; ws holds two ping-pong record arrays.
hipError_t run_wyllie(const RunArgs& a, uint64_t n, bool weighted);

// Batch staging, all on the device: the request table from descriptors passed
// as kernel arguments, its bases and chunk offsets (with dev_sizes also the
// level sizes in Ctrl.dm), then the requests' successor arrays copied into
// one forest over the concatenated id range (ids shifted by the request's
// base), chunk by chunk; each chunk also writes its request's partial head
// sum and terminal count. max_chunks bounds the chunks (grid size only).
hipError_t run_batch_table(const lr_request* reqs, uint32_t count, const Plan& p, char* ws, bool dev_sizes,
                           uint32_t max_chunks, hipStream_t st);

// Euler-tour arc weights by grouping (see kernels.hip); *done false: the
// caller scatters the weights itself.
hipError_t tree_arc_weights(const uint32_t* down, uint32_t V, uint32_t root, int8_t* w, uint32_t m, void* ws,
                            const lr_opts* opts, hipStream_t st, bool* done);

// Validation pass before ranking: range and in-degree check on the input.
hipError_t run_validate_input(const uint32_t* succ, uint32_t n, uint32_t* counts, uint32_t* err,
                              hipStream_t st);

// Result check: the local equations of the ranking on the device (err: one
// 32-bit word, cleared first; see k_verify for its bits).
hipError_t run_verify(const uint32_t* succ, const void* weight, int wt, const uint32_t* rank, const uint32_t* root,
                      const int64_t* sum, uint32_t n, uint32_t* err, hipStream_t st);

int device_cus();
size_t device_max_lds();

}  // namespace lr
