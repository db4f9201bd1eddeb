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
constexpr uint32_t HEADSUM_BLOCKS = 2048;      // partial sums of the one-list head search
#ifndef LR_LOG_CHUNK
#define LR_LOG_CHUNK 1024
#endif
constexpr uint32_t LOG_CHUNK = LR_LOG_CHUNK;  // records per visit-log chunk
constexpr uint32_t LOG_MAX_WAVES = 8192;     // chase waves in log mode (caps the log slack)
#ifndef LR_LOG_MIN_LOG2
#define LR_LOG_MIN_LOG2 25
#endif
static_assert(LR_LOG_MIN_LOG2 >= 16 && LR_LOG_MIN_LOG2 <= 31, "visit-log threshold: 2^16 .. 2^31 elements");
constexpr uint64_t LOG_MIN_N = 1ull << LR_LOG_MIN_LOG2;  // smallest level 0 that uses the visit log
constexpr uint64_t LOG_FORCE_MIN_N = 1ull << 16;          // smallest level 0 LR_VISIT_LOG applies to
// Packed visit-log records (one 64-bit word) up to 2^28 elements: then the
// element field takes at most 29 bits and the walk field (walks plus
// continuations, fewer than 2^29) at most 29, which leaves the offset field
// at least LOG_BO_MIN bits. Larger inputs keep the wide 12-byte records.
constexpr uint64_t LOG_PACK_MAX_N = 1ull << 28;
constexpr uint32_t LOG_BO_MIN = 6;
#ifndef LR_PLACE_FINE_SHIFT
#define LR_PLACE_FINE_SHIFT 13
#endif
constexpr uint32_t PLACE_FINE_SHIFT = LR_PLACE_FINE_SHIFT;  // fine placement ranges of 8192 elements (LDS of one workgroup)
// bits of the grouping fan-out moved from the first pass to the second
// (unweighted / weighted records)
#ifndef LR_PLACE_COARSE_BIAS
#define LR_PLACE_COARSE_BIAS 1
#endif
#ifndef LR_PLACE_COARSE_BIAS_W
#define LR_PLACE_COARSE_BIAS_W 2
#endif
// Grouping counters: every tile of the first pass reserves space in every
// coarse range, so each coarse range has two counters, a front one that fills
// the range upward and a back one that fills it downward (even tiles take the
// front, odd tiles the back), each on a 128 B line of its own: atomics on one
// line are serialised, and packed counters made the first pass wait on them.
// The fine ranges' counters follow, packed (few tiles reach each of them).
constexpr uint32_t FILL_LINE = 32;
inline uint64_t fill_words(uint32_t nb1, uint32_t nb2) { return 2ull * nb1 * FILL_LINE + nb2; }
constexpr uint32_t LOCAL_SHIFT = 12;         // tile-local contraction: tiles of 4096 consecutive ids
constexpr uint32_t LOCAL_TILE = 1u << LOCAL_SHIFT;
// automatic contraction: considered from this size on; the contracted levels
// hold at most LR_LOCAL_AUTO_16THS / 16 of the elements
constexpr uint64_t LOCAL_AUTO_MIN_N = 1ull << 21;
#ifndef LR_LOCAL_AUTO_16THS
#define LR_LOCAL_AUTO_16THS 5
#endif
constexpr uint64_t local_auto_cap(uint64_t n) { return (n * LR_LOCAL_AUTO_16THS + 15) / 16; }
// the choice is a guess from every LOCAL_SAMPLE_STRIDE-th tile, taken when the
// extrapolated contracted list is at most LR_LOCAL_GUESS_16THS / 16 of the
// elements (below the capacity, so a wrong guess is rare; the contracted
// path checks the exact size and falls back to the plain path)
constexpr uint32_t LOCAL_SAMPLE_STRIDE = 16;
#ifndef LR_LOCAL_GUESS_16THS
#define LR_LOCAL_GUESS_16THS 4
#endif
constexpr uint64_t local_guess_cap(uint64_t n) { return n * LR_LOCAL_GUESS_16THS / 16; }
// ruler spawning: default sampling spacing k of the input level, the cap of
// its walks in multiples of k, and the spacing k2 (a power of two) at which
// rulers are spawned among the elements the capped walks left
#ifndef LR_SPAWN_K0
#define LR_SPAWN_K0 32
#endif
constexpr uint32_t SPAWN_K0 = LR_SPAWN_K0;
#ifndef LR_SPAWN_CAP
#define LR_SPAWN_CAP 2
#endif
#ifndef LR_SPAWN_K2
#define LR_SPAWN_K2 4
#endif
static_assert((LR_SPAWN_K2 & (LR_SPAWN_K2 - 1)) == 0, "k2 is a power of two");
// grouping tiles: lanes x LR_PLACE_PER records (half as many weighted); the
// passes whose records carry roots or weights use wider workgroups (measured
// faster there, slower for plain ranks)
// Debug builds (LR_DEBUG_WRITES=1, a separate library): the plain path counts
// the writes to every slot and predecessor mark of every level that writes
// them at the element's address, and a call returns LR_ERR_BAD_LIST unless
// every slot was written exactly once and every mark at most once.
#ifndef LR_DEBUG_WRITES
#define LR_DEBUG_WRITES 0
#endif

#ifndef LR_PLACE_TPB
#define LR_PLACE_TPB 512
#endif
#ifndef LR_PLACE_TPB_ROOT
#define LR_PLACE_TPB_ROOT 1024
#endif
#ifndef LR_PLACE_PER
#define LR_PLACE_PER 8
#endif
constexpr int place_tpb(bool weighted, bool root) { return (weighted || root) ? LR_PLACE_TPB_ROOT : LR_PLACE_TPB; }
constexpr uint32_t place_tile_records(bool weighted, bool root) {
    return (weighted ? LR_PLACE_PER / 2 : LR_PLACE_PER) * (uint32_t)place_tpb(weighted, root);
}

// Compile-time limits of the tuning overrides above, so a variant built with
// -DNAME=VALUE that cannot launch fails here and not at run time. LDS: gfx950
// gives one workgroup at most 160 KiB. A grouping tile holds T records (4 B
// element + 4 B rank [+ 4 B root] [+ 8 B sum]) and two 4 B counters per range
// of its pass; the plan keeps every pass at most 2^11 ranges (split of the
// fan-out over two passes up to 2^31 elements).
constexpr size_t LDS_MAX = 160 * 1024;
constexpr uint32_t PLACE_MAX_RANGES = 1u << 11;
constexpr size_t place_tile_lds(bool weighted, bool root) {
    return (size_t)place_tile_records(weighted, root) * (8 + (root ? 4 : 0) + (weighted ? 8 : 0)) + 8 +
           8 * (size_t)PLACE_MAX_RANGES;
}
static_assert(LR_PLACE_TPB % 64 == 0 && LR_PLACE_TPB >= 64 && LR_PLACE_TPB <= 1024, "grouping workgroup width");
static_assert(LR_PLACE_TPB_ROOT % 64 == 0 && LR_PLACE_TPB_ROOT >= 64 && LR_PLACE_TPB_ROOT <= 1024,
              "grouping workgroup width (roots, weights)");
static_assert(LR_PLACE_PER >= 2 && LR_PLACE_PER % 2 == 0, "records per lane (halved for weighted records)");
static_assert(place_tile_lds(false, false) <= LDS_MAX && place_tile_lds(false, true) <= LDS_MAX &&
                  place_tile_lds(true, false) <= LDS_MAX && place_tile_lds(true, true) <= LDS_MAX,
              "a grouping tile must fit one workgroup's LDS: lower LR_PLACE_PER or the workgroup width");
static_assert(PLACE_FINE_SHIFT >= 10 && ((size_t)1 << PLACE_FINE_SHIFT) * 16 <= LDS_MAX,
              "a fine placement range (4 B rank + 4 B root + 8 B sum per id) must fit one workgroup's LDS");
static_assert(LOG_CHUNK >= 256 && (LOG_CHUNK & (LOG_CHUNK - 1)) == 0,
              "a visit-log chunk takes at least two steps of a wavefront (64 walks x 2 per lane)");
static_assert(LR_LOCAL_GUESS_16THS <= LR_LOCAL_AUTO_16THS && LR_LOCAL_AUTO_16THS <= 16,
              "the contracted path's guess threshold lies within its capacity");
static_assert(LR_SPAWN_K0 >= 2 && LR_SPAWN_K0 <= 4096 && (LR_SPAWN_K0 & (LR_SPAWN_K0 - 1)) == 0 &&
                  LR_SPAWN_CAP >= 1 && LR_SPAWN_K2 >= 2,
              "spawning spacing and cap");
static_assert(LR_PLACE_COARSE_BIAS <= 4 && LR_PLACE_COARSE_BIAS_W <= 4, "fan-out bias");

// Batches: the concatenation is cut into chunks of BATCH_CHUNK ids that never
// cross a request, each reducing its request's head sum; the host uploads the
// request bases and each request's first chunk (two tables of count + 1).
constexpr uint32_t BATCH_CHUNK = 4096;
constexpr uint32_t BATCH_ARG_DESC = 96;  // request descriptors passed by value per table-writer launch
inline size_t batch_table_bytes(uint32_t count) { return 2 * ((size_t)count + 1) * 4; }

struct Plan {
    bool weighted = false;
    uint32_t levels = 0;                   // ruling-set levels before the base case
    uint32_t base_max = 0;
    uint64_t m[LR_MAX_LEVELS + 1] = {};
    uint32_t log2k[LR_MAX_LEVELS] = {};
    uint32_t lseed[LR_MAX_LEVELS] = {};
    uint32_t refill = 0;
    uint32_t lane_walks = 1;               // level-0 chase: walks held per lane (1 or 2)
    uint32_t ntiles[LR_MAX_LEVELS] = {};
    size_t rec_bytes = 0;                  // slot / record / result size (8 or 16)
    // workspace layout (byte offsets)
    size_t off_ctrl = 0;
    size_t off_hsum = 0;                   // HEADSUM_BLOCKS x 16 B partial sums
    size_t off_fb = 0;                     // the bounded fallback's two record arrays (over every path's
                                           // arrays, which are dead when it runs)
    size_t off_slot[LR_MAX_LEVELS] = {};
    size_t off_eb[LR_MAX_LEVELS] = {};
    size_t off_tile[LR_MAX_LEVELS] = {};
    size_t off_batch_succ = 0, off_batch_desc = 0, off_batch_bases = 0;  // bases: then the chunk offsets
    size_t off_batch_hdr = 0;
    size_t off_batch_part = 0, off_batch_sums = 0;  // per chunk, per request: (head sum, terminals)
    // level 0 in log mode: the chase appends (element, walk, offset) records to
    // a chunked visit log instead of storing at random addresses; after the
    // recursion the records are resolved and grouped by element range in two
    // passes (ranges of 2^s1, then 2^s2 ids) and written range by range from
    // LDS. The fine-grouped records reuse the log arrays.
    bool log0 = false;
    bool pack = false;       // packed records; else wide
    uint32_t ccap = 0;       // packed: continuation entries
    uint32_t bocap = 31;     // packed: most offset bits per record
    size_t off_conts = 0;    // packed: continuation entries, 8 B each
    uint32_t chunk = 0, max_chunks = 0, s1 = 0, s2 = 0, nb1 = 0, nb2 = 0;
    size_t off_log[4] = {}, off_p[4] = {}, off_fill = 0;  // fill: nb1 then nb2 counters
    uint32_t batch_count = 0;
    // tile-local contraction (LR_LOCAL): the ruling-set levels run on the
    // contracted list, whose size is known only on the device; m[] are then
    // capacities (m[0] = n) and the kernels read the actual sizes from Ctrl.
    bool local = false;
    uint64_t lc_n = 0;       // input elements (m[0] is the contracted list's capacity)
    uint32_t lc_ntiles = 0;
    size_t off_lc_cnt = 0;   // lc_ntiles + 1 start counts, scanned in place
    size_t off_lc_dir = 0;   // per 32 ids: start bits and starts before the word in its tile
    size_t off_lc_pos = 0;   // per element: chain start (compact, tile-relative) << 16 | distance
    size_t off_lc_wd = 0;    // per element: weight from its chain start (weighted only)
    size_t off_lc_stage = 0; // contracted records at their tile's offset, before compaction
    size_t off_lrec = 0;     // contracted records, then their results
    // ruler spawning (LR_SPAWN): the input level is a chase whose lanes spawn
    // rulers; its walks form the contracted list (records at off_lrec, at
    // most n of them: m[0] = n), which the levels above rank
    bool spawn = false;
    uint64_t sp_n = 0;       // input elements
    uint32_t sp_log2k = 0, sp_seed = 0;  // input level sampling
    uint32_t sp_ntiles = 0;  // head-compaction tiles of the input
    size_t off_sp_slot = 0;  // per element: walk id (flagged for spawned rulers) and offset
    size_t off_sp_hp = 0;    // per element: has-a-predecessor byte
    size_t off_sp_tile = 0;  // head counts per tile, scanned in place
    size_t off_dbg = 0;      // debug builds: per level, slot then mark write counters (4 B each)
    size_t total = 0;
};

// The plans of one call: p runs alone, or, with automatic contraction
// (autol), p is the plain path and lp the contracted path over the same
// workspace (common header: control block and head-sum partials).
struct PlanSet {
    Plan p;
    Plan lp;
    bool autol = false;
};

// Build the plans for n elements. batch_count > 0 adds the batch staging
// areas (concatenated successor array and request table).
lr_status make_plans(uint64_t n, bool weighted, const lr_opts* o, uint32_t batch_count, PlanSet* ps);
// The same, keeping only p (its total covers every path).
lr_status make_plan(uint64_t n, bool weighted, const lr_opts* o, uint32_t batch_count, Plan* p);

// Autotune cache (tune.cpp): fills o's plan options (spacing of the first
// two levels, base size, walks per lane, refill) from the entry of the
// current device, n's size bucket (floor(log2 n)) and weighted, if any.
bool tune_lookup(uint64_t n, bool weighted, lr_opts* o);

// Base-case shared memory bytes for m elements.
inline size_t base_lds_bytes(uint64_t m, bool weighted) {
    // one 8 B (count, successor) word per slot, 4096, 8192 or 16384 slots
    // (whole columns of the 1024-lane workgroup), weighted with an 8 B sum
    // per slot as well; weighted levels above 8192 elements: 8 B sum, 4 B
    // count and 2 B successor arrays
    const uint64_t slots = (m <= 4096) ? 4096 : (m <= 8192) ? 8192 : 16384;
    if (weighted) return m <= 8192 ? (size_t)slots * 16 + 64 : (size_t)m * 14 + 64;
    return (size_t)(m > slots ? m : slots) * 8 + 64;
}

}  // namespace lr
