/*
 * lr.h -- C ABI of the MI355X (gfx950) list-ranking library (liblr.so).
 *
 * Problem (Section 1.1 of "Engineering Scalable Distributed List Ranking"):
 * a successor array succ[0..n) describes a forest of singly linked lists; a
 * terminal element points to itself, an initial element has no predecessor.
 * For every element i the library computes
 *   root[i] = the terminal of i's list (the paper "identifies i with i_term"),
 *   rank[i] = the number of links followed from i to reach root[i],
 *   sum[i]  = the weighted rank: the sum of the link weights w[j] over the
 *             elements j on the path from i to root[i], root excluded (the
 *             terminal has no outgoing link, so its weight never counts).
 * The paper's in-place convention (succ becomes the terminal, rank goes from
 * weight to weighted rank) is replaced by const inputs and separate outputs.
 *
 * Method: sparse ruling set (Section 2.1, Fig. 1): rulers are sampled, every
 * ruler and every initial element walks the list to the next ruler or to a
 * terminal, the rulers form a smaller weighted instance that is solved
 * recursively down to a pointer-doubling base case (Wyllie), and every element
 * then takes its rank from the walk that reached it.
 *
 * Conventions shared by every entry point:
 *   - All array pointers are DEVICE pointers owned by the caller. Inputs are
 *     never written; requested outputs are fully overwritten.
 *   - `ws` is caller-owned device workspace of at least the size the matching
 *     *_workspace_bytes call reports. The library allocates no device memory
 *     in these calls. A workspace must not be used by two calls that may run
 *     at the same time.
 *   - `stream` is a hipStream_t (NULL = the default stream). Calls only
 *     enqueue work and return; results are valid once the stream reaches that
 *     point (event or stream synchronisation). Without LR_VALIDATE no call
 *     synchronises, so a call can be captured into a HIP graph.
 *   - Indices and ranks are uint32; n must be below 2^31.
 *   - Without LR_VALIDATE, input that is not a forest of lists (an index out
 *     of range, two predecessors, a cycle) gives unspecified outputs but never
 *     an out-of-bounds access or a non-terminating kernel. With LR_VALIDATE
 *     the call checks the input and the result on the device, synchronises the
 *     stream, and returns LR_ERR_BAD_LIST for such input.
 *   - Errors are returned as lr_status; nothing is thrown across the ABI.
 *
 * Debug build: the same sources built with LR_DEBUG_WRITES=1 (liblr_debug.so)
 * export the same functions. There lr_rank and lr_prefix_sum count the writes
 * of every store that relies on a single writer (a walk's slot per visited
 * element, a predecessor mark per element), synchronise, and return
 * LR_ERR_BAD_LIST unless every slot was written exactly once and every mark
 * at most once, also without LR_VALIDATE. Their workspaces are larger
 * (*_workspace_bytes of that library), automatic contraction is off, and
 * calls must not run on several streams at once.
 */
#ifndef LR_H
#define LR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lr_status {
    LR_OK = 0,
    LR_ERR_INVALID_ARG = 1,   /* null required pointer, bad enum, bad option */
    LR_ERR_UNSUPPORTED = 2,   /* n >= 2^31, or an option the device cannot run */
    LR_ERR_WORKSPACE = 3,     /* ws NULL or smaller than required */
    LR_ERR_OUT_OF_MEMORY = 4, /* server creation could not allocate its pool */
    LR_ERR_BAD_LIST = 5,      /* LR_VALIDATE found input that is not a forest of lists */
    LR_ERR_HIP = 6            /* a HIP runtime call failed */
} lr_status;

/* Element type of the weight array of lr_prefix_sum. */
typedef enum lr_wtype {
    LR_W_NONE = 0,  /* no weight array: every link weighs 1 (sum == rank) */
    LR_W_I32 = 1,   /* int32 weights, widened to int64 */
    LR_W_I64 = 2    /* int64 weights */
} lr_wtype;

enum {
    LR_VALIDATE = 1u,  /* check input and result; synchronises the stream */
    LR_PROFILE = 2u,   /* record per-phase times, read with lr_profile_last */
    LR_LOCAL = 4u,     /* always contract tile-local chains first (Section 2.3) */
    LR_NO_LOCAL = 8u,  /* never contract tile-local chains */
    LR_SPAWN = 16u,    /* first level with ruler spawning (Section 2.2); not with LR_LOCAL */
    LR_VISIT_LOG = 32u /* first level through the visit log even below 2^25 elements
                          (inputs of at least 2^16); a tuning and testing option */
};
/* Visit log: on inputs of 2^25 elements or more the first level's chase does
 * not store each element's walk and offset at the element (one random store
 * per element) but appends them to per-wavefront logs written in whole lines;
 * two grouping passes then bring every record to its element's range, and
 * the outputs are written range by range. Below 2^25 the random stores are
 * cheaper (the arrays are small enough for the caches to absorb them). Up to
 * 2^28 elements a record is one 64-bit word (element, walk, offset; a walk
 * whose offset outgrows its field goes on under a continuation id, see
 * log_off_bits), above 2^28 three 32-bit words. */
/* Walk cap and bounded fallback: how long a walk runs depends on where the
 * next sampled ruler sits in list order (Section 2.2: the longest sublist
 * decides the number of rounds). On an order unrelated to the sampling the
 * walks at spacing k are about geometric with mean k; an order built against
 * the sampling (every sampled ruler placed after all other elements, say)
 * would make one walk cover almost the whole list. Every walk therefore
 * stops after 64 k steps; if any does, the call ranks its input by pointer
 * doubling with J-fold jumps per round (J = 128 up to 2^21 elements, at most
 * 3 rounds; J = 16 above, at most 8 rounds), independent of the order, with
 * identical results. The fallback's kernels are enqueued with every call and
 * return at once when no walk was capped (a few microseconds per call);
 * lr_profile_last reports whether it ran. Under LR_VALIDATE a cycle reached
 * by a walk is reported through the same fallback. */
/* Ruler spawning (Section 2.2): the first level is chased in two rounds. The
 * walks of the sampled rulers and heads stop after 2k steps, each marking the
 * element it would have taken next; then new rulers are spawned at every such
 * element and, at a rate of 1/4, at the elements no walk has reached, and
 * their walks finish the list. This cuts the long stretches between sampled
 * rulers that decide how long a chase runs. The walks of both rounds form a
 * list, numbered and sized on the device, which the ruling-set levels rank;
 * spacing[0] is then the first level's sampling spacing k and spacing[1..]
 * the spacings of the levels above (0 = defaults). No element is claimed
 * atomically and the walks do not depend on timing; results are identical to
 * the default path. On MI355X the extra passes cost about what the shorter
 * chase saves (slower below 2^22 elements, within a few percent from 2^22 to
 * 2^25), so it is an option, not a default. */
/* Tile-local contraction (Section 2.3): chains of links that stay inside a
 * tile of 4096 consecutive ids are contracted to their first element, the
 * ruling-set levels rank the contracted list, and every element then takes
 * its rank from its chain's first element. It pays off when most links are
 * local (a list stored mostly in list order) and costs extra passes when few
 * are. By default (neither flag) inputs of 2^21 elements or more choose on
 * the device: the local links of every 16th tile are counted, and the
 * contracted path runs when they extrapolate to a contracted list of at most
 * 4/16 of the elements (at least 75% of the links local). The contracted path
 * counts its list exactly and, if it holds more than 5/16 of the elements
 * (the most its workspace takes), hands over to the plain path on the
 * device. Nothing is synchronised: both paths are enqueued and the one not
 * taken returns at once. Results are identical in every mode. Applies to
 * lr_rank, lr_prefix_sum and lr_rank_batch. */

#define LR_MAX_LEVELS 8

/* Options; a NULL lr_opts* means all defaults. */
typedef struct lr_opts {
    uint64_t seed;                     /* seed of the ruler sampling hash */
    uint32_t flags;                    /* LR_VALIDATE | LR_PROFILE | LR_LOCAL |
                                          LR_NO_LOCAL | LR_SPAWN | LR_VISIT_LOG */
    uint32_t base_max;                 /* largest level solved by the one-workgroup
                                          base case; 0 = default (8192 unweighted,
                                          4096 weighted) */
    uint32_t spacing[LR_MAX_LEVELS];   /* ruler spacing k per recursion level: one
                                          ruler per k consecutive ids; powers of
                                          two in [2, 4096]; the list ends at the
                                          first 0. spacing[0] == 0 = planner
                                          default. Levels are added with the
                                          default spacing until the last level
                                          fits base_max. */
    uint32_t refill;                   /* chase: idle walk slots of a wavefront
                                          that trigger taking new walks
                                          (1 .. 64 x lane_walks); 0 = default (1) */
    uint32_t lane_walks;               /* level-0 chase: walks each lane holds at
                                          once (1 or 2); 0 = default (1) */
    uint32_t log_off_bits;             /* visit log of up to 2^28 elements (one
                                          64-bit record per visit: element,
                                          walk, offset): the most bits of the
                                          offset field, 1 .. 31; 0 = as many as
                                          fit. A walk whose offset outgrows the
                                          field goes on under a continuation
                                          id; smaller values only make that
                                          more frequent (results are the same) */
} lr_opts;

/* The plan a call will follow (host-only query, no device needed). */
typedef struct lr_plan {
    uint32_t levels;                   /* ruling-set levels before the base case */
    uint32_t base_max;
    uint64_t m[LR_MAX_LEVELS + 1];     /* elements per level; m[0] = n,
                                          m[l+1] = ceil(m[l] / spacing[l]) */
    uint32_t spacing[LR_MAX_LEVELS];
    uint64_t workspace_bytes;
} lr_plan;

/* Fill *out with the plan for n elements (LR_W_NONE = lr_rank). Host only. */
lr_status lr_plan_query(uint64_t n, lr_wtype w, const lr_opts* opts, lr_plan* out);

/* Workspace bytes for n elements with these options: w == LR_W_NONE sizes an
 * lr_rank call, LR_W_I32 / LR_W_I64 an lr_prefix_sum call (the same size for
 * both, and also for lr_prefix_sum without weights). Host only; returns 0
 * for invalid arguments. */
size_t lr_workspace_bytes(uint64_t n, lr_wtype w, const lr_opts* opts);

/* Unweighted list ranking (Section 1.1).
 *   succ  [n] uint32, input: successor array (succ[t] == t marks a terminal).
 *   rank  [n] uint32, output: links from i to its terminal. Required.
 *   root  [n] uint32, output: terminal of i's list. May be NULL.
 * n == 0 returns LR_OK and does nothing. */
lr_status lr_rank(const uint32_t* succ, uint32_t* rank, uint32_t* root, uint64_t n,
                  void* ws, size_t ws_bytes, const lr_opts* opts, void* stream);

/* Weighted list ranking = list prefix sums (Section 1.1, weighted problem).
 *   weight [n] int32 or int64 as `w` says (NULL iff w == LR_W_NONE); w[t] of a
 *          terminal t is ignored.
 *   sum    [n] int64, output: weighted rank (the suffix sum toward the
 *          terminal, terminal excluded). Required. The caller guarantees
 *          |sum| < 2^63.
 *   rank, root: as lr_rank, both may be NULL.
 * Head-anchored prefix sums follow: exclusive = sum[head] - sum[i]. */
lr_status lr_prefix_sum(const uint32_t* succ, const void* weight, lr_wtype w, int64_t* sum,
                        uint32_t* rank, uint32_t* root, uint64_t n,
                        void* ws, size_t ws_bytes, const lr_opts* opts, void* stream);

/* lr_rank without a caller workspace and without any allocation, for callers
 * that cannot allocate device memory (code under HIP graph capture, serving
 * loops that must not call hipMalloc, harnesses that forbid it). The
 * workspace is a static device array of LR_NOALLOC_SCRATCH_BYTES (128 MiB)
 * that each GPU the call runs on holds until the process ends; its device
 * address is looked up on the first call on a device. The call makes no
 * hipMalloc, hipFree or other allocating call.
 *   succ, rank, root, n, opts: as lr_rank. The stream must belong to the
 *   current device.
 * Limit: n whose lr_rank workspace (lr_workspace_bytes(n, LR_W_NONE, opts))
 * exceeds LR_NOALLOC_SCRATCH_BYTES returns LR_ERR_WORKSPACE and does
 * nothing; with default options that is n above 6,632,960 (about 2^22.7).
 * LR_PROFILE is rejected with LR_ERR_INVALID_ARG (profiling creates events).
 * Every call on one GPU uses the same array, and each call rewrites what it
 * reads: calls that may overlap on one GPU (other streams, other threads)
 * race and give unspecified results. Calls on one stream are ordered and
 * safe. */
#define LR_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
lr_status lr_rank_noalloc(const uint32_t* succ, uint32_t* rank, uint32_t* root, uint64_t n,
                          const lr_opts* opts, void* stream);

/* One unweighted ranking request of a batch. All pointers are device
 * pointers; rank is required, root may be NULL; root ids are local to the
 * request (in [0, n)). */
typedef struct lr_request {
    const uint32_t* succ;
    uint32_t* rank;
    uint32_t* root;
    uint64_t n;
} lr_request;

/* Workspace bytes for lr_rank_batch over these requests (host only). */
size_t lr_batch_workspace_bytes(const lr_request* reqs, uint32_t count, const lr_opts* opts);

/* Rank many independent requests in one pass: the requests are treated as one
 * forest over the concatenation of their index ranges (lists never cross
 * requests), so every kernel of the method runs once for the whole batch.
 * `reqs` is a HOST array of `count` descriptors; they reach the device as
 * kernel arguments (96 per launch of a small table-writing kernel), so the
 * array may be reused as soon as the call returns, the call never
 * synchronises (without LR_VALIDATE) and it can be captured into a HIP graph.
 * The sum of the n must be below 2^31.
 * Results are identical to ranking each request alone. When every request is
 * one list (exactly one terminal), each request's head comes from its own
 * streaming sum (the one-list test of Fig. 1's findInit, per request) and no
 * predecessor marks are computed; a batch with a forest among its requests
 * marks predecessors over the whole concatenation, which costs more. */
lr_status lr_rank_batch(const lr_request* reqs, uint32_t count,
                        void* ws, size_t ws_bytes, const lr_opts* opts, void* stream);

/* A batch captured once as a HIP graph and replayed with other requests.
 * The graph is planned for a capacity: at most max_requests requests and
 * max_elements elements in all per launch. Every launch writes the request
 * table on the device from kernel arguments (one small kernel per 96
 * requests) and replays the graph; its kernels read the actual sizes from
 * the device, so any requests within the capacity run with the same graph
 * and give the same results as lr_rank_batch (the plain path: no automatic
 * contraction). The graph is bound to the workspace given at creation (at
 * least lr_batch_graph_workspace_bytes); launches of one graph must not
 * overlap (stream-ordered launches on one stream are fine); device buffers
 * of the requests must stay valid until the launch completes. Options: no
 * LR_VALIDATE, LR_PROFILE, LR_SPAWN or LR_LOCAL (LR_ERR_INVALID_ARG). A
 * launch over the capacity returns LR_ERR_WORKSPACE; a request with a root
 * output on a graph created without want_root returns LR_ERR_INVALID_ARG.
 * Creation captures on a stream of its own and synchronises nothing else;
 * launches never synchronise. */
typedef struct lr_batch_graph lr_batch_graph;
typedef struct lr_batch_graph_config {
    uint64_t max_elements;   /* most elements over the requests of one launch (< 2^31) */
    uint32_t max_requests;   /* most requests of one launch */
    uint32_t want_root;      /* nonzero: requests may ask for root outputs */
    lr_opts opts;            /* ruler spacings, base size, seed, ... for every launch */
} lr_batch_graph_config;
size_t lr_batch_graph_workspace_bytes(const lr_batch_graph_config* cfg);
lr_status lr_batch_graph_create(const lr_batch_graph_config* cfg, void* ws, size_t ws_bytes, lr_batch_graph** out);
lr_status lr_batch_graph_launch(lr_batch_graph* g, const lr_request* reqs, uint32_t count, void* stream);
void lr_batch_graph_destroy(lr_batch_graph* g);

/* GPU baseline: Wyllie pointer doubling over the whole input (Section 1,
 * Section 2.6: pointer doubling, ceil(log2 n) rounds of
 * rank[i] += rank[succ[i]], succ[i] = succ[succ[i]]). Same outputs as
 * lr_rank / lr_prefix_sum. Workspace from lr_wyllie_workspace_bytes. */
size_t lr_wyllie_workspace_bytes(uint64_t n, lr_wtype w);
lr_status lr_rank_wyllie(const uint32_t* succ, uint32_t* rank, uint32_t* root, uint64_t n,
                         void* ws, size_t ws_bytes, void* stream);
lr_status lr_prefix_sum_wyllie(const uint32_t* succ, const void* weight, lr_wtype w, int64_t* sum,
                               uint32_t* rank, uint32_t* root, uint64_t n,
                               void* ws, size_t ws_bytes, void* stream);

/* Tree computations by the Euler-tour technique (the paper ranks Euler tours
 * of BFS trees as an input family, Section 3, and names tree algorithms as
 * the users of list ranking, Section 1). One lr_prefix_sum over the tour with
 * weight +1 on down arcs and -1 on up arcs gives, for every arc a, the number
 * of arcs (rank) and #down - #up (sum) from a to the end of the tour; depth,
 * preorder number and subtree size of every vertex follow from the values at
 * the vertex's two arcs (those of the tour's first arc are fixed by V: rank
 * 2V - 3, sum 1).
 *   succ  [m] uint32, m = 2(V-1): the tour as a successor array over its arcs
 *         (one list; its last arc is the terminal). Ignored when V == 1.
 *   down  [V] uint32: down[v] = id of the arc parent(v) -> v.
 *   up    [V] uint32: up[v] = id of the arc v -> parent(v). The root's entries
 *         of down and up are ignored.
 *   root  the root vertex (< V).
 *   depth    [V] uint32 output: edges from the root (root 0). May be NULL.
 *   preorder [V] uint32 output: position of v in the depth-first order the
 *         tour follows (root 0). May be NULL.
 *   size     [V] uint32 output: vertices in v's subtree (root V). May be NULL.
 * V <= 2^30. Workspace from lr_euler_tree_workspace_bytes (it holds the
 * weights, a (rank, sum) record per arc and an lr_prefix_sum workspace). With
 * LR_VALIDATE the call also checks that down/up name every arc exactly once
 * and that the tour is one list starting with rank 2V - 3 and sum 1
 * (LR_ERR_BAD_LIST otherwise); without it such
 * input gives unspecified outputs, never an out-of-bounds access. opts apply
 * to the inner lr_prefix_sum. */
size_t lr_euler_tree_workspace_bytes(uint64_t V, const lr_opts* opts);
lr_status lr_euler_tree(const uint32_t* succ, const uint32_t* down, const uint32_t* up, uint64_t V, uint32_t root,
                        uint32_t* depth, uint32_t* preorder, uint32_t* size,
                        void* ws, size_t ws_bytes, const lr_opts* opts, void* stream);

/* Plan autotuner (the paper fixes its ruler-count constants by a parameter
 * study, Section 3 "Methodology"; this does the same on the caller's input).
 * Times lr_rank (w == LR_W_NONE, weight NULL) or lr_prefix_sum (any other w)
 * on `succ` in three stages, each keeping the fastest so far and varying one
 * group: the ruler spacings of the first two levels (16..128 x 8..32), then
 * the base-case size, then walks per lane and the refill threshold. It keeps
 * `base`'s seed and flags other than LR_VALIDATE / LR_PROFILE, writes the
 * fastest option set to *best (its spacing list filled for every level) and
 * stores it in the autotune cache under (device, floor(log2 n), weighted):
 * every later call of this process on that device whose options leave
 * spacing[0], base_max, lane_walks and refill at 0 (NULL options included)
 * and do not ask for LR_SPAWN takes the cached entry; its results are the
 * same whatever the plan, but its workspace size may change, so query
 * *_workspace_bytes after tuning. The trial calls write their outputs to
 * the tail of `ws` (n x 4 B, weighted n x 8 B) and use the rest as their
 * workspace; candidates that do not fit are skipped (LR_ERR_WORKSPACE if
 * none fits). `ms` (may be NULL) receives up to `cap` timings, in the order
 * the candidates were tried; *tried (may be NULL) their number. Synchronises
 * `stream`. */
lr_status lr_autotune(const uint32_t* succ, const void* weight, lr_wtype w, uint64_t n, void* ws, size_t ws_bytes,
                      const lr_opts* base, lr_opts* best, double* ms, int cap, int* tried, void* stream);

/* The autotune cache (host memory, per process, thread-safe). Entries are
 * keyed by the device ("gfx950:256": architecture and compute units of the
 * device current at the first use; "none" without a device), the input size
 * bucket floor(log2 n) and whether the call is weighted.
 *   lr_autotune_arch: the device key lookups use.
 *   lr_autotune_cache_save / _load: a text file, one entry per line
 *     (arch log2n weighted k0 k1 base_max lane_walks refill ms); loading
 *     checks every value as the planner checks user options, adds or
 *     replaces entries, and changes nothing on LR_ERR_INVALID_ARG. */
const char* lr_autotune_arch(void);
int lr_autotune_cache_entries(void);
void lr_autotune_cache_clear(void);
lr_status lr_autotune_cache_save(const char* path);
lr_status lr_autotune_cache_load(const char* path);

/* Device-side check of a result (a debugging and serving aid, not part of
 * any ranking call): the local equations of Section 1.1's definition, each
 * element against its successor -- a terminal t has rank 0, root t and sum 0;
 * any other x has rank[x] = rank[succ x] + 1, root[x] = root[succ x] and
 * sum[x] = sum[succ x] + w[x]. On a forest of lists these have exactly one
 * solution, so LR_OK proves the given outputs exact (checked: the ones not
 * NULL; at least one of rank, root, sum). A cycle cannot satisfy them, so it
 * is reported; input with two predecessors of one element may pass (that is
 * LR_VALIDATE's check). weight as in lr_prefix_sum (only with sum; NULL with
 * LR_W_NONE means unit weights). ws: at least 512 bytes of device memory.
 * Returns LR_ERR_BAD_LIST when an equation fails. Synchronises `stream`. */
lr_status lr_verify(const uint32_t* succ, const void* weight, lr_wtype w, const uint32_t* rank,
                    const uint32_t* root, const int64_t* sum, uint64_t n, void* ws, size_t ws_bytes, void* stream);

/* Per-phase device times (milliseconds) of the last call made with
 * LR_PROFILE on this thread: [0] predecessor marks, [1] head compaction,
 * [2] level-0 chase, [3] upper levels, base case and their propagation,
 * [4] level-0 record resolution and first grouping pass (0 for inputs
 * without the visit log), [5] level-0 propagation to the outputs, [6] total,
 * [7] 1 if the call ran the bounded fallback (a walk reached its step cap,
 * see below), else 0 (read from the device: the workspace must still hold
 * the call's state). Synchronises on the recorded events. Returns the number
 * of values written. The phase times of a call that ran the fallback cover
 * the stopped ruling-set path; [6] then excludes the fallback's rounds. */
int lr_profile_last(double* ms, int cap);

/* Device calibration (diagnostic, not part of any ranking call): on the
 * current device, with `ws` as scratch (at least lr_calibrate_workspace_bytes,
 * about 4 GiB, contents destroyed), times 2^28 accesses of each kind and
 * writes up to `cap` rates to `out`: [0] streaming copy of 1 GiB (GB/s, read +
 * written bytes), [1] 4 B gathers at hashed positions of a 1 GiB array, [2] 8 B
 * stores into 1 GiB, [3] 8 B stores into 256 MiB, [4] 1 B stores into 256 MiB,
 * [5] bit sets (atomic OR) in a 32 MiB bitmap, [6] records (x, v) streamed
 * from two 1 GiB arrays and v stored at x, the x grouped by ranges of 2^15
 * ids and every range stored by the workgroups of one XCD (G accesses/s).
 * These are the
 * ceilings the ranking kernels' random accesses are measured against.
 * Synchronises `stream`. Returns the number of rates written, or a negative
 * lr_status. */
size_t lr_calibrate_workspace_bytes(void);
int lr_calibrate(void* ws, size_t ws_bytes, double* out, int cap, void* stream);

/* Human-readable name of a status code (static storage). */
const char* lr_status_string(lr_status s);

/* ------------------------------------------------------------- serving ----
 * Continuous batching (project-defined; the paper has no serving layer).
 * A server owns `hbm_budget` bytes of device workspace split across
 * `max_inflight` batch slots, each with its own stream. Submitted requests
 * wait in FIFO order; whenever a slot is free, the waiting requests whose
 * workspace fits in the slot are launched together as one lr_rank_batch, so
 * requests arriving while other batches run join the next batch and their
 * work overlaps on the device. A request whose workspace can never fit a slot
 * is rejected with LR_ERR_WORKSPACE; a batch that fails fails only its own
 * requests. */
typedef struct lr_server lr_server;

typedef struct lr_server_config {
    uint64_t hbm_budget;      /* device workspace bytes the server allocates */
    uint32_t max_inflight;    /* concurrent batches (streams), >= 1 */
    uint32_t max_batch;       /* most requests per batch (1 = one launch per request) */
    lr_opts opts;             /* options for every batch */
    uint32_t graphs;          /* nonzero: a batch replays a captured lr_batch_graph of its
                                 size bucket (capacities 2^(j/2) elements from 2^16 on,
                                 max_batch requests; captured per slot when the server
                                 is created, those with root outputs on first use);
                                 batches whose bucket does not fit a slot, or options a
                                 graph cannot take, are enqueued as lr_rank_batch */
    uint32_t pad;
} lr_server_config;

lr_status lr_server_create(const lr_server_config* cfg, lr_server** out);
/* Enqueue a request (device buffers stay owned by the caller and must stay
 * valid until the ticket completes). */
lr_status lr_server_submit(lr_server* s, const lr_request* req, uint64_t* ticket);
/* 0 = pending, 1 = done (*status and *latency_s, seconds from submit to the
 * server observing completion, are filled; the submit time is taken when
 * lr_server_submit is entered, before any lock), -1 = unknown ticket. */
int lr_server_poll(lr_server* s, uint64_t ticket, lr_status* status, double* latency_s);
/* Block until every submitted request has completed. */
lr_status lr_server_drain(lr_server* s);
void lr_server_destroy(lr_server* s);

/* Replay a request trace through a server created from cfg: request i is
 * submitted at arrival_s[i] seconds after the start (host clock). Writes
 * each request's latency (scheduled arrival -> completion observed) to
 * latency_s[i] and the time
 * from the start to the last completion to *makespan_s; status[i] (may be
 * NULL) receives each request's status. */
lr_status lr_server_replay(const lr_server_config* cfg, const lr_request* reqs, const double* arrival_s,
                           uint32_t count, double* latency_s, lr_status* status, double* makespan_s);

#ifdef __cplusplus
}
#endif

#endif /* LR_H */
