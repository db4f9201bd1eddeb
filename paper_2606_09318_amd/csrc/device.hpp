// Device-side building blocks of the sparse ruling-set list ranker (gfx950).
//
// Data layout per recursion level l (m_l elements, S_l = m_{l+1} rulers):
//   slot_l[m_l]         walk id and offset of every element, written by the
//                       chase (the element's position inside its walk)
//   eb_l[S_l + m_l]     one record per walk. Entries [0, S_l) are the walks of
//                       the sampled rulers; after the chase they hold the
//                       elements of level l+1 (successor ruler + segment
//                       weight), after level l+1 is solved they hold its
//                       results (rank + root). Entries [S_l, ...) are the walks
//                       of initial elements that are not rulers; the compaction
//                       pass parks each such walk's start element in the entry's
//                       first word, the chase replaces it by the walk's end and
//                       weight, and the resolve pass by the walk's result.
//   hp_l[m_l] (bytes)   "has a predecessor" marks, aliased onto slot_l: they
//                       are read by the compaction pass before the chase of the
//                       same level overwrites slot_l.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lr {

constexpr uint32_t TERM = 0x80000000u;      // record flag: element is a terminal
constexpr uint32_t IDX = 0x7fffffffu;       // payload bits (ids are < 2^31)
constexpr uint32_t NONE = 0xffffffffu;
constexpr int MAXL = 8;

struct Ctrl {
    struct Lv { uint32_t H, q; } lv[MAXL];  // per level: #initial-element walks, chase queue head
    uint32_t err;                           // validation error bits
    uint32_t chunks;                        // visit-log chunks handed out (level 0, log mode)
    uint32_t nterm;                         // level 0: number of terminals (= number of lists)
    uint32_t single;                        // level 0: one list, whose head is known from hsum
    uint64_t hsum;                          // level 0: sum of ids minus sum of successors of non-terminals
    uint32_t dm[MAXL + 1];                  // element count per level when sizes are known only on the
                                            // device (the contracted list of tile-local contraction)
    uint32_t mode;                          // the path that runs (MODE_*): set by each path's first
                                            // kernels, MODE_FALLBACK once a walk reached its cap
    uint32_t multi;                         // plain path with more than one list: predecessor marks needed
    uint32_t spn;                           // ruler spawning: number of spawned rulers
    uint32_t conts;                         // packed visit log: continuation ids handed out
    uint32_t hc_done;                       // workgroups of a head-count kernel that have finished
    uint32_t pad[28];
};
static_assert(sizeof(Ctrl) == 256, "Ctrl layout");

// Device-side choice between enqueued kernel sequences: a kernel whose gate
// is set runs only when the word it points to (Ctrl.mode) holds `want`, and
// otherwise returns before touching memory. A null gate always runs.
struct Gate {
    const uint32_t* p;
    uint32_t want;
    __device__ __forceinline__ bool off() const { return p && *p != want; }
};

// Values of Ctrl.mode: the path whose kernels run. Each path's first kernels
// set it (the automatic choice between plain and contracted path included),
// and a walk that reaches its step cap turns it to MODE_FALLBACK, so every
// later kernel of the path returns and only the fallback runs.
enum : uint32_t { MODE_PLAIN = 0, MODE_LOCAL = 1, MODE_FALLBACK = 2, MODE_SPAWN = 3 };

// Ctrl.err bits (LR_VALIDATE): the input check sets ERR_INPUT (an index out
// of range, two predecessors); the ranking path's consistency checks set
// others; the fallback sets ERR_FALLBACK_CYCLE for a path that never reaches
// a terminal. After a fallback only ERR_INPUT and ERR_FALLBACK_CYCLE count:
// a path stopped by a cap leaves inconsistent state behind.
constexpr uint32_t ERR_INPUT = 1u | 2u;
constexpr uint32_t ERR_FALLBACK_CYCLE = 256u;
constexpr uint32_t ERR_DEBUG_WRITES = 512u;  // debug builds: a slot or mark with another write count

// Walk step cap: a walk at level spacing k stops after WALK_CAP_MULT * k
// steps. On a list whose order is independent of the sampling, walk lengths
// are about geometric with mean k, so R walks exceed the cap with
// probability about R * e^-64 (never, in practice); only an order built
// against the sampling reaches it. The fallback then ranks the input by
// pointer doubling, whose rounds do not depend on the order.
// A walk that outgrows its level (a cycle: input that is not a forest) is
// stopped the same way; the fallback then reports it under LR_VALIDATE.
// Spacings are at most 2^12, so the cap fits 32 bits.
constexpr uint32_t WALK_CAP_MULT = 64;
__device__ __forceinline__ uint32_t walk_cap(uint32_t m, uint32_t log2k) { return min(m, WALK_CAP_MULT << log2k); }

// Visit log of the level-0 chase (log mode): one record (element, walk,
// offset) per visited element, in one of two formats.
//   wide:   three 32-bit arrays x, w, c.
//   packed: one 64-bit word r = x << (bw + bo) | walk << bo | offset, field
//           widths from LogFmt. A walk whose offset outgrows its bo bits goes
//           on under a continuation id nw + j (nw = walks of the level), whose
//           entry cont[j] = (walk, offset where the continuation starts); the
//           offset field then counts from there. Continuation ids are handed
//           out in blocks of CONT_GRAB per wavefront.
// Weighted levels add the 64-bit weight sum s in both formats.
template <bool W>
struct LogArrays {
    uint32_t* x;
    uint32_t* w;
    uint32_t* c;
    int64_t* s;  // weighted levels only
    uint64_t* r;     // packed records
    uint2* cont;     // packed: continuation entries (walk, base offset)
    uint32_t ccap;   // packed: continuation entries available
    uint32_t bocap;  // packed: most offset bits a record may use
};

constexpr uint32_t CONT_GRAB = 128;  // continuation ids a wavefront takes at a time (>= its lanes' walks)

// Field widths of the packed visit log for n elements and nw walks: 2^bx > n,
// so an all-ones record (chunk padding) names no element; 2^bw > nw + ccap
// (walks and continuations); bo gets the rest of the 64 bits, at most bocap
// and 31. Chase and grouping derive the same widths from the same numbers.
struct LogFmt {
    uint32_t bx, bw, bo;
    __device__ __forceinline__ LogFmt(uint32_t n, uint32_t nw, uint32_t ccap, uint32_t bocap) {
        bx = 32u - (uint32_t)__clz((int)n);
        bw = 32u - (uint32_t)__clz((int)(nw + ccap));
        bo = min(64u - bx - bw, min(bocap, 31u));
    }
    __device__ __forceinline__ uint64_t pack(uint32_t x, uint32_t w, uint32_t o) const {
        return ((uint64_t)x << (bw + bo)) | ((uint64_t)w << bo) | o;
    }
    __device__ __forceinline__ uint32_t x(uint64_t r) const { return (uint32_t)(r >> (bw + bo)); }
    __device__ __forceinline__ uint32_t w(uint64_t r) const { return (uint32_t)(r >> bo) & ((1u << bw) - 1u); }
    __device__ __forceinline__ uint32_t o(uint64_t r) const { return (uint32_t)r & ((1u << bo) - 1u); }
};

// ---------------------------------------------------------------- values --
// Unweighted levels carry a link count; weighted levels carry (count, sum).
template <bool W> struct Lay;

template <> struct Lay<false> {
    struct Val { uint32_t c; };
    struct alignas(8) Slot { uint32_t w, c; };
    struct alignas(8) Rec { uint32_t nxt, c; };       // level element / walk end
    struct alignas(8) Res { uint32_t c, root; };      // solved rank + terminal id
    static __device__ __forceinline__ Val zero() { return {0u}; }
    static __device__ __forceinline__ Val one_link(int64_t) { return {1u}; }
    static __device__ __forceinline__ Val add(Val a, Val b) { return {a.c + b.c}; }
    static __device__ __forceinline__ Val sub(Val a, Val b) { return {a.c - b.c}; }
    static __device__ __forceinline__ Slot slot(uint32_t w, Val v) { return {w, v.c}; }
    static __device__ __forceinline__ Val val(Slot s) { return {s.c}; }
    static __device__ __forceinline__ Rec rec(uint32_t nxt, Val v) { return {nxt, v.c}; }
    static __device__ __forceinline__ Val val(Rec r) { return {r.c}; }
    static __device__ __forceinline__ Res res(Val v, uint32_t root) { return {v.c, root}; }
    static __device__ __forceinline__ Val val(Res r) { return {r.c}; }
    static __device__ __forceinline__ Val junk() { return {NONE}; }
};

template <> struct Lay<true> {
    struct Val { uint32_t c; int64_t s; };
    struct alignas(16) Slot { uint32_t w, c; int64_t s; };
    struct alignas(16) Rec { uint32_t nxt, c; int64_t s; };
    struct alignas(16) Res { uint32_t c, root; int64_t s; };
    static __device__ __forceinline__ Val zero() { return {0u, 0}; }
    static __device__ __forceinline__ Val one_link(int64_t w) { return {1u, w}; }
    static __device__ __forceinline__ Val add(Val a, Val b) { return {a.c + b.c, a.s + b.s}; }
    static __device__ __forceinline__ Val sub(Val a, Val b) { return {a.c - b.c, a.s - b.s}; }
    static __device__ __forceinline__ Slot slot(uint32_t w, Val v) { return {w, v.c, v.s}; }
    static __device__ __forceinline__ Val val(Slot s) { return {s.c, s.s}; }
    static __device__ __forceinline__ Rec rec(uint32_t nxt, Val v) { return {nxt, v.c, v.s}; }
    static __device__ __forceinline__ Val val(Rec r) { return {r.c, r.s}; }
    static __device__ __forceinline__ Res res(Val v, uint32_t root) { return {v.c, root, v.s}; }
    static __device__ __forceinline__ Val val(Res r) { return {r.c, r.s}; }
    static __device__ __forceinline__ Val junk() { return {NONE, INT64_MIN}; }
};

// ------------------------------------------------------------ sampling --
// Ruler sampling by strata: level l cuts its index range into blocks of
// k = 2^log2k consecutive ids and makes exactly one element of every block a
// ruler, at a position drawn by a hash of (level seed, block). This is the
// per-PE quota of Section 2.1 (r/p rulers drawn locally) taken down to blocks
// of k ids, so the ruler count of every level is exactly ceil(m / k), known
// before the data is read, and the ruler of block c has compact id c.
// Hash: "lowbias32" integer finaliser (C. Wellons, hash-prospector).
__device__ __forceinline__ uint32_t hash32(uint32_t seed, uint32_t x) {
    uint32_t h = (x * 0x9e3779b9u) ^ seed;
    h ^= h >> 16;
    h *= 0x7feb352du;
    h ^= h >> 15;
    h *= 0x846ca68bu;
    h ^= h >> 16;
    return h;
}

struct Sampler {
    uint32_t m, log2k, seed;
    __device__ __forceinline__ uint32_t pos(uint32_t blk) const {
        const uint32_t base = blk << log2k;
        const uint32_t k = 1u << log2k;
        const uint32_t len = (m - base < k) ? (m - base) : k;
        const uint32_t h = hash32(seed, blk);
        return (len == k) ? (h & (k - 1u)) : (h % len);
    }
    __device__ __forceinline__ bool sampled(uint32_t y) const {
        const uint32_t blk = y >> log2k;
        return (y - (blk << log2k)) == pos(blk);
    }
    __device__ __forceinline__ uint32_t start(uint32_t c) const { return (c << log2k) + pos(c); }
};

// --------------------------------------------------------------- sources --
// A source yields, for element x of a level, its successor (TERM | terminal
// id when x is a terminal) and its value: the link weight for a non-terminal,
// the terminal's own weight for a terminal (0 on the input level).
// Out-of-range successors are read as terminals, so no walk leaves the array.
template <bool W, int WT>  // WT: 0 = every link weighs 1, 1 = int32, 2 = int64, 3 = int8 weights (internal)
struct SrcIn {
    const uint32_t* succ;
    const void* weight;
    uint32_t m;
    using L = Lay<W>;
    static constexpr bool kLinks = true;  // every record is one link: a walk's count is its step count
    __device__ __forceinline__ void load(uint32_t x, uint32_t& nxt, typename L::Val& v) const {
        const uint32_t s = succ[x];
        int64_t w = 1;
        if constexpr (WT == 1) w = static_cast<const int32_t*>(weight)[x];
        if constexpr (WT == 3) w = static_cast<const int8_t*>(weight)[x];
        if constexpr (WT == 2) w = static_cast<const int64_t*>(weight)[x];
        const bool t = (s == x) | (s >= m);
        nxt = t ? (TERM | x) : s;
        v = t ? L::zero() : L::one_link(w);
    }
};

// The input's successor and weight interleaved into one record, so a chase
// step gathers one line instead of two (int32 weights: 8 B, int64: 16 B).
template <int WT> struct PairRec;
template <> struct alignas(8) PairRec<1> { uint32_t s; int32_t w; };
template <> struct alignas(16) PairRec<2> { uint32_t s, pad; int64_t w; };
template <> struct alignas(8) PairRec<3> { uint32_t s; int32_t w; };  // int8 weights, widened

template <int WT>
struct SrcPair {
    const PairRec<WT>* r;
    uint32_t m;
    using L = Lay<true>;
    static constexpr bool kLinks = true;
    __device__ __forceinline__ void load(uint32_t x, uint32_t& nxt, typename L::Val& v) const {
        const PairRec<WT> p = r[x];
        const bool t = (p.s == x) | (p.s >= m);
        nxt = t ? (TERM | x) : p.s;
        v = t ? L::zero() : L::one_link((int64_t)p.w);
    }
};

template <bool W>
struct SrcLvl {
    const typename Lay<W>::Rec* e;
    uint32_t m;
    using L = Lay<W>;
    static constexpr bool kLinks = false;  // records are segments: counts exceed step counts
    __device__ __forceinline__ void load(uint32_t x, uint32_t& nxt, typename L::Val& v) const {
        const typename L::Rec r = e[x];
        nxt = r.nxt;
        v = L::val(r);
        if (!(nxt & TERM) && nxt >= m) { nxt = TERM | IDX; v = L::zero(); }
    }
};

// --------------------------------------------------------------- outputs --
// Outputs take (element, value, root). A cursor lets an output keep state
// between consecutive elements of one lane (the batch output walks its
// request table forward instead of searching it per element).
// The caller's outputs. RK / RT say at compile time whether rank and root are
// written (the ranking kernels are instantiated per combination, so their
// store loops carry no branches); DYN checks the pointers at run time instead.
template <bool W, bool RK = true, bool RT = true, bool DYN = false>
struct OutUser {
    uint32_t* rank;
    uint32_t* root;
    int64_t* sum;
    using L = Lay<W>;
    struct Cur {};
    __device__ __forceinline__ Cur begin(uint32_t) const { return {}; }
    __device__ __forceinline__ void store(Cur&, uint32_t i, typename L::Val v, uint32_t r) const {
        if constexpr (DYN) {
            if (rank) rank[i] = v.c;
            if (root) root[i] = r;
            if constexpr (W) { if (sum) sum[i] = v.s; }
        } else {
            if constexpr (RK) rank[i] = v.c;
            if constexpr (RT) root[i] = r;
            if constexpr (W) sum[i] = v.s;
        }
    }
};

template <bool W>
struct OutLvl {
    typename Lay<W>::Res* e;
    using L = Lay<W>;
    struct Cur {};
    __device__ __forceinline__ Cur begin(uint32_t) const { return {}; }
    __device__ __forceinline__ void store(Cur&, uint32_t i, typename L::Val v, uint32_t r) const {
        e[i] = L::res(v, r);
    }
};

// Batch request table in device memory: bases[q] is the first global id of
// request q, bases[count] the total. The table is written on the device from
// descriptors passed by value as kernel arguments (no host staging, nothing
// for a graph replay to read from host memory); the header holds the sizes.
struct BatchDesc {
    const uint32_t* succ;
    uint32_t* rank;
    uint32_t* root;
    uint64_t n;
};
struct BatchHdr {
    uint32_t count;    // requests
    uint32_t nchunks;  // BATCH_CHUNK-id chunks over all requests (none crosses a request)
    uint32_t total;    // elements (= bases[count])
    uint32_t pad;
};

__device__ __forceinline__ uint32_t batch_find(const uint32_t* bases, uint32_t count, uint32_t g) {
    uint32_t lo = 0, hi = count;  // invariant: bases[lo] <= g < bases[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (bases[mid] <= g) lo = mid; else hi = mid;
    }
    return lo;
}

struct OutBatch {
    const BatchDesc* d;
    const uint32_t* bases;
    const BatchHdr* hdr;
    using L = Lay<false>;
    // the request holding the current element, with its output arrays
    struct Cur { uint32_t q, lo, hi, count; uint32_t* rank; uint32_t* root; };
    __device__ __forceinline__ Cur begin(uint32_t g) const {
        const uint32_t count = hdr->count;
        const uint32_t q = batch_find(bases, count, g);
        return {q, bases[q], bases[q + 1], count, d[q].rank, d[q].root};
    }
    __device__ __forceinline__ void store(Cur& c, uint32_t g, L::Val v, uint32_t r) const {
        if (g >= c.hi && c.q + 1 < c.count) {
            while (g >= c.hi && c.q + 1 < c.count) { c.q++; c.lo = c.hi; c.hi = bases[c.q + 1]; }
            c.rank = d[c.q].rank;
            c.root = d[c.q].root;
        }
        if (g >= c.hi) return;  // past the last request (cannot happen for ids below the total)
        const uint32_t l = g - c.lo;
        c.rank[l] = v.c;
        if (c.root) c.root[l] = r - c.lo;
    }
};

// ------------------------------------------------------------ wave utils --
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t mbcnt(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

}  // namespace lr
