// HIP kernels for gfx950 (wave64) and the launch sequences that chain them.
//
// Sparse ruling set (Section 2.1, Fig. 1), per level l of the recursion:
//   detect   (level 0 only) mark every element that has a predecessor;
//            unmarked elements are the initial elements (findInit).
//   heads    compact the initial elements that are not sampled rulers into a
//            walk list (tile count -> one-workgroup scan -> tile write).
//   chase    one lane per walk: from its start, follow succ and record in
//            slot[x] the walk id and the weight from the start to x, until the
//            next sampled ruler or a terminal (the ruler chasing loop). The
//            walk's end and total weight form the next level's element (for a
//            sampled ruler) or a parked record (for an initial element).
//   base     the last level (<= base_max elements) is ranked by pointer
//            doubling in LDS by one workgroup (the base case).
//   resolve  walks of initial elements take the result of the ruler (or
//            terminal) they ended on.
//   expand   every element takes rank = rank(walk) - offset and the walk's
//            root (ruler propagation).
// Walks run forward along succ, so ranks toward the terminal come out
// directly and no list reversal is needed.
//
// Level 0 of large inputs (n >= 2^25) logs the chase's visits and places the
// results by element range (place1/2/3) instead of storing at random
// addresses; with more than one list its predecessor marks are grouped by
// range the same way (mark1, place2 on ids, mark3), and weighted inputs are
// interleaved into one record per element first (pair).
//
// Tile-local contraction (Section 2.3): chains of links inside 4096-id tiles
// are contracted first (lc_chain, lc_scan, lc_compact), the levels above rank
// the contracted list with sizes read from the device, and lc_expand restores
// every element. By default a sample of the tiles chooses on the device
// between this path and the plain one (lsample, ldecide; the exact count in
// lc_scan can still hand over to the plain path); both are enqueued and the
// kernels of the path not taken return at once (Gate).
//
// Ruler spawning (Section 2.2, LR_SPAWN): the input level is chased in two
// rounds (sp_chase1 capped at 2k steps; sp_count/scan/write spawn rulers at
// the cap targets and among the unreached elements; sp_chase2 walks from
// them), and all walks form the list the levels above rank (run_clevels, as
// for the contracted list); sp_expand restores every element.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "device.hpp"
#include "runner.hpp"

namespace lr {

constexpr int TPB = 256;
#ifndef LR_CHASE_TPB
#define LR_CHASE_TPB 256
#endif
constexpr int CHASE_TPB = LR_CHASE_TPB;
constexpr int BASE_TPB = 1024;
constexpr int BASE_PER = BASE_MAX_LIMIT / BASE_TPB;  // 16 elements per lane
constexpr int EXPAND_CH = 8;                         // elements per lane per wave tile
#ifndef LR_CHASE_POOL
#define LR_CHASE_POOL 2   // sixteenths of a level's walks handed out from a shared pool at the end
#endif
constexpr uint32_t CHASE_GRAB = 64;  // walks a wavefront takes from the pool at a time
#ifndef LR_XCD_GROUPS
#define LR_XCD_GROUPS 1   // second grouping pass: the tiles of one coarse range on one XCD
#endif
static_assert(LR_XCD_GROUPS == 0 || LR_XCD_GROUPS == 1, "XCD grouping is on (1) or off (0)");
static_assert(CHASE_TPB % 64 == 0 && CHASE_TPB >= 64 && CHASE_TPB <= 1024, "chase workgroup width");
static_assert(LR_CHASE_POOL >= 0 && LR_CHASE_POOL < 16, "pool share of the walks, in sixteenths");

// ----------------------------------------------------------- debug writes --
// Debug builds (LR_DEBUG_WRITES): the stores that rely on having one writer
// per address (a slot per visited element, a predecessor mark per element)
// also count themselves, per level, into counters the call sets up; a check
// after the call wants every slot of a chased level written exactly once and
// every mark at most once. Null pointers (release builds, and calls outside
// the plain path) count nothing.
struct DbgWrites {
    uint32_t* slot[MAXL];
    uint32_t* mark[MAXL];
};
struct DbgSizes {
    uint32_t m[MAXL];
};
#if LR_DEBUG_WRITES
__device__ DbgWrites g_dbg;
#define LR_DBG_COUNT(kind, lvl, i)                  \
    do {                                            \
        uint32_t* c_ = g_dbg.kind[(lvl)];           \
        if (c_) atomicAdd(&c_[(i)], 1u);            \
    } while (0)
#else
#define LR_DBG_COUNT(kind, lvl, i) \
    do {                           \
    } while (0)
#endif

// ------------------------------------------------------------------ fill --
__global__ __launch_bounds__(TPB) void k_fill(uint32_t* __restrict__ p, uint64_t words, uint32_t val,
                                              const Ctrl* skip_if_single, Gate gate) {
    if (gate.off()) return;
    if (skip_if_single && skip_if_single->single) return;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t n4 = words / 4;
    uint4 v = make_uint4(val, val, val, val);
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
        reinterpret_cast<uint4*>(p)[i] = v;
    for (uint64_t i = n4 * 4 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride) p[i] = val;
}

// ---------------------------------------------------------------- detect --
// hp[succ[i]] = 1 for every non-terminal i. In a forest each element has at
// most one predecessor, so every byte has at most one writer and plain byte
// stores suffice (no atomics, no cross-XCD coherence traffic).
template <bool VEC>
__global__ __launch_bounds__(TPB) void k_detect(const uint32_t* __restrict__ succ, uint32_t m,
                                                uint8_t* __restrict__ hp, const Ctrl* ctrl, const uint32_t* dm,
                                                Gate gate) {
    if (gate.off()) return;
    if (ctrl->single) return;
    if (dm) m = dm[0];
    const uint32_t stride = gridDim.x * blockDim.x;
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t done = 0;
    if constexpr (VEC) {
        const uint32_t m4 = m / 4;
        for (uint32_t i = g; i < m4; i += stride) {
            const uint4 s = reinterpret_cast<const uint4*>(succ)[i];
            const uint32_t x = 4 * i;
            if (s.x != x && s.x < m) { hp[s.x] = 1; LR_DBG_COUNT(mark, 0, s.x); }
            if (s.y != x + 1 && s.y < m) { hp[s.y] = 1; LR_DBG_COUNT(mark, 0, s.y); }
            if (s.z != x + 2 && s.z < m) { hp[s.z] = 1; LR_DBG_COUNT(mark, 0, s.z); }
            if (s.w != x + 3 && s.w < m) { hp[s.w] = 1; LR_DBG_COUNT(mark, 0, s.w); }
        }
        done = m4 * 4;
    }
    for (uint32_t i = done + g; i < m; i += stride) {
        const uint32_t s = succ[i];
        if (s != i && s < m) {
            hp[s] = 1;
            LR_DBG_COUNT(mark, 0, s);
        }
    }
}

// One list shortcut for finding the initial elements. Every non-head element
// has exactly one predecessor, so over a forest
//   sum(all ids) - sum(succ[x] over non-terminals x) = sum of the heads,
// and the number of terminals is the number of lists. With one list this
// sum IS the head, found by one streaming reduction instead of a random
// store per element; the marking passes then do nothing.
template <bool VEC>
__global__ __launch_bounds__(TPB) void k_headsum(const uint32_t* __restrict__ succ, uint32_t m,
                                                 uint32_t* __restrict__ partial, Gate gate) {
    if (gate.off()) return;
    const uint32_t stride = gridDim.x * blockDim.x;
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t hs = 0;
    uint32_t nt = 0;
    auto one = [&](uint32_t x, uint32_t s) {
        if (s == x || s >= m) { ++nt; hs += x; }
        else hs += (uint64_t)x - s;
    };
    uint32_t done = 0;
    if constexpr (VEC) {
        const uint32_t m4 = m / 4;
        for (uint32_t i = g; i < m4; i += stride) {
            const uint4 s = reinterpret_cast<const uint4*>(succ)[i];
            one(4 * i, s.x);
            one(4 * i + 1, s.y);
            one(4 * i + 2, s.z);
            one(4 * i + 3, s.w);
        }
        done = m4 * 4;
    }
    for (uint32_t i = done + g; i < m; i += stride) one(i, succ[i]);
    __shared__ uint64_t shs[TPB / 64];
    __shared__ uint32_t snt[TPB / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        hs += __shfl_xor(hs, o);
        nt += __shfl_xor(nt, o);
    }
    if ((threadIdx.x & 63) == 0) { shs[threadIdx.x >> 6] = hs; snt[threadIdx.x >> 6] = nt; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < TPB / 64; ++i) { hs += shs[i]; nt += snt[i]; }
        partial[4 * blockIdx.x] = nt;
        partial[4 * blockIdx.x + 1] = 0;
        reinterpret_cast<uint64_t*>(partial)[2 * blockIdx.x + 1] = hs;
    }
}

// Automatic contraction, the guess: local links counted on every
// LOCAL_SAMPLE_STRIDE-th tile (one workgroup per sampled tile at a time);
// partial[4b] = local links, partial[4b + 1] = elements looked at.
template <bool VEC>
__global__ __launch_bounds__(TPB) void k_lsample(const uint32_t* __restrict__ succ, uint32_t m,
                                                 uint32_t* __restrict__ partial) {
    const uint32_t ntiles = (m + LOCAL_TILE - 1) / LOCAL_TILE;
    const uint32_t nsamp = (ntiles + LOCAL_SAMPLE_STRIDE - 1) / LOCAL_SAMPLE_STRIDE;
    uint32_t loc = 0, seen = 0;
    for (uint32_t q = blockIdx.x; q < nsamp; q += gridDim.x) {
        const uint32_t b = q * LOCAL_SAMPLE_STRIDE * LOCAL_TILE;
        const uint32_t len = min(LOCAL_TILE, m - b);
        for (uint32_t i = threadIdx.x; i < len; i += TPB) {
            const uint32_t s = succ[b + i];
            loc += s != b + i && s < m && (s >> LOCAL_SHIFT) == (b >> LOCAL_SHIFT);
        }
        seen += len;
    }
    __shared__ uint32_t sl[TPB / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) loc += __shfl_xor(loc, o);
    if ((threadIdx.x & 63) == 0) sl[threadIdx.x >> 6] = loc;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < TPB / 64; ++i) loc += sl[i];
        partial[4 * blockIdx.x] = loc;
        partial[4 * blockIdx.x + 1] = seen;
    }
}

// The guess: contract when the sampled tiles extrapolate to a contracted
// list of at most thr elements. The contracted path's scan checks the exact
// size against its capacity and falls back to the plain path if it is larger.
__global__ __launch_bounds__(TPB) void k_ldecide(const uint32_t* __restrict__ partial, uint32_t nparts, uint32_t m,
                                                 uint32_t thr, Ctrl* ctrl) {
    uint64_t loc = 0, seen = 0;
    for (uint32_t i = threadIdx.x; i < nparts; i += TPB) {
        loc += partial[4 * i];
        seen += partial[4 * i + 1];
    }
    __shared__ uint64_t sl[TPB / 64], ss[TPB / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        loc += __shfl_xor(loc, o);
        seen += __shfl_xor(seen, o);
    }
    if ((threadIdx.x & 63) == 0) { sl[threadIdx.x >> 6] = loc; ss[threadIdx.x >> 6] = seen; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < TPB / 64; ++i) { loc += sl[i]; seen += ss[i]; }
        const uint64_t est_local = seen ? loc * (uint64_t)m / seen : 0;
        ctrl->mode = (seen && (uint64_t)m - est_local <= thr) ? 1u : 0u;
        ctrl->single = 0;  // set by the plain path's head sum if that path runs
        ctrl->multi = 0;
    }
}

// Sums the partials (plain path). With exactly one terminal (and a head
// inside the range) it publishes the head as the level's only
// initial-element walk; multi says whether predecessor marks are needed.
__global__ __launch_bounds__(TPB) void k_headsum_final(const uint32_t* __restrict__ partial, uint32_t nparts,
                                                       Ctrl* ctrl, Sampler smp, char* __restrict__ eb, uint32_t S,
                                                       uint32_t rec_bytes, int lvl, uint32_t mode, Gate gate) {
    if (gate.off()) return;
    uint64_t hs = 0;
    uint32_t nt = 0;
    for (uint32_t i = threadIdx.x; i < nparts; i += TPB) {
        nt += partial[4 * i];
        hs += reinterpret_cast<const uint64_t*>(partial)[2 * i + 1];
    }
    __shared__ uint64_t shs[TPB / 64];
    __shared__ uint32_t snt[TPB / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        hs += __shfl_xor(hs, o);
        nt += __shfl_xor(nt, o);
    }
    if ((threadIdx.x & 63) == 0) { shs[threadIdx.x >> 6] = hs; snt[threadIdx.x >> 6] = nt; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < TPB / 64; ++i) { hs += shs[i]; nt += snt[i]; }
        ctrl->nterm = nt;
        ctrl->hsum = hs;
        ctrl->hc_done = 0;  // the head-count kernels' workgroup counter starts the call at zero
        if (mode != NONE) ctrl->mode = mode;
        const bool single = nt == 1 && hs < smp.m;
        ctrl->single = single ? 1u : 0u;
        ctrl->multi = single ? 0u : 1u;
        if (single) {
            const uint32_t h = (uint32_t)hs;
            uint32_t H = 0;
            if (!smp.sampled(h)) {
                *reinterpret_cast<uint32_t*>(eb + (size_t)S * rec_bytes) = h;
                H = 1;
            }
            ctrl->lv[lvl].H = H;
            ctrl->lv[lvl].q = 0;
            ctrl->chunks = 0;
            ctrl->conts = 0;
        }
    }
}

// Validation: counts[s]++ per link (counts zeroed before); any element with
// two predecessors or an out-of-range successor sets an error bit.
__global__ __launch_bounds__(TPB) void k_validate_in(const uint32_t* __restrict__ succ, uint32_t m,
                                                     uint32_t* __restrict__ counts, uint32_t* err) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
        const uint32_t s = succ[i];
        if (s >= m) { atomicOr(err, 1u); continue; }
        if (s != i && atomicAdd(&counts[s], 1u) != 0) atomicOr(err, 2u);
    }
}

// Result check (lr_verify): the local equations of the ranking, each
// element against its successor (one gather per output). err |= 1 for a
// successor out of range, 2 for a terminal whose values are not (0, itself,
// 0), 4 for an element whose values do not follow from its successor's.
template <int WT>
__global__ __launch_bounds__(TPB) void k_verify(const uint32_t* __restrict__ succ, const void* __restrict__ weight,
                                                const uint32_t* __restrict__ rank, const uint32_t* __restrict__ root,
                                                const int64_t* __restrict__ sum, uint32_t m, uint32_t* err) {
    const uint32_t stride = gridDim.x * blockDim.x;
    uint32_t bad = 0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
        const uint32_t s = succ[i];
        if (s >= m) { bad |= 1u; continue; }
        if (s == i) {
            if ((rank && rank[i] != 0) || (root && root[i] != i) || (sum && sum[i] != 0)) bad |= 2u;
            continue;
        }
        if (rank && rank[i] != rank[s] + 1u) bad |= 4u;
        if (root && root[i] != root[s]) bad |= 4u;
        if (sum) {
            int64_t w = 1;
            if constexpr (WT == 1) w = static_cast<const int32_t*>(weight)[i];
            if constexpr (WT == 2) w = static_cast<const int64_t*>(weight)[i];
            // two's complement wrap, as the prefix sums themselves
            if ((uint64_t)sum[i] != (uint64_t)sum[s] + (uint64_t)w) bad |= 4u;
        }
    }
    if (bad) atomicOr(err, bad);
}


// ----------------------------------------------------------------- heads --
// A tile of TILE elements per block: each lane owns 16 consecutive bytes of
// the hp bytemap. An element starts a walk of its own when it has no
// predecessor and is not the sampled ruler of its block.
__device__ __forceinline__ uint32_t tile_heads(const uint8_t* __restrict__ hp, const Sampler& smp, uint32_t x0,
                                               uint32_t& bits) {
    bits = 0;
    const uint32_t m = smp.m;
    if (x0 >= m) return 0;
    uint8_t b[16];
    if (x0 + 16 <= m) {
        const uint4 v = *reinterpret_cast<const uint4*>(hp + x0);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int j = 0; j < 16; ++j) b[j] = (uint8_t)(w[j >> 2] >> (8 * (j & 3)));
    } else {
#pragma unroll
        for (int j = 0; j < 16; ++j) b[j] = (x0 + j < m) ? hp[x0 + j] : 1;
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const uint32_t x = x0 + j;
        if (b[j] == 0 && x < m && !smp.sampled(x)) bits |= 1u << j;
    }
    return __popc(bits);
}

__device__ __forceinline__ uint32_t block_sum(uint32_t v, uint32_t* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const uint32_t wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[wv] = v;
    __syncthreads();
    uint32_t t = 0;
    for (uint32_t i = 0; i < blockDim.x / 64; ++i) t += sh[i];
    return t;
}

// Exclusive block scan (all lanes get their prefix; *total = block sum).
__device__ __forceinline__ uint32_t block_exscan(uint32_t v, uint32_t* sh, uint32_t* total) {
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o);
        if (lane >= (uint32_t)o) inc += y;
    }
    if (lane == 63) sh[wv] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
    const uint32_t nw = blockDim.x / 64;
    for (uint32_t i = 0; i < nw; ++i) {
        const uint32_t s = sh[i];
        if (i < wv) before += s;
        all += s;
    }
    *total = all;
    return before + inc - v;
}

// In-place exclusive scan of a[0, n) by one workgroup of 1024 lanes; returns
// the total to every lane. Each lane owns a contiguous run of a multiple of 4
// entries, read and written as 16-byte vectors, so both passes issue all of a
// lane's loads at once (a must be 16-byte aligned).
__device__ uint32_t wg_exscan_inplace(uint32_t* __restrict__ a, uint32_t n, uint32_t* sh) {
    const uint32_t per = (((n + blockDim.x - 1u) / blockDim.x) + 3u) & ~3u;
    const uint32_t lo = min(threadIdx.x * per, n);
    const uint32_t hi = min(lo + per, n);
    const uint32_t nv = (hi - lo) >> 2;  // whole vectors; the rest one by one
    uint4* av = reinterpret_cast<uint4*>(a + lo);
    uint32_t s = 0;
    for (uint32_t k = 0; k < nv; ++k) {
        const uint4 v = av[k];
        s += v.x + v.y + v.z + v.w;
    }
    for (uint32_t i = lo + 4 * nv; i < hi; ++i) s += a[i];
    uint32_t total;
    uint32_t run = block_exscan(s, sh, &total);
    for (uint32_t k = 0; k < nv; ++k) {
        const uint4 v = av[k];
        uint4 o;
        o.x = run;
        o.y = o.x + v.x;
        o.z = o.y + v.y;
        o.w = o.z + v.z;
        run = o.w + v.w;
        av[k] = o;
    }
    for (uint32_t i = lo + 4 * nv; i < hi; ++i) {
        const uint32_t v = a[i];
        a[i] = run;
        run += v;
    }
    return total;
}

constexpr int SPL = MAXL - 1;  // Ctrl level entry of the spawning path's input level

// Counts, per tile of TILE elements, the initial elements that are not
// sampled rulers. With scan_last (levels of at most HEADS_SCAN_LAST_TILES
// tiles) the last workgroup to finish then scans the counts in place
// (exclusive) and publishes the walk count of the level, which saves a launch;
// larger levels leave that to k_heads_scan's wider workgroup. Ctrl.hc_done
// counts finished workgroups: each writes its tiles' counts, fences, and
// takes a ticket; the one with the last ticket fences again, sees every
// count, and resets the counter for the next level. The first kernels of
// every path (head sum, batch heads, contraction scan) clear it at the start
// of a call.
constexpr uint32_t HEADS_SCAN_LAST_TILES = 1024;
__global__ __launch_bounds__(TPB) void k_heads_count(const uint8_t* __restrict__ hp, Sampler smp,
                                                     uint32_t* __restrict__ tilecnt, uint32_t ntiles, uint32_t* zero_p,
                                                     uint32_t zero_words, uint32_t skip_single, uint32_t scan_last,
                                                     Ctrl* ctrl, int lvl, const uint32_t* dm, Gate gate) {
    if (gate.off()) return;
    __shared__ uint32_t sh[TPB / 64];
    __shared__ uint32_t last;
    if (dm) smp.m = dm[0];
    // clear the next level's predecessor marks (free memory at this point)
    if (zero_p) {
        const uint32_t stride = gridDim.x * blockDim.x;
        for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < zero_words; i += stride) zero_p[i] = 0;
    }
    // one list: its head is known (head sum) and no workgroup counts or scans
    if (skip_single && ctrl->single) return;
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        uint32_t bits;
        const uint32_t c = tile_heads(hp, smp, tile * TILE + threadIdx.x * 16, bits);
        const uint32_t t = block_sum(c, sh);
        if (threadIdx.x == 0) tilecnt[tile] = t;
        __syncthreads();  // sh is reused by the next tile
    }
    if (!scan_last) return;
    if (threadIdx.x == 0) {
        __threadfence();  // this workgroup's counts before its ticket
        last = atomicAdd(&ctrl->hc_done, 1u) == gridDim.x - 1u;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();  // every other workgroup's counts after the last ticket
    const uint32_t total = wg_exscan_inplace(tilecnt, ntiles, sh);
    if (threadIdx.x == 0) {
        ctrl->hc_done = 0;
        ctrl->lv[lvl].H = total;
        ctrl->lv[lvl].q = 0;
        if (lvl == 0) {
            ctrl->chunks = 0;
            ctrl->conts = 0;
        }
    }
}

// One workgroup: exclusive scan of the tile counts in place (levels of more
// than HEADS_SCAN_LAST_TILES tiles); publishes the walk count and resets the
// chase queue of this level.
__global__ __launch_bounds__(1024) void k_heads_scan(uint32_t* __restrict__ tilecnt, uint32_t ntiles,
                                                     Ctrl* ctrl, int lvl, uint32_t skip_single, Gate gate) {
    if (gate.off()) return;
    __shared__ uint32_t sh[1024 / 64];
    if (skip_single && ctrl->single) return;
    const uint32_t total = wg_exscan_inplace(tilecnt, ntiles, sh);
    if (threadIdx.x == 0) {
        ctrl->lv[lvl].H = total;
        ctrl->lv[lvl].q = 0;
        if (lvl == 0) {
            ctrl->chunks = 0;
            ctrl->conts = 0;
        }
    }
}

// Writes walk start j into the first word of walk record S + j.
__global__ __launch_bounds__(TPB) void k_heads_write(const uint8_t* __restrict__ hp, Sampler smp,
                                                     const uint32_t* __restrict__ tileoff, uint32_t ntiles,
                                                     char* __restrict__ eb, uint32_t S, uint32_t rec_bytes,
                                                     const Ctrl* skip_if_single, const uint32_t* dm, Gate gate) {
    if (gate.off()) return;
    __shared__ uint32_t sh[TPB / 64];
    if (skip_if_single && skip_if_single->single) return;
    if (dm) { smp.m = dm[0]; S = dm[1]; }
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint32_t x0 = tile * TILE + threadIdx.x * 16;
        uint32_t bits;
        const uint32_t c = tile_heads(hp, smp, x0, bits);
        uint32_t total;
        uint32_t pos = tileoff[tile] + block_exscan(c, sh, &total);
        while (bits) {
            const int j = __ffs(bits) - 1;
            bits &= bits - 1;
            *reinterpret_cast<uint32_t*>(eb + (size_t)(S + pos) * rec_bytes) = x0 + j;
            ++pos;
        }
        __syncthreads();  // sh is reused by the next tile
    }
}

// ----------------------------------------------------------------- chase --
// Pads the rest of a wavefront's visit-log chunk with records that name no
// element (x = NONE wide, all ones packed).
template <int LOG, bool W>
__device__ __forceinline__ void pad_chunk(const LogArrays<W>& lg, uint32_t cbase, uint32_t cfill, uint32_t lane) {
    for (uint32_t q = cfill + lane; q < LOG_CHUNK; q += 64) {
        if constexpr (LOG == 2) lg.r[cbase + q] = ~0ull;
        else lg.x[cbase + q] = NONE;
    }
}

// Persistent kernel: each lane holds one walk; a wavefront refills its idle
// lanes from its own range of walk ids (ballot + mbcnt hand out consecutive
// ids) once `refill` lanes are idle. Each step is
// one dependent gather (the record of x), one store (slot[x]) and a few ALU
// operations for the ruler test, so the loop is bound by memory latency and
// the lanes resident on the chip keep that many gathers in flight.
//
// LOG mode (level 0 of large inputs): instead of storing slot[x] at a random
// address, the active lanes of a wavefront append their (x, walk, offset)
// records to a chunk of the visit log that the wavefront owns, at consecutive
// positions (mbcnt over the active lanes), so every step writes whole lines.
// A chunk that cannot take another step's records is padded and a new one is
// taken with one atomic. LOG = 1 writes wide records, LOG = 2 packed ones.
//
// NW walks per lane: the lane issues the loads of all its walks before it
// uses any of them, so NW independent gathers are in flight per lane.
// At most 80 scalar registers: the persistent grid is 8 waves per SIMD, and
// waves allocated 96 scalar registers (the next granule) measured 1.5-2 %
// slower at 2^28 elements, although the compiler's occupancy estimate is 8
// either way.
template <bool W, class Src, int LOG, int NW>
__global__ __launch_bounds__(CHASE_TPB) __attribute__((amdgpu_num_sgpr(80))) void k_chase(Src src, Sampler smp, uint32_t S, Ctrl* ctrl, int lvl,
                                                     typename Lay<W>::Slot* __restrict__ slot,
                                                     typename Lay<W>::Rec* __restrict__ eb,
                                                     uint8_t* __restrict__ hp_next, uint32_t refill,
                                                     LogArrays<W> lg, uint32_t max_chunks, const uint32_t* dm, Gate gate) {
    if (gate.off()) return;
    using L = Lay<W>;
    using Val = typename L::Val;
    if (dm) { smp.m = src.m = dm[0]; S = dm[1]; }
    const uint32_t lane = lane_id();
    const uint32_t total = S + ctrl->lv[lvl].H;
    const uint32_t m = smp.m;
    const uint32_t cap = walk_cap(m, smp.log2k);
    uint32_t w[NW], x[NW], steps[NW];
    Val off[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        w[k] = NONE;
        x[k] = 0;
        steps[k] = 0;
        off[k] = L::zero();
    }
    // Each wavefront owns a contiguous range of walk ids and refills its lanes
    // from it, so no queue is contended while the chip is busy. In LOG mode
    // with at least 64 walks per wavefront (level 0 of large inputs) the last
    // LR_CHASE_POOL sixteenths of the walk ids form a pool instead: a
    // wavefront done with its own range takes CHASE_GRAB of them at a time
    // with one atomic, so the wavefronts finish closer together. With few walks
    // per wavefront (upper levels, short contracted lists) every wavefront
    // would reach the pool at once, and the contended counter costs more than
    // the balance gains.
    const uint32_t gwave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwave = (gridDim.x * blockDim.x) >> 6;
    const uint32_t pool16 = (LOG != 0 && total >= 64u * nwave) ? LR_CHASE_POOL : 0u;  // many walks per wavefront
    const uint32_t own = (uint32_t)((uint64_t)total * (16u - pool16) / 16u);
    const uint32_t per = own / nwave + 1;
    uint32_t whi = (uint32_t)min<uint64_t>((uint64_t)(gwave + 1) * per, own);
    uint32_t cursor = (uint32_t)min<uint64_t>((uint64_t)gwave * per, own);
    bool exhausted = false;
    uint32_t cbase = 0, cfill = LOG_CHUNK;  // visit-log chunk held by this wavefront (LOG mode)
    bool have = false, dead = false;
    // packed records (LOG == 2): field widths, and per walk slot the id its
    // records carry (the walk, or its current continuation) and the offset
    // that id's records count from; continuation ids come from a block of
    // CONT_GRAB held by the wavefront
    const LogFmt fmt(m, total, lg.ccap, lg.bocap);
    uint32_t rw[NW], rb[NW];
    uint32_t kbase = 0, kfill = CONT_GRAB;
    for (;;) {
        uint64_t idle[NW];
        uint32_t nidle = 0;
        bool all_idle = true;
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            idle[k] = __ballot(w[k] == NONE);
            nidle += __popcll(idle[k]);
            all_idle &= idle[k] == ~0ull;
        }
        const bool want = nidle >= refill || all_idle;
        if (!exhausted && want && cursor >= whi && own >= total) exhausted = true;  // no pool
        if (!exhausted && want && cursor >= whi) {  // own range (or last grab) used up: the pool
            uint32_t g = 0;
            if (lane == 0) g = atomicAdd(&ctrl->lv[lvl].q, CHASE_GRAB);
            g = __shfl(g, 0);
            if ((uint64_t)own + g < total) {
                cursor = own + g;
                whi = (uint32_t)min<uint64_t>((uint64_t)cursor + CHASE_GRAB, total);
            } else {
                exhausted = true;
            }
        }
        if (all_idle && exhausted) break;
        if (!exhausted && want) {
            const uint32_t base = cursor;
            cursor = min(cursor + nidle, whi);
            uint32_t acc = base;
#pragma unroll
            for (int k = 0; k < NW; ++k) {
                if (w[k] == NONE) {
                    const uint32_t my = acc + mbcnt(idle[k]);
                    if (my < whi) {
                        w[k] = my;
                        off[k] = L::zero();
                        steps[k] = 0;
                        rw[k] = my;
                        rb[k] = 0;
                        x[k] = (my < S) ? smp.start(my) : reinterpret_cast<const uint32_t*>(eb + my)[0];
                        if (x[k] >= m) {  // corrupt start (cannot happen for valid input)
                            eb[w[k]] = L::rec(TERM | IDX, L::zero());
                            atomicOr(&ctrl->err, 8u);
                            w[k] = NONE;
                        }
                    }
                }
                acc += __popcll(idle[k]);
            }
        }
        uint32_t nxt[NW];
        Val v[NW];
#pragma unroll
        for (int k = 0; k < NW; ++k)
            if (w[k] != NONE) src.load(x[k], nxt[k], v[k]);
        uint32_t pos[NW];
        if constexpr (LOG != 0) {
            uint64_t act[NW];
            uint32_t na = 0;
#pragma unroll
            for (int k = 0; k < NW; ++k) {
                act[k] = __ballot(w[k] != NONE);
                na += __popcll(act[k]);
            }
            if (na && !dead) {
                if (cfill + na > LOG_CHUNK) {
                    if (have) pad_chunk<LOG>(lg, cbase, cfill, lane);
                    uint32_t c = 0;
                    if (lane == 0) c = atomicAdd(&ctrl->chunks, 1u);
                    c = __shfl(c, 0);
                    if (c >= max_chunks) {  // more visits than elements: the input is not a forest
                        dead = true;
                        have = false;
                        if (lane == 0) atomicOr(&ctrl->err, 32u);
                    } else {
                        cbase = c * LOG_CHUNK;
                        cfill = 0;
                        have = true;
                    }
                }
                uint32_t acc = cbase + cfill;
#pragma unroll
                for (int k = 0; k < NW; ++k) {
                    pos[k] = acc + mbcnt(act[k]);
                    acc += __popcll(act[k]);
                }
                cfill += na;
            }
            if constexpr (LOG == 2) {
                // walks whose offset no longer fits the field take a continuation id
                uint64_t nc[NW];
                uint32_t ncs = 0;
#pragma unroll
                for (int k = 0; k < NW; ++k) {
                    nc[k] = __ballot(!dead && w[k] != NONE && off[k].c - rb[k] >= (1u << fmt.bo));
                    ncs += __popcll(nc[k]);
                }
                if (ncs) {
                    if (kfill + ncs > CONT_GRAB) {
                        uint32_t b = 0;
                        if (lane == 0) b = atomicAdd(&ctrl->conts, CONT_GRAB);
                        kbase = __shfl(b, 0);
                        kfill = 0;
                    }
                    if ((uint64_t)kbase + kfill + ncs > lg.ccap) {
                        // cannot happen: the table holds every continuation a full log can need
                        if (lane == 0) atomicOr(&ctrl->err, 32u);
                        dead = true;
                    } else {
                        uint32_t acc = kbase + kfill;
#pragma unroll
                        for (int k = 0; k < NW; ++k) {
                            if ((nc[k] >> lane) & 1ull) {
                                const uint32_t j = acc + mbcnt(nc[k]);
                                lg.cont[j] = make_uint2(w[k], off[k].c);
                                rw[k] = total + j;
                                rb[k] = off[k].c;
                            }
                            acc += __popcll(nc[k]);
                        }
                        kfill += ncs;
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            if (w[k] == NONE) continue;
            if constexpr (LOG == 1) {
                if (!dead) {
                    lg.x[pos[k]] = x[k];
                    lg.w[pos[k]] = w[k];
                    lg.c[pos[k]] = off[k].c;
                    if constexpr (W) lg.s[pos[k]] = off[k].s;
                }
            } else if constexpr (LOG == 2) {
                if (!dead) {
                    lg.r[pos[k]] = fmt.pack(x[k], rw[k], off[k].c - rb[k]);
                    if constexpr (W) lg.s[pos[k]] = off[k].s;
                }
            } else {
                slot[x[k]] = L::slot(w[k], off[k]);
                LR_DBG_COUNT(slot, lvl, x[k]);
            }
            if (nxt[k] & TERM) {                    // x is a terminal: the walk ends on it
                eb[w[k]] = L::rec(nxt[k], L::add(off[k], v[k]));
                w[k] = NONE;
            } else {
                off[k] = L::add(off[k], v[k]);
                // steps so far: on the input level every record is one link,
                // so the walk's count is its step count and no counter is kept
                uint32_t walked;
                if constexpr (Src::kLinks) walked = off[k].c;
                else walked = ++steps[k];
                if (walked >= cap) {                // too long (or a cycle): the bounded fallback takes over
                    eb[w[k]] = L::rec(TERM | IDX, off[k]);
                    ctrl->mode = MODE_FALLBACK;
                    w[k] = NONE;
                } else if (smp.sampled(nxt[k])) {   // reached the next ruler
                    const uint32_t c = nxt[k] >> smp.log2k;
                    eb[w[k]] = L::rec(c, off[k]);
                    if (hp_next && w[k] < S) {
                        hp_next[c] = 1;
                        LR_DBG_COUNT(mark, lvl + 1, c);  // hp_next exists below the last level only
                    }
                    w[k] = NONE;
                } else {
                    x[k] = nxt[k];
                }
            }
        }
    }
    if constexpr (LOG != 0) {
        if (have) pad_chunk<LOG>(lg, cbase, cfill, lane);
    }
}

// ------------------------------------------------------------------ base --
// Pointer doubling (Wyllie) on <= 16384 elements in LDS by one workgroup.
// d[i] is the weight from i up to (not including) f[i]; terminals point to
// themselves with d = 0, so a round d[i] += d[f[i]], f[i] = f[f[i]] leaves
// them fixed, and after ceil(log2 len) rounds f[i] is i's terminal. The
// result adds the terminal's own value (its weight at this level).
//
// Unweighted levels: lane t holds slots t + j * BASE_TPB for j < COLS (4, 8
// or 16 columns, the fewest that cover the planned size) as (d << 32) | f
// words in registers, and publishes them to LDS after every round. Slots
// past m hold self-loops (0, i), which never change, so a round has no
// per-lane branch: the lane's COLS gathers are in flight together. The
// round is bound by the LDS gathers (random 8 B words); the branch-free
// form took 18-28 % off calls of 2^10-2^13 elements (the base case alone).
template <int COLS, class Src>
__device__ __forceinline__ void base_pd_unweighted(Src& src, uint32_t m, unsigned char* lds, uint32_t* f_,
                                                   uint32_t* dc_) {
    using Val = typename Lay<false>::Val;
    uint64_t* fd = reinterpret_cast<uint64_t*>(lds);
    const uint32_t t = threadIdx.x;
    uint64_t e_[COLS];
#pragma unroll
    for (int j = 0; j < COLS; ++j) {
        const uint32_t i = t + j * BASE_TPB;
        e_[j] = (uint64_t)i;
        if (i < m) {
            uint32_t nxt;
            Val v;
            src.load(i, nxt, v);
            if (!((nxt & TERM) || nxt >= m)) e_[j] = ((uint64_t)v.c << 32) | nxt;
        }
        fd[i] = e_[j];
    }
    __syncthreads();
    for (int round = 0; round < 40; ++round) {
        uint32_t changed = 0;
        uint64_t w_[COLS];
#pragma unroll
        for (int j = 0; j < COLS; ++j) w_[j] = fd[(uint32_t)e_[j]];
#pragma unroll
        for (int j = 0; j < COLS; ++j) {
            changed |= (uint32_t)w_[j] ^ (uint32_t)e_[j];
            e_[j] = ((uint64_t)((uint32_t)(e_[j] >> 32) + (uint32_t)(w_[j] >> 32)) << 32) | (uint32_t)w_[j];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < COLS; ++j) fd[t + j * BASE_TPB] = e_[j];
        if (!__syncthreads_or(changed != 0)) break;
    }
#pragma unroll
    for (int j = 0; j < COLS; ++j) {
        f_[j] = (uint32_t)e_[j];
        dc_[j] = (uint32_t)(e_[j] >> 32);
    }
}

// Weighted levels of at most 8192 elements, the same way: a (d << 32) | f
// word and the 8 B sum per slot, two gathers per element and round.
template <int COLS, class Src>
__device__ __forceinline__ void base_pd_weighted(Src& src, uint32_t m, unsigned char* lds, uint32_t* f_,
                                                 uint32_t* dc_, int64_t* ds_) {
    using Val = typename Lay<true>::Val;
    uint64_t* fd = reinterpret_cast<uint64_t*>(lds);
    int64_t* sd = reinterpret_cast<int64_t*>(lds + 8 * (size_t)(COLS * BASE_TPB));
    const uint32_t t = threadIdx.x;
    uint64_t e_[COLS];
    int64_t s_[COLS];
#pragma unroll
    for (int j = 0; j < COLS; ++j) {
        const uint32_t i = t + j * BASE_TPB;
        e_[j] = (uint64_t)i;
        s_[j] = 0;
        if (i < m) {
            uint32_t nxt;
            Val v;
            src.load(i, nxt, v);
            if (!((nxt & TERM) || nxt >= m)) {
                e_[j] = ((uint64_t)v.c << 32) | nxt;
                s_[j] = v.s;
            }
        }
        fd[i] = e_[j];
        sd[i] = s_[j];
    }
    __syncthreads();
    for (int round = 0; round < 40; ++round) {
        uint32_t changed = 0;
        uint64_t w_[COLS];
        int64_t v_[COLS];
#pragma unroll
        for (int j = 0; j < COLS; ++j) {
            w_[j] = fd[(uint32_t)e_[j]];
            v_[j] = sd[(uint32_t)e_[j]];
        }
#pragma unroll
        for (int j = 0; j < COLS; ++j) {
            changed |= (uint32_t)w_[j] ^ (uint32_t)e_[j];
            e_[j] = ((uint64_t)((uint32_t)(e_[j] >> 32) + (uint32_t)(w_[j] >> 32)) << 32) | (uint32_t)w_[j];
            s_[j] += v_[j];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < COLS; ++j) {
            fd[t + j * BASE_TPB] = e_[j];
            sd[t + j * BASE_TPB] = s_[j];
        }
        if (!__syncthreads_or(changed != 0)) break;
    }
#pragma unroll
    for (int j = 0; j < COLS; ++j) {
        f_[j] = (uint32_t)e_[j];
        dc_[j] = (uint32_t)(e_[j] >> 32);
        ds_[j] = s_[j];
    }
}

template <bool W, class Src, class Out>
__global__ __launch_bounds__(BASE_TPB) void k_base(Src src, Out out, uint32_t m, Ctrl* ctrl, const uint32_t* dm, Gate gate) {
    if (gate.off()) return;
    using L = Lay<W>;
    using Val = typename L::Val;
    extern __shared__ __align__(16) unsigned char lds[];
    const uint32_t mcap = m;            // LDS is carved for the planned size
    if (dm) m = src.m = min(dm[0], m);  // a device-side size is at most that
    const uint32_t t = threadIdx.x;
    // each lane keeps its own elements' (f, d) in registers and writes them
    // to LDS after every round, where the other lanes gather them
    uint32_t f_[BASE_PER], dc_[BASE_PER];
    int64_t ds_[BASE_PER];
    if constexpr (!W) {
        if (mcap <= 4 * BASE_TPB) base_pd_unweighted<4>(src, m, lds, f_, dc_);
        else if (mcap <= 8 * BASE_TPB) base_pd_unweighted<8>(src, m, lds, f_, dc_);
        else base_pd_unweighted<16>(src, m, lds, f_, dc_);
    } else if (mcap <= 4 * BASE_TPB) {
        base_pd_weighted<4>(src, m, lds, f_, dc_, ds_);
    } else if (mcap <= 8 * BASE_TPB) {
        base_pd_weighted<8>(src, m, lds, f_, dc_, ds_);
    } else {
        // larger weighted levels (a user base size above 8192): 8 B sum,
        // 4 B count and 2 B successor arrays
        int64_t* ds = reinterpret_cast<int64_t*>(lds);
        uint32_t* dc = reinterpret_cast<uint32_t*>(lds + 8 * (size_t)m);
        uint16_t* f = reinterpret_cast<uint16_t*>(lds + 12 * (size_t)m);
        for (uint32_t i = t; i < m; i += BASE_TPB) {
            uint32_t nxt;
            Val v;
            src.load(i, nxt, v);
            const bool term = (nxt & TERM) || nxt >= m;
            f[i] = (uint16_t)(term ? i : nxt);
            dc[i] = term ? 0u : v.c;
            ds[i] = term ? 0 : v.s;
        }
        __syncthreads();
        for (int round = 0; round < 40; ++round) {
            uint16_t ff[BASE_PER];
            uint32_t fc[BASE_PER];
            int64_t fs[BASE_PER];
            int changed = 0;
#pragma unroll
            for (int j = 0; j < BASE_PER; ++j) {
                const uint32_t i = t + j * BASE_TPB;
                if (i < m) {
                    const uint32_t fi = f[i];
                    ff[j] = f[fi];
                    fc[j] = dc[fi];
                    fs[j] = ds[fi];
                    changed |= (ff[j] != fi);
                }
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < BASE_PER; ++j) {
                const uint32_t i = t + j * BASE_TPB;
                if (i < m) {
                    f[i] = ff[j];
                    dc[i] += fc[j];
                    ds[i] += fs[j];
                }
            }
            if (!__syncthreads_or(changed)) break;
        }
#pragma unroll
        for (int j = 0; j < BASE_PER; ++j) {
            const uint32_t i = t + j * BASE_TPB;
            if (i < m) {
                f_[j] = f[i];
                dc_[j] = dc[i];
                ds_[j] = ds[i];
            }
        }
    }
    Val rv[BASE_PER];
    uint32_t rr[BASE_PER];
#pragma unroll
    for (int j = 0; j < BASE_PER; ++j) {
        const uint32_t i = t + j * BASE_TPB;
        if (i < m) {
            const uint32_t ti = f_[j];
            uint32_t nxt;
            Val v;
            src.load(ti, nxt, v);
            Val d;
            d.c = dc_[j];
            if constexpr (W) d.s = ds_[j];
            if (nxt & TERM) {
                rv[j] = L::add(d, v);
                rr[j] = nxt & IDX;
            } else {  // never reached a terminal: the input has a cycle
                rv[j] = L::junk();
                rr[j] = NONE;
                atomicOr(&ctrl->err, 16u);
            }
        }
    }
    __syncthreads();  // every read of the level's records happens before any in-place write
#pragma unroll
    for (int j = 0; j < BASE_PER; ++j) {
        const uint32_t i = t + j * BASE_TPB;
        if (i < m) {
            auto cur = out.begin(i);
            out.store(cur, i, rv[j], rr[j]);
        }
    }
}

// --------------------------------------------------------------- resolve --
// Walk S + j of an initial element: its result is its own weight plus the
// result of the ruler it ended on, or plus nothing when it ended on a
// terminal (whose weight the chase already added).
template <bool W>
__global__ __launch_bounds__(TPB) void k_resolve(char* __restrict__ eb_raw, uint32_t S, const Ctrl* ctrl, int lvl,
                                                 const uint32_t* dm, Gate gate) {
    if (gate.off()) return;
    using L = Lay<W>;
    if (dm) S = dm[1];
    auto* rec = reinterpret_cast<typename L::Rec*>(eb_raw);
    auto* res = reinterpret_cast<typename L::Res*>(eb_raw);
    const uint32_t H = ctrl->lv[lvl].H;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < H; j += stride) {
        const typename L::Rec r = rec[S + j];
        typename L::Res o;
        if (r.nxt & TERM) {
            o = L::res(L::val(r), r.nxt & IDX);
        } else if (r.nxt < S) {
            const typename L::Res b = res[r.nxt];
            o = L::res(L::add(L::val(r), L::val(b)), b.root);
        } else {
            o = L::res(L::junk(), NONE);
        }
        res[S + j] = o;
    }
}

// ---------------------------------------------------------------- expand --
// rank(x) = result(walk(x)) - offset(x); root(x) = root(walk(x)).
// Wave tiles of 64 * EXPAND_CH elements, lane-strided (coalesced slot reads
// and output writes); the result gather hits the small per-walk table.
template <bool W, class Out>
__global__ __launch_bounds__(TPB) void k_expand(const typename Lay<W>::Slot* __restrict__ slot, uint32_t m,
                                                const typename Lay<W>::Res* __restrict__ res, uint32_t S,
                                                Ctrl* ctrl, int lvl, Out out, const uint32_t* dm, Gate gate) {
    if (gate.off()) return;
    using L = Lay<W>;
    if (dm) { m = dm[0]; S = dm[1]; }
    const uint32_t nw = S + ctrl->lv[lvl].H;
    const uint32_t lane = lane_id();
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    const uint32_t ntile = (m + 64 * EXPAND_CH - 1) / (64 * EXPAND_CH);
    bool bad = false;
    for (uint32_t tile = wave; tile < ntile; tile += nwaves) {
        const uint32_t base = tile * 64 * EXPAND_CH;
        if (base + lane >= m) continue;
        auto cur = out.begin(base + lane);
        typename L::Slot sv[EXPAND_CH];
#pragma unroll
        for (int j = 0; j < EXPAND_CH; ++j) {
            const uint32_t i = base + j * 64 + lane;
            if (i < m) sv[j] = slot[i];
        }
        // all gathers before any store: the outputs may alias nothing here,
        // but the compiler cannot know that and would order each gather
        // after the previous element's store
        typename L::Res rv[EXPAND_CH];
#pragma unroll
        for (int j = 0; j < EXPAND_CH; ++j) {
            const uint32_t i = base + j * 64 + lane;
            if (i < m && sv[j].w < nw) rv[j] = res[sv[j].w];
        }
        // all values first, then the stores (see k_lc_expand)
        typename L::Val ov[EXPAND_CH];
        uint32_t orr[EXPAND_CH];
#pragma unroll
        for (int j = 0; j < EXPAND_CH; ++j) {
            const typename L::Slot s = sv[j];
            const bool ok = s.w < nw;
            bad |= !ok && (base + j * 64 + lane < m);
            ov[j] = ok ? L::sub(L::val(rv[j]), L::val(s)) : L::junk();
            orr[j] = ok ? rv[j].root : NONE;
        }
#pragma unroll
        for (int j = 0; j < EXPAND_CH; ++j) {
            const uint32_t i = base + j * 64 + lane;
            if (i < m) out.store(cur, i, ov[j], orr[j]);
        }
    }
    if (__ballot(bad) && lane == 0) atomicOr(&ctrl->err, 4u);
}

// ---------------------------------------------------------- placement ----
// Log mode, after the recursion: every visit-log record (x, walk, offset)
// becomes (x, rank[, root][, sum]) and must land at x. Records are grouped by
// element range in two passes and a third pass writes each range of 2^s2
// elements from LDS, so every output line is written whole:
//   place1  resolve each record against its walk's result (records of one
//           walk sit close together in the log, so these gathers mostly hit
//           the caches) and group by x >> s1 (coarse ranges);
//   place2  within each coarse range, group by x >> s2 (fine ranges);
//   place3  one workgroup per fine range: scatter into LDS by x, then write
//           the outputs in order.
// Every element is visited exactly once, so range r receives exactly as many
// records as it has ids; its group starts at r << shift and a fill counter per
// range hands out positions inside it. All tiles append at the same few
// frontiers, so the partially written lines there complete quickly.
template <bool W>
struct PlaceArrays {
    uint32_t* x;
    uint32_t* r;   // rank (link count)
    uint32_t* t;   // root
    int64_t* s;    // weighted rank (weighted levels only)
};

template <bool W, bool ROOT>
constexpr int place_per() { return (int)place_tile_records(W, ROOT) / place_tpb(W, ROOT); }

// LDS bytes of one grouping tile over nb ranges (device and host agree);
// without values only the element ids are grouped.
__host__ __device__ constexpr size_t place_lds_bytes(bool weighted, bool root, uint32_t nb, bool vals = true) {
    const size_t T = place_tile_records(weighted, root);
    size_t o = 8 * (size_t)nb + (vals ? (root ? 12 : 8) : 4) * T;
    if (weighted) o = ((o + 7) & ~(size_t)7) + 8 * T;
    return o;
}

// LDS counting sort of one tile by range, then coalesced writes of each
// range's run at [group(lo_bucket + b) + reserved, ...), space reserved with
// one atomic per range and tile. TWO: the ranges' two-sided counters (front
// and back, one line each), the tile taking the given side.
template <bool W, bool ROOT, int PER, bool VALS = true, bool TWO = false>
__device__ void place_tile(const uint32_t (&xs)[PER], const uint32_t (&rs)[PER], const uint32_t (&ts)[PER],
                           const int64_t (&ss)[PER], const uint32_t (&bs)[PER], uint32_t nb, uint32_t shift,
                           uint32_t lo_bucket, uint32_t n, uint32_t* __restrict__ fill, PlaceArrays<W> out,
                           Ctrl* ctrl, unsigned char* lds, uint32_t side = 0) {
    constexpr int TPB_ = place_tpb(W, ROOT);
    constexpr uint32_t T = (uint32_t)PER * TPB_;
    size_t o = 0;
    uint32_t* hist = reinterpret_cast<uint32_t*>(lds + o);
    o += 4 * (size_t)nb;
    uint32_t* gbase = reinterpret_cast<uint32_t*>(lds + o);
    o += 4 * (size_t)nb;
    uint32_t* sx = reinterpret_cast<uint32_t*>(lds + o);
    o += 4 * (size_t)T;
    uint32_t* sr = reinterpret_cast<uint32_t*>(lds + o);
    if constexpr (VALS) o += 4 * (size_t)T;
    uint32_t* st = nullptr;
    if constexpr (ROOT) {
        st = reinterpret_cast<uint32_t*>(lds + o);
        o += 4 * (size_t)T;
    }
    int64_t* sw = nullptr;
    if constexpr (W) {
        o = (o + 7) & ~(size_t)7;
        sw = reinterpret_cast<int64_t*>(lds + o);
        o += 8 * (size_t)T;
    }
    __shared__ uint32_t scan_sh[TPB_ / 64];
    __shared__ uint32_t tile_total;
    const uint32_t t = threadIdx.x;
    uint32_t lr[PER];
    for (uint32_t b = t; b < nb; b += TPB_) hist[b] = 0;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PER; ++j)
        if (xs[j] < n) lr[j] = atomicAdd(&hist[bs[j]], 1u);
    __syncthreads();
    // exclusive scan of hist (each lane owns a run of consecutive ranges) and reservations
    const uint32_t chunk = (nb + TPB_ - 1) / TPB_;
    const uint32_t a = min(t * chunk, nb), e = min(a + chunk, nb);
    uint32_t sum = 0;
    for (uint32_t b = a; b < e; ++b) sum += hist[b];
    uint32_t total;
    uint32_t run = block_exscan(sum, scan_sh, &total);
    for (uint32_t b = a; b < e; ++b) {
        const uint32_t h = hist[b];
        uint32_t g = 0;
        if (h) {
            if constexpr (TWO) {
                const uint32_t r = lo_bucket + b;
                const uint32_t old = atomicAdd(&fill[(2 * r + side) * FILL_LINE], h);
                // the back side's run ends where the previous back run began
                // (wraps past the range, and is caught below, on overflow)
                const uint32_t len = (uint32_t)min((uint64_t)1 << shift, (uint64_t)n - ((uint64_t)r << shift));
                g = side ? len - old - h : old;
            } else {
                g = atomicAdd(&fill[lo_bucket + b], h);
            }
        }
        gbase[b] = g;
        hist[b] = run;
        run += h;
    }
    if (t == 0) tile_total = total;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        if (xs[j] < n) {
            const uint32_t p = hist[bs[j]] + lr[j];
            sx[p] = xs[j];
            if constexpr (VALS) sr[p] = rs[j];
            if constexpr (ROOT) st[p] = ts[j];
            if constexpr (W) sw[p] = ss[j];
        }
    }
    __syncthreads();
    const uint32_t cnt = tile_total;
    for (uint32_t i = t; i < cnt; i += TPB_) {
        const uint32_t b = (sx[i] >> shift) - lo_bucket;  // the record's range, from its element id
        const uint64_t lo = (uint64_t)(lo_bucket + b) << shift;
        const uint64_t hi = min(lo + (1ull << shift), (uint64_t)n);
        const uint64_t p = lo + gbase[b] + (i - hist[b]);
        if (p < hi) {
            out.x[p] = sx[i];
            if constexpr (VALS) out.r[p] = sr[i];
            if constexpr (ROOT) out.t[p] = st[i];
            if constexpr (W) out.s[p] = sw[i];
        } else {
            atomicOr(&ctrl->err, 64u);  // a range overflowed: some element was visited twice
        }
    }
    __syncthreads();
}

template <bool W, bool ROOT, bool PACK>
__global__ __launch_bounds__(place_tpb(W, ROOT)) void k_place1(LogArrays<W> lg, uint32_t max_chunks,
                                                const typename Lay<W>::Res* __restrict__ res, uint32_t S,
                                                Ctrl* ctrl, uint32_t n, uint32_t s1, uint32_t nb1,
                                                uint32_t* __restrict__ fill1, PlaceArrays<W> out, const uint32_t* dm,
                                                Gate gate) {
    if (gate.off()) return;
    if (dm) { n = dm[0]; S = dm[1]; }
    using L = Lay<W>;
    extern __shared__ __align__(16) unsigned char lds[];
    constexpr int PER = place_per<W, ROOT>();
    constexpr int TPB_ = place_tpb(W, ROOT);
    constexpr uint32_t T = PER * TPB_;
    const uint32_t used = min(ctrl->chunks, max_chunks) * LOG_CHUNK;
    const uint32_t nw = S + ctrl->lv[0].H;
    const uint32_t tiles = (used + T - 1) / T;
    // The fields of every record of a tile in one round of loads (a padding
    // record names no element and is read like the others: it shares their
    // lines). The next tile's round is issued before this tile is grouped:
    // the grouping's barriers wait for LDS only, so those loads stay in
    // flight meanwhile. Packed records are decoded when they are used.
    const LogFmt fmt(n, nw, lg.ccap, lg.bocap);
    uint32_t nx[PER], nwl[PER];
    uint64_t nr[PER];
    typename L::Val noff[PER];
    auto load_tile = [&](uint32_t tile) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const uint32_t i = tile * T + j * TPB_ + threadIdx.x;
            if constexpr (PACK) {
                nr[j] = ~0ull;
                if (i < used) {
                    nr[j] = lg.r[i];
                    if constexpr (W) noff[j].s = lg.s[i];
                }
            } else {
                nx[j] = NONE;
                nwl[j] = NONE;
                if (i < used) {
                    nx[j] = lg.x[i];
                    nwl[j] = lg.w[i];
                    noff[j].c = lg.c[i];
                    if constexpr (W) noff[j].s = lg.s[i];
                }
            }
        }
    };
    if (blockIdx.x < tiles) load_tile(blockIdx.x);
    for (uint32_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        uint32_t xs[PER], rs[PER], ts[PER], bs[PER], wl[PER];
        int64_t ss[PER];
        typename L::Val offs[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            if constexpr (PACK) {
                xs[j] = fmt.x(nr[j]);
                wl[j] = fmt.w(nr[j]);
                offs[j].c = fmt.o(nr[j]);
                if constexpr (W) offs[j].s = noff[j].s;
            } else {
                xs[j] = nx[j];
                wl[j] = nwl[j];
                offs[j] = noff[j];
            }
        }
        if constexpr (PACK) {
            // a continuation id stands for (walk, offset its records count from)
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                if (xs[j] < n && wl[j] >= nw) {
                    const uint32_t cid = wl[j] - nw;
                    if (cid < lg.ccap) {
                        const uint2 e = lg.cont[cid];
                        wl[j] = e.x;
                        offs[j].c += e.y;
                    } else {
                        wl[j] = NONE;
                    }
                }
            }
        }
        // every walk result (the records of a walk sit together, so these
        // mostly hit the caches), all issued before any is used
        typename L::Res bres[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j)
            if (xs[j] < n && wl[j] < nw) bres[j] = res[wl[j]];
        if (tile + gridDim.x < tiles) load_tile(tile + gridDim.x);
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            if (xs[j] < n) {
                const uint32_t w = wl[j];
                const typename L::Val off = offs[j];
                if (w < nw) {
                    const typename L::Res b = bres[j];
                    const typename L::Val v = L::sub(L::val(b), off);
                    rs[j] = v.c;
                    ts[j] = b.root;
                    if constexpr (W) ss[j] = v.s;
                } else {
                    rs[j] = NONE;
                    ts[j] = NONE;
                    if constexpr (W) ss[j] = INT64_MIN;
                    atomicOr(&ctrl->err, 4u);
                }
                bs[j] = xs[j] >> s1;
            }
        }
        place_tile<W, ROOT, PER, true, true>(xs, rs, ts, ss, bs, nb1, s1, 0, n, fill1, out, ctrl, lds, tile & 1u);
    }
}

// fill1: the coarse ranges' two-sided counters. With values (VALS) every
// coarse range is full, and its front and back counts must add up to its
// length; VALS = false groups element ids only: then a coarse range need not
// be full and its records are its front and back segments.
template <bool W, bool ROOT, bool VALS = true>
__global__ __launch_bounds__(place_tpb(W, ROOT)) void k_place2(PlaceArrays<W> in, Ctrl* ctrl, uint32_t n, uint32_t s1, uint32_t s2,
                                                uint32_t* __restrict__ fill2, PlaceArrays<W> out, const uint32_t* dm,
                                                const uint32_t* __restrict__ fill1, Gate gate) {
    if (gate.off()) return;
    if (dm) n = dm[0];
    extern __shared__ __align__(16) unsigned char lds[];
    constexpr int PER = place_per<W, ROOT>();
    constexpr int TPB_ = place_tpb(W, ROOT);
    constexpr uint32_t T = PER * TPB_;
    const uint32_t tiles = (n + T - 1) / T;
    const uint32_t fan = 1u << (s1 - s2);
    // All tiles of one coarse range append to the same fan frontiers. Workgroup
    // i runs on XCD i mod 8, so the tiles of coarse range c go to workgroups
    // on XCD c mod 8: the partial lines at a frontier then meet in one L2.
    const uint32_t tpc = (1u << s1) / T;                        // tiles per coarse range
    const bool xcd = LR_XCD_GROUPS && (gridDim.x % 8) == 0;
    const uint32_t lane8 = blockIdx.x % 8, step = xcd ? gridDim.x / 8 : gridDim.x;
    // the workgroup's tiles in order: q advances by step; NONE when done
    uint32_t q = xcd ? blockIdx.x / 8 : blockIdx.x;
    auto next_tile = [&]() -> uint32_t {
        for (;; q += step) {
            if (!xcd) return q < tiles ? q : NONE;
            const uint32_t c = lane8 + 8 * (q / tpc);
            if (c * tpc >= tiles) return NONE;
            const uint32_t tile = c * tpc + q % tpc;
            if (tile < tiles) return tile;
        }
    };
    // every field of a tile's records in one round of loads (the value loads
    // do not wait for the element id); the next tile's round is issued while
    // this tile is grouped (the grouping's barriers wait for LDS only)
    uint32_t nx[PER], nr[PER], nt[PER];
    int64_t ns[PER];
    auto load_tile = [&](uint32_t tile) {
        const uint32_t c = (tile * T) >> s1;
        const uint32_t lo = c << s1;
        const uint32_t len = min(1u << s1, n - lo);
        uint32_t front = len, back_at = len;  // records at [lo, lo + front) and [lo + back_at, lo + len)
        if constexpr (!VALS) {
            front = fill1[2 * c * FILL_LINE];
            const uint32_t back = fill1[(2 * c + 1) * FILL_LINE];
            back_at = back < len ? len - back : 0u;
        }
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const uint32_t i = tile * T + j * TPB_ + threadIdx.x;
            nx[j] = NONE;
            if (i < n && (i - lo < front || i - lo >= back_at)) {
                nx[j] = in.x[i];
                if constexpr (VALS) {
                    nr[j] = in.r[i];
                    if constexpr (ROOT) nt[j] = in.t[i];
                    if constexpr (W) ns[j] = in.s[i];
                }
            }
        }
    };
    uint32_t tile = next_tile();
    if (tile != NONE) load_tile(tile);
    while (tile != NONE) {
        const uint32_t c = (tile * T) >> s1;  // coarse range of this tile (T divides 2^s1)
        if (threadIdx.x == 0 && tile % tpc == 0) {
            // the range's two sides met exactly (more records than ids: some
            // element was visited twice, or a target has two links)
            const uint32_t len = min(1u << s1, n - (c << s1));
            const uint64_t got = (uint64_t)fill1[2 * c * FILL_LINE] + fill1[(2 * c + 1) * FILL_LINE];
            if (VALS ? got != len : got > len) atomicOr(&ctrl->err, 64u);
        }
        uint32_t xs[PER], rs[PER], ts[PER], bs[PER];
        int64_t ss[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            xs[j] = nx[j];
            if constexpr (VALS) {
                rs[j] = nr[j];
                if constexpr (ROOT) ts[j] = nt[j];
                if constexpr (W) ss[j] = ns[j];
            }
        }
        q += step;
        const uint32_t nxt_tile = next_tile();
        if (nxt_tile != NONE) load_tile(nxt_tile);
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            if (xs[j] < n && (xs[j] >> s1) != c) {  // stale record: the input is not a forest
                atomicOr(&ctrl->err, 64u);
                xs[j] = NONE;
            }
            if (xs[j] < n) bs[j] = (xs[j] >> s2) - c * fan;
        }
        place_tile<W, ROOT, PER, VALS>(xs, rs, ts, ss, bs, fan, s2, c * fan, n, fill2, out, ctrl, lds);
        tile = nxt_tile;
    }
}

// One workgroup per fine range of 2^s2 elements: place the records by x in
// LDS, then write the outputs in element order.
template <bool W, bool ROOT, class Out>
__global__ __launch_bounds__(place_tpb(W, ROOT)) void k_place3(PlaceArrays<W> in, Ctrl* ctrl, uint32_t n, uint32_t s2, uint32_t nb2,
                                                const uint32_t* __restrict__ fill2, int check, Out out,
                                                const uint32_t* dm, Gate gate) {
    if (gate.off()) return;
    if (dm) {  // a device-side size: only the ranges it covers
        n = dm[0];
        nb2 = (n + (1u << s2) - 1) >> s2;
    }
    using L = Lay<W>;
    extern __shared__ __align__(16) unsigned char lds[];
    const uint32_t R = 1u << s2;
    int64_t* ls = reinterpret_cast<int64_t*>(lds);
    uint32_t* lr = reinterpret_cast<uint32_t*>(lds + (W ? 8 * (size_t)R : 0));
    uint32_t* lt = lr + R;
    const uint32_t t = threadIdx.x;
    for (uint32_t f = blockIdx.x; f < nb2; f += gridDim.x) {
        const uint32_t base = f << s2;
        const uint32_t len = min(R, n - base);
        for (uint32_t i = t; i < len; i += place_tpb(W, ROOT)) {
            lr[i] = NONE;
            if constexpr (ROOT) lt[i] = NONE;
            if constexpr (W) ls[i] = INT64_MIN;
        }
        if (check && t == 0 && fill2[f] != len) atomicOr(&ctrl->err, 128u);
        __syncthreads();
        // four records per lane per round, every field loaded before any LDS
        // store (the value loads do not wait for the element id)
        constexpr int U = 4;
        for (uint32_t i0 = t; i0 < len; i0 += U * place_tpb(W, ROOT)) {
            uint32_t kk[U], rv[U], tv[U];
            int64_t sv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t i = i0 + u * place_tpb(W, ROOT);
                kk[u] = NONE;
                if (i < len) {
                    kk[u] = in.x[base + i] - base;
                    rv[u] = in.r[base + i];
                    if constexpr (ROOT) tv[u] = in.t[base + i];
                    if constexpr (W) sv[u] = in.s[base + i];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (kk[u] < len) {
                    lr[kk[u]] = rv[u];
                    if constexpr (ROOT) lt[kk[u]] = tv[u];
                    if constexpr (W) ls[kk[u]] = sv[u];
                }
            }
        }
        __syncthreads();
        if (t < len) {
            auto cur = out.begin(base + t);
            for (uint32_t i = t; i < len; i += place_tpb(W, ROOT)) {
                typename L::Val v;
                v.c = lr[i];
                if constexpr (W) v.s = ls[i];
                out.store(cur, base + i, v, ROOT ? lt[i] : NONE);
            }
        }
        __syncthreads();
    }
}

// Interleave successor and weight (weighted level 0 in log mode).
template <int WT>
__global__ __launch_bounds__(TPB) void k_pair(const uint32_t* __restrict__ succ, const void* __restrict__ weight,
                                              uint32_t n, PairRec<WT>* __restrict__ out, Gate gate) {
    if (gate.off()) return;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        PairRec<WT> r{};
        r.s = succ[i];
        if constexpr (WT == 1) r.w = static_cast<const int32_t*>(weight)[i];
        if constexpr (WT == 3) r.w = static_cast<const int8_t*>(weight)[i];
        if constexpr (WT == 2) r.w = static_cast<const int64_t*>(weight)[i];
        out[i] = r;
    }
}

// ------------------------------------------------- predecessor marks ----
// Level 0 in log mode with more than one list: instead of one random byte
// store per link, the link targets are grouped by element range with the
// placement passes (ids only) and each range of 2^s2 ids writes its marks
// from LDS in order. Every id is the target of at most one link, so no range
// receives more targets than it has ids.
// TGT: the input is a plain list of nin target ids below n (entry `skip`
// excluded) instead of a successor array of n entries.
template <bool VEC, bool TGT = false>
__global__ __launch_bounds__(place_tpb(false, false)) void k_mark1(const uint32_t* __restrict__ succ, uint32_t n, uint32_t s1,
                                                            uint32_t nb1, uint32_t* __restrict__ fill1,
                                                            PlaceArrays<false> out, Ctrl* ctrl, Gate gate,
                                                            uint32_t nin = 0, uint32_t skip = NONE,
                                                            const uint32_t* dm = nullptr) {
    if (gate.off()) return;
    extern __shared__ __align__(16) unsigned char lds[];
    constexpr int PER = place_per<false, false>();
    constexpr int TPB_ = place_tpb(false, false);
    constexpr uint32_t T = PER * TPB_;
    if (dm) n = dm[0];
    if constexpr (!TGT) nin = n;
    const uint32_t tiles = (nin + T - 1) / T;
    // the next tile's successors are loaded while this tile is grouped (the
    // grouping's barriers wait for LDS only)
    uint32_t ns[PER];
    auto load_tile = [&](uint32_t tile) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const uint32_t i = tile * T + j * TPB_ + threadIdx.x;
            ns[j] = (i < nin) ? succ[i] : NONE;
        }
    };
    if (blockIdx.x < tiles) load_tile(blockIdx.x);
    for (uint32_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        uint32_t xs[PER], rs[PER], ts[PER], bs[PER];
        int64_t ss[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const uint32_t i = tile * T + j * TPB_ + threadIdx.x;
            const uint32_t s = ns[j];
            if constexpr (TGT) xs[j] = (i != skip && s < n) ? s : NONE;  // a target id
            else xs[j] = (s != i && s < n) ? s : NONE;                  // the target of a link
            bs[j] = xs[j] >> s1;
        }
        if (tile + gridDim.x < tiles) load_tile(tile + gridDim.x);
        place_tile<false, false, PER, false, true>(xs, rs, ts, ss, bs, nb1, s1, 0, n, fill1, out, ctrl, lds, tile & 1u);
    }
}

// One workgroup per fine range: the range's targets set bytes in LDS, then
// the range's marks are written in order (all n bytes get written).
// WEIGHTS: write +1 for a marked id and -1 for the others (as int8) instead
// of 1 / 0.
template <bool WEIGHTS = false>
__global__ __launch_bounds__(place_tpb(false, false)) void k_mark3(const uint32_t* __restrict__ tx, uint32_t n, uint32_t s2,
                                                            uint32_t nb2, const uint32_t* __restrict__ fill2,
                                                            uint8_t* __restrict__ hp, Gate gate,
                                                            const uint32_t* dm = nullptr) {
    if (gate.off()) return;
    extern __shared__ __align__(16) unsigned char lds[];
    uint32_t* mk = reinterpret_cast<uint32_t*>(lds);
    constexpr int TPB_ = place_tpb(false, false);
    const uint32_t R = 1u << s2;
    if (dm) n = dm[0];
    for (uint32_t f = blockIdx.x; f < nb2; f += gridDim.x) {
        const uint32_t base = f << s2;
        if (base >= n) break;  // device-side size: the ranges past it hold no ids
        const uint32_t len = min(R, n - base);
        for (uint32_t i = threadIdx.x; i < R / 4; i += TPB_) mk[i] = 0;
        __syncthreads();
        const uint32_t cnt = min(fill2[f], len);
        uint8_t* mb = reinterpret_cast<uint8_t*>(mk);
        for (uint32_t i0 = threadIdx.x; i0 < cnt; i0 += 4 * TPB_) {  // four loads in flight per lane
            uint32_t kk[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t i = i0 + u * TPB_;
                kk[u] = (i < cnt) ? tx[base + i] - base : NONE;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (kk[u] < len) mb[kk[u]] = 1;
        }
        __syncthreads();
        if ((len & 3) == 0) {
            uint32_t* hw = reinterpret_cast<uint32_t*>(hp + base);
            // bytes 1 -> 0x01 and 0 -> 0xFF: each byte times 0xFE stays in its byte
            for (uint32_t i = threadIdx.x; i < len / 4; i += TPB_)
                hw[i] = WEIGHTS ? 0xFFFFFFFFu - mk[i] * 0xFEu : mk[i];
        } else {
            for (uint32_t i = threadIdx.x; i < len; i += TPB_)
                hp[base + i] = WEIGHTS ? (mb[i] ? 0x01 : 0xFF) : mb[i];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- Wyllie --
template <bool W, class Src>
__global__ __launch_bounds__(TPB) void k_wy_init(Src src, typename Lay<W>::Rec* __restrict__ a, uint32_t m) {
    using L = Lay<W>;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
        uint32_t nxt;
        typename L::Val v;
        src.load(i, nxt, v);
        a[i] = (nxt & TERM) ? L::rec(i, L::zero()) : L::rec(nxt, v);
    }
}

// One doubling round: d[i] += d[f[i]]; f[i] = f[f[i]] (ping-pong buffers).
// The last round writes the outputs instead (terminal weight is 0 here).
template <bool W, bool LAST>
__global__ __launch_bounds__(TPB) void k_wy_round(const typename Lay<W>::Rec* __restrict__ a,
                                                  typename Lay<W>::Rec* __restrict__ b, uint32_t m,
                                                  OutUser<W, true, true, true> out) {
    using L = Lay<W>;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
        const typename L::Rec r = a[i];
        const typename L::Rec q = a[r.nxt];
        const typename L::Val d = L::add(L::val(r), L::val(q));
        if constexpr (LAST) {
            typename OutUser<W, true, true, true>::Cur c;
            out.store(c, i, d, q.nxt);
        } else {
            b[i] = L::rec(q.nxt, d);
        }
    }
}

template <bool W>
__global__ __launch_bounds__(TPB) void k_wy_copy(const typename Lay<W>::Rec* __restrict__ a, uint32_t m,
                                                 OutUser<W, true, true, true> out) {
    using L = Lay<W>;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
        const typename L::Rec r = a[i];
        typename OutUser<W, true, true, true>::Cur c;
        out.store(c, i, L::val(r), r.nxt);
    }
}

// ------------------------------------------------------------- fallback --
// The bounded fallback, run only when a walk of the ruling-set path reached
// its step cap (an order built against the sampling): pointer doubling with
// J-fold jumps per round, so a round follows up to J - 1 records and
// ceil(log_J n) rounds reach every terminal, whatever the order. A record
// (nxt, value) spans its value's links from its element to nxt; nxt =
// TERM | t once the path has reached its terminal t. Every kernel of the
// fallback is enqueued with every call and returns at once unless the cap
// was hit, so the rounds are few: J = 128 up to 2^21 elements (at most 3
// rounds), 16 above (at most 8).
constexpr uint32_t FB_GRID_PER_CU = 2;

// One round: compose up to J consecutive records (the first round reads the
// input itself). The last round writes the outputs; with err set, a path
// that has not reached a terminal (a cycle) is reported.
template <bool W, bool FIRST, bool LAST, class Src, class Out>
__global__ __launch_bounds__(TPB) void k_fb_round(Src src, const typename Lay<W>::Rec* __restrict__ a,
                                                  typename Lay<W>::Rec* __restrict__ b, uint32_t m, uint32_t J,
                                                  Out out, uint32_t* err, const uint32_t* dm, Gate gate) {
    if (gate.off()) return;
    using L = Lay<W>;
    if (dm) m = src.m = dm[0];
    const uint32_t stride = gridDim.x * blockDim.x;
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    typename Out::Cur cur = out.begin(i);
    for (; i < m; i += stride) {
        typename L::Val acc;
        uint32_t j;
        if constexpr (FIRST) src.load(i, j, acc);  // a terminal t: TERM | t, value 0
        else {
            const typename L::Rec r = a[i];
            acc = L::val(r);
            j = r.nxt;
        }
        for (uint32_t t = 1; t < J && !(j & TERM); ++t) {
            typename L::Val v;
            uint32_t nj;
            if constexpr (FIRST) src.load(j, nj, v);
            else {
                const typename L::Rec q = a[j];
                v = L::val(q);
                nj = q.nxt;
            }
            acc = L::add(acc, v);
            j = nj;
        }
        if constexpr (LAST) {
            if (!(j & TERM) && err) atomicOr(err, ERR_FALLBACK_CYCLE);
            out.store(cur, i, acc, j & IDX);
        } else {
            b[i] = L::rec(j, acc);
        }
    }
}

// Per level, log2 of the ruler spacing (device-side level sizes follow from them).
struct LevelShifts { uint8_t lg[MAXL]; };

// ----------------------------------------------------------------- batch --
// The request table is built on the device: k_batch_desc copies descriptors
// passed by value (up to BATCH_ARG_DESC per launch) into the workspace, and
// k_batch_index scans their sizes into the request bases and first chunks and
// fills the header. With device-side sizes (a batch planned for a capacity,
// as a replayed graph is) it also publishes the level sizes.
struct BatchDescArg {
    BatchDesc d[BATCH_ARG_DESC];
    uint32_t first;  // table index of d[0]
    uint32_t cnt;    // descriptors in this launch
    uint32_t count;  // requests of the whole batch (written to the header)
};
static_assert(sizeof(BatchDescArg) <= 4096, "kernel arguments");

__global__ __launch_bounds__(64) void k_batch_desc(BatchDescArg a, BatchDesc* __restrict__ dst,
                                                   BatchHdr* __restrict__ hdr) {
    for (uint32_t i = threadIdx.x; i < a.cnt; i += 64) dst[a.first + i] = a.d[i];
    if (a.first == 0 && threadIdx.x == 0) hdr->count = a.count;
}

// One workgroup: bases[q] = elements before request q, boff[q] = chunks
// before it (count + 1 entries each); the header's chunk and element totals;
// with levels > 0 (device-side sizes) dm[0] = total and dm[l + 1] =
// ceil(dm[l] / k_l).
__global__ __launch_bounds__(1024) void k_batch_index(const BatchDesc* __restrict__ d, uint32_t* __restrict__ bases,
                                                      uint32_t* __restrict__ boff, BatchHdr* __restrict__ hdr,
                                                      Ctrl* ctrl, uint32_t levels, LevelShifts ks) {
    __shared__ uint32_t sh[2 * (1024 / 64)];
    const uint32_t count = hdr->count;
    const uint32_t per = (count + 1023u) >> 10;
    const uint32_t lo = min(threadIdx.x * per, count), hi = min(lo + per, count);
    uint32_t sn = 0, sc = 0;
    for (uint32_t q = lo; q < hi; ++q) {
        const uint32_t n = (uint32_t)d[q].n;
        sn += n;
        sc += (n + BATCH_CHUNK - 1) / BATCH_CHUNK;
    }
    uint32_t tn, tc;
    uint32_t an = block_exscan(sn, sh, &tn);
    uint32_t ac = block_exscan(sc, sh + 1024 / 64, &tc);
    for (uint32_t q = lo; q < hi; ++q) {
        const uint32_t n = (uint32_t)d[q].n;
        bases[q] = an;
        boff[q] = ac;
        an += n;
        ac += (n + BATCH_CHUNK - 1) / BATCH_CHUNK;
    }
    if (threadIdx.x == 0) {
        bases[count] = tn;
        boff[count] = tc;
        hdr->nchunks = tc;
        hdr->total = tn;
        if (levels) {
            uint32_t m = tn;
            ctrl->dm[0] = m;
            for (uint32_t l = 0; l < levels; ++l) {
                m = (m + (1u << ks.lg[l]) - 1u) >> ks.lg[l];
                ctrl->dm[l + 1] = m;
            }
        }
    }
}

// One workgroup per chunk of BATCH_CHUNK ids of one request:
// concat[g] = base(q) + succ_q[g - base(q)]; out-of-range successors become
// terminals (no list leaves its request). The chunk also sums, for the one-list
// head test, ids minus successors of non-terminals and counts terminals.
__global__ __launch_bounds__(TPB) void k_batch_gather(const BatchDesc* __restrict__ d,
                                                      const uint32_t* __restrict__ bases,
                                                      const uint32_t* __restrict__ boff, const BatchHdr* hdr,
                                                      uint32_t* __restrict__ concat, uint2* __restrict__ part) {
    __shared__ uint64_t shs[TPB / 64];
    __shared__ uint32_t snt[TPB / 64];
    const uint32_t count = hdr->count, nchunks = hdr->nchunks;
    for (uint32_t b = blockIdx.x; b < nchunks; b += gridDim.x) {
        const uint32_t q = batch_find(boff, count, b);  // the request whose chunks hold b
        const uint32_t lo = bases[q], nq = bases[q + 1] - lo;
        const uint32_t start = (b - boff[q]) * BATCH_CHUNK;
        const uint32_t end = min(start + BATCH_CHUNK, nq);
        const uint32_t* sq = d[q].succ;
        uint64_t hs = 0;
        uint32_t nt = 0;
        for (uint32_t i = start + threadIdx.x; i < end; i += TPB) {
            const uint32_t s = sq[i];
            const uint32_t g = lo + i;
            const uint32_t c = (s < nq) ? lo + s : g;
            concat[g] = c;
            if (c == g) { ++nt; hs += g; }
            else hs += (uint64_t)g - c;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            hs += __shfl_xor(hs, o);
            nt += __shfl_xor(nt, o);
        }
        if ((threadIdx.x & 63) == 0) { shs[threadIdx.x >> 6] = hs; snt[threadIdx.x >> 6] = nt; }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int i = 1; i < TPB / 64; ++i) { hs += shs[i]; nt += snt[i]; }
            part[2 * b] = make_uint2((uint32_t)hs, (uint32_t)(hs >> 32));
            part[2 * b + 1] = make_uint2(nt, 0u);
        }
        __syncthreads();  // shs, snt are reused by the next chunk
    }
}

// One workgroup per request: its chunks' partial sums -> (head sum, terminals).
__global__ __launch_bounds__(TPB) void k_batch_reduce(const uint2* __restrict__ part,
                                                      const uint32_t* __restrict__ boff, const BatchHdr* hdr,
                                                      uint2* __restrict__ sums, Gate gate) {
    if (gate.off()) return;
    __shared__ uint64_t shs[TPB / 64];
    __shared__ uint32_t snt[TPB / 64];
    const uint32_t count = hdr->count;
    for (uint32_t q = blockIdx.x; q < count; q += gridDim.x) {
        uint64_t hs = 0;
        uint32_t nt = 0;
        for (uint32_t b = boff[q] + threadIdx.x; b < boff[q + 1]; b += TPB) {
            const uint2 h = part[2 * b];
            hs += (uint64_t)h.x | ((uint64_t)h.y << 32);
            nt += part[2 * b + 1].x;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            hs += __shfl_xor(hs, o);
            nt += __shfl_xor(nt, o);
        }
        if ((threadIdx.x & 63) == 0) { shs[threadIdx.x >> 6] = hs; snt[threadIdx.x >> 6] = nt; }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int i = 1; i < TPB / 64; ++i) { hs += shs[i]; nt += snt[i]; }
            sums[2 * q] = make_uint2((uint32_t)hs, (uint32_t)(hs >> 32));
            sums[2 * q + 1] = make_uint2(nt, 0u);
        }
        __syncthreads();
    }
}

// One workgroup, in place of the head-sum pass for a batch: if every
// non-empty request holds exactly one terminal, each is one list whose head is
// its head sum (the one-list shortcut per request). Then the heads that are
// not sampled rulers become the level-0 walk list in request order, and the
// level-0 marking and compaction are skipped as for a single list; otherwise
// the forest path runs. dm (device-side sizes) gives the level-0 size and
// walk count.
__global__ __launch_bounds__(1024) void k_batch_heads(const uint2* __restrict__ sums,
                                                      const uint32_t* __restrict__ bases, const BatchHdr* hdr,
                                                      Ctrl* ctrl, Sampler smp, char* __restrict__ eb, uint32_t S,
                                                      uint32_t rec_bytes, const uint32_t* dm, Gate gate) {
    if (gate.off()) return;
    __shared__ uint32_t sh[1024 / 64];
    if (threadIdx.x == 0) ctrl->hc_done = 0;  // the head-count kernels' workgroup counter
    if (dm) { smp.m = dm[0]; S = dm[1]; }
    const uint32_t count = hdr->count;
    int ok = 1;
    for (uint32_t q = threadIdx.x; q < count; q += 1024) {
        const uint32_t lo = bases[q], hi = bases[q + 1];
        if (lo == hi) continue;
        const uint64_t hs = (uint64_t)sums[2 * q].x | ((uint64_t)sums[2 * q].y << 32);
        if (sums[2 * q + 1].x != 1 || hs < lo || hs >= hi) ok = 0;
    }
    if (!__syncthreads_and(ok)) {
        if (threadIdx.x == 0) {
            ctrl->single = 0;
            ctrl->multi = 1;
            ctrl->mode = MODE_PLAIN;
        }
        return;
    }
    uint32_t run = 0;  // heads written so far
    for (uint32_t q0 = 0; q0 < count; q0 += 1024) {
        const uint32_t q = q0 + threadIdx.x;
        uint32_t h = NONE;
        if (q < count && bases[q] != bases[q + 1]) {
            h = sums[2 * q].x;  // < 2^31: the check above
            if (smp.sampled(h)) h = NONE;
        }
        uint32_t tot;
        const uint32_t pos = run + block_exscan(h != NONE ? 1u : 0u, sh, &tot);
        if (h != NONE) *reinterpret_cast<uint32_t*>(eb + (size_t)(S + pos) * rec_bytes) = h;
        run += tot;
        __syncthreads();  // sh is reused by the next round
    }
    if (threadIdx.x == 0) {
        ctrl->single = 1;
        ctrl->multi = 0;
        ctrl->mode = MODE_PLAIN;
        ctrl->lv[0].H = run;
        ctrl->lv[0].q = 0;
        ctrl->chunks = 0;
        ctrl->conts = 0;
    }
}

// ------------------------------------------------ tile-local contraction --
// Section 2.3: sublists whose links stay inside one tile of LOCAL_TILE
// consecutive ids are contracted before the ruling-set levels run. A local
// chain starts at an element that no element of its tile links to and ends at
// the first element whose successor lies outside the tile (or that is a
// terminal). The contracted list has one element per chain start, linked to
// the start that the chain's exit leads to, with the chain's link count (and
// weight) as its value; after it is ranked, every element takes the rank of
// its chain start minus its distance from that start.
//   chain    one workgroup per tile: chains by pointer jumping in LDS; per
//            element its chain start and distance; per 32 ids the start
//            bits; per chain its record, staged at the tile's own offset
//   scan     start counts -> compact ids of the first start of every tile
//   compact  staged records -> compact positions, exit successors -> compact
//            ids, predecessor marks for the first ruling-set level
//   expand   every element from its chain start's result
// Elements are owned lane-strided (element j * LC_TPB + lane), so every
// global access of the tile kernels is coalesced.
constexpr int LC_TPB = 512;
#ifndef LR_LC_GRID_PER_CU
#define LR_LC_GRID_PER_CU 64  // chain kernel workgroups per CU, each looping over tiles; 0 = one per tile
#endif
static_assert(LR_LC_GRID_PER_CU >= 0 && LR_LC_GRID_PER_CU <= 1024, "chain kernel workgroups per CU");
constexpr uint32_t LC_T = LOCAL_TILE;
constexpr int LC_PER = LC_T / LC_TPB;   // elements per lane
constexpr int LC_ROUNDS = 14;           // > log2(LC_T): chains of a tile converge within this many rounds
constexpr int LC_CHUNKS = LC_T / 64;    // 64-id chunks of a tile (one wave ballot each)
constexpr uint32_t LC_TGT = 0xffffu;    // jump entry: target (tile-relative id); link count in bits 16-31

static_assert(LC_T == (1u << LOCAL_SHIFT) && LC_T <= LC_TGT + 1 && LC_CHUNKS <= 64, "local tile");

// start ids are compact: tile base (scanned start counts) + starts before the
// element in its tile (word prefix + bits below it in its 32-id word)
__device__ __forceinline__ uint32_t lc_below(uint2 d, uint32_t y) {
    return d.y + __popc(d.x & ((1u << (y & 31)) - 1u));
}

// Chains by pointer jumping toward their starts. PD packs the current jump
// target (low 16 bits, tile-relative) and the link count to it (high 16
// bits); starts point to themselves. Writes pos (start's tile-relative
// compact index << 16 | distance, NONE on a cycle inside the tile), wd (weight
// from the start, weighted only), the tile's start bits and word prefixes
// (dir), its start count (cnt), and per chain its record at stage[tile *
// LC_T + index] with the exit's successor still a global id.
template <bool W, int WT>
__global__ __launch_bounds__(LC_TPB) void k_lc_chain(const uint32_t* __restrict__ succ, const void* __restrict__ weight,
                                                     uint32_t n, uint32_t ntiles, uint32_t* __restrict__ cnt,
                                                     uint2* __restrict__ dir,
                                                     typename Lay<W>::Rec* __restrict__ stage,
                                                     uint32_t* __restrict__ pos, int64_t* __restrict__ wd,
                                                     Ctrl* ctrl, Gate gate) {
    if (gate.off()) return;
    using L = Lay<W>;
    using Val = typename L::Val;
    __shared__ uint32_t PD[LC_T];
    __shared__ int64_t WS[W ? LC_T : 1];
    __shared__ uint2 DIR[LC_T / 32];
    __shared__ uint32_t CH[LC_CHUNKS];
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint32_t b = tile * LC_T;
        const uint32_t len = min(LC_T, n - b);
        const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        uint32_t sv[LC_PER];
        int64_t wv[LC_PER];
#pragma unroll
        for (int j = 0; j < LC_PER; ++j) {
            const uint32_t i = j * LC_TPB + threadIdx.x;
            sv[j] = NONE;
            wv[j] = 1;
            if (i < len) {
                sv[j] = succ[b + i];
                if constexpr (WT == 1) wv[j] = static_cast<const int32_t*>(weight)[b + i];
                if constexpr (WT == 3) wv[j] = static_cast<const int8_t*>(weight)[b + i];
                if constexpr (WT == 2) wv[j] = static_cast<const int64_t*>(weight)[b + i];
                PD[i] = i;
                if constexpr (W) WS[i] = 0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < LC_PER; ++j) {
            const uint32_t i = j * LC_TPB + threadIdx.x;
            const uint32_t d = sv[j] - b;
            if (i < len && d < len && d != i) {
                PD[d] = i | (1u << 16);
                if constexpr (W) WS[d] = wv[j];
            }
        }
        __syncthreads();
        uint32_t v[LC_PER];
        int64_t ws[LC_PER];
#pragma unroll
        for (int j = 0; j < LC_PER; ++j) {
            const uint32_t i = j * LC_TPB + threadIdx.x;
            v[j] = (i < len) ? PD[i] : i;
            ws[j] = 0;
            if constexpr (W) if (i < len) ws[j] = WS[i];
            // chunk j * 8 + wave covers ids [64 (j * 8 + wave), +64), lane = id offset
            const uint64_t starts = __ballot(i < len && (v[j] >> 16) == 0);
            if (lane == 0) CH[j * (LC_TPB / 64) + wave] = __popcll(starts);
            if (lane < 2) DIR[2 * (j * (LC_TPB / 64) + wave) + lane] = make_uint2((uint32_t)(starts >> (32 * lane)), 0u);
        }
        __syncthreads();
        if (wave == 0) {  // exclusive scan of the 64 chunk counts, then the word prefixes
            const uint32_t c = (lane < (uint32_t)LC_CHUNKS) ? CH[lane] : 0u;
            uint32_t inc = c;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t y = __shfl_up(inc, o);
                if (lane >= (uint32_t)o) inc += y;
            }
            if (lane < (uint32_t)LC_CHUNKS) {
                const uint32_t pre = inc - c;
                const uint32_t lo = DIR[2 * lane].x;
                DIR[2 * lane].y = pre;
                DIR[2 * lane + 1].y = pre + __popc(lo);
            }
            if (lane == 63) cnt[tile] = inc;
        }
        for (int round = 0; round < LC_ROUNDS; ++round) {
            int changed = 0;
            if constexpr (!W) {
                // in place: a 32-bit entry always holds a consistent (target, count)
                // pair, so reading a neighbour's newer value only jumps further
#pragma unroll
                for (int j = 0; j < LC_PER; ++j) {
                    const uint32_t i = j * LC_TPB + threadIdx.x;
                    const uint32_t p = v[j] & LC_TGT;
                    if (i < len && p != i) {
                        const uint32_t u = PD[p];
                        const uint32_t q = u & LC_TGT;
                        if (q != p) {
                            v[j] = q | (((v[j] >> 16) + (u >> 16)) << 16);
                            PD[i] = v[j];
                            changed = 1;
                        }
                    }
                }
            } else {
                // target, count and weight live in two words: read all, then write all
                uint32_t nv[LC_PER];
                int64_t nw[LC_PER];
#pragma unroll
                for (int j = 0; j < LC_PER; ++j) {
                    const uint32_t i = j * LC_TPB + threadIdx.x;
                    const uint32_t p = v[j] & LC_TGT;
                    nv[j] = v[j];
                    nw[j] = ws[j];
                    if (i < len && p != i) {
                        const uint32_t u = PD[p];
                        const uint32_t q = u & LC_TGT;
                        if (q != p) {
                            nv[j] = q | (((v[j] >> 16) + (u >> 16)) << 16);
                            nw[j] = ws[j] + WS[p];
                        }
                    }
                }
                __syncthreads();
#pragma unroll
                for (int j = 0; j < LC_PER; ++j) {
                    const uint32_t i = j * LC_TPB + threadIdx.x;
                    if (nv[j] != v[j]) {
                        v[j] = nv[j];
                        ws[j] = nw[j];
                        PD[i] = v[j];
                        WS[i] = ws[j];
                        changed = 1;
                    }
                }
            }
            if (!__syncthreads_or(changed)) break;
        }
        if (threadIdx.x < (len + 31) / 32) dir[(b >> 5) + threadIdx.x] = DIR[threadIdx.x];
#pragma unroll
        for (int j = 0; j < LC_PER; ++j) {
            const uint32_t i = j * LC_TPB + threadIdx.x;
            if (i >= len) continue;
            const uint32_t x = b + i;
            const uint32_t p = v[j] & LC_TGT;
            const uint32_t dist = v[j] >> 16;
            // a start has no predecessor in the tile (its start bit); on a cycle inside
            // the tile the jumps never reach one, even where a target comes back to itself
            if (!((DIR[p >> 5].x >> (p & 31)) & 1u)) {
                pos[x] = NONE;
                atomicOr(&ctrl->err, 8u);
                continue;
            }
            const uint32_t lid = lc_below(DIR[p >> 5], p);
            pos[x] = (lid << 16) | dist;
            if constexpr (W) wd[x] = ws[j];
            const uint32_t s = sv[j];
            const uint32_t d = s - b;
            if (d < len && d != i) continue;  // the chain continues inside the tile
            Val val;
            uint32_t nxt;
            if (s == x || s >= n) {           // the chain ends at the terminal x
                val.c = dist;
                if constexpr (W) val.s = ws[j];
                nxt = TERM | x;
            } else {                          // the chain leaves the tile for the start s
                val.c = dist + 1;
                if constexpr (W) val.s = ws[j] + wv[j];
                nxt = s;
            }
            stage[(size_t)tile * LC_T + lid] = L::rec(nxt, val);
        }
        __syncthreads();  // LDS is reused by the next tile
    }
}

// Exclusive scan of the per-tile start counts (one workgroup); publishes the
// contracted list's size and the sizes of the ruling-set levels above it.

// forced: the contracted path runs alone and this kernel sets its mode
__global__ __launch_bounds__(1024) void k_lc_scan(uint32_t* __restrict__ cnt, uint32_t ntiles, Ctrl* ctrl,
                                                  uint32_t levels, LevelShifts ks, uint32_t cap, uint32_t forced,
                                                  Gate gate) {
    if (gate.off()) return;
    __shared__ uint32_t sh[1024 / 64];
    const uint32_t total = wg_exscan_inplace(cnt, ntiles, sh);
    if (threadIdx.x == 0) {
        ctrl->hc_done = 0;  // the head-count kernels' workgroup counter
        if (forced) ctrl->mode = MODE_LOCAL;
        if (total > cap) {  // the guess was wrong: more than the contracted levels hold
            ctrl->mode = MODE_PLAIN;  // every later kernel of this path returns; the plain path runs
            return;
        }
        cnt[ntiles] = total;
        uint32_t m = total;
        ctrl->dm[0] = m;
        for (uint32_t l = 0; l < levels; ++l) {
            m = (m + (1u << ks.lg[l]) - 1u) >> ks.lg[l];
            ctrl->dm[l + 1] = m;
        }
        ctrl->single = 0;
    }
}

// Zero the first dm bytes of p (the contracted level's predecessor marks).
__global__ __launch_bounds__(TPB) void k_zero_dyn(uint32_t* __restrict__ p, const uint32_t* dm, Gate gate) {
    if (gate.off()) return;
    const uint32_t words = (dm[0] + 3) / 4;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride) p[i] = 0;
}

// One wave per tile: move the tile's staged records to their compact
// positions; an exit successor s (a chain start of another tile) becomes its
// compact id, whose record is marked as having a predecessor.
template <bool W>
__global__ __launch_bounds__(TPB) void k_lc_compact(const typename Lay<W>::Rec* __restrict__ stage,
                                                    const uint32_t* __restrict__ cnt, const uint2* __restrict__ dir,
                                                    uint32_t ntiles, uint32_t n, typename Lay<W>::Rec* __restrict__ lrec,
                                                    uint8_t* __restrict__ hp, Gate gate) {
    if (gate.off()) return;
    const uint32_t lane = lane_id();
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t t = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; t < ntiles; t += nwaves) {
        const uint32_t base = cnt[t];
        const uint32_t c = cnt[t + 1] - base;
        for (uint32_t k = lane; k < c; k += 64) {
            typename Lay<W>::Rec r = stage[(size_t)t * LC_T + k];
            if (!(r.nxt & TERM)) {
                const uint32_t s = r.nxt < n ? r.nxt : n - 1;
                r.nxt = cnt[s >> LOCAL_SHIFT] + lc_below(dir[s >> 5], s);
                if (hp) hp[r.nxt] = 1;
            }
            lrec[base + k] = r;
        }
    }
}

// Pass 3: every element from its chain start's result (lane-strided wave
// tiles like the level expansion; the result gathers stay inside the tile's
// compact range).
template <bool W, class Out>
__global__ __launch_bounds__(TPB) void k_lc_expand(const uint32_t* __restrict__ pos, const int64_t* __restrict__ wd,
                                                   const uint32_t* __restrict__ cnt,
                                                   const typename Lay<W>::Res* __restrict__ res, uint32_t n,
                                                   Ctrl* ctrl, Out out, Gate gate) {
    if (gate.off()) return;
    using L = Lay<W>;
    const uint32_t mc = ctrl->dm[0];
    const uint32_t lane = lane_id();
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    const uint32_t ntile = (n + 64 * EXPAND_CH - 1) / (64 * EXPAND_CH);
    static_assert((64 * EXPAND_CH) <= LC_T && LC_T % (64 * EXPAND_CH) == 0, "a wave tile lies in one chain tile");
    bool bad = false;
    for (uint32_t tile = wave; tile < ntile; tile += nwaves) {
        const uint32_t base = tile * 64 * EXPAND_CH;
        // one chain tile per wave tile: its first compact id is one load
        const uint32_t cb = cnt[base >> LOCAL_SHIFT];
        if (base + lane >= n) continue;
        auto cur = out.begin(base + lane);
        uint32_t pv[EXPAND_CH];
#pragma unroll
        for (int j = 0; j < EXPAND_CH; ++j) {
            const uint32_t i = base + j * 64 + lane;
            pv[j] = (i < n) ? pos[i] : NONE;
        }
        // every gather issued before any store (see k_expand)
        uint32_t cv[EXPAND_CH];
        typename L::Res rv[EXPAND_CH];
        int64_t wv[EXPAND_CH];
#pragma unroll
        for (int j = 0; j < EXPAND_CH; ++j) {
            const uint32_t i = base + j * 64 + lane;
            cv[j] = (pv[j] == NONE) ? NONE : cb + (pv[j] >> 16);
            if (cv[j] < mc) rv[j] = res[cv[j]];
            wv[j] = 0;
            if constexpr (W) if (i < n) wv[j] = wd[i];
        }
        // all values first, then the stores: vector-memory counters also count
        // stores, so a store between two dependent gathers would make every
        // later gather wait for it
        typename L::Val ov[EXPAND_CH];
        uint32_t orr[EXPAND_CH];
#pragma unroll
        for (int j = 0; j < EXPAND_CH; ++j) {
            const bool ok = cv[j] < mc;
            bad |= !ok && (base + j * 64 + lane < n);
            typename L::Val v = L::val(rv[j]);
            v.c -= pv[j] & 0xffffu;
            if constexpr (W) v.s -= wv[j];
            ov[j] = ok ? v : L::junk();
            orr[j] = ok ? rv[j].root : NONE;
        }
#pragma unroll
        for (int j = 0; j < EXPAND_CH; ++j) {
            const uint32_t i = base + j * 64 + lane;
            if (i < n) out.store(cur, i, ov[j], orr[j]);
        }
    }
    if (__ballot(bad) && lane == 0) atomicOr(&ctrl->err, 4u);
}

// ------------------------------------------------------- ruler spawning --
// Section 2.2 on one GPU, in two chases with no atomics on the elements.
// Spawning exists to cut the long stretches between sampled rulers, whose
// walks decide how long a chase runs. Phase 1 is the ordinary chase from the
// sampled rulers and the heads, except that a walk stops after `cap` steps:
// it marks the next element, which no walk has reached, as its cap target
// (slot = SPF | walk, offset) and ends there. Between the phases every
// element whose slot is still free (reached by no walk) is known, and new
// rulers are spawned among exactly those: each cap target, and each free
// element that a hash picks at rate 1/k2. Phase 2 walks from the spawned
// rulers; its lanes tell a spawned ruler from a free element by one plain
// load of the slot, so every step is one round trip of plain loads. With
// phase 1 capped at c k steps only a fraction of about exp(-c) of the
// elements is left for phase 2, where walks are k2 long on average.
//
// Walk ids: [0, S0) sampled rulers (block b's ruler is walk b), [S0, T0)
// heads that are not sampled (start parked in the record), [T0, T0 + R2)
// spawned rulers (start parked in the record), numbered in tile order.
// Slots: all ones = free; (walk, offset) = reached; SPF | walk = a phase-1
// cap target (before the spawn pass) or a spawned ruler (after it).
constexpr uint32_t SPF = TERM;        // slot flag: cap target / spawned ruler
constexpr uint32_t LOG2_SPAWN_K2 = 31 - __builtin_clz((unsigned)LR_SPAWN_K2);  // second chase: mean walk 2^this
constexpr int SP_TPB = 256;

// Every slot free (all ones), and the control words of the path reset.
__global__ __launch_bounds__(TPB) void k_sp_prep(uint32_t* __restrict__ slotw, uint64_t words, Ctrl* ctrl,
                                                 Gate gate) {
    if (gate.off()) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctrl->spn = 0;
        ctrl->single = 0;
        ctrl->multi = 0;
        ctrl->mode = MODE_SPAWN;
    }
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t n4 = words / 4;
    const uint4 v = make_uint4(NONE, NONE, NONE, NONE);
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
        reinterpret_cast<uint4*>(slotw)[i] = v;
    for (uint64_t i = n4 * 4 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride)
        slotw[i] = NONE;
}

// Phase 1: the chase of the sampled rulers' and heads' walks (one walk per
// lane, wavefront walk ranges as in k_chase), capped at `cap` steps. Unlike
// the levels' chase every walk is an element of the next list, so every walk
// that ends on a ruler marks that ruler as having a predecessor.
template <bool W, int WT>
__global__ __launch_bounds__(SP_TPB) void k_sp_chase1(SrcIn<W, WT> src, Sampler smp, Ctrl* ctrl,
                                                      typename Lay<W>::Slot* __restrict__ slot,
                                                      typename Lay<W>::Rec* __restrict__ lrec,
                                                      uint8_t* __restrict__ hp_c, uint32_t cap, Gate gate) {
    if (gate.off()) return;
    using L = Lay<W>;
    using Val = typename L::Val;
    const uint32_t m = smp.m;
    const uint32_t S0 = (m + (1u << smp.log2k) - 1u) >> smp.log2k;
    const uint32_t T0 = S0 + ctrl->lv[SPL].H;
    const uint32_t gwave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwave = (gridDim.x * blockDim.x) >> 6;
    const uint32_t per = T0 / nwave + 1;
    uint32_t cursor = (uint32_t)min<uint64_t>((uint64_t)gwave * per, T0);
    const uint32_t whi = (uint32_t)min<uint64_t>((uint64_t)(gwave + 1) * per, T0);
    uint32_t w = NONE, x = 0, steps = 0;
    Val off = L::zero();
    for (;;) {
        const uint64_t idle = __ballot(w == NONE);
        if (idle == ~0ull && cursor >= whi) break;
        if (idle && cursor < whi) {
            const uint32_t my = cursor + mbcnt(idle);
            cursor = min(cursor + (uint32_t)__popcll(idle), whi);
            if (w == NONE && my < whi) {
                const uint32_t s0 = (my < S0) ? smp.start(my) : lrec[my].nxt;
                if (s0 < m) {
                    w = my;
                    x = s0;
                    off = L::zero();
                    steps = 0;
                } else {  // corrupt parked start (cannot happen for valid input)
                    lrec[my] = L::rec(TERM | IDX, L::zero());
                    atomicOr(&ctrl->err, 8u);
                }
            }
        }
        if (w == NONE) continue;
        uint32_t nxt;
        Val v;
        src.load(x, nxt, v);
        slot[x] = L::slot(w, off);
        if (nxt & TERM) {                           // x is a terminal: the walk ends on it
            lrec[w] = L::rec(nxt, L::add(off, v));
            w = NONE;
            continue;
        }
        off = L::add(off, v);
        if (smp.sampled(nxt)) {                     // reached the next sampled ruler
            const uint32_t c = nxt >> smp.log2k;
            lrec[w] = L::rec(c, off);
            hp_c[c] = 1;
            if (c == w) atomicOr(&ctrl->err, 8u);   // back at its own start: a cycle
            w = NONE;
        } else if (++steps >= cap) {                // capped: nxt becomes a spawned ruler
            slot[nxt] = L::slot(SPF | w, off);
            w = NONE;
        } else {
            x = nxt;
        }
    }
}

// Spawned rulers: per tile of TILE ids, lane j looks at ids tile*TILE + i*TPB
// + j (i < TILE / TPB), coalesced. A ruler is a cap target or a free element
// picked by the hash.
constexpr int SP_PER = TILE / TPB;

template <bool W>
__device__ __forceinline__ bool sp_ruler(const typename Lay<W>::Slot* slot, uint32_t z, uint32_t seed,
                                         uint32_t k2mask) {
    const uint32_t w = slot[z].w;
    if (w == NONE) return (hash32(seed, z) & k2mask) == 0u;
    return (w & SPF) != 0u;
}

template <bool W>
__global__ __launch_bounds__(TPB) void k_sp_count(const typename Lay<W>::Slot* __restrict__ slot, uint32_t n,
                                                  uint32_t seed, uint32_t k2mask, uint32_t* __restrict__ tilecnt,
                                                  uint32_t ntiles, Gate gate) {
    if (gate.off()) return;
    __shared__ uint32_t sh[TPB / 64];
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        uint32_t c = 0;
#pragma unroll
        for (int i = 0; i < SP_PER; ++i) {
            const uint32_t z = t * TILE + i * TPB + threadIdx.x;
            if (z < n) c += sp_ruler<W>(slot, z, seed, k2mask);
        }
        const uint32_t tot = block_sum(c, sh);
        if (threadIdx.x == 0) tilecnt[t] = tot;
        __syncthreads();
    }
}

// One workgroup: scan of the spawned-ruler counts; publishes their number.
__global__ __launch_bounds__(1024) void k_sp_scan(uint32_t* __restrict__ tilecnt, uint32_t ntiles, Ctrl* ctrl,
                                                  Gate gate) {
    if (gate.off()) return;
    __shared__ uint32_t sh[1024 / 64];
    const uint32_t total = wg_exscan_inplace(tilecnt, ntiles, sh);
    if (threadIdx.x == 0) ctrl->spn = total;
}

// Numbers the spawned rulers, parks each one's start in its record, flags its
// slot, and ends the capped walk whose target it is on it.
template <bool W>
__global__ __launch_bounds__(TPB) void k_sp_write(typename Lay<W>::Slot* __restrict__ slot, uint32_t n,
                                                  uint32_t seed, uint32_t k2mask,
                                                  const uint32_t* __restrict__ tileoff, uint32_t ntiles,
                                                  const Ctrl* ctrl, uint32_t S0, typename Lay<W>::Rec* __restrict__ lrec,
                                                  uint8_t* __restrict__ hp_c, Gate gate) {
    if (gate.off()) return;
    using L = Lay<W>;
    __shared__ uint32_t sh[TPB / 64];
    const uint32_t T0 = S0 + ctrl->lv[SPL].H;
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        uint32_t bits = 0;
#pragma unroll
        for (int i = 0; i < SP_PER; ++i) {
            const uint32_t z = t * TILE + i * TPB + threadIdx.x;
            if (z < n && sp_ruler<W>(slot, z, seed, k2mask)) bits |= 1u << i;
        }
        uint32_t total;
        uint32_t pos = T0 + tileoff[t] + block_exscan((uint32_t)__popc(bits), sh, &total);
        while (bits) {
            const int i = __ffs(bits) - 1;
            bits &= bits - 1;
            const uint32_t z = t * TILE + i * TPB + threadIdx.x;
            const typename L::Slot sv = slot[z];
            if (sv.w != NONE) {  // a cap target: its walk ends on this ruler
                lrec[sv.w & IDX] = L::rec(pos, L::val(sv));
                hp_c[pos] = 1;
            }
            slot[z] = L::slot(SPF | pos, L::zero());
            *reinterpret_cast<uint32_t*>(&lrec[pos]) = z;  // parked start
            ++pos;
        }
        __syncthreads();
    }
}

// Phase 2: the walks of the spawned rulers. A lane holds the record of x and
// the pending successor; each step loads the successor's slot and record
// together and then decides: a spawned ruler ends the walk, a free element is
// taken.
template <bool W, int WT>
__global__ __launch_bounds__(SP_TPB) void k_sp_chase2(SrcIn<W, WT> src, Sampler smp, Ctrl* ctrl,
                                                      typename Lay<W>::Slot* __restrict__ slot,
                                                      typename Lay<W>::Rec* __restrict__ lrec,
                                                      uint8_t* __restrict__ hp_c, Gate gate) {
    if (gate.off()) return;
    using L = Lay<W>;
    using Val = typename L::Val;
    const uint32_t m = smp.m;
    const uint32_t S0 = (m + (1u << smp.log2k) - 1u) >> smp.log2k;
    const uint32_t T0 = S0 + ctrl->lv[SPL].H;
    const uint32_t R2 = ctrl->spn;
    const uint32_t gwave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwave = (gridDim.x * blockDim.x) >> 6;
    const uint32_t per = R2 / nwave + 1;
    uint32_t cursor = T0 + (uint32_t)min<uint64_t>((uint64_t)gwave * per, R2);
    const uint32_t whi = T0 + (uint32_t)min<uint64_t>((uint64_t)(gwave + 1) * per, R2);
    uint32_t w = NONE, x = 0, nxt = 0, steps = 0;
    Val v = L::zero(), off = L::zero();
    bool fresh = false;  // walk just started: the record of x is not loaded yet
    const uint32_t cap = walk_cap(m, LOG2_SPAWN_K2);
    for (;;) {
        const uint64_t idle = __ballot(w == NONE);
        if (idle == ~0ull && cursor >= whi) break;
        if (idle && cursor < whi) {
            const uint32_t my = cursor + mbcnt(idle);
            cursor = min(cursor + (uint32_t)__popcll(idle), whi);
            if (w == NONE && my < whi) {
                const uint32_t s0 = lrec[my].nxt;
                if (s0 < m) {
                    w = my;
                    x = s0;
                    off = L::zero();
                    fresh = true;
                    steps = 0;
                } else {
                    lrec[my] = L::rec(TERM | IDX, L::zero());
                    atomicOr(&ctrl->err, 8u);
                }
            }
        }
        if (w == NONE) continue;
        bool adv = false;
        Val o2 = off;
        if (!fresh) {
            o2 = L::add(off, v);
            if (nxt & TERM) {
                lrec[w] = L::rec(nxt, o2);
                w = NONE;
            } else if (smp.sampled(nxt)) {
                const uint32_t c = nxt >> smp.log2k;
                lrec[w] = L::rec(c, o2);
                hp_c[c] = 1;
                w = NONE;
            } else {
                adv = true;
            }
        }
        if (w == NONE) continue;
        const uint32_t q = fresh ? x : nxt;
        uint32_t sw = NONE, ln;
        Val lv;
        if (adv) sw = slot[q].w;
        src.load(q, ln, lv);
        if (fresh) {
            nxt = ln;
            v = lv;
            fresh = false;
        } else if (sw == NONE) {                    // a free element: the walk takes it
            slot[q] = L::slot(w, o2);
            x = q;
            off = o2;
            nxt = ln;
            v = lv;
            if (++steps >= cap) {                   // the bounded fallback takes over
                lrec[w] = L::rec(TERM | IDX, o2);
                ctrl->mode = MODE_FALLBACK;
                w = NONE;
            }
        } else if (sw & SPF) {                      // a spawned ruler: the walk ends on it
            const uint32_t c = sw & IDX;
            lrec[w] = L::rec(c, o2);
            hp_c[c] = 1;
            if (c == w) atomicOr(&ctrl->err, 8u);
            w = NONE;
        } else {                                    // reached twice: two predecessors
            lrec[w] = L::rec(TERM | IDX, o2);
            atomicOr(&ctrl->err, 2u);
            w = NONE;
        }
    }
}

// The walks' list: its size and the sizes of the levels above.
__global__ void k_sp_publish(Ctrl* ctrl, uint32_t S0, uint32_t cap, uint32_t levels, LevelShifts ks, Gate gate) {
    if (gate.off()) return;
    if (threadIdx.x == 0) {
        uint64_t t = (uint64_t)S0 + ctrl->lv[SPL].H + ctrl->spn;
        uint32_t m = (uint32_t)min<uint64_t>(t, cap);
        ctrl->dm[0] = m;
        for (uint32_t l = 0; l < levels; ++l) {
            m = (m + (1u << ks.lg[l]) - 1u) >> ks.lg[l];
            ctrl->dm[l + 1] = m;
        }
        ctrl->single = 0;
    }
}

// rank(x) = result(walk(x)) - offset(x), as k_expand, with the walk id taken
// from the slot without its spawned-ruler flag.
template <bool W, class Out>
__global__ __launch_bounds__(TPB) void k_sp_expand(const typename Lay<W>::Slot* __restrict__ slot, uint32_t n,
                                                   const typename Lay<W>::Res* __restrict__ res, Ctrl* ctrl,
                                                   Out out, Gate gate) {
    if (gate.off()) return;
    using L = Lay<W>;
    const uint32_t mc = ctrl->dm[0];
    const uint32_t lane = lane_id();
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    const uint32_t ntile = (n + 64 * EXPAND_CH - 1) / (64 * EXPAND_CH);
    bool bad = false;
    for (uint32_t tile = wave; tile < ntile; tile += nwaves) {
        const uint32_t base = tile * 64 * EXPAND_CH;
        if (base + lane >= n) continue;
        auto cur = out.begin(base + lane);
        typename L::Slot sv[EXPAND_CH];
#pragma unroll
        for (int j = 0; j < EXPAND_CH; ++j) {
            const uint32_t i = base + j * 64 + lane;
            if (i < n) sv[j] = slot[i];
        }
        typename L::Res rv[EXPAND_CH];
        uint32_t wv[EXPAND_CH];
#pragma unroll
        for (int j = 0; j < EXPAND_CH; ++j) {
            const uint32_t i = base + j * 64 + lane;
            wv[j] = (i < n) ? (sv[j].w & IDX) : NONE;
            if (wv[j] < mc) rv[j] = res[wv[j]];
        }
        typename L::Val ov[EXPAND_CH];
        uint32_t orr[EXPAND_CH];
#pragma unroll
        for (int j = 0; j < EXPAND_CH; ++j) {
            const bool ok = wv[j] < mc;
            bad |= !ok && (base + j * 64 + lane < n);
            ov[j] = ok ? L::sub(L::val(rv[j]), L::val(sv[j])) : L::junk();
            orr[j] = ok ? rv[j].root : NONE;
        }
#pragma unroll
        for (int j = 0; j < EXPAND_CH; ++j) {
            const uint32_t i = base + j * 64 + lane;
            if (i < n) out.store(cur, i, ov[j], orr[j]);
        }
    }
    if (__ballot(bad) && lane == 0) atomicOr(&ctrl->err, 4u);
}

// ============================================================== host side ==

// Device properties, looked up once (thread-safe initialisation of local
// statics) on the device current at the first call.
int device_cus() {
    static const int cus = [] {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            return v;
        return 256;
    }();
    return cus;
}

size_t device_max_lds() {
    static const size_t lds = [] {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
            return (size_t)v;
        return (size_t)65536;
    }();
    return lds;
}

static inline uint32_t grid_for(uint64_t work, uint32_t per_block, uint32_t cap_per_cu = 8) {
    uint64_t g = (work + per_block - 1) / per_block;
    const uint64_t cap = (uint64_t)device_cus() * cap_per_cu;
    if (g > cap) g = cap;
    if (g == 0) g = 1;
    return (uint32_t)g;
}

template <class K>
static uint32_t persistent_grid(K kernel, int tpb) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, tpb, 0) != hipSuccess || nb <= 0) nb = 4;
    return (uint32_t)nb * (uint32_t)device_cus();
}

static hipError_t fill(void* p, uint64_t bytes, uint32_t val, hipStream_t st, const Ctrl* skip_if_single = nullptr,
                       Gate gate = Gate{}) {
    const uint64_t words = (bytes + 3) / 4;
    if (!words) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(words, TPB * 4)), dim3(TPB), 0, st, (uint32_t*)p, words, val,
                       skip_if_single, gate);
    return hipGetLastError();
}

static inline void rec_ev(const RunArgs& a, int i) {
    if (a.ev) (void)hipEventRecord(a.ev[i], a.stream);
}

template <bool W, class Src, class Out>
static hipError_t launch_base(Src src, Out out, uint32_t m, Ctrl* ctrl, hipStream_t st,
                             const uint32_t* dm = nullptr, Gate gate = Gate{}) {
    const size_t lds = base_lds_bytes(m, W);
    auto kern = k_base<W, Src, Out>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(1), dim3(BASE_TPB), lds, st, src, out, m, ctrl, dm, gate);
    return hipGetLastError();
}

template <bool W>
static LogArrays<W> log_arrays(char* ws, const Plan& p) {
    LogArrays<W> a{};
    a.x = reinterpret_cast<uint32_t*>(ws + p.off_log[0]);
    a.w = reinterpret_cast<uint32_t*>(ws + p.off_log[1]);
    a.c = reinterpret_cast<uint32_t*>(ws + p.off_log[2]);
    a.s = W ? reinterpret_cast<int64_t*>(ws + p.off_log[3]) : nullptr;
    a.r = reinterpret_cast<uint64_t*>(ws + p.off_log[0]);  // packed: over the first two arrays
    if (p.pack) {
        a.cont = reinterpret_cast<uint2*>(ws + p.off_conts);
        a.ccap = p.ccap;
        a.bocap = p.bocap;
    }
    return a;
}

template <bool W, int LOG, int NW, class Src>
static hipError_t launch_chase(const Plan& p, int l, Src src, Sampler smp, Ctrl* ctrl, char* ws, hipStream_t st,
                               const uint32_t* dm = nullptr, Gate gate = Gate{}) {
    using L = Lay<W>;
    auto kern = k_chase<W, Src, LOG, NW>;
    static const uint32_t grid = [kern] {  // one per template instance, found once
        const uint32_t g = persistent_grid(kern, CHASE_TPB);
        return LOG != 0 ? std::min<uint32_t>(g, LOG_MAX_WAVES / (CHASE_TPB / 64)) : g;  // bounds the log slack
    }();
    const uint32_t S = (uint32_t)p.m[l + 1];
    auto* slot = reinterpret_cast<typename L::Slot*>(ws + p.off_slot[l]);
    auto* eb = reinterpret_cast<typename L::Rec*>(ws + p.off_eb[l]);
    uint8_t* hp_next = (l + 1 < (int)p.levels) ? reinterpret_cast<uint8_t*>(ws + p.off_slot[l + 1]) : nullptr;
    LogArrays<W> lg = LOG != 0 ? log_arrays<W>(ws, p) : LogArrays<W>{};
    hipLaunchKernelGGL(kern, dim3(grid), dim3(CHASE_TPB), 0, st, src, smp, S, ctrl, l, slot, eb, hp_next,
                       p.refill, lg, p.max_chunks, dm, gate);
    return hipGetLastError();
}

// Level-0 chase into the visit log, in the plan's record format.
template <bool W, int NW, class Src>
static hipError_t launch_chase_log(const Plan& p, Src src, Sampler smp, Ctrl* ctrl, char* ws, hipStream_t st,
                                   const uint32_t* dm, Gate gate) {
    if (p.pack) return launch_chase<W, 2, NW>(p, 0, src, smp, ctrl, ws, st, dm, gate);
    return launch_chase<W, 1, NW>(p, 0, src, smp, ctrl, ws, st, dm, gate);
}

#define LR_TRY(x)                              \
    do {                                       \
        hipError_t e_ = (x);                   \
        if (e_ != hipSuccess) return e_;       \
    } while (0)

template <bool W>
static PlaceArrays<W> place_arrays(char* ws, const size_t* off) {
    PlaceArrays<W> a;
    a.x = reinterpret_cast<uint32_t*>(ws + off[0]);
    a.r = reinterpret_cast<uint32_t*>(ws + off[1]);
    a.t = reinterpret_cast<uint32_t*>(ws + off[2]);
    a.s = W ? reinterpret_cast<int64_t*>(ws + off[3]) : nullptr;
    return a;
}

template <class K>
static hipError_t allow_lds(K kern, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Level-0 propagation in log mode: resolve + coarse grouping, fine grouping,
// placement. The fine-grouped records reuse the visit-log arrays.
template <bool W, bool ROOT, class Out0>
static hipError_t run_place_t(const RunArgs& a, const Plan& p, const typename Lay<W>::Res* res, uint32_t S,
                              Ctrl* ctrl, Out0 out0, const uint32_t* dm) {
    char* ws = a.ws;
    hipStream_t st = a.stream;
    const uint32_t n = (uint32_t)p.m[0];
    uint32_t* fill1 = reinterpret_cast<uint32_t*>(ws + p.off_fill);
    uint32_t* fill2 = fill1 + 2 * (size_t)p.nb1 * FILL_LINE;
    const PlaceArrays<W> P = place_arrays<W>(ws, p.off_p);
    const PlaceArrays<W> Q = place_arrays<W>(ws, p.off_log);
    constexpr uint32_t T = place_tile_records(W, ROOT);
    const dim3 tpb(place_tpb(W, ROOT));
    const size_t cap = (size_t)p.max_chunks * LOG_CHUNK;
    const size_t l1 = place_lds_bytes(W, ROOT, p.nb1);
    if (p.pack) {
        LR_TRY(allow_lds(k_place1<W, ROOT, true>, l1));
        hipLaunchKernelGGL((k_place1<W, ROOT, true>), dim3(grid_for(cap, T)), tpb, l1, st, log_arrays<W>(ws, p),
                           p.max_chunks, res, S, ctrl, n, p.s1, p.nb1, fill1, P, dm, a.gate);
    } else {
        LR_TRY(allow_lds(k_place1<W, ROOT, false>, l1));
        hipLaunchKernelGGL((k_place1<W, ROOT, false>), dim3(grid_for(cap, T)), tpb, l1, st, log_arrays<W>(ws, p),
                           p.max_chunks, res, S, ctrl, n, p.s1, p.nb1, fill1, P, dm, a.gate);
    }
    LR_TRY(hipGetLastError());
    rec_ev(a, EV_PART);
    const size_t l2 = place_lds_bytes(W, ROOT, 1u << (p.s1 - p.s2));
    LR_TRY(allow_lds(k_place2<W, ROOT>, l2));
    hipLaunchKernelGGL((k_place2<W, ROOT>), dim3(grid_for(n, T)), tpb, l2, st, P, ctrl, n, p.s1, p.s2, fill2,
                       Q, dm, fill1, a.gate);
    LR_TRY(hipGetLastError());
    const size_t l3 = ((size_t)1 << p.s2) * (4 + (ROOT ? 4 : 0) + (W ? 8 : 0));
    LR_TRY(allow_lds(k_place3<W, ROOT, Out0>, l3));
    hipLaunchKernelGGL((k_place3<W, ROOT, Out0>), dim3(std::min<uint32_t>(p.nb2, (uint32_t)device_cus() * 8)),
                       tpb, l3, st, Q, ctrl, n, p.s2, p.nb2, fill2, (int)a.validate, out0, dm, a.gate);
    return hipGetLastError();
}

template <bool W, class Out0>
static hipError_t run_place(const RunArgs& a, const Plan& p, const typename Lay<W>::Res* res, uint32_t S, Ctrl* ctrl,
                            Out0 out0, bool root, const uint32_t* dm) {
    if (root) return run_place_t<W, true>(a, p, res, S, ctrl, out0, dm);
    return run_place_t<W, false>(a, p, res, S, ctrl, out0, dm);
}


// Predecessor marks of level 0 in log mode (more than one list): link targets
// grouped by range in two passes, then written range by range from LDS. The
// grouping arrays of the placement are free at this point; the marks land on
// the first of them (hp0), after its grouped targets have been consumed.
static hipError_t run_marks(const RunArgs& a, const Plan& p, uint8_t* hp0, Ctrl* ctrl, const uint32_t* dm) {
    char* ws = a.ws;
    hipStream_t st = a.stream;
    const uint32_t n = (uint32_t)p.m[0];
    const Gate mg{&ctrl->multi, 1u};  // plain path taken and more than one list
    uint32_t* fill1 = reinterpret_cast<uint32_t*>(ws + p.off_fill);
    uint32_t* fill2 = fill1 + 2 * (size_t)p.nb1 * FILL_LINE;
    LR_TRY(fill(fill1, fill_words(p.nb1, p.nb2) * 4, 0u, st, nullptr, mg));
    const PlaceArrays<false> P = place_arrays<false>(ws, p.off_p);
    const PlaceArrays<false> Q = place_arrays<false>(ws, p.off_log);
    constexpr uint32_t T = place_tile_records(false, false);
    const dim3 tpb(place_tpb(false, false));
    const bool vec = ((uintptr_t)a.succ % 16) == 0;
    const size_t l1 = place_lds_bytes(false, false, p.nb1, false);
    if (vec) {
        LR_TRY(allow_lds(k_mark1<true>, l1));
        hipLaunchKernelGGL(k_mark1<true>, dim3(grid_for(n, T)), tpb, l1, st, a.succ, n, p.s1, p.nb1, fill1, P, ctrl, mg,
                           0u, NONE, dm);
    } else {
        LR_TRY(allow_lds(k_mark1<false>, l1));
        hipLaunchKernelGGL(k_mark1<false>, dim3(grid_for(n, T)), tpb, l1, st, a.succ, n, p.s1, p.nb1, fill1, P, ctrl,
                           mg, 0u, NONE, dm);
    }
    LR_TRY(hipGetLastError());
    const size_t l2 = place_lds_bytes(false, false, 1u << (p.s1 - p.s2), false);
    LR_TRY(allow_lds(k_place2<false, false, false>, l2));
    hipLaunchKernelGGL((k_place2<false, false, false>), dim3(grid_for(n, T)), tpb, l2, st, P, ctrl, n, p.s1, p.s2,
                       fill2, Q, dm, fill1, mg);
    LR_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_mark3<false>, dim3(std::min<uint32_t>(p.nb2, (uint32_t)device_cus() * 8)), tpb,
                       (size_t)1 << p.s2, st, Q.x, n, p.s2, p.nb2, fill2, hp0, mg, dm);
    return hipGetLastError();
}

// Euler-tour arc weights (+1 for the down arcs named in `down`, -1 for the
// rest) without one random byte store per vertex: the down arcs' ids are
// grouped by range with the predecessor-mark passes and every 8192-id range
// writes its weights from LDS in order. Uses the grouping arrays of the
// workspace of the prefix sum that follows (weighted, m elements), which are
// free until that call; *done stays false when its plan has none (no visit
// log at this size) and the caller scatters instead.
hipError_t tree_arc_weights(const uint32_t* down, uint32_t V, uint32_t root, int8_t* w, uint32_t m, void* ws,
                            const lr_opts* opts, hipStream_t st, bool* done) {
    *done = false;
    PlanSet ps;
    if (make_plans(m, true, opts, 0, &ps) != LR_OK) return hipSuccess;
    const Plan& p = ps.p;
    if (!p.log0 || p.levels == 0) return hipSuccess;
    char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + ALIGN - 1) / ALIGN * ALIGN);
    Ctrl* ctrl = reinterpret_cast<Ctrl*>(base + p.off_ctrl);
    uint32_t* fill1 = reinterpret_cast<uint32_t*>(base + p.off_fill);
    uint32_t* fill2 = fill1 + 2 * (size_t)p.nb1 * FILL_LINE;
    LR_TRY(fill(fill1, fill_words(p.nb1, p.nb2) * 4, 0u, st));
    const PlaceArrays<false> P = place_arrays<false>(base, p.off_p);
    const PlaceArrays<false> Q = place_arrays<false>(base, p.off_log);
    constexpr uint32_t T = place_tile_records(false, false);
    const dim3 tpb(place_tpb(false, false));
    const size_t l1 = place_lds_bytes(false, false, p.nb1, false);
    LR_TRY(allow_lds(k_mark1<false, true>, l1));
    hipLaunchKernelGGL((k_mark1<false, true>), dim3(grid_for(V, T)), tpb, l1, st, down, m, p.s1, p.nb1, fill1, P, ctrl,
                       Gate{}, V, root);
    LR_TRY(hipGetLastError());
    const size_t l2 = place_lds_bytes(false, false, 1u << (p.s1 - p.s2), false);
    LR_TRY(allow_lds(k_place2<false, false, false>, l2));
    hipLaunchKernelGGL((k_place2<false, false, false>), dim3(grid_for(m, T)), tpb, l2, st, P, ctrl, m, p.s1, p.s2,
                       fill2, Q, nullptr, fill1, Gate{});
    LR_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_mark3<true>, dim3(std::min<uint32_t>(p.nb2, (uint32_t)device_cus() * 8)), tpb,
                       (size_t)1 << p.s2, st, Q.x, m, p.s2, p.nb2, fill2, reinterpret_cast<uint8_t*>(w), Gate{});
    LR_TRY(hipGetLastError());
    *done = true;
    return hipSuccess;
}

// Validation of the input (LR_VALIDATE): range and in-degree counts.
static hipError_t run_validate(const RunArgs& a, const Plan& p, uint32_t n) {
    Ctrl* ctrl = reinterpret_cast<Ctrl*>(a.ws + p.off_ctrl);
    LR_TRY(fill(ctrl, sizeof(Ctrl), 0u, a.stream));
    uint32_t* counts = reinterpret_cast<uint32_t*>(a.ws + p.off_slot[0]);
    LR_TRY(fill(counts, (uint64_t)n * 4, 0u, a.stream));
    return run_validate_input(a.succ, n, counts, &ctrl->err, a.stream);
}

// One streaming pass over the input: terminal count, head sum (the one-list
// shortcut); the plain path's gate (mode 0) when the choice is automatic.
static hipError_t run_headsum(const RunArgs& a, const Plan& p, Gate g) {
    const uint32_t n = (uint32_t)p.m[0];
    hipStream_t st = a.stream;
    const bool vec = ((uintptr_t)a.succ % 16) == 0;
    const uint32_t gs = std::min<uint32_t>(grid_for(n, TPB * 16), HEADSUM_BLOCKS);
    uint32_t* part = reinterpret_cast<uint32_t*>(a.ws + p.off_hsum);
    if (vec) hipLaunchKernelGGL(k_headsum<true>, dim3(gs), dim3(TPB), 0, st, a.succ, n, part, g);
    else hipLaunchKernelGGL(k_headsum<false>, dim3(gs), dim3(TPB), 0, st, a.succ, n, part, g);
    LR_TRY(hipGetLastError());
    const Sampler smp0{n, p.log2k[0], p.lseed[0]};
    hipLaunchKernelGGL(k_headsum_final, dim3(1), dim3(TPB), 0, st, part, gs,
                       reinterpret_cast<Ctrl*>(a.ws + p.off_ctrl), smp0, a.ws + p.off_eb[0], (uint32_t)p.m[1],
                       (uint32_t)p.rec_bytes, 0, (uint32_t)MODE_PLAIN, g);
    return hipGetLastError();
}

// Batches, in place of the head-sum pass: the per-request head sums (from
// the gather pass) and, when every request is one list, their heads as the
// level-0 walks (see k_batch_heads); else the forest path.
static hipError_t run_batch_heads(const RunArgs& a, const Plan& p, Gate g) {
    hipStream_t st = a.stream;
    const uint2* part = reinterpret_cast<const uint2*>(a.ws + p.off_batch_part);
    uint2* sums = reinterpret_cast<uint2*>(a.ws + p.off_batch_sums);
    Ctrl* ctrl = reinterpret_cast<Ctrl*>(a.ws + p.off_ctrl);
    const uint32_t grid = std::max(1u, std::min<uint32_t>(a.count, (uint32_t)device_cus() * 8));
    hipLaunchKernelGGL(k_batch_reduce, dim3(grid), dim3(TPB), 0, st, part, a.boff, a.bhdr, sums, g);
    LR_TRY(hipGetLastError());
    const Sampler smp0{(uint32_t)p.m[0], p.log2k[0], p.lseed[0]};
    hipLaunchKernelGGL(k_batch_heads, dim3(1), dim3(1024), 0, st, sums, a.bases, a.bhdr, ctrl, smp0,
                       a.ws + p.off_eb[0], (uint32_t)p.m[1], (uint32_t)p.rec_bytes,
                       a.dev_sizes ? (const uint32_t*)&ctrl->dm[0] : nullptr, g);
    return hipGetLastError();
}

// Automatic contraction, the device-side guess (sets Ctrl.mode).
static hipError_t run_guess(const RunArgs& a, const Plan& p, uint32_t thr) {
    const uint32_t n = (uint32_t)p.m[0];
    hipStream_t st = a.stream;
    const uint32_t ntiles = (n + LOCAL_TILE - 1) / LOCAL_TILE;
    const uint32_t nsamp = (ntiles + LOCAL_SAMPLE_STRIDE - 1) / LOCAL_SAMPLE_STRIDE;
    const uint32_t gs = std::max(1u, std::min<uint32_t>(nsamp, HEADSUM_BLOCKS));
    uint32_t* part = reinterpret_cast<uint32_t*>(a.ws + p.off_hsum);
    hipLaunchKernelGGL(k_lsample<true>, dim3(gs), dim3(TPB), 0, st, a.succ, n, part);
    LR_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_ldecide, dim3(1), dim3(TPB), 0, st, part, gs, n, thr,
                       reinterpret_cast<Ctrl*>(a.ws + p.off_ctrl));
    return hipGetLastError();
}

// The plain path. With a.prologue the call starts here (validation, head
// sum); otherwise the caller ran them and a.gate selects this path.
template <bool W, int WT, class Out0>
static hipError_t run_srs_t(const RunArgs& a, Out0 out0) {
    using L = Lay<W>;
    const Plan& p = *a.plan;
    char* ws = a.ws;
    hipStream_t st = a.stream;
    const Gate g = a.gate;
    Ctrl* ctrl = reinterpret_cast<Ctrl*>(ws + p.off_ctrl);
    const uint32_t n = (uint32_t)p.m[0];
    // device-side sizes (a batch planned for a capacity): level l's actual
    // size and walk count are dm[l], dm[l + 1]; p.m[] are capacities
    auto dm_at = [&](uint32_t l) -> const uint32_t* { return a.dev_sizes ? &ctrl->dm[l] : nullptr; };
    SrcIn<W, WT> src0{a.succ, a.weight, n};
    if (a.prologue) {
        rec_ev(a, EV_START);
        if (a.validate) LR_TRY(run_validate(a, p, n));
    }
    if (p.levels == 0) {
        LR_TRY((launch_base<W>(src0, out0, n, ctrl, st, dm_at(0), g)));
        for (int i = EV_DETECT; i < EV_COUNT; ++i) rec_ev(a, i);
        return hipSuccess;
    }
    // level 0: initial elements. One list: its head from a streaming sum.
    // Otherwise: predecessor marks (the one-list case skips these kernels).
    uint8_t* hp0 = reinterpret_cast<uint8_t*>(ws + p.off_slot[0]);
    {
        if (a.prologue) LR_TRY(a.desc ? run_batch_heads(a, p, Gate{}) : run_headsum(a, p, Gate{}));
        if (p.log0) {
            LR_TRY(run_marks(a, p, hp0, ctrl, dm_at(0)));
        } else {
            LR_TRY(fill(hp0, n, 0u, st, ctrl, g));
            const bool vec = ((uintptr_t)a.succ % 16) == 0;
            const uint32_t gd = grid_for(n, TPB * 4 * 4);
            if (vec) hipLaunchKernelGGL(k_detect<true>, dim3(gd), dim3(TPB), 0, st, a.succ, n, hp0, ctrl, dm_at(0), g);
            else hipLaunchKernelGGL(k_detect<false>, dim3(gd), dim3(TPB), 0, st, a.succ, n, hp0, ctrl, dm_at(0), g);
            LR_TRY(hipGetLastError());
        }
    }
    rec_ev(a, EV_DETECT);
    for (uint32_t l = 0; l < p.levels; ++l) {
        const uint32_t m = (uint32_t)p.m[l];
        const uint32_t S = (uint32_t)p.m[l + 1];
        const Sampler smp{m, p.log2k[l], p.lseed[l]};
        const uint8_t* hp = reinterpret_cast<const uint8_t*>(ws + p.off_slot[l]);
        uint32_t* tile = reinterpret_cast<uint32_t*>(ws + p.off_tile[l]);
        const bool more = l + 1 < p.levels;
        uint32_t* zp = more ? reinterpret_cast<uint32_t*>(ws + p.off_slot[l + 1]) : nullptr;
        const uint32_t zw = more ? (S + 3) / 4 : 0;
        const uint32_t gt = std::min<uint32_t>(p.ntiles[l], (uint32_t)device_cus() * 8);
        const uint32_t last = p.ntiles[l] <= HEADS_SCAN_LAST_TILES;
        hipLaunchKernelGGL(k_heads_count, dim3(gt), dim3(TPB), 0, st, hp, smp, tile, p.ntiles[l], zp, zw,
                           (uint32_t)(l == 0), last, ctrl, (int)l, dm_at(l), g);
        LR_TRY(hipGetLastError());
        if (!last) {
            hipLaunchKernelGGL(k_heads_scan, dim3(1), dim3(1024), 0, st, tile, p.ntiles[l], ctrl, (int)l,
                               (uint32_t)(l == 0), g);
            LR_TRY(hipGetLastError());
        }
        hipLaunchKernelGGL(k_heads_write, dim3(gt), dim3(TPB), 0, st, hp, smp, tile, p.ntiles[l], ws + p.off_eb[l],
                           S, (uint32_t)p.rec_bytes, (l == 0) ? ctrl : nullptr, dm_at(l), g);
        LR_TRY(hipGetLastError());
        if (a.validate && !(l == 0 && p.log0))
            LR_TRY(fill(ws + p.off_slot[l], (uint64_t)m * p.rec_bytes, 0xffffffffu, st, nullptr, g));
        if (l == 0) rec_ev(a, EV_HEADS);
        if (l == 0) {
            if (p.log0) {
                LR_TRY(fill(ws + p.off_fill, fill_words(p.nb1, p.nb2) * 4, 0u, st, nullptr, g));
                if constexpr (W && WT != 0) {
                    // weighted input: one record per element, interleaved into the
                    // grouping arrays after the first (free until the placement)
                    auto* pr = reinterpret_cast<PairRec<WT>*>(ws + p.off_p[1]);
                    hipLaunchKernelGGL(k_pair<WT>, dim3(grid_for(n, TPB * 4)), dim3(TPB), 0, st, a.succ, a.weight, n,
                                       pr, g);
                    LR_TRY(hipGetLastError());
                    SrcPair<WT> srcp{pr, n};
                    LR_TRY((launch_chase_log<W, 1>(p, srcp, smp, ctrl, ws, st, dm_at(0), g)));
                } else if (p.lane_walks == 2) {
                    LR_TRY((launch_chase_log<W, 2>(p, src0, smp, ctrl, ws, st, dm_at(0), g)));
                } else {
                    LR_TRY((launch_chase_log<W, 1>(p, src0, smp, ctrl, ws, st, dm_at(0), g)));
                }
            } else {
                if (p.lane_walks == 2) LR_TRY((launch_chase<W, 0, 2>(p, 0, src0, smp, ctrl, ws, st, dm_at(0), g)));
                else LR_TRY((launch_chase<W, 0, 1>(p, 0, src0, smp, ctrl, ws, st, dm_at(0), g)));
            }
            rec_ev(a, EV_CHASE0);
        } else {
            SrcLvl<W> src{reinterpret_cast<const typename L::Rec*>(ws + p.off_eb[l - 1]), m};
            LR_TRY((launch_chase<W, 0, 1>(p, (int)l, src, smp, ctrl, ws, st, dm_at(l), g)));
        }
    }
    {
        const uint32_t L_ = p.levels;
        const uint32_t mL = (uint32_t)p.m[L_];
        SrcLvl<W> src{reinterpret_cast<const typename L::Rec*>(ws + p.off_eb[L_ - 1]), mL};
        OutLvl<W> out{reinterpret_cast<typename L::Res*>(ws + p.off_eb[L_ - 1])};
        LR_TRY((launch_base<W>(src, out, mL, ctrl, st, dm_at(L_), g)));
    }
    for (int l = (int)p.levels - 1; l >= 0; --l) {
        const uint32_t m = (uint32_t)p.m[l];
        const uint32_t S = (uint32_t)p.m[l + 1];
        hipLaunchKernelGGL(k_resolve<W>, dim3(grid_for(m, TPB * 4, 4)), dim3(TPB), 0, st, ws + p.off_eb[l], S,
                           ctrl, l, dm_at((uint32_t)l), g);
        LR_TRY(hipGetLastError());
        const auto* slot = reinterpret_cast<const typename L::Slot*>(ws + p.off_slot[l]);
        const auto* res = reinterpret_cast<const typename L::Res*>(ws + p.off_eb[l]);
        const uint32_t ge = grid_for(m, TPB * EXPAND_CH);
        if (l == 0) {
            rec_ev(a, EV_UPPER);
            if (p.log0) {
                LR_TRY((run_place<W, Out0>(a, p, res, S, ctrl, out0, a.desc ? a.any_root : a.root != nullptr,
                                           dm_at(0))));
            } else {
                rec_ev(a, EV_PART);
                hipLaunchKernelGGL((k_expand<W, Out0>), dim3(ge), dim3(TPB), 0, st, slot, m, res, S, ctrl, 0, out0,
                                   dm_at(0), g);
            }
        } else {
            OutLvl<W> out{reinterpret_cast<typename L::Res*>(ws + p.off_eb[l - 1])};
            hipLaunchKernelGGL((k_expand<W, OutLvl<W>>), dim3(ge), dim3(TPB), 0, st, slot, m, res, S, ctrl, l,
                               out, dm_at((uint32_t)l), g);
        }
        LR_TRY(hipGetLastError());
    }
    rec_ev(a, EV_EXPAND);
    return hipSuccess;
}

// The ruling-set levels over a contracted list (records at lrec, sizes in
// Ctrl.dm): on return lrec holds every contracted element's result.
template <bool W>
static hipError_t run_clevels(const RunArgs& a, const Plan& p, typename Lay<W>::Rec* lrec, Ctrl* ctrl, Gate g,
                              bool ev_chase0) {
    using L = Lay<W>;
    char* ws = a.ws;
    hipStream_t st = a.stream;
    const uint32_t Lv = p.levels;
    for (uint32_t l = 0; l < Lv; ++l) {
        const uint32_t* dm = &ctrl->dm[l];
        const Sampler smp{(uint32_t)p.m[l], p.log2k[l], p.lseed[l]};
        const uint32_t S = (uint32_t)p.m[l + 1];
        const uint8_t* hp = reinterpret_cast<const uint8_t*>(ws + p.off_slot[l]);
        uint32_t* tile = reinterpret_cast<uint32_t*>(ws + p.off_tile[l]);
        const bool more = l + 1 < Lv;
        uint32_t* zp = more ? reinterpret_cast<uint32_t*>(ws + p.off_slot[l + 1]) : nullptr;
        const uint32_t zw = more ? (S + 3) / 4 : 0;
        const uint32_t gt = std::min<uint32_t>(p.ntiles[l], (uint32_t)device_cus() * 8);
        const uint32_t last = p.ntiles[l] <= HEADS_SCAN_LAST_TILES;
        hipLaunchKernelGGL(k_heads_count, dim3(gt), dim3(TPB), 0, st, hp, smp, tile, p.ntiles[l], zp, zw, 0u, last,
                           ctrl, (int)l, dm, g);
        LR_TRY(hipGetLastError());
        if (!last) {
            hipLaunchKernelGGL(k_heads_scan, dim3(1), dim3(1024), 0, st, tile, p.ntiles[l], ctrl, (int)l, 0u, g);
            LR_TRY(hipGetLastError());
        }
        hipLaunchKernelGGL(k_heads_write, dim3(gt), dim3(TPB), 0, st, hp, smp, tile, p.ntiles[l], ws + p.off_eb[l],
                           S, (uint32_t)p.rec_bytes, nullptr, dm, g);
        LR_TRY(hipGetLastError());
        if (a.validate && !(l == 0 && p.log0))
            LR_TRY(fill(ws + p.off_slot[l], (uint64_t)p.m[l] * p.rec_bytes, 0xffffffffu, st, nullptr, g));
        const auto* rec = (l == 0) ? lrec : reinterpret_cast<const typename L::Rec*>(ws + p.off_eb[l - 1]);
        SrcLvl<W> src{rec, (uint32_t)p.m[l]};
        if (l == 0 && p.log0) {  // a long contracted list: visit log and grouped placement, as the plain path
            LR_TRY(fill(ws + p.off_fill, fill_words(p.nb1, p.nb2) * 4, 0u, st, nullptr, g));
            LR_TRY((launch_chase_log<W, 1>(p, src, smp, ctrl, ws, st, dm, g)));
        } else {
            LR_TRY((launch_chase<W, 0, 1>(p, (int)l, src, smp, ctrl, ws, st, dm, g)));
        }
        if (l == 0 && ev_chase0) rec_ev(a, EV_CHASE0);
    }
    {
        auto* top = Lv ? reinterpret_cast<typename L::Rec*>(ws + p.off_eb[Lv - 1]) : lrec;
        SrcLvl<W> src{top, (uint32_t)p.m[Lv]};
        OutLvl<W> out{reinterpret_cast<typename L::Res*>(top)};
        LR_TRY((launch_base<W>(src, out, (uint32_t)p.m[Lv], ctrl, st, &ctrl->dm[Lv], g)));
    }
    for (int l = (int)Lv - 1; l >= 0; --l) {
        const uint32_t m = (uint32_t)p.m[l];
        const uint32_t S = (uint32_t)p.m[l + 1];
        const uint32_t* dm = &ctrl->dm[l];
        hipLaunchKernelGGL(k_resolve<W>, dim3(grid_for(m, TPB * 4, 4)), dim3(TPB), 0, st, ws + p.off_eb[l], S,
                           ctrl, l, dm, g);
        LR_TRY(hipGetLastError());
        const auto* slot = reinterpret_cast<const typename L::Slot*>(ws + p.off_slot[l]);
        const auto* res = reinterpret_cast<const typename L::Res*>(ws + p.off_eb[l]);
        auto* below = (l == 0) ? reinterpret_cast<typename L::Res*>(lrec)
                               : reinterpret_cast<typename L::Res*>(ws + p.off_eb[l - 1]);
        OutLvl<W> out{below};
        if (l == 0 && p.log0) {
            LR_TRY((run_place<W, OutLvl<W>>(a, p, res, S, ctrl, out, true, dm)));
        } else {
            hipLaunchKernelGGL((k_expand<W, OutLvl<W>>), dim3(grid_for(m, TPB * EXPAND_CH)), dim3(TPB), 0, st, slot,
                               m, res, S, ctrl, l, out, dm, g);
        }
        LR_TRY(hipGetLastError());
    }
    return hipSuccess;
}

// Tile-local contraction, then the ruling-set levels on the contracted list
// (sizes from the device), then every element from its chain start. The plan
// sizes the levels for a contracted list of at most m[0] elements; lc_n is
// the input's length.
template <bool W, int WT, class Out0>
static hipError_t run_local_t(const RunArgs& a, Out0 out0) {
    using L = Lay<W>;
    const Plan& p = *a.plan;
    char* ws = a.ws;
    hipStream_t st = a.stream;
    const Gate g = a.gate;
    Ctrl* ctrl = reinterpret_cast<Ctrl*>(ws + p.off_ctrl);
    const uint32_t n = (uint32_t)p.lc_n;
    const uint32_t Lv = p.levels;
    if (a.prologue) {
        rec_ev(a, EV_START);
        if (a.validate) LR_TRY(run_validate(a, p, n));
    }
    uint32_t* cnt = reinterpret_cast<uint32_t*>(ws + p.off_lc_cnt);
    uint2* dir = reinterpret_cast<uint2*>(ws + p.off_lc_dir);
    uint32_t* pos = reinterpret_cast<uint32_t*>(ws + p.off_lc_pos);
    int64_t* wd = W ? reinterpret_cast<int64_t*>(ws + p.off_lc_wd) : nullptr;
    auto* lrec = reinterpret_cast<typename L::Rec*>(ws + p.off_lrec);
    auto* stage = reinterpret_cast<typename L::Rec*>(ws + p.off_lc_stage);
    uint8_t* hp0 = Lv ? reinterpret_cast<uint8_t*>(ws + p.off_slot[0]) : nullptr;
    const uint32_t gc = LR_LC_GRID_PER_CU ? std::min<uint32_t>(p.lc_ntiles, (uint32_t)device_cus() * LR_LC_GRID_PER_CU)
                                          : p.lc_ntiles;
    // alone (forced), the path's mode is set by the scan: the kernels up to it
    // run ungated
    const Gate gpre = a.prologue ? Gate{} : g;
    hipLaunchKernelGGL((k_lc_chain<W, WT>), dim3(gc), dim3(LC_TPB), 0, st, a.succ, a.weight, n, p.lc_ntiles, cnt, dir,
                       stage, pos, wd, ctrl, gpre);
    LR_TRY(hipGetLastError());
    LevelShifts ks{};
    for (uint32_t l = 0; l < Lv; ++l) ks.lg[l] = (uint8_t)p.log2k[l];
    hipLaunchKernelGGL(k_lc_scan, dim3(1), dim3(1024), 0, st, cnt, p.lc_ntiles, ctrl, Lv, ks, (uint32_t)p.m[0],
                       (uint32_t)a.prologue, gpre);
    LR_TRY(hipGetLastError());
    rec_ev(a, EV_DETECT);
    if (hp0) {
        hipLaunchKernelGGL(k_zero_dyn, dim3(grid_for(p.m[0] / 4 + 1, TPB * 4)), dim3(TPB), 0, st,
                           reinterpret_cast<uint32_t*>(hp0), (const uint32_t*)&ctrl->dm[0], g);
        LR_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL((k_lc_compact<W>), dim3(grid_for((uint64_t)p.lc_ntiles * 64, TPB)), dim3(TPB), 0, st, stage,
                       cnt, dir, p.lc_ntiles, n, lrec, hp0, g);
    LR_TRY(hipGetLastError());
    rec_ev(a, EV_HEADS);
    LR_TRY(run_clevels<W>(a, p, lrec, ctrl, g, true));
    rec_ev(a, EV_UPPER);
    rec_ev(a, EV_PART);
    hipLaunchKernelGGL((k_lc_expand<W, Out0>), dim3(grid_for(n, TPB * EXPAND_CH)), dim3(TPB), 0, st, pos, wd, cnt,
                       reinterpret_cast<const typename L::Res*>(lrec), n, ctrl, out0, g);
    LR_TRY(hipGetLastError());
    rec_ev(a, EV_EXPAND);
    return hipSuccess;
}

// Ruler spawning: predecessor bytes and heads of the input, the capped chase,
// the spawned rulers, their chase (all walks form the contracted list, sized
// on the device), the ruling-set levels on that list, then every element
// from its walk.
template <bool W, int WT, class Out0>
static hipError_t run_spawn_t(const RunArgs& a, Out0 out0) {
    using L = Lay<W>;
    const Plan& p = *a.plan;
    char* ws = a.ws;
    hipStream_t st = a.stream;
    const Gate g = a.gate;
    Ctrl* ctrl = reinterpret_cast<Ctrl*>(ws + p.off_ctrl);
    const uint32_t n = (uint32_t)p.sp_n;
    const uint32_t Lv = p.levels;
    if (a.prologue) {
        rec_ev(a, EV_START);
        if (a.validate) LR_TRY(run_validate(a, p, n));
    }
    auto* slot = reinterpret_cast<typename L::Slot*>(ws + p.off_sp_slot);
    uint8_t* hp_in = reinterpret_cast<uint8_t*>(ws + p.off_sp_hp);
    uint32_t* tile = reinterpret_cast<uint32_t*>(ws + p.off_sp_tile);
    auto* lrec = reinterpret_cast<typename L::Rec*>(ws + p.off_lrec);
    uint8_t* hp_c = reinterpret_cast<uint8_t*>(ws + p.off_slot[0]);  // the walks' predecessor bytes
    const Sampler smp{n, p.sp_log2k, p.sp_seed};
    const uint32_t S0 = (n + (1u << p.sp_log2k) - 1u) >> p.sp_log2k;
    {
        const uint64_t words = (uint64_t)n * p.rec_bytes / 4;
        hipLaunchKernelGGL(k_sp_prep, dim3(grid_for(words, TPB * 4)), dim3(TPB), 0, st,
                           reinterpret_cast<uint32_t*>(slot), words, ctrl, Gate{});
        LR_TRY(hipGetLastError());
    }
    {  // one list: its head from the streaming sum, and no predecessor marks
        const bool vec = ((uintptr_t)a.succ % 16) == 0;
        const uint32_t gs = std::min<uint32_t>(grid_for(n, TPB * 16), HEADSUM_BLOCKS);
        uint32_t* part = reinterpret_cast<uint32_t*>(ws + p.off_hsum);
        if (vec) hipLaunchKernelGGL(k_headsum<true>, dim3(gs), dim3(TPB), 0, st, a.succ, n, part, g);
        else hipLaunchKernelGGL(k_headsum<false>, dim3(gs), dim3(TPB), 0, st, a.succ, n, part, g);
        LR_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_headsum_final, dim3(1), dim3(TPB), 0, st, part, gs, ctrl, smp,
                           reinterpret_cast<char*>(lrec), S0, (uint32_t)p.rec_bytes, SPL, NONE, g);
        LR_TRY(hipGetLastError());
    }
    LR_TRY(fill(hp_in, n, 0u, st, ctrl, g));
    {
        const bool vec = ((uintptr_t)a.succ % 16) == 0;
        const uint32_t gd = grid_for(n, TPB * 4 * 4);
        if (vec) hipLaunchKernelGGL(k_detect<true>, dim3(gd), dim3(TPB), 0, st, a.succ, n, hp_in, ctrl, nullptr, g);
        else hipLaunchKernelGGL(k_detect<false>, dim3(gd), dim3(TPB), 0, st, a.succ, n, hp_in, ctrl, nullptr, g);
        LR_TRY(hipGetLastError());
    }
    rec_ev(a, EV_DETECT);
    const uint32_t gt = std::min<uint32_t>(p.sp_ntiles, (uint32_t)device_cus() * 8);
    const uint32_t last = p.sp_ntiles <= HEADS_SCAN_LAST_TILES;
    hipLaunchKernelGGL(k_heads_count, dim3(gt), dim3(TPB), 0, st, hp_in, smp, tile, p.sp_ntiles,
                       reinterpret_cast<uint32_t*>(hp_c), (n + 3) / 4, 1u, last, ctrl, SPL, nullptr, g);
    LR_TRY(hipGetLastError());
    if (!last) {
        hipLaunchKernelGGL(k_heads_scan, dim3(1), dim3(1024), 0, st, tile, p.sp_ntiles, ctrl, SPL, 1u, g);
        LR_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(k_heads_write, dim3(gt), dim3(TPB), 0, st, hp_in, smp, tile, p.sp_ntiles,
                       reinterpret_cast<char*>(lrec), S0, (uint32_t)p.rec_bytes, ctrl, nullptr, g);
    LR_TRY(hipGetLastError());
    rec_ev(a, EV_HEADS);
    {
        SrcIn<W, WT> src{a.succ, a.weight, n};
        auto k1 = k_sp_chase1<W, WT>;
        auto k2 = k_sp_chase2<W, WT>;
        static const uint32_t g1 = persistent_grid(k1, SP_TPB);  // one per template instance, found once
        static const uint32_t g2 = persistent_grid(k2, SP_TPB);
        const uint32_t cap = (uint32_t)std::min<uint64_t>((uint64_t)LR_SPAWN_CAP << p.sp_log2k, n);
        hipLaunchKernelGGL(k1, dim3(g1), dim3(SP_TPB), 0, st, src, smp, ctrl, slot, lrec, hp_c, cap, g);
        LR_TRY(hipGetLastError());
        const uint32_t seed2 = p.sp_seed ^ 0x5bd1e995u, k2mask = LR_SPAWN_K2 - 1u;
        hipLaunchKernelGGL(k_sp_count<W>, dim3(gt), dim3(TPB), 0, st, slot, n, seed2, k2mask, tile, p.sp_ntiles, g);
        LR_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_sp_scan, dim3(1), dim3(1024), 0, st, tile, p.sp_ntiles, ctrl, g);
        LR_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_sp_write<W>, dim3(gt), dim3(TPB), 0, st, slot, n, seed2, k2mask, tile, p.sp_ntiles, ctrl,
                           S0, lrec, hp_c, g);
        LR_TRY(hipGetLastError());
        hipLaunchKernelGGL(k2, dim3(g2), dim3(SP_TPB), 0, st, src, smp, ctrl, slot, lrec, hp_c, g);
        LR_TRY(hipGetLastError());
    }
    LevelShifts ks{};
    for (uint32_t l = 0; l < Lv; ++l) ks.lg[l] = (uint8_t)p.log2k[l];
    hipLaunchKernelGGL(k_sp_publish, dim3(1), dim3(64), 0, st, ctrl, S0, (uint32_t)p.m[0], Lv, ks, g);
    LR_TRY(hipGetLastError());
    rec_ev(a, EV_CHASE0);
    LR_TRY(run_clevels<W>(a, p, lrec, ctrl, g, false));
    rec_ev(a, EV_UPPER);
    rec_ev(a, EV_PART);
    hipLaunchKernelGGL((k_sp_expand<W, Out0>), dim3(grid_for(n, TPB * EXPAND_CH)), dim3(TPB), 0, st, slot, n,
                       reinterpret_cast<const typename L::Res*>(lrec), ctrl, out0, g);
    LR_TRY(hipGetLastError());
    rec_ev(a, EV_EXPAND);
    return hipSuccess;
}

// Forced paths run alone. Automatic contraction: a sample of the tiles
// decides on the device, the contracted path's scan may still hand over to the
// plain path, and the plain path's head-sum pass runs only if that path is
// taken. Both paths are enqueued and the one not chosen returns from every
// kernel at once (no host synchronisation, so the call stays capturable).
template <bool W, int WT, class Out0>
static hipError_t run_path_t(const RunArgs& a, Out0 out0) {
    if (a.plan->spawn) return run_spawn_t<W, WT>(a, out0);
    if (!a.lplan) return a.plan->local ? run_local_t<W, WT>(a, out0) : run_srs_t<W, WT>(a, out0);
    const Plan& p = *a.plan;
    Ctrl* ctrl = reinterpret_cast<Ctrl*>(a.ws + p.off_ctrl);
    rec_ev(a, EV_START);
    if (a.validate) LR_TRY(run_validate(a, p, (uint32_t)p.m[0]));
    LR_TRY(run_guess(a, p, (uint32_t)local_guess_cap(p.m[0])));
    RunArgs la = a;
    la.plan = a.lplan;
    la.prologue = false;
    la.gate = Gate{&ctrl->mode, MODE_LOCAL};
    LR_TRY((run_local_t<W, WT>(la, out0)));  // its scan falls back to mode 0 if the list is too long
    RunArgs pa = a;
    pa.prologue = false;
    pa.gate = Gate{&ctrl->mode, MODE_PLAIN};
    LR_TRY(a.desc ? run_batch_heads(pa, p, pa.gate) : run_headsum(pa, p, pa.gate));
    return run_srs_t<W, WT>(pa, out0);
}

// The bounded fallback over the input (see k_fb_round); every kernel returns
// at once unless some walk reached its cap.
template <bool W, int WT, class Out0>
static hipError_t run_fallback_t(const RunArgs& a, Out0 out0) {
    using L = Lay<W>;
    using Src = SrcIn<W, WT>;
    const Plan& p = *a.plan;
    Ctrl* ctrl = reinterpret_cast<Ctrl*>(a.ws + p.off_ctrl);
    const uint64_t n64 = p.spawn ? p.sp_n : (p.local ? p.lc_n : p.m[0]);
    const uint32_t n = (uint32_t)n64;
    const Gate g{&ctrl->mode, MODE_FALLBACK};
    auto* A = reinterpret_cast<typename L::Rec*>(a.ws + p.off_fb);
    auto* B = reinterpret_cast<typename L::Rec*>(a.ws + p.off_fb + (n64 * sizeof(typename L::Rec) + 16 + ALIGN - 1) /
                                                                     ALIGN * ALIGN);
    const uint32_t grid = std::min(grid_for(n, TPB * 4), (uint32_t)device_cus() * FB_GRID_PER_CU);
    const uint32_t J = n64 <= (1ull << 21) ? 128u : 16u;
    uint32_t rounds = 1;
    for (uint64_t span = J; span < n64; span *= J) ++rounds;
    const Src src{a.succ, a.weight, n};
    uint32_t* err = a.validate ? &ctrl->err : nullptr;
    const uint32_t* dm = a.dev_sizes ? &ctrl->dm[0] : nullptr;
    for (uint32_t r = 0; r < rounds; ++r) {
        const bool first = r == 0, last = r + 1 == rounds;
        if (first && last)
            hipLaunchKernelGGL((k_fb_round<W, true, true, Src, Out0>), dim3(grid), dim3(TPB), 0, a.stream, src, A, B,
                               n, J, out0, err, dm, g);
        else if (first)
            hipLaunchKernelGGL((k_fb_round<W, true, false, Src, Out0>), dim3(grid), dim3(TPB), 0, a.stream, src, A,
                               B, n, J, out0, err, dm, g);
        else if (last)
            hipLaunchKernelGGL((k_fb_round<W, false, true, Src, Out0>), dim3(grid), dim3(TPB), 0, a.stream, src, A,
                               B, n, J, out0, err, dm, g);
        else
            hipLaunchKernelGGL((k_fb_round<W, false, false, Src, Out0>), dim3(grid), dim3(TPB), 0, a.stream, src, A,
                               B, n, J, out0, err, dm, g);
        LR_TRY(hipGetLastError());
        std::swap(A, B);  // the round's output is the next round's input
    }
    return hipSuccess;
}

// Every path's first kernels set Ctrl.mode and a capped walk turns it to
// MODE_FALLBACK; the fallback runs after the path and returns at once unless
// that happened. A path that runs alone has no gates (a gate costs every
// kernel a dependent load): after a cap it runs on to its end, bounded (every
// walk stops at its cap, every other kernel is bounded whatever its input),
// and the fallback then overwrites its outputs. Under automatic contraction
// both paths are gated on the mode anyway, so they stop at once. A plan
// without levels (the base case alone) has no walks and no fallback.
template <bool W, int WT, class Out0>
static hipError_t run_any_t(const RunArgs& a, Out0 out0) {
    const Plan& p = *a.plan;
    const bool walks = p.levels >= 1 || p.spawn;
    LR_TRY((run_path_t<W, WT>(a, out0)));
    return walks ? run_fallback_t<W, WT>(a, out0) : hipSuccess;
}

template <int WT>
static hipError_t run_weighted(const RunArgs& a) {
    if (a.rank && a.root) return run_any_t<true, WT>(a, OutUser<true, true, true>{a.rank, a.root, a.sum});
    if (a.rank) return run_any_t<true, WT>(a, OutUser<true, true, false>{a.rank, nullptr, a.sum});
    if (a.root) return run_any_t<true, WT>(a, OutUser<true, false, true>{nullptr, a.root, a.sum});
    return run_any_t<true, WT>(a, OutUser<true, false, false>{nullptr, nullptr, a.sum});
}

hipError_t run_srs(const RunArgs& a) {
    const Plan& p = *a.plan;
    if (a.desc) {
        OutBatch out{a.desc, a.bases, a.bhdr};
        return run_any_t<false, 0>(a, out);
    }
    if (!p.weighted) {  // rank is required
        if (a.root) return run_any_t<false, 0>(a, OutUser<false, true, true>{a.rank, a.root, nullptr});
        return run_any_t<false, 0>(a, OutUser<false, true, false>{a.rank, nullptr, nullptr});
    }
    if (a.rec) {  // records for an internal caller
        OutLvl<true> out{reinterpret_cast<typename Lay<true>::Res*>(a.rec)};
        switch (a.wt) {
            case 1: return run_any_t<true, 1>(a, out);
            case 2: return run_any_t<true, 2>(a, out);
            case 3: return run_any_t<true, 3>(a, out);
            default: return run_any_t<true, 0>(a, out);
        }
    }
    switch (a.wt) {  // the sum is required; rank and root are optional
        case 1: return run_weighted<1>(a);
        case 2: return run_weighted<2>(a);
        default: return run_weighted<0>(a);
    }
}

template <bool W, int WT>
static hipError_t run_wyllie_t(const RunArgs& a, uint64_t n64) {
    using L = Lay<W>;
    const uint32_t n = (uint32_t)n64;
    auto* A = reinterpret_cast<typename L::Rec*>(a.ws);
    auto* B = reinterpret_cast<typename L::Rec*>(a.ws + ((n64 * sizeof(typename L::Rec) + ALIGN - 1) / ALIGN) * ALIGN);
    OutUser<W, true, true, true> out{a.rank, a.root, W ? a.sum : nullptr};
    const uint32_t g = grid_for(n, TPB * 4);
    SrcIn<W, WT> src{a.succ, a.weight, n};
    rec_ev(a, EV_START);
    hipLaunchKernelGGL((k_wy_init<W, SrcIn<W, WT>>), dim3(g), dim3(TPB), 0, a.stream, src, A, n);
    LR_TRY(hipGetLastError());
    uint32_t rounds = 0;
    while ((1ull << rounds) < n64) ++rounds;
    if (rounds == 0) {
        hipLaunchKernelGGL(k_wy_copy<W>, dim3(g), dim3(TPB), 0, a.stream, A, n, out);
        LR_TRY(hipGetLastError());
    }
    for (uint32_t r = 0; r < rounds; ++r) {
        if (r + 1 == rounds)
            hipLaunchKernelGGL((k_wy_round<W, true>), dim3(g), dim3(TPB), 0, a.stream, A, B, n, out);
        else
            hipLaunchKernelGGL((k_wy_round<W, false>), dim3(g), dim3(TPB), 0, a.stream, A, B, n, out);
        LR_TRY(hipGetLastError());
        std::swap(A, B);
    }
    for (int i = EV_DETECT; i < EV_COUNT; ++i) rec_ev(a, i);
    return hipSuccess;
}

hipError_t run_wyllie(const RunArgs& a, uint64_t n, bool weighted) {
    if (!weighted) return run_wyllie_t<false, 0>(a, n);
    switch (a.wt) {
        case 1: return run_wyllie_t<true, 1>(a, n);
        case 2: return run_wyllie_t<true, 2>(a, n);
        default: return run_wyllie_t<true, 0>(a, n);
    }
}

hipError_t run_batch_table(const lr_request* reqs, uint32_t count, const Plan& p, char* ws, bool dev_sizes,
                           uint32_t max_chunks, hipStream_t st) {
    auto* desc = reinterpret_cast<BatchDesc*>(ws + p.off_batch_desc);
    auto* bases = reinterpret_cast<uint32_t*>(ws + p.off_batch_bases);
    uint32_t* boff = bases + p.batch_count + 1;
    auto* hdr = reinterpret_cast<BatchHdr*>(ws + p.off_batch_hdr);
    Ctrl* ctrl = reinterpret_cast<Ctrl*>(ws + p.off_ctrl);
    BatchDescArg arg{};
    arg.count = count;
    for (uint32_t first = 0; first < count || first == 0; first += BATCH_ARG_DESC) {
        arg.first = first;
        arg.cnt = std::min<uint32_t>(BATCH_ARG_DESC, count - first);
        for (uint32_t i = 0; i < arg.cnt; ++i) {
            const lr_request& r = reqs[first + i];
            arg.d[i] = BatchDesc{r.succ, r.rank, r.root, r.n};
        }
        hipLaunchKernelGGL(k_batch_desc, dim3(1), dim3(64), 0, st, arg, desc, hdr);
        LR_TRY(hipGetLastError());
        if (count == 0) break;
    }
    LevelShifts ks{};
    for (uint32_t l = 0; l < p.levels; ++l) ks.lg[l] = (uint8_t)p.log2k[l];
    hipLaunchKernelGGL(k_batch_index, dim3(1), dim3(1024), 0, st, desc, bases, boff, hdr, ctrl,
                       dev_sizes ? p.levels : 0u, ks);
    LR_TRY(hipGetLastError());
    const uint32_t grid = std::max(1u, std::min<uint32_t>(max_chunks, (uint32_t)device_cus() * 16));
    hipLaunchKernelGGL(k_batch_gather, dim3(grid), dim3(TPB), 0, st, desc, bases, boff, hdr,
                       reinterpret_cast<uint32_t*>(ws + p.off_batch_succ),
                       reinterpret_cast<uint2*>(ws + p.off_batch_part));
    return hipGetLastError();
}

hipError_t run_validate_input(const uint32_t* succ, uint32_t n, uint32_t* counts, uint32_t* err, hipStream_t st) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_validate_in, dim3(grid_for(n, TPB * 4)), dim3(TPB), 0, st, succ, n, counts, err);
    return hipGetLastError();
}

hipError_t run_verify(const uint32_t* succ, const void* weight, int wt, const uint32_t* rank, const uint32_t* root,
                      const int64_t* sum, uint32_t n, uint32_t* err, hipStream_t st) {
    const dim3 g(grid_for(n, TPB * 4)), b(TPB);
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(TPB), 0, st, err, 1ull, 0u, (const Ctrl*)nullptr, Gate{});
    if (wt == 1) hipLaunchKernelGGL(k_verify<1>, g, b, 0, st, succ, weight, rank, root, sum, n, err);
    else if (wt == 2) hipLaunchKernelGGL(k_verify<2>, g, b, 0, st, succ, weight, rank, root, sum, n, err);
    else hipLaunchKernelGGL(k_verify<0>, g, b, 0, st, succ, weight, rank, root, sum, n, err);
    return hipGetLastError();
}


// ----------------------------------------------------------- debug writes --
// Sets the counters of a call (null: count nothing) and clears them and the
// control block's debug bit (without validation nothing else clears it).
__global__ __launch_bounds__(TPB) void k_dbg_begin(DbgWrites d, uint32_t* __restrict__ base, uint64_t words,
                                                   Ctrl* ctrl) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
#if LR_DEBUG_WRITES
        g_dbg = d;
#endif
        ctrl->err &= ~ERR_DEBUG_WRITES;
    }
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride) base[i] = 0;
}

// Every slot of the levels from `slot_from` on written once, every mark at
// most once (only when the plain path ran to its end); then counting stops.
__global__ __launch_bounds__(TPB) void k_dbg_check(DbgWrites d, DbgSizes sz, uint32_t levels, uint32_t slot_from,
                                                   Ctrl* ctrl) {
#if LR_DEBUG_WRITES
    if (blockIdx.x == 0 && threadIdx.x == 0) g_dbg = DbgWrites{};
#endif
    if (ctrl->mode != MODE_PLAIN) return;
    const uint32_t stride = gridDim.x * blockDim.x;
    bool bad = false;
    for (uint32_t l = 0; l < levels; ++l) {
        for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < sz.m[l]; i += stride) {
            if (l >= slot_from && d.slot[l][i] != 1u) bad = true;
            if (d.mark[l][i] > 1u) bad = true;
        }
    }
    if (bad) atomicOr(&ctrl->err, ERR_DEBUG_WRITES);
}

hipError_t run_debug_begin(const RunArgs& a, const Plan& p) {
    if (!LR_DEBUG_WRITES) return hipSuccess;
    DbgWrites d{};
    uint64_t words = 0;
    const bool plain = !p.local && !p.spawn && !a.lplan;
    if (plain) {
        size_t off = p.off_dbg;
        for (uint32_t l = 0; l < p.levels; ++l) {
            d.slot[l] = reinterpret_cast<uint32_t*>(a.ws + off);
            d.mark[l] = d.slot[l] + p.m[l];
            off += (p.m[l] * 8 + ALIGN - 1) / ALIGN * ALIGN;
        }
        words = (off - p.off_dbg) / 4;
    }
    uint32_t* base = reinterpret_cast<uint32_t*>(a.ws + p.off_dbg);
    hipLaunchKernelGGL(k_dbg_begin, dim3(std::max<uint32_t>(1, grid_for(words, TPB * 4))), dim3(TPB), 0, a.stream, d,
                       base, words, reinterpret_cast<Ctrl*>(a.ws + p.off_ctrl));
    return hipGetLastError();
}

hipError_t run_debug_check(const RunArgs& a, const Plan& p) {
    if (!LR_DEBUG_WRITES) return hipSuccess;
    const bool plain = !p.local && !p.spawn && !a.lplan;
    DbgWrites d{};
    DbgSizes sz{};
    uint32_t levels = 0;
    if (plain) {
        size_t off = p.off_dbg;
        levels = p.levels;
        for (uint32_t l = 0; l < p.levels; ++l) {
            d.slot[l] = reinterpret_cast<uint32_t*>(a.ws + off);
            d.mark[l] = d.slot[l] + p.m[l];
            sz.m[l] = (uint32_t)p.m[l];
            off += (p.m[l] * 8 + ALIGN - 1) / ALIGN * ALIGN;
        }
    }
    Ctrl* ctrl = reinterpret_cast<Ctrl*>(a.ws + p.off_ctrl);
    // level 0 writes slots only when it is not chased through the visit log
    hipLaunchKernelGGL(k_dbg_check, dim3(std::max<uint32_t>(1, grid_for(p.m[0], TPB * 4))), dim3(TPB), 0, a.stream, d,
                       sz, levels, p.log0 ? 1u : 0u, ctrl);
    return hipGetLastError();
}

}  // namespace lr
