// C ABI of liblr.so: argument checks, planning, workspace carving, dispatch.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "device.hpp"
#include "lr.h"
#include "plan.hpp"
#include "runner.hpp"

namespace lr {

static inline size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

static uint64_t mix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static bool pow2_in(uint32_t k, uint32_t lo, uint32_t hi) { return k >= lo && k <= hi && (k & (k - 1)) == 0; }

static uint32_t ilog2(uint32_t k) {
    uint32_t r = 0;
    while ((1u << r) < k) ++r;
    return r;
}

// Default spacing: long first-level walks amortise the per-ruler work on big
// inputs; upper levels are cache resident and use short walks to keep the
// longest walk (about k ln(m/k) steps) short. Inputs below 2^25 elements are
// bound by that longest walk on every level (each step a dependent load), so
// they take shorter walks: 8 on the first level below 2^23 elements, 16 up to
// 2^24, 32 beyond; above the first level 4 below 2^17 elements, 8 up to 2^20,
// 16 beyond (measured per size on MI355X: 6-18 % faster from 2^17 to 2^23;
// from 2^25 on the longer walks stay ahead). From 2^25 the first level takes
// 32 up to 3 * 2^26 elements and 64 beyond (32 is 7 % faster at 2^26 and
// 2 % at 2^27, 64 is 2 % faster at 2^28); weighted inputs (16 B records)
// take 64 from 2^27 (32 is 2-6 % faster at 2^26, 2 % slower on a 2^27
// forest), a plan sized for a capacity (capped) from 2^26. The last level
// takes the smallest spacing that brings it under base_max.
constexpr uint64_t SHORT_WALKS_BELOW = 1ull << 25;
static uint32_t default_spacing(uint32_t l, uint64_t m, uint32_t base_max, bool short_walks, bool weighted,
                                bool capped) {
    uint32_t k;
    if (short_walks) {
        if (l == 0) k = (m >= (1ull << 24)) ? 32 : (m >= (1ull << 23)) ? 16 : 8;
        else k = (m >= (1ull << 20)) ? 16 : (m >= (1ull << 17)) ? 8 : 4;
    } else {
        const uint64_t k64 = capped ? (1ull << 26) : weighted ? (1ull << 27) : (3ull << 26);
        if (l == 0) k = (m >= k64) ? 64 : (m >= (1ull << 23) ? 32 : 16);
        else k = 16;
    }
    uint32_t kmin = 2;
    while ((m + kmin - 1) / kmin > base_max && kmin < 4096) kmin <<= 1;
    return (kmin <= k) ? kmin : k;
}

// Levels, spacing and seeds for a level-0 list of (at most) m0 elements.
// capped: m0 is a capacity (the contracted path's plan), whose actual size
// is usually far below it; its first level switches to spacing 64 from
// 2^26, which keeps its level count (and the launches it enqueues on every
// call) down.
static lr_status plan_levels(uint64_t m0, bool weighted, const lr_opts* o, bool user_spacing, Plan* p,
                             uint32_t max_levels = LR_MAX_LEVELS, bool capped = false) {
    p->weighted = weighted;
    p->rec_bytes = weighted ? 16 : 8;
    uint32_t bm = (o && o->base_max) ? o->base_max : (weighted ? 4096u : 8192u);
    if (bm < 1 || bm > BASE_MAX_LIMIT) return LR_ERR_INVALID_ARG;
    const bool user_spacing_set = user_spacing && o && o->spacing[0];
    const bool short_walks = m0 < SHORT_WALKS_BELOW;
    if (!(o && o->base_max) && !user_spacing_set && short_walks) {
        // inputs below 2^25: a base case of twice the size (16384 elements
        // unweighted, 8192 weighted) where it saves a level (a level costs
        // more than the larger base case)
        auto levels_for = [m0](uint32_t b) {
            uint64_t m = m0;
            uint32_t L = 0;
            while (m > b && L < (uint32_t)LR_MAX_LEVELS) {
                const uint32_t k = default_spacing(L, m, b, true, false, false);
                m = (m + k - 1) / k;
                ++L;
            }
            return L;
        };
        if (levels_for(2 * bm) < levels_for(bm)) bm = 2 * bm;
    }
    p->base_max = bm;
    const uint32_t lw = (o && o->lane_walks) ? o->lane_walks : 1u;
    if (lw > 2) return LR_ERR_INVALID_ARG;
    p->lane_walks = lw;
    uint32_t rf = (o && o->refill) ? o->refill : 1u;
    if (rf > 64 * lw) return LR_ERR_INVALID_ARG;
    p->refill = rf;
    const uint32_t bo = (o && o->log_off_bits) ? o->log_off_bits : 31u;
    if (bo > 31) return LR_ERR_INVALID_ARG;
    p->bocap = bo;
    const uint64_t seed = o ? o->seed : 0;
    if (o) {
        for (int l = 0; l < LR_MAX_LEVELS && o->spacing[l]; ++l)
            if (!pow2_in(o->spacing[l], 2, 4096)) return LR_ERR_INVALID_ARG;
    }
    auto fill = [&](bool sw) {
        uint64_t m = m0;
        uint32_t L = 0;
        bool user = user_spacing_set;
        p->m[0] = m0;
        while (m > bm) {
            if (L >= max_levels) return LR_ERR_UNSUPPORTED;
            uint32_t k;
            if (user && o->spacing[L]) k = o->spacing[L];
            else { user = false; k = default_spacing(L, m, bm, sw, weighted, capped); }
            p->log2k[L] = ilog2(k);
            p->lseed[L] = (uint32_t)mix64(seed * 0x2545f4914f6cdd1dULL + 0x1000 + L);
            m = (m + k - 1) / k;
            ++L;
            p->m[L] = m;
        }
        p->levels = L;
        return LR_OK;
    };
    // short walks need more levels: where they would pass the level limit (a
    // tiny base_max, many user levels of spacing 2, spawning's extra input
    // level) the long walks are taken
    if (short_walks && fill(true) == LR_OK) return LR_OK;
    return fill(false);
}

// Visit log and grouping areas (level 0 in log mode), then per level the
// slot, walk-record and tile-count arrays. Returns the end offset.
static size_t layout_levels(Plan* p, size_t off) {
    const uint64_t n = p->m[0];
    const uint32_t L = p->levels;
    const bool weighted = p->weighted;
    if (p->log0) {
        p->chunk = LOG_CHUNK;
        // a chunk is given up only when a step's records (at most 64 per walk a lane holds) do not fit
        p->max_chunks = (uint32_t)((n + LOG_CHUNK - 128) / (LOG_CHUNK - 127)) + LOG_MAX_WAVES + 1;
        const size_t cap = (size_t)p->max_chunks * LOG_CHUNK;
        uint32_t lg = 0;
        while ((1ull << lg) < n) ++lg;
        p->s2 = PLACE_FINE_SHIFT;                               // a fine range's outputs fit one workgroup's LDS
        // split the fan-out over the two passes, a little more of it in the
        // second: the first pass's frontiers are shared by every XCD, so its
        // partial lines are written back from several L2s, while the second
        // pass's frontiers stay in one XCD's L2. Weighted records (four
        // arrays) gain more from longer first-pass runs.
        const uint32_t bias = weighted ? LR_PLACE_COARSE_BIAS_W : LR_PLACE_COARSE_BIAS;
        p->s1 = p->s2 + std::max(1u, (lg - p->s2 + 1) / 2 + bias);
        if ((1ull << p->s1) >= 2 * n) p->s1 = std::max(p->s2 + 1, lg);
        p->nb1 = (uint32_t)((n + (1ull << p->s1) - 1) >> p->s1);
        p->nb2 = (uint32_t)((n + (1ull << p->s2) - 1) >> p->s2);
        const int arrays = weighted ? 4 : 3;
        for (int i = 0; i < arrays; ++i) {
            p->off_log[i] = off;
            off += align_up(cap * (i == 3 ? 8 : 4));
        }
        // packed records: 8 B per entry over the first two arrays (adjacent:
        // cap * 4 is a multiple of the alignment), then the continuations.
        // Successive continuations of one walk are at least 2^bo apart in
        // offset (bo >= the smallest offset width), so a level has at most
        // (its offsets' range) >> bo of them: the visits for a plain level 0,
        // the input's elements for a contracted list, whose steps count
        // whole chains. A wavefront's block wastes fewer ids than the next
        // block's first step uses.
        static_assert((LOG_CHUNK * 4) % ALIGN == 0, "packed records span the first two log arrays");
        p->pack = n <= LOG_PACK_MAX_N;
        if (p->pack) {
            const uint32_t bo_min = std::min(p->bocap, LOG_BO_MIN);
            const uint64_t range = std::max<uint64_t>(cap, p->local ? p->lc_n : n);
            p->ccap = (uint32_t)(2 * (range >> bo_min) + (uint64_t)CONT_GRAB * (LOG_MAX_WAVES + 1));
            p->off_conts = off;
            off += align_up((size_t)p->ccap * 8);
        }
        for (int i = 0; i < arrays; ++i) {
            p->off_p[i] = off;
            off += align_up((size_t)n * (i == 3 ? 8 : 4));
        }
        // weighted: the arrays after the first hold the interleaved (successor,
        // weight) records during the level-0 chase (16 B per element)
        p->off_fill = off;
        off += align_up((size_t)fill_words(p->nb1, p->nb2) * 4);
    }
    for (uint32_t l = 0; l < std::max(L, 1u); ++l) {
        const uint64_t ml = p->m[l];
        const uint64_t S = (l < L) ? p->m[l + 1] : 0;
        if (l == 0 && p->log0) {
            p->off_slot[0] = p->off_p[0];  // no slot array: marks and counts live in the grouping area
        } else {
            p->off_slot[l] = off;
            off += align_up(std::max<size_t>((size_t)ml * p->rec_bytes, 16));
        }
        if (l < L) {
            p->ntiles[l] = (uint32_t)((ml + TILE - 1) / TILE);
            p->off_eb[l] = off;
            off += align_up((size_t)(S + ml) * p->rec_bytes);
            p->off_tile[l] = off;
            off += align_up((size_t)(p->ntiles[l] + 1) * 4);
        }
    }
    return off;
}

// Tile-local contraction of an n-element input: start counts, start bits,
// per-element chain positions (and weights), staged and final contracted
// records (the latter for at most m[0] of them). Returns the end offset.
static size_t layout_local(Plan* p, uint64_t n, size_t off) {
    p->local = true;
    p->lc_n = n;
    p->lc_ntiles = (uint32_t)((n + LOCAL_TILE - 1) / LOCAL_TILE);
    p->off_lc_cnt = off;
    off += align_up((size_t)(p->lc_ntiles + 1) * 4);
    p->off_lc_dir = off;
    off += align_up((size_t)((n + 31) / 32) * 8);
    p->off_lc_pos = off;
    off += align_up((size_t)n * 4);
    if (p->weighted) {
        p->off_lc_wd = off;
        off += align_up((size_t)n * 8);
    }
    p->off_lc_stage = off;
    off += align_up(std::max<size_t>((size_t)n * p->rec_bytes, 16));
    p->off_lrec = off;
    off += align_up(std::max<size_t>((size_t)p->m[0] * p->rec_bytes, 16));
    return off;
}

// Ruler spawning over an n-element input: slots, predecessor bytes and head
// tile counts of the input level, and the records of its walks (at most n).
static size_t layout_spawn(Plan* p, uint64_t n, size_t off) {
    p->spawn = true;
    p->sp_n = n;
    p->sp_ntiles = (uint32_t)((n + TILE - 1) / TILE);
    p->off_sp_slot = off;
    off += align_up(std::max<size_t>((size_t)n * p->rec_bytes, 16));
    p->off_sp_hp = off;
    off += align_up((size_t)n + 16);
    p->off_sp_tile = off;
    off += align_up((size_t)(p->sp_ntiles + 1) * 4);
    p->off_lrec = off;
    off += align_up(std::max<size_t>((size_t)n * p->rec_bytes, 16));
    return off;
}

// Level 0 through the visit log: from LOG_MIN_N elements on, or on request.
static bool use_log(uint64_t m0, uint32_t levels, const lr_opts* o) {
    if (levels < 1) return false;
    return m0 >= LOG_MIN_N || (o && (o->flags & LR_VISIT_LOG) && m0 >= LOG_FORCE_MIN_N);
}

lr_status make_plans(uint64_t n, bool weighted, const lr_opts* o, uint32_t batch_count, PlanSet* ps) {
    *ps = PlanSet{};
    if (n >= (1ull << 31)) return LR_ERR_UNSUPPORTED;
    // plan options left at their defaults take the autotune cache's entry
    // for this device and size bucket, if there is one
    lr_opts tuned;
    if (!(o && ((o->flags & LR_SPAWN) || o->spacing[0] || o->base_max || o->lane_walks || o->refill))) {
        tuned = o ? *o : lr_opts{};
        if (tune_lookup(n, weighted, &tuned)) o = &tuned;
    }
    const bool force = o && (o->flags & LR_LOCAL);
    const bool never = o && (o->flags & LR_NO_LOCAL);
    const bool spawn = o && (o->flags & LR_SPAWN);
    if (force && never) return LR_ERR_INVALID_ARG;
    if (force && spawn) return LR_ERR_INVALID_ARG;
    Plan* p = &ps->p;
    lr_opts upper = o ? *o : lr_opts{};  // spawning: spacing[0] samples the input, the rest the levels above
    if (spawn) {
        for (int l = 0; l + 1 < LR_MAX_LEVELS; ++l) upper.spacing[l] = o->spacing[l + 1];
        upper.spacing[LR_MAX_LEVELS - 1] = 0;
        if (o->spacing[0] && !pow2_in(o->spacing[0], 2, 4096)) return LR_ERR_INVALID_ARG;
    }
    // the input level of the spawning chase keeps its head count in the last
    // Ctrl level entry
    lr_status s = plan_levels(n, weighted, spawn ? &upper : o, true, p, spawn ? MAXL - 2 : LR_MAX_LEVELS);
    if (s != LR_OK) return s;
    size_t off = 0;
    p->off_ctrl = off;
    off += align_up(sizeof(Ctrl));
    p->off_hsum = off;
    off += align_up((size_t)HEADSUM_BLOCKS * 16);
    const size_t body = off;
    if (spawn) {
        const uint32_t k0 = o->spacing[0] ? o->spacing[0] : SPAWN_K0;
        p->sp_log2k = ilog2(k0);
        p->sp_seed = (uint32_t)mix64(o->seed * 0x2545f4914f6cdd1dULL + 0x2000);
        p->log0 = false;  // the walks' list is a small fraction of n on the inputs spawning is for
        off = layout_levels(p, layout_spawn(p, n, body));
    } else if (force) {
        p->log0 = use_log(n, p->levels, o);
        off = layout_levels(p, layout_local(p, n, body));
    } else {
        p->log0 = use_log(n, p->levels, o);
        off = layout_levels(p, body);
    }
    // Automatic contraction: the contracted path's arrays share the workspace
    // with the plain path's (only one of them runs), after the common header.
    // (debug builds count the plain path's writes: no automatic contraction there)
    ps->autol = !force && !never && !spawn && p->levels >= 1 && n >= LOCAL_AUTO_MIN_N && !LR_DEBUG_WRITES;
    if (ps->autol) {
        Plan* q = &ps->lp;
        lr_opts lo = o ? *o : lr_opts{};
        for (int l = 0; l < LR_MAX_LEVELS; ++l) lo.spacing[l] = 0;  // user spacing describes the plain levels
        s = plan_levels(local_auto_cap(n), weighted, &lo, false, q, LR_MAX_LEVELS, true);
        if (s != LR_OK) return s;
        q->off_ctrl = p->off_ctrl;
        q->off_hsum = p->off_hsum;
        q->log0 = use_log(q->m[0], q->levels, o);
        off = std::max(off, layout_levels(q, layout_local(q, n, body)));
    }
    // the bounded fallback (a walk reached its step cap): two record arrays
    // over the input, after the common header
    if (p->levels >= 1 || spawn) {
        p->off_fb = body;
        off = std::max(off, body + 2 * align_up((size_t)n * p->rec_bytes + 16));
        ps->lp.off_fb = body;
    }
    if (batch_count) {
        p->batch_count = batch_count;
        p->off_batch_succ = off;
        off += align_up((size_t)n * 4 + 16);
        p->off_batch_desc = off;
        off += align_up((size_t)batch_count * sizeof(BatchDesc));
        p->off_batch_bases = off;
        off += align_up(batch_table_bytes(batch_count));
        p->off_batch_hdr = off;
        off += align_up(sizeof(BatchHdr));
        p->off_batch_part = off;  // at most n / BATCH_CHUNK + one partial chunk per request
        off += align_up(((size_t)n / BATCH_CHUNK + batch_count + 1) * 16);
        p->off_batch_sums = off;
        off += align_up((size_t)batch_count * 16);
    }
    if (LR_DEBUG_WRITES) {
        p->off_dbg = off;
        for (uint32_t l = 0; l < p->levels; ++l) off += align_up((size_t)p->m[l] * 8);
    }
    p->total = off + ALIGN;  // room to align the caller's base pointer
    ps->lp.total = p->total;
    return LR_OK;
}

lr_status make_plan(uint64_t n, bool weighted, const lr_opts* o, uint32_t batch_count, Plan* p) {
    PlanSet ps;
    const lr_status s = make_plans(n, weighted, o, batch_count, &ps);
    *p = ps.p;
    return s;
}

// ------------------------------------------------------------- profiling --
struct ProfState {
    hipEvent_t ev[EV_COUNT] = {};
    bool made = false, valid = false;
    const uint32_t* mode = nullptr;  // the profiled call's path word (device), null without walks
};
static thread_local ProfState g_prof;

// The profiled call's path word, for lr_profile_last (plans with walks only).
static void prof_capped(const RunArgs& a, const Plan& p) {
    if (a.ev) g_prof.mode = (p.levels >= 1 || p.spawn) ? &reinterpret_cast<const Ctrl*>(a.ws + p.off_ctrl)->mode
                                                        : nullptr;
}

static hipEvent_t* prof_events(bool on) {
    if (!on) return nullptr;
    if (!g_prof.made) {
        for (auto& e : g_prof.ev)
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
        g_prof.made = true;
    }
    g_prof.valid = true;
    return g_prof.ev;
}

static char* carve(void* ws) { return reinterpret_cast<char*>(align_up(reinterpret_cast<uintptr_t>(ws))); }

static lr_status finish(hipError_t e, const RunArgs& a, const Plan& p) {
    if (e != hipSuccess) return LR_ERR_HIP;
    if (a.validate) {
        Ctrl c{};
        if (hipMemcpyAsync(&c, a.ws + p.off_ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, a.stream) != hipSuccess)
            return LR_ERR_HIP;
        if (hipStreamSynchronize(a.stream) != hipSuccess) return LR_ERR_HIP;
        const bool walks = p.levels >= 1 || p.spawn;
        const uint32_t err = (walks && c.mode == MODE_FALLBACK) ? (c.err & (ERR_INPUT | ERR_FALLBACK_CYCLE)) : c.err;
        if (err) return LR_ERR_BAD_LIST;
    }
    return LR_OK;
}

static lr_status check_base_lds(const Plan& p) {
    const uint64_t mL = p.m[p.levels];
    if (base_lds_bytes(mL, p.weighted) > device_max_lds()) return LR_ERR_UNSUPPORTED;
    if (p.log0 && ((size_t)1 << p.s2) * (p.weighted ? 16 : 8) > device_max_lds()) return LR_ERR_UNSUPPORTED;
    // the grouping tiles' LDS is sized for at most PLACE_MAX_RANGES ranges per pass
    if (p.log0 && (p.nb1 > PLACE_MAX_RANGES || (1u << (p.s1 - p.s2)) > PLACE_MAX_RANGES)) return LR_ERR_UNSUPPORTED;
    return LR_OK;
}

static lr_status rank_common(const uint32_t* succ, const void* weight, int wt, bool weighted, int64_t* sum,
                             uint32_t* rank, uint32_t* root, uint64_t n, void* ws, size_t ws_bytes,
                             const lr_opts* opts, void* stream, void* rec = nullptr) {
    PlanSet ps;
    lr_status s = make_plans(n, weighted, opts, 0, &ps);
    if (s != LR_OK) return s;
    const Plan& p = ps.p;
    if (!ws || ws_bytes < p.total) return LR_ERR_WORKSPACE;
    if ((s = check_base_lds(p)) != LR_OK) return s;
    if (ps.autol && (s = check_base_lds(ps.lp)) != LR_OK) return s;
    RunArgs a;
    a.plan = &p;
    a.lplan = ps.autol ? &ps.lp : nullptr;
    a.succ = succ;
    a.weight = weight;
    a.wt = wt;
    a.rank = rank;
    a.root = root;
    a.sum = sum;
    a.rec = rec;
    a.ws = carve(ws);
    a.stream = static_cast<hipStream_t>(stream);
    a.validate = opts && (opts->flags & LR_VALIDATE);
    a.ev = prof_events(opts && (opts->flags & LR_PROFILE));
    prof_capped(a, p);
    if (LR_DEBUG_WRITES) {
        hipError_t e = run_debug_begin(a, p);
        if (e == hipSuccess) e = run_srs(a);
        if (e == hipSuccess) e = run_debug_check(a, p);
        if (e != hipSuccess) return LR_ERR_HIP;
        Ctrl c{};
        if (hipMemcpyAsync(&c, a.ws + p.off_ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, a.stream) != hipSuccess ||
            hipStreamSynchronize(a.stream) != hipSuccess)
            return LR_ERR_HIP;
        if (c.err & ERR_DEBUG_WRITES) return LR_ERR_BAD_LIST;
        return finish(hipSuccess, a, p);
    }
    return finish(run_srs(a), a, p);
}

lr_status prefix_sum_records(const uint32_t* succ, const void* weight, int wt, void* rec, uint64_t n, void* ws,
                             size_t ws_bytes, const lr_opts* opts, void* stream) {
    if (wt < 0 || wt > 3) return LR_ERR_INVALID_ARG;
    if (n == 0) return LR_OK;
    if (!succ || !rec || (wt == 0) != (weight == nullptr)) return LR_ERR_INVALID_ARG;
    if (n >= (1ull << 31)) return LR_ERR_UNSUPPORTED;
    return rank_common(succ, weight, wt, true, nullptr, nullptr, nullptr, n, ws, ws_bytes, opts, stream, rec);
}

}  // namespace lr

using namespace lr;

extern "C" {

const char* lr_status_string(lr_status s) {
    switch (s) {
        case LR_OK: return "LR_OK";
        case LR_ERR_INVALID_ARG: return "LR_ERR_INVALID_ARG: null required pointer, bad enum or bad option";
        case LR_ERR_UNSUPPORTED: return "LR_ERR_UNSUPPORTED: size or option beyond what the library or device supports";
        case LR_ERR_WORKSPACE: return "LR_ERR_WORKSPACE: workspace missing or smaller than required";
        case LR_ERR_OUT_OF_MEMORY: return "LR_ERR_OUT_OF_MEMORY: device allocation failed";
        case LR_ERR_BAD_LIST: return "LR_ERR_BAD_LIST: input is not a forest of lists";
        case LR_ERR_HIP: return "LR_ERR_HIP: a HIP runtime call failed";
    }
    return "unknown lr_status";
}

lr_status lr_plan_query(uint64_t n, lr_wtype w, const lr_opts* opts, lr_plan* out) {
    if (!out) return LR_ERR_INVALID_ARG;
    if (w != LR_W_NONE && w != LR_W_I32 && w != LR_W_I64) return LR_ERR_INVALID_ARG;
    Plan p;
    lr_status s = make_plan(n, w != LR_W_NONE, opts, 0, &p);
    if (s != LR_OK) return s;
    memset(out, 0, sizeof(*out));
    out->levels = p.levels;
    out->base_max = p.base_max;
    for (uint32_t l = 0; l <= p.levels; ++l) out->m[l] = p.m[l];
    for (uint32_t l = 0; l < p.levels; ++l) out->spacing[l] = 1u << p.log2k[l];
    out->workspace_bytes = p.total;
    return LR_OK;
}

size_t lr_workspace_bytes(uint64_t n, lr_wtype w, const lr_opts* opts) {
    if (w != LR_W_NONE && w != LR_W_I32 && w != LR_W_I64) return 0;
    Plan p;
    if (make_plan(n, w != LR_W_NONE, opts, 0, &p) != LR_OK) return 0;
    return p.total;
}

lr_status lr_rank(const uint32_t* succ, uint32_t* rank, uint32_t* root, uint64_t n, void* ws, size_t ws_bytes,
                  const lr_opts* opts, void* stream) {
    if (n == 0) return LR_OK;
    if (!succ || !rank) return LR_ERR_INVALID_ARG;
    if (n >= (1ull << 31)) return LR_ERR_UNSUPPORTED;
    return rank_common(succ, nullptr, 0, false, nullptr, rank, root, n, ws, ws_bytes, opts, stream);
}

lr_status lr_prefix_sum(const uint32_t* succ, const void* weight, lr_wtype w, int64_t* sum, uint32_t* rank,
                        uint32_t* root, uint64_t n, void* ws, size_t ws_bytes, const lr_opts* opts, void* stream) {
    if (w != LR_W_NONE && w != LR_W_I32 && w != LR_W_I64) return LR_ERR_INVALID_ARG;
    if (n == 0) return LR_OK;
    if (!succ || !sum) return LR_ERR_INVALID_ARG;
    if ((w == LR_W_NONE) != (weight == nullptr)) return LR_ERR_INVALID_ARG;
    if (n >= (1ull << 31)) return LR_ERR_UNSUPPORTED;
    return rank_common(succ, weight, (int)w, true, sum, rank, root, n, ws, ws_bytes, opts, stream);
}

size_t lr_wyllie_workspace_bytes(uint64_t n, lr_wtype w) {
    if (w != LR_W_NONE && w != LR_W_I32 && w != LR_W_I64) return 0;
    if (n >= (1ull << 31)) return 0;
    const size_t rec = (w == LR_W_NONE) ? 8 : 16;
    return 2 * align_up((size_t)n * rec + 16) + ALIGN;
}

static lr_status wyllie_common(const uint32_t* succ, const void* weight, lr_wtype w, bool weighted, int64_t* sum,
                               uint32_t* rank, uint32_t* root, uint64_t n, void* ws, size_t ws_bytes, void* stream) {
    const size_t need = lr_wyllie_workspace_bytes(n, weighted ? (w == LR_W_NONE ? LR_W_I64 : w) : LR_W_NONE);
    if (!ws || ws_bytes < need) return LR_ERR_WORKSPACE;
    RunArgs a;
    a.succ = succ;
    a.weight = weight;
    a.wt = (int)w;
    a.rank = rank;
    a.root = root;
    a.sum = sum;
    a.ws = carve(ws);
    a.stream = static_cast<hipStream_t>(stream);
    return run_wyllie(a, n, weighted) == hipSuccess ? LR_OK : LR_ERR_HIP;
}

lr_status lr_rank_wyllie(const uint32_t* succ, uint32_t* rank, uint32_t* root, uint64_t n, void* ws,
                         size_t ws_bytes, void* stream) {
    if (n == 0) return LR_OK;
    if (!succ || !rank) return LR_ERR_INVALID_ARG;
    if (n >= (1ull << 31)) return LR_ERR_UNSUPPORTED;
    return wyllie_common(succ, nullptr, LR_W_NONE, false, nullptr, rank, root, n, ws, ws_bytes, stream);
}

lr_status lr_prefix_sum_wyllie(const uint32_t* succ, const void* weight, lr_wtype w, int64_t* sum, uint32_t* rank,
                               uint32_t* root, uint64_t n, void* ws, size_t ws_bytes, void* stream) {
    if (w != LR_W_NONE && w != LR_W_I32 && w != LR_W_I64) return LR_ERR_INVALID_ARG;
    if (n == 0) return LR_OK;
    if (!succ || !sum) return LR_ERR_INVALID_ARG;
    if ((w == LR_W_NONE) != (weight == nullptr)) return LR_ERR_INVALID_ARG;
    if (n >= (1ull << 31)) return LR_ERR_UNSUPPORTED;
    return wyllie_common(succ, weight, w, true, sum, rank, root, n, ws, ws_bytes, stream);
}

size_t lr_batch_workspace_bytes(const lr_request* reqs, uint32_t count, const lr_opts* opts) {
    if (!reqs && count) return 0;
    uint64_t N = 0;
    for (uint32_t i = 0; i < count; ++i) N += reqs[i].n;
    Plan p;
    if (make_plan(N, false, opts, std::max(count, 1u), &p) != LR_OK) return 0;
    return p.total;
}

}  // extern "C"

namespace lr {

// Enqueue a batch: the request table is written on the device from kernel
// arguments (no host staging, no synchronisation), then the method runs once
// over the concatenation.
lr_status batch_enqueue(const lr_request* reqs, uint32_t count, void* ws, size_t ws_bytes, const lr_opts* opts,
                        hipStream_t st) {
    uint64_t N = 0;
    for (uint32_t i = 0; i < count; ++i) {
        if (reqs[i].n && (!reqs[i].succ || !reqs[i].rank)) return LR_ERR_INVALID_ARG;
        N += reqs[i].n;
    }
    if (N >= (1ull << 31)) return LR_ERR_UNSUPPORTED;
    if (N == 0) return LR_OK;
    PlanSet ps;
    lr_status s = make_plans(N, false, opts, count, &ps);
    if (s != LR_OK) return s;
    const Plan& p = ps.p;
    if (!ws || ws_bytes < p.total) return LR_ERR_WORKSPACE;
    if ((s = check_base_lds(p)) != LR_OK) return s;
    if (ps.autol && (s = check_base_lds(ps.lp)) != LR_OK) return s;
    uint32_t chunks = 0;
    for (uint32_t i = 0; i < count; ++i) chunks += (uint32_t)((reqs[i].n + BATCH_CHUNK - 1) / BATCH_CHUNK);
    char* w = carve(ws);
    if (run_batch_table(reqs, count, p, w, false, chunks, st) != hipSuccess) return LR_ERR_HIP;
    RunArgs a;
    a.plan = &p;
    a.lplan = ps.autol ? &ps.lp : nullptr;
    a.succ = reinterpret_cast<const uint32_t*>(w + p.off_batch_succ);
    a.desc = reinterpret_cast<const BatchDesc*>(w + p.off_batch_desc);
    a.bases = reinterpret_cast<const uint32_t*>(w + p.off_batch_bases);
    a.boff = a.bases + count + 1;
    a.bhdr = reinterpret_cast<const BatchHdr*>(w + p.off_batch_hdr);
    a.count = count;
    for (uint32_t i = 0; i < count; ++i) a.any_root |= reqs[i].root != nullptr;
    a.ws = w;
    a.stream = st;
    a.validate = opts && (opts->flags & LR_VALIDATE);
    a.ev = prof_events(opts && (opts->flags & LR_PROFILE));
    prof_capped(a, p);
    if (LR_DEBUG_WRITES) {
        hipError_t e = run_debug_begin(a, p);
        if (e == hipSuccess) e = run_srs(a);
        if (e == hipSuccess) e = run_debug_check(a, p);
        if (e != hipSuccess) return LR_ERR_HIP;
        Ctrl c{};
        if (hipMemcpyAsync(&c, a.ws + p.off_ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, a.stream) != hipSuccess ||
            hipStreamSynchronize(a.stream) != hipSuccess)
            return LR_ERR_HIP;
        if (c.err & ERR_DEBUG_WRITES) return LR_ERR_BAD_LIST;
        return finish(hipSuccess, a, p);
    }
    return finish(run_srs(a), a, p);
}

}  // namespace lr

extern "C" lr_status lr_rank_batch(const lr_request* reqs, uint32_t count, void* ws, size_t ws_bytes,
                                   const lr_opts* opts, void* stream) {
    if (count == 0) return LR_OK;
    if (!reqs) return LR_ERR_INVALID_ARG;
    return batch_enqueue(reqs, count, ws, ws_bytes, opts, static_cast<hipStream_t>(stream));
}

// ------------------------------------------------------------ batch graph --
// A batch planned for a capacity (max_elements, max_requests) and captured
// once as a HIP graph; each launch writes the request table (kernel
// arguments, a few small launches) and replays the graph, whose kernels read
// the actual sizes from the device.
struct lr_batch_graph {
    lr::Plan plan;
    char* ws = nullptr;
    uint32_t max_requests = 0;
    uint64_t max_elements = 0;
    uint32_t max_chunks = 0;
    bool want_root = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace lr {

static lr_status graph_plan(const lr_batch_graph_config* c, Plan* p) {
    if (!c || c->max_requests == 0 || c->max_elements == 0) return LR_ERR_INVALID_ARG;
    if (c->max_elements >= (1ull << 31)) return LR_ERR_UNSUPPORTED;
    // no synchronising or event-recording options in a graph; the path with
    // device-side sizes is the plain one (no automatic contraction, no spawning)
    if (c->opts.flags & (LR_VALIDATE | LR_PROFILE | LR_SPAWN | LR_LOCAL)) return LR_ERR_INVALID_ARG;
    lr_opts o = c->opts;
    o.flags |= LR_NO_LOCAL;
    return make_plan(c->max_elements, false, &o, c->max_requests, p);
}

}  // namespace lr

extern "C" {

size_t lr_batch_graph_workspace_bytes(const lr_batch_graph_config* cfg) {
    Plan p;
    if (lr::graph_plan(cfg, &p) != LR_OK) return 0;
    return p.total;
}

lr_status lr_batch_graph_create(const lr_batch_graph_config* cfg, void* ws, size_t ws_bytes, lr_batch_graph** out) {
    if (!out) return LR_ERR_INVALID_ARG;
    *out = nullptr;
    Plan p;
    lr_status s = lr::graph_plan(cfg, &p);
    if (s != LR_OK) return s;
    if (!ws || ws_bytes < p.total) return LR_ERR_WORKSPACE;
    if ((s = check_base_lds(p)) != LR_OK) return s;
    auto* g = new lr_batch_graph();
    g->plan = p;
    g->ws = carve(ws);
    g->max_requests = cfg->max_requests;
    g->max_elements = cfg->max_elements;
    g->max_chunks = (uint32_t)(cfg->max_elements / BATCH_CHUNK + cfg->max_requests);
    g->want_root = cfg->want_root != 0;
    // capture the ranking sequence on a stream of our own
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
        delete g;
        return LR_ERR_HIP;
    }
    RunArgs a;
    a.plan = &g->plan;
    a.succ = reinterpret_cast<const uint32_t*>(g->ws + p.off_batch_succ);
    a.desc = reinterpret_cast<const BatchDesc*>(g->ws + p.off_batch_desc);
    a.bases = reinterpret_cast<const uint32_t*>(g->ws + p.off_batch_bases);
    a.boff = a.bases + cfg->max_requests + 1;
    a.bhdr = reinterpret_cast<const BatchHdr*>(g->ws + p.off_batch_hdr);
    a.count = cfg->max_requests;
    a.any_root = g->want_root;
    a.dev_sizes = true;
    a.ws = g->ws;
    a.stream = cs;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    hipError_t er = (e == hipSuccess) ? run_srs(a) : e;
    hipGraph_t graph = nullptr;
    if (e == hipSuccess) e = hipStreamEndCapture(cs, &graph);
    if (e == hipSuccess) e = er;
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    g->graph = graph;
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        lr_batch_graph_destroy(g);
        return LR_ERR_HIP;
    }
    *out = g;
    return LR_OK;
}

lr_status lr_batch_graph_launch(lr_batch_graph* g, const lr_request* reqs, uint32_t count, void* stream) {
    if (!g || (count && !reqs)) return LR_ERR_INVALID_ARG;
    if (count == 0) return LR_OK;
    if (count > g->max_requests) return LR_ERR_WORKSPACE;
    uint64_t N = 0;
    for (uint32_t i = 0; i < count; ++i) {
        if (reqs[i].n && (!reqs[i].succ || !reqs[i].rank)) return LR_ERR_INVALID_ARG;
        if (reqs[i].root && !g->want_root) return LR_ERR_INVALID_ARG;
        N += reqs[i].n;
    }
    if (N > g->max_elements) return LR_ERR_WORKSPACE;
    if (N == 0) return LR_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (run_batch_table(reqs, count, g->plan, g->ws, true, g->max_chunks, st) != hipSuccess) return LR_ERR_HIP;
    return hipGraphLaunch(g->exec, st) == hipSuccess ? LR_OK : LR_ERR_HIP;
}

void lr_batch_graph_destroy(lr_batch_graph* g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

}  // extern "C"

extern "C" int lr_profile_last(double* ms, int cap) {
    if (!ms || cap <= 0 || !g_prof.valid) return 0;
    for (auto& e : g_prof.ev)
        if (hipEventSynchronize(e) != hipSuccess) return 0;
    float v[EV_COUNT] = {};
    for (int i = 1; i < EV_COUNT; ++i) (void)hipEventElapsedTime(&v[i], g_prof.ev[i - 1], g_prof.ev[i]);
    float total = 0;
    (void)hipEventElapsedTime(&total, g_prof.ev[0], g_prof.ev[EV_COUNT - 1]);
    uint32_t mode = MODE_PLAIN;
    if (cap > 7 && g_prof.mode && hipMemcpy(&mode, g_prof.mode, 4, hipMemcpyDeviceToHost) != hipSuccess) return 0;
    double out[8] = {v[EV_DETECT], v[EV_HEADS], v[EV_CHASE0], v[EV_UPPER], v[EV_PART], v[EV_EXPAND], total,
                     mode == MODE_FALLBACK ? 1.0 : 0.0};
    int k = std::min(cap, 8);
    for (int i = 0; i < k; ++i) ms[i] = out[i];
    return k;
}

extern "C" lr_status lr_verify(const uint32_t* succ, const void* weight, lr_wtype w, const uint32_t* rank,
                               const uint32_t* root, const int64_t* sum, uint64_t n, void* ws, size_t ws_bytes,
                               void* stream) {
    if (w != LR_W_NONE && w != LR_W_I32 && w != LR_W_I64) return LR_ERR_INVALID_ARG;
    if (n == 0) return LR_OK;
    if (!succ || (!rank && !root && !sum)) return LR_ERR_INVALID_ARG;
    if ((w != LR_W_NONE) && (!weight || !sum)) return LR_ERR_INVALID_ARG;
    if (n >= (1ull << 31)) return LR_ERR_UNSUPPORTED;
    if (!ws || ws_bytes < 2 * ALIGN) return LR_ERR_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint32_t* err = reinterpret_cast<uint32_t*>(carve(ws));
    if (run_verify(succ, weight, (int)w, rank, root, sum, (uint32_t)n, err, st) != hipSuccess) return LR_ERR_HIP;
    uint32_t e = 0;
    if (hipMemcpyAsync(&e, err, 4, hipMemcpyDeviceToHost, st) != hipSuccess) return LR_ERR_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return LR_ERR_HIP;
    return e ? LR_ERR_BAD_LIST : LR_OK;
}
