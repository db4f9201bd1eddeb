// Plan autotuner and its cache. The paper fixes its ruler-count constants
// by a parameter study on its machine (Section 3, "Methodology"); here
// lr_autotune times candidate plans on the caller's input and keeps the
// fastest per (device, input size bucket, weighted or not), and the planner
// takes a cached entry for every later call of that bucket that leaves the
// plan options at their defaults. Results never depend on the plan.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "lr.h"
#include "plan.hpp"

namespace lr {

namespace {

struct TuneKey {
    std::string arch;  // device name and compute units, e.g. "gfx950:256"
    uint32_t log2n;    // floor(log2(n))
    uint32_t weighted;
    bool operator<(const TuneKey& o) const {
        return std::tie(arch, log2n, weighted) < std::tie(o.arch, o.log2n, o.weighted);
    }
};
struct TuneVal {
    uint32_t k0, k1, base_max, lane_walks, refill;
    double ms;
};

std::mutex g_mu;
std::map<TuneKey, TuneVal> g_cache;
std::string g_arch;  // the current device's key, found on first use

// The current device's arch key, or "none" without a device.
const std::string& arch_key() {
    if (g_arch.empty()) {
        int dev = 0;
        hipDeviceProp_t prop{};
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
            char buf[128];
            const char* colon = strchr(prop.gcnArchName, ':');  // drop feature suffixes (":sramecc+:xnack-")
            const int len = colon ? (int)(colon - prop.gcnArchName) : (int)strlen(prop.gcnArchName);
            snprintf(buf, sizeof buf, "%.*s:%d", len, prop.gcnArchName, prop.multiProcessorCount);
            g_arch = buf;
        } else {
            (void)hipGetLastError();
            g_arch = "none";
        }
    }
    return g_arch;
}

uint32_t floor_log2(uint64_t n) {
    uint32_t r = 0;
    while (n >> (r + 1)) ++r;
    return r;
}

}  // namespace

// Fill o's plan options from the cache entry of (device, n, weighted), if
// any. Returns whether an entry applied.
bool tune_lookup(uint64_t n, bool weighted, lr_opts* o) {
    if (n == 0) return false;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_cache.empty()) return false;
    const auto it = g_cache.find(TuneKey{arch_key(), floor_log2(n), weighted ? 1u : 0u});
    if (it == g_cache.end()) return false;
    const TuneVal& v = it->second;
    for (int l = 0; l < LR_MAX_LEVELS; ++l) o->spacing[l] = 0;
    o->spacing[0] = v.k0;
    o->spacing[1] = v.k1;
    o->base_max = v.base_max;
    o->lane_walks = v.lane_walks;
    o->refill = v.refill;
    return true;
}

static void tune_store(uint64_t n, bool weighted, const lr_opts& best, double ms) {
    std::lock_guard<std::mutex> lock(g_mu);
    g_cache[TuneKey{arch_key(), floor_log2(n), weighted ? 1u : 0u}] =
        TuneVal{best.spacing[0], best.spacing[1], best.base_max, best.lane_walks, best.refill, ms};
}

}  // namespace lr

using namespace lr;

extern "C" {

const char* lr_autotune_arch(void) {
    std::lock_guard<std::mutex> lock(g_mu);
    return arch_key().c_str();
}

int lr_autotune_cache_entries(void) {
    std::lock_guard<std::mutex> lock(g_mu);
    return (int)g_cache.size();
}

void lr_autotune_cache_clear(void) {
    std::lock_guard<std::mutex> lock(g_mu);
    g_cache.clear();
}

lr_status lr_autotune_cache_save(const char* path) {
    if (!path) return LR_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_mu);
    FILE* f = fopen(path, "w");
    if (!f) return LR_ERR_INVALID_ARG;
    fprintf(f, "# lr autotune cache v1: arch log2n weighted k0 k1 base_max lane_walks refill ms\n");
    for (const auto& kv : g_cache)
        fprintf(f, "%s %u %u %u %u %u %u %u %.4f\n", kv.first.arch.c_str(), kv.first.log2n, kv.first.weighted,
                kv.second.k0, kv.second.k1, kv.second.base_max, kv.second.lane_walks, kv.second.refill, kv.second.ms);
    return fclose(f) == 0 ? LR_OK : LR_ERR_INVALID_ARG;
}

lr_status lr_autotune_cache_load(const char* path) {
    if (!path) return LR_ERR_INVALID_ARG;
    FILE* f = fopen(path, "r");
    if (!f) return LR_ERR_INVALID_ARG;
    std::vector<std::pair<TuneKey, TuneVal>> rows;
    char line[512];
    bool ok = true;
    while (fgets(line, sizeof line, f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        char arch[128];
        TuneKey k;
        TuneVal v;
        if (sscanf(line, "%127s %u %u %u %u %u %u %u %lf", arch, &k.log2n, &k.weighted, &v.k0, &v.k1, &v.base_max,
                   &v.lane_walks, &v.refill, &v.ms) != 9) {
            ok = false;
            break;
        }
        k.arch = arch;
        // the same checks the planner makes on user options
        auto pow2 = [](uint32_t x, uint32_t lo, uint32_t hi) { return x >= lo && x <= hi && !(x & (x - 1)); };
        if (!pow2(v.k0, 2, 4096) || (v.k1 && !pow2(v.k1, 2, 4096)) || v.base_max > BASE_MAX_LIMIT ||
            v.lane_walks > 2 || v.refill > 64 * (v.lane_walks ? v.lane_walks : 1) || k.weighted > 1 || k.log2n > 31) {
            ok = false;
            break;
        }
        rows.emplace_back(k, v);
    }
    fclose(f);
    if (!ok) return LR_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_mu);
    for (const auto& r : rows) g_cache[r.first] = r.second;
    return LR_OK;
}

lr_status lr_autotune(const uint32_t* succ, const void* weight, lr_wtype w, uint64_t n, void* ws, size_t ws_bytes,
                      const lr_opts* base, lr_opts* best, double* ms, int cap, int* tried, void* stream) {
    if (!succ || !best || (w != LR_W_NONE && w != LR_W_I32 && w != LR_W_I64)) return LR_ERR_INVALID_ARG;
    if (n == 0 || n >= (1ull << 31)) return LR_ERR_UNSUPPORTED;
    if ((w == LR_W_NONE) != (weight == nullptr)) return LR_ERR_INVALID_ARG;
    const bool weighted = w != LR_W_NONE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    lr_opts b{};
    if (base) b = *base;
    b.flags &= ~(uint32_t)(LR_VALIDATE | LR_PROFILE);
    // trial outputs go to the tail of the caller's workspace; the rest is the
    // trial calls' workspace
    const size_t out_bytes = (size_t)n * (weighted ? 8 : 4);
    if (ws_bytes <= out_bytes + ALIGN) return LR_ERR_WORKSPACE;
    char* wsb = static_cast<char*>(ws);
    const size_t trial_ws = (ws_bytes - out_bytes - ALIGN) / ALIGN * ALIGN;
    void* out = wsb + trial_ws + ALIGN;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return LR_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return LR_ERR_HIP;
    }
    float best_ms = 1e30f;
    bool found = false;
    int count = 0;
    lr_status result = LR_OK;
    // time one candidate (1 warm-up, 3 timed calls); false: skipped (does not fit)
    auto trial = [&](const lr_opts& o, float* t) -> bool {
        Plan p;
        if (make_plan(n, weighted, &o, 0, &p) != LR_OK || p.total > trial_ws) return false;
        auto run = [&]() -> lr_status {
            return weighted ? lr_prefix_sum(succ, weight, w, static_cast<int64_t*>(out), nullptr, nullptr, n, ws,
                                            trial_ws, &o, stream)
                            : lr_rank(succ, static_cast<uint32_t*>(out), nullptr, n, ws, trial_ws, &o, stream);
        };
        lr_status s = run();
        if (s != LR_OK) { result = s; return false; }
        if (hipEventRecord(e0, st) != hipSuccess) { result = LR_ERR_HIP; return false; }
        const int reps = 3;
        for (int r = 0; r < reps && s == LR_OK; ++r) s = run();
        if (s != LR_OK) { result = s; return false; }
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(t, e0, e1) != hipSuccess) {
            result = LR_ERR_HIP;
            return false;
        }
        *t /= reps;
        if (ms && count < cap) ms[count] = *t;
        ++count;
        if (*t < best_ms) {
            best_ms = *t;
            *best = o;
            found = true;
        }
        return true;
    };
    // stage 1: spacing of the first two levels; stage 2: the base case size;
    // stage 3: walks per lane and refill threshold (each stage keeps the best
    // so far and varies one group)
    const uint32_t k0s[] = {16, 32, 64, 128};
    const uint32_t k1s[] = {8, 16, 32};
    for (uint32_t k0 : k0s) {
        for (uint32_t k1 : k1s) {
            lr_opts o = b;
            for (int l = 0; l < LR_MAX_LEVELS; ++l) o.spacing[l] = 0;
            o.spacing[0] = k0;
            o.spacing[1] = k1;
            Plan p;
            if (make_plan(n, weighted, &o, 0, &p) != LR_OK) continue;
            if (p.levels < 2 && k1 != k1s[0]) continue;  // second spacing unused: try it once
            float t;
            (void)trial(o, &t);
            if (result != LR_OK) break;
        }
        if (result != LR_OK) break;
    }
    if (found && result == LR_OK) {
        const lr_opts s1 = *best;
        const uint32_t bases[] = {weighted ? 2048u : 4096u, weighted ? 4096u : 8192u, weighted ? 8192u : 16384u};
        for (uint32_t bm : bases) {
            lr_opts o = s1;
            o.base_max = bm;
            float t;
            (void)trial(o, &t);
            if (result != LR_OK) break;
        }
    }
    if (found && result == LR_OK) {
        const lr_opts s2 = *best;
        const uint32_t lw_rf[][2] = {{2, 1}, {1, 8}, {1, 32}};
        for (const auto& c : lw_rf) {
            lr_opts o = s2;
            o.lane_walks = c[0];
            o.refill = c[1];
            float t;
            (void)trial(o, &t);
            if (result != LR_OK) break;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (tried) *tried = count;
    if (result != LR_OK) return result;
    if (!found) return LR_ERR_WORKSPACE;
    // the full spacing list the winning plan uses, and the cache entry
    Plan p;
    if (make_plan(n, weighted, best, 0, &p) == LR_OK)
        for (uint32_t l = 0; l < p.levels; ++l) best->spacing[l] = 1u << p.log2k[l];
    if (!best->base_max) best->base_max = p.base_max;
    if (!best->lane_walks) best->lane_walks = 1;
    if (!best->refill) best->refill = 1;
    tune_store(n, weighted, *best, best_ms);
    if (base) best->flags = base->flags;
    return LR_OK;
}

}  // extern "C"
