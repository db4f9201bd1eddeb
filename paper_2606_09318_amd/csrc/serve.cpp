// Serving layer: the HIP executor behind the continuous-batching scheduler,
// and the C ABI of lr_server_*.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <chrono>
#include <map>
#include <memory>
#include <thread>
#include <vector>

#include "device.hpp"
#include "lr.h"
#include "plan.hpp"
#include "sched.hpp"

namespace lr {

lr_status batch_enqueue(const lr_request* reqs, uint32_t count, void* ws, size_t ws_bytes, const lr_opts* opts,
                        hipStream_t st);

// Graph buckets: a batch of N elements replays the graph planned for the
// smallest capacity 2^(j/2) >= N (j >= 2 * GRAPH_MIN_LOG2), captured on first
// use per slot; all graphs of a slot share its workspace (its batches run one
// after another on its stream).
constexpr uint32_t GRAPH_MIN_LOG2 = 16;

class HipExecutor : public Executor {
public:
    lr_status init(const lr_server_config& c) {
        cfg_ = c;
        if (cfg_.max_inflight == 0 || cfg_.hbm_budget == 0) return LR_ERR_INVALID_ARG;
        if (hipGetDevice(&dev_) != hipSuccess) return LR_ERR_HIP;
        if (hipMalloc(&pool_, cfg_.hbm_budget) != hipSuccess) {
            pool_ = nullptr;
            return LR_ERR_OUT_OF_MEMORY;
        }
        bytes_ = (cfg_.hbm_budget / cfg_.max_inflight) / 256 * 256;
        slots_.resize(cfg_.max_inflight);
        for (uint32_t i = 0; i < cfg_.max_inflight; ++i) {
            Slot& s = slots_[i];
            if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess) return LR_ERR_HIP;
            if (hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) return LR_ERR_HIP;
            s.ws = static_cast<char*>(pool_) + (size_t)i * bytes_;
        }
        // capture every bucket that fits a slot now (rank-only graphs), so no
        // capture runs while requests wait; graphs with roots are captured on
        // first use
        if (cfg_.graphs) {
            for (Slot& s : slots_) {
                for (uint32_t j = 2 * GRAPH_MIN_LOG2; bucket_cap(j) < (1ull << 31); ++j) {
                    const lr_batch_graph_config gc = graph_config(j, false);
                    const size_t need = lr_batch_graph_workspace_bytes(&gc);
                    if (need == 0 || need > bytes_) break;
                    lr_batch_graph* g = nullptr;
                    if (lr_batch_graph_create(&gc, s.ws, bytes_, &g) != LR_OK) break;
                    s.graphs.emplace(2 * j, g);
                }
            }
        }
        return LR_OK;
    }

    ~HipExecutor() override {
        for (Slot& s : slots_) {
            if (s.stream) (void)hipStreamSynchronize(s.stream);
            for (auto& kv : s.graphs) lr_batch_graph_destroy(kv.second);
            if (s.done) (void)hipEventDestroy(s.done);
            if (s.stream) (void)hipStreamDestroy(s.stream);
        }
        if (pool_) (void)hipFree(pool_);
    }

    uint32_t slots() const override { return (uint32_t)slots_.size(); }
    size_t slot_bytes() const override { return bytes_; }

    size_t workspace(const lr_request* reqs, uint32_t count) const override {
        return lr_batch_workspace_bytes(reqs, count, &cfg_.opts);
    }

    // A batch after a failed launch needs no wait: every launch of a slot is
    // ordered on the slot's stream, and no host buffer outlives a call.
    lr_status launch(uint32_t i, const lr_request* reqs, uint32_t count) override {
        Slot& s = slots_[i];
        (void)hipSetDevice(dev_);
        lr_status st = LR_ERR_UNSUPPORTED;
        if (cfg_.graphs) st = launch_graph(s, reqs, count);
        if (st == LR_ERR_UNSUPPORTED) st = batch_enqueue(reqs, count, s.ws, bytes_, &cfg_.opts, s.stream);
        if (hipEventRecord(s.done, s.stream) != hipSuccess && st == LR_OK) st = LR_ERR_HIP;
        return st;
    }

    int poll(uint32_t i) override {
        const hipError_t e = hipEventQuery(slots_[i].done);
        if (e == hipSuccess) return 1;
        if (e == hipErrorNotReady) return 0;
        return -1;
    }

    uint64_t graph_launches() const { return graph_launches_.load(); }

private:
    struct Slot {
        hipStream_t stream = nullptr;
        hipEvent_t done = nullptr;
        char* ws = nullptr;
        std::map<uint32_t, lr_batch_graph*> graphs;  // by 2 j + roots (capacity 2^(j/2) elements)
    };

    // Replays the bucket's graph; LR_ERR_UNSUPPORTED when the batch should take
    // the plain enqueue instead (its bucket's workspace does not fit the slot,
    // or options a graph cannot take).
    lr_status launch_graph(Slot& s, const lr_request* reqs, uint32_t count) {
        uint64_t N = 0;
        bool root = false;
        for (uint32_t q = 0; q < count; ++q) {
            N += reqs[q].n;
            root |= reqs[q].root != nullptr;
        }
        uint32_t j = 2 * GRAPH_MIN_LOG2;
        while (j < 62 && bucket_cap(j) < N) ++j;
        if (bucket_cap(j) >= (1ull << 31)) return LR_ERR_UNSUPPORTED;
        const lr_batch_graph_config gc = graph_config(j, root);
        const uint32_t key = 2 * j + (root ? 1u : 0u);  // the root column costs placement bandwidth
        auto it = s.graphs.find(key);
        if (it == s.graphs.end()) {
            const size_t need = lr_batch_graph_workspace_bytes(&gc);
            if (need == 0 || need > bytes_) return LR_ERR_UNSUPPORTED;
            lr_batch_graph* g = nullptr;
            const lr_status st = lr_batch_graph_create(&gc, s.ws, bytes_, &g);
            if (st != LR_OK) return st == LR_ERR_INVALID_ARG ? LR_ERR_UNSUPPORTED : st;
            it = s.graphs.emplace(key, g).first;
        }
        const lr_status st = lr_batch_graph_launch(it->second, reqs, count, s.stream);
        if (st == LR_OK) graph_launches_++;
        return st;
    }

    lr_batch_graph_config graph_config(uint32_t j, bool root) const {
        lr_batch_graph_config gc{};
        gc.max_elements = bucket_cap(j);
        gc.max_requests = cfg_.max_batch ? cfg_.max_batch : 1;
        gc.want_root = root ? 1u : 0u;
        gc.opts = cfg_.opts;
        return gc;
    }

    static uint64_t bucket_cap(uint32_t j) {  // 2^(j/2), rounded up
        const uint64_t b = 1ull << (j / 2);
        return (j & 1) ? (uint64_t)((double)b * 1.4142135623730951) + 1 : b;
    }

    lr_server_config cfg_{};
    int dev_ = 0;
    void* pool_ = nullptr;
    size_t bytes_ = 0;
    std::vector<Slot> slots_;
    std::atomic<uint64_t> graph_launches_{0};
};

}  // namespace lr

struct lr_server {
    std::unique_ptr<lr::HipExecutor> ex;
    std::unique_ptr<lr::Scheduler> sched;
};

extern "C" {

lr_status lr_server_create(const lr_server_config* cfg, lr_server** out) {
    if (!cfg || !out) return LR_ERR_INVALID_ARG;
    if (cfg->max_inflight == 0 || cfg->hbm_budget == 0) return LR_ERR_INVALID_ARG;
    *out = nullptr;
    auto s = std::make_unique<lr_server>();
    s->ex = std::make_unique<lr::HipExecutor>();
    lr_status st = s->ex->init(*cfg);
    if (st != LR_OK) return st;
    s->sched = std::make_unique<lr::Scheduler>(s->ex.get(), cfg->max_batch);
    *out = s.release();
    return LR_OK;
}

lr_status lr_server_submit(lr_server* s, const lr_request* req, uint64_t* ticket) {
    if (!s || !req || !ticket) return LR_ERR_INVALID_ARG;
    if (req->n && (!req->succ || !req->rank)) return LR_ERR_INVALID_ARG;
    *ticket = s->sched->submit(*req);
    return LR_OK;
}

int lr_server_poll(lr_server* s, uint64_t ticket, lr_status* status, double* latency_s) {
    if (!s) return -1;
    return s->sched->poll(ticket, status, latency_s);
}

lr_status lr_server_drain(lr_server* s) {
    if (!s) return LR_ERR_INVALID_ARG;
    s->sched->drain();
    return LR_OK;
}

void lr_server_destroy(lr_server* s) {
    if (!s) return;
    s->sched.reset();  // joins the worker after the queue drains
    s->ex.reset();
    delete s;
}

lr_status lr_server_replay(const lr_server_config* cfg, const lr_request* reqs, const double* arrival_s,
                           uint32_t count, double* latency_s, lr_status* status, double* makespan_s) {
    if (!cfg || (count && (!reqs || !arrival_s || !latency_s))) return LR_ERR_INVALID_ARG;
    lr_server* s = nullptr;
    lr_status st = lr_server_create(cfg, &s);
    if (st != LR_OK) return st;
    using clock = std::chrono::steady_clock;
    std::vector<uint64_t> tickets(count);
    const auto t0 = clock::now();
    for (uint32_t i = 0; i < count; ++i) {
        const auto due = t0 + std::chrono::duration_cast<clock::duration>(std::chrono::duration<double>(arrival_s[i]));
        for (;;) {
            const auto now = clock::now();
            if (now >= due) break;
            if (due - now > std::chrono::microseconds(300)) std::this_thread::sleep_for(std::chrono::microseconds(100));
            else std::this_thread::yield();
        }
        if (reqs[i].n && (!reqs[i].succ || !reqs[i].rank)) {
            lr_server_destroy(s);
            return LR_ERR_INVALID_ARG;
        }
        // latency counts from the scheduled arrival, so a late submission
        // (the replay loop itself delayed) is not hidden
        tickets[i] = s->sched->submit(reqs[i], due);
    }
    s->sched->drain();
    auto last = t0;
    for (uint32_t i = 0; i < count; ++i) {
        lr_status r = LR_OK;
        double lat = 0;
        s->sched->poll(tickets[i], &r, &lat);
        latency_s[i] = lat;
        if (status) status[i] = r;
        const auto d = s->sched->done_time(tickets[i]);
        if (d > last) last = d;
    }
    if (makespan_s) *makespan_s = std::chrono::duration<double>(last - t0).count();
    lr_server_destroy(s);
    return LR_OK;
}

}  // extern "C"
