// Serving layer: the HIP executor behind the continuous-batching scheduler,
// and the C ABI of lr_server_*.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <chrono>
#include <memory>
#include <thread>
#include <vector>

#include "device.hpp"
#include "lr.h"
#include "plan.hpp"
#include "sched.hpp"

namespace lr {

lr_status batch_enqueue(const lr_request* reqs, uint32_t count, void* ws, size_t ws_bytes, const lr_opts* opts,
                        hipStream_t st, void* host_stage, size_t host_cap, hipEvent_t* copy_done);

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
        const uint32_t mb = cfg_.max_batch ? cfg_.max_batch : 1;
        stage_cap_ = (size_t)mb * sizeof(BatchDesc) + batch_table_bytes(mb);
        slots_.resize(cfg_.max_inflight);
        for (uint32_t i = 0; i < cfg_.max_inflight; ++i) {
            Slot& s = slots_[i];
            if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess) return LR_ERR_HIP;
            if (hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) return LR_ERR_HIP;
            if (hipHostMalloc(&s.stage, stage_cap_, hipHostMallocDefault) != hipSuccess) return LR_ERR_HIP;
            s.ws = static_cast<char*>(pool_) + (size_t)i * bytes_;
        }
        return LR_OK;
    }

    ~HipExecutor() override {
        for (Slot& s : slots_) {
            if (s.stream) (void)hipStreamSynchronize(s.stream);
            if (s.done) (void)hipEventDestroy(s.done);
            if (s.stream) (void)hipStreamDestroy(s.stream);
            if (s.stage) (void)hipHostFree(s.stage);
        }
        if (pool_) (void)hipFree(pool_);
    }

    uint32_t slots() const override { return (uint32_t)slots_.size(); }
    size_t slot_bytes() const override { return bytes_; }

    size_t workspace(const lr_request* reqs, uint32_t count) const override {
        return lr_batch_workspace_bytes(reqs, count, &cfg_.opts);
    }

    lr_status launch(uint32_t i, const lr_request* reqs, uint32_t count) override {
        Slot& s = slots_[i];
        (void)hipSetDevice(dev_);
        if (s.failed) {  // a failed launch may have left copies from the staging buffer in flight
            if (hipEventSynchronize(s.done) != hipSuccess) return LR_ERR_HIP;
            s.failed = false;
        }
        lr_status st = batch_enqueue(reqs, count, s.ws, bytes_, &cfg_.opts, s.stream, s.stage, stage_cap_, nullptr);
        const bool recorded = hipEventRecord(s.done, s.stream) == hipSuccess;
        if (st == LR_OK && !recorded) st = LR_ERR_HIP;
        if (st != LR_OK) s.failed = true;  // the scheduler frees the slot at once
        return st;
    }

    int poll(uint32_t i) override {
        const hipError_t e = hipEventQuery(slots_[i].done);
        if (e == hipSuccess) return 1;
        if (e == hipErrorNotReady) return 0;
        return -1;
    }

private:
    struct Slot {
        hipStream_t stream = nullptr;
        hipEvent_t done = nullptr;
        void* stage = nullptr;
        char* ws = nullptr;
        bool failed = false;  // the last launch failed: wait for s.done before reusing the staging
    };
    lr_server_config cfg_{};
    int dev_ = 0;
    void* pool_ = nullptr;
    size_t bytes_ = 0, stage_cap_ = 0;
    std::vector<Slot> slots_;
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
