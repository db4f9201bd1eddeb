// Continuous-batching scheduler for ranking requests, independent of the
// device: an Executor runs batches on a fixed number of slots, the scheduler
// admits waiting requests (FIFO) into whichever slot is free, as many as fit
// the slot's workspace, and records each request's completion time.
// Host-only C++ (no HIP), so it can be tested with a fake executor.
//
// Latency is measured from a request's arrival: the time the caller passes
// to submit (a trace replay passes the scheduled arrival), else the time
// submit was entered, taken before any lock, so time spent waiting for the
// scheduler's lock counts. Launches run outside the lock, so submissions and
// polls never wait for a batch being enqueued.
#pragma once
#include <stdint.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "lr.h"

namespace lr {

class Executor {
public:
    virtual ~Executor() = default;
    virtual uint32_t slots() const = 0;
    virtual size_t slot_bytes() const = 0;
    // Workspace a batch of these requests needs (0 = cannot be served).
    virtual size_t workspace(const lr_request* reqs, uint32_t count) const = 0;
    // Start a batch on a free slot; returns LR_OK once it is enqueued. Called
    // from the scheduler's worker thread only, never under its lock.
    virtual lr_status launch(uint32_t slot, const lr_request* reqs, uint32_t count) = 0;
    // 1 = the slot's batch has finished, 0 = still running, -1 = it failed.
    virtual int poll(uint32_t slot) = 0;
};

class Scheduler {
public:
    using clock = std::chrono::steady_clock;

    Scheduler(Executor* ex, uint32_t max_batch) : ex_(ex), max_batch_(max_batch ? max_batch : 1) {
        busy_.assign(ex_->slots(), {});
        worker_ = std::thread([this] { loop(); });
    }

    ~Scheduler() {
        {
            std::lock_guard<std::mutex> g(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        worker_.join();
    }

    // Enqueue a request that arrived at `arrival`.
    uint64_t submit(const lr_request& r, clock::time_point arrival) {
        std::lock_guard<std::mutex> g(mu_);
        const uint64_t id = tickets_.size();
        tickets_.push_back(Ticket{r, arrival, {}, LR_OK, 0});
        queue_.push_back(id);
        cv_.notify_all();
        return id;
    }
    uint64_t submit(const lr_request& r) { return submit(r, clock::now()); }

    int poll(uint64_t id, lr_status* st, double* lat) {
        std::lock_guard<std::mutex> g(mu_);
        if (id >= tickets_.size()) return -1;
        const Ticket& t = tickets_[id];
        if (t.state != 2) return 0;
        if (st) *st = t.status;
        if (lat) *lat = std::chrono::duration<double>(t.t_done - t.t_submit).count();
        return 1;
    }

    void drain() {
        std::unique_lock<std::mutex> g(mu_);
        done_cv_.wait(g, [this] { return queue_.empty() && running_ == 0; });
    }

    // Completion time of a ticket (valid once poll returned 1).
    clock::time_point done_time(uint64_t id) {
        std::lock_guard<std::mutex> g(mu_);
        return tickets_[id].t_done;
    }

    uint64_t batches() const { return batches_.load(); }

private:
    struct Ticket {
        lr_request req;
        clock::time_point t_submit, t_done;
        lr_status status;
        int state;  // 0 waiting, 1 running, 2 done
    };
    struct Busy {
        bool on = false;
        std::vector<uint64_t> ids;
    };

    void finish(uint64_t id, lr_status s, clock::time_point now) {
        Ticket& t = tickets_[id];
        t.status = s;
        t.state = 2;
        t.t_done = now;
    }

    // Retire finished slots. Caller holds mu_.
    bool retire() {
        bool progress = false;
        for (uint32_t s = 0; s < busy_.size(); ++s) {
            if (!busy_[s].on) continue;
            const int r = ex_->poll(s);
            if (r == 0) continue;
            const auto now = clock::now();
            for (uint64_t id : busy_[s].ids) finish(id, r > 0 ? LR_OK : LR_ERR_HIP, now);
            running_ -= (uint32_t)busy_[s].ids.size();
            busy_[s].on = false;
            busy_[s].ids.clear();
            progress = true;
        }
        return progress;
    }

    // Take the next batch for a free slot off the queue (FIFO, as many as fit
    // the slot); requests that can never fit are rejected alone. Caller holds
    // mu_. Returns false when no slot is free or nothing is waiting.
    bool admit(uint32_t* slot, std::vector<lr_request>* reqs, std::vector<uint64_t>* ids, bool* progress) {
        for (uint32_t s = 0; s < busy_.size() && !queue_.empty(); ++s) {
            if (busy_[s].on) continue;
            reqs->clear();
            ids->clear();
            uint64_t total = 0;
            while (!queue_.empty() && reqs->size() < max_batch_) {
                const uint64_t id = queue_.front();
                const lr_request& r = tickets_[id].req;
                reqs->push_back(r);
                const size_t need = ex_->workspace(reqs->data(), (uint32_t)reqs->size());
                if (need == 0 || need > ex_->slot_bytes() || total + r.n >= (1ull << 31)) {
                    reqs->pop_back();
                    if (reqs->empty()) {  // can never be served: reject alone
                        queue_.pop_front();
                        finish(id, LR_ERR_WORKSPACE, clock::now());
                        *progress = true;
                        continue;
                    }
                    break;
                }
                total += r.n;
                ids->push_back(id);
                queue_.pop_front();
            }
            if (reqs->empty()) continue;
            // the slot and its requests are taken before the lock is released
            for (uint64_t id : *ids) tickets_[id].state = 1;
            busy_[s].on = true;
            busy_[s].ids = *ids;
            running_ += (uint32_t)ids->size();
            *slot = s;
            return true;
        }
        return false;
    }

    void loop() {
        std::unique_lock<std::mutex> g(mu_);
        std::vector<lr_request> reqs;
        std::vector<uint64_t> ids;
        for (;;) {
            bool progress = retire();
            uint32_t slot = 0;
            while (admit(&slot, &reqs, &ids, &progress)) {
                g.unlock();
                const lr_status st = ex_->launch(slot, reqs.data(), (uint32_t)reqs.size());
                g.lock();
                if (st != LR_OK) {  // the batch fails alone; its slot is free again
                    const auto now = clock::now();
                    for (uint64_t id : ids) finish(id, st, now);
                    running_ -= (uint32_t)ids.size();
                    busy_[slot].on = false;
                    busy_[slot].ids.clear();
                } else {
                    batches_++;
                }
                progress = true;
            }
            if (queue_.empty() && running_ == 0) done_cv_.notify_all();
            if (stop_ && queue_.empty() && running_ == 0) break;
            if (!progress) {
                if (running_ == 0) {
                    // a timed wait on the system clock (pthread_cond_timedwait,
                    // which thread sanitizers model); 5 ms either way
                    cv_.wait_until(g, std::chrono::system_clock::now() + std::chrono::milliseconds(5));
                } else {  // batches in flight: poll their completion closely
                    g.unlock();
                    std::this_thread::yield();
                    g.lock();
                }
            }
        }
    }

    Executor* ex_;
    uint32_t max_batch_;
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    std::deque<uint64_t> queue_;
    std::vector<Ticket> tickets_;
    std::vector<Busy> busy_;
    uint32_t running_ = 0;
    std::atomic<uint64_t> batches_{0};
    bool stop_ = false;
    std::thread worker_;
};

}  // namespace lr
