// CPU tests of the continuous-batching scheduler (csrc/sched.hpp) with a fake
// executor: no device, no HIP. Built and run by tests/test_sched_cpu.py; each
// case prints "ok <name>" and any failure exits non-zero with a message.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <chrono>
#include <future>
#include <mutex>
#include <thread>
#include <vector>

#include "sched.hpp"

using clk = std::chrono::steady_clock;
using namespace std::chrono_literals;

#define CHECK(c)                                                               \
    do {                                                                       \
        if (!(c)) {                                                            \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            exit(1);                                                           \
        }                                                                      \
    } while (0)

// Requests are tagged through their succ pointer (an integer, never read).
static lr_request req(uint64_t tag, uint64_t n) {
    lr_request r{};
    r.succ = reinterpret_cast<const uint32_t*>(tag + 1);
    r.rank = reinterpret_cast<uint32_t*>(tag + 1);
    r.n = n;
    return r;
}
static uint64_t tag_of(const lr_request& r) { return reinterpret_cast<uint64_t>(r.succ) - 1; }

// A fake executor: a batch "runs" for run_time after launch; launch or
// completion fails for batches holding a chosen tag. Workspace of a batch:
// 64 B per request + 1 B per element.
class Mock : public lr::Executor {
public:
    struct Launch {
        uint32_t slot;
        std::vector<uint64_t> tags;
        bool launch_failed;
    };
    Mock(uint32_t nslots, size_t bytes) : nslots_(nslots), bytes_(bytes), ready_(nslots), result_(nslots, 0) {}

    uint32_t slots() const override { return nslots_; }
    size_t slot_bytes() const override { return bytes_; }
    size_t workspace(const lr_request* r, uint32_t count) const override {
        size_t b = 0;
        for (uint32_t i = 0; i < count; ++i) b += 64 + r[i].n;
        return b;
    }
    lr_status launch(uint32_t slot, const lr_request* r, uint32_t count) override {
        CHECK(slot < nslots_);
        std::vector<uint64_t> tags;
        for (uint32_t i = 0; i < count; ++i) tags.push_back(tag_of(r[i]));
        CHECK(workspace(r, count) <= bytes_);
        if (launch_delay.count()) std::this_thread::sleep_for(launch_delay);
        const bool fail = std::find(tags.begin(), tags.end(), fail_launch_tag) != tags.end();
        {
            std::lock_guard<std::mutex> g(mu_);
            CHECK(result_[slot] == 0);  // never launched on a busy slot
            log.push_back({slot, tags, fail});
            if (fail) return LR_ERR_HIP;
            ready_[slot] = clk::now() + run_time;
            result_[slot] = std::find(tags.begin(), tags.end(), fail_poll_tag) != tags.end() ? -1 : 1;
        }
        return LR_OK;
    }
    int poll(uint32_t slot) override {
        std::lock_guard<std::mutex> g(mu_);
        CHECK(result_[slot] != 0);  // only busy slots are polled
        if (clk::now() < ready_[slot]) return 0;
        const int r = result_[slot];
        result_[slot] = 0;
        return r;
    }

    std::vector<Launch> log;
    std::chrono::microseconds run_time{200};
    std::chrono::microseconds launch_delay{0};
    uint64_t fail_launch_tag = ~0ull, fail_poll_tag = ~0ull;

private:
    uint32_t nslots_;
    size_t bytes_;
    std::mutex mu_;
    std::vector<clk::time_point> ready_;
    std::vector<int> result_;
};

// drain() must return within a few seconds: a stuck queue is a failure.
static void drain_or_fail(lr::Scheduler& s) {
    auto f = std::async(std::launch::async, [&] { s.drain(); });
    CHECK(f.wait_for(10s) == std::future_status::ready);
}

static lr_status status_of(lr::Scheduler& s, uint64_t id, double* lat = nullptr) {
    lr_status st = LR_OK;
    CHECK(s.poll(id, &st, lat) == 1);
    return st;
}

// Requests are admitted in submission order: one slot, one request per batch.
static void fifo() {
    Mock ex(1, 1 << 20);
    std::vector<uint64_t> ids;
    {
        lr::Scheduler s(&ex, 1);
        for (uint64_t i = 0; i < 64; ++i) ids.push_back(s.submit(req(i, 100 + i)));
        drain_or_fail(s);
        for (uint64_t id : ids) CHECK(status_of(s, id) == LR_OK);
    }
    CHECK(ex.log.size() == 64);
    for (uint64_t i = 0; i < 64; ++i) CHECK(ex.log[i].tags.size() == 1 && ex.log[i].tags[0] == i);
    puts("ok fifo");
}

// A budget that holds only a few requests per batch: everything still
// completes (no deadlock), every batch fits its slot, and the batches taken
// in launch order list the requests in submission order.
static void tiny_budget() {
    Mock ex(2, 3 * 64 + 3 * 100);  // at most three 100-element requests per slot
    std::vector<uint64_t> ids;
    {
        lr::Scheduler s(&ex, 1000);
        for (uint64_t i = 0; i < 200; ++i) ids.push_back(s.submit(req(i, 1 + (i * 37) % 100)));
        drain_or_fail(s);
        for (uint64_t id : ids) CHECK(status_of(s, id) == LR_OK);
    }
    std::vector<uint64_t> order;
    size_t most = 0;
    for (const auto& l : ex.log) {
        most = std::max(most, l.tags.size());
        order.insert(order.end(), l.tags.begin(), l.tags.end());
    }
    CHECK(order.size() == 200);
    for (uint64_t i = 0; i < 200; ++i) CHECK(order[i] == i);
    CHECK(most >= 3);  // batches do form
    puts("ok tiny_budget");
}

// A request that can never fit a slot is rejected alone; the requests
// around it run.
static void oversize_rejected_alone() {
    Mock ex(1, 1000);
    std::vector<uint64_t> ids;
    lr::Scheduler s(&ex, 8);
    ids.push_back(s.submit(req(0, 10)));
    ids.push_back(s.submit(req(1, 5000)));  // 64 + 5000 > 1000
    ids.push_back(s.submit(req(2, 10)));
    drain_or_fail(s);
    CHECK(status_of(s, ids[0]) == LR_OK);
    CHECK(status_of(s, ids[1]) == LR_ERR_WORKSPACE);
    CHECK(status_of(s, ids[2]) == LR_OK);
    for (const auto& l : ex.log)
        for (uint64_t t : l.tags) CHECK(t != 1);
    puts("ok oversize_rejected_alone");
}

// A batch whose launch fails, and a batch that fails while running, fail only
// their own requests; the slot is reused afterwards.
static void failure_isolation(bool at_launch) {
    Mock ex(2, 1 << 20);
    ex.run_time = 2000us;
    if (at_launch) ex.fail_launch_tag = 13;
    else ex.fail_poll_tag = 13;
    std::vector<uint64_t> ids;
    lr::Scheduler s(&ex, 4);
    for (uint64_t i = 0; i < 40; ++i) {
        ids.push_back(s.submit(req(i, 50)));
        if (i % 5 == 4) std::this_thread::sleep_for(300us);
    }
    drain_or_fail(s);
    std::vector<uint64_t> failed;
    for (const auto& l : ex.log)
        if (std::find(l.tags.begin(), l.tags.end(), 13ull) != l.tags.end()) failed = l.tags;
    CHECK(!failed.empty());
    for (uint64_t i = 0; i < 40; ++i) {
        const bool in_failed = std::find(failed.begin(), failed.end(), i) != failed.end();
        CHECK(status_of(s, ids[i]) == (in_failed ? LR_ERR_HIP : LR_OK));
    }
    puts(at_launch ? "ok failure_isolation_launch" : "ok failure_isolation_running");
}

// Latency counts from the arrival the caller states, and from the moment
// submit is entered otherwise.
static void latency_from_arrival() {
    Mock ex(1, 1 << 20);
    ex.run_time = 1000us;
    lr::Scheduler s(&ex, 1);
    const auto t0 = clk::now();
    const uint64_t a = s.submit(req(0, 10), t0 - 20ms);  // arrived 20 ms before its submission
    const uint64_t b = s.submit(req(1, 10));
    drain_or_fail(s);
    double la = 0, lb = 0;
    CHECK(status_of(s, a, &la) == LR_OK && status_of(s, b, &lb) == LR_OK);
    CHECK(la >= 0.020 + 0.001);
    CHECK(lb >= 0.001 && lb < la);
    const double da = std::chrono::duration<double>(s.done_time(a) - (t0 - 20ms)).count();
    CHECK(da == la);
    // request b ran after a: at least two run times from t0 to its completion
    CHECK(std::chrono::duration<double>(s.done_time(b) - t0).count() >= 0.002);
    puts("ok latency_from_arrival");
}

// Launches run outside the scheduler's lock: while a launch takes 200 ms,
// submissions and polls return at once.
static void launch_outside_lock() {
    Mock ex(1, 1 << 20);
    ex.launch_delay = 200000us;
    lr::Scheduler s(&ex, 1);
    const uint64_t a = s.submit(req(0, 10));
    std::this_thread::sleep_for(50ms);  // the worker is inside launch(a) now
    const auto t = clk::now();
    const uint64_t b = s.submit(req(1, 10));
    lr_status st;
    double lat;
    (void)s.poll(a, &st, &lat);
    const double waited = std::chrono::duration<double>(clk::now() - t).count();
    CHECK(waited < 0.05);
    drain_or_fail(s);
    CHECK(status_of(s, a) == LR_OK && status_of(s, b) == LR_OK);
    puts("ok launch_outside_lock");
}

int main() {
    fifo();
    tiny_budget();
    oversize_rejected_alone();
    failure_isolation(true);
    failure_isolation(false);
    latency_from_arrival();
    launch_outside_lock();
    return 0;
}
