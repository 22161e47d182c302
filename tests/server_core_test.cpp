// CPU tests of the request loop's scheduling core (paper_2408_09066_amd/csrc/server_core.h)
// with a simulated executor: no device.  Built and run by tests/test_server_core.py under
// AddressSanitizer + UndefinedBehaviorSanitizer and under ThreadSanitizer.  Exit status 0 when
// every check passes; each failed check prints its line.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <memory>
#include <mutex>
#include <random>
#include <set>
#include <thread>
#include <vector>

#include "server_core.h"

using namespace vsaogm;

static int g_failures = 0;
#define CHECK(c)                                                                 \
    do {                                                                         \
        if (!(c)) {                                                              \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            ++g_failures;                                                        \
        }                                                                        \
    } while (0)

// A payload the simulated executor understands: a per-map sequence number and what to inject.
struct FakeReq {
    int map = 0;
    int seq = 0;              // submission order within the map
    bool fail_launch = false;
    bool fail_run = false;
};

// Runs batches by counting polls: a batch finishes after 1..max_polls queries (seeded), so
// completions arrive out of submission order.  Records what it saw for the checks.
class FakeExecutor : public Executor {
public:
    FakeExecutor(int slots, unsigned seed, int max_polls, int64_t budget)
        : polls_left_(slots, 0), fail_(slots, 0), rng_(seed), max_polls_(max_polls), budget_(budget) {}

    int launch(int slot, const std::vector<CoreRequest*>& batch) override {
        std::lock_guard<std::mutex> lk(mu_);
        ++batches;
        max_batch_seen = std::max(max_batch_seen, (int)batch.size());
        std::set<int> maps;
        int failing = kCoreOk;
        for (CoreRequest* q : batch) {
            FakeReq* f = static_cast<FakeReq*>(q->payload);
            if (!maps.insert(f->map).second) duplicate_map_in_batch = true;
            if (q->precision != batch.front()->precision) mixed_precision = true;
            if (!q->batchable && batch.size() > 1) lone_shared = true;
            if (in_flight_maps.count(f->map)) map_twice_in_flight = true;
            in_flight_maps.insert(f->map);
            // per-map order: sequence numbers launch strictly in order
            auto it = last_seq.find(f->map);
            if (it != last_seq.end() && f->seq != it->second + 1) order_broken = true;
            last_seq[f->map] = f->seq;
            bytes_in_flight += q->bytes;
            if (f->fail_launch) failing = kCoreDevice;
            if (f->fail_run) fail_[slot] = kCoreNomem;
        }
        peak_bytes = std::max(peak_bytes, bytes_in_flight);
        if (bytes_in_flight > budget_) over_budget = true;
        polls_left_[slot] = 1 + (int)(rng_() % (unsigned)max_polls_);
        return failing;
    }
    int query(int slot) override {
        std::lock_guard<std::mutex> lk(mu_);
        if (hold) return kCoreAgain;
        if (--polls_left_[slot] > 0) return kCoreAgain;
        const int st = fail_[slot];
        fail_[slot] = 0;
        return st == 0 ? kCoreOk : st;
    }
    void complete(int, const std::vector<CoreRequest*>& batch, int status) override {
        std::lock_guard<std::mutex> lk(mu_);
        for (CoreRequest* q : batch) {
            FakeReq* f = static_cast<FakeReq*>(q->payload);
            in_flight_maps.erase(f->map);
            bytes_in_flight -= q->bytes;
            q->status = status;
            q->result[0] = (float)f->seq;
            delete f;
            q->payload = nullptr;
        }
    }
    void release(CoreRequest* q) override {
        delete static_cast<FakeReq*>(q->payload);
        q->payload = nullptr;
    }

    std::atomic<bool> hold{false};
    std::mutex mu_;
    std::map<int, int> last_seq;
    std::set<int> in_flight_maps;
    int64_t bytes_in_flight = 0, peak_bytes = 0;
    int batches = 0, max_batch_seen = 0;
    bool duplicate_map_in_batch = false, mixed_precision = false, lone_shared = false, map_twice_in_flight = false,
         order_broken = false, over_budget = false;

private:
    std::vector<int> polls_left_, fail_;
    std::mt19937 rng_;
    int max_polls_;
    int64_t budget_;
};

std::unique_ptr<CoreRequest> make(int map, int seq, int64_t bytes, int precision, bool batchable,
                                  bool fail_launch = false, bool fail_run = false) {
    auto q = std::make_unique<CoreRequest>();
    q->map = map;
    q->bytes = bytes;
    q->precision = precision;
    q->batchable = batchable;
    auto* f = new FakeReq();
    f->map = map;
    f->seq = seq;
    f->fail_launch = fail_launch;
    f->fail_run = fail_run;
    q->payload = f;
    return q;
}

// Many requests over a few maps, several slots and workers, random completion order.
void test_stream_order_batches_budget() {
    SchedulerConfig cfg;
    cfg.slots = 4;
    cfg.workers = 2;
    cfg.max_batch = 3;
    cfg.max_queue = 1000;
    cfg.budget = 1000;
    cfg.poll_us = 1;
    FakeExecutor ex(cfg.slots, 7u, 6, cfg.budget);
    Scheduler s(cfg, &ex);
    const int nmaps = 5;
    for (int m = 0; m < nmaps; ++m) CHECK(s.add_map() == m);
    s.start();
    std::mt19937 rng(11);
    std::vector<int> seq(nmaps, 0);
    std::vector<uint64_t> tickets;
    std::vector<int> expect_seq;
    for (int i = 0; i < 300; ++i) {
        const int m = (int)(rng() % nmaps);
        const int prec = (rng() % 4 == 0) ? 1 : 3;
        const bool batchable = rng() % 5 != 0;
        auto q = make(m, seq[m]++, 50 + (int64_t)(rng() % 200), prec, batchable);
        uint64_t t = 0;
        CHECK(s.submit(q, &t) == kCoreOk);
        tickets.push_back(t);
        expect_seq.push_back(seq[m] - 1);
    }
    for (size_t i = 0; i < tickets.size(); ++i) {
        CoreRequest r;
        CHECK(s.wait(tickets[i], &r) == kCoreOk);
        CHECK(r.status == kCoreOk);
        CHECK(r.result[0] == (float)expect_seq[i]);
        CHECK(r.t_submit_ns <= r.t_start_ns && r.t_start_ns <= r.t_done_ns);
        CoreRequest again;
        CHECK(s.poll(tickets[i], &again) == kCoreNotFound);   // retired
    }
    s.drain();
    int64_t completed = 0, peak = 0, budget = 0, batches = 0;
    s.stats(&completed, &peak, &budget, &batches);
    CHECK(completed == 300);
    CHECK(peak <= budget && peak > 0);
    CHECK(batches < 300);   // some requests shared a batch
    CHECK(!ex.duplicate_map_in_batch);
    CHECK(!ex.mixed_precision);
    CHECK(!ex.lone_shared);
    CHECK(!ex.map_twice_in_flight);
    CHECK(!ex.order_broken);
    CHECK(!ex.over_budget);
    CHECK(ex.max_batch_seen <= cfg.max_batch && ex.max_batch_seen > 1);
    s.stop();
}

// A full queue refuses (EBUSY) without taking the request; a request above the budget alone is
// invalid; an unknown map is not found.
void test_backpressure_and_refusals() {
    SchedulerConfig cfg;
    cfg.slots = 1;
    cfg.workers = 1;
    cfg.max_queue = 4;
    cfg.budget = 100;
    cfg.poll_us = 1;
    FakeExecutor ex(cfg.slots, 3u, 2, cfg.budget);
    ex.hold = true;   // nothing completes until released
    Scheduler s(cfg, &ex);
    s.add_map();
    s.start();
    std::vector<uint64_t> tickets;
    int queued_ok = 0, busy = 0;
    for (int i = 0; i < 12; ++i) {
        auto q = make(0, i, 10, 3, true);
        uint64_t t = 0;
        const int rc = s.submit(q, &t);
        if (rc == kCoreOk) {
            ++queued_ok;
            tickets.push_back(t);
        } else {
            CHECK(rc == kCoreBusy);
            CHECK(q != nullptr && q->payload != nullptr);   // still the caller's
            ex.release(q.get());
            ++busy;
        }
        // give the worker time to admit the first one (one map: one in flight, the rest pend)
        if (i == 0) std::this_thread::sleep_for(std::chrono::milliseconds(20));
    }
    CHECK(queued_ok == 5);   // one running + four pending
    CHECK(busy == 7);
    auto big = make(0, 99, 1000, 3, true);
    uint64_t t = 0;
    CHECK(s.submit(big, &t) == kCoreInval);
    ex.release(big.get());
    auto lost = make(5, 0, 10, 3, true);
    CHECK(s.submit(lost, &t) == kCoreNotFound);
    ex.release(lost.get());
    ex.hold = false;
    for (uint64_t tk : tickets) {
        CoreRequest r;
        CHECK(s.wait(tk, &r) == kCoreOk);
        CHECK(r.status == kCoreOk);
    }
    s.stop();
}

// A failed launch and a failed run reach poll as the request's status; the others succeed.
void test_injected_failures() {
    SchedulerConfig cfg;
    cfg.slots = 2;
    cfg.workers = 1;
    cfg.max_batch = 1;   // one request per batch, so each failure hits only its request
    cfg.budget = 1 << 20;
    cfg.poll_us = 1;
    FakeExecutor ex(cfg.slots, 5u, 3, cfg.budget);
    Scheduler s(cfg, &ex);
    for (int m = 0; m < 3; ++m) s.add_map();
    s.start();
    std::vector<uint64_t> tickets;
    std::vector<int> expect;
    for (int i = 0; i < 30; ++i) {
        const bool fl = i == 7, fr = i == 19;
        auto q = make(i % 3, i / 3, 10, 3, true, fl, fr);
        uint64_t t = 0;
        CHECK(s.submit(q, &t) == kCoreOk);
        tickets.push_back(t);
        expect.push_back(fl ? kCoreDevice : (fr ? kCoreNomem : kCoreOk));
    }
    for (size_t i = 0; i < tickets.size(); ++i) {
        CoreRequest r;
        CHECK(s.wait(tickets[i], &r) == kCoreOk);
        CHECK(r.status == expect[i]);
    }
    CHECK(!ex.order_broken && !ex.map_twice_in_flight);
    s.stop();
}

// Budget admission is first come, first served: a request that does not fit stops admission of
// everything behind it until bytes are released.
void test_budget_blocks_later_requests() {
    SchedulerConfig cfg;
    cfg.slots = 4;
    cfg.workers = 1;
    cfg.max_batch = 4;
    cfg.budget = 100;
    cfg.poll_us = 1;
    FakeExecutor ex(cfg.slots, 9u, 4, cfg.budget);
    Scheduler s(cfg, &ex);
    for (int m = 0; m < 6; ++m) s.add_map();
    s.start();
    std::vector<uint64_t> tickets;
    const int64_t bytes[] = {60, 60, 30, 30, 90, 10, 10, 100};
    for (int i = 0; i < 8; ++i) {
        auto q = make(i % 6, i / 6, bytes[i], 3, true);
        uint64_t t = 0;
        CHECK(s.submit(q, &t) == kCoreOk);
        tickets.push_back(t);
    }
    for (uint64_t tk : tickets) {
        CoreRequest r;
        CHECK(s.wait(tk, &r) == kCoreOk);
        CHECK(r.status == kCoreOk);
    }
    CHECK(!ex.over_budget);
    CHECK(ex.peak_bytes <= 100);
    s.stop();
}

int main() {
    test_stream_order_batches_budget();
    test_backpressure_and_refusals();
    test_injected_failures();
    test_budget_blocks_later_requests();
    if (g_failures) {
        std::fprintf(stderr, "%d check(s) failed\n", g_failures);
        return 1;
    }
    std::printf("server core: all checks passed\n");
    return 0;
}
