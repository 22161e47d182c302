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

// Maps that cache grids: each request decodes one of a few grids; a grid not yet cached costs
// kGrid resident bytes from its run on.  The executor tracks the bytes it really holds (maps'
// resident bytes plus in-flight transient buffers) and checks them against the budget at every
// launch; reclaim drops every cached grid.
class CachingExecutor : public Executor {
public:
    static constexpr int64_t kBase = 100, kGrid = 300;
    CachingExecutor(int slots, int nmaps, int64_t budget)
        : cached_(nmaps), running_(slots), budget_(budget) {}

    struct Req {
        int map, grid;
        int64_t transient;
        bool ran = false;
    };
    int64_t resident_of(int m) const { return kBase + (int64_t)cached_[m].size() * kGrid; }

    void admission(const CoreRequest* q, int64_t* now, int64_t* growth) override {
        std::lock_guard<std::mutex> lk(mu_);
        const Req* r = static_cast<const Req*>(q->payload);
        *now = resident_of(r->map);
        *growth = cached_[r->map].count(r->grid) ? 0 : kGrid;
    }
    int launch(int slot, const std::vector<CoreRequest*>& batch) override {
        std::lock_guard<std::mutex> lk(mu_);
        for (CoreRequest* q : batch) {
            Req* r = static_cast<Req*>(q->payload);
            cached_[r->map].insert(r->grid);   // the run builds the grid's tables
            transient_ += r->transient;
            r->ran = true;
        }
        running_[slot] = batch.size();
        int64_t held = transient_;
        for (size_t m = 0; m < cached_.size(); ++m) held += resident_of((int)m);
        peak_held = std::max(peak_held, held);
        if (held > budget_) over_budget = true;
        return kCoreOk;
    }
    int query(int) override { return kCoreOk; }
    void complete(int, const std::vector<CoreRequest*>& batch, int status) override {
        std::lock_guard<std::mutex> lk(mu_);
        for (CoreRequest* q : batch) {
            Req* r = static_cast<Req*>(q->payload);
            transient_ -= r->transient;
            q->status = status;
            q->resident_after = resident_of(r->map);
            delete r;
            q->payload = nullptr;
        }
    }
    void release(CoreRequest* q) override {
        delete static_cast<Req*>(q->payload);
        q->payload = nullptr;
        ++released;
    }
    void reclaim(std::vector<int64_t>* res) override {
        std::lock_guard<std::mutex> lk(mu_);
        ++reclaims;
        for (size_t m = 0; m < cached_.size(); ++m) {
            cached_[m].clear();
            if (m < res->size()) (*res)[m] = resident_of((int)m);
        }
    }

    std::mutex mu_;
    std::vector<std::set<int>> cached_;
    std::vector<size_t> running_;
    int64_t budget_, transient_ = 0, peak_held = 0;
    int reclaims = 0, released = 0;
    bool over_budget = false;
};

std::unique_ptr<CoreRequest> make_cached(int map, int grid, int64_t transient) {
    auto q = std::make_unique<CoreRequest>();
    q->map = map;
    q->bytes = transient;
    q->precision = 3;
    q->batchable = true;
    q->payload = new CachingExecutor::Req{map, grid, transient};
    return q;
}

// Resident bytes count against the budget, grid caches are reclaimed when nothing runs and the
// next request does not fit, and a request too large even then completes with kCoreNomem.
void test_resident_bytes_and_reclaim() {
    SchedulerConfig cfg;
    cfg.slots = 4;
    cfg.workers = 2;
    cfg.max_batch = 2;
    cfg.poll_us = 1;
    const int nmaps = 4;
    cfg.budget = nmaps * CachingExecutor::kBase + 3 * CachingExecutor::kGrid + 200;   // 4 maps, 3 grids
    CachingExecutor ex(cfg.slots, nmaps, cfg.budget);
    Scheduler s(cfg, &ex);
    for (int m = 0; m < nmaps; ++m) CHECK(s.add_map(CachingExecutor::kBase) == m);
    CHECK(s.add_map(cfg.budget) == -1);   // a map as large as the budget does not fit beside them
    s.start();
    std::mt19937 rng(5);
    std::vector<uint64_t> tickets;
    std::vector<int> expect;
    for (int i = 0; i < 200; ++i) {
        const bool huge = (i == 120);
        const int m = (int)(rng() % nmaps), g = (int)(rng() % 5);
        auto q = make_cached(m, g, huge ? cfg.budget - nmaps * CachingExecutor::kBase : 20 + (int64_t)(rng() % 60));
        uint64_t t = 0;
        CHECK(s.submit(q, &t) == kCoreOk);
        tickets.push_back(t);
        expect.push_back(huge ? kCoreNomem : kCoreOk);
    }
    for (size_t i = 0; i < tickets.size(); ++i) {
        CoreRequest r;
        CHECK(s.wait(tickets[i], &r) == kCoreOk);
        CHECK(r.status == expect[i]);
    }
    int64_t completed = 0, peak = 0, budget = 0, batches = 0, resident = 0, reclaims = 0;
    s.stats(&completed, &peak, &budget, &batches, &resident, &reclaims);
    CHECK(completed == 200);
    CHECK(peak <= budget);
    CHECK(reclaims >= 1 && reclaims == ex.reclaims);
    CHECK(ex.released == 1);   // the refused one
    CHECK(!ex.over_budget);
    CHECK(ex.peak_held <= cfg.budget);
    s.stop();
}

int main() {
    test_stream_order_batches_budget();
    test_backpressure_and_refusals();
    test_injected_failures();
    test_budget_blocks_later_requests();
    test_resident_bytes_and_reclaim();
    if (g_failures) {
        std::fprintf(stderr, "%d check(s) failed\n", g_failures);
        return 1;
    }
    std::printf("server core: all checks passed\n");
    return 0;
}
