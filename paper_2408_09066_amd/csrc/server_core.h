// Scheduling core of the request loop: tickets, the queue of pending requests, per-map order,
// admission against a device-byte budget and a number of execution slots, and the grouping of
// admitted requests into batches.  It makes no device call: an Executor runs the batches (the
// HIP executor of server.hip on a GPU, a simulated one in the CPU tests), so the admission and
// ordering rules can be tested without a device.
//
// Rules.  Requests are considered in submission order.  A request whose map has an update in
// flight, or an earlier request still pending, waits (updates of one map run in submission
// order: memories are state); requests of other maps pass it.  A request that does not fit the
// remaining budget stops admission (first come, first served: nothing behind it is admitted
// until running requests release their bytes).
//
// Budget.  The bytes counted against it are those of the requests in flight (each charged its
// transient bytes plus an upper bound on what its run can add to its map's resident memory,
// asked of the executor at admission, when the map is idle), the resident bytes of every map
// (reported at admission and at completion) and the executor's fixed buffers.  When nothing
// is in flight and the first waiting request still does not fit, the executor is asked once to
// reclaim what the maps rebuild on demand; if it still does not fit, it completes with
// kCoreNomem without running.  Requests of distinct maps with the same
// precision and the batchable flag are admitted together into one batch of at most max_batch;
// a request that is not batchable runs alone in its slot.
#pragma once

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

namespace vsaogm {

inline int64_t steady_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// Status codes (the values of vsaogm_status).
enum CoreStatus { kCoreOk = 0, kCoreInval = -1, kCoreNomem = -2, kCoreDevice = -3, kCoreAgain = -4, kCoreBusy = -5,
                  kCoreNotFound = -6 };

struct CoreRequest {
    uint64_t ticket = 0;
    int32_t map = 0;
    int64_t bytes = 0;           // device bytes held from admission to completion
    int32_t precision = 0;
    bool batchable = false;      // may share a batch with other maps' requests of its precision
    int32_t status = kCoreAgain; // the update's status once done
    int32_t slot = -1;
    bool done = false;
    int64_t t_submit_ns = 0, t_start_ns = 0, t_done_ns = 0;
    float result[2] = {0.f, 0.f}; // values the executor reports with the status (class maxima)
    void* payload = nullptr;     // the executor's view of the request (inputs, outputs)
    int64_t charge = 0;          // bytes held against the budget while in flight
    int64_t resident_after = -1; // the map's resident bytes after the run (set by complete)
};

// Runs batches on execution slots.  launch() enqueues the batch's work on the slot and returns
// at once (a launch failure is returned, and the batch then completes with that status);
// query() reports kCoreAgain while the slot's work runs, kCoreOk when it finished and an error
// status when it failed; complete() hands the results back (called once per batch, after query
// stopped returning kCoreAgain, or after a failed launch).  Each slot is driven by one worker
// thread.
class Executor {
public:
    virtual ~Executor() = default;
    virtual int launch(int slot, const std::vector<CoreRequest*>& batch) = 0;
    virtual int query(int slot) = 0;
    virtual void complete(int slot, const std::vector<CoreRequest*>& batch, int status) = 0;
    // called when the request is dropped without running (server shut down with it pending,
    // or refused for memory)
    virtual void release(CoreRequest*) {}
    // At admission (scheduler lock held, the request's map idle): the map's resident bytes now
    // (-1: unchanged) and an upper bound on what the request's run can add to them.
    virtual void admission(const CoreRequest*, int64_t* resident_now, int64_t* growth) {
        *resident_now = -1;
        *growth = 0;
    }
    // Device bytes of the executor's own buffers (read under the scheduler lock; thread-safe).
    virtual int64_t fixed_bytes() { return 0; }
    // Nothing in flight: release what can be rebuilt on demand; resident[m] = map m's bytes
    // after (entries left at -1 are unchanged).
    virtual void reclaim(std::vector<int64_t>* resident) { (void)resident; }
};

struct SchedulerConfig {
    int slots = 4;              // execution slots (batches in flight)
    int max_queue = 1024;       // pending requests before submit refuses
    int max_batch = 8;          // requests per batch
    int workers = 1;            // threads driving the slots
    int64_t budget = 1 << 30;   // device bytes for in-flight requests
    int poll_us = 20;           // sleep between queries while the worker's slots run
};

class Scheduler {
public:
    Scheduler(const SchedulerConfig& cfg, Executor* ex) : cfg_(cfg), ex_(ex), slots_(cfg.slots) {}
    ~Scheduler() { stop(); }
    Scheduler(const Scheduler&) = delete;
    Scheduler& operator=(const Scheduler&) = delete;

    void start() {
        for (int w = 0; w < cfg_.workers; ++w) threads_.emplace_back([this, w] { run(w); });
    }
    // Finish everything admitted and pending, then join the workers.
    void stop() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (stopping_ && threads_.empty()) return;
            stopping_ = true;
        }
        cv_work_.notify_all();
        for (auto& t : threads_)
            if (t.joinable()) t.join();
        threads_.clear();
    }

    // A new map holding resident bytes already; -1 (and no map) if they do not fit the budget.
    int add_map(int64_t resident = 0) {
        std::lock_guard<std::mutex> lk(mu_);
        if (resident_ + resident + ex_->fixed_bytes() > cfg_.budget) return -1;
        map_busy_.push_back(0);
        map_resident_.push_back(resident);
        resident_ += resident;
        peak_ = std::max(peak_, used_ + resident_ + ex_->fixed_bytes());
        return (int)map_busy_.size() - 1;
    }
    int num_maps() {
        std::lock_guard<std::mutex> lk(mu_);
        return (int)map_busy_.size();
    }

    // Queue one prepared request; kCoreBusy when the queue is full (the request is not queued and
    // stays the caller's), kCoreInval when it alone exceeds the budget, kCoreNotFound for an
    // unknown map.  On success the scheduler owns it.
    int submit(std::unique_ptr<CoreRequest>& q, uint64_t* ticket) {
        std::vector<std::unique_ptr<CoreRequest>*> one{&q};
        int n = 0;
        return submit_many(one, ticket, &n);
    }
    // Queue in order until the first failure; *queued = how many were queued.
    int submit_many(const std::vector<std::unique_ptr<CoreRequest>*>& qs, uint64_t* tickets, int* queued) {
        int rc = kCoreOk;
        *queued = 0;
        {
            std::lock_guard<std::mutex> lk(mu_);
            for (auto* qp : qs) {
                CoreRequest* q = qp->get();
                if (q->map < 0 || q->map >= (int)map_busy_.size()) {
                    rc = kCoreNotFound;
                    break;
                }
                if (q->bytes > cfg_.budget) {
                    rc = kCoreInval;
                    break;
                }
                if ((int)pending_.size() >= cfg_.max_queue) {
                    rc = kCoreBusy;
                    break;
                }
                q->ticket = next_ticket_++;
                q->t_submit_ns = steady_ns();
                q->status = kCoreAgain;
                q->done = false;
                tickets[*queued] = q->ticket;
                pending_.push_back(q);
                tickets_.emplace(q->ticket, std::move(*qp));
                ++*queued;
            }
        }
        if (*queued) cv_work_.notify_all();
        return rc;
    }

    // Non-blocking: kCoreAgain while running; kCoreOk with *out filled (and the ticket retired)
    // once done; kCoreNotFound for an unknown or retired ticket.
    int poll(uint64_t ticket, CoreRequest* out) {
        std::lock_guard<std::mutex> lk(mu_);
        return poll_locked(ticket, out);
    }
    int wait(uint64_t ticket, CoreRequest* out) {
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            const int rc = poll_locked(ticket, out);
            if (rc != kCoreAgain) return rc;
            cv_done_.wait(lk);
        }
    }
    void drain() {
        std::unique_lock<std::mutex> lk(mu_);
        cv_done_.wait(lk, [&] { return pending_.empty() && inflight_ == 0; });
    }
    void stats(int64_t* completed, int64_t* peak, int64_t* budget, int64_t* batches, int64_t* resident = nullptr,
               int64_t* reclaims = nullptr) {
        std::lock_guard<std::mutex> lk(mu_);
        if (completed) *completed = completed_;
        if (peak) *peak = peak_;
        if (budget) *budget = cfg_.budget;
        if (batches) *batches = batches_;
        if (resident) *resident = resident_;
        if (reclaims) *reclaims = reclaims_;
    }
    int64_t budget() const { return cfg_.budget; }
    // Bytes counted against the budget now: in-flight charges, maps' resident bytes, the
    // executor's fixed buffers; and how many reclaims ran.
    void memory(int64_t* in_flight, int64_t* resident, int64_t* fixed, int64_t* reclaims) {
        std::lock_guard<std::mutex> lk(mu_);
        if (in_flight) *in_flight = used_;
        if (resident) *resident = resident_;
        if (fixed) *fixed = ex_->fixed_bytes();
        if (reclaims) *reclaims = reclaims_;
    }

private:
    struct SlotState {
        std::vector<CoreRequest*> batch;
        int launch_status = kCoreOk;
    };

    int poll_locked(uint64_t ticket, CoreRequest* out) {
        auto it = tickets_.find(ticket);
        if (it == tickets_.end()) return kCoreNotFound;
        if (!it->second->done) return kCoreAgain;
        if (out) {
            *out = *it->second;
            out->payload = nullptr;
        }
        tickets_.erase(it);
        return kCoreOk;
    }

    // Admission for one free slot (lock held): the batch to launch there, possibly empty.
    std::vector<CoreRequest*> admit_locked() {
        std::vector<CoreRequest*> batch;
        if (reclaiming_) return batch;
        std::unordered_set<int32_t> blocked;   // maps with an earlier request still waiting
        for (auto it = pending_.begin(); it != pending_.end();) {
            CoreRequest* q = *it;
            if (map_busy_[q->map] || blocked.count(q->map)) {
                blocked.insert(q->map);
                ++it;
                continue;
            }
            if (!batch.empty()) {
                const CoreRequest* f = batch.front();
                if (!f->batchable) break;   // a lone request fills its slot
                if (!q->batchable || q->precision != f->precision) {
                    blocked.insert(q->map);  // keeps its map's order; may run in another slot
                    ++it;
                    continue;
                }
            }
            int64_t now = -1, grow = 0;
            ex_->admission(q, &now, &grow);
            if (now >= 0) {
                resident_ += now - map_resident_[q->map];
                map_resident_[q->map] = now;
            }
            const int64_t charge = q->bytes + std::max<int64_t>(grow, 0);
            const int64_t fixed = ex_->fixed_bytes();
            if (used_ + resident_ + fixed + charge > cfg_.budget) {   // first come, first served
                if (inflight_ == 0 && batch.empty()) {
                    if (!reclaimed_) {
                        want_reclaim_ = true;   // the worker reclaims outside the lock
                    } else {
                        // cannot fit even with everything reclaimed: refuse it
                        it = pending_.erase(it);
                        q->status = kCoreNomem;
                        q->t_start_ns = q->t_done_ns = steady_ns();
                        q->done = true;
                        ++completed_;
                        ex_->release(q);
                        refused_ = true;
                        continue;
                    }
                }
                break;
            }
            q->charge = charge;
            used_ += charge;
            peak_ = std::max(peak_, used_ + resident_ + fixed);
            map_busy_[q->map] = 1;
            ++inflight_;
            batch.push_back(q);
            it = pending_.erase(it);
            if ((int)batch.size() >= cfg_.max_batch || !q->batchable) break;
        }
        return batch;
    }

    // Worker w drives a contiguous block of slots: streams are spread over the device's hardware
    // queues in creation order, so a worker's concurrent batches land on different queues.
    int slot_begin(int w) const { return (int)((int64_t)w * (int64_t)slots_.size() / cfg_.workers); }

    void run(int w) {
        const int s0 = slot_begin(w), s1 = slot_begin(w + 1);
        std::vector<int> free_slots;
        for (int i = s1 - 1; i >= s0; --i) free_slots.push_back(i);
        for (;;) {
            bool progressed = false;
            for (int i = s0; i < s1; ++i) {
                SlotState& s = slots_[i];
                if (s.batch.empty()) continue;
                int st = s.launch_status;
                if (st == kCoreOk) {
                    st = ex_->query(i);
                    if (st == kCoreAgain) continue;
                }
                ex_->complete(i, s.batch, st);
                const int64_t t = steady_ns();
                {
                    std::lock_guard<std::mutex> lk(mu_);
                    for (CoreRequest* q : s.batch) {
                        if (q->status == kCoreAgain) q->status = st;
                        q->t_done_ns = t;
                        used_ -= q->charge;
                        if (q->resident_after >= 0) {
                            resident_ += q->resident_after - map_resident_[q->map];
                            map_resident_[q->map] = q->resident_after;
                        }
                        reclaimed_ = false;   // progress: a later blockage may reclaim again
                        map_busy_[q->map] = 0;
                        q->done = true;
                        ++completed_;
                        --inflight_;
                    }
                }
                cv_done_.notify_all();
                cv_work_.notify_all();   // a map or budget freed up for the other workers
                s.batch.clear();
                s.launch_status = kCoreOk;
                free_slots.push_back(i);
                progressed = true;
            }
            std::vector<std::pair<int, std::vector<CoreRequest*>>> to_launch;
            bool reclaim = false;
            {
                std::unique_lock<std::mutex> lk(mu_);
                if (stopping_ && pending_.empty() && inflight_ == 0) break;
                while (!free_slots.empty()) {
                    std::vector<CoreRequest*> b = admit_locked();
                    if (refused_) {
                        refused_ = false;
                        cv_done_.notify_all();
                    }
                    if (want_reclaim_ && inflight_ == 0 && !reclaiming_) {
                        want_reclaim_ = false;
                        reclaiming_ = true;   // no admission anywhere until it is done
                        reclaim = true;
                        break;
                    }
                    if (b.empty()) break;
                    const int si = free_slots.back();
                    free_slots.pop_back();
                    ++batches_;
                    for (CoreRequest* q : b) q->slot = si;
                    slots_[si].batch = b;
                    to_launch.emplace_back(si, std::move(b));
                }
                if (to_launch.empty() && !progressed && !reclaim) {
                    bool mine = false;
                    for (int i = s0; i < s1; ++i) mine = mine || !slots_[i].batch.empty();
                    // a system-clock deadline (pthread_cond_timedwait), which thread sanitizers
                    // follow; a short poll interval does not mind clock adjustments
                    cv_work_.wait_until(lk, std::chrono::system_clock::now() +
                                                std::chrono::microseconds(mine ? cfg_.poll_us : 2000));
                    continue;
                }
            }
            for (auto& [si, b] : to_launch) {
                const int64_t t = steady_ns();
                for (CoreRequest* q : b) q->t_start_ns = t;
                slots_[si].launch_status = ex_->launch(si, b);
            }
            if (reclaim) {
                std::vector<int64_t> res;
                {
                    std::lock_guard<std::mutex> lk(mu_);
                    res.assign(map_resident_.size(), -1);
                }
                ex_->reclaim(&res);
                std::lock_guard<std::mutex> lk(mu_);
                for (size_t m = 0; m < res.size() && m < map_resident_.size(); ++m)
                    if (res[m] >= 0) {
                        resident_ += res[m] - map_resident_[m];
                        map_resident_[m] = res[m];
                    }
                ++reclaims_;
                reclaimed_ = true;
                reclaiming_ = false;
                cv_work_.notify_all();
            }
        }
    }

    SchedulerConfig cfg_;
    Executor* ex_;
    std::vector<SlotState> slots_;
    std::vector<std::thread> threads_;
    std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    bool stopping_ = false;
    std::deque<CoreRequest*> pending_;
    std::unordered_map<uint64_t, std::unique_ptr<CoreRequest>> tickets_;
    std::vector<char> map_busy_;
    std::vector<int64_t> map_resident_;
    uint64_t next_ticket_ = 1;
    int64_t used_ = 0, resident_ = 0, peak_ = 0, completed_ = 0, batches_ = 0, reclaims_ = 0;
    int inflight_ = 0;
    bool want_reclaim_ = false, reclaiming_ = false, reclaimed_ = false, refused_ = false;
};

}  // namespace vsaogm
