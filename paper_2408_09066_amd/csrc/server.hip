// Request server for map updates (vsaogm_server_* / vsaogm_submit / vsaogm_poll).
//
// Worker threads (up to four) own the device side, each a share of the execution slots.  Each
// slot is a HIP stream with its own device and pinned host buffers; a request admitted to a
// slot runs its whole update there:
// one host-to-device copy of the points (staged by submit in pooled pinned memory), encode into its map (Algorithm 1), decode of its grid
// (eqs. vector-normalization, loc-query), classification (Algorithm 2, eqs. softmax, psd,
// classification) and device-to-host copies of the outputs, closed by an event.  Slots run
// concurrently, so updates of different maps overlap on the GPU; a map is bound to at most one
// slot at a time and its requests are admitted in submission order.  Admission is first come,
// first served against a device-memory budget: a request that does not fit blocks the ones
// behind it until running requests finish and release their bytes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "internal.h"
#include "vsaogm.h"

namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}


struct Fail : std::runtime_error {
    int code;
    Fail(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void check_hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return;
    throw Fail(e == hipErrorOutOfMemory ? VSAOGM_ENOMEM : VSAOGM_EDEVICE,
               std::string(what) + ": " + hipGetErrorString(e));
}

template <class F>
int guard(F&& f) {
    try {
        f();
        return VSAOGM_OK;
    } catch (const Fail& e) {
        vsaogm::set_last_error(e.what());
        return e.code;
    } catch (const std::bad_alloc&) {
        vsaogm::set_last_error("host allocation failed");
        return VSAOGM_ENOMEM;
    } catch (const std::exception& e) {
        vsaogm::set_last_error(e.what());
        return VSAOGM_EDEVICE;
    }
}

// Device buffer of a slot, grown in the order of the slot's stream (no device-wide sync).
struct DevMem {
    void* p = nullptr;
    size_t bytes = 0;
    void ensure(size_t need, hipStream_t s, const char* what) {
        if (need <= bytes) return;
        if (p) check_hip(hipFreeAsync(p, s), what);
        p = nullptr;
        bytes = 0;
        size_t cap = 1 << 21;
        while (cap < need) cap *= 2;
        check_hip(hipMallocAsync(&p, cap, s), what);
        bytes = cap;
    }
    ~DevMem() {
        if (p) (void)hipFree(p);
    }
};

struct HostMem {
    void* p = nullptr;
    size_t bytes = 0;
    void ensure(size_t need, const char* what) {
        if (need <= bytes) return;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
        size_t cap = 1 << 21;
        while (cap < need) cap *= 2;
        check_hip(hipHostMalloc(&p, cap, hipHostMallocDefault), what);
        bytes = cap;
    }
    ~HostMem() {
        if (p) (void)hipHostFree(p);
    }
};

// Pinned host blocks of power-of-two sizes, reused across requests (allocating pinned memory
// per request would cost more than the request's copies).
struct PinnedPool {
    std::mutex mu;
    std::vector<std::pair<size_t, void*>> free_blocks;
    std::vector<void*> all;
    std::pair<void*, size_t> get(size_t need) {
        size_t cap = 1 << 16;
        while (cap < need) cap *= 2;
        {
            std::lock_guard<std::mutex> lk(mu);
            for (size_t i = 0; i < free_blocks.size(); ++i)
                if (free_blocks[i].first == cap) {
                    void* p = free_blocks[i].second;
                    free_blocks[i] = free_blocks.back();
                    free_blocks.pop_back();
                    return {p, cap};
                }
        }
        void* p = nullptr;
        check_hip(hipHostMalloc(&p, cap, hipHostMallocDefault), "pinned request buffer");
        std::lock_guard<std::mutex> lk(mu);
        all.push_back(p);
        return {p, cap};
    }
    void put(void* p, size_t cap) {
        std::lock_guard<std::mutex> lk(mu);
        free_blocks.emplace_back(cap, p);
    }
    ~PinnedPool() {
        for (void* p : all) (void)hipHostFree(p);
    }
};

struct Request {
    uint64_t ticket = 0;
    vsaogm_request r{};
    void* in = nullptr;       // pinned [n][2] float32 points, then [n] labels
    size_t in_cap = 0;
    int64_t footprint = 0;
    vsaogm_result res{};
    bool done = false;
};

// Output block on the device and in pinned memory: maxima, labels, map, heatmaps, each
// 256-byte aligned; one copy brings back the prefix holding what the request asked for.
struct OutLayout {
    size_t lab, ogm, heat, end_lab, end_ogm, end_heat;
    explicit OutLayout(int64_t cells) {
        auto up = [](size_t v) { return (v + 255) / 256 * 256; };
        lab = 256;
        ogm = up(lab + cells);
        heat = up(ogm + cells * 4);
        end_lab = lab + cells;
        end_ogm = ogm + cells * 4;
        end_heat = heat + cells * 8;
    }
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    Request* req = nullptr;
    DevMem d_in, d_out;
    HostMem h_out;
};

// Bytes a request holds while it runs: its inputs and outputs on the device plus the map's
// working buffers for its points (sorted coordinates, keys, partial spectra) and grid.
int64_t footprint_of(const vsaogm_request& r, int32_t dim, int64_t nkeys) {
    const int64_t n = r.n, cells = (int64_t)r.grid.nx * r.grid.ny;
    const int64_t halfp = ((int64_t)dim / 2 + 63) / 64 * 64;
    const int64_t inputs = n * 9;
    const int64_t outputs = cells * 13 + 8;
    // work items hold at least 64 points, plus one partial item per memory
    const int64_t encode_ws = n * 20 + (n / 64 + 1 + nkeys) * halfp * 8;
    const int64_t decode_ws = (int64_t)256 * 2 * 2 * 256 * 64 * 4;  // stream-K partial sums (upper bound)
    return inputs + outputs + encode_ws + decode_ws;
}

}  // namespace

struct vsaogm_server {
    int device = 0;
    int64_t budget = 0, used = 0, peak = 0;
    int max_inflight = 4, max_queue = 1024;
    std::vector<vsaogm_map*> maps;
    std::vector<int32_t> map_dim;
    std::vector<int64_t> map_keys;
    std::vector<char> map_busy;
    // heat kept per map for VSAOGM_REQUEST_LOCAL (only the map's own running request uses it)
    struct LocalHeat {
        DevMem heat;
        vsaogm_grid_desc grid{};
    };
    std::vector<std::unique_ptr<LocalHeat>> local_heat;
    std::deque<Request*> pending;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> tickets;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    uint64_t next_ticket = 1;
    int64_t completed = 0;
    int inflight = 0;

    int nworkers = 1;
    std::vector<std::thread> workers;
    PinnedPool pool;

    void run(int w);
    void launch(Slot& s, int slot_index);
    void finish(Slot& s);
};

void vsaogm_server::launch(Slot& s, int slot_index) {
    Request* q = s.req;
    const vsaogm_request& r = q->r;
    q->res.slot = slot_index;
    q->res.t_start_ns = now_ns();
    int rc = VSAOGM_OK;
    try {
        const int64_t n = r.n, cells = (int64_t)r.grid.nx * r.grid.ny;
        const OutLayout L(cells);
        const size_t back = r.heat ? L.end_heat : (r.ogm ? L.end_ogm : (r.label_out ? L.end_lab : 8));
        s.d_in.ensure(std::max<int64_t>(n, 1) * 9, s.stream, "slot inputs");
        s.d_out.ensure(L.end_heat, s.stream, "slot outputs");
        s.h_out.ensure(back, "slot pinned outputs");
        unsigned char* din = static_cast<unsigned char*>(s.d_in.p);
        unsigned char* dout = static_cast<unsigned char*>(s.d_out.p);
        if (n > 0)
            check_hip(hipMemcpyAsync(din, q->in, n * 9, hipMemcpyHostToDevice, s.stream), "copy inputs");
        vsaogm_map* m = maps[r.map_id];
        auto call = [&](int code) {
            if (code != VSAOGM_OK) throw Fail(code, vsaogm_last_error());
        };
        float* hmax = reinterpret_cast<float*>(dout);
        float* heat = reinterpret_cast<float*>(dout + L.heat);
        call(vsaogm_encode(m, reinterpret_cast<float*>(din), din + n * 8, n, s.stream));
        if (r.flags & VSAOGM_REQUEST_LOCAL) {
            LocalHeat& lh = *local_heat[r.map_id];
            const bool same = lh.heat.p && lh.grid.nx == r.grid.nx && lh.grid.ny == r.grid.ny &&
                              lh.grid.x0 == r.grid.x0 && lh.grid.y0 == r.grid.y0 && lh.grid.res == r.grid.res;
            if (!same) {
                lh.heat.ensure(cells * 8, s.stream, "map heat");
                lh.grid = r.grid;
            }
            float* mheat = static_cast<float*>(lh.heat.p);
            // a buffer that held another grid is decoded in full: its address alone cannot tell
            // the localized decode that its contents changed
            if (same)
                call(vsaogm_decode_incremental(m, &r.grid, r.precision, mheat, hmax, s.stream));
            else
                call(vsaogm_decode(m, &r.grid, r.precision, mheat, hmax, s.stream));
            if (r.heat)
                check_hip(hipMemcpyAsync(heat, mheat, cells * 8, hipMemcpyDeviceToDevice, s.stream), "copy heat");
            heat = mheat;
        } else {
            call(vsaogm_decode(m, &r.grid, r.precision, heat, hmax, s.stream));
        }
        call(vsaogm_classify(&r.grid, heat, hmax, r.r_occ, r.r_emp, r.rho,
                             reinterpret_cast<float*>(dout + L.ogm), dout + L.lab, device, s.stream));
        check_hip(hipMemcpyAsync(s.h_out.p, dout, back, hipMemcpyDeviceToHost, s.stream), "copy outputs");
    } catch (const Fail& e) {
        rc = e.code;
    } catch (const std::exception&) {
        rc = VSAOGM_EDEVICE;
    }
    q->res.status = rc;
    if (hipEventRecord(s.done, s.stream) != hipSuccess && q->res.status == VSAOGM_OK)
        q->res.status = VSAOGM_EDEVICE;
}

void vsaogm_server::finish(Slot& s) {
    Request* q = s.req;
    const vsaogm_request& r = q->r;
    if (q->res.status == VSAOGM_OK) {
        const int64_t cells = (int64_t)r.grid.nx * r.grid.ny;
        const OutLayout L(cells);
        const unsigned char* h = static_cast<const unsigned char*>(s.h_out.p);
        std::memcpy(q->res.hmax, h, 8);
        if (r.label_out) std::memcpy(r.label_out, h + L.lab, cells);
        if (r.ogm) std::memcpy(r.ogm, h + L.ogm, cells * 4);
        if (r.heat) std::memcpy(r.heat, h + L.heat, cells * 8);
    }
    if (q->in) pool.put(q->in, q->in_cap);
    q->in = nullptr;
    q->res.t_done_ns = now_ns();
}

void vsaogm_server::run(int w) {
    (void)hipSetDevice(device);
    std::vector<int> free_slots;
    for (int i = (int)slots.size() - 1; i >= 0; --i)
        if (i % nworkers == w) free_slots.push_back(i);
    for (;;) {
        bool progressed = false;
        // completions of this worker's slots
        for (int i = w; i < (int)slots.size(); i += nworkers) {
            Slot& s = slots[i];
            if (!s.req) continue;
            const hipError_t e = hipEventQuery(s.done);
            if (e == hipErrorNotReady) continue;
            if (e != hipSuccess && s.req->res.status == VSAOGM_OK) s.req->res.status = VSAOGM_EDEVICE;
            finish(s);
            {
                std::lock_guard<std::mutex> lk(mu);
                used -= s.req->footprint;
                map_busy[s.req->r.map_id] = 0;
                s.req->done = true;
                ++completed;
                --inflight;
            }
            cv_done.notify_all();
            cv_work.notify_all();  // a map or budget freed up for the other workers
            s.req = nullptr;
            free_slots.push_back(i);
            progressed = true;
        }
        // admissions, first come first served: a request whose map is busy waits (and so do
        // later requests of that map); a request that does not fit the budget stops admission
        std::vector<std::pair<int, Request*>> to_launch;
        {
            std::unique_lock<std::mutex> lk(mu);
            if (stop && pending.empty() && inflight == 0) break;
            std::unordered_set<int32_t> blocked;
            for (auto it = pending.begin(); it != pending.end() && !free_slots.empty();) {
                Request* q = *it;
                const int32_t mid = q->r.map_id;
                if (map_busy[mid] || blocked.count(mid)) {
                    blocked.insert(mid);
                    ++it;
                    continue;
                }
                if (used + q->footprint > budget) break;
                used += q->footprint;
                peak = std::max(peak, used);
                map_busy[mid] = 1;
                ++inflight;
                const int si = free_slots.back();
                free_slots.pop_back();
                slots[si].req = q;
                to_launch.emplace_back(si, q);
                it = pending.erase(it);
            }
            if (to_launch.empty() && !progressed) {
                // nothing to do right now: sleep until a submit or a completion, or a short
                // timeout while this worker's slots run (they are polled every 20 us)
                bool mine = false;
                for (int i = w; i < (int)slots.size(); i += nworkers) mine = mine || slots[i].req;
                cv_work.wait_for(lk, std::chrono::microseconds(mine ? 20 : 2000));
                continue;
            }
        }
        for (auto& [si, q] : to_launch) launch(slots[si], si);
    }
}

extern "C" {

int vsaogm_server_create(const vsaogm_server_desc* d, vsaogm_server** out) {
    return guard([&] {
        if (!d || !out) throw Fail(VSAOGM_EINVAL, "desc and out must not be NULL");
        *out = nullptr;
        if (d->max_inflight < 1 || d->max_inflight > 32) throw Fail(VSAOGM_EINVAL, "max_inflight must be 1..32");
        if (d->max_queue < 1) throw Fail(VSAOGM_EINVAL, "max_queue must be >= 1");
        int ndev = 0;
        check_hip(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
        if (d->device < 0 || d->device >= ndev) throw Fail(VSAOGM_EINVAL, "no such device");
        check_hip(hipSetDevice(d->device), "hipSetDevice");
        auto s = std::make_unique<vsaogm_server>();
        s->device = d->device;
        s->max_inflight = d->max_inflight;
        s->max_queue = d->max_queue;
        s->budget = d->hbm_budget_bytes;
        if (s->budget <= 0) {
            size_t free_b = 0, total_b = 0;
            check_hip(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
            s->budget = (int64_t)(free_b / 4);
        }
        s->slots.resize(d->max_inflight);
        for (auto& sl : s->slots) {
            check_hip(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking), "create stream");
            check_hip(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming), "create event");
        }
        vsaogm_server* raw = s.get();
        raw->nworkers = std::min(d->max_inflight, 4);
        for (int w = 0; w < raw->nworkers; ++w) raw->workers.emplace_back([raw, w] { raw->run(w); });
        *out = s.release();
    });
}

int vsaogm_server_destroy(vsaogm_server* s) {
    if (!s) return VSAOGM_OK;
    return guard([&] {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
        }
        s->cv_work.notify_all();
        for (auto& t : s->workers)
            if (t.joinable()) t.join();
        (void)hipSetDevice(s->device);
        for (auto& sl : s->slots) {
            if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        }
        for (auto* m : s->maps) vsaogm_map_destroy(m);
        for (auto& sl : s->slots) {
            if (sl.done) (void)hipEventDestroy(sl.done);
            if (sl.stream) (void)hipStreamDestroy(sl.stream);
        }
        delete s;
    });
}

int vsaogm_server_add_map(vsaogm_server* s, const vsaogm_map_desc* d, int32_t* map_id) {
    return guard([&] {
        if (!s || !d || !map_id) throw Fail(VSAOGM_EINVAL, "server, desc and map_id must not be NULL");
        vsaogm_map_desc dd = *d;
        dd.device = s->device;
        vsaogm_map* m = nullptr;
        const int rc = vsaogm_map_create(&dd, &m);
        if (rc != VSAOGM_OK) throw Fail(rc, vsaogm_last_error());
        std::lock_guard<std::mutex> lk(s->mu);
        s->maps.push_back(m);
        s->map_dim.push_back(dd.dim);
        s->map_keys.push_back(2 * (int64_t)dd.tiles_x * dd.tiles_y);
        s->map_busy.push_back(0);
        s->local_heat.push_back(std::make_unique<vsaogm_server::LocalHeat>());
        *map_id = (int32_t)s->maps.size() - 1;
    });
}

int vsaogm_server_get_map(vsaogm_server* s, int32_t map_id, vsaogm_map** out) {
    return guard([&] {
        if (!s || !out) throw Fail(VSAOGM_EINVAL, "server and out must not be NULL");
        std::lock_guard<std::mutex> lk(s->mu);
        if (map_id < 0 || map_id >= (int32_t)s->maps.size()) throw Fail(VSAOGM_ENOTFOUND, "unknown map");
        *out = s->maps[map_id];
    });
}

}  // extern "C"

namespace {

// Validate one request and stage its inputs in pinned memory (no server lock held).
std::unique_ptr<Request> prepare(vsaogm_server* s, const vsaogm_request* r) {
    if (!r) throw Fail(VSAOGM_EINVAL, "request must not be NULL");
    if (r->n < 0) throw Fail(VSAOGM_EINVAL, "n must be >= 0");
    if (r->n > 0 && (!r->xy || !r->label)) throw Fail(VSAOGM_EINVAL, "xy and label must not be NULL");
    if (r->grid.nx < 1 || r->grid.ny < 1 || !(r->grid.res > 0)) throw Fail(VSAOGM_EINVAL, "invalid grid");
    if (r->precision < VSAOGM_FP32 || r->precision > VSAOGM_BF16X3) throw Fail(VSAOGM_EINVAL, "unknown precision");
    if (r->r_occ < 0 || r->r_emp < 0 || r->r_occ > 24 || r->r_emp > 24)
        throw Fail(VSAOGM_EINVAL, "disk radii must be in 0..24");
    auto q = std::make_unique<Request>();
    q->r = *r;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (r->map_id < 0 || r->map_id >= (int32_t)s->maps.size()) throw Fail(VSAOGM_ENOTFOUND, "unknown map");
        q->footprint = footprint_of(*r, s->map_dim[r->map_id], s->map_keys[r->map_id]);
    }
    if (q->footprint > s->budget) throw Fail(VSAOGM_EINVAL, "request exceeds the memory budget");
    if (r->n > 0) {
        auto blk = s->pool.get((size_t)r->n * 9);
        q->in = blk.first;
        q->in_cap = blk.second;
        std::memcpy(q->in, r->xy, (size_t)r->n * 8);
        std::memcpy(static_cast<unsigned char*>(q->in) + r->n * 8, r->label, (size_t)r->n);
    }
    q->r.xy = nullptr;
    q->r.label = nullptr;
    q->res.status = VSAOGM_EAGAIN;
    q->res.slot = -1;
    return q;
}

// Queue a prepared request (server lock held); false when the queue is full.
bool enqueue_locked(vsaogm_server* s, std::unique_ptr<Request>& q, uint64_t* ticket) {
    if ((int)s->pending.size() >= s->max_queue) return false;
    q->ticket = s->next_ticket++;
    q->res.t_submit_ns = now_ns();
    *ticket = q->ticket;
    s->pending.push_back(q.get());
    s->tickets.emplace(q->ticket, std::move(q));
    return true;
}

}  // namespace

extern "C" {

int vsaogm_submit(vsaogm_server* s, const vsaogm_request* r, uint64_t* ticket) {
    return guard([&] {
        if (!s || !r || !ticket) throw Fail(VSAOGM_EINVAL, "server, request and ticket must not be NULL");
        auto q = prepare(s, r);
        bool ok;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            ok = enqueue_locked(s, q, ticket);
        }
        if (!ok) {
            if (q->in) s->pool.put(q->in, q->in_cap);
            throw Fail(VSAOGM_EBUSY, "queue full");
        }
        s->cv_work.notify_all();
    });
}

int vsaogm_submit_many(vsaogm_server* s, const vsaogm_request* reqs, int32_t count, uint64_t* tickets,
                       int32_t* n_queued) {
    int32_t queued = 0;
    const int rc = guard([&] {
        if (!s || (!reqs && count > 0) || (!tickets && count > 0))
            throw Fail(VSAOGM_EINVAL, "server, requests and tickets must not be NULL");
        std::vector<std::unique_ptr<Request>> qs;
        qs.reserve(count > 0 ? count : 0);
        int err = VSAOGM_OK;
        std::string msg;
        for (int32_t i = 0; i < count; ++i) {
            try {
                qs.push_back(prepare(s, reqs + i));
            } catch (const Fail& e) {
                err = e.code;
                msg = e.what();
                break;
            }
        }
        {
            std::lock_guard<std::mutex> lk(s->mu);
            for (auto& q : qs) {
                if (!enqueue_locked(s, q, tickets + queued)) {
                    err = VSAOGM_EBUSY;
                    msg = "queue full";
                    break;
                }
                ++queued;
            }
        }
        for (auto& q : qs)
            if (q && q->in) s->pool.put(q->in, q->in_cap);  // the ones not queued
        if (queued) s->cv_work.notify_all();
        if (err != VSAOGM_OK) throw Fail(err, msg);
    });
    if (n_queued) *n_queued = queued;
    return rc;
}

static int poll_locked(vsaogm_server* s, uint64_t ticket, vsaogm_result* out) {
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) {
        vsaogm::set_last_error("unknown or retired ticket");
        return VSAOGM_ENOTFOUND;
    }
    if (!it->second->done) return VSAOGM_EAGAIN;
    if (out) *out = it->second->res;
    s->tickets.erase(it);
    return VSAOGM_OK;
}

int vsaogm_poll(vsaogm_server* s, uint64_t ticket, vsaogm_result* out) {
    if (!s) return VSAOGM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    return poll_locked(s, ticket, out);
}

int vsaogm_wait(vsaogm_server* s, uint64_t ticket, vsaogm_result* out) {
    if (!s) return VSAOGM_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        const int rc = poll_locked(s, ticket, out);
        if (rc != VSAOGM_EAGAIN) return rc;
        s->cv_done.wait(lk);
    }
}

int vsaogm_server_drain(vsaogm_server* s) {
    if (!s) return VSAOGM_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->pending.empty() && s->inflight == 0; });
    return VSAOGM_OK;
}

int vsaogm_server_stats(vsaogm_server* s, int64_t* completed, int64_t* peak_bytes, int64_t* budget_bytes) {
    if (!s) return VSAOGM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (completed) *completed = s->completed;
    if (peak_bytes) *peak_bytes = s->peak;
    if (budget_bytes) *budget_bytes = s->budget;
    return VSAOGM_OK;
}

int vsaogm_request_bytes(vsaogm_server* s, const vsaogm_request* r, int64_t* bytes) {
    if (!s || !r || !bytes) return VSAOGM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (r->map_id < 0 || r->map_id >= (int32_t)s->maps.size()) return VSAOGM_ENOTFOUND;
    *bytes = footprint_of(*r, s->map_dim[r->map_id], s->map_keys[r->map_id]);
    return VSAOGM_OK;
}

}  // extern "C"
