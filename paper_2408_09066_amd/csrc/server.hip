// Request server for map updates (vsaogm_server_* / vsaogm_submit / vsaogm_poll).
//
// One worker thread owns the device side.  Each execution slot is a HIP stream with its own
// device and pinned host buffers; a request admitted to a slot runs its whole update there:
// host-to-device copy of the points, encode into its map (Algorithm 1), decode of its grid
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

struct Request {
    uint64_t ticket = 0;
    vsaogm_request r{};
    std::vector<float> xy;
    std::vector<uint8_t> label;
    int64_t footprint = 0;
    vsaogm_result res{};
    bool done = false;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    Request* req = nullptr;
    DevMem d_xy, d_label, d_heat, d_hmax, d_ogm, d_lab;
    HostMem h_xy, h_label, h_heat, h_hmax, h_ogm, h_lab;
};

// Bytes a request holds while it runs: its inputs and outputs on the device plus the map's
// working buffers for its points (sorted coordinates, keys, partial spectra) and grid.
int64_t footprint_of(const vsaogm_request& r, int32_t dim) {
    const int64_t n = r.n, cells = (int64_t)r.grid.nx * r.grid.ny;
    const int64_t halfp = ((int64_t)dim / 2 + 63) / 64 * 64;
    const int64_t inputs = n * 9;
    const int64_t outputs = cells * 13 + 8;
    const int64_t encode_ws = n * 20 + (n / 64 + 1024) * halfp * 8;
    const int64_t decode_ws = 512 * 2 * 2 * 112 * 64 * 4;  // stream-K partial sums (upper bound)
    return inputs + outputs + encode_ws + decode_ws;
}

}  // namespace

struct vsaogm_server {
    int device = 0;
    int64_t budget = 0, used = 0, peak = 0;
    int max_inflight = 4, max_queue = 1024;
    std::vector<vsaogm_map*> maps;
    std::vector<int32_t> map_dim;
    std::vector<char> map_busy;
    std::deque<Request*> pending;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> tickets;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stop = false;
    uint64_t next_ticket = 1;
    int64_t completed = 0;
    int inflight = 0;

    void run();
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
        s.d_xy.ensure(std::max<int64_t>(n, 1) * 8, s.stream, "slot points");
        s.d_label.ensure(std::max<int64_t>(n, 1), s.stream, "slot labels");
        s.d_heat.ensure(cells * 8, s.stream, "slot heatmaps");
        s.d_hmax.ensure(8, s.stream, "slot maxima");
        s.d_ogm.ensure(cells * 4, s.stream, "slot map");
        s.d_lab.ensure(cells, s.stream, "slot labels");
        s.h_xy.ensure(std::max<int64_t>(n, 1) * 8, "slot pinned points");
        s.h_label.ensure(std::max<int64_t>(n, 1), "slot pinned labels");
        s.h_hmax.ensure(8, "slot pinned maxima");
        if (r.heat) s.h_heat.ensure(cells * 8, "slot pinned heatmaps");
        if (r.ogm) s.h_ogm.ensure(cells * 4, "slot pinned map");
        if (r.label_out) s.h_lab.ensure(cells, "slot pinned labels");
        if (n > 0) {
            std::memcpy(s.h_xy.p, q->xy.data(), n * 8);
            std::memcpy(s.h_label.p, q->label.data(), n);
            check_hip(hipMemcpyAsync(s.d_xy.p, s.h_xy.p, n * 8, hipMemcpyHostToDevice, s.stream), "copy points");
            check_hip(hipMemcpyAsync(s.d_label.p, s.h_label.p, n, hipMemcpyHostToDevice, s.stream), "copy labels");
        }
        vsaogm_map* m = maps[r.map_id];
        auto call = [&](int code) {
            if (code != VSAOGM_OK) throw Fail(code, vsaogm_last_error());
        };
        call(vsaogm_encode(m, static_cast<float*>(s.d_xy.p), static_cast<uint8_t*>(s.d_label.p), n, s.stream));
        call(vsaogm_decode(m, &r.grid, r.precision, static_cast<float*>(s.d_heat.p),
                           static_cast<float*>(s.d_hmax.p), s.stream));
        call(vsaogm_classify(&r.grid, static_cast<float*>(s.d_heat.p), static_cast<float*>(s.d_hmax.p), r.r_occ,
                             r.r_emp, r.rho, static_cast<float*>(s.d_ogm.p), static_cast<uint8_t*>(s.d_lab.p),
                             device, s.stream));
        check_hip(hipMemcpyAsync(s.h_hmax.p, s.d_hmax.p, 8, hipMemcpyDeviceToHost, s.stream), "copy maxima");
        if (r.heat)
            check_hip(hipMemcpyAsync(s.h_heat.p, s.d_heat.p, cells * 8, hipMemcpyDeviceToHost, s.stream),
                      "copy heatmaps");
        if (r.ogm)
            check_hip(hipMemcpyAsync(s.h_ogm.p, s.d_ogm.p, cells * 4, hipMemcpyDeviceToHost, s.stream), "copy map");
        if (r.label_out)
            check_hip(hipMemcpyAsync(s.h_lab.p, s.d_lab.p, cells, hipMemcpyDeviceToHost, s.stream), "copy labels");
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
        std::memcpy(q->res.hmax, s.h_hmax.p, 8);
        if (r.heat) std::memcpy(r.heat, s.h_heat.p, cells * 8);
        if (r.ogm) std::memcpy(r.ogm, s.h_ogm.p, cells * 4);
        if (r.label_out) std::memcpy(r.label_out, s.h_lab.p, cells);
    }
    q->res.t_done_ns = now_ns();
}

void vsaogm_server::run() {
    (void)hipSetDevice(device);
    std::vector<int> free_slots;
    for (int i = (int)slots.size() - 1; i >= 0; --i) free_slots.push_back(i);
    for (;;) {
        bool progressed = false;
        // completions
        for (int i = 0; i < (int)slots.size(); ++i) {
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
                // nothing to do right now: sleep until a submit or a short timeout (running
                // slots are polled every 20 microseconds)
                cv_work.wait_for(lk, std::chrono::microseconds(inflight > 0 ? 20 : 2000));
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
        raw->worker = std::thread([raw] { raw->run(); });
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
        if (s->worker.joinable()) s->worker.join();
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
        s->map_busy.push_back(0);
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

int vsaogm_submit(vsaogm_server* s, const vsaogm_request* r, uint64_t* ticket) {
    return guard([&] {
        if (!s || !r || !ticket) throw Fail(VSAOGM_EINVAL, "server, request and ticket must not be NULL");
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
            q->footprint = footprint_of(*r, s->map_dim[r->map_id]);
            if (q->footprint > s->budget) throw Fail(VSAOGM_EINVAL, "request exceeds the memory budget");
            if ((int)s->pending.size() >= s->max_queue) throw Fail(VSAOGM_EBUSY, "queue full");
        }
        if (r->n > 0) {
            q->xy.assign(r->xy, r->xy + 2 * r->n);
            q->label.assign(r->label, r->label + r->n);
        }
        q->r.xy = nullptr;
        q->r.label = nullptr;
        q->res.status = VSAOGM_EAGAIN;
        q->res.slot = -1;
        q->res.t_submit_ns = now_ns();
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if ((int)s->pending.size() >= s->max_queue) throw Fail(VSAOGM_EBUSY, "queue full");
            q->ticket = s->next_ticket++;
            *ticket = q->ticket;
            s->pending.push_back(q.get());
            s->tickets.emplace(q->ticket, std::move(q));
        }
        s->cv_work.notify_all();
    });
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

}  // extern "C"
