// Request server for map updates (vsaogm_server_* / vsaogm_submit / vsaogm_poll).
//
// The scheduling (tickets, per-map order, admission by device bytes and execution slots,
// batching) is the device-free core of server_core.h; this file is its HIP executor and the C
// ABI.  Each execution slot is a HIP stream with its own device and pinned staging buffers.  A
// batch of admitted requests of distinct maps runs as one launch per stage (run_update_batch):
// one host-to-device copy of all the batch's points (gathered from the pinned blocks submit
// staged them in), encode into each map (Algorithm 1), norm and decode of each request's grid
// (eqs. vector-normalization, loc-query), classification (Algorithm 2, eqs. softmax, psd,
// classification), one device-to-host copy of the outputs, closed by an event.  Requests with
// the fp32 contraction or with localized decoding run alone in a slot through the map API.
// Slots run concurrently, so batches overlap on the GPU; a map is in at most one batch at a time
// and its requests run in submission order.  A request's results do not depend on the other
// requests of its batch: every kernel works per request, and the similarity's work split
// (decode_units) depends on the request alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "internal.h"
#include "server_core.h"
#include "vsaogm.h"

namespace {

using vsaogm::CoreRequest;

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
        const size_t cap = round_up(need);
        check_hip(hipMallocAsync(&p, cap, s), what);
        bytes = cap;
    }
    // 2 MiB granules, so that a block exceeds what was asked for by less than one granule
    static size_t round_up(size_t need) { return (need + kGranule - 1) / kGranule * kGranule; }
    static constexpr size_t kGranule = size_t(1) << 21;
    // the block ensure(need) would hold (0 if the current one suffices)
    size_t growth(size_t need) const { return need <= bytes ? 0 : round_up(need); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    ~DevMem() { release(); }
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
        dev = nullptr;
        if (hipHostGetDevicePointer(&dev, p, 0) != hipSuccess) {
            (void)hipGetLastError();
            dev = nullptr;
        }
    }
    void* dev = nullptr;   // the block's device address (kernels write results into it), or null
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

// The heat a map keeps for VSAOGM_REQUEST_LOCAL requests (only its own running request uses it).
struct LocalHeat {
    DevMem heat;
    vsaogm_grid_desc grid{};
};

// What the executor needs of one request: its arguments, the map (captured under the server
// lock at submit), the staged inputs and the results handed back.
struct Payload {
    vsaogm_request r{};
    vsaogm_map* map = nullptr;
    LocalHeat* local = nullptr;
    void* in = nullptr;       // pinned [n][2] float32 points, then [n] labels
    size_t in_cap = 0;
    float hmax[2] = {0.f, 0.f};
    // outputs in pinned host memory: copied there from the device directly, not staged; their
    // device addresses (null where the runtime gives none: a copy call then)
    bool pin_ogm = false, pin_label = false, pin_heat = false;
    void* dev_ogm = nullptr;
    void* dev_label = nullptr;
    void* dev_heat = nullptr;
};

// The device address of pinned host memory, or null.
void* device_address(void* host) {
    void* d = nullptr;
    if (!host || hipHostGetDevicePointer(&d, host, 0) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return d;
}

// Results of a batch written into pinned host buffers by one launch: segment k copies bytes[k]
// from src[k] (device) to dst[k] (device address of pinned host memory), 16 KiB per block.
constexpr int kMaxOutSegs = 32;
constexpr size_t kOutChunk = 16384;
struct OutSegs {
    const unsigned char* src[kMaxOutSegs];
    unsigned char* dst[kMaxOutSegs];
    unsigned long long bytes[kMaxOutSegs];
    int n;
};

__global__ __launch_bounds__(256) void k_results_to_host(OutSegs sg) {
    const int k = blockIdx.y;
    if (k >= sg.n) return;
    const size_t nb = sg.bytes[k];
    const size_t c0 = (size_t)blockIdx.x * kOutChunk;
    if (c0 >= nb) return;
    const size_t c1 = c0 + kOutChunk < nb ? c0 + kOutChunk : nb;
    const unsigned char* src = sg.src[k];
    unsigned char* dst = sg.dst[k];
    if ((((uintptr_t)src | (uintptr_t)dst) & 15) == 0) {
        const size_t w0 = c0 / 16, w1 = c1 / 16;
        for (size_t w = w0 + threadIdx.x; w < w1; w += 256)
            reinterpret_cast<uint4*>(dst)[w] = reinterpret_cast<const uint4*>(src)[w];
        for (size_t b = w1 * 16 + threadIdx.x; b < c1; b += 256) dst[b] = src[b];
    } else {
        for (size_t b = c0 + threadIdx.x; b < c1; b += 256) dst[b] = src[b];
    }
}

// Host memory the device can copy into directly (allocated pinned, e.g. hipHostMalloc).
bool is_pinned_host(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();   // pageable memory may report an error: not pinned
        return false;
    }
    return a.type == hipMemoryTypeHost;
}

// Bytes a request holds while it runs: its inputs and outputs on the device plus the map's
// working buffers for its points (sorted coordinates, keys, partial spectra) and the similarity's
// partial sums.
int64_t footprint_of(const vsaogm_request& r, int32_t dim, int64_t nkeys) {
    const int64_t n = r.n, cells = (int64_t)r.grid.nx * r.grid.ny;
    const int64_t halfp = ((int64_t)dim / 2 + 63) / 64 * 64;
    const int64_t inputs = n * 9;
    const int64_t outputs = cells * 13 + 8;
    // work items hold at least 64 points, plus one partial item per memory
    const int64_t encode_ws = n * 20 + (n / 64 + 1 + nkeys) * halfp * 8;
    const int64_t decode_ws = (int64_t)256 * 2 * 2 * 256 * 64 * 4;  // split-tile partial sums (upper bound)
    // the slot's input and output blocks are rounded up to 2 MiB granules
    return inputs + outputs + encode_ws + decode_ws + 2 * ((int64_t)1 << 21);
}

size_t up256(size_t v) { return (v + 255) / 256 * 256; }

// Output block of one request run alone: maxima, labels, map, heatmaps, each 256-byte aligned;
// one copy brings back the prefix holding what the request asked for.
struct OutLayout {
    size_t lab, ogm, heat, end_lab, end_ogm, end_heat;
    explicit OutLayout(int64_t cells) {
        lab = 256;
        ogm = up256(lab + cells);
        heat = up256(ogm + cells * 4);
        end_lab = lab + cells;
        end_ogm = ogm + cells * 4;
        end_heat = heat + cells * 8;
    }
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    DevMem d_in, d_out;
    HostMem h_out;
    vsaogm::UpdateBatchWork* work = nullptr;
    // layout of the current batch's outputs (section-major: maxima, labels, maps, heatmaps)
    std::vector<size_t> o_hmax, o_lab, o_ogm, o_heat;
    size_t back = 0;
    bool single = false;
    int64_t counted = 0;   // device bytes of this slot counted in the executor's fixed bytes
};

class HipExecutor : public vsaogm::Executor {
public:
    // trim_maps: release what every map rebuilds on demand and report each one's bytes after
    HipExecutor(int device, int nslots, PinnedPool* pool, std::function<void(std::vector<int64_t>*)> trim_maps)
        : device_(device), pool_(pool), slots_(nslots), trim_maps_(std::move(trim_maps)) {}
    ~HipExecutor() override {
        (void)hipSetDevice(device_);
        for (auto& s : slots_) {
            if (s.stream) (void)hipStreamSynchronize(s.stream);
            if (s.work) vsaogm::update_batch_work_destroy(s.work);
            if (s.done) (void)hipEventDestroy(s.done);
            if (s.stream) (void)hipStreamDestroy(s.stream);
        }
    }
    void init() {
        for (auto& s : slots_) {
            check_hip(hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking), "create stream");
            check_hip(hipEventCreateWithFlags(&s.done, hipEventDisableTiming), "create event");
            s.work = vsaogm::update_batch_work_create();
        }
    }

    int launch(int si, const std::vector<CoreRequest*>& batch) override {
        thread_local int cur = -1;
        if (cur != device_) {
            (void)hipSetDevice(device_);
            cur = device_;
        }
        Slot& s = slots_[si];
        int rc = VSAOGM_OK;
        try {
            const Payload* f = static_cast<const Payload*>(batch.front()->payload);
            const bool single = batch.size() == 1 && ((f->r.flags & VSAOGM_REQUEST_LOCAL) || f->r.precision == VSAOGM_FP32);
            s.single = single;
            if (single) launch_single(s, *static_cast<Payload*>(batch.front()->payload));
            else launch_batch(s, batch);
        } catch (const Fail& e) {
            rc = e.code;
        } catch (const std::exception&) {
            rc = VSAOGM_EDEVICE;
        }
        // the event closes whatever was enqueued, so that completion waits for it
        if (hipEventRecord(s.done, s.stream) != hipSuccess && rc == VSAOGM_OK) rc = VSAOGM_EDEVICE;
        if (rc != VSAOGM_OK) (void)hipEventSynchronize(s.done);
        count_slot(s);
        return rc;
    }

    void admission(const CoreRequest* q, int64_t* resident_now, int64_t* growth) override {
        const Payload* p = static_cast<const Payload*>(q->payload);
        const vsaogm_request& r = p->r;
        const bool local = (r.flags & VSAOGM_REQUEST_LOCAL) != 0;
        *resident_now = map_bytes(*p);
        int64_t g = vsaogm::map_growth_bytes(p->map, &r.grid, r.precision, r.n, local);
        if (local) {
            const LocalHeat& lh = *p->local;
            const bool same = lh.heat.p && lh.grid.nx == r.grid.nx && lh.grid.ny == r.grid.ny;
            if (!same) g += (int64_t)lh.heat.growth((size_t)r.grid.nx * r.grid.ny * 8);
        }
        *growth = g;
    }

    int64_t fixed_bytes() override { return fixed_.load(); }

    void reclaim(std::vector<int64_t>* resident) override {
        (void)hipSetDevice(device_);
        for (auto& s : slots_) {
            (void)hipStreamSynchronize(s.stream);
            s.d_in.release();
            s.d_out.release();
            vsaogm::update_batch_work_trim(s.work);
            count_slot(s);
        }
        try {
            trim_maps_(resident);
        } catch (const std::exception&) {
            // a map that could not be trimmed keeps its bytes (entries stay -1: unchanged)
        }
    }

    int query(int si) override {
        const hipError_t e = hipEventQuery(slots_[si].done);
        if (e == hipErrorNotReady) return vsaogm::kCoreAgain;
        return e == hipSuccess ? VSAOGM_OK : VSAOGM_EDEVICE;
    }

    void complete(int si, const std::vector<CoreRequest*>& batch, int status) override {
        Slot& s = slots_[si];
        const unsigned char* h = static_cast<const unsigned char*>(s.h_out.p);
        for (size_t i = 0; i < batch.size(); ++i) {
            CoreRequest* q = batch[i];
            Payload* p = static_cast<Payload*>(q->payload);
            if (status == VSAOGM_OK) {
                const vsaogm_request& r = p->r;
                const int64_t cells = (int64_t)r.grid.nx * r.grid.ny;
                std::memcpy(p->hmax, h + s.o_hmax[i], 8);
                if (r.label_out && !p->pin_label) std::memcpy(r.label_out, h + s.o_lab[i], cells);
                if (r.ogm && !p->pin_ogm) std::memcpy(r.ogm, h + s.o_ogm[i], cells * 4);
                if (r.heat && !p->pin_heat) std::memcpy(r.heat, h + s.o_heat[i], cells * 8);
            }
            q->status = status;
            q->result[0] = p->hmax[0];
            q->result[1] = p->hmax[1];
            q->resident_after = map_bytes(*p);   // the map is still this batch's alone
            release(q);
        }
    }

    void release(CoreRequest* q) override {
        Payload* p = static_cast<Payload*>(q->payload);
        if (!p) return;
        if (p->in) pool_->put(p->in, p->in_cap);
        delete p;
        q->payload = nullptr;
    }

private:
    static int64_t map_bytes(const Payload& p) {
        return vsaogm::map_resident_bytes(p.map) + (int64_t)p.local->heat.bytes;
    }
    // device bytes a slot keeps between batches (its streams' buffers and batch workspace)
    void count_slot(Slot& s) {
        const int64_t b = (int64_t)s.d_in.bytes + (int64_t)s.d_out.bytes + vsaogm::update_batch_work_bytes(s.work);
        fixed_ += b - s.counted;
        s.counted = b;
    }

    void launch_single(Slot& s, Payload& p) {
        const vsaogm_request& r = p.r;
        const int64_t n = r.n, cells = (int64_t)r.grid.nx * r.grid.ny;
        const OutLayout L(cells);
        const bool st_heat = r.heat && !p.pin_heat, st_ogm = r.ogm && !p.pin_ogm, st_lab = r.label_out && !p.pin_label;
        s.back = st_heat ? L.end_heat : (st_ogm ? L.end_ogm : (st_lab ? L.end_lab : 8));
        s.o_hmax.assign(1, 0);
        s.o_lab.assign(1, L.lab);
        s.o_ogm.assign(1, L.ogm);
        s.o_heat.assign(1, L.heat);
        s.d_in.ensure(std::max<int64_t>(n, 1) * 9, s.stream, "slot inputs");
        s.d_out.ensure(L.end_heat, s.stream, "slot outputs");
        s.h_out.ensure(s.back, "slot pinned outputs");
        unsigned char* din = static_cast<unsigned char*>(s.d_in.p);
        unsigned char* dout = static_cast<unsigned char*>(s.d_out.p);
        if (n > 0) check_hip(hipMemcpyAsync(din, p.in, n * 9, hipMemcpyHostToDevice, s.stream), "copy inputs");
        vsaogm_map* m = p.map;
        auto call = [&](int code) {
            if (code != VSAOGM_OK) throw Fail(code, vsaogm_last_error());
        };
        float* hmax = reinterpret_cast<float*>(dout);
        float* heat = reinterpret_cast<float*>(dout + L.heat);
        call(vsaogm_encode(m, reinterpret_cast<float*>(din), din + n * 8, n, s.stream));
        if (r.flags & VSAOGM_REQUEST_LOCAL) {
            LocalHeat& lh = *p.local;
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
        // the map of values only when the caller asked for it
        call(vsaogm_classify(&r.grid, heat, hmax, r.r_occ, r.r_emp, r.rho,
                             r.ogm ? reinterpret_cast<float*>(dout + L.ogm) : nullptr, dout + L.lab, device_,
                             s.stream));
        check_hip(hipMemcpyAsync(s.h_out.p, dout, s.back, hipMemcpyDeviceToHost, s.stream), "copy outputs");
        // pinned outputs: one kernel writes them through their device addresses (copy calls
        // where the runtime gave none)
        OutSegs sg{};
        bool direct = true;
        size_t max_bytes = 0;
        auto add = [&](const unsigned char* src, void* dst, size_t bytes) {
            if (!dst) return false;
            sg.src[sg.n] = src;
            sg.dst[sg.n] = static_cast<unsigned char*>(dst);
            sg.bytes[sg.n] = bytes;
            ++sg.n;
            max_bytes = std::max(max_bytes, bytes);
            return true;
        };
        if (r.label_out && p.pin_label) direct = add(dout + L.lab, p.dev_label, (size_t)cells) && direct;
        if (r.ogm && p.pin_ogm) direct = add(dout + L.ogm, p.dev_ogm, (size_t)cells * 4) && direct;
        if (r.heat && p.pin_heat) direct = add(dout + L.heat, p.dev_heat, (size_t)cells * 8) && direct;
        if (!direct) {
            copy_pinned(s, p, dout + L.lab, dout + L.ogm, dout + L.heat, cells);
        } else if (sg.n > 0) {
            const dim3 grid((unsigned)((max_bytes + kOutChunk - 1) / kOutChunk), (unsigned)sg.n);
            hipLaunchKernelGGL(k_results_to_host, grid, dim3(256), 0, s.stream, sg);
            check_hip(hipGetLastError(), "results to host");
        }
    }

    // outputs the caller holds in pinned memory go there straight from the device
    void copy_pinned(Slot& s, const Payload& p, const unsigned char* lab, const unsigned char* ogm,
                     const unsigned char* heat, int64_t cells) {
        const vsaogm_request& r = p.r;
        if (r.label_out && p.pin_label)
            check_hip(hipMemcpyAsync(r.label_out, lab, (size_t)cells, hipMemcpyDeviceToHost, s.stream), "copy labels");
        if (r.ogm && p.pin_ogm)
            check_hip(hipMemcpyAsync(r.ogm, ogm, (size_t)cells * 4, hipMemcpyDeviceToHost, s.stream), "copy map");
        if (r.heat && p.pin_heat)
            check_hip(hipMemcpyAsync(r.heat, heat, (size_t)cells * 8, hipMemcpyDeviceToHost, s.stream), "copy heat");
    }

    void launch_batch(Slot& s, const std::vector<CoreRequest*>& batch) {
        const size_t count = batch.size();
        bool want_lab = false, want_ogm = false, want_heat = false;   // staged through h_out
        bool want_ogm_dev = false;                                     // the map computed at all
        size_t cells_total = 0;
        for (size_t i = 0; i < count; ++i) {
            const Payload* p = static_cast<const Payload*>(batch[i]->payload);
            want_lab = want_lab || (p->r.label_out && !p->pin_label);
            want_ogm = want_ogm || (p->r.ogm && !p->pin_ogm);
            want_heat = want_heat || (p->r.heat && !p->pin_heat);
            want_ogm_dev = want_ogm_dev || p->r.ogm;
            cells_total += (size_t)p->r.grid.nx * p->r.grid.ny;
        }
        // outputs, section-major so that one copy brings back what any request asked for
        s.o_hmax.resize(count);
        s.o_lab.resize(count);
        s.o_ogm.resize(count);
        s.o_heat.resize(count);
        size_t o = 0;
        for (size_t i = 0; i < count; ++i) s.o_hmax[i] = o, o += 16;
        o = up256(o);
        for (size_t i = 0; i < count; ++i) {
            const Payload* p = static_cast<const Payload*>(batch[i]->payload);
            s.o_lab[i] = o;
            o = up256(o + (size_t)p->r.grid.nx * p->r.grid.ny);
        }
        const size_t end_lab = o;
        for (size_t i = 0; i < count; ++i) {
            const Payload* p = static_cast<const Payload*>(batch[i]->payload);
            s.o_ogm[i] = o;
            o = up256(o + (size_t)p->r.grid.nx * p->r.grid.ny * 4);
        }
        const size_t end_ogm = o;
        for (size_t i = 0; i < count; ++i) {
            const Payload* p = static_cast<const Payload*>(batch[i]->payload);
            s.o_heat[i] = o;
            o = up256(o + (size_t)p->r.grid.nx * p->r.grid.ny * 8);
        }
        const size_t end_heat = o;
        (void)cells_total;
        s.back = want_heat ? end_heat : (want_ogm ? end_ogm : (want_lab ? end_lab : 16 * count));
        s.d_out.ensure(end_heat, s.stream, "batch outputs");
        s.h_out.ensure(s.back, "batch pinned outputs");
        unsigned char* dout = static_cast<unsigned char*>(s.d_out.p);
        std::vector<vsaogm::UpdateItem> items(count);
        int precision = VSAOGM_BF16X3;
        for (size_t i = 0; i < count; ++i) {
            const Payload* p = static_cast<const Payload*>(batch[i]->payload);
            const vsaogm_request& r = p->r;
            // the request's pinned block travels with the batch's descriptors (it goes back to
            // the pool only after the slot's work ended)
            vsaogm::UpdateItem& it = items[i];
            it.map = p->map;
            it.xy = nullptr;
            it.label = nullptr;
            it.host_in = r.n > 0 ? p->in : nullptr;
            it.n = r.n;
            it.grid = r.grid;
            it.r_occ = r.r_occ;
            it.r_emp = r.r_emp;
            it.rho = r.rho;
            it.heat = reinterpret_cast<float*>(dout + s.o_heat[i]);
            it.hmax = reinterpret_cast<float*>(dout + s.o_hmax[i]);
            it.ogm = want_ogm_dev ? reinterpret_cast<float*>(dout + s.o_ogm[i]) : nullptr;
            it.label_out = dout + s.o_lab[i];
            precision = r.precision;
        }
        const int rc = vsaogm::run_update_batch(items.data(), (int)count, precision, s.stream, s.work);
        if (rc != VSAOGM_OK) throw Fail(rc, vsaogm_last_error());
        // results: what is staged comes back with one copy; pinned outputs (and the maxima, when
        // nothing is staged) are written by one kernel where the runtime gave device addresses
        OutSegs sg{};
        size_t max_bytes = 0;
        bool direct = true;
        auto add = [&](const unsigned char* src, void* dst, size_t n) {
            if (!dst || sg.n >= kMaxOutSegs) return false;
            sg.src[sg.n] = src;
            sg.dst[sg.n] = static_cast<unsigned char*>(dst);
            sg.bytes[sg.n] = n;
            ++sg.n;
            max_bytes = std::max(max_bytes, n);
            return true;
        };
        const bool staged = want_lab || want_ogm || want_heat;
        if (staged) check_hip(hipMemcpyAsync(s.h_out.p, dout, s.back, hipMemcpyDeviceToHost, s.stream), "copy outputs");
        else direct = add(dout, s.h_out.dev, 16 * count);
        for (size_t i = 0; i < count && direct; ++i) {
            const Payload* p = static_cast<const Payload*>(batch[i]->payload);
            const vsaogm_request& r = p->r;
            const size_t cells = (size_t)r.grid.nx * r.grid.ny;
            if (r.label_out && p->pin_label) direct = direct && add(dout + s.o_lab[i], p->dev_label, cells);
            if (r.ogm && p->pin_ogm) direct = direct && add(dout + s.o_ogm[i], p->dev_ogm, cells * 4);
            if (r.heat && p->pin_heat) direct = direct && add(dout + s.o_heat[i], p->dev_heat, cells * 8);
        }
        if (direct) {
            if (sg.n > 0) {
                const dim3 grid((unsigned)((max_bytes + kOutChunk - 1) / kOutChunk), (unsigned)sg.n);
                hipLaunchKernelGGL(k_results_to_host, grid, dim3(256), 0, s.stream, sg);
                check_hip(hipGetLastError(), "results to host");
            }
        } else {
            // a buffer without a device address, or too many: copy calls
            if (!staged) check_hip(hipMemcpyAsync(s.h_out.p, dout, 16 * count, hipMemcpyDeviceToHost, s.stream),
                                   "copy maxima");
            for (size_t i = 0; i < count; ++i) {
                const Payload* p = static_cast<const Payload*>(batch[i]->payload);
                copy_pinned(s, *p, dout + s.o_lab[i], dout + s.o_ogm[i], dout + s.o_heat[i],
                            (int64_t)p->r.grid.nx * p->r.grid.ny);
            }
        }
    }

    int device_;
    PinnedPool* pool_;
    std::vector<Slot> slots_;
    std::function<void(std::vector<int64_t>*)> trim_maps_;
    std::atomic<int64_t> fixed_{0};
};

}  // namespace

struct vsaogm_server {
    int device = 0;
    int64_t budget = 0;
    std::mutex mu;                          // guards the map tables below
    std::vector<vsaogm_map*> maps;
    std::vector<int32_t> map_dim;
    std::vector<int64_t> map_keys;
    std::vector<std::unique_ptr<LocalHeat>> local_heat;
    PinnedPool pool;
    std::unique_ptr<HipExecutor> exec;
    std::unique_ptr<vsaogm::Scheduler> sched;
};

namespace {

// Requests one batch takes when the descriptor does not say (distinct maps, one precision):
// pairs measured best on the serving stream (batches of 1, 2, 3, 4, 8 over 4-16 slots).
constexpr int kMaxDefaultBatch = 2;

// Validate one request and stage its inputs in pinned memory.
std::unique_ptr<CoreRequest> prepare(vsaogm_server* s, const vsaogm_request* r) {
    if (!r) throw Fail(VSAOGM_EINVAL, "request must not be NULL");
    if (r->n < 0) throw Fail(VSAOGM_EINVAL, "n must be >= 0");
    if (r->n > 0 && (!r->xy || !r->label)) throw Fail(VSAOGM_EINVAL, "xy and label must not be NULL");
    if (r->grid.nx < 1 || r->grid.ny < 1 || !(r->grid.res > 0)) throw Fail(VSAOGM_EINVAL, "invalid grid");
    if (r->precision < VSAOGM_FP32 || r->precision > VSAOGM_BF16X3) throw Fail(VSAOGM_EINVAL, "unknown precision");
    if (r->r_occ < 0 || r->r_emp < 0 || r->r_occ > 24 || r->r_emp > 24)
        throw Fail(VSAOGM_EINVAL, "disk radii must be in 0..24");
    auto p = std::make_unique<Payload>();
    p->r = *r;
    p->pin_label = is_pinned_host(r->label_out);
    p->pin_ogm = is_pinned_host(r->ogm);
    p->pin_heat = is_pinned_host(r->heat);
    if (p->pin_label) p->dev_label = device_address(r->label_out);
    if (p->pin_ogm) p->dev_ogm = device_address(r->ogm);
    if (p->pin_heat) p->dev_heat = device_address(r->heat);
    auto q = std::make_unique<CoreRequest>();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (r->map_id < 0 || r->map_id >= (int32_t)s->maps.size()) throw Fail(VSAOGM_ENOTFOUND, "unknown map");
        p->map = s->maps[r->map_id];
        p->local = s->local_heat[r->map_id].get();
        q->bytes = footprint_of(*r, s->map_dim[r->map_id], s->map_keys[r->map_id]);
    }
    if (q->bytes > s->budget) throw Fail(VSAOGM_EINVAL, "request exceeds the memory budget");
    q->map = r->map_id;
    q->precision = r->precision;
    q->batchable = r->precision != VSAOGM_FP32 && !(r->flags & VSAOGM_REQUEST_LOCAL);
    if (r->n > 0) {
        auto blk = s->pool.get((size_t)r->n * 9);
        p->in = blk.first;
        p->in_cap = blk.second;
        std::memcpy(p->in, r->xy, (size_t)r->n * 8);
        std::memcpy(static_cast<unsigned char*>(p->in) + r->n * 8, r->label, (size_t)r->n);
    }
    p->r.xy = nullptr;
    p->r.label = nullptr;
    q->payload = p.release();
    return q;
}

void drop(vsaogm_server* s, std::unique_ptr<CoreRequest>& q) {
    if (q && q->payload) s->exec->release(q.get());
}

vsaogm_result to_result(const CoreRequest& q) {
    vsaogm_result r{};
    r.status = q.status;
    r.slot = q.slot;
    r.t_submit_ns = q.t_submit_ns;
    r.t_start_ns = q.t_start_ns;
    r.t_done_ns = q.t_done_ns;
    r.hmax[0] = q.result[0];
    r.hmax[1] = q.result[1];
    return r;
}

}  // namespace

extern "C" {

int vsaogm_server_create(const vsaogm_server_desc* d, vsaogm_server** out) {
    return guard([&] {
        if (!d || !out) throw Fail(VSAOGM_EINVAL, "desc and out must not be NULL");
        *out = nullptr;
        if (d->max_inflight < 1 || d->max_inflight > 32) throw Fail(VSAOGM_EINVAL, "max_inflight must be 1..32");
        if (d->max_queue < 1) throw Fail(VSAOGM_EINVAL, "max_queue must be >= 1");
        if (d->max_batch > 64) throw Fail(VSAOGM_EINVAL, "max_batch must be <= 64");
        int ndev = 0;
        check_hip(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
        if (d->device < 0 || d->device >= ndev) throw Fail(VSAOGM_EINVAL, "no such device");
        check_hip(hipSetDevice(d->device), "hipSetDevice");
        auto s = std::make_unique<vsaogm_server>();
        s->device = d->device;
        s->budget = d->hbm_budget_bytes;
        if (s->budget <= 0) {
            size_t free_b = 0, total_b = 0;
            check_hip(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
            s->budget = (int64_t)(free_b / 4);
        }
        vsaogm_server* sp = s.get();
        s->exec = std::make_unique<HipExecutor>(d->device, d->max_inflight, &s->pool, [sp](std::vector<int64_t>* res) {
            // nothing is in flight: trim every map (the local heat buffers are rebuilt too)
            std::lock_guard<std::mutex> lk(sp->mu);
            for (size_t m = 0; m < sp->maps.size(); ++m) {
                vsaogm::map_trim(sp->maps[m]);
                sp->local_heat[m]->heat.release();
                sp->local_heat[m]->grid = vsaogm_grid_desc{};
                if (m < res->size()) (*res)[m] = vsaogm::map_resident_bytes(sp->maps[m]);
            }
        });
        s->exec->init();
        vsaogm::SchedulerConfig cfg;
        cfg.slots = d->max_inflight;
        cfg.max_queue = d->max_queue;
        cfg.max_batch = d->max_batch > 0 ? d->max_batch : kMaxDefaultBatch;
        cfg.workers = std::min(d->max_inflight, 4);
        cfg.budget = s->budget;
        s->sched = std::make_unique<vsaogm::Scheduler>(cfg, s->exec.get());
        s->sched->start();
        *out = s.release();
    });
}

int vsaogm_server_destroy(vsaogm_server* s) {
    if (!s) return VSAOGM_OK;
    return guard([&] {
        s->sched->stop();
        s->sched.reset();
        (void)hipSetDevice(s->device);
        s->exec.reset();
        for (auto* m : s->maps) vsaogm_map_destroy(m);
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
        s->local_heat.push_back(std::make_unique<LocalHeat>());
        const int id = s->sched->add_map(vsaogm::map_resident_bytes(m));
        if (id < 0) {
            s->maps.pop_back();
            s->map_dim.pop_back();
            s->map_keys.pop_back();
            s->local_heat.pop_back();
            vsaogm_map_destroy(m);
            throw Fail(VSAOGM_ENOMEM, "the map's memories do not fit the server's memory budget");
        }
        *map_id = (int32_t)s->maps.size() - 1;
        if (id != *map_id) throw Fail(VSAOGM_EDEVICE, "map tables out of step");
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
        auto q = prepare(s, r);
        const int rc = s->sched->submit(q, ticket);
        if (rc != VSAOGM_OK) {
            drop(s, q);
            throw Fail(rc, rc == VSAOGM_EBUSY ? "queue full" : "request refused");
        }
    });
}

int vsaogm_submit_many(vsaogm_server* s, const vsaogm_request* reqs, int32_t count, uint64_t* tickets,
                       int32_t* n_queued) {
    int queued = 0;
    const int rc = guard([&] {
        if (!s || (!reqs && count > 0) || (!tickets && count > 0))
            throw Fail(VSAOGM_EINVAL, "server, requests and tickets must not be NULL");
        // each request is queued as soon as it is staged, so that the workers start on the first
        // ones while the later ones are copied
        for (int32_t i = 0; i < count; ++i) {
            std::unique_ptr<CoreRequest> q = prepare(s, reqs + i);
            const int rc2 = s->sched->submit(q, tickets + i);
            if (rc2 != VSAOGM_OK) {
                drop(s, q);   // not queued: still ours
                throw Fail(rc2, rc2 == VSAOGM_EBUSY ? "queue full" : "request refused");
            }
            ++queued;
        }
    });
    if (n_queued) *n_queued = queued;
    return rc;
}

int vsaogm_poll(vsaogm_server* s, uint64_t ticket, vsaogm_result* out) {
    if (!s) return VSAOGM_EINVAL;
    CoreRequest q;
    const int rc = s->sched->poll(ticket, &q);
    if (rc == VSAOGM_OK && out) *out = to_result(q);
    if (rc == VSAOGM_ENOTFOUND) vsaogm::set_last_error("unknown or retired ticket");
    return rc;
}

int vsaogm_wait(vsaogm_server* s, uint64_t ticket, vsaogm_result* out) {
    if (!s) return VSAOGM_EINVAL;
    CoreRequest q;
    const int rc = s->sched->wait(ticket, &q);
    if (rc == VSAOGM_OK && out) *out = to_result(q);
    if (rc == VSAOGM_ENOTFOUND) vsaogm::set_last_error("unknown or retired ticket");
    return rc;
}

int vsaogm_server_drain(vsaogm_server* s) {
    if (!s) return VSAOGM_EINVAL;
    s->sched->drain();
    return VSAOGM_OK;
}

int vsaogm_server_stats(vsaogm_server* s, int64_t* completed, int64_t* peak_bytes, int64_t* budget_bytes) {
    if (!s) return VSAOGM_EINVAL;
    s->sched->stats(completed, peak_bytes, budget_bytes, nullptr);
    return VSAOGM_OK;
}

int vsaogm_server_memory(vsaogm_server* s, int64_t* in_flight, int64_t* resident, int64_t* fixed,
                         int64_t* reclaims) {
    if (!s) return VSAOGM_EINVAL;
    s->sched->memory(in_flight, resident, fixed, reclaims);
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
