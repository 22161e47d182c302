// Host side of the C ABI (include/vsaogm.h): map objects, validation, buffer management and
// the order of launches.  Every entry point catches C++ exceptions and returns a status.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <tuple>
#include <vector>

#include "internal.h"
#include "vsaogm.h"

using namespace vsaogm;

namespace {

thread_local std::string g_last_error;

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] void fail(int code, const std::string& msg) { throw Error(code, msg); }

void hip_check(hipError_t e, const char* what) {
    if (e == hipSuccess) return;
    if (e == hipErrorOutOfMemory) fail(VSAOGM_ENOMEM, std::string(what) + ": out of device memory");
    fail(VSAOGM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

template <class F>
int guarded(F&& f) {
    try {
        g_last_error.clear();
        f();
        return VSAOGM_OK;
    } catch (const Error& e) {
        g_last_error = e.what();
        return e.code;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return VSAOGM_ENOMEM;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return VSAOGM_EDEVICE;
    } catch (...) {
        g_last_error = "unknown error";
        return VSAOGM_EDEVICE;
    }
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        hip_check(hipGetDevice(&prev), "hipGetDevice");
        if (prev != dev) hip_check(hipSetDevice(dev), "hipSetDevice");
    }
    ~DeviceGuard() {
        int cur = -1;
        if (hipGetDevice(&cur) == hipSuccess && cur != prev && prev >= 0) (void)hipSetDevice(prev);
    }
};

template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    void alloc(size_t count, const char* what) {
        release();
        void* q = nullptr;
        hip_check(hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)), what);
        p = static_cast<T*>(q);
        n = count;
    }
    // Stream-ordered replacement: the old block is released and the new one obtained in the
    // order of stream s, so growing a buffer never synchronises the device.
    void alloc_async(size_t count, hipStream_t s, const char* what) {
        if (p) hip_check(hipFreeAsync(p, s), what);
        p = nullptr;
        n = 0;
        void* q = nullptr;
        hip_check(hipMallocAsync(&q, std::max<size_t>(count, 1) * sizeof(T), s), what);
        p = static_cast<T*>(q);
        n = count;
    }
};

// Work units of the 16-bit GEMM over one tile list (decode_units): the host copy, and the device
// copy the kernels read.
struct UnitPlan {
    std::vector<DUnit> units;
    std::vector<int> tile_u0, wg_u0;   // [ntiles + 1], [workgroups + 1]
    void build(int ntiles, int ksteps, int num_cus) {
        units.clear();
        tile_u0.clear();
        wg_u0.clear();
        decode_units(ntiles, ksteps, num_cus, 0, 0, units, tile_u0, wg_u0);
        tile_u0.push_back((int)units.size());
        wg_u0.push_back((int)units.size());
    }
    int nwg() const { return (int)wg_u0.size() - 1; }
};
struct DevUnits {
    DevBuf<DUnit> units;
    DevBuf<int> tile_u0, wg_u0;
    void upload(const UnitPlan& h) {
        units.alloc(h.units.size(), "decode work units");
        tile_u0.alloc(h.tile_u0.size(), "decode tile units");
        wg_u0.alloc(h.wg_u0.size(), "decode workgroup units");
        hip_check(hipMemcpy(units.p, h.units.data(), h.units.size() * sizeof(DUnit), hipMemcpyHostToDevice),
                  "copy units");
        hip_check(hipMemcpy(tile_u0.p, h.tile_u0.data(), h.tile_u0.size() * sizeof(int), hipMemcpyHostToDevice),
                  "copy tile units");
        hip_check(hipMemcpy(wg_u0.p, h.wg_u0.data(), h.wg_u0.size() * sizeof(int), hipMemcpyHostToDevice),
                  "copy workgroup units");
    }
    // stream-ordered; h must stay unchanged until the stream has passed the copies
    void upload_async(const UnitPlan& h, hipStream_t s) {
        if (units.n < h.units.size()) units.alloc_async(h.units.size(), s, "decode work units");
        if (tile_u0.n < h.tile_u0.size()) tile_u0.alloc_async(h.tile_u0.size(), s, "decode tile units");
        if (wg_u0.n < h.wg_u0.size()) wg_u0.alloc_async(h.wg_u0.size(), s, "decode workgroup units");
        hip_check(hipMemcpyAsync(units.p, h.units.data(), h.units.size() * sizeof(DUnit), hipMemcpyHostToDevice, s),
                  "copy units");
        hip_check(hipMemcpyAsync(tile_u0.p, h.tile_u0.data(), h.tile_u0.size() * sizeof(int),
                                 hipMemcpyHostToDevice, s),
                  "copy tile units");
        hip_check(hipMemcpyAsync(wg_u0.p, h.wg_u0.data(), h.wg_u0.size() * sizeof(int), hipMemcpyHostToDevice, s),
                  "copy workgroup units");
    }
};
// The 16-bit GEMM's work units of a decode; returns the partial-sum floats it needs.
size_t set_units(DecodeLaunch& d, const UnitPlan& h, const DevUnits& dv, int ntiles) {
    d.units = dv.units.p;
    d.nunits = (int)h.units.size();
    d.tile_u0 = dv.tile_u0.p;
    d.wg_u0 = dv.wg_u0.p;
    d.nwg = h.nwg();
    d.any_split = d.nunits > ntiles;   // every tile has a unit, so some tile has several
    return d.any_split ? decode_unit_partial_floats(2 * d.nwg) : 0;   // blocks 2w, 2w + 1
}

__global__ void k_zero_words(unsigned* p, size_t n) {
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Reset of a map in one launch: zero the memories and bump every memory's version.
__global__ void k_reset_map(unsigned* words, size_t n, unsigned* version, int nkeys) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) words[i] = 0u;
    if (i < (size_t)nkeys) version[i] += 1u;
}

void zero_async(void* p, size_t bytes, hipStream_t s) {
    size_t words = bytes / 4;
    if (words == 0) return;
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s,
                       static_cast<unsigned*>(p), words);
    hip_check(hipGetLastError(), "zero kernel");
}

bool is_finite(double v) { return std::isfinite(v); }

struct GridKey {
    double x0, y0, res;
    int nx, ny;
    bool operator<(const GridKey& o) const {
        return std::tie(x0, y0, res, nx, ny) < std::tie(o.x0, o.y0, o.res, o.nx, o.ny);
    }
};

// Per-grid decode state: cell-to-tile split, local coordinates, work tiles, tables.
struct GridCache {
    int nx = 0, ny = 0;
    DevBuf<double> local_x, local_y;
    // work tiles of each tile set (decode_tile_set)
    DevBuf<DTile> tiles[kDecodeTileSets];
    int ntiles[kDecodeTileSets] = {};
    std::vector<DTile> host_tiles[kDecodeTileSets];
    // work units of the 16-bit GEMM per tile set
    UnitPlan uplan[kDecodeTileSets];
    DevUnits dunits[kDecodeTileSets];
    DevBuf<int> col_tx;              // [nx] tile column of every grid column
    DevBuf<float2> ex32, ey32;       // fp32 tables [n][halfp]
    DevBuf<uint16_t> ey_bf, ey_bf_lo, ey_h;  // 16-bit y tables (rows16(ny) x 2*halfp, operand order), built on first use
    // localized decoding state (planned on the device: IncPlan)
    std::vector<int> tcol;                   // tile column of every grid column
    std::vector<RegionBox> boxes;            // [tiles] cell range of every tile (row0 == row1: none)
    DevBuf<RegionBox> d_boxes;
    DevBuf<unsigned> d_seen;                 // memory versions at the last localized decode
    const float* inc_heat = nullptr;         // heat buffer of that decode
    int inc_precision = -1;                  // and its operand precision
    bool inc_valid = false;
    DevBuf<unsigned> region_max;             // [tiles][2] ordered maxima (order_key)
    DevBuf<DTile> inc_tiles;                 // changed tiles, regions and the GEMM's work units
    DevBuf<RegionBox> inc_boxes;             // (capacities for the whole tile list)
    DevBuf<DUnit> inc_units;
    DevBuf<int> inc_tile_u0, inc_wg_u0, inc_dyn;
};

struct ProfileSlot {
    hipEvent_t begin = nullptr, end = nullptr;
};
ProfileSlot g_profile[kNumStages];

}  // namespace

namespace vsaogm {
void set_last_error(const char* msg) { g_last_error = msg ? msg : ""; }

std::vector<DTile> build_decode_tiles(const std::vector<DBand>& bands, const std::vector<int>& tcol, int nx,
                                      int set) {
    // Work tiles: per band, its rows in blocks of 16 split evenly into groups of at most
    // kDecodeSetRowBlocks blocks, times the grid's columns in slices of up to 64.
    const int maxrb = kDecodeSetRowBlocks[set];
    // column slices (the same for every band): 64 columns; for 16-bit operands cut short where
    // a slice would reach a third tile column (its kernel stages two tiles' memories)
    std::vector<std::pair<int, int>> slices;
    for (int c = 0; c < nx;) {
        int end = std::min(c + 64, nx);
        if (set > 0 && tcol[end - 1] > tcol[c] + 1)
            end = (int)(std::lower_bound(tcol.begin(), tcol.end(), tcol[c] + 2) - tcol.begin());
        slices.emplace_back(c, end);
        c = end;
    }
    std::vector<DTile> groups;  // row groups, columns unset
    for (const DBand& bd : bands) {
        const int nblocks = (bd.row1 - bd.row0 + 15) / 16;
        const int ngroups = (nblocks + maxrb - 1) / maxrb;
        int b0 = 0;
        for (int gi = 0; gi < ngroups; ++gi) {
            const int nb = nblocks / ngroups + (gi < nblocks % ngroups ? 1 : 0);
            DTile d{};
            d.ty = bd.key_row;
            d.row0 = bd.row0 + 16 * b0;
            d.row_end = bd.row1;
            d.nrb = nb;
            d.pad = 0;
            groups.push_back(d);
            b0 += nb;
        }
    }
    // order: blocks of kBlockRows row groups x kBlockCols slices, so that the workgroups
    // resident on one XCD at a time work on tiles that share rows and columns
    constexpr int kBlockRows = 4, kBlockCols = 8;
    std::vector<DTile> tl;
    for (size_t gb = 0; gb < groups.size(); gb += kBlockRows)
        for (size_t sb = 0; sb < slices.size(); sb += kBlockCols)
            for (size_t gi = gb; gi < std::min(groups.size(), gb + kBlockRows); ++gi)
                for (size_t si = sb; si < std::min(slices.size(), sb + kBlockCols); ++si) {
                    DTile d = groups[gi];
                    d.col0 = slices[si].first;
                    d.ncol = slices[si].second - slices[si].first;
                    d.tx0 = tcol[d.col0];
                    tl.push_back(d);
                }
    return tl;
}
hipEvent_t profile_start(int stage) { return g_profile[stage].begin; }
hipEvent_t profile_stop(int stage) { return g_profile[stage].end; }
}  // namespace vsaogm

struct vsaogm_map {
    int device = 0;
    int D = 0, half = 0, halfp = 0;
    int tiles_x = 1, tiles_y = 1, nkeys = 2;
    double x0 = 0, y0 = 0, x1 = 0, y1 = 0;
    std::vector<double> theta;          // host copy [D][2]
    std::vector<double> cx, cy;         // tile centres
    float max_rev_x = 0.f, max_rev_y = 0.f;

    DevBuf<double> d_cx, d_cy;
    DevBuf<float2> d_rev;               // [halfp] Theta / (2 pi), fp32
    DevBuf<double> d_rev_d;             // [halfp][2] Theta / (2 pi), fp64
    DevBuf<double> d_theta;             // [half][2] Theta, rad/m
    DevBuf<float2> d_omega;             // [nkeys][halfp] local-frame memories
    DevBuf<float> d_scale;              // [nkeys] 1/||w||
    DevBuf<float2> d_omega_s;           // [nkeys][halfp] conj(Omega)/||w|| for the decode
    DevBuf<float> d_partial;            // stream-K partial sums of the decode
    int num_cus = 0;
    DevBuf<unsigned> d_hmax_u;          // [2] ordered class maxima
    DevBuf<unsigned long long> d_bad;   // [1]
    DevBuf<unsigned> d_version;         // [nkeys] change counters of the memories

    // encode workspace
    int64_t cap_n = 0;
    int cap_chunks = 0, cap_echunks = 0;
    DevBuf<int> w_key, w_hist, w_meta;
    DevBuf<float2> w_sorted, w_sorted_lo, w_partial;
    DevBuf<EChunk> w_table;

    std::map<GridKey, std::unique_ptr<GridCache>> grids;

    LayoutDev layout() const {
        LayoutDev L;
        L.x0 = x0;
        L.y0 = y0;
        L.inv_wx = (double)tiles_x / (x1 - x0);
        L.inv_wy = (double)tiles_y / (y1 - y0);
        L.tiles_x = tiles_x;
        L.tiles_y = tiles_y;
        L.cx = d_cx.p;
        L.cy = d_cy.p;
        return L;
    }
};

// A volume (3-D map) and its one cached grid.
struct Grid3Cache {
    vsaogm_grid3_desc key{};
    DevBuf<double> local_x, local_y, local_z;
    DevBuf<int> col_tx;
    DevBuf<DTile> tiles[kDecodeTileSets];
    int ntiles[kDecodeTileSets] = {};
    UnitPlan uplan[kDecodeTileSets];           // work units of the 16-bit GEMM
    DevUnits dunits[kDecodeTileSets];
    DevBuf<float2> ex32;                       // [nx][halfp]
    int nrows = 0;                             // joint (z, y) rows = nz * ny
    DevBuf<int> row_map;                       // [nrows] voxel plane offset slice * ny + y
    DevBuf<uint16_t> eyz_bf, eyz_bf_lo, eyz_h; // joint (z, y) tables, rows16(nrows) x 2 halfp, operand order
};

struct vsaogm_volume {
    int device = 0, D = 0, half = 0, halfp = 0, tiles_x = 1, tiles_y = 1, tiles_z = 1, nkeys = 0, num_cus = 1;
    double lay[6] = {};
    std::vector<double> cx, cy, cz;
    float max_rev[3] = {0.f, 0.f, 0.f};
    DevBuf<double> d_cx, d_cy, d_cz;
    DevBuf<float4> d_rev;                      // [halfp] revolutions per metre (x, y, z, 0)
    DevBuf<double> d_rev_d;                    // [halfp][3]
    DevBuf<double> d_theta_xy, d_theta_z;      // [half][2] rad/m: (x, y) and (z, 0) for the tables
    DevBuf<float2> d_omega, d_omega_s;         // [nkeys][halfp]
    DevBuf<float> d_scale;
    DevBuf<unsigned> d_hmax_u;
    DevBuf<unsigned long long> d_bad;
    DevBuf<int> w_key, w_hist, w_meta;
    DevBuf<float4> w_sorted, w_sorted_lo;
    DevBuf<EChunk> w_table;
    DevBuf<float2> w_partial;
    int64_t cap_n = 0;
    int cap_chunks = 0, cap_echunks = 0;
    DevBuf<float> d_partial;                   // split-tile partial sums of the decode
    std::unique_ptr<Grid3Cache> grid;
};

namespace {

#pragma clang fp contract(off)
// Tile centres exactly as written: x0 + (t + 0.5) * ((x1 - x0) / tiles), in double.
std::vector<double> centres(double a0, double a1, int tiles) {
    std::vector<double> c(tiles);
    const double w = (a1 - a0) / (double)tiles;
    for (int t = 0; t < tiles; ++t) c[t] = a0 + ((double)t + 0.5) * w;
    return c;
}

double sq_dist(double x, double y, double mx, double my) {
    const double dx = x - mx, dy = y - my;
    return dx * dx + dy * dy;
}
#pragma clang fp contract(on)

// Nearest centre along one axis (strict <, lowest index on ties).
int nearest_1d(const std::vector<double>& c, double v) {
    int best = 0;
    double bd = INFINITY;
    for (int t = 0; t < (int)c.size(); ++t) {
        const double d = (v - c[t]) * (v - c[t]);
        if (d < bd) {
            bd = d;
            best = t;
        }
    }
    return best;
}

void ensure_encode_workspace(vsaogm_map* m, int64_t n, hipStream_t s) {
    const EncodePlan p = encode_plan(n, m->halfp, m->nkeys);
    if (n <= m->cap_n && p.nchunks <= m->cap_chunks && p.max_echunks <= m->cap_echunks) return;
    const int64_t cap = std::max<int64_t>(n + n / 2, 4096);
    const EncodePlan q = encode_plan(cap, m->halfp, m->nkeys);
    const int chunks = std::max(q.nchunks, p.nchunks);
    const int echunks = std::max(q.max_echunks, p.max_echunks);
    m->w_key.alloc_async(cap, s, "encode keys");
    m->w_sorted.alloc_async(cap, s, "encode sorted");
    m->w_sorted_lo.alloc_async(cap, s, "encode sorted residuals");
    // the scan reads the histogram in aligned groups of kHistPad entries
    m->w_hist.alloc_async((size_t)chunks * m->nkeys + kHistPad, s, "encode histogram");
    m->w_table.alloc_async(echunks, s, "encode table");
    m->w_partial.alloc_async((size_t)echunks * m->halfp, s, "encode partial spectra");
    if (!m->w_meta.p) m->w_meta.alloc_async(1 + 3 * (size_t)m->nkeys, s, "encode meta");
    m->cap_n = cap;
    m->cap_chunks = chunks;
    m->cap_echunks = echunks;
}

GridCache* grid_cache(vsaogm_map* m, const vsaogm_grid_desc* g, hipStream_t s) {
    GridKey key{g->x0, g->y0, g->res, g->nx, g->ny};
    auto it = m->grids.find(key);
    if (it != m->grids.end()) return it->second.get();

    // Columns and rows of each tile: every cell belongs to the tile with the nearest
    // centre.  Along one axis the nearest centre is non-decreasing in the cell index, so
    // each tile owns a contiguous range of columns and of rows.
    std::vector<int> tcol(g->nx), trow(g->ny);
    std::vector<double> lx(g->nx), ly(g->ny);
    std::vector<char> near_tie_col(g->nx, 0), near_tie_row(g->ny, 0);
    auto axis = [&](int ncell, double o, const std::vector<double>& c, std::vector<int>& t,
                    std::vector<double>& loc, std::vector<char>& tie) {
        for (int i = 0; i < ncell; ++i) {
            const double v = o + ((double)i + 0.5) * g->res;
            t[i] = nearest_1d(c, v);
            loc[i] = v - c[t[i]];
            if (i > 0 && t[i] < t[i - 1]) fail(VSAOGM_EINVAL, "grid cells are not ordered along an axis");
            for (int u = 0; u < (int)c.size(); ++u) {
                if (u == t[i]) continue;
                const double d1 = (v - c[t[i]]) * (v - c[t[i]]), d2 = (v - c[u]) * (v - c[u]);
                if (std::fabs(d2 - d1) <= 1e-9 * (d1 + d2) + 1e-300) tie[i] = 1;
            }
        }
    };
    axis(g->nx, g->x0, m->cx, tcol, lx, near_tie_col);
    axis(g->ny, g->y0, m->cy, trow, ly, near_tie_row);
    // Where an axis is close to a tie, confirm that the two-dimensional argmin (the
    // definition) agrees with the per-axis split for every affected cell.
    for (int j = 0; j < g->ny; ++j)
        for (int i = 0; i < g->nx; ++i) {
            if (!near_tie_col[i] && !near_tie_row[j]) continue;
            const double x = g->x0 + ((double)i + 0.5) * g->res;
            const double y = g->y0 + ((double)j + 0.5) * g->res;
            int best = 0;
            double bd = INFINITY;
            for (int b = 0; b < m->tiles_x * m->tiles_y; ++b) {
                const double d = sq_dist(x, y, m->cx[b % m->tiles_x], m->cy[b / m->tiles_x]);
                if (d < bd) {
                    bd = d;
                    best = b;
                }
            }
            if (best != trow[j] * m->tiles_x + tcol[i])
                fail(VSAOGM_EINVAL, "a grid cell centre lies on a tile boundary in a way that "
                                    "does not split into per-tile rows and columns");
        }

    auto gc = std::make_unique<GridCache>();
    gc->nx = g->nx;
    gc->ny = g->ny;
    std::vector<DBand> bands;
    for (int ty = 0; ty < m->tiles_y; ++ty) {
        const int r0 = (int)(std::lower_bound(trow.begin(), trow.end(), ty) - trow.begin());
        const int r1 = (int)(std::upper_bound(trow.begin(), trow.end(), ty) - trow.begin());
        if (r0 < r1) bands.push_back(DBand{ty, r0, r1});
    }
    for (int set = 0; set < kDecodeTileSets; ++set) {
        gc->host_tiles[set] = build_decode_tiles(bands, tcol, g->nx, set);
        gc->ntiles[set] = (int)gc->host_tiles[set].size();
    }
    gc->tcol = tcol;
    gc->boxes.resize((size_t)m->tiles_x * m->tiles_y);
    for (int ty = 0; ty < m->tiles_y; ++ty)
        for (int tx = 0; tx < m->tiles_x; ++tx) {
            RegionBox b{};
            b.beta = ty * m->tiles_x + tx;
            b.row0 = (int)(std::lower_bound(trow.begin(), trow.end(), ty) - trow.begin());
            b.row1 = (int)(std::upper_bound(trow.begin(), trow.end(), ty) - trow.begin());
            b.col0 = (int)(std::lower_bound(tcol.begin(), tcol.end(), tx) - tcol.begin());
            b.col1 = (int)(std::upper_bound(tcol.begin(), tcol.end(), tx) - tcol.begin());
            if (b.row0 >= b.row1 || b.col0 >= b.col1) b.row0 = b.row1 = b.col0 = b.col1 = 0;
            gc->boxes[b.beta] = b;
        }
    for (int set = 1; set < kDecodeTileSets; ++set) {
        gc->uplan[set].build(gc->ntiles[set], m->halfp / 32, m->num_cus);
        gc->dunits[set].upload(gc->uplan[set]);
    }
    for (int set = 0; set < kDecodeTileSets; ++set)
        gc->tiles[set].alloc(gc->host_tiles[set].size(), "decode tile list");
    gc->col_tx.alloc(g->nx, "column tiles");
    gc->local_x.alloc(g->nx, "local x");
    gc->local_y.alloc(g->ny, "local y");
    gc->ex32.alloc((size_t)g->nx * m->halfp, "x location table");
    for (int set = 0; set < kDecodeTileSets; ++set)
        hip_check(hipMemcpy(gc->tiles[set].p, gc->host_tiles[set].data(),
                            gc->host_tiles[set].size() * sizeof(DTile), hipMemcpyHostToDevice),
                  "copy tile list");
    hip_check(hipMemcpy(gc->col_tx.p, tcol.data(), tcol.size() * sizeof(int), hipMemcpyHostToDevice),
              "copy column tiles");
    hip_check(hipMemcpy(gc->local_x.p, lx.data(), lx.size() * sizeof(double), hipMemcpyHostToDevice),
              "copy local x");
    hip_check(hipMemcpy(gc->local_y.p, ly.data(), ly.size() * sizeof(double), hipMemcpyHostToDevice),
              "copy local y");
    hip_check(launch_table_f32(m->d_theta.p, 0, gc->local_x.p, g->nx, m->half, m->halfp, gc->ex32.p, s),
              "x table");
    GridCache* raw = gc.get();
    m->grids.emplace(key, std::move(gc));
    return raw;
}

// The y table in the operand format of the requested precision (built on first use).
const void* y_table(vsaogm_map* m, GridCache* gc, int precision, const void** lo, hipStream_t s) {
    *lo = nullptr;
    const size_t n16 = (size_t)rows16(gc->ny) * 2 * m->halfp;
    switch (precision) {
        case VSAOGM_FP32:
            if (!gc->ey32.p) {
                gc->ey32.alloc((size_t)gc->ny * m->halfp, "y location table");
                hip_check(launch_table_f32(m->d_theta.p, 1, gc->local_y.p, gc->ny, m->half, m->halfp,
                                           gc->ey32.p, s), "y table");
            }
            return gc->ey32.p;
        case VSAOGM_FP16:
            if (!gc->ey_h.p) {
                gc->ey_h.alloc(n16, "y location table (fp16)");
                hip_check(launch_table_split(m->d_theta.p, 1, gc->local_y.p, gc->ny, m->half, m->halfp,
                                             true, gc->ey_h.p, nullptr, s), "y table");
            }
            return gc->ey_h.p;
        default:
            if (!gc->ey_bf.p || !gc->ey_bf_lo.p) {
                gc->ey_bf.alloc(n16, "y location table (bf16)");
                gc->ey_bf_lo.alloc(n16, "y location table (bf16 residual)");
                hip_check(launch_table_split(m->d_theta.p, 1, gc->local_y.p, gc->ny, m->half, m->halfp,
                                             false, gc->ey_bf.p, gc->ey_bf_lo.p, s), "y table");
            }
            if (precision == VSAOGM_BF16X3) *lo = gc->ey_bf_lo.p;
            return gc->ey_bf.p;
    }
}

void check_grid(const vsaogm_grid_desc* g) {
    if (!g) fail(VSAOGM_EINVAL, "grid is NULL");
    if (g->nx < 1 || g->ny < 1) fail(VSAOGM_EINVAL, "grid nx and ny must be >= 1");
    if ((int64_t)g->nx * g->ny > (int64_t)1 << 31) fail(VSAOGM_EINVAL, "grid too large");
    if (!is_finite(g->x0) || !is_finite(g->y0) || !is_finite(g->res) || !(g->res > 0))
        fail(VSAOGM_EINVAL, "grid origin must be finite and res > 0");
}

void check_grid3(const vsaogm_grid3_desc* g) {
    if (!g) fail(VSAOGM_EINVAL, "grid is NULL");
    if (g->nx < 1 || g->ny < 1 || g->nz < 1) fail(VSAOGM_EINVAL, "grid nx, ny and nz must be >= 1");
    if ((int64_t)g->nx * g->ny * g->nz > (int64_t)1 << 31) fail(VSAOGM_EINVAL, "grid too large");
    if (!is_finite(g->x0) || !is_finite(g->y0) || !is_finite(g->z0) || !is_finite(g->res) || !(g->res > 0))
        fail(VSAOGM_EINVAL, "grid origin must be finite and res > 0");
}

// Per-axis nearest centres of a volume grid, with the exact 3-D argmin confirmed wherever an
// axis is close to a tie (as for plane maps).
Grid3Cache* grid3_cache(vsaogm_volume* v, const vsaogm_grid3_desc* g, hipStream_t s) {
    if (v->grid && std::memcmp(&v->grid->key, g, sizeof(*g)) == 0) return v->grid.get();
    const int nx = g->nx, ny = g->ny, nz = g->nz;
    std::vector<int> t[3];
    std::vector<double> loc[3];
    std::vector<char> tie[3];
    const double o[3] = {g->x0, g->y0, g->z0};
    const std::vector<double>* c[3] = {&v->cx, &v->cy, &v->cz};
    const int nc[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a) {
        t[a].resize(nc[a]);
        loc[a].resize(nc[a]);
        tie[a].assign(nc[a], 0);
        for (int i = 0; i < nc[a]; ++i) {
            const double val = o[a] + ((double)i + 0.5) * g->res;
            t[a][i] = nearest_1d(*c[a], val);
            loc[a][i] = val - (*c[a])[t[a][i]];
            if (i > 0 && t[a][i] < t[a][i - 1]) fail(VSAOGM_EINVAL, "grid voxels are not ordered along an axis");
            for (int u = 0; u < (int)c[a]->size(); ++u) {
                if (u == t[a][i]) continue;
                const double d1 = (val - (*c[a])[t[a][i]]) * (val - (*c[a])[t[a][i]]);
                const double d2 = (val - (*c[a])[u]) * (val - (*c[a])[u]);
                if (std::fabs(d2 - d1) <= 1e-9 * (d1 + d2) + 1e-300) tie[a][i] = 1;
            }
        }
    }
    for (int l = 0; l < nz; ++l)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                if (!tie[0][i] && !tie[1][j] && !tie[2][l]) continue;
                const double x = g->x0 + ((double)i + 0.5) * g->res, y = g->y0 + ((double)j + 0.5) * g->res,
                             z = g->z0 + ((double)l + 0.5) * g->res;
                int best = 0;
                double bd = INFINITY;
                for (int b = 0; b < v->tiles_x * v->tiles_y * v->tiles_z; ++b) {
                    const int tx = b % v->tiles_x, ty = (b / v->tiles_x) % v->tiles_y, tz = b / (v->tiles_x * v->tiles_y);
                    const double dx = x - v->cx[tx], dy = y - v->cy[ty], dz = z - v->cz[tz];
                    const double d = dx * dx + dy * dy + dz * dz;
                    if (d < bd) {
                        bd = d;
                        best = b;
                    }
                }
                if (best != (t[2][l] * v->tiles_y + t[1][j]) * v->tiles_x + t[0][i])
                    fail(VSAOGM_EINVAL, "a voxel centre lies on a tile boundary in a way that does not "
                                        "split into per-tile slabs");
            }
    auto gc = std::make_unique<Grid3Cache>();
    gc->key = *g;
    // joint (z, y) rows grouped by tile block: for each (tz, ty), its slices, and in each slice
    // its grid rows; every block is one band (its rows share the memories of (tz, ty))
    std::vector<DBand> bands;
    std::vector<int> row_map;
    row_map.reserve((size_t)nz * ny);
    for (int tz = 0; tz < v->tiles_z; ++tz) {
        const int l0 = (int)(std::lower_bound(t[2].begin(), t[2].end(), tz) - t[2].begin());
        const int l1 = (int)(std::upper_bound(t[2].begin(), t[2].end(), tz) - t[2].begin());
        for (int ty = 0; ty < v->tiles_y; ++ty) {
            const int y0 = (int)(std::lower_bound(t[1].begin(), t[1].end(), ty) - t[1].begin());
            const int y1 = (int)(std::upper_bound(t[1].begin(), t[1].end(), ty) - t[1].begin());
            if (l0 >= l1 || y0 >= y1) continue;
            const int r0 = (int)row_map.size();
            for (int l = l0; l < l1; ++l)
                for (int y = y0; y < y1; ++y) row_map.push_back(l * ny + y);
            bands.push_back(DBand{tz * v->tiles_y + ty, r0, (int)row_map.size()});
        }
    }
    gc->nrows = (int)row_map.size();   // every voxel row once: the axes split into per-tile slabs
    gc->row_map.alloc(row_map.size(), "volume row map");
    hip_check(hipMemcpy(gc->row_map.p, row_map.data(), row_map.size() * sizeof(int), hipMemcpyHostToDevice),
              "copy row map");
    for (int set = 1; set < kDecodeTileSets; ++set) {
        std::vector<DTile> tl = build_decode_tiles(bands, t[0], nx, set);
        gc->ntiles[set] = (int)tl.size();
        gc->tiles[set].alloc(tl.size(), "volume tile list");
        hip_check(hipMemcpy(gc->tiles[set].p, tl.data(), tl.size() * sizeof(DTile), hipMemcpyHostToDevice),
                  "copy tile list");
        gc->uplan[set].build((int)tl.size(), v->halfp / 32, v->num_cus);
        gc->dunits[set].upload(gc->uplan[set]);
    }
    gc->col_tx.alloc(nx, "column tiles");
    hip_check(hipMemcpy(gc->col_tx.p, t[0].data(), nx * sizeof(int), hipMemcpyHostToDevice), "copy column tiles");
    DevBuf<double>* lb[3] = {&gc->local_x, &gc->local_y, &gc->local_z};
    for (int a = 0; a < 3; ++a) {
        lb[a]->alloc(nc[a], "local coordinates");
        hip_check(hipMemcpy(lb[a]->p, loc[a].data(), nc[a] * sizeof(double), hipMemcpyHostToDevice), "copy local");
    }
    gc->ex32.alloc((size_t)nx * v->halfp, "x location table");
    hip_check(launch_table_f32(v->d_theta_xy.p, 0, gc->local_x.p, nx, v->half, v->halfp, gc->ex32.p, s), "x table");
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    v->grid = std::move(gc);
    return v->grid.get();
}

EncodeWork map_work(vsaogm_map* m) {
    EncodeWork w;
    w.key = m->w_key.p;
    w.sorted = m->w_sorted.p;
    w.sorted_lo = m->w_sorted_lo.p;
    w.hist = m->w_hist.p;
    w.table = m->w_table.p;
    w.meta = m->w_meta.p;
    w.partial = m->w_partial.p;
    w.n_bad = m->d_bad.p;
    w.version = m->d_version.p;
    return w;
}

}  // namespace

// ---- batched map updates ---------------------------------------------------------------
// Several whole map updates (one per map) run as one launch per stage: the per-request
// descriptors, block prefixes and the concatenated decode tile list are packed into one staging
// block and copied to the device with one copy, then encode (assign, scan, scatter, encode,
// reduce), norm, the similarity GEMM (+ fix-up) and the classification each cover every request.
namespace vsaogm {

namespace {
template <class T>
int64_t nbytes(const DevBuf<T>& b) {
    return b.p ? (int64_t)std::max<size_t>(b.n, 1) * (int64_t)sizeof(T) : 0;
}

// Every device buffer of a cached grid (keep in step with GridCache).
int64_t grid_bytes(const GridCache& g) {
    int64_t b = nbytes(g.local_x) + nbytes(g.local_y) + nbytes(g.col_tx) + nbytes(g.ex32) + nbytes(g.ey32) +
                nbytes(g.ey_bf) + nbytes(g.ey_bf_lo) + nbytes(g.ey_h) + nbytes(g.d_boxes) + nbytes(g.d_seen) +
                nbytes(g.region_max) + nbytes(g.inc_tiles) + nbytes(g.inc_boxes) + nbytes(g.inc_units) +
                nbytes(g.inc_tile_u0) + nbytes(g.inc_wg_u0) + nbytes(g.inc_dyn);
    for (int t = 0; t < kDecodeTileSets; ++t)
        b += nbytes(g.tiles[t]) + nbytes(g.dunits[t].units) + nbytes(g.dunits[t].tile_u0) +
             nbytes(g.dunits[t].wg_u0);
    return b;
}

// Bytes of a 16-bit y table or of an fp32 table of n cells.
int64_t table16_bytes(const vsaogm_map* m, int n) { return (int64_t)rows16(n) * 2 * m->halfp * 2; }
int64_t table32_bytes(const vsaogm_map* m, int n) { return (int64_t)n * m->halfp * 8; }

int64_t y_tables_bytes(const vsaogm_map* m, int ny, int precision) {
    switch (precision) {
        case VSAOGM_FP32: return table32_bytes(m, ny);
        case VSAOGM_FP16: return table16_bytes(m, ny);
        default: return 2 * table16_bytes(m, ny);   // bf16 hi + residual, built together
    }
}
}  // namespace

int64_t map_resident_bytes(const vsaogm_map* m) {
    int64_t b = nbytes(m->d_cx) + nbytes(m->d_cy) + nbytes(m->d_rev) + nbytes(m->d_rev_d) + nbytes(m->d_theta) +
                nbytes(m->d_omega) + nbytes(m->d_scale) + nbytes(m->d_omega_s) + nbytes(m->d_partial) +
                nbytes(m->d_hmax_u) + nbytes(m->d_bad) + nbytes(m->d_version) + nbytes(m->w_key) +
                nbytes(m->w_hist) + nbytes(m->w_meta) + nbytes(m->w_sorted) + nbytes(m->w_sorted_lo) +
                nbytes(m->w_partial) + nbytes(m->w_table);
    for (const auto& kv : m->grids) b += grid_bytes(*kv.second);
    return b;
}

int64_t map_growth_bytes(const vsaogm_map* m, const vsaogm_grid_desc* g, int precision, int64_t n, bool local) {
    int64_t b = 0;
    // encode workspace (ensure_encode_workspace): a new block replaces the old in stream order,
    // so both are counted while the old one may still be in use
    const EncodePlan p = encode_plan(n, m->halfp, m->nkeys);
    if (n > m->cap_n || p.nchunks > m->cap_chunks || p.max_echunks > m->cap_echunks) {
        const int64_t cap = std::max<int64_t>(n + n / 2, 4096);
        const EncodePlan q = encode_plan(cap, m->halfp, m->nkeys);
        const int64_t chunks = std::max(q.nchunks, p.nchunks), echunks = std::max(q.max_echunks, p.max_echunks);
        b += cap * (4 + 8 + 8) + (chunks * m->nkeys + kHistPad) * 4 + echunks * (int64_t)sizeof(EChunk) +
             echunks * m->halfp * 8 + (1 + 3 * (int64_t)m->nkeys) * 4;
    }
    // partial sums: at most the largest block any decode uses
    const int64_t partial = (int64_t)decode_partial_floats_max(m->num_cus) * 4;
    if (nbytes(m->d_partial) < partial) b += partial;
    // grid: the whole cache when new, else the table of a precision not built yet
    const GridKey key{g->x0, g->y0, g->res, g->nx, g->ny};
    auto it = m->grids.find(key);
    const GridCache* gc = it == m->grids.end() ? nullptr : it->second.get();
    if (!gc) {
        // tiles per set: bands of at least 16 rows (plus one per tile row), 64 columns
        // (plus one per tile column); units at most two per tile plus one per slot
        const int64_t tiles = ((int64_t)g->ny / 16 + 1 + m->tiles_y) * ((int64_t)g->nx / 64 + 1 + m->tiles_x);
        const int64_t slots = std::max(decode_slots16(m->num_cus), decode_slots32(m->num_cus));
        const int64_t per_set = tiles * (int64_t)sizeof(DTile) + (2 * tiles + slots) * (int64_t)sizeof(DUnit) +
                                (2 * tiles + slots + 2) * 4;
        b += kDecodeTileSets * per_set + ((int64_t)g->nx + g->ny) * 12 + table32_bytes(m, g->nx) +
             y_tables_bytes(m, g->ny, precision);
        if (local) {
            const int64_t nreg = (int64_t)m->tiles_x * m->tiles_y;
            b += nreg * (int64_t)(2 * sizeof(RegionBox) + 8 + 8) + tiles * (int64_t)(sizeof(DTile) + sizeof(DUnit)) +
                 (2 * tiles + 2 * slots + 8) * 4 + slots * (int64_t)sizeof(DUnit);
        }
    } else {
        const bool have = precision == VSAOGM_FP32 ? gc->ey32.p != nullptr
                          : precision == VSAOGM_FP16 ? gc->ey_h.p != nullptr
                                                     : gc->ey_bf.p != nullptr && gc->ey_bf_lo.p != nullptr;
        if (!have) b += y_tables_bytes(m, g->ny, precision);
        if (local && !gc->d_seen.p) {
            int nmax = 0;
            for (int t = 0; t < kDecodeTileSets; ++t) nmax = std::max(nmax, gc->ntiles[t]);
            const int64_t nreg = (int64_t)m->tiles_x * m->tiles_y;
            const int64_t slots = decode_slots16(m->num_cus);
            b += nreg * (int64_t)(2 * sizeof(RegionBox) + 8 + 8) + nmax * (int64_t)(sizeof(DTile) + sizeof(DUnit)) +
                 (2 * nmax + 2 * slots + 8) * 4 + slots * (int64_t)sizeof(DUnit);
        }
    }
    return b;
}

void map_trim(vsaogm_map* m) {
    DeviceGuard guard(m->device);
    hip_check(hipDeviceSynchronize(), "trim: synchronise");
    m->grids.clear();
    m->d_partial.release();
    m->w_key.release();
    m->w_hist.release();
    m->w_meta.release();
    m->w_sorted.release();
    m->w_sorted_lo.release();
    m->w_partial.release();
    m->w_table.release();
    m->cap_n = 0;
    m->cap_chunks = 0;
    m->cap_echunks = 0;
}

struct UpdateBatchWork {
    DevBuf<unsigned char> d_meta;
    unsigned char* h_meta = nullptr;
    size_t h_cap = 0;
    DevBuf<float> d_partial;
    ~UpdateBatchWork() {
        if (h_meta) (void)hipHostFree(h_meta);
    }
};

UpdateBatchWork* update_batch_work_create() { return new UpdateBatchWork(); }
void update_batch_work_destroy(UpdateBatchWork* w) { delete w; }
int64_t update_batch_work_bytes(const UpdateBatchWork* w) { return nbytes(w->d_meta) + nbytes(w->d_partial); }
void update_batch_work_trim(UpdateBatchWork* w) {
    w->d_meta.release();
    w->d_partial.release();
}

int run_update_batch(const UpdateItem* items, int count, int precision, hipStream_t s, UpdateBatchWork* w) {
    return guarded([&] {
        if (!items || count < 1 || !w) fail(VSAOGM_EINVAL, "batch: items, count >= 1 and workspace required");
        if (precision < VSAOGM_BF16 || precision > VSAOGM_BF16X3)
            fail(VSAOGM_EINVAL, "batch: the batched similarity runs the 16-bit formats");
        const int device = items[0].map ? items[0].map->device : 0;
        for (int i = 0; i < count; ++i) {
            const UpdateItem& it = items[i];
            if (!it.map) fail(VSAOGM_EINVAL, "batch: map is NULL");
            if (it.map->device != device) fail(VSAOGM_EINVAL, "batch: maps on different devices");
            for (int j = 0; j < i; ++j)
                if (items[j].map == it.map) fail(VSAOGM_EINVAL, "batch: a map appears twice");
            check_grid(&it.grid);
            if (it.n < 0) fail(VSAOGM_EINVAL, "batch: n must be >= 0");
            if (it.n > 0 && !it.host_in && (!it.xy || !it.label))
                fail(VSAOGM_EINVAL, "batch: xy and label (or host_in) must not be NULL");
            if (it.n > ((int64_t)1 << 31) - (int64_t)kAssignChunk * 2) fail(VSAOGM_EINVAL, "batch: n too large");
            if (!it.heat || !it.hmax || !it.label_out) fail(VSAOGM_EINVAL, "batch: heat, hmax and label required");
            if (it.r_occ < 0 || it.r_emp < 0 || it.r_occ > kMaxRadius || it.r_emp > kMaxRadius)
                fail(VSAOGM_EINVAL, "batch: radii must be in 0..24");
            if (!is_finite(it.rho)) fail(VSAOGM_EINVAL, "batch: rho must be finite");
        }
        DeviceGuard guard(device);
        const int set = decode_tile_set(precision);
        std::vector<EncodeReq> eq(count);
        std::vector<DecodeReq> dq(count);
        std::vector<ClassifyReq> cq(count);
        std::vector<DTile> tiles;
        std::vector<DUnit> units;
        std::vector<int> tile_u0, wg_u0;
        int pblocks = 0;   // partial-sum blocks of the requests with split tiles
        int num_cus = 1, max_r = 0;
        for (int i = 0; i < count; ++i) {
            const UpdateItem& it = items[i];
            vsaogm_map* m = it.map;
            num_cus = m->num_cus;
            if (it.n > 0) ensure_encode_workspace(m, it.n, s);
            GridCache* gc = grid_cache(m, &it.grid, s);
            const void* ey_lo = nullptr;
            const void* ey = y_table(m, gc, precision, &ey_lo, s);
            EncodeReq q = encode_req(it.xy, it.label, it.n, m->layout(), m->nkeys, m->d_rev.p, m->d_rev_d.p,
                                     m->max_rev_x, m->max_rev_y, m->half, m->halfp, map_work(m), m->d_omega.p);
            q.D = m->D;
            q.scale = m->d_scale.p;
            q.omega_s = m->d_omega_s.p;
            q.hmax_u = m->d_hmax_u.p;
            eq[i] = q;
            DecodeReq& d = dq[i];
            d.col_tx = gc->col_tx.p;
            d.ex = gc->ex32.p;
            d.ey = ey;
            d.ey_lo = ey_lo;
            d.omega_s = m->d_omega_s.p;
            d.halfp = m->halfp;
            d.nx = it.grid.nx;
            d.ny = it.grid.ny;
            d.tiles_x = m->tiles_x;
            d.out_scale = (float)(2.0 / (double)m->D);
            d.heat = it.heat;
            d.class_stride = (size_t)it.grid.nx * it.grid.ny;
            d.row_map = nullptr;
            d.hmax_u = m->d_hmax_u.p;
            d.ksteps = m->halfp / 32;
            ClassifyReq& c = cq[i];
            c.heat = it.heat;
            c.hmax_u = m->d_hmax_u.p;
            c.hmax_out = it.hmax;
            c.nx = it.grid.nx;
            c.ny = it.grid.ny;
            c.r_occ = it.r_occ;
            c.r_emp = it.r_emp;
            c.rho = it.rho;
            c.ogm = it.ogm;
            c.label = it.label_out;
            max_r = std::max(max_r, std::max(it.r_occ, it.r_emp));
            // the request's own units (as vsaogm_decode runs them), renumbered into the batch
            const int tile_base = (int)tiles.size(), unit_base = (int)units.size();
            for (DTile t : gc->host_tiles[set]) {
                t.pad = i;
                tiles.push_back(t);
            }
            const UnitPlan& up = gc->uplan[set];
            const bool split = up.units.size() > gc->host_tiles[set].size();
            for (DUnit u : up.units) {
                u.tile += tile_base;
                u.part += pblocks;   // partial blocks of the request's workgroups, after the others'
                units.push_back(u);
            }
            if (split) pblocks += 2 * up.nwg();
            for (size_t t = 0; t + 1 < up.tile_u0.size(); ++t) tile_u0.push_back(up.tile_u0[t] + unit_base);
            for (size_t g = 0; g + 1 < up.wg_u0.size(); ++g) wg_u0.push_back(up.wg_u0[g] + unit_base);
        }
        // encode groups by bins per thread (the encode kernel's template argument)
        std::vector<int> order;
        int ngroup[3] = {0, 0, 0};
        for (int g = 1; g <= 2; ++g)
            for (int i = 0; i < count; ++i)
                if (eq[i].bpt == g) {
                    order.push_back(i);
                    ++ngroup[g];
                }
        if ((int)order.size() != count) fail(VSAOGM_EDEVICE, "batch: unexpected encode geometry");
        std::vector<EncodeReq> eq_sorted(count);
        for (int j = 0; j < count; ++j) eq_sorted[j] = eq[order[j]];
        // block prefixes: per group [kEncodeStages][n_g + 1]; classification [count + 1]
        std::vector<int> enc_b0;
        EncodeBatch eb[3] = {};
        size_t enc_b0_off[3] = {0, 0, 0};
        int first = 0;
        for (int g = 1; g <= 2; ++g) {
            const int ng = ngroup[g];
            eb[g].nreq = ng;
            eb[g].bpt = g;
            enc_b0_off[g] = enc_b0.size();
            if (ng == 0) continue;
            std::vector<int> pre((size_t)kEncodeStages * (ng + 1), 0);
            for (int j = 0; j < ng; ++j) {
                int b[kEncodeStages];
                encode_batch_blocks(eq_sorted[first + j], b);
                for (int st = 0; st < kEncodeStages; ++st) pre[(size_t)st * (ng + 1) + j + 1] = pre[(size_t)st * (ng + 1) + j] + b[st];
                eb[g].max_keys = std::max(eb[g].max_keys, eq_sorted[first + j].nkeys);
            }
            for (int st = 0; st < kEncodeStages; ++st) eb[g].blocks[st] = pre[(size_t)st * (ng + 1) + ng];
            enc_b0.insert(enc_b0.end(), pre.begin(), pre.end());
            first += ng;
        }
        std::vector<int> cls_b0(count + 1, 0);
        for (int i = 0; i < count; ++i) cls_b0[i + 1] = cls_b0[i] + classify_blocks(cq[i].nx, cq[i].ny);
        tile_u0.push_back((int)units.size());
        wg_u0.push_back((int)units.size());
        const bool any_split = units.size() > tiles.size();
        (void)num_cus;

        // one staging block: encode requests, encode prefixes, decode requests, classify requests,
        // classify prefixes, tiles, work units, first units of tiles and workgroups (each
        // 16-byte aligned)
        size_t off = 0;
        auto place = [&](size_t bytes) {
            const size_t o = off;
            off = (off + bytes + 15) / 16 * 16;
            return o;
        };
        const size_t o_eq = place(sizeof(EncodeReq) * count);
        const size_t o_eb0 = place(sizeof(int) * enc_b0.size());
        const size_t o_dq = place(sizeof(DecodeReq) * count);
        const size_t o_cq = place(sizeof(ClassifyReq) * count);
        const size_t o_cb0 = place(sizeof(int) * cls_b0.size());
        const size_t o_t = place(sizeof(DTile) * std::max<size_t>(tiles.size(), 1));
        const size_t o_u = place(sizeof(DUnit) * std::max<size_t>(units.size(), 1));
        const size_t o_ti = place(sizeof(int) * tile_u0.size());
        const size_t o_wi = place(sizeof(int) * wg_u0.size());
        // inputs given in pinned host memory travel with the descriptors
        std::vector<size_t> o_in(count, 0);
        for (int i = 0; i < count; ++i)
            if (items[i].host_in && items[i].n > 0) o_in[i] = place((size_t)items[i].n * 9);
        const size_t bytes = off;
        if (w->h_cap < bytes) {
            if (w->h_meta) (void)hipHostFree(w->h_meta);
            w->h_meta = nullptr;
            w->h_cap = 0;
            size_t cap = 1 << 16;
            while (cap < bytes) cap *= 2;
            hip_check(hipHostMalloc((void**)&w->h_meta, cap, hipHostMallocDefault), "batch staging");
            w->h_cap = cap;
        }
        if (w->d_meta.n < bytes) w->d_meta.alloc_async(std::max<size_t>(bytes, w->h_cap), s, "batch descriptors");
        unsigned char* h = w->h_meta;
        unsigned char* dm = w->d_meta.p;
        for (int j = 0; j < count; ++j) {
            const UpdateItem& it = items[order[j]];
            if (!it.host_in || it.n <= 0) continue;
            std::memcpy(h + o_in[order[j]], it.host_in, (size_t)it.n * 9);
            eq_sorted[j].xy = reinterpret_cast<const float2*>(dm + o_in[order[j]]);
            eq_sorted[j].label = dm + o_in[order[j]] + (size_t)it.n * 8;
        }
        std::memcpy(h + o_eq, eq_sorted.data(), sizeof(EncodeReq) * count);
        std::memcpy(h + o_eb0, enc_b0.data(), sizeof(int) * enc_b0.size());
        std::memcpy(h + o_dq, dq.data(), sizeof(DecodeReq) * count);
        std::memcpy(h + o_cq, cq.data(), sizeof(ClassifyReq) * count);
        std::memcpy(h + o_cb0, cls_b0.data(), sizeof(int) * cls_b0.size());
        if (!tiles.empty()) std::memcpy(h + o_t, tiles.data(), sizeof(DTile) * tiles.size());
        if (!units.empty()) std::memcpy(h + o_u, units.data(), sizeof(DUnit) * units.size());
        std::memcpy(h + o_ti, tile_u0.data(), sizeof(int) * tile_u0.size());
        std::memcpy(h + o_wi, wg_u0.data(), sizeof(int) * wg_u0.size());
        const size_t partial = decode_unit_partial_floats(pblocks);
        if (any_split && w->d_partial.n < partial) w->d_partial.alloc_async(partial, s, "batch partial sums");
        hip_check(hipMemcpyAsync(dm, h, bytes, hipMemcpyHostToDevice, s), "copy batch descriptors");
        const EncodeReq* d_eq = reinterpret_cast<const EncodeReq*>(dm + o_eq);
        int done = 0;
        for (int g = 1; g <= 2; ++g) {
            if (eb[g].nreq == 0) continue;
            eb[g].reqs = d_eq + done;
            eb[g].block0 = reinterpret_cast<const int*>(dm + o_eb0) + enc_b0_off[g];
            hip_check(launch_encode_batch(eb[g], s), "batched encode");
            done += eb[g].nreq;
        }
        DecodeBatch db;
        db.tiles = reinterpret_cast<const DTile*>(dm + o_t);
        db.ntiles = (int)tiles.size();
        db.reqs = reinterpret_cast<const DecodeReq*>(dm + o_dq);
        db.units = reinterpret_cast<const DUnit*>(dm + o_u);
        db.nunits = (int)units.size();
        db.tile_u0 = reinterpret_cast<const int*>(dm + o_ti);
        db.wg_u0 = reinterpret_cast<const int*>(dm + o_wi);
        db.nwg = (int)wg_u0.size() - 1;
        db.partial = w->d_partial.p;
        db.any_split = any_split;
        hip_check(launch_decode_batch(precision, db, s), "batched decode");
        hip_check(launch_classify_batch(reinterpret_cast<const ClassifyReq*>(dm + o_cq),
                                        reinterpret_cast<const int*>(dm + o_cb0), count, cls_b0[count], max_r, s),
                  "batched classify");
    });
}

}  // namespace vsaogm

extern "C" {

int32_t vsaogm_version(void) { return 100; }

const char* vsaogm_last_error(void) { return g_last_error.c_str(); }

int vsaogm_map_create(const vsaogm_map_desc* d, vsaogm_map** out) {
    return guarded([&] {
        if (!d || !out) fail(VSAOGM_EINVAL, "desc and out must not be NULL");
        *out = nullptr;
        const int D = d->dim;
        if (D < 4 || (D & 1)) fail(VSAOGM_EINVAL, "dim must be even and >= 4");
        if (D > (1 << 22)) fail(VSAOGM_EINVAL, "dim too large");
        if (!d->theta) fail(VSAOGM_EINVAL, "theta is NULL");
        if (d->tiles_x < 1 || d->tiles_y < 1 || d->tiles_x > kMaxTilesPerAxis ||
            d->tiles_y > kMaxTilesPerAxis)
            fail(VSAOGM_EINVAL, "tiles per axis must be in 1..64");
        if (!is_finite(d->x0) || !is_finite(d->x1) || !is_finite(d->y0) || !is_finite(d->y1) ||
            !(d->x1 > d->x0) || !(d->y1 > d->y0))
            fail(VSAOGM_EINVAL, "layout rectangle must be finite with x1 > x0 and y1 > y0");
        const double* th = d->theta;
        for (int k = 0; k < 2 * D; ++k)
            if (!is_finite(th[k])) fail(VSAOGM_EINVAL, "theta must be finite");
        const int half = D / 2;
        if (th[0] != 0.0 || th[1] != 0.0 || th[2 * half] != 0.0 || th[2 * half + 1] != 0.0)
            fail(VSAOGM_EINVAL, "theta[0] and theta[D/2] must be zero");
        for (int k = 1; k < half; ++k)
            for (int a = 0; a < 2; ++a)
                if (th[2 * (D - k) + a] != -th[2 * k + a])
                    fail(VSAOGM_EINVAL, "theta must be conjugate-symmetric: theta[D-k] = -theta[k]");
        int ndev = 0;   // arguments are checked before the device is touched
        hip_check(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
        if (d->device < 0 || d->device >= ndev) fail(VSAOGM_EINVAL, "no such device");

        auto m = std::make_unique<vsaogm_map>();
        m->device = d->device;
        m->D = D;
        m->half = half;
        m->halfp = (half + kBinPad - 1) / kBinPad * kBinPad;
        m->tiles_x = d->tiles_x;
        m->tiles_y = d->tiles_y;
        m->nkeys = 2 * d->tiles_x * d->tiles_y;
        m->x0 = d->x0;
        m->y0 = d->y0;
        m->x1 = d->x1;
        m->y1 = d->y1;
        m->theta.assign(th, th + 2 * (size_t)D);
        m->cx = centres(d->x0, d->x1, d->tiles_x);
        m->cy = centres(d->y0, d->y1, d->tiles_y);

        std::vector<float2> rev(m->halfp, make_float2(0.f, 0.f));
        std::vector<double> rev_d(2 * (size_t)m->halfp, 0.0);
        const double inv2pi = 1.0 / (2.0 * M_PI);
        for (int k = 0; k < half; ++k) {
            const double a = th[2 * k] * inv2pi, b = th[2 * k + 1] * inv2pi;
            rev[k] = make_float2((float)a, (float)b);
            rev_d[2 * k] = a;
            rev_d[2 * k + 1] = b;
            m->max_rev_x = std::max(m->max_rev_x, std::fabs(rev[k].x));
            m->max_rev_y = std::max(m->max_rev_y, std::fabs(rev[k].y));
        }

        DeviceGuard guard(m->device);
        hip_check(hipDeviceGetAttribute(&m->num_cus, hipDeviceAttributeMultiprocessorCount, m->device),
                  "device attribute");
        if (m->num_cus < 1) m->num_cus = 1;
        m->d_cx.alloc(m->tiles_x, "tile centres x");
        m->d_cy.alloc(m->tiles_y, "tile centres y");
        m->d_rev.alloc(m->halfp, "theta (rev, fp32)");
        m->d_rev_d.alloc(2 * (size_t)m->halfp, "theta (rev, fp64)");
        m->d_theta.alloc(2 * (size_t)half, "theta (rad)");
        m->d_omega.alloc((size_t)m->nkeys * m->halfp, "memories");
        m->d_scale.alloc(m->nkeys, "memory scales");
        m->d_omega_s.alloc((size_t)m->nkeys * m->halfp, "scaled memories");
        m->d_hmax_u.alloc(2, "class maxima");
        m->d_bad.alloc(1, "rejected-label counter");
        m->d_version.alloc(m->nkeys, "memory versions");
        hip_check(hipMemcpy(m->d_cx.p, m->cx.data(), m->cx.size() * 8, hipMemcpyHostToDevice), "copy");
        hip_check(hipMemcpy(m->d_cy.p, m->cy.data(), m->cy.size() * 8, hipMemcpyHostToDevice), "copy");
        hip_check(hipMemcpy(m->d_rev.p, rev.data(), rev.size() * sizeof(float2), hipMemcpyHostToDevice),
                  "copy");
        hip_check(hipMemcpy(m->d_rev_d.p, rev_d.data(), rev_d.size() * 8, hipMemcpyHostToDevice), "copy");
        hip_check(hipMemcpy(m->d_theta.p, th, 2 * (size_t)half * 8, hipMemcpyHostToDevice), "copy");
        zero_async(m->d_omega.p, m->d_omega.n * sizeof(float2), nullptr);
        zero_async(m->d_bad.p, sizeof(unsigned long long), nullptr);
        zero_async(m->d_version.p, sizeof(unsigned) * m->nkeys, nullptr);
        hip_check(hipStreamSynchronize(nullptr), "hipStreamSynchronize");
        *out = m.release();
    });
}

int vsaogm_map_destroy(vsaogm_map* m) {
    if (!m) return VSAOGM_OK;
    return guarded([&] {
        DeviceGuard guard(m->device);
        (void)hipDeviceSynchronize();
        delete m;
    });
}

int vsaogm_map_info(const vsaogm_map* m, int64_t* n_memories, int32_t* dim) {
    return guarded([&] {
        if (!m) fail(VSAOGM_EINVAL, "map is NULL");
        if (n_memories) *n_memories = m->nkeys;
        if (dim) *dim = m->D;
    });
}

int vsaogm_map_reset(vsaogm_map* m, vsaogm_stream stream) {
    return guarded([&] {
        if (!m) fail(VSAOGM_EINVAL, "map is NULL");
        DeviceGuard guard(m->device);
        const size_t words = m->d_omega.n * 2;
        const size_t n = std::max(words, (size_t)m->nkeys);
        hipLaunchKernelGGL(k_reset_map, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                           reinterpret_cast<unsigned*>(m->d_omega.p), words, m->d_version.p, m->nkeys);
        hip_check(hipGetLastError(), "reset kernel");
    });
}

int vsaogm_encode(vsaogm_map* m, const float* xy, const uint8_t* label, int64_t n,
                  vsaogm_stream stream) {
    return guarded([&] {
        if (!m) fail(VSAOGM_EINVAL, "map is NULL");
        if (n < 0) fail(VSAOGM_EINVAL, "n must be >= 0");
        if (n == 0) return;
        if (!xy || !label) fail(VSAOGM_EINVAL, "xy and label must not be NULL");
        if (n > ((int64_t)1 << 31) - (int64_t)kAssignChunk * 2)
            fail(VSAOGM_EINVAL, "n too large for one call");
        DeviceGuard guard(m->device);
        hipStream_t s = (hipStream_t)stream;
        ensure_encode_workspace(m, n, s);
        EncodeWork w;
        w.key = m->w_key.p;
        w.sorted = m->w_sorted.p;
        w.sorted_lo = m->w_sorted_lo.p;
        w.hist = m->w_hist.p;
        w.table = m->w_table.p;
        w.meta = m->w_meta.p;
        w.partial = m->w_partial.p;
        w.n_bad = m->d_bad.p;
        w.version = m->d_version.p;
        hip_check(launch_encode(xy, label, n, m->layout(), m->nkeys, m->d_rev.p, m->d_rev_d.p,
                                m->max_rev_x, m->max_rev_y, m->half, m->halfp, w, m->d_omega.p, s),
                  "encode launch");
    });
}

int vsaogm_map_take_rejected(vsaogm_map* m, vsaogm_stream stream, int64_t* n_rejected) {
    return guarded([&] {
        if (!m || !n_rejected) fail(VSAOGM_EINVAL, "map and n_rejected must not be NULL");
        DeviceGuard guard(m->device);
        hipStream_t s = (hipStream_t)stream;
        unsigned long long v = 0;
        hip_check(hipMemcpyAsync(&v, m->d_bad.p, sizeof(v), hipMemcpyDeviceToHost, s), "read counter");
        hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
        zero_async(m->d_bad.p, sizeof(v), s);
        *n_rejected = (int64_t)v;
    });
}

int vsaogm_decode(vsaogm_map* m, const vsaogm_grid_desc* g, int32_t precision, float* heat,
                  float* hmax, vsaogm_stream stream) {
    return guarded([&] {
        if (!m) fail(VSAOGM_EINVAL, "map is NULL");
        check_grid(g);
        if (!heat || !hmax) fail(VSAOGM_EINVAL, "heat and hmax must not be NULL");
        if (precision < VSAOGM_FP32 || precision > VSAOGM_BF16X3) fail(VSAOGM_EINVAL, "unknown precision");
        DeviceGuard guard(m->device);
        hipStream_t s = (hipStream_t)stream;
        GridCache* gc = grid_cache(m, g, s);
        const void* ey_lo = nullptr;
        const void* ey = y_table(m, gc, precision, &ey_lo, s);
        const int set = decode_tile_set(precision);
        DecodeLaunch d;
        d.plan = decode_plan(precision, gc->ntiles[set], m->halfp, m->num_cus);
        size_t need = decode_partial_floats(precision, d.plan);
        if (precision != VSAOGM_FP32) need = set_units(d, gc->uplan[set], gc->dunits[set], gc->ntiles[set]);
        if (m->d_partial.n < need) m->d_partial.alloc_async(need, s, "decode partial sums");
        hip_check(launch_norm(m->d_omega.p, m->nkeys, m->half, m->halfp, m->D, m->d_scale.p,
                              m->d_omega_s.p, m->d_hmax_u.p, s),
                  "norm launch");
        d.tiles = gc->tiles[set].p;
        d.ntiles = gc->ntiles[set];
        d.col_tx = gc->col_tx.p;
        d.ex = gc->ex32.p;
        d.ey = ey;
        d.ey_lo = ey_lo;
        d.omega_s = m->d_omega_s.p;
        d.halfp = m->halfp;
        d.nx = g->nx;
        d.ny = g->ny;
        d.tiles_x = m->tiles_x;
        d.out_scale = (float)(2.0 / (double)m->D);
        d.heat = heat;
        d.hmax_u = m->d_hmax_u.p;
        d.hmax = hmax;
        d.partial = m->d_partial.p;
        hip_check(launch_decode(precision, d, s), "decode launch");
    });
}

int vsaogm_decode_incremental(vsaogm_map* m, const vsaogm_grid_desc* g, int32_t precision, float* heat,
                              float* hmax, vsaogm_stream stream) {
    return guarded([&] {
        if (!m) fail(VSAOGM_EINVAL, "map is NULL");
        check_grid(g);
        if (!heat || !hmax) fail(VSAOGM_EINVAL, "heat and hmax must not be NULL");
        if (precision < VSAOGM_FP32 || precision > VSAOGM_BF16X3) fail(VSAOGM_EINVAL, "unknown precision");
        DeviceGuard guard(m->device);
        hipStream_t s = (hipStream_t)stream;
        GridCache* gc = grid_cache(m, g, s);
        const void* ey_lo = nullptr;
        const void* ey = y_table(m, gc, precision, &ey_lo, s);
        const int nregions = m->tiles_x * m->tiles_y;
        if (!gc->region_max.p) gc->region_max.alloc_async(2 * (size_t)nregions, s, "region maxima");
        const int set = decode_tile_set(precision);
        const int N = gc->ntiles[set];
        const int slots16 = decode_slots16(m->num_cus), slots32 = decode_slots32(m->num_cus);
        if (!gc->d_seen.p) {
            gc->d_seen.alloc_async(m->nkeys, s, "seen versions");
            gc->d_boxes.alloc_async(nregions, s, "region boxes");
            hip_check(hipMemcpyAsync(gc->d_boxes.p, gc->boxes.data(), sizeof(RegionBox) * nregions,
                                     hipMemcpyHostToDevice, s),
                      "copy region boxes");
            gc->inc_boxes.alloc_async(nregions, s, "changed regions");
            gc->inc_dyn.alloc_async(4, s, "localized decode counts");
        }
        // capacities for every tile of the largest tile set
        int nmax = 0;
        for (int t = 0; t < kDecodeTileSets; ++t) nmax = std::max(nmax, gc->ntiles[t]);
        if (gc->inc_tiles.n < (size_t)std::max(nmax, 1)) {
            gc->inc_tiles.alloc_async(std::max(nmax, 1), s, "changed tiles");
            gc->inc_units.alloc_async((size_t)nmax + slots16, s, "localized work units");
            gc->inc_tile_u0.alloc_async((size_t)nmax + 1, s, "localized tile units");
            gc->inc_wg_u0.alloc_async((size_t)std::max(nmax, slots16) + 1, s, "localized workgroup units");
        }
        const bool all = !gc->inc_valid || gc->inc_heat != heat || gc->inc_precision != precision;
        gc->inc_valid = true;
        gc->inc_heat = heat;
        gc->inc_precision = precision;
        // which memories changed since this grid's last localized decode, the tiles to decode
        // and the GEMM's work units: planned on the device, so nothing here waits for it
        IncPlan ip;
        ip.version = m->d_version.p;
        ip.seen = gc->d_seen.p;
        ip.all = all ? 1 : 0;
        ip.nregions = nregions;
        ip.tiles_x = m->tiles_x;
        ip.tiles = gc->tiles[set].p;
        ip.ntiles = N;
        ip.col_tx = gc->col_tx.p;
        ip.boxes = gc->d_boxes.p;
        ip.ksteps16 = m->halfp / 32;
        ip.ksteps32 = m->halfp / 16;
        ip.slots16 = slots16;
        ip.slots32 = slots32;
        ip.out_tiles = gc->inc_tiles.p;
        ip.out_boxes = gc->inc_boxes.p;
        ip.units = gc->inc_units.p;
        ip.tile_u0 = gc->inc_tile_u0.p;
        ip.wg_u0 = gc->inc_wg_u0.p;
        ip.dyn = gc->inc_dyn.p;
        ip.region_u = gc->region_max.p;
        hip_check(launch_inc_plan(ip, s), "localized decode plan");
        // partial sums: 16-bit, split tiles only when fewer tiles than slots (at most two units
        // per workgroup); fp32, two blocks per workgroup of at most slots32 workgroups
        DecodeLaunch d;
        d.plan = decode_plan(precision, N, m->halfp, m->num_cus);
        size_t need;
        if (precision != VSAOGM_FP32) {
            need = decode_unit_partial_floats(2 * slots16);
            d.units = gc->inc_units.p;
            d.nunits = 0;   // read on the device
            d.tile_u0 = gc->inc_tile_u0.p;
            d.wg_u0 = gc->inc_wg_u0.p;
            d.nwg = std::max(N, slots16);
            d.fix_tiles = N;   // with more changed tiles than slots, any of them can be split
        } else {
            d.plan.grid = slots32;
            d.plan.steps_per_wg = 0;   // read on the device
            DecodePlan worst{};   // at most slots32 workgroups, each with split tiles
            worst.ksteps = 2;
            worst.steps_per_wg = 1;
            worst.grid = slots32;
            need = decode_partial_floats(precision, worst);
            d.fix_tiles = N;
        }
        if (m->d_partial.n < need) m->d_partial.alloc_async(need, s, "decode partial sums");
        hip_check(launch_norm(m->d_omega.p, m->nkeys, m->half, m->halfp, m->D, m->d_scale.p, m->d_omega_s.p,
                              m->d_hmax_u.p, s),
                  "norm launch");
        d.dyn = gc->inc_dyn.p;
        d.tiles = gc->inc_tiles.p;
        d.ntiles = N;
        d.col_tx = gc->col_tx.p;
        d.ex = gc->ex32.p;
        d.ey = ey;
        d.ey_lo = ey_lo;
        d.omega_s = m->d_omega_s.p;
        d.halfp = m->halfp;
        d.nx = g->nx;
        d.ny = g->ny;
        d.tiles_x = m->tiles_x;
        d.out_scale = (float)(2.0 / (double)m->D);
        d.heat = heat;
        d.hmax_u = nullptr;
        d.hmax = hmax;
        d.partial = m->d_partial.p;
        if (N > 0) hip_check(launch_decode(precision, d, s), "decode launch");
        hip_check(launch_region_max_dyn(heat, g->nx, g->ny, gc->inc_boxes.p, gc->inc_dyn.p + 2, nregions,
                                        gc->region_max.p, nregions, hmax, s),
                  "region maxima");
    });
}

int vsaogm_classify_ex(const vsaogm_grid_desc* g, const float* heat, const float* hmax,
                       int32_t r_occ, int32_t r_emp, float rho, int32_t normalize, int32_t square,
                       int32_t activation, float* ogm, uint8_t* label, int32_t device,
                       vsaogm_stream stream) {
    return guarded([&] {
        if (!g || g->nx < 1 || g->ny < 1) fail(VSAOGM_EINVAL, "grid nx and ny must be >= 1");
        if (!heat || !hmax || !label) fail(VSAOGM_EINVAL, "heat, hmax and label must not be NULL");
        if (r_occ < 0 || r_emp < 0 || r_occ > kMaxRadius || r_emp > kMaxRadius)
            fail(VSAOGM_EINVAL, "disk radii must be in 0..24");
        if (!std::isfinite(rho)) fail(VSAOGM_EINVAL, "rho must be finite");
        if (activation < VSAOGM_ACT_ENTROPY || activation > VSAOGM_ACT_SIGMOID)
            fail(VSAOGM_EINVAL, "unknown activation");
        int ndev = 0;
        hip_check(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
        if (device < 0 || device >= ndev) fail(VSAOGM_EINVAL, "no such device");
        DeviceGuard guard(device);
        hip_check(launch_classify(heat, hmax, g->nx, g->ny, r_occ, r_emp, rho, normalize ? 1 : 0,
                                  square ? 1 : 0, activation, ogm, label, (hipStream_t)stream),
                  "classify launch");
    });
}

int vsaogm_classify(const vsaogm_grid_desc* g, const float* heat, const float* hmax, int32_t r_occ,
                    int32_t r_emp, float rho, float* ogm, uint8_t* label, int32_t device,
                    vsaogm_stream stream) {
    return vsaogm_classify_ex(g, heat, hmax, r_occ, r_emp, rho, 1, 1, VSAOGM_ACT_ENTROPY, ogm, label,
                              device, stream);
}

int vsaogm_memories(const vsaogm_map* m, float* out, vsaogm_stream stream) {
    return guarded([&] {
        if (!m || !out) fail(VSAOGM_EINVAL, "map and out must not be NULL");
        DeviceGuard guard(m->device);
        hip_check(launch_memories_export(m->d_omega.p, m->d_theta.p, m->layout(), m->nkeys, m->half,
                                         m->halfp, out, (hipStream_t)stream),
                  "export launch");
    });
}

int vsaogm_fuse(vsaogm_map* dst, const vsaogm_map* src, vsaogm_stream stream) {
    return guarded([&] {
        if (!dst || !src) fail(VSAOGM_EINVAL, "maps must not be NULL");
        if (dst == src) fail(VSAOGM_EINVAL, "cannot fuse a map into itself");
        if (dst->device != src->device) fail(VSAOGM_EINVAL, "maps live on different devices");
        if (dst->D != src->D || dst->theta != src->theta)
            fail(VSAOGM_EINVAL, "maps must share the axis vectors (same Theta)");
        if (dst->tiles_x != src->tiles_x || dst->tiles_y != src->tiles_y || dst->x0 != src->x0 ||
            dst->y0 != src->y0 || dst->x1 != src->x1 || dst->y1 != src->y1)
            fail(VSAOGM_EINVAL, "maps must share the tiling of the global frame");
        DeviceGuard guard(dst->device);
        hip_check(launch_add(dst->d_omega.p, src->d_omega.p, dst->d_omega.n, (hipStream_t)stream),
                  "fuse launch");
        hip_check(launch_bump_versions(dst->d_version.p, dst->nkeys, (hipStream_t)stream), "versions");
    });
}

int vsaogm_fuse_many(vsaogm_map* dst, const vsaogm_map* const* srcs, int32_t n, vsaogm_stream stream) {
    return guarded([&] {
        if (!dst) fail(VSAOGM_EINVAL, "dst must not be NULL");
        if (n < 0 || (n > 0 && !srcs)) fail(VSAOGM_EINVAL, "srcs must hold n >= 0 maps");
        std::vector<const float2*> p((size_t)n);
        for (int j = 0; j < n; ++j) {
            const vsaogm_map* src = srcs[j];
            if (!src) fail(VSAOGM_EINVAL, "a source map is NULL");
            if (src == dst) fail(VSAOGM_EINVAL, "cannot fuse a map into itself");
            if (dst->device != src->device) fail(VSAOGM_EINVAL, "maps live on different devices");
            if (dst->D != src->D || dst->theta != src->theta)
                fail(VSAOGM_EINVAL, "maps must share the axis vectors (same Theta)");
            if (dst->tiles_x != src->tiles_x || dst->tiles_y != src->tiles_y || dst->x0 != src->x0 ||
                dst->y0 != src->y0 || dst->x1 != src->x1 || dst->y1 != src->y1)
                fail(VSAOGM_EINVAL, "maps must share the tiling of the global frame");
            p[(size_t)j] = src->d_omega.p;
        }
        if (n == 0) return;
        DeviceGuard guard(dst->device);
        hip_check(launch_add_many(dst->d_omega.p, p.data(), n, dst->d_omega.n, (hipStream_t)stream), "fuse launch");
        hip_check(launch_bump_versions(dst->d_version.p, dst->nkeys, (hipStream_t)stream), "versions");
    });
}

int vsaogm_profile_events(int32_t stage, void* begin_event, void* end_event) {
    return guarded([&] {
        if (stage < 0 || stage >= kNumStages) fail(VSAOGM_EINVAL, "unknown stage");
        g_profile[stage].begin = static_cast<hipEvent_t>(begin_event);
        g_profile[stage].end = static_cast<hipEvent_t>(end_event);
    });
}

int vsaogm_volume_create(const vsaogm_volume_desc* d, vsaogm_volume** out) {
    return guarded([&] {
        if (!d || !out) fail(VSAOGM_EINVAL, "desc and out must not be NULL");
        *out = nullptr;
        const int D = d->dim;
        if (D < 4 || (D & 1)) fail(VSAOGM_EINVAL, "dim must be even and >= 4");
        if (D > (1 << 22)) fail(VSAOGM_EINVAL, "dim too large");
        if (!d->theta) fail(VSAOGM_EINVAL, "theta is NULL");
        const int tn[3] = {d->tiles_x, d->tiles_y, d->tiles_z};
        for (int a = 0; a < 3; ++a)
            if (tn[a] < 1 || tn[a] > kMaxTilesPerAxis) fail(VSAOGM_EINVAL, "tiles per axis must be in 1..64");
        if (2 * tn[0] * tn[1] * tn[2] > kMaxKeys) fail(VSAOGM_EINVAL, "at most 4096 tiles");
        const double box[6] = {d->x0, d->y0, d->z0, d->x1, d->y1, d->z1};
        for (int a = 0; a < 3; ++a)
            if (!is_finite(box[a]) || !is_finite(box[3 + a]) || !(box[3 + a] > box[a]))
                fail(VSAOGM_EINVAL, "layout box must be finite with x1 > x0, y1 > y0 and z1 > z0");
        const double* th = d->theta;
        for (int k = 0; k < 3 * D; ++k)
            if (!is_finite(th[k])) fail(VSAOGM_EINVAL, "theta must be finite");
        const int half = D / 2;
        for (int a = 0; a < 3; ++a) {
            if (th[a] != 0.0 || th[3 * half + a] != 0.0) fail(VSAOGM_EINVAL, "theta[0] and theta[D/2] must be zero");
            for (int k = 1; k < half; ++k)
                if (th[3 * (D - k) + a] != -th[3 * k + a])
                    fail(VSAOGM_EINVAL, "theta must be conjugate-symmetric: theta[D-k] = -theta[k]");
        }
        int ndev = 0;   // arguments are checked before the device is touched
        hip_check(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
        if (d->device < 0 || d->device >= ndev) fail(VSAOGM_EINVAL, "no such device");
        auto v = std::make_unique<vsaogm_volume>();
        v->device = d->device;
        v->D = D;
        v->half = half;
        v->halfp = (half + kBinPad - 1) / kBinPad * kBinPad;
        v->tiles_x = tn[0];
        v->tiles_y = tn[1];
        v->tiles_z = tn[2];
        v->nkeys = 2 * tn[0] * tn[1] * tn[2];
        std::copy(box, box + 6, v->lay);
        v->cx = centres(d->x0, d->x1, tn[0]);
        v->cy = centres(d->y0, d->y1, tn[1]);
        v->cz = centres(d->z0, d->z1, tn[2]);
        std::vector<float4> rev(v->halfp, make_float4(0.f, 0.f, 0.f, 0.f));
        std::vector<double> rev_d(3 * (size_t)v->halfp, 0.0), txy(2 * (size_t)half), tz(2 * (size_t)half, 0.0);
        const double inv2pi = 1.0 / (2.0 * M_PI);
        for (int k = 0; k < half; ++k) {
            double r3[3];
            for (int a = 0; a < 3; ++a) {
                r3[a] = th[3 * k + a] * inv2pi;
                rev_d[3 * k + a] = r3[a];
                v->max_rev[a] = std::max(v->max_rev[a], (float)std::fabs(r3[a]));
            }
            rev[k] = make_float4((float)r3[0], (float)r3[1], (float)r3[2], 0.f);
            txy[2 * k] = th[3 * k];
            txy[2 * k + 1] = th[3 * k + 1];
            tz[2 * k] = th[3 * k + 2];
        }
        DeviceGuard guard(v->device);
        hip_check(hipDeviceGetAttribute(&v->num_cus, hipDeviceAttributeMultiprocessorCount, v->device),
                  "device attribute");
        if (v->num_cus < 1) v->num_cus = 1;
        v->d_cx.alloc(tn[0], "tile centres x");
        v->d_cy.alloc(tn[1], "tile centres y");
        v->d_cz.alloc(tn[2], "tile centres z");
        v->d_rev.alloc(v->halfp, "theta (rev, fp32)");
        v->d_rev_d.alloc(3 * (size_t)v->halfp, "theta (rev, fp64)");
        v->d_theta_xy.alloc(2 * (size_t)half, "theta xy");
        v->d_theta_z.alloc(2 * (size_t)half, "theta z");
        v->d_omega.alloc((size_t)v->nkeys * v->halfp, "memories");
        v->d_omega_s.alloc((size_t)v->nkeys * v->halfp, "scaled memories");
        v->d_scale.alloc(v->nkeys, "memory scales");
        v->d_hmax_u.alloc(2, "class maxima");
        v->d_bad.alloc(1, "rejected-label counter");
        hip_check(hipMemcpy(v->d_cx.p, v->cx.data(), tn[0] * 8, hipMemcpyHostToDevice), "copy");
        hip_check(hipMemcpy(v->d_cy.p, v->cy.data(), tn[1] * 8, hipMemcpyHostToDevice), "copy");
        hip_check(hipMemcpy(v->d_cz.p, v->cz.data(), tn[2] * 8, hipMemcpyHostToDevice), "copy");
        hip_check(hipMemcpy(v->d_rev.p, rev.data(), rev.size() * sizeof(float4), hipMemcpyHostToDevice), "copy");
        hip_check(hipMemcpy(v->d_rev_d.p, rev_d.data(), rev_d.size() * 8, hipMemcpyHostToDevice), "copy");
        hip_check(hipMemcpy(v->d_theta_xy.p, txy.data(), txy.size() * 8, hipMemcpyHostToDevice), "copy");
        hip_check(hipMemcpy(v->d_theta_z.p, tz.data(), tz.size() * 8, hipMemcpyHostToDevice), "copy");
        zero_async(v->d_omega.p, v->d_omega.n * sizeof(float2), nullptr);
        zero_async(v->d_bad.p, sizeof(unsigned long long), nullptr);
        hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
        *out = v.release();
    });
}

int vsaogm_volume_destroy(vsaogm_volume* v) {
    return guarded([&] {
        if (!v) return;
        DeviceGuard guard(v->device);
        (void)hipDeviceSynchronize();
        delete v;
    });
}

int vsaogm_volume_reset(vsaogm_volume* v, vsaogm_stream stream) {
    return guarded([&] {
        if (!v) fail(VSAOGM_EINVAL, "volume is NULL");
        DeviceGuard guard(v->device);
        zero_async(v->d_omega.p, v->d_omega.n * sizeof(float2), (hipStream_t)stream);
    });
}

int vsaogm_volume_encode(vsaogm_volume* v, const float* xyz, const uint8_t* label, int64_t n,
                         vsaogm_stream stream) {
    return guarded([&] {
        if (!v) fail(VSAOGM_EINVAL, "volume is NULL");
        if (n < 0) fail(VSAOGM_EINVAL, "n must be >= 0");
        if (n == 0) return;
        if (!xyz || !label) fail(VSAOGM_EINVAL, "xyz and label must not be NULL");
        if (n > ((int64_t)1 << 31) - (int64_t)kAssignChunk * 2)
            fail(VSAOGM_EINVAL, "n too large for one call");
        DeviceGuard guard(v->device);
        hipStream_t s = (hipStream_t)stream;
        const EncodePlan p = encode_plan(n, v->halfp, v->nkeys);
        if (n > v->cap_n || p.nchunks > v->cap_chunks || p.max_echunks > v->cap_echunks) {
            const int64_t cap = std::max<int64_t>(n + n / 2, 4096);
            const EncodePlan q = encode_plan(cap, v->halfp, v->nkeys);
            const int chunks = std::max(q.nchunks, p.nchunks), echunks = std::max(q.max_echunks, p.max_echunks);
            v->w_key.alloc_async(cap, s, "volume keys");
            v->w_sorted.alloc_async(cap, s, "volume sorted local coordinates");
            v->w_sorted_lo.alloc_async(cap, s, "volume sorted residuals");
            // the scan reads the histogram in aligned groups of kHistPad entries
            v->w_hist.alloc_async((size_t)chunks * v->nkeys + kHistPad, s, "volume histogram");
            v->w_table.alloc_async(echunks, s, "volume work table");
            v->w_partial.alloc_async((size_t)echunks * v->halfp, s, "volume partial spectra");
            if (!v->w_meta.p) v->w_meta.alloc_async(1 + 3 * (size_t)v->nkeys, s, "volume encode meta");
            v->cap_n = cap;
            v->cap_chunks = chunks;
            v->cap_echunks = echunks;
        }
        Volume3Dev V{v->d_cx.p, v->d_cy.p, v->d_cz.p, v->tiles_x, v->tiles_y, v->tiles_z, v->lay[0], v->lay[1],
                     v->lay[2], (v->lay[3] - v->lay[0]) / v->tiles_x, (v->lay[4] - v->lay[1]) / v->tiles_y,
                     (v->lay[5] - v->lay[2]) / v->tiles_z};
        Encode3Work w{v->w_key.p, v->w_sorted.p, v->w_sorted_lo.p, v->w_hist.p, v->w_table.p, v->w_meta.p,
                      v->w_partial.p, v->d_bad.p};
        hip_check(launch_encode3(xyz, label, n, V, v->d_rev.p, v->d_rev_d.p,
                                 make_float4(v->max_rev[0], v->max_rev[1], v->max_rev[2], 0.f), v->nkeys, v->half,
                                 v->halfp, w, v->d_omega.p, s),
                  "volume encode");
    });
}

int vsaogm_volume_take_rejected(vsaogm_volume* v, vsaogm_stream stream, int64_t* n_rejected) {
    return guarded([&] {
        if (!v || !n_rejected) fail(VSAOGM_EINVAL, "volume and n_rejected must not be NULL");
        DeviceGuard guard(v->device);
        hipStream_t s = (hipStream_t)stream;
        unsigned long long c = 0;
        hip_check(hipMemcpyAsync(&c, v->d_bad.p, sizeof(c), hipMemcpyDeviceToHost, s), "read counter");
        hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
        zero_async(v->d_bad.p, sizeof(c), s);
        *n_rejected = (int64_t)c;
    });
}

int vsaogm_volume_decode(vsaogm_volume* v, const vsaogm_grid3_desc* g, int32_t precision, float* heat,
                         float* hmax, vsaogm_stream stream) {
    return guarded([&] {
        if (!v) fail(VSAOGM_EINVAL, "volume is NULL");
        check_grid3(g);
        if (!heat || !hmax) fail(VSAOGM_EINVAL, "heat and hmax must not be NULL");
        if (precision != VSAOGM_BF16 && precision != VSAOGM_FP16 && precision != VSAOGM_BF16X3)
            fail(VSAOGM_EINVAL, "volumes decode with VSAOGM_BF16, VSAOGM_FP16 or VSAOGM_BF16X3");
        DeviceGuard guard(v->device);
        hipStream_t s = (hipStream_t)stream;
        Grid3Cache* gc = grid3_cache(v, g, s);
        const size_t n16 = (size_t)rows16(gc->nrows) * 2 * v->halfp;
        const void* ey = nullptr;
        const void* ey_lo = nullptr;
        auto table = [&](DevBuf<uint16_t>& hi, DevBuf<uint16_t>* lo, bool fp16, const char* what) {
            hi.alloc(n16, what);
            if (lo) lo->alloc(n16, what);
            hip_check(launch_table_yz_split(v->d_theta_xy.p, v->d_theta_z.p, gc->local_y.p, gc->local_z.p,
                                            gc->row_map.p, gc->nrows, g->ny, v->half, v->halfp, fp16, hi.p,
                                            lo ? lo->p : nullptr, s),
                      what);
        };
        if (precision == VSAOGM_FP16) {
            if (!gc->eyz_h.p) table(gc->eyz_h, nullptr, true, "joint (z, y) table (fp16)");
            ey = gc->eyz_h.p;
        } else {
            if (!gc->eyz_bf.p) table(gc->eyz_bf, &gc->eyz_bf_lo, false, "joint (z, y) table (bf16 hi + lo)");
            ey = gc->eyz_bf.p;
            if (precision == VSAOGM_BF16X3) ey_lo = gc->eyz_bf_lo.p;
        }
        const int set = decode_tile_set(precision);
        DecodeLaunch d;
        d.plan = decode_plan(precision, gc->ntiles[set], v->halfp, v->num_cus);
        const size_t need = set_units(d, gc->uplan[set], gc->dunits[set], gc->ntiles[set]);
        if (v->d_partial.n < need) v->d_partial.alloc_async(need, s, "decode partial sums");
        hip_check(launch_norm(v->d_omega.p, v->nkeys, v->half, v->halfp, v->D, v->d_scale.p, v->d_omega_s.p,
                              v->d_hmax_u.p, s),
                  "norm launch");
        d.tiles = gc->tiles[set].p;
        d.ntiles = gc->ntiles[set];
        d.col_tx = gc->col_tx.p;
        d.ex = gc->ex32.p;
        d.ey = ey;
        d.ey_lo = ey_lo;
        d.omega_s = v->d_omega_s.p;
        d.halfp = v->halfp;
        d.nx = g->nx;
        d.ny = g->ny;
        d.tiles_x = v->tiles_x;
        d.out_scale = (float)(2.0 / (double)v->D);
        d.heat = heat;
        d.class_stride = (size_t)g->nx * g->ny * g->nz;
        d.row_map = gc->row_map.p;
        d.hmax_u = v->d_hmax_u.p;
        d.hmax = hmax;
        d.partial = v->d_partial.p;
        hip_check(launch_decode(precision, d, s), "volume decode launch");
    });
}

int vsaogm_classify3(const vsaogm_grid3_desc* g, const float* heat, const float* hmax, int32_t r_occ,
                     int32_t r_emp, float rho, float* ogm, uint8_t* label, int32_t device, vsaogm_stream stream) {
    return guarded([&] {
        check_grid3(g);
        if (!heat || !hmax || !label) fail(VSAOGM_EINVAL, "heat, hmax and label must not be NULL");
        if (r_occ < 0 || r_emp < 0 || r_occ > kMaxRadius || r_emp > kMaxRadius)
            fail(VSAOGM_EINVAL, "radii must be in 0..24");
        if (!is_finite(rho)) fail(VSAOGM_EINVAL, "rho must be finite");
        DeviceGuard guard(device);
        hipStream_t s = (hipStream_t)stream;
        const size_t nvox = (size_t)g->nx * g->ny * g->nz;
        float* gbuf = nullptr;   // entropy scratch, only for radii beyond the tiled kernel's
        if (std::max(r_occ, r_emp) > kClassify3TiledRadius)
            hip_check(hipMallocAsync((void**)&gbuf, 2 * nvox * sizeof(float), s), "classify scratch");
        const hipError_t e = launch_classify3(heat, hmax, g->nx, g->ny, g->nz, r_emp, r_occ, rho, gbuf, ogm, label, s);
        if (gbuf) (void)hipFreeAsync(gbuf, s);
        hip_check(e, "classify launch");
    });
}

}  // extern "C"

// ---- allocation-free volume classification -------------------------------------------------
// vsaogm_classify3_noalloc keeps the entropy terms of the two-pass path (radii above the tiled
// kernel's) in this file-scope device array instead of a stream-ordered allocation.  Host code
// never uses the array's name as an address: each device's copy is found once with
// hipGetSymbolAddress (with that device current) and the kernels receive that pointer.
namespace {
constexpr int64_t kNoAllocVoxels = int64_t(1) << 21;   // 2 floats per voxel: 16 MiB per device
constexpr int kNoAllocMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kNoAllocMaxDevices] = {};
}  // namespace

static __device__ __align__(256) float scratch[2 * kNoAllocVoxels];

namespace {
// The calling thread's current device must be `device`.
float* scratch_on_device(int device) {
    if (device < 0 || device >= kNoAllocMaxDevices) fail(VSAOGM_EINVAL, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "scratch symbol address");
        if (!ptr) fail(VSAOGM_EDEVICE, "scratch symbol address is NULL");
        g_scratch_ptr[device] = static_cast<float*>(ptr);
    }
    return g_scratch_ptr[device];
}
}  // namespace

extern "C" {

int vsaogm_classify3_noalloc(const vsaogm_grid3_desc* g, const float* heat, const float* hmax, int32_t r_occ,
                             int32_t r_emp, float rho, float* ogm, uint8_t* label, int32_t device,
                             vsaogm_stream stream) {
    return guarded([&] {
        check_grid3(g);
        if (!heat || !hmax || !label) fail(VSAOGM_EINVAL, "heat, hmax and label must not be NULL");
        if (r_occ < 0 || r_emp < 0 || r_occ > kMaxRadius || r_emp > kMaxRadius)
            fail(VSAOGM_EINVAL, "radii must be in 0..24");
        if (!is_finite(rho)) fail(VSAOGM_EINVAL, "rho must be finite");
        const int64_t nvox = (int64_t)g->nx * g->ny * g->nz;
        const bool two_pass = std::max(r_occ, r_emp) > kClassify3TiledRadius;
        if (two_pass && nvox > kNoAllocVoxels)
            fail(VSAOGM_EINVAL, "vsaogm_classify3_noalloc: radii above 4 need nx*ny*nz <= 2097152 voxels "
                                "(the fixed scratch holds 2 floats per voxel)");
        DeviceGuard guard(device);
        hipStream_t s = (hipStream_t)stream;
        float* gbuf = two_pass ? scratch_on_device(device) : nullptr;
        hip_check(launch_classify3(heat, hmax, g->nx, g->ny, g->nz, r_emp, r_occ, rho, gbuf, ogm, label, s),
                  "classify launch");
    });
}

}  // extern "C"
