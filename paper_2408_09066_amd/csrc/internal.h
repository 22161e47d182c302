// Internal declarations of the gfx950 VSA-OGM library: launch helpers and the
// small structs the kernels share.  Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <cstddef>
#include <cstdint>
#include <vector>

#include "vsaogm.h"

namespace vsaogm {

constexpr int kMaxTilesPerAxis = 64;
constexpr int kMaxKeys = 2 * kMaxTilesPerAxis * kMaxTilesPerAxis;  // 8192 memories
constexpr int kAssignChunk = 1024;   // points per histogram / stable-scatter chunk
constexpr int kHistPad = 16;         // entries of padding after a key histogram (aligned group reads)
constexpr int kEncodeChunk = 512;    // points per encode work item (even, so pairs never straddle)
constexpr int kEncodeThreads = 256;
constexpr int kEncodeBpt = 2;        // spectrum bins per encode thread (at most)
constexpr int kBinPad = 64;          // stored half spectra are padded to a multiple of this
constexpr int kMaxRadius = 24;       // largest disk radius of the entropy filter
// A phase bound (revolutions) above which a chunk is encoded with double-precision
// phases; below it single precision keeps the phase error under ~4e-6 revolutions.
constexpr float kWidePhaseRev = 64.0f;

// Lanes of this wavefront holding the same value v < 2^bits as this lane, as a mask (one ballot
// per bit).  Every lane of the wavefront must take part; the result includes inactive lanes
// only if they are, so callers run it with the whole wavefront active.
__device__ inline uint64_t same_value_lanes(unsigned v, int bits) {
    uint64_t same = ~0ull;
    for (int b = 0; b < bits; ++b) {
        const bool bit = (v >> b) & 1u;
        const uint64_t m = __ballot(bit);
        same &= bit ? m : ~m;
    }
    return same;
}

// Pointers into global memory (address space 1), so that loads and stores through pointers
// read from a descriptor (batched launches) still compile to global, not flat, instructions.
// The qualifier only exists in the device pass; the host pass parses the same bodies with plain
// pointers (it compiles no device code).
#if defined(__HIP_DEVICE_COMPILE__)
template <class T>
using gmem = const __attribute__((address_space(1))) T;
template <class T>
using gmem_rw = __attribute__((address_space(1))) T;
#else
template <class T>
using gmem = const T;
template <class T>
using gmem_rw = T;
#endif
template <class T>
__device__ inline gmem<T>* as_global(const T* p) {
    return (gmem<T>*)p;
}
template <class T>
__device__ inline gmem_rw<T>* as_global_rw(T* p) {
    return (gmem_rw<T>*)p;
}

// Monotone map float -> unsigned so that unsigned max = float max (class maxima by atomicMax).
__device__ inline unsigned order_key(float f) {
    unsigned u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float order_value(unsigned u) {
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

// Tile layout as the kernels see it.  Centres are computed on the host in double
// precision, cx[tx] = x0 + (tx + 0.5) * (x1 - x0) / tiles_x.
struct LayoutDev {
    double x0, y0;
    double inv_wx, inv_wy;  // used only to guess the nearest tile before the exact check
    int tiles_x, tiles_y;
    const double* cx;       // [tiles_x]
    const double* cy;       // [tiles_y]
};

// One encode work item: a run of points of one memory (key) in the sorted buffer.
struct EChunk {
    int key;
    int start;
    int len;
    int pad;
};

// One decode work tile: up to kDecodeSetRowBlocks[decode_tile_set(precision)] blocks of 16 rows
// of one tile band (rows whose cells share a tile row) by 64 consecutive grid columns, both
// classes.  Tile sets: 0 fp32 operands, 1 bf16 / fp16, 2 bf16 hi+lo.
constexpr int kDecodeTileSets = 3;
constexpr int kDecodeSetRowBlocks[kDecodeTileSets] = {7, 16, 16};
inline int decode_tile_set(int precision) { return precision == 0 ? 0 : (precision == 3 ? 2 : 1); }
struct DTile {
    int ty;           // tile row of the band
    int row0;         // first grid row of the block
    int row_end;      // one past the band's last row
    int nrb;          // row blocks of 16 in this tile (1..kDecodeSetRowBlocks of its set)
    int col0;         // first grid column
    int ncol;         // columns of this tile (1..64)
    int tx0;          // tile column of its first column; 16-bit tiles span at most tx0, tx0 + 1
    int pad;          // unused (keeps the record 32 bytes)
};

// Rows of one band of decode work: its memories are those of tile row key_row (for volumes
// tz * tiles_y + ty), its rows [row0, row1) (grid rows of a map; joint (z, y) rows of a volume).
struct DBand {
    int key_row, row0, row1;
};
// Work tiles of a tile set over the bands, the grid's columns with their tile columns tcol.
std::vector<DTile> build_decode_tiles(const std::vector<DBand>& bands, const std::vector<int>& tcol, int nx,
                                      int set);

// ---- volumes (volume.hip) -------------------------------------------------------------
struct Volume3Dev {
    const double* cx;   // [tx] tile centres per axis
    const double* cy;   // [ty]
    const double* cz;   // [tz]
    int tx, ty, tz;
    double x0, y0, z0, wx, wy, wz;   // layout origin and tile widths
};
// Volume encode workspace: keys [n], local coordinates sorted by key (fp32 and residual,
// (x, y, z, 0)) [n], histogram / table / meta / partial spectra as for planes (encode_plan).
struct Encode3Work {
    int* key;
    float4* sorted;
    float4* sorted_lo;
    int* hist;
    EChunk* table;
    int* meta;
    float2* partial;
    unsigned long long* n_bad;
};
// Bucketing, encoding and bundling of n labelled points into omega [nkeys][halfp] (local frame).
// rev: fp32 [halfp] (x, y, z, 0) revolutions per metre, 0 past half; rev_d: double [halfp][3].
hipError_t launch_encode3(const float* xyz, const uint8_t* label, int64_t n, const Volume3Dev& V,
                          const float4* rev, const double* rev_d, float4 max_rev, int nkeys, int half,
                          int halfp, const Encode3Work& w, float2* omega, hipStream_t s);
// Ball entropy classification of a volume's heat [2][nz][ny][nx].  Radii up to
// kClassify3TiledRadius run in one kernel through LDS (g unused, may be NULL); larger radii need g,
// 2*nvox floats of scratch.
constexpr int kClassify3TiledRadius = 4;
hipError_t launch_classify3(const float* heat, const float* hmax, int nx, int ny, int nz, int r_emp, int r_occ,
                            float rho, float* g, float* ogm, uint8_t* label, hipStream_t s);

// ---- batched map updates (map.hip) ------------------------------------------------------
// One whole map update: bundle n points into the map, decode its grid, classify it.  Device
// pointers; ogm may be null.
struct UpdateItem {
    vsaogm_map* map;
    const float* xy;          // device inputs, or
    const uint8_t* label;
    const void* host_in;      // pinned host [n][2] float32 points then [n] labels, staged with
                              // the batch's descriptors (one copy for the batch)
    int64_t n;
    vsaogm_grid_desc grid;
    int32_t r_occ, r_emp;
    float rho;
    float* heat;        // [2][ny][nx]
    float* hmax;        // [2]
    float* ogm;         // [ny][nx] or null
    uint8_t* label_out; // [ny][nx]
};
struct UpdateBatchWork;   // staging and device buffers of one in-flight batch
UpdateBatchWork* update_batch_work_create();
void update_batch_work_destroy(UpdateBatchWork* w);
int64_t update_batch_work_bytes(const UpdateBatchWork* w);   // device bytes it holds
void update_batch_work_trim(UpdateBatchWork* w);             // release them (nothing in flight)
// count updates of distinct maps on one device as one launch per stage (precision: a 16-bit
// format), asynchronously on s.  Results equal the same updates through vsaogm_encode,
// vsaogm_decode and vsaogm_classify up to the order of the similarity's fp32 accumulation (the
// stream-K split of the K loop depends on the batch).  w must not be reused before s passes the
// batch.  Returns a vsaogm_status (message in vsaogm_last_error).
int run_update_batch(const UpdateItem* items, int count, int precision, hipStream_t s, UpdateBatchWork* w);

// ---- error text shared by every entry point (map.hip) -------------------------------
void set_last_error(const char* msg);

// ---- profiling hook (map.hip) --------------------------------------------------------
enum ProfileStage { kStageEncode = 0, kStageDecode = 1, kStageClassify = 2, kNumStages = 3 };
// The events a stage is being timed with (NULL when it is not): the stage's first kernel is
// launched with the start event and its last with the stop event through hipExtLaunchKernelGGL,
// so that the dispatches record them themselves (no marker packets between kernels).
hipEvent_t profile_start(int stage);
hipEvent_t profile_stop(int stage);

// ---- encode (encode.hip) -----------------------------------------------------------
struct EncodeWork {
    int* key;            // [cap_n]
    float2* sorted;      // [cap_n] tile-local coordinates, grouped by key
    float2* sorted_lo;   // [cap_n] rounding residuals of the local coordinates
    int* hist;           // [nkeys][cap_chunks] per-chunk key counts, then bases
    EChunk* table;       // [cap_echunks]
    int* meta;           // [1 + 3 * nkeys]: n_echunks, key_ec_start[nkeys], key_ec_count[nkeys], key_count[nkeys]
    float2* partial;     // [cap_echunks][halfp]
    unsigned long long* n_bad;
    unsigned* version;   // [nkeys] bumped for every memory that receives points
};

// Everything one map's encode chain (assign, scan, scatter, encode, reduce) and its memory norm
// need: the kernels take it by value for one map, or read it from a device array in a batched
// launch that covers the encodes of several maps (one request each) with one dispatch per stage.
struct EncodeReq {
    const float2* xy;                 // [n] world metres
    const uint8_t* label;             // [n]
    int64_t n;
    LayoutDev L;
    int nkeys, key_bits;
    int nchunks, echunk, max_echunks, binblocks, bpt;   // encode_plan
    int* key;
    int* hist;
    EChunk* table;
    int* meta;
    float2* sorted;
    float2* sorted_lo;
    float2* partial;
    unsigned long long* n_bad;
    unsigned* version;
    const float2* rev;
    const double2* rev_d;
    float max_rev_x, max_rev_y;
    int half, halfp, D;
    // the encode adds the sums of a memory that has one work item straight into it (the
    // reduction then skips that memory); 0 where the encode writes every work item's partials
    int direct_single;
    float2* omega;                    // [nkeys][halfp] local-frame memories
    float* scale;                     // norm: [nkeys] 1/||w||
    float2* omega_s;                  // norm: [nkeys][halfp] conj(Omega)/||w||
    unsigned* hmax_u;                 // norm: [2] ordered class maxima, zeroed
};

// Batched launches: job r covers blocks [block0[r], block0[r+1]) of a stage's grid; the job of
// block b is the last r with block0[r] <= b (jobs with no blocks are passed over).
__device__ inline int batch_job(const int* __restrict__ block0, int njobs, int b) {
    int lo = 0, hi = njobs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (block0[mid] <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Stages of a batched encode: assign, scan, scatter, encode, reduce, norm.
constexpr int kEncodeStages = 6;
struct EncodeBatch {
    const EncodeReq* reqs;            // device [nreq]
    const int* block0;                // device [kEncodeStages][nreq + 1] block prefixes
    int nreq;
    int blocks[kEncodeStages];        // total blocks per stage
    int max_keys;                     // largest nkeys (dynamic LDS)
    int bpt;                          // bins per encode thread, the same for every request
};
hipError_t launch_encode_batch(const EncodeBatch& b, hipStream_t s);
// Blocks of each stage for one request (0 for the encode stages when it has no points).
void encode_batch_blocks(const EncodeReq& q, int out[kEncodeStages]);

// Launch geometry of one encode, shared by the host (buffer sizing) and the launcher.
struct EncodePlan {
    int nchunks;      // histogram / scatter chunks of kAssignChunk points
    int bpt;          // bins per encode thread
    int binblocks;    // bin blocks of kEncodeThreads * bpt bins
    int echunk;       // points per encode work item (even)
    int max_echunks;  // upper bound on work items: ceil(n / echunk) + nkeys
};
EncodePlan encode_plan(int64_t n, int halfp, int nkeys);

// Shared by plane and volume encodes.  hist: key-major per-chunk key counts [nkeys][nchunks]
// (+4 padding), turned in place into the stable counting sort's destination bases; then per
// key its point count and work items of at most echunk points (table, meta as in EncodeWork;
// version, if not NULL, is bumped for every key that received points).  One block.
void launch_key_scan(int* hist, int nchunks, int nkeys, int echunk, EChunk* table, int* meta, unsigned* version,
                     hipStream_t s);
// omega[key] += the key's work-item partial spectra in work-item order.  With direct_single, keys
// with exactly one work item are skipped (their encode added its sums into omega itself).
void launch_key_reduce(const float2* partial, const int* meta, int nkeys, int half, int halfp, int direct_single,
                       float2* omega, hipStream_t s);

hipError_t launch_encode(const float* xy, const uint8_t* label, int64_t n, const LayoutDev& L,
                         int nkeys, const float2* theta_rev, const double* theta_rev_d,
                         float max_rev_x, float max_rev_y, int half, int halfp,
                         const EncodeWork& w, float2* omega, hipStream_t s);
// The request launch_encode runs (the norm fields are left for the caller).
EncodeReq encode_req(const float* xy, const uint8_t* label, int64_t n, const LayoutDev& L, int nkeys,
                     const float2* theta_rev, const double* theta_rev_d, float max_rev_x, float max_rev_y,
                     int half, int halfp, const EncodeWork& w, float2* omega);

// inv_norm[key] = 1/||w_key|| (0 for an empty memory) and omega_s = conj(Omega) * inv_norm.
// Also zeroes hmax_u[0..1], the ordered class maxima of the decode that follows.
hipError_t launch_norm(const float2* omega, int nkeys, int half, int halfp, int D, float* inv_norm,
                       float2* omega_s, unsigned* hmax_u, hipStream_t s);

hipError_t launch_memories_export(const float2* omega, const double* theta_rad, const LayoutDev& L,
                                  int nkeys, int half, int halfp, float* out, hipStream_t s);

hipError_t launch_add(float2* dst, const float2* src, size_t n, hipStream_t s);
// dst[i] += srcs[0][i] + ... in source order (as nsrc pairwise launch_add calls would add), one
// launch per kFuseSources sources.
constexpr int kFuseSources = 16;
hipError_t launch_add_many(float2* dst, const float2* const* srcs, int nsrc, size_t n, hipStream_t s);
hipError_t launch_bump_versions(unsigned* version, int nkeys, hipStream_t s);

// ---- decode (decode.hip) -----------------------------------------------------------
// Location tables: tab[c][k] = exp(i * Theta_axis[k] * local[c]) for k < half, 0 for
// half <= k < halfp; computed in double precision.  Stored as fp32 complex pairs.
hipError_t launch_table_f32(const double* theta_rad, int axis, const double* local, int ncells,
                            int half, int halfp, float2* tab, hipStream_t s);
// Same table split into bf16 (or fp16) hi and lo parts, hi and lo tables of rows16(ncells) x
// 2*halfp elements each, in the matrix-core operand order of the 16-bit decode (decode.hip); the
// rows past ncells are zero.
// Joint (z, y) table of a volume, 16-bit, rows16(nrows) x 2 halfp (+ residual when lo is given),
// same order: row r is the voxel plane offset row_map[r] = slice * ny + y.  theta_xy [half][2],
// theta_z [half][2] rad/m.
hipError_t launch_table_yz_split(const double* theta_xy, const double* theta_z, const double* local_y,
                                 const double* local_z, const int* row_map, int nrows, int ny, int half, int halfp,
                                 bool fp16, uint16_t* hi, uint16_t* lo, hipStream_t s);
hipError_t launch_table_split(const double* theta_rad, int axis, const double* local, int ncells,
                              int half, int halfp, bool fp16, void* hi, void* lo, hipStream_t s);

// Rows of a 16-bit row table of n rows (whole blocks of 32).
__host__ __device__ constexpr int rows16(int n) { return (n + 31) / 32 * 32; }

struct DUnit {
    int tile, kb0, kb1;
    int part;   // partial-sum block, used when the unit is not a whole tile
};

// One request of a batched similarity GEMM (the per-map, per-grid fields of a decode).
struct DecodeReq {
    const int* col_tx;
    const float2* ex;
    const void* ey;
    const void* ey_lo;
    const float2* omega_s;
    int halfp, nx, ny, tiles_x;
    float out_scale;
    float* heat;
    size_t class_stride;
    const int* row_map;
    unsigned* hmax_u;
    int ksteps;
};

// Stream-K launch geometry of the similarity GEMM.
struct DecodePlan {
    int ksteps;            // K steps per tile
    int steps_per_wg;      // contiguous (tile, K step) iterations per workgroup
    int grid;              // workgroups
    long long total_steps; // tiles * ksteps
};
DecodePlan decode_plan(int precision, int ntiles, int halfp, int num_cus);
// Work units of the 16-bit similarity GEMM: a K range of one tile.  Each workgroup runs a
// range of consecutive K steps of the request (whole tiles, or equal ranges when that balances
// the CUs better), one unit per tile the range touches; a unit that is part of a tile writes
// partial block DUnit::part (2w or 2w + 1 for the request's workgroup w).  A request's units
// depend only on its own tile count and K steps, so its fp32 accumulation order is the same
// whether it is decoded alone or in a batch.  Appends the units of tiles tile_base ..
// tile_base + ntiles - 1 (numbered from unit_base), each tile's first unit and each
// workgroup's first unit; the caller appends the closing entries of tile_u0 and wg_u0.
void decode_units(int ntiles, int ksteps, int num_cus, int tile_base, int unit_base, std::vector<DUnit>& units,
                  std::vector<int>& tile_u0, std::vector<int>& wg_u0);
size_t decode_unit_partial_floats(int nblocks);   // partial-sum blocks of split tiles

// A batched 16-bit similarity GEMM: tiles of several requests (DTile::pad = request index).
struct DecodeBatch {
    const DTile* tiles;        // device [ntiles]
    int ntiles;
    const DecodeReq* reqs;     // device [requests]
    const DUnit* units;        // device [nunits]
    int nunits;
    const int* tile_u0;        // device [ntiles + 1]
    const int* wg_u0;          // device [nwg + 1]
    int nwg;                   // workgroups of the GEMM
    float* partial;            // decode_unit_partial_floats(partial blocks) when any_split
    bool any_split;            // some tile has several units (a fix-up pass runs)
};
hipError_t launch_decode_batch(int precision, const DecodeBatch& b, hipStream_t s);
size_t decode_partial_floats(int precision, const DecodePlan& plan);  // 0 when no tile is split

struct DecodeLaunch {
    const DTile* tiles;
    int ntiles;
    const int* col_tx;
    const float2* ex;       // fp32 [nx][halfp]
    const void* ey;         // fp32 [ny][halfp] (FP32) or 16-bit [ny][2*halfp]
    const void* ey_lo;      // bf16 residual table (BF16X3) or null
    const float2* omega_s;  // conj(Omega) / ||w||, [nkeys][halfp]
    int halfp, nx, ny, tiles_x;
    float out_scale;        // 2 / D
    float* heat;
    size_t class_stride = 0;   // floats between the class planes of heat (0: nx * ny)
    const int* row_map = nullptr;  // volumes: voxel plane offset of every joint (z, y) row (16-bit kernels only)
    unsigned* hmax_u;       // zeroed by launch_norm
    float* hmax;
    float* partial;         // fp32: decode_partial_floats(precision, plan); 16-bit: decode_unit_partial_floats
    DecodePlan plan;        // fp32 kernel
    const DUnit* units = nullptr;   // 16-bit kernels: work units (decode_units), each tile's
    int nunits = 0;                 // first unit [ntiles + 1] and each workgroup's [nwg + 1]
    const int* tile_u0 = nullptr;
    const int* wg_u0 = nullptr;
    int nwg = 0;
    bool any_split = false;
    // Localized decode: the counts come from the device (an IncPlan's dyn) and ntiles, nwg and
    // plan.grid are upper bounds for the grids; fix_tiles bounds the tiles a fix-up may touch.
    const int* dyn = nullptr;
    int fix_tiles = 0;
};
// Similarity GEMM over the tile list (precision: 0 fp32, 1 bf16, 2 fp16, 3 bf16 hi+lo).
// With hmax_u == nullptr no class maxima are folded and hmax is not written.
hipError_t launch_decode(int precision, const DecodeLaunch& d, hipStream_t s);

// Per-region class maxima of a heatmap, for localized decoding: the ordered maxima (order_key)
// region_u[beta][psi] of the *nboxes_dev listed regions (max_boxes at most) are raised to the
// maxima of their cells (the entries start from 0, which no cell value maps to), then
// hmax[psi] = max over all nregions regions (-inf if none has a cell).
struct RegionBox {
    int beta, row0, row1, col0, col1, pad[3];
};
hipError_t launch_region_max_dyn(const float* heat, int nx, int ny, const RegionBox* boxes, const int* nboxes_dev,
                                 int max_boxes, unsigned* region_u, int nregions, float* hmax, hipStream_t s);

// Plan of a localized decode, made on the device so that the host never waits for the memory
// versions: the regions whose memories changed since the last localized decode (or all),
// the tiles touching them and the GEMM's work units over those tiles (the cut of
// decode_units for the 16-bit kernels; steps per workgroup for the fp32 kernel).
struct IncPlan {
    const unsigned* version;   // [2 nregions] memory versions
    unsigned* seen;            // [2 nregions] versions at the last localized decode (updated)
    int all;                   // every region counts as changed
    int nregions, tiles_x;
    const DTile* tiles;        // the grid's full tile list [ntiles]
    int ntiles;
    const int* col_tx;         // tile column of every grid column
    const RegionBox* boxes;    // [nregions] cell range of every region
    int ksteps16, ksteps32;    // K steps per tile of the 16-bit and fp32 kernels
    int slots16, slots32;      // resident workgroups of the 16-bit and fp32 kernels
    DTile* out_tiles;          // [ntiles] changed tiles
    RegionBox* out_boxes;      // [nregions] changed regions
    unsigned* region_u;        // [nregions][2] ordered region maxima: the changed regions' zeroed
    DUnit* units;              // [ntiles + slots16] 16-bit work units
    int* tile_u0;              // [ntiles + 1]
    int* wg_u0;                // [max(ntiles, slots16) + 1]
    int* dyn;                  // [4]: changed tiles, 16-bit workgroups, changed regions, fp32 steps per workgroup
};
hipError_t launch_inc_plan(const IncPlan& p, hipStream_t s);
// Resident workgroups of the 16-bit and fp32 GEMMs on num_cus CUs (the plans' slot counts).
int decode_slots16(int num_cus);
int decode_slots32(int num_cus);
// Largest partial-sum block any decode of a map needs (full or localized, any precision).
size_t decode_partial_floats_max(int num_cus);

// ---- device memory of a map (the request loop's budget) ----------------------------------
// Bytes of device memory the map holds now: memories, workspaces, partial sums, every cached
// grid (tables, tile lists, localized-decode state).
int64_t map_resident_bytes(const vsaogm_map* m);
// Upper bound on the bytes one update (n points, decode of grid g at precision, localized or
// not) can add to map_resident_bytes: a new grid cache or table format, workspace growth.
int64_t map_growth_bytes(const vsaogm_map* m, const vsaogm_grid_desc* g, int precision, int64_t n, bool local);
// Release what the map rebuilds on demand (grid caches, encode workspace, partial sums); the
// memories stay.  The caller makes sure no work on the map is in flight.
void map_trim(vsaogm_map* m);

// ---- classify (classify.hip) -------------------------------------------------------
// One request of a batched classification (entropy decoding, Sec. III-B defaults).
struct ClassifyReq {
    const float* heat;         // [2][ny][nx]
    const unsigned* hmax_u;    // [2] ordered class maxima of the decode
    float* hmax_out;           // [2] the maxima as floats, or null
    int nx, ny, r_occ, r_emp;
    float rho;
    float* ogm;                // [ny][nx] or null
    uint8_t* label;            // [ny][nx]
};
int classify_blocks(int nx, int ny);
hipError_t launch_classify_batch(const ClassifyReq* reqs, const int* block0, int nreq, int total_blocks, int max_radius,
                                 hipStream_t s);
// act: 0 entropy (disk radii used), 1 ReLU, 2 tanh, 3 sigmoid (per cell)
hipError_t launch_classify(const float* heat, const float* hmax, int nx, int ny, int r_occ,
                           int r_emp, float rho, int normalize, int square, int act, float* ogm,
                           uint8_t* label, hipStream_t s);

}  // namespace vsaogm
