// Decoding: similarity of every grid cell with the normalised memories of its tile
// (Sec. III-B eqs. vector-normalization and loc-query) on gfx950 matrix cores.
//
// The location vector of cell c = (x, y) has the spectrum exp(i*Theta[k].c), which factors
// per axis: exp(i*Theta_x[k]*x) * exp(i*Theta_y[k]*y).  In tile-local coordinates, and
// using the conjugate symmetry of the spectra, the similarity of cell (row y, column x)
// of tile beta with memory key = 2*beta+psi is
//   P[psi][y][x] = (2/D) * sum_{k < D/2} Re( conj(Omega[key][k]) / ||w_key|| * Ex[x][k] * Ey[y][k] )
// Written over real and imaginary parts this is a real contraction of length D:
//   L[y][2k] = Re Ey[y][k],  L[y][2k+1] = Im Ey[y][k]
//   R[x][2k] = Re(conj(Om) Ex[x][k]) / ||w||,  R[x][2k+1] = -Im(conj(Om) Ex[x][k]) / ||w||
//   P = (2/D) * L . R^T
// so the heatmaps are dense GEMMs run on MFMA.  The per-axis tables Ex, Ey (the paper's
// precomputed location vectors, factored) are built once per grid in double precision; the
// memory factor conj(Omega)/||w|| is applied to R while it is staged into LDS, which also
// keeps R of order one for the 16-bit formats.
//
// Work layout.  Rows of one tile band (cells sharing a tile row) are grouped in blocks of
// 16; a work tile is up to kRowBlocks row blocks of one band by 64 consecutive grid columns
// (the columns may belong to different tiles: each column stages its own memory).  Each of
// the 4 waves owns one 16-column block and all row blocks, for both classes.  The K loop
// (the spectrum) is split "stream-K" style: the (tile, K step) iteration space is cut into
// equal contiguous ranges, one per workgroup, so every CU gets the same work however few
// tiles there are.  A tile finished by one workgroup is stored from registers; a tile split
// across workgroups is written as partial sums that a second kernel adds in workgroup order
// (deterministic) and stores.  Nothing in the GEMM waits on another workgroup: a device-scope
// fence on this multi-XCD part writes back and invalidates the whole L2 of the XCD, which
// would evict the location tables of every resident workgroup.  Every store folds the class
// maxima (eq. non-linearities) into order-preserving unsigned atomics; a one-block kernel
// converts them once all stores are done.
#include <algorithm>
#include <type_traits>

#include "internal.h"

namespace vsaogm {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

// Two floats to packed bf16 / fp16 (round to nearest even; v_cvt_pk_* on gfx950).
__device__ inline uint32_t pack_bf16(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{a, b}, bf16x2));
}
__device__ inline uint32_t pack_f16(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{a, b}, f16x2));
}
// The residuals a - bf16(a), b - bf16(b) of a packed pair, packed again.
__device__ inline uint32_t pack_bf16_lo(float a, float b, uint32_t hi) {
    const float ha = __uint_as_float(hi << 16), hb = __uint_as_float(hi & 0xffff0000u);
    return pack_bf16(a - ha, b - hb);
}

constexpr int kRowBlocks = kDecodeSetRowBlocks[0];
constexpr int kTileRows = 16 * kRowBlocks;
constexpr int kTileCols = 64;
constexpr int kRowPitchBytes = 144;  // LDS row: 128 data bytes + 16 padding

__global__ __launch_bounds__(256) void k_table_f32(const double* __restrict__ theta_rad, int axis,
                                                   const double* __restrict__ local, int half,
                                                   int halfp, float2* __restrict__ tab) {
    const int c = blockIdx.y;
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= halfp) return;
    float2 v = make_float2(0.f, 0.f);
    if (k < half) {
        double s, co;
        sincos(theta_rad[2 * k + axis] * local[c], &s, &co);
        v = make_float2((float)co, (float)s);
    }
    tab[(size_t)c * halfp + k] = v;
}

__device__ inline uint16_t bf16_bits(float f) {  // round to nearest even (finite inputs)
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf16_value(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ inline uint16_t f16_bits(float f) {
    _Float16 h = (_Float16)f;
    return __builtin_bit_cast(uint16_t, h);
}

// 16-bit row tables are stored in the operand order of v_mfma_f32_32x32x16: rows in blocks of
// 32, and for every block, K step (32 bins = 64 reals, re and im interleaved) and 16-real chunk of
// the step, one contiguous 1 KB fragment whose 16-byte piece l holds reals 8 (l / 32) .. + 7 of
// the chunk for row l % 32 of the block.  A wavefront's operand load is then 1 KB of consecutive
// bytes (a row-major table would touch 32 lines and use 32 bytes of each).  Element e of row r
// (K step kb = e / 64, chunk ch = (e / 16) % 4, half h = (e / 8) % 2, j = e % 8) sits at
//   (((r / 32) * ksteps + kb) * 4 + ch) * 512 + ((r % 32) + 32 h) * 8 + j.

// Eight table values (four bins, re and im) of one lane's 16-byte piece, rounded to the 16-bit
// format (hi) and, for the split form, the rounding residuals (lo).
__device__ inline void pack16x8(const double (&v)[8], int fp16, uint32_t (&h)[4], uint32_t (&l)[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint16_t hb[2], lb[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const double x = v[2 * q + u];
            if (fp16) {
                hb[u] = f16_bits((float)x);
                lb[u] = f16_bits((float)(x - (double)__builtin_bit_cast(_Float16, hb[u])));
            } else {
                hb[u] = bf16_bits((float)x);
                lb[u] = bf16_bits((float)(x - (double)bf16_value(hb[u])));
            }
        }
        h[q] = (uint32_t)hb[0] | ((uint32_t)hb[1] << 16);
        l[q] = (uint32_t)lb[0] | ((uint32_t)lb[1] << 16);
    }
}

// Block (K step kb, 32-row block b) of a 16-bit table: thread t writes lane t % 64 of chunk t / 64,
// i.e. bins kb*32 + 8*(t/64) + 4*h .. + 3 of row 32*b + l % 32 (h = l / 32), as one 16-byte store,
// so each wavefront writes one whole 1 KB fragment.
struct Frag16Lane {
    int r, k0;
    size_t off;   // element offset of the lane's 16-byte piece
};
__device__ inline Frag16Lane frag16_lane(int ks) {
    const int kb = blockIdx.x, b = blockIdx.y, ch = threadIdx.x >> 6, l = threadIdx.x & 63;
    Frag16Lane f;
    f.r = 32 * b + (l & 31);
    f.k0 = kb * 32 + 8 * ch + 4 * (l >> 5);
    f.off = (((size_t)b * ks + kb) * 4 + ch) * 512 + (size_t)l * 8;
    return f;
}
__device__ inline void store16x8(const double (&v)[8], size_t off, int fp16, uint16_t* __restrict__ hi,
                                 uint16_t* __restrict__ lo) {
    uint32_t h[4], l[4];
    pack16x8(v, fp16, h, l);
    *reinterpret_cast<uint4*>(hi + off) = make_uint4(h[0], h[1], h[2], h[3]);
    if (lo) *reinterpret_cast<uint4*>(lo + off) = make_uint4(l[0], l[1], l[2], l[3]);
}

// 16-bit tables of nrows rows (re, im per bin, in the order above); lo holds the rounding
// residual (split form).  Grid (K steps, rows16(nrows) / 32); rows past nrows are zero.
__global__ __launch_bounds__(256) void k_table_16(const double* __restrict__ theta_rad, int axis,
                                                  const double* __restrict__ local, int nrows, int half,
                                                  int halfp, int fp16, uint16_t* __restrict__ hi,
                                                  uint16_t* __restrict__ lo) {
    const Frag16Lane f = frag16_lane(halfp / 32);
    double v[8];
    const double c = f.r < nrows ? local[f.r] : 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int k = f.k0 + i;
        v[2 * i] = v[2 * i + 1] = 0.0;
        if (f.r < nrows && k < half) sincos(theta_rad[2 * k + axis] * c, &v[2 * i + 1], &v[2 * i]);
    }
    store16x8(v, f.off, fp16, hi, lo);
}

// Joint (z, y) rows of a volume, row r of the row space being voxel plane offset
// row_map[r] = slice * ny + y: spectrum exp(i (Theta_y[k] y + Theta_z[k] z)) with the phase
// formed in double precision from the tile-local coordinates.  Same order, grid and padding.
__global__ __launch_bounds__(256) void k_table_yz_16(const double* __restrict__ theta_xy,
                                                     const double* __restrict__ theta_z,
                                                     const double* __restrict__ local_y,
                                                     const double* __restrict__ local_z,
                                                     const int* __restrict__ row_map, int nrows, int ny,
                                                     int half, int halfp, int fp16, uint16_t* __restrict__ hi,
                                                     uint16_t* __restrict__ lo) {
    const Frag16Lane f = frag16_lane(halfp / 32);
    double y = 0.0, z = 0.0;
    if (f.r < nrows) {
        const int rm = row_map[f.r];
        y = local_y[rm % ny];
        z = local_z[rm / ny];
    }
    double v[8];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int k = f.k0 + i;
        v[2 * i] = v[2 * i + 1] = 0.0;
        if (f.r < nrows && k < half) sincos(theta_xy[2 * k + 1] * y + theta_z[2 * k] * z, &v[2 * i + 1], &v[2 * i]);
    }
    store16x8(v, f.off, fp16, hi, lo);
}

// Logical index of workgroup b of n when consecutive hardware indices land on different XCDs
// (round-robin over kXcds): XCD x receives the logical range [x*n/kXcds, (x+1)*n/kXcds).
constexpr int kXcds = 8;
__device__ inline int xcd_local_index(int b, int n) {
    if (n % kXcds != 0) return b;
    return (b % kXcds) * (n / kXcds) + b / kXcds;
}

struct DecodeArgs {
    const DTile* tiles;
    int ntiles;
    const int* col_tx;         // [nx] tile column of every grid column
    const float2* ex;          // [nx][halfp] fp32
    const void* ey;            // fp32 [ny][halfp] or 16-bit [ny][2*halfp]
    const void* ey_lo;         // 16-bit residual (split form) or null
    const float2* omega_s;     // [nkeys][halfp] conj(Omega) / ||w|| (0 for an empty memory)
    int halfp, nx, ny, tiles_x;
    float out_scale;           // 2 / D
    float* heat;               // [2][slices][ny][nx]: class planes class_stride apart
    size_t class_stride;
    const int* row_map;        // volumes: voxel plane offset (slice * ny + y) of every row of the
                               // joint (z, y) row space; null for maps
    unsigned* hmax_u;          // [2] ordered maxima (zeroed by the norm kernel)
    float* partial;            // [grid][2][2][kTileRows][kTileCols]
    int ksteps;                // K steps per tile
    int steps_per_wg;          // fp32 kernel: L, stream-K iterations per workgroup
    long long total_steps;     // fp32 kernel: ntiles * ksteps
    // 16-bit kernels: work units (a K range of one tile), in K order within a tile; tile t's
    // units are tile_u0[t] .. tile_u0[t + 1] - 1 and workgroup w runs units wg_u0[w] ..
    // wg_u0[w + 1] - 1; a unit that is not a whole tile writes partial block unit.part.
    const DUnit* units;
    int nunits;
    const int* tile_u0;
    const int* wg_u0;
    int nwg;
    // Batched launches (16-bit kernels): tiles of several requests, tile t belonging to request
    // reqs[t.pad], whose fields replace the per-request ones above.  Null for one request.
    const DecodeReq* reqs;
    // Localized decode: [0] tiles, [1] 16-bit workgroups, [3] fp32 steps per workgroup, written
    // on the device by the plan kernel (the grids are upper bounds).  Null: the fields above.
    const int* dyn;
};

// Launch width and logical index of this workgroup when the real workgroup count n comes from
// the device: the first round_up(n, kXcds) workgroups are spread over the XCDs as usual, the
// rest of the (upper-bound) grid leaves at once (returns -1).
__device__ inline int dyn_wg_index(int n) {
    const int n8 = (n + kXcds - 1) / kXcds * kXcds;
    if ((int)blockIdx.x >= n8) return -1;
    return xcd_local_index(blockIdx.x, n8);
}

// The per-request view of a batched launch for tile t (unchanged for a single request).
__device__ inline void apply_request(DecodeArgs& r, const DTile& t) {
    if (!r.reqs) return;
    const DecodeReq q = r.reqs[t.pad];
    r.col_tx = q.col_tx;
    r.ex = q.ex;
    r.ey = q.ey;
    r.ey_lo = q.ey_lo;
    r.omega_s = q.omega_s;
    r.halfp = q.halfp;
    r.nx = q.nx;
    r.ny = q.ny;
    r.tiles_x = q.tiles_x;
    r.out_scale = q.out_scale;
    r.heat = q.heat;
    r.class_stride = q.class_stride;
    r.row_map = q.row_map;
    r.hmax_u = q.hmax_u;
    r.ksteps = q.ksteps;
}

// Operand formats: FP32 (0), BF16 (1), FP16 (2), BF16 hi+lo (3).  k_decode below takes FP32
// operands; the 16-bit formats run k_decode16.

__device__ inline void store_tile(const DecodeArgs& a, const DTile& t, int wave, int lane,
                                  const v4f (&acc)[2][kRowBlocks]) {
    const int g = lane >> 4, i16 = lane & 15;
    const int col = t.col0 + 16 * wave + i16;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        float mx = -INFINITY;
        float* out = a.heat + (size_t)p * a.class_stride;
#pragma unroll
        for (int rb = 0; rb < kRowBlocks; ++rb) {
            if (rb < t.nrb) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int row = t.row0 + 16 * rb + 4 * g + j;
                    if (row < t.row_end && col < a.nx) {
                        const float v = acc[p][rb][j] * a.out_scale;
                        out[(size_t)row * a.nx + col] = v;
                        mx = fmaxf(mx, v);
                    }
                }
            }
        }
        for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
        if (lane == 0 && mx > -INFINITY && a.hmax_u) atomicMax(a.hmax_u + p, order_key(mx));
    }
}

// Workgroups of the fp32 kernel resident per CU.
constexpr int kDecodeOccupancy32 = 2;

// FP32 operands (PREC 0 only).
template <int PREC>
__global__ __launch_bounds__(256, kDecodeOccupancy32) void k_decode(DecodeArgs a) {
    static_assert(PREC == 0, "the 16-bit formats run k_decode16");
    constexpr int KB = 16;    // complex bins per K step (128-byte rows)
    constexpr int NSPLIT = 1;
    // LDS, two stages: A rows [kTileRows], B rows [2 classes][kTileCols], each kRowPitchBytes.
    constexpr int STAGE = NSPLIT * (kTileRows + 2 * kTileCols) * kRowPitchBytes;
    __shared__ __attribute__((aligned(16))) unsigned char smem[2 * STAGE];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, i16 = lane & 15;
    // Workgroups are dispatched round-robin over the XCDs; give each XCD a contiguous share of
    // the iteration space, so that its resident workgroups work on neighbouring tiles (the
    // same row group of a band) and share those rows' table lines in the XCD's L2.
    long long steps_per_wg = a.steps_per_wg, total_steps = a.total_steps;
    int wg;
    if (a.dyn) {
        steps_per_wg = a.dyn[3];
        total_steps = (long long)a.dyn[0] * a.ksteps;
        wg = dyn_wg_index((int)((total_steps + steps_per_wg - 1) / steps_per_wg));
        if (wg < 0) return;
    } else {
        wg = xcd_local_index(blockIdx.x, gridDim.x);
    }
    const long long it0 = (long long)wg * steps_per_wg;
    const long long it1 = min(it0 + steps_per_wg, total_steps);
    const int first_tile = (int)(it0 / a.ksteps);

    // A: 128-byte rows, 8 units of 16 bytes; B: 64 columns x KB complex, units of 2 complex
    constexpr int A_UNITS_MAX = kTileRows * 8;
    constexpr int A_PER_T = (A_UNITS_MAX + 255) / 256;
    constexpr int B_UNITS = kTileCols * KB / 2;
    constexpr int B_PER_T = B_UNITS / 256;

    long long it = it0;
    while (it < it1) {
        const int ti = (int)(it / a.ksteps);
        const int kb0 = (int)(it - (long long)ti * a.ksteps);
        const int kb1 = (int)min((long long)a.ksteps, it1 - (long long)ti * a.ksteps);
        it = (long long)ti * a.ksteps + kb1;
        const DTile t = a.tiles[ti];
        const int nrows = 16 * t.nrb;
        const int ty = t.ty;

        u32x4 ra[A_PER_T * NSPLIT];
        f32x4 rx[B_PER_T], ro[B_PER_T][2];
        // per-tile column data, hoisted out of the K loop: every load of a K step then has a
        // ready address and the first wait on them comes after the step's MFMAs
        const f32x4* ex_row[B_PER_T];
        const f32x4* om_row[B_PER_T];
#pragma unroll
        for (int u = 0; u < B_PER_T; ++u) {
            const int idx = tid + 256 * u;
            const int c = idx / (KB / 2), part = idx % (KB / 2);
            const int gcol = min(t.col0 + c, a.nx - 1);
            const int key0 = 2 * (ty * a.tiles_x + a.col_tx[gcol]);
            ex_row[u] = reinterpret_cast<const f32x4*>(a.ex + (size_t)gcol * a.halfp + 2 * part);
            om_row[u] = reinterpret_cast<const f32x4*>(a.omega_s + (size_t)key0 * a.halfp + 2 * part);
        }
        const size_t om_class = (size_t)a.halfp / 2;  // one key further, in f32x4 units

        // Global loads of one K step into registers.  Rows past the tile's last row block (but
        // inside the kTileRows LDS rows) load a clamped valid row that the MFMAs never read.
        auto gload = [&](int kb) {
#pragma unroll
            for (int u = 0; u < A_PER_T; ++u) {
                const int idx = tid + 256 * u;
                if (idx >= A_UNITS_MAX) break;  // only the last unit round is partial
                const int r = idx >> 3, part = idx & 7;
                const int grow = min(t.row0 + min(r, nrows - 1), t.row_end - 1);
                const float2* src = static_cast<const float2*>(a.ey) + (size_t)grow * a.halfp + (size_t)kb * KB + 2 * part;
                ra[u * NSPLIT] = *reinterpret_cast<const u32x4*>(src);
            }
#pragma unroll
            for (int u = 0; u < B_PER_T; ++u) {
                const size_t boff = (size_t)kb * (KB / 2);  // f32x4 = two complex bins
                rx[u] = ex_row[u][boff];
                ro[u][0] = om_row[u][boff];
                ro[u][1] = om_row[u][boff + om_class];
            }
        };

        // Registers of one K step into LDS stage `st`; the column operand becomes
        // conj(Omega)/||w|| * Ex written as (Re, -Im).
        auto lstore = [&](int st) {
            unsigned char* As = smem + st * STAGE;
            unsigned char* Bs = As + NSPLIT * kTileRows * kRowPitchBytes;
#pragma unroll
            for (int u = 0; u < A_PER_T; ++u) {
                const int idx = tid + 256 * u;
                if (idx >= A_UNITS_MAX) break;  // LDS rows stop at kTileRows
                const int r = idx >> 3, part = idx & 7;
#pragma unroll
                for (int h = 0; h < NSPLIT; ++h)
                    *reinterpret_cast<u32x4*>(As + (h * kTileRows + r) * kRowPitchBytes + 16 * part) = ra[u * NSPLIT + h];
            }
#pragma unroll
            for (int u = 0; u < B_PER_T; ++u) {
                const int idx = tid + 256 * u;
                const int c = idx / (KB / 2), part = idx % (KB / 2);
                const f32x4 e = rx[u];
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    const f32x4 o = ro[u][p];
                    // (o.x + i o.y)(e.x + i e.y) -> (Re, -Im)
                    const float r0 = __builtin_fmaf(o.x, e.x, -o.y * e.y);
                    const float r1 = __builtin_fmaf(-o.x, e.y, -o.y * e.x);   // -(o.x e.y + o.y e.x), same bits
                    const float r2 = __builtin_fmaf(o.z, e.z, -o.w * e.w);
                    const float r3 = __builtin_fmaf(-o.z, e.w, -o.w * e.z);
                    unsigned char* dst = Bs + (p * kTileCols + c) * kRowPitchBytes;
                    *reinterpret_cast<f32x4*>(dst + 16 * part) = f32x4{r0, r1, r2, r3};
                }
            }
        };

        v4f acc[2][kRowBlocks];
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int rb = 0; rb < kRowBlocks; ++rb) acc[p][rb] = v4f{0.f, 0.f, 0.f, 0.f};

        // Pipeline: stage k+1 is loaded and written to the other LDS stage while the MFMAs
        // of stage k run; one barrier per K step.
        __syncthreads();  // the previous tile's last reads of both stages are done
        gload(kb0);
        lstore(0);
        __syncthreads();
        for (int kb = kb0; kb < kb1; ++kb) {
            const int st = (kb - kb0) & 1;
            const bool more = kb + 1 < kb1;
            if (more) gload(kb + 1);
            const unsigned char* As = smem + st * STAGE;
            const unsigned char* Bs = As + NSPLIT * kTileRows * kRowPitchBytes;
            const int bcol = 16 * wave + i16;
            // MFMAs are issued with the row-block loop innermost so that consecutive
            // instructions update different accumulators (no back-to-back dependency).
            {
                float b[2][8];
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    const f32x4* src = reinterpret_cast<const f32x4*>(Bs + (p * kTileCols + bcol) * kRowPitchBytes + 32 * g);
                    const f32x4 u = src[0], v = src[1];
                    b[p][0] = u.x; b[p][1] = u.y; b[p][2] = u.z; b[p][3] = u.w;
                    b[p][4] = v.x; b[p][5] = v.y; b[p][6] = v.z; b[p][7] = v.w;
                }
                float av[kRowBlocks][8];
#pragma unroll
                for (int rb = 0; rb < kRowBlocks; ++rb) {
                    if (rb < t.nrb) {
                        const f32x4* src = reinterpret_cast<const f32x4*>(As + (16 * rb + i16) * kRowPitchBytes + 32 * g);
                        const f32x4 u = src[0], v = src[1];
                        av[rb][0] = u.x; av[rb][1] = u.y; av[rb][2] = u.z; av[rb][3] = u.w;
                        av[rb][4] = v.x; av[rb][5] = v.y; av[rb][6] = v.z; av[rb][7] = v.w;
                    }
                }
#pragma unroll
                for (int s = 0; s < 8; ++s)
#pragma unroll
                    for (int rb = 0; rb < kRowBlocks; ++rb)
                        if (rb < t.nrb)
#pragma unroll
                            for (int p = 0; p < 2; ++p)
                                acc[p][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[rb][s], b[p][s], acc[p][rb], 0, 0, 0);
            }
            if (more) lstore(st ^ 1);
            __syncthreads();
        }

        if (kb0 == 0 && kb1 == a.ksteps) {  // the whole tile: store it
            store_tile(a, t, wave, lane, acc);
            continue;
        }
        // a tile split across workgroups: store this segment's partial sums (slot 0 if the
        // tile is the workgroup's first, else slot 1); k_decode_fix adds the segments
        const int slot = (ti == first_tile) ? 0 : 1;
        float* part = a.partial + ((size_t)wg * 2 + slot) * 2 * kTileRows * kTileCols;
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int rb = 0; rb < kRowBlocks; ++rb)
                if (rb < t.nrb)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        part[((size_t)p * kTileRows + 16 * rb + 4 * g + j) * kTileCols + 16 * wave + i16] = acc[p][rb][j];
    }
}

// 16-bit operand formats.  Work tiles of 256 rows x 64 columns x 2 classes on the 32x32x16
// matrix instructions (the 16x16x32 form of the same formats issues at about half their rate on
// gfx950).  Each of the NW waves owns one block of 32 consecutive rows and both 32-column blocks
// of the tile, for both classes (four 32x32 accumulators).  A wave reads its row operand -- the
// location table, already in the MFMA input format -- straight from global memory into
// registers, DEPTH K steps ahead; only the column operand, which needs the memory factor
// applied, goes through LDS (its sources are loaded one step ahead), where every wave reads it.
// So LDS carries one operand instead of two, and each wave reads only its own rows' table data.
// One workgroup of eight waves per CU: two waves per SIMD, so that one wave's matrix
// instructions run while the other forms, stores or waits for operands.
//
// Lane layout of v_mfma_f32_32x32x16 (16-bit inputs): lane l holds eight consecutive K elements
// 8*(l/32) .. +7 of row (A) / column (B) l%32; output register v of lane l is row
// 8*(v/4) + 4*(l/32) + v%4, column l%32.  A K step (64 reals) is four 16-real chunks.
template <int PREC>
struct Wide {
    static constexpr bool kSplit = (PREC == 3);
    static constexpr int NW = 8;                        // waves per workgroup (two per SIMD)
    static constexpr int NT = 64 * NW;                  // threads per workgroup
    static constexpr int WR = 32;                       // rows per wave
    static constexpr int OCC = 1;                       // workgroups per CU
    static constexpr int TR = WR * NW;                  // tile rows
    static constexpr int NS = kSplit ? 2 : 1;           // hi (+ lo) parts
    static constexpr int DEPTH = 1;                     // K steps the row operand is loaded ahead
    static constexpr int NSETS = DEPTH + 1;             // register sets in rotation
    static constexpr int KB = 32;                       // complex bins per K step
    static constexpr int NCH = 2 * KB / 16;             // 16-real MFMA chunks per K step
    static constexpr int BROWS = 2 * kTileCols;         // LDS rows: class-major columns
    static constexpr int BSTAGE = NS * BROWS * kRowPitchBytes;
    static constexpr int B_PER_T = kTileCols * KB / 2 / NT;  // f32x4 units per thread
    static constexpr int OSTAGE = 2 * 2 * KB;           // float2: [key slot][class][bin]
};

static_assert(Wide<1>::KB == 32 && Wide<1>::NCH == 4 && Wide<1>::WR == 32, "the row tables' operand order (k_table_16)");
static_assert(Wide<1>::TR == 16 * kDecodeSetRowBlocks[1] && Wide<3>::TR == 16 * kDecodeSetRowBlocks[2],
              "tile sets match the kernels");

template <int PREC>
__device__ inline v16f mfma32(u32x4 x, u32x4 y, v16f c) {
    if constexpr (PREC == 2)
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(v8h, x), __builtin_bit_cast(v8h, y), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, x), __builtin_bit_cast(v8bf, y), c, 0,
                                                       0, 0);
}

// Z: volumes; rows are the joint (z, y) rows of the volume (the row operand is their joint table)
// and row_map places them in the heat planes.
template <int PREC, bool Z>
__global__ __launch_bounds__(Wide<PREC>::NT, Wide<PREC>::OCC) void k_decode16(DecodeArgs ab) {
    using W = Wide<PREC>;
    constexpr int NS = W::NS, NSETS = W::NSETS, DEPTH = W::DEPTH, KB = W::KB, NCH = W::NCH, TR = W::TR;
    constexpr int B_PER_T = W::B_PER_T, NT = W::NT;
    __shared__ __attribute__((aligned(16))) unsigned char smem[2 * W::BSTAGE];
    __shared__ __attribute__((aligned(16))) float2 om_lds[2][W::OSTAGE];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, l32 = lane & 31;
    const int wg = ab.dyn ? dyn_wg_index(ab.dyn[1]) : xcd_local_index(blockIdx.x, gridDim.x);
    if (wg < 0 || wg >= (ab.dyn ? ab.dyn[1] : ab.nwg)) return;   // grid padding (uniform over the workgroup)
    const int u_end = ab.wg_u0[wg + 1];
    for (int ui = ab.wg_u0[wg]; ui < u_end; ++ui) {
        const DUnit unit = ab.units[ui];
        const int ti = unit.tile, kb0 = unit.kb0, kb1 = unit.kb1;
        const DTile t = ab.tiles[ti];
        DecodeArgs a = ab;
        apply_request(a, t);
        const int ks = a.ksteps;
        // the tables are global memory (the pointers of a batched launch come from a descriptor,
        // so the address space is stated for the compiler)
        const gmem<uint16_t>* ey_hi = as_global(static_cast<const uint16_t*>(a.ey));
        const gmem<uint16_t>* ey_lo = as_global(static_cast<const uint16_t*>(a.ey_lo));
        const int n = kb1 - kb0;
        // does this wave's 32-row block hold any row of the tile (wave-uniform)
        const int wv = __builtin_amdgcn_readfirstlane(wave);
        const bool active = t.nrb > 2 * wv;

        // row operand: row l32 of the wave's block (clamped to the tile's last row), K offset 8*h
        // within a 16-real chunk, in the table's operand order (chunk ch of step kb of the row's
        // 32-row block is the 1 KB at (kb * NCH + ch) * 512 elements from the block's first)
        const int arow_idx = min(t.row0 + W::WR * wave + l32, t.row_end - 1);
        const size_t arow = ((size_t)(arow_idx >> 5) * ks * NCH * 64 + (arow_idx & 31) + 32 * h) * 8;
        // column operand sources: the x table per column; the memories of the (at most two)
        // tile columns of the slice are staged in LDS, two K steps ahead, by the first wave
        const gmem<f32x4>* ex_row[B_PER_T];
        int oslot[B_PER_T];
        const int part16 = tid % (KB / 2);
#pragma unroll
        for (int u = 0; u < B_PER_T; ++u) {
            const int c = (tid + NT * u) / (KB / 2);
            const int gcol = min(t.col0 + c, a.nx - 1);
            ex_row[u] = as_global(reinterpret_cast<const f32x4*>(a.ex + (size_t)gcol * a.halfp + 2 * part16));
            oslot[u] = min(max(as_global(a.col_tx)[gcol] - t.tx0, 0), 1);
        }
        const int oks = (lane >> 5) & 1, ocls = (lane >> 4) & 1;  // this lane's staging item
        const gmem<f32x4>* om_src = as_global(reinterpret_cast<const f32x4*>(
            a.omega_s + (size_t)(2 * (t.ty * a.tiles_x + min(t.tx0 + oks, a.tiles_x - 1)) + ocls) * a.halfp +
            2 * part16));
        f32x4 OM;
        auto load_om = [&](int kk) { OM = om_src[(size_t)(kb0 + min(kk, n - 1)) * (KB / 2)]; };
        auto store_om = [&](int st) {
            if (wave == 0)
                *reinterpret_cast<f32x4*>(&om_lds[st][(oks * 2 + ocls) * KB + 2 * part16]) = OM;
        };

        u32x4 A[NSETS][NCH][NS];     // [set][16-real chunk][hi, lo]
        f32x4 BX[B_PER_T];

        // Loads are issued without branches (rows past the tile's last one reload a clamped row,
        // steps past the segment's last one reload its last step), so that the compiler can count
        // them exactly and waits only for the data a step actually consumes.
        auto load_a = [&](auto SET, int kk) {  // row operand of K step kb0 + kk into set SET
            constexpr int S = decltype(SET)::value;
            const int kb = kb0 + min(kk, n - 1);
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                const size_t off = arow + ((size_t)kb * NCH + ch) * 512;
                A[S][ch][0] = *reinterpret_cast<const gmem<u32x4>*>(ey_hi + off);
                if (W::kSplit) A[S][ch][NS - 1] = *reinterpret_cast<const gmem<u32x4>*>(ey_lo + off);
            }
        };
        auto load_b = [&](int kk) {  // column operand sources of K step kb0 + kk
            const size_t boff = (size_t)(kb0 + min(kk, n - 1)) * (KB / 2);
#pragma unroll
            for (int u = 0; u < B_PER_T; ++u) BX[u] = ex_row[u][boff];
        };
        // column operand into LDS stage st: conj(Omega)/||w|| * Ex as (Re, -Im)
        auto bstore = [&](int st) {
            unsigned char* Bs = smem + st * W::BSTAGE;
#pragma unroll
            for (int u = 0; u < B_PER_T; ++u) {
                const int idx = tid + NT * u;
                const int c = idx / (KB / 2), part = idx % (KB / 2);
                f32x4 e = BX[u];
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    const f32x4 o = *reinterpret_cast<const f32x4*>(&om_lds[st][(oslot[u] * 2 + p) * KB + 2 * part]);
                    const float r0 = __builtin_fmaf(o.x, e.x, -o.y * e.y);
                    const float r1 = __builtin_fmaf(-o.x, e.y, -o.y * e.x);   // -(o.x e.y + o.y e.x), same bits
                    const float r2 = __builtin_fmaf(o.z, e.z, -o.w * e.w);
                    const float r3 = __builtin_fmaf(-o.z, e.w, -o.w * e.z);
                    unsigned char* dst = Bs + (p * kTileCols + c) * kRowPitchBytes + 8 * part;
                    if (PREC == 2) {
                        *reinterpret_cast<u32x2*>(dst) = u32x2{pack_f16(r0, r1), pack_f16(r2, r3)};
                    } else {
                        const uint32_t h01 = pack_bf16(r0, r1), h23 = pack_bf16(r2, r3);
                        *reinterpret_cast<u32x2*>(dst) = u32x2{h01, h23};
                        if (W::kSplit)
                            *reinterpret_cast<u32x2*>(dst + W::BROWS * kRowPitchBytes) =
                                u32x2{pack_bf16_lo(r0, r1, h01), pack_bf16_lo(r2, r3, h23)};
                    }
                }
            }
        };

        v16f acc[2][2];   // [column block][class]
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int e = 0; e < 16; ++e) acc[cb][p][e] = 0.f;

        // one K step from register set SET: loads for step kk + DEPTH go out first, then the
        // MFMAs of step kk (column operand from LDS stage kk & 1), then step kk + 1's column
        // operand is written to the other stage; one barrier per step
        auto step = [&](auto SET, int kk) {
            constexpr int S = decltype(SET)::value;
            load_b(kk + 1);  // first: the wait for it at the end of the step leaves the row loads in flight
            load_om(kk + 2);
            load_a(std::integral_constant<int, (S + DEPTH) % NSETS>{}, kk + DEPTH);
            const unsigned char* Bs = smem + (kk & 1) * W::BSTAGE;
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                u32x4 bh[2][2], bl[2][2];
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                    for (int p = 0; p < 2; ++p) {
                        const unsigned char* src = Bs + (p * kTileCols + 32 * cb + l32) * kRowPitchBytes + 32 * ch + 16 * h;
                        bh[cb][p] = *reinterpret_cast<const u32x4*>(src);
                        if (W::kSplit) bl[cb][p] = *reinterpret_cast<const u32x4*>(src + W::BROWS * kRowPitchBytes);
                    }
                constexpr int NTERM = W::kSplit ? 3 : 1;
                if (active) {
#pragma unroll
                    for (int term = 0; term < NTERM; ++term)
#pragma unroll
                        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                            for (int p = 0; p < 2; ++p) {
                                const u32x4 x = (term == 2) ? A[S][ch][NS - 1] : A[S][ch][0];
                                const u32x4 y = (term == 1) ? bl[cb][p] : bh[cb][p];
                                acc[cb][p] = mfma32<PREC>(x, y, acc[cb][p]);
                            }
                }
            }
            bstore((kk + 1) & 1);  // past the segment's end: a stage nobody reads
            store_om(kk & 1);      // memories of step kk + 2, into the stage step kk's used
            __syncthreads();
        };

        __syncthreads();  // the previous tile's reads of every LDS stage are done
        load_om(0);
        store_om(0);
        load_om(1);
        store_om(1);
        load_b(0);
        load_a(std::integral_constant<int, 0>{}, 0);
        if (DEPTH > 1) load_a(std::integral_constant<int, 1 % NSETS>{}, 1);
        __syncthreads();
        bstore(0);
        __syncthreads();
        int kk = 0;
        for (; kk + NSETS <= n; kk += NSETS) {  // straight-line bodies
            step(std::integral_constant<int, 0>{}, kk);
            step(std::integral_constant<int, 1>{}, kk + 1);
            if (NSETS > 2) step(std::integral_constant<int, 2 % NSETS>{}, kk + 2);
        }
        if (kk < n) step(std::integral_constant<int, 0>{}, kk);
        if (NSETS > 2 && kk + 1 < n) step(std::integral_constant<int, 1>{}, kk + 1);

        const bool whole = (kb0 == 0 && kb1 == ks);
        gmem_rw<float>* part = as_global_rw(a.partial + (size_t)unit.part * 2 * TR * kTileCols);
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            float mx = -INFINITY;
            gmem_rw<float>* out = as_global_rw(a.heat + (size_t)p * a.class_stride);
            if (active) {
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                    for (int v = 0; v < 16; ++v) {
                        const int r = W::WR * wave + 8 * (v >> 2) + 4 * h + (v & 3), c = 32 * cb + l32;
                        if (whole) {
                            const int row = t.row0 + r, col = t.col0 + c;
                            if (row < t.row_end && c < t.ncol) {
                                const float val = acc[cb][p][v] * a.out_scale;
                                out[(size_t)(Z ? as_global(a.row_map)[row] : row) * a.nx + col] = val;
                                mx = fmaxf(mx, val);
                            }
                        } else {
                            part[((size_t)p * TR + r) * kTileCols + c] = acc[cb][p][v];
                        }
                    }
            }
            if (whole) {
                for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
                if (lane == 0 && mx > -INFINITY && a.hmax_u) atomicMax(a.hmax_u + p, order_key(mx));
            }
        }
    }
}

// Split tiles: add the segments' partial sums in workgroup order (deterministic), scale, store,
// fold the maxima.  Block (tile, part): about 8 elements per thread, all loads of a thread in
// flight together; one atomic per block and class.  Tiles finished whole by one workgroup are
// skipped.  Runs after the GEMM, so the kernel boundary makes the partial sums visible.
template <int TR>
struct Fix {
    static constexpr int PER_TILE = 2 * TR * kTileCols;
    static constexpr int PARTS = PER_TILE / 256 / 8 > 0 ? PER_TILE / (256 * 8) : 1;  // ~8 elements per thread
    static constexpr int PER = PER_TILE / PARTS / 256;
    static_assert(PER * 256 * PARTS == PER_TILE, "fix-up split");
};

template <int TR>
__global__ __launch_bounds__(256) void k_decode_fix(DecodeArgs ab) {
    using X = Fix<TR>;
    constexpr int PER_TILE = X::PER_TILE, PARTS = X::PARTS, PER = X::PER;
    const int ti = blockIdx.x / PARTS, partk = blockIdx.x % PARTS;
    if (ti >= (ab.dyn ? ab.dyn[0] : ab.ntiles)) return;   // localized decode: fewer tiles than the grid
    const long long steps_per_wg = ab.dyn ? ab.dyn[3] : ab.steps_per_wg;
    // segments of the tile: its work units (16-bit kernels, one partial block per unit), or the
    // workgroups whose stream-K ranges cover it (fp32 kernel, two partial blocks per workgroup)
    int w_first, w_last;
    if (ab.units) {
        w_first = ab.tile_u0[ti];
        w_last = ab.tile_u0[ti + 1] - 1;
    } else {
        const long long t0 = (long long)ti * ab.ksteps;
        w_first = (int)(t0 / steps_per_wg);
        w_last = (int)((t0 + ab.ksteps - 1) / steps_per_wg);
    }
    if (w_first >= w_last) return;  // whole tile, stored by the GEMM
    const DTile t = ab.tiles[ti];
    // a part of rows at or past the tile's last row block holds nothing to add (parts of whole
    // rows of one class: rows r0 .. r0 + PART_ROWS - 1)
    constexpr int PART_ROWS = PER_TILE / PARTS / kTileCols;
    if constexpr (TR % PART_ROWS == 0) {
        const int r0 = (partk * PART_ROWS) % TR;
        if (r0 >= 16 * t.nrb) return;
    }
    DecodeArgs a = ab;
    apply_request(a, t);
    float sum[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) sum[j] = 0.f;
    // segments in workgroup order, four at a time so that their loads are in flight together
    // (a segment past the last one reloads the last and adds nothing)
    auto seg = [&](int w) {
        if (ab.units) return as_global(a.partial + (size_t)ab.units[w].part * PER_TILE + partk * (PER_TILE / PARTS));
        const int slot = ((long long)w * steps_per_wg / ab.ksteps == ti) ? 0 : 1;
        return as_global(a.partial + ((size_t)w * 2 + slot) * PER_TILE + partk * (PER_TILE / PARTS));
    };
    for (int w = w_first; w <= w_last; w += 4) {
        float v[4][PER];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const gmem<float>* src = seg(min(w + q, w_last));
#pragma unroll
            for (int j = 0; j < PER; ++j) v[q][j] = src[threadIdx.x + 256 * j];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (w + q <= w_last)
#pragma unroll
                for (int j = 0; j < PER; ++j) sum[j] += v[q][j];
    }
    float mx[2] = {-INFINITY, -INFINITY};
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int rem = partk * (PER_TILE / PARTS) + threadIdx.x + 256 * j;
        const int p = rem / (TR * kTileCols);
        const int r = (rem / kTileCols) % TR, c = rem % kTileCols;
        const int row = t.row0 + r, col = t.col0 + c;
        if (r < 16 * t.nrb && row < t.row_end && c < t.ncol) {
            const float v = sum[j] * a.out_scale;
            const size_t orow = a.row_map ? (size_t)as_global(a.row_map)[row] : (size_t)row;
            as_global_rw(a.heat)[(size_t)p * a.class_stride + orow * a.nx + col] = v;
            mx[p] = fmaxf(mx[p], v);
        }
    }
    __shared__ float sh[2][4];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        float m = mx[q];
        for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
        if ((threadIdx.x & 63) == 0) sh[q][threadIdx.x >> 6] = m;
    }
    __syncthreads();
    if (threadIdx.x < 2 && a.hmax_u) {
        const float m = fmaxf(fmaxf(sh[threadIdx.x][0], sh[threadIdx.x][1]), fmaxf(sh[threadIdx.x][2], sh[threadIdx.x][3]));
        if (m > -INFINITY) atomicMax(a.hmax_u + threadIdx.x, order_key(m));
    }
}

// Maxima of both classes over the listed regions' cells, folded into their ordered maxima
// (order_key; 0 = no cell seen: the localized plan zeroes the entries of the regions it lists).
// Block (region, stripe): kRegionStripes blocks share a region's rows; the block's threads run
// across each row, four rows' loads in flight.
constexpr int kRegionStripes = 16;
__global__ __launch_bounds__(256) void k_region_max(const float* __restrict__ heat, int nx, int ny,
                                                    const RegionBox* __restrict__ boxes,
                                                    const int* __restrict__ nboxes_dev,
                                                    unsigned* __restrict__ region_u) {
    if ((int)blockIdx.x >= *nboxes_dev) return;
    const RegionBox b = boxes[blockIdx.x];
    const int h = b.row1 - b.row0, sh_rows = (h + kRegionStripes - 1) / kRegionStripes;
    const int r0 = b.row0 + (int)blockIdx.y * sh_rows, r1 = min(b.row1, r0 + sh_rows);
    const size_t plane = (size_t)nx * ny;
    float mx[2] = {-INFINITY, -INFINITY};
    for (int c = b.col0 + (int)threadIdx.x; c < b.col1; c += 256) {
        int r = r0;
        for (; r + 4 <= r1; r += 4) {
            float v[2][4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int p = 0; p < 2; ++p) v[p][u] = heat[(size_t)p * plane + (size_t)(r + u) * nx + c];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int p = 0; p < 2; ++p) mx[p] = fmaxf(mx[p], v[p][u]);
        }
        for (; r < r1; ++r)
#pragma unroll
            for (int p = 0; p < 2; ++p) mx[p] = fmaxf(mx[p], heat[(size_t)p * plane + (size_t)r * nx + c]);
    }
    __shared__ float sh[2][4];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        float m = mx[p];
        for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
        if ((threadIdx.x & 63) == 0) sh[p][threadIdx.x >> 6] = m;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        const float m = fmaxf(fmaxf(sh[threadIdx.x][0], sh[threadIdx.x][1]), fmaxf(sh[threadIdx.x][2], sh[threadIdx.x][3]));
        if (m > -INFINITY) atomicMax(region_u + 2 * b.beta + threadIdx.x, order_key(m));
    }
}

// hmax over all regions (a region with no cell counts as -inf).
__global__ __launch_bounds__(256) void k_region_final(const unsigned* __restrict__ region_u, int nregions,
                                                      float* __restrict__ hmax) {
    unsigned mx[2] = {0u, 0u};
    for (int i = threadIdx.x; i < nregions; i += 256) {
        mx[0] = max(mx[0], region_u[2 * i]);
        mx[1] = max(mx[1], region_u[2 * i + 1]);
    }
    __shared__ unsigned sh[2][4];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        unsigned m = mx[p];
        for (int off = 32; off > 0; off >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, off));
        if ((threadIdx.x & 63) == 0) sh[p][threadIdx.x >> 6] = m;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        const unsigned m = max(max(sh[threadIdx.x][0], sh[threadIdx.x][1]), max(sh[threadIdx.x][2], sh[threadIdx.x][3]));
        hmax[threadIdx.x] = m ? order_value(m) : -INFINITY;
    }
}

__global__ void k_hmax_final(const unsigned* __restrict__ hmax_u, float* __restrict__ hmax) {
    if (threadIdx.x < 2) hmax[threadIdx.x] = order_value(hmax_u[threadIdx.x]);
}

}  // namespace

hipError_t launch_table_f32(const double* theta_rad, int axis, const double* local, int ncells,
                            int half, int halfp, float2* tab, hipStream_t s) {
    hipLaunchKernelGGL(k_table_f32, dim3((halfp + 255) / 256, ncells), dim3(256), 0, s, theta_rad,
                       axis, local, half, halfp, tab);
    return hipGetLastError();
}

hipError_t launch_table_yz_split(const double* theta_xy, const double* theta_z, const double* local_y,
                                 const double* local_z, const int* row_map, int nrows, int ny, int half, int halfp,
                                 bool fp16, uint16_t* hi, uint16_t* lo, hipStream_t s) {
    if (nrows > 0)
        hipLaunchKernelGGL(k_table_yz_16, dim3((unsigned)(halfp / 32), (unsigned)(rows16(nrows) / 32)), dim3(256), 0, s,
                           theta_xy, theta_z, local_y, local_z, row_map, nrows, ny, half, halfp, fp16 ? 1 : 0, hi, lo);
    return hipGetLastError();
}

hipError_t launch_table_split(const double* theta_rad, int axis, const double* local, int ncells,
                              int half, int halfp, bool fp16, void* hi, void* lo, hipStream_t s) {
    if (ncells > 0)
        hipLaunchKernelGGL(k_table_16, dim3((unsigned)(halfp / 32), (unsigned)(rows16(ncells) / 32)), dim3(256), 0, s,
                           theta_rad, axis, local, ncells, half, halfp, fp16 ? 1 : 0, static_cast<uint16_t*>(hi),
                           static_cast<uint16_t*>(lo));
    return hipGetLastError();
}

DecodePlan decode_plan(int precision, int ntiles, int halfp, int num_cus) {
    DecodePlan p;
    const int kb = precision == 0 ? 16 : 32;
    p.ksteps = halfp / kb;
    const long long total = (long long)ntiles * p.ksteps;
    const int occ = precision == 0 ? kDecodeOccupancy32 : Wide<1>::OCC;
    const int slots = occ * num_cus;
    const long long rounds = (ntiles + slots - 1) / slots;
    if (precision != 0 && ntiles >= slots && (double)ntiles >= 0.9 * (double)(rounds * slots)) {
        // whole tiles per workgroup: every workgroup walks K from the start, in step with the
        // others on its XCD, and no tile needs a fix-up (grid padded to a multiple of the XCDs)
        p.steps_per_wg = p.ksteps;
        p.grid = (ntiles + kXcds - 1) / kXcds * kXcds;
        p.total_steps = total;
        return p;
    }
    long long L = (total + slots - 1) / slots;
    if (L < 4) L = 4;
    p.steps_per_wg = (int)L;
    p.grid = (int)((total + L - 1) / L);
    p.total_steps = total;
    return p;
}

size_t decode_partial_floats(int precision, const DecodePlan& p) {
    if (p.steps_per_wg % p.ksteps == 0 && p.steps_per_wg >= p.ksteps) return 0;  // no split tile
    const int tr = precision == 0 ? kTileRows : Wide<1>::TR;
    return (size_t)p.grid * 2 * 2 * tr * kTileCols;
}

hipError_t launch_region_max_dyn(const float* heat, int nx, int ny, const RegionBox* boxes, const int* nboxes_dev,
                                 int max_boxes, unsigned* region_u, int nregions, float* hmax, hipStream_t s) {
    if (max_boxes > 0)
        hipLaunchKernelGGL(k_region_max, dim3(max_boxes, kRegionStripes), dim3(256), 0, s, heat, nx, ny, boxes,
                           nboxes_dev, region_u);
    hipLaunchKernelGGL(k_region_final, dim3(1), dim3(256), 0, s, region_u, nregions, hmax);
    return hipGetLastError();
}

hipError_t launch_decode(int precision, const DecodeLaunch& d, hipStream_t s) {
    DecodeArgs a{};
    a.tiles = d.tiles;
    a.ntiles = d.ntiles;
    a.col_tx = d.col_tx;
    a.ex = d.ex;
    a.ey = d.ey;
    a.ey_lo = d.ey_lo;
    a.omega_s = d.omega_s;
    a.halfp = d.halfp;
    a.nx = d.nx;
    a.ny = d.ny;
    a.tiles_x = d.tiles_x;
    a.out_scale = d.out_scale;
    a.heat = d.heat;
    a.class_stride = d.class_stride ? d.class_stride : (size_t)d.nx * d.ny;
    a.row_map = d.row_map;
    a.hmax_u = d.hmax_u;
    a.partial = d.partial;
    a.ksteps = d.plan.ksteps;
    a.steps_per_wg = d.plan.steps_per_wg;
    a.total_steps = d.plan.total_steps;
    a.units = precision == 0 ? nullptr : d.units;
    a.nunits = d.nunits;
    a.tile_u0 = d.tile_u0;
    a.wg_u0 = d.wg_u0;
    a.nwg = d.nwg;
    a.reqs = nullptr;
    a.dyn = d.dyn;
    if (precision != 0 && (!d.units || !d.wg_u0 || d.nwg < 1 || (!d.dyn && d.nunits < 1)))
        return d.ntiles == 0 ? hipSuccess : hipErrorInvalidValue;
    const dim3 grid(precision == 0 ? d.plan.grid : (unsigned)((d.nwg + kXcds - 1) / kXcds * kXcds)), block(256),
        block16(Wide<1>::NT);
    // the GEMM records the stage's start event, and its stop event unless a fix-up follows
    // (a localized decode does not know on the host whether a tile is split: its fix-up always
    // runs, over at most fix_tiles tiles, and leaves at once where nothing is split)
    const bool fix = d.dyn ? true
                           : precision == 0 ? (d.plan.steps_per_wg % d.plan.ksteps != 0 || d.plan.steps_per_wg < d.plan.ksteps)
                                            : d.any_split;
    const unsigned fix_tiles = (unsigned)(d.dyn ? d.fix_tiles : d.ntiles);
    const hipEvent_t e0 = profile_start(kStageDecode), e1 = profile_stop(kStageDecode);
    const hipEvent_t g1 = fix ? nullptr : e1;
    switch (precision) {
        case 0:
            if (d.row_map) return hipErrorInvalidValue;  // volumes run the 16-bit kernels
            hipExtLaunchKernelGGL(k_decode<0>, grid, block, 0, s, e0, g1, 0, a);
            break;
        case 1:
            if (d.row_map) hipExtLaunchKernelGGL(k_decode16<1, true>, grid, block16, 0, s, e0, g1, 0, a);
            else hipExtLaunchKernelGGL(k_decode16<1, false>, grid, block16, 0, s, e0, g1, 0, a);
            break;
        case 2:
            if (d.row_map) hipExtLaunchKernelGGL(k_decode16<2, true>, grid, block16, 0, s, e0, g1, 0, a);
            else hipExtLaunchKernelGGL(k_decode16<2, false>, grid, block16, 0, s, e0, g1, 0, a);
            break;
        case 3:
            if (d.row_map) hipExtLaunchKernelGGL(k_decode16<3, true>, grid, block16, 0, s, e0, g1, 0, a);
            else hipExtLaunchKernelGGL(k_decode16<3, false>, grid, block16, 0, s, e0, g1, 0, a);
            break;
        default: return hipErrorInvalidValue;
    }
    if (fix) {
        if (precision == 0)
            hipExtLaunchKernelGGL(k_decode_fix<kTileRows>, dim3(fix_tiles * Fix<kTileRows>::PARTS),
                                  dim3(256), 0, s, nullptr, e1, 0, a);
        else if (precision == 3)
            hipExtLaunchKernelGGL(k_decode_fix<Wide<3>::TR>, dim3(fix_tiles * Fix<Wide<3>::TR>::PARTS),
                                  dim3(256), 0, s, nullptr, e1, 0, a);
        else
            hipExtLaunchKernelGGL(k_decode_fix<Wide<1>::TR>, dim3(fix_tiles * Fix<Wide<1>::TR>::PARTS),
                                  dim3(256), 0, s, nullptr, e1, 0, a);
    }
    if (d.hmax_u) hipLaunchKernelGGL(k_hmax_final, dim3(1), dim3(64), 0, s, d.hmax_u, d.hmax);
    return hipGetLastError();
}

// Shortest K range of a workgroup when tiles are split (longer ranges amortise the unit's
// prologue, epilogue and partial-sum traffic).
constexpr int kMinUnitSteps = 16;

// K steps per workgroup for n tiles of ks steps on slots resident workgroups: whole tiles when
// there are at least slots of them and the last round of workgroups is at least 90 % full;
// otherwise equal consecutive ranges, about one per slot (at least kMinUnitSteps steps, at most
// one tile when the tiles are fewer than the slots).
__host__ __device__ inline long long unit_range(long long n, long long ks, long long slots) {
    if (n <= 0) return ks;
    const long long rounds = (n + slots - 1) / slots;
    if (n >= slots && 10 * n >= 9 * rounds * slots) return ks;
    long long L = (n * ks + slots - 1) / slots;
    if (L < kMinUnitSteps) L = kMinUnitSteps;
    if (n < slots && L > ks) L = ks;
    return L;
}

void decode_units(int ntiles, int ksteps, int num_cus, int tile_base, int unit_base, std::vector<DUnit>& units,
                  std::vector<int>& tile_u0, std::vector<int>& wg_u0) {
    // The request's ntiles * ksteps K steps are cut into consecutive ranges, one per workgroup
    // (unit_range); a range is one unit per tile it touches.  Only a range's first and last
    // units can be parts of a tile; they write partial blocks 2w and 2w + 1 (w: the
    // workgroup within the request).  The cut depends on the request alone, so its tiles' sums
    // (partials added in unit order) are the same whatever else shares the launch.
    const int slots = Wide<1>::OCC * num_cus;
    const long long ks = ksteps, total = (long long)ntiles * ks;
    const long long L = unit_range(ntiles, ks, slots);
    int u = unit_base, cur = -1, w = 0;
    for (long long it0 = 0; it0 < total; it0 += L, ++w) {
        const long long it1 = std::min(total, it0 + L);
        wg_u0.push_back(u);
        for (long long it = it0; it < it1;) {
            const int t = (int)(it / ks);
            const int kb0 = (int)(it - (long long)t * ks);
            const int kb1 = (int)std::min<long long>(ks, it1 - (long long)t * ks);
            for (; cur < t; ++cur) tile_u0.push_back(u);   // tile t starts at this unit
            units.push_back(DUnit{tile_base + t, kb0, kb1, 2 * w + (it == it0 ? 0 : 1)});
            ++u;
            it = (long long)t * ks + kb1;
        }
    }
    for (; cur + 1 < ntiles; ++cur) tile_u0.push_back(u);   // no K steps: tiles without units
}

size_t decode_unit_partial_floats(int nblocks) { return (size_t)nblocks * 2 * Wide<1>::TR * kTileCols; }

hipError_t launch_decode_batch(int precision, const DecodeBatch& b, hipStream_t s) {
    if (precision < 1 || precision > 3) return hipErrorInvalidValue;
    if (b.ntiles == 0 || b.nunits == 0 || b.nwg == 0) return hipSuccess;
    DecodeArgs a{};
    a.tiles = b.tiles;
    a.ntiles = b.ntiles;
    a.partial = b.partial;
    a.units = b.units;
    a.nunits = b.nunits;
    a.tile_u0 = b.tile_u0;
    a.wg_u0 = b.wg_u0;
    a.nwg = b.nwg;
    a.reqs = b.reqs;
    a.dyn = nullptr;
    const dim3 grid((unsigned)((b.nwg + kXcds - 1) / kXcds * kXcds)), block16(Wide<1>::NT);
    const hipEvent_t e0 = profile_start(kStageDecode), e1 = profile_stop(kStageDecode);
    const hipEvent_t g1 = b.any_split ? nullptr : e1;
    switch (precision) {
        case 1: hipExtLaunchKernelGGL(k_decode16<1, false>, grid, block16, 0, s, e0, g1, 0, a); break;
        case 2: hipExtLaunchKernelGGL(k_decode16<2, false>, grid, block16, 0, s, e0, g1, 0, a); break;
        default: hipExtLaunchKernelGGL(k_decode16<3, false>, grid, block16, 0, s, e0, g1, 0, a); break;
    }
    if (b.any_split) {
        constexpr int TR = Wide<1>::TR;
        static_assert(Wide<3>::TR == TR, "one fix-up geometry for the 16-bit formats");
        hipExtLaunchKernelGGL(k_decode_fix<TR>, dim3((unsigned)b.ntiles * Fix<TR>::PARTS), dim3(256), 0, s, nullptr,
                              e1, 0, a);
    }
    return hipGetLastError();
}

namespace {

constexpr int kPlanThreads = 1024;
constexpr int kMaxRegions = kMaxTilesPerAxis * kMaxTilesPerAxis;

// Exclusive prefix sum of v over the block (kPlanThreads threads); *total = the block's sum.
__device__ inline int plan_scan(int v, int* s_w, int* total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_w[w] = x;
    __syncthreads();
    int off = 0, tot = 0;
    for (int i = 0; i < kPlanThreads / 64; ++i) {
        const int t = s_w[i];
        if (i < w) off += t;
        tot += t;
    }
    __syncthreads();   // s_w is reused by the next scan
    *total = tot;
    return off + x - v;
}

// One block: changed regions (memory versions against the last localized decode), the tiles
// touching them and the boxes of those regions, compacted in list order, then the 16-bit
// GEMM's work units over the changed tiles (the cut decode_units makes: equal consecutive
// K ranges per workgroup, two units where a range crosses a tile border) and the fp32
// kernel's steps per workgroup.
__global__ __launch_bounds__(kPlanThreads) void k_inc_plan(IncPlan a) {
    __shared__ unsigned char dirty[kMaxRegions];
    __shared__ int s_w[kPlanThreads / 64];
    const int tid = threadIdx.x;
    for (int b = tid; b < a.nregions; b += kPlanThreads) {
        const unsigned v0 = a.version[2 * b], v1 = a.version[2 * b + 1];
        dirty[b] = (a.all || v0 != a.seen[2 * b] || v1 != a.seen[2 * b + 1]) ? 1 : 0;
        a.seen[2 * b] = v0;
        a.seen[2 * b + 1] = v1;
    }
    __syncthreads();
    int n = 0;   // changed tiles so far (uniform)
    for (int c0 = 0; c0 < a.ntiles; c0 += kPlanThreads) {
        const int i = c0 + tid;
        int f = 0;
        DTile t{};
        if (i < a.ntiles) {
            t = a.tiles[i];
            const int tx0 = a.col_tx[t.col0], tx1 = a.col_tx[t.col0 + t.ncol - 1];
            for (int tx = tx0; tx <= tx1 && !f; ++tx) f = dirty[t.ty * a.tiles_x + tx];
        }
        int tot;
        const int pos = plan_scan(f, s_w, &tot);
        if (f) a.out_tiles[n + pos] = t;
        n += tot;
    }
    int nb = 0;   // changed regions
    for (int c0 = 0; c0 < a.nregions; c0 += kPlanThreads) {
        const int b = c0 + tid;
        const int f = b < a.nregions ? dirty[b] : 0;
        int tot;
        const int pos = plan_scan(f, s_w, &tot);
        if (f) {
            a.out_boxes[nb + pos] = a.boxes[b];
            a.region_u[2 * b] = 0u;   // their maxima are taken again after the decode
            a.region_u[2 * b + 1] = 0u;
        }
        nb += tot;
    }
    const long long ks = a.ksteps16, total = (long long)n * ks;
    const long long L = unit_range(n, ks, a.slots16);
    const int nwg = total > 0 ? (int)((total + L - 1) / L) : 0;
    int extra = 0;   // units so far beyond one per workgroup (tile borders inside ranges)
    for (int c0 = 0; c0 < nwg; c0 += kPlanThreads) {
        const int w = c0 + tid;
        long long it0 = 0, it1 = 0;
        int t0 = 0, pieces = 0;
        if (w < nwg) {
            it0 = (long long)w * L;
            it1 = min(total, it0 + L);
            t0 = (int)(it0 / ks);
            pieces = (int)((it1 - 1) / ks) - t0 + 1;
        }
        int tot;
        const int pos = plan_scan(pieces > 0 ? pieces - 1 : 0, s_w, &tot);
        if (w < nwg) {
            const int u = w + extra + pos;
            a.wg_u0[w] = u;
            for (int j = 0; j < pieces; ++j) {
                const int t = t0 + j;
                const int kb0 = j == 0 ? (int)(it0 - (long long)t0 * ks) : 0;
                const int kb1 = (int)min(ks, it1 - (long long)t * ks);
                if (kb0 == 0) a.tile_u0[t] = u + j;
                a.units[u + j] = DUnit{t, kb0, kb1, 2 * w + (j == 0 ? 0 : 1)};
            }
        }
        extra += tot;
    }
    if (tid == 0) {
        const int nunits = nwg + extra;
        a.wg_u0[nwg] = nunits;
        a.tile_u0[n] = nunits;
        const long long total32 = (long long)n * a.ksteps32;
        long long L32 = (total32 + a.slots32 - 1) / a.slots32;
        if (L32 < 4) L32 = 4;   // the fp32 plan's shortest range (decode_plan)
        a.dyn[0] = n;
        a.dyn[1] = nwg;
        a.dyn[2] = nb;
        a.dyn[3] = (int)L32;
    }
}

}  // namespace

hipError_t launch_inc_plan(const IncPlan& p, hipStream_t s) {
    if (p.nregions < 1 || p.nregions > kMaxRegions || p.ntiles < 0 || p.ksteps16 < 1 || p.ksteps32 < 1 ||
        p.slots16 < 1 || p.slots32 < 1)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_inc_plan, dim3(1), dim3(kPlanThreads), 0, s, p);
    return hipGetLastError();
}

size_t decode_partial_floats_max(int num_cus) {
    const size_t u16 = decode_unit_partial_floats(2 * decode_slots16(num_cus));
    const size_t f32 = (size_t)decode_slots32(num_cus) * 2 * 2 * kTileRows * kTileCols;
    return std::max(u16, f32);
}

int decode_slots16(int num_cus) { return Wide<1>::OCC * num_cus; }
int decode_slots32(int num_cus) { return kDecodeOccupancy32 * num_cus; }

}  // namespace vsaogm
