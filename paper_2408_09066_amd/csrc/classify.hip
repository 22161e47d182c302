// Entropy-based classification (Sec. III-B: eq. non-linearities, Algorithm 2 with the
// local Shannon entropy and disk-mask equations, eqs. softmax, psd and classification).
//
// One block covers TX x TY cells.  The entropy terms g = -Q ln Q, Q = (P / max P)^2, of the
// block and a halo of R = max(r_occ, r_emp) cells are computed once into LDS (zero outside
// the grid, which excludes those neighbours), then each cell sums its disk of integer
// offsets dx^2 + dy^2 <= r^2 per class, and the softmax of the two entropies minus each other
// is tanh((H1 - H0) / 2).  The heatmaps are read once and the map written once.  The ablation
// variants (normalisation / square off, per-cell ReLU, tanh or sigmoid in place of the
// entropy) change only the per-cell value and use a radius of 0.
#include "internal.h"

namespace vsaogm {
namespace {

constexpr int TX = 32, TY = 16;

// Disk sum around the LDS element at `centre` (row pitch W) for a radius known at compile
// time: straight-line reads at constant offsets within each row.
template <int R>
__device__ inline float disk_sum(const float* centre, int W) {
    float s = 0.f;
#pragma unroll
    for (int dy = -R; dy <= R; ++dy) {
        const float* row = centre + dy * W;
#pragma unroll
        for (int dx = -R; dx <= R; ++dx)
            if (dx * dx + dy * dy <= R * R) s += row[dx];
    }
    return s;
}

// Radii up to kFastRadius use the unrolled sums; larger ones the table-driven loop.
constexpr int kFastRadius = 6;

__device__ inline float disk_sum_fast(int r, const float* centre, int W) {
    switch (r) {
        case 0: return disk_sum<0>(centre, W);
        case 1: return disk_sum<1>(centre, W);
        case 2: return disk_sum<2>(centre, W);
        case 3: return disk_sum<3>(centre, W);
        case 4: return disk_sum<4>(centre, W);
        case 5: return disk_sum<5>(centre, W);
        default: return disk_sum<6>(centre, W);
    }
}

// Pre-softmax value of one cell of one class (decoding of Sec. III-B and its ablation of
// Sec. IV-B): q = P (/ max P if normalising, as P times the block's reciprocal inv_m of the class
// maximum, 0 when the maximum is not positive) (squared if squaring), then -q ln q (entropy, to
// be summed over the disk; 0 for q <= 0) or the per-cell activation ReLU / tanh / sigmoid.
__device__ inline float recip_max(float m) { return (m > 0.f) ? 1.f / m : 0.f; }
__device__ inline float cell_value(float p, float inv_m, int normalize, int square, int act) {
    float q = p;
    if (normalize) q = p * inv_m;
    if (square) q = q * q;
    switch (act) {
        case 0: return (q > 0.f) ? -q * __logf(q) : 0.f;
        case 1: return fmaxf(q, 0.f);
        case 2: return tanhf(q);
        default: return 1.f / (1.f + expf(-q));
    }
}

// One block of TX x TY cells, block column bxi and row byi; m0, m1 the class maxima.
__device__ __attribute__((always_inline)) inline void classify_body(const float* __restrict__ heat_, float m0, float m1,
                                                                    int nx, int ny, int r_occ, int r_emp, float rho,
                                                                    int normalize, int square, int act,
                                                                    float* __restrict__ ogm_, uint8_t* __restrict__ label_,
                                                                    int bxi, int byi, float* sg /* LDS */) {
    gmem<float>* __restrict__ heat = as_global(heat_);
    gmem_rw<float>* __restrict__ ogm = ogm_ ? as_global_rw(ogm_) : nullptr;
    gmem_rw<uint8_t>* __restrict__ label = as_global_rw(label_);
    const int R = max(r_occ, r_emp);
    const int W = TX + 2 * R, H = TY + 2 * R;
    __shared__ int half_w[2][2 * kMaxRadius + 1];
    const int bx = bxi * TX, by = byi * TY;
    if (threadIdx.x < 2 * (2 * kMaxRadius + 1)) {
        const int p = threadIdx.x / (2 * kMaxRadius + 1);
        const int dy = threadIdx.x % (2 * kMaxRadius + 1) - kMaxRadius;
        const int r = p ? r_occ : r_emp;
        int w = -1;  // no cell in this row of the disk
        if (dy >= -r && dy <= r) {
            w = 0;
            while ((w + 1) * (w + 1) + dy * dy <= r * r) ++w;
        }
        half_w[p][dy + kMaxRadius] = w;
    }
    const size_t plane = (size_t)nx * ny;
    const float inv0 = recip_max(m0), inv1 = recip_max(m1);
    // the block's cells and halo, both classes, kLoadBatch loads in flight per thread; element
    // idx = class * W * H + yy * W + xx, walked in steps of 256 without integer division (one
    // per thread to start; W >= 32 and H >= 16, so a step moves at most 8 rows and wraps the
    // class at most once)
    constexpr int kLoadBatch = 8;
    const int total = 2 * W * H;
    const int sy = 256 / W, sx = 256 - sy * W;
    int cp = 0, cyy = threadIdx.x / W, cxx = threadIdx.x - (threadIdx.x / W) * W;
    for (int base = 0; base < total; base += 256 * kLoadBatch) {
        float raw[kLoadBatch];
        bool in[kLoadBatch];
        int cls[kLoadBatch];
#pragma unroll
        for (int u = 0; u < kLoadBatch; ++u) {
            const int idx = base + u * 256 + threadIdx.x;
            const int gx = bx - R + cxx, gy = by - R + cyy;
            in[u] = idx < total && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
            cls[u] = cp;
            // outside the grid: a clamped in-bounds address, the value is discarded
            const size_t off = in[u] ? (size_t)cp * plane + (size_t)gy * nx + gx : 0;
            raw[u] = heat[off];
            cxx += sx;
            cyy += sy;
            if (cxx >= W) {
                cxx -= W;
                ++cyy;
            }
            if (cyy >= H) {
                cyy -= H;
                ++cp;
            }
        }
#pragma unroll
        for (int u = 0; u < kLoadBatch; ++u) {
            const int idx = base + u * 256 + threadIdx.x;
            if (idx < total) sg[idx] = in[u] ? cell_value(raw[u], cls[u] ? inv1 : inv0, normalize, square, act) : 0.f;
        }
    }
    __syncthreads();
    for (int c = threadIdx.x; c < TX * TY; c += 256) {
        const int cx = c % TX, cy = c / TX;
        const int gx = bx + cx, gy = by + cy;
        if (gx >= nx || gy >= ny) continue;
        float h[2];
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const int r = p ? r_occ : r_emp;
            const float* base = sg + p * W * H;
            float s = 0.f;
            if (r <= kFastRadius) {
                s = disk_sum_fast(r, base + (cy + R) * W + (cx + R), W);
            } else {
                for (int dy = -r; dy <= r; ++dy) {
                    const int w = half_w[p][dy + kMaxRadius];
                    const float* row = base + (cy + R + dy) * W + (cx + R);
                    for (int dx = -w; dx <= w; ++dx) s += row[dx];
                }
            }
            h[p] = s;
        }
        const float o = tanhf(0.5f * (h[1] - h[0]));
        const size_t off = (size_t)gy * nx + gx;
        if (ogm) ogm[off] = o;
        label[off] = (o >= rho) ? 1 : 0;
    }
}

__global__ __launch_bounds__(256) void k_classify(const float* __restrict__ heat,
                                                  const float* __restrict__ hmax, int nx, int ny,
                                                  int r_occ, int r_emp, float rho, int normalize,
                                                  int square, int act,
                                                  float* __restrict__ ogm,
                                                  uint8_t* __restrict__ label) {
    extern __shared__ float sg[];
    classify_body(heat, hmax[0], hmax[1], nx, ny, r_occ, r_emp, rho, normalize, square, act, ogm, label, blockIdx.x,
                  blockIdx.y, sg);
}

// Batched: the blocks of request r are [block0[r], block0[r + 1]), numbered block column
// fastest; the class maxima come from the ordered maxima of the request's decode, and the
// request's first block also writes them out as floats.
__global__ __launch_bounds__(256) void k_classify_b(const ClassifyReq* __restrict__ qs,
                                                    const int* __restrict__ block0, int nq) {
    extern __shared__ float sg[];
    const int r = batch_job(block0, nq, blockIdx.x);
    const ClassifyReq q = qs[r];
    const int b = blockIdx.x - block0[r];
    const int gx = (q.nx + TX - 1) / TX;
    const float m0 = order_value(as_global(q.hmax_u)[0]), m1 = order_value(as_global(q.hmax_u)[1]);
    if (b == 0 && threadIdx.x == 0 && q.hmax_out) {
        gmem_rw<float>* ho = as_global_rw(q.hmax_out);
        ho[0] = m0;
        ho[1] = m1;
    }
    classify_body(q.heat, m0, m1, q.nx, q.ny, q.r_occ, q.r_emp, q.rho, 1, 1, 0, q.ogm, q.label, b % gx, b / gx, sg);
}

}  // namespace

int classify_blocks(int nx, int ny) { return ((nx + TX - 1) / TX) * ((ny + TY - 1) / TY); }

hipError_t launch_classify_batch(const ClassifyReq* reqs, const int* block0, int nreq, int total_blocks, int max_radius,
                                 hipStream_t s) {
    if (total_blocks == 0) return hipSuccess;
    const size_t lds = 2 * (size_t)(TX + 2 * max_radius) * (TY + 2 * max_radius) * sizeof(float);
    hipExtLaunchKernelGGL(k_classify_b, dim3(total_blocks), dim3(256), lds, s, profile_start(kStageClassify),
                          profile_stop(kStageClassify), 0, reqs, block0, nreq);
    return hipGetLastError();
}

hipError_t launch_classify(const float* heat, const float* hmax, int nx, int ny, int r_occ,
                           int r_emp, float rho, int normalize, int square, int act, float* ogm,
                           uint8_t* label, hipStream_t s) {
    if (act != 0) r_occ = r_emp = 0;  // per-cell activations: the "disk" is the cell itself
    const int R = r_occ > r_emp ? r_occ : r_emp;
    const size_t lds = 2 * (size_t)(TX + 2 * R) * (TY + 2 * R) * sizeof(float);
    hipExtLaunchKernelGGL(k_classify, dim3((nx + TX - 1) / TX, (ny + TY - 1) / TY), dim3(256), lds, s,
                          profile_start(kStageClassify), profile_stop(kStageClassify), 0, heat, hmax, nx, ny,
                          r_occ, r_emp, rho, normalize, square, act, ogm, label);
    return hipGetLastError();
}

}  // namespace vsaogm
