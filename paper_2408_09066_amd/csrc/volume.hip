// Volumes: the method of Sec. III with a third axis (the 3-D mapping the paper names as
// future work in Sec. V).  A point's spectrum is exp(i Theta[k].(x, y, z)); tiles are boxes
// numbered beta = (tz * ty_n + ty) * tx_n + tx; the entropy window is the ball of integer voxel
// offsets dx^2 + dy^2 + dz^2 <= r^2.
//
//   k3_assign, k3_scatter, k3_encode   the map's encode stages (bundle.h) on VolumeGeom: nearest
//               tile (exact double-precision argmin over the 3x3x3 neighbourhood of the per-axis
//               guess, lowest index on ties), key 2*beta+psi, per-chunk key histogram; stable
//               counting sort of the tile-local coordinates; per (work item, block of bins) sum of
//               exp(2 pi i t), two points per step.  The scan of the histogram into sort offsets
//               and work items, and the final reduction, are the map encoder's (encode.hip)
//   k3_classify_tiled  radii <= kClassify3TiledRadius: per 8x8x8 block, -Q ln Q with
//               Q = (P / max P)^2 of the block and its halo into LDS, ball sums there, softmax
//               difference tanh((H1 - H0)/2), threshold
//   k3_entropy, k3_classify  larger radii: the same in two passes through a scratch buffer
// The similarity of every voxel is the same GEMM as for maps: its rows are the volume's joint
// (z, y) rows, with a cached table of exp(i (Theta_y y + Theta_z z)) as the row operand
// (decode.hip).
#include "bundle.h"

namespace vsaogm {
namespace {


struct Layout3Dev {
    const double* cx;
    const double* cy;
    const double* cz;
    int tx, ty, tz;
    double x0, y0, z0, wx, wy, wz;   // layout origin and tile widths
};

__device__ inline int axis_guess(double v, double o, double w, int n) {
    double f = floor((v - o) / w);
    f = fmin(fmax(f, 0.0), (double)(n - 1));
    return (int)f;
}

// Exact argmin of ((dx*dx + dy*dy) + dz*dz) over the 3x3x3 tiles around the per-axis guess,
// candidates visited in increasing beta so that the lowest index wins a tie.
__device__ int nearest_tile3(double x, double y, double z, const Layout3Dev& L) {
    const int gx = axis_guess(x, L.x0, L.wx, L.tx), gy = axis_guess(y, L.y0, L.wy, L.ty),
              gz = axis_guess(z, L.z0, L.wz, L.tz);
    int best = -1;
    double bd = INFINITY;
    for (int tz = max(gz - 1, 0); tz <= min(gz + 1, L.tz - 1); ++tz)
        for (int ty = max(gy - 1, 0); ty <= min(gy + 1, L.ty - 1); ++ty)
            for (int tx = max(gx - 1, 0); tx <= min(gx + 1, L.tx - 1); ++tx) {
                const double dx = __dadd_rn(x, -L.cx[tx]), dy = __dadd_rn(y, -L.cy[ty]),
                             dz = __dadd_rn(z, -L.cz[tz]);
                const double d = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
                if (d < bd) {
                    bd = d;
                    best = (tz * L.ty + ty) * L.tx + tx;
                }
            }
    return best;
}

// The encode of a volume, as one record that the shared bodies read (member names as for a map's
// encode).
struct EncodeReq3 {
    const float* xyz;               // [n][3] world metres
    const uint8_t* label;           // [n]
    int64_t n;
    Layout3Dev L;
    int nkeys, key_bits, nchunks, max_echunks;
    int* key;
    int* hist;
    EChunk* table;
    int* meta;
    float4* sorted;                 // [n] local (x, y, z, 0)
    float4* sorted_lo;              // [n] rounding residuals
    float2* partial;
    unsigned long long* n_bad;
    const float4* rev;              // [halfp] (x, y, z, 0) revolutions per metre
    const double* rev_d;            // [halfp][3]
    float4 max_rev;
    int half, halfp;
    int direct_single;              // as for maps: a memory with one work item is written directly
    float2* omega;
};

struct D3 {
    double x, y, z;
};
struct Pair3 {
    float4 m, d;   // mid-point, half-difference (w unused)
};

// The volume: points (x, y, z), tiles numbered beta = (tz * ty_n + ty) * tx_n + tx.
struct VolumeGeom {
    using Src = float3;
    using Pt = float4;
    using Rev = float4;
    using RevD = D3;
    using Pair = Pair3;
    __device__ static float3 src0() { return make_float3(0.f, 0.f, 0.f); }
    __device__ static float3 load(const EncodeReq3& q, int64_t i) {
        gmem<float>* __restrict__ p = as_global(q.xyz) + 3 * i;
        return make_float3(p[0], p[1], p[2]);
    }
    __device__ static int nearest(const EncodeReq3& q, float3 p) { return nearest_tile3(p.x, p.y, p.z, q.L); }
    __device__ static void local(const EncodeReq3& q, int beta, float3 s, float4& h, float4& l) {
        const Layout3Dev& L = q.L;
        const int tx = beta % L.tx, ty = (beta / L.tx) % L.ty, tz = beta / (L.tx * L.ty);
        const double lx = (double)s.x - as_global(L.cx)[tx], ly = (double)s.y - as_global(L.cy)[ty],
                     lz = (double)s.z - as_global(L.cz)[tz];
        const float fx = (float)lx, fy = (float)ly, fz = (float)lz;
        h = make_float4(fx, fy, fz, 0.f);
        l = make_float4((float)(lx - (double)fx), (float)(ly - (double)fy), (float)(lz - (double)fz), 0.f);
    }
    __device__ static float reach(float4 v, float4 m) {
        return fabsf(v.x) * m.x + fabsf(v.y) * m.y + fabsf(v.z) * m.z;
    }
    __device__ static Pair3 pair(float4 a, float4 b) {
        return Pair3{make_float4(0.5f * (a.x + b.x), 0.5f * (a.y + b.y), 0.5f * (a.z + b.z), 0.f),
                     make_float4(0.5f * (a.x - b.x), 0.5f * (a.y - b.y), 0.5f * (a.z - b.z), 0.f)};
    }
    __device__ static float phase(float4 r, float4 p) {
        return __builtin_fmaf(r.x, p.x, __builtin_fmaf(r.y, p.y, r.z * p.z));
    }
    __device__ static float mid(float4 r, const Pair3& pr) { return phase(r, pr.m); }
    __device__ static float half(float4 r, const Pair3& pr) { return phase(r, pr.d); }
    __device__ static double wide(const D3& r, float4 h, float4 l) {
        const double x = (double)h.x + (double)l.x, y = (double)h.y + (double)l.y, z = (double)h.z + (double)l.z;
        return r.x * x + r.y * y + r.z * z;
    }
    __device__ static float4 rev0() { return make_float4(0.f, 0.f, 0.f, 0.f); }
    __device__ static float4 rev(const EncodeReq3& q, int k) { return as_global(q.rev)[k]; }
    __device__ static D3 rev_d0() { return D3{0.0, 0.0, 0.0}; }
    __device__ static D3 rev_d(const EncodeReq3& q, int k) {
        gmem<double>* __restrict__ p = as_global(q.rev_d) + 3 * k;
        return D3{p[0], p[1], p[2]};
    }
    __device__ static float4 max_rev(const EncodeReq3& q) { return q.max_rev; }
};

__global__ __launch_bounds__(kAssignChunk) void k3_assign(EncodeReq3 q) {
    extern __shared__ int sh_hist[];
    assign_points<VolumeGeom>(q, blockIdx.x, sh_hist);
}
template <int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k3_scatter(EncodeReq3 q) {
    extern __shared__ int run[];   // [WAVES][nkeys]
    scatter_points<WAVES, VolumeGeom>(q, blockIdx.x, run);
}
template <int BPT>
__global__ __launch_bounds__(kEncodeThreads) void k3_encode(EncodeReq3 q) {
    encode_points<BPT, VolumeGeom>(q, blockIdx.x);
}

// Entropy term -Q ln Q of one similarity, Q = (P / max P)^2 (0 when the class maximum is not
// positive or Q is 0).
__device__ inline float entropy_term(float h, float m) {
    if (!(m > 0.f)) return 0.f;
    const float q = (h / m) * (h / m);
    return (q > 0.f) ? -q * __logf(q) : 0.f;
}

__global__ __launch_bounds__(256) void k3_entropy(const float* __restrict__ heat, const float* __restrict__ hmax,
                                                  int64_t nvox, float* __restrict__ g) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= nvox) return;
#pragma unroll
    for (int p = 0; p < 2; ++p) g[p * nvox + i] = entropy_term(heat[p * nvox + i], hmax[p]);
}

// Radii up to R in one kernel: a block of kB3^3 voxels computes the entropy terms of its voxels
// and a halo of R into LDS (zero outside the volume, which excludes those neighbours), then sums
// each voxel's balls there (offsets with dz, then dy, then dx increasing).
constexpr int kB3 = 8;
template <int R>
__global__ __launch_bounds__(256) void k3_classify_tiled(const float* __restrict__ heat,
                                                         const float* __restrict__ hmax, int nx, int ny, int nz,
                                                         int r_emp, int r_occ, float rho,
                                                         float* __restrict__ ogm, uint8_t* __restrict__ label) {
    constexpr int W = kB3 + 2 * R, W3 = W * W * W;
    __shared__ float sg[2 * W3];
    const int bx = blockIdx.x * kB3, by = blockIdx.y * kB3, bz = blockIdx.z * kB3;
    const int64_t nvox = (int64_t)nx * ny * nz;
    const float m0 = hmax[0], m1 = hmax[1];
    constexpr int kLoadBatch = 8;   // loads in flight per thread
    for (int base = 0; base < 2 * W3; base += 256 * kLoadBatch) {
        float raw[kLoadBatch];
        bool in[kLoadBatch];
#pragma unroll
        for (int u = 0; u < kLoadBatch; ++u) {
            const int idx = base + u * 256 + threadIdx.x;
            const int p = idx >= W3, rem = idx - p * W3;
            const int gx = bx - R + rem % W, gy = by - R + (rem / W) % W, gz = bz - R + rem / (W * W);
            in[u] = idx < 2 * W3 && gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz;
            raw[u] = heat[in[u] ? p * nvox + ((int64_t)gz * ny + gy) * nx + gx : 0];
        }
#pragma unroll
        for (int u = 0; u < kLoadBatch; ++u) {
            const int idx = base + u * 256 + threadIdx.x;
            if (idx < 2 * W3) sg[idx] = in[u] ? entropy_term(raw[u], idx >= W3 ? m1 : m0) : 0.f;
        }
    }
    __syncthreads();
    for (int c = threadIdx.x; c < kB3 * kB3 * kB3; c += 256) {
        const int cx = c % kB3, cy = (c / kB3) % kB3, cz = c / (kB3 * kB3);
        const int gx = bx + cx, gy = by + cy, gz = bz + cz;
        if (gx >= nx || gy >= ny || gz >= nz) continue;
        float h[2];
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const int r = p ? r_occ : r_emp;
            const float* ctr = sg + p * W3 + ((cz + R) * W + (cy + R)) * W + (cx + R);
            float sum = 0.f;
            if (r == R) {   // the ball of the tile's radius: offsets known at compile time
#pragma unroll
                for (int dz = -R; dz <= R; ++dz)
#pragma unroll
                    for (int dy = -R; dy <= R; ++dy)
#pragma unroll
                        for (int dx = -R; dx <= R; ++dx)
                            if (dx * dx + dy * dy + dz * dz <= R * R) sum += ctr[(dz * W + dy) * W + dx];
            } else {
                for (int dz = -r; dz <= r; ++dz)
                    for (int dy = -r; dy <= r; ++dy) {
                        const int e2 = r * r - dz * dz - dy * dy;
                        if (e2 < 0) continue;
                        const float* row = ctr + (dz * W + dy) * W;
                        for (int dx = -r; dx <= r; ++dx)
                            if (dx * dx <= e2) sum += row[dx];
                    }
            }
            h[p] = sum;
        }
        const float o = tanhf(0.5f * (h[1] - h[0]));
        const int64_t v = ((int64_t)gz * ny + gy) * nx + gx;
        if (ogm) ogm[v] = o;
        label[v] = (o >= rho) ? 1 : 0;
    }
}

// Sum of g over the ball |d| <= r around voxel (i, j, l), offsets visited with dz, then dy, then
// dx increasing; voxels outside the volume contribute nothing.
__device__ inline float ball_sum(const float* __restrict__ g, int i, int j, int l, int nx, int ny, int nz, int r) {
    float s = 0.f;
    const int r2 = r * r;
    for (int dz = -r; dz <= r; ++dz) {
        const int ll = l + dz;
        for (int dy = -r; dy <= r; ++dy) {
            const int jj = j + dy;
            const int e2 = r2 - dz * dz - dy * dy;
            if (e2 < 0 || ll < 0 || ll >= nz || jj < 0 || jj >= ny) continue;
            const float* row = g + ((int64_t)ll * ny + jj) * nx;
            for (int dx = -r; dx <= r; ++dx) {
                const int ii = i + dx;
                if (dx * dx <= e2 && ii >= 0 && ii < nx) s += row[ii];
            }
        }
    }
    return s;
}

// The same sum for a radius known at compile time: straight-line code whose loads do not depend
// on the running sum, so they can all be in flight together (addresses clamped into the
// volume, values outside it masked to zero); same offset order.
template <int R>
__device__ inline float ball_sum_fixed(const float* __restrict__ g, int i, int j, int l, int nx, int ny, int nz) {
    float s = 0.f;
#pragma unroll
    for (int dz = -R; dz <= R; ++dz)
#pragma unroll
        for (int dy = -R; dy <= R; ++dy)
#pragma unroll
            for (int dx = -R; dx <= R; ++dx)
                if (dx * dx + dy * dy + dz * dz <= R * R) {   // compile-time after unrolling
                    const int ii = i + dx, jj = j + dy, ll = l + dz;
                    const bool in = ii >= 0 && ii < nx && jj >= 0 && jj < ny && ll >= 0 && ll < nz;
                    const float x = g[in ? ((int64_t)ll * ny + jj) * nx + ii : 0];
                    s += in ? x : 0.f;
                }
    return s;
}

__device__ inline float ball_sum_any(const float* __restrict__ g, int i, int j, int l, int nx, int ny, int nz,
                                     int r) {
    switch (r) {
        case 0: return ball_sum_fixed<0>(g, i, j, l, nx, ny, nz);
        case 1: return ball_sum_fixed<1>(g, i, j, l, nx, ny, nz);
        case 2: return ball_sum_fixed<2>(g, i, j, l, nx, ny, nz);
        default: return ball_sum(g, i, j, l, nx, ny, nz, r);
    }
}

// Class 0 sums over the ball of radius r_emp, class 1 over radius r_occ.
__global__ __launch_bounds__(256) void k3_classify(const float* __restrict__ g, int nx, int ny, int nz, int r_emp,
                                                   int r_occ, float rho, float* __restrict__ ogm,
                                                   uint8_t* __restrict__ label) {
    const int64_t nvox = (int64_t)nx * ny * nz;
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= nvox) return;
    const int i = (int)(v % nx), j = (int)((v / nx) % ny), l = (int)(v / ((int64_t)nx * ny));
    const float h0 = ball_sum_any(g, i, j, l, nx, ny, nz, r_emp);
    const float h1 = ball_sum_any(g + nvox, i, j, l, nx, ny, nz, r_occ);
    const float o = tanhf(0.5f * (h1 - h0));
    if (ogm) ogm[v] = o;
    label[v] = (o >= rho) ? 1 : 0;
}

int key_bits_for(int v) {
    int b = 0;
    while ((1 << b) <= v) ++b;
    return b;
}

}  // namespace

hipError_t launch_encode3(const float* xyz, const uint8_t* label, int64_t n, const Volume3Dev& V,
                          const float4* rev, const double* rev_d, float4 max_rev, int nkeys, int half,
                          int halfp, const Encode3Work& w, float2* omega, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const EncodePlan p = encode_plan(n, halfp, nkeys);
    EncodeReq3 q{};
    q.xyz = xyz;
    q.label = label;
    q.n = n;
    q.L = Layout3Dev{V.cx, V.cy, V.cz, V.tx, V.ty, V.tz, V.x0, V.y0, V.z0, V.wx, V.wy, V.wz};
    q.nkeys = nkeys;
    q.key_bits = key_bits_for(nkeys);
    q.nchunks = p.nchunks;
    q.max_echunks = p.max_echunks;
    q.key = w.key;
    q.hist = w.hist;
    q.table = w.table;
    q.meta = w.meta;
    q.sorted = w.sorted;
    q.sorted_lo = w.sorted_lo;
    q.partial = w.partial;
    q.n_bad = w.n_bad;
    q.rev = rev;
    q.rev_d = rev_d;
    q.max_rev = max_rev;
    q.half = half;
    q.halfp = halfp;
    q.direct_single = 1;
    q.omega = omega;
    hipLaunchKernelGGL(k3_assign, dim3(p.nchunks), dim3(kAssignChunk), nkeys * sizeof(int), s, q);
    launch_key_scan(w.hist, p.nchunks, nkeys, p.echunk, w.table, w.meta, nullptr, s);
    if (4 * nkeys * (int)sizeof(int) <= 65536)
        hipLaunchKernelGGL(k3_scatter<4>, dim3(p.nchunks), dim3(256), 4 * nkeys * sizeof(int), s, q);
    else
        hipLaunchKernelGGL(k3_scatter<1>, dim3(p.nchunks), dim3(64), nkeys * sizeof(int), s, q);
    const unsigned eblocks = (unsigned)p.max_echunks * (unsigned)p.binblocks;
    const hipEvent_t e0 = profile_start(kStageEncode), e1 = profile_stop(kStageEncode);
    static_assert(kEncodeBpt == 2, "instantiations below");
    if (p.bpt == 1)
        hipExtLaunchKernelGGL(k3_encode<1>, dim3(eblocks), dim3(kEncodeThreads), 0, s, e0, e1, 0, q);
    else
        hipExtLaunchKernelGGL(k3_encode<2>, dim3(eblocks), dim3(kEncodeThreads), 0, s, e0, e1, 0, q);
    launch_key_reduce(w.partial, w.meta, nkeys, half, halfp, 1, omega, s);
    return hipGetLastError();
}

hipError_t launch_classify3(const float* heat, const float* hmax, int nx, int ny, int nz, int r_emp, int r_occ,
                            float rho, float* g, float* ogm, uint8_t* label, hipStream_t s) {
    const int R = r_emp > r_occ ? r_emp : r_occ;
    const hipEvent_t e0 = profile_start(kStageClassify), e1 = profile_stop(kStageClassify);
    if (R <= kClassify3TiledRadius) {
        const dim3 grid((nx + kB3 - 1) / kB3, (ny + kB3 - 1) / kB3, (nz + kB3 - 1) / kB3);
        const dim3 block(256);
        switch (R) {
            case 0: hipExtLaunchKernelGGL(k3_classify_tiled<0>, grid, block, 0, s, e0, e1, 0, heat, hmax, nx, ny, nz, r_emp, r_occ, rho, ogm, label); break;
            case 1: hipExtLaunchKernelGGL(k3_classify_tiled<1>, grid, block, 0, s, e0, e1, 0, heat, hmax, nx, ny, nz, r_emp, r_occ, rho, ogm, label); break;
            case 2: hipExtLaunchKernelGGL(k3_classify_tiled<2>, grid, block, 0, s, e0, e1, 0, heat, hmax, nx, ny, nz, r_emp, r_occ, rho, ogm, label); break;
            case 3: hipExtLaunchKernelGGL(k3_classify_tiled<3>, grid, block, 0, s, e0, e1, 0, heat, hmax, nx, ny, nz, r_emp, r_occ, rho, ogm, label); break;
            default: hipExtLaunchKernelGGL(k3_classify_tiled<4>, grid, block, 0, s, e0, e1, 0, heat, hmax, nx, ny, nz, r_emp, r_occ, rho, ogm, label); break;
        }
        return hipGetLastError();
    }
    if (!g) return hipErrorInvalidValue;   // larger radii need the entropy scratch
    const int64_t nvox = (int64_t)nx * ny * nz;
    const unsigned blocks = (unsigned)((nvox + 255) / 256);
    hipExtLaunchKernelGGL(k3_entropy, dim3(blocks), dim3(256), 0, s, e0, nullptr, 0, heat, hmax, nvox, g);
    hipExtLaunchKernelGGL(k3_classify, dim3(blocks), dim3(256), 0, s, nullptr, e1, 0, g, nx, ny, nz, r_emp, r_occ,
                          rho, ogm, label);
    return hipGetLastError();
}

}  // namespace vsaogm
