// Volumes: the method of Sec. III with a third axis (the 3-D mapping the paper names as
// future work in Sec. V).  A point's spectrum is exp(i Theta[k].(x, y, z)); tiles are boxes
// numbered beta = (tz * ty_n + ty) * tx_n + tx; the entropy window is the ball of integer voxel
// offsets dx^2 + dy^2 + dz^2 <= r^2.
//
//   k3_assign   nearest tile (exact double-precision argmin over the 3x3x3 neighbourhood of the
//               per-axis guess, lowest index on ties), key 2*beta+psi, tile-local coordinates
//   k3_encode   per (bin block, memory, range of points): sum of exp(2 pi i t) over the range's
//               points of that memory, in point order (deterministic), t in revolutions; a range
//               whose phases could exceed kWidePhaseRev forms and wraps them in double precision
//   k3_reduce   memories += the ranges' partial sums, in range order
//   k3_entropy  -Q ln Q with Q = (P / max P)^2 per voxel and class
//   k3_classify ball sums of the entropy terms, softmax difference tanh((H1 - H0)/2), threshold
// The similarity of every voxel is the same GEMM as for maps, per z slice, with the slice's
// third-axis table folded into the column operand (decode.hip).
#include "internal.h"

namespace vsaogm {
namespace {

constexpr int kV3Threads = 256;
constexpr int kV3Bpt = 4;          // bins per thread
constexpr int kV3Range = 4096;     // points per encode range
constexpr int kV3Stage = 1024;     // points staged in LDS at a time

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

__global__ __launch_bounds__(256) void k3_assign(const float* __restrict__ xyz, const uint8_t* __restrict__ label,
                                                 int64_t n, Layout3Dev L, int* __restrict__ key,
                                                 float4* __restrict__ loc, float4* __restrict__ loc_lo,
                                                 unsigned long long* __restrict__ n_bad) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
    const unsigned l = label[i];
    int k = -1;
    float4 hi = make_float4(0.f, 0.f, 0.f, 0.f), lo = hi;
    if (l <= 1u) {
        const int b = nearest_tile3(x, y, z, L);
        k = 2 * b + (int)l;
        const int tx = b % L.tx, ty = (b / L.tx) % L.ty, tz = b / (L.tx * L.ty);
        const double lx = x - L.cx[tx], ly = y - L.cy[ty], lz = z - L.cz[tz];
        hi = make_float4((float)lx, (float)ly, (float)lz, 0.f);
        lo = make_float4((float)(lx - (double)hi.x), (float)(ly - (double)hi.y), (float)(lz - (double)hi.z), 0.f);
    } else {
        atomicAdd(n_bad, 1ull);
    }
    key[i] = k;
    loc[i] = hi;
    loc_lo[i] = lo;
}

// Block (bin block, key, range): the range's points are staged in LDS; each matching point
// (a uniform test) adds exp(2 pi i t) to the thread's kV3Bpt bins.
__global__ __launch_bounds__(kV3Threads) void k3_encode(const int* __restrict__ key,
                                                        const float4* __restrict__ loc,
                                                        const float4* __restrict__ loc_lo, int64_t n,
                                                        const float4* __restrict__ rev,
                                                        const double* __restrict__ rev_d, float4 max_rev,
                                                        int halfp, int nkeys, float2* __restrict__ partial) {
    const int bb = blockIdx.x, kq = blockIdx.y, range = blockIdx.z;
    const int64_t p0 = (int64_t)range * kV3Range, p1 = min(p0 + kV3Range, n);
    __shared__ int sh_key[kV3Stage];
    __shared__ float4 sh_loc[kV3Stage];
    __shared__ float sh_max[kV3Threads / 64];

    // largest phase (revolutions) the key's points of this range can reach
    float bound = 0.f;
    for (int64_t i = p0 + threadIdx.x; i < p1; i += kV3Threads)
        if (key[i] == kq) {
            const float4 v = loc[i];
            bound = fmaxf(bound, fabsf(v.x) * max_rev.x + fabsf(v.y) * max_rev.y + fabsf(v.z) * max_rev.z);
        }
    for (int off = 32; off > 0; off >>= 1) bound = fmaxf(bound, __shfl_xor(bound, off));
    if ((threadIdx.x & 63) == 0) sh_max[threadIdx.x >> 6] = bound;
    __syncthreads();
    float wmax = 0.f;
#pragma unroll
    for (int w = 0; w < kV3Threads / 64; ++w) wmax = fmaxf(wmax, sh_max[w]);
    const bool wide = wmax > kWidePhaseRev;

    const int b0 = bb * (kV3Threads * kV3Bpt) + threadIdx.x;
    float ax[kV3Bpt], ay[kV3Bpt], az[kV3Bpt], re[kV3Bpt], im[kV3Bpt];
#pragma unroll
    for (int j = 0; j < kV3Bpt; ++j) {
        const int k = b0 + j * kV3Threads;
        const float4 t = (k < halfp) ? rev[k] : make_float4(0.f, 0.f, 0.f, 0.f);
        ax[j] = t.x;
        ay[j] = t.y;
        az[j] = t.z;
        re[j] = im[j] = 0.f;
    }
    for (int64_t s0 = p0; s0 < p1; s0 += kV3Stage) {
        const int m = (int)min((int64_t)kV3Stage, p1 - s0);
        __syncthreads();  // the previous stage's reads are done
        for (int q = threadIdx.x; q < m; q += kV3Threads) {
            sh_key[q] = key[s0 + q];
            sh_loc[q] = loc[s0 + q];
        }
        __syncthreads();
        for (int q = 0; q < m; ++q) {
            if (sh_key[q] != kq) continue;   // uniform over the block
            const float4 v = sh_loc[q];
            if (!wide) {
#pragma unroll
                for (int j = 0; j < kV3Bpt; ++j) {
                    const float t = __builtin_fmaf(ax[j], v.x, __builtin_fmaf(ay[j], v.y, az[j] * v.z));
                    re[j] += __builtin_amdgcn_cosf(t);
                    im[j] += __builtin_amdgcn_sinf(t);
                }
            } else {
                const float4 lo = loc_lo[s0 + q];
                const double x = (double)v.x + (double)lo.x, y = (double)v.y + (double)lo.y,
                             z = (double)v.z + (double)lo.z;
#pragma unroll
                for (int j = 0; j < kV3Bpt; ++j) {
                    const int k = min(b0 + j * kV3Threads, halfp - 1);
                    const double t = rev_d[3 * k] * x + rev_d[3 * k + 1] * y + rev_d[3 * k + 2] * z;
                    const float r = (float)(t - rint(t));
                    re[j] += __builtin_amdgcn_cosf(r);
                    im[j] += __builtin_amdgcn_sinf(r);
                }
            }
        }
    }
    float2* out = partial + ((size_t)range * nkeys + kq) * halfp;
#pragma unroll
    for (int j = 0; j < kV3Bpt; ++j) {
        const int k = b0 + j * kV3Threads;
        if (k < halfp) out[k] = make_float2(re[j], im[j]);
    }
}

__global__ __launch_bounds__(256) void k3_reduce(const float2* __restrict__ partial, int nranges, int nkeys,
                                                 int half, int halfp, float2* __restrict__ omega) {
    const int key = blockIdx.y;
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= half) return;
    float sr = 0.f, si = 0.f;
    for (int r = 0; r < nranges; ++r) {
        const float2 v = partial[((size_t)r * nkeys + key) * halfp + k];
        sr += v.x;
        si += v.y;
    }
    float2* o = omega + (size_t)key * halfp + k;
    const float2 w = *o;
    *o = make_float2(w.x + sr, w.y + si);
}

__global__ __launch_bounds__(256) void k3_entropy(const float* __restrict__ heat, const float* __restrict__ hmax,
                                                  int64_t nvox, float* __restrict__ g) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= nvox) return;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const float m = hmax[p];
        float v = 0.f;
        if (m > 0.f) {
            const float q = (heat[p * nvox + i] / m) * (heat[p * nvox + i] / m);
            v = (q > 0.f) ? -q * __logf(q) : 0.f;
        }
        g[p * nvox + i] = v;
    }
}

// Ball offsets of both classes: off[0 .. n_emp) class 0, off[n_emp .. n_emp + n_occ) class 1.
__global__ __launch_bounds__(256) void k3_classify(const float* __restrict__ g, int nx, int ny, int nz,
                                                   const int4* __restrict__ off, int n_emp, int n_occ,
                                                   float rho, float* __restrict__ ogm, uint8_t* __restrict__ label) {
    const int64_t nvox = (int64_t)nx * ny * nz;
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= nvox) return;
    const int i = (int)(v % nx), j = (int)((v / nx) % ny), l = (int)(v / ((int64_t)nx * ny));
    float h[2] = {0.f, 0.f};
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const int o0 = p ? n_emp : 0, o1 = p ? n_emp + n_occ : n_emp;
        const float* gp = g + p * nvox;
        float s = 0.f;
        for (int o = o0; o < o1; ++o) {
            const int4 d = off[o];
            const int ii = i + d.x, jj = j + d.y, ll = l + d.z;
            if (ii < 0 || jj < 0 || ll < 0 || ii >= nx || jj >= ny || ll >= nz) continue;
            s += gp[((int64_t)ll * ny + jj) * nx + ii];
        }
        h[p] = s;
    }
    const float o = tanhf(0.5f * (h[1] - h[0]));
    if (ogm) ogm[v] = o;
    label[v] = (o >= rho) ? 1 : 0;
}

}  // namespace

int encode3_ranges(int64_t n) { return (int)((n + kV3Range - 1) / kV3Range); }

hipError_t launch_encode3(const float* xyz, const uint8_t* label, int64_t n, const Volume3Dev& V,
                          const float4* rev, const double* rev_d, float4 max_rev, int nkeys, int half,
                          int halfp, int* key, float4* loc, float4* loc_lo, float2* partial,
                          unsigned long long* n_bad, float2* omega, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    Layout3Dev L{V.cx, V.cy, V.cz, V.tx, V.ty, V.tz, V.x0, V.y0, V.z0, V.wx, V.wy, V.wz};
    hipLaunchKernelGGL(k3_assign, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, xyz, label, n, L, key, loc,
                       loc_lo, n_bad);
    const int nranges = encode3_ranges(n);
    const int binblocks = (halfp + kV3Threads * kV3Bpt - 1) / (kV3Threads * kV3Bpt);
    profile_begin(kStageEncode, s);
    hipLaunchKernelGGL(k3_encode, dim3(binblocks, nkeys, nranges), dim3(kV3Threads), 0, s, key, loc, loc_lo, n, rev,
                       rev_d, max_rev, halfp, nkeys, partial);
    profile_end(kStageEncode, s);
    hipLaunchKernelGGL(k3_reduce, dim3((half + 255) / 256, nkeys), dim3(256), 0, s, partial, nranges, nkeys, half,
                       halfp, omega);
    return hipGetLastError();
}

hipError_t launch_classify3(const float* heat, const float* hmax, int nx, int ny, int nz, const int4* offsets,
                            int n_emp, int n_occ, float rho, float* g, float* ogm, uint8_t* label, hipStream_t s) {
    const int64_t nvox = (int64_t)nx * ny * nz;
    const unsigned blocks = (unsigned)((nvox + 255) / 256);
    profile_begin(kStageClassify, s);
    hipLaunchKernelGGL(k3_entropy, dim3(blocks), dim3(256), 0, s, heat, hmax, nvox, g);
    hipLaunchKernelGGL(k3_classify, dim3(blocks), dim3(256), 0, s, g, nx, ny, nz, offsets, n_emp, n_occ, rho, ogm,
                       label);
    profile_end(kStageClassify, s);
    return hipGetLastError();
}

}  // namespace vsaogm
