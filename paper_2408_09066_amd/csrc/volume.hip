// Volumes: the method of Sec. III with a third axis (the 3-D mapping the paper names as
// future work in Sec. V).  A point's spectrum is exp(i Theta[k].(x, y, z)); tiles are boxes
// numbered beta = (tz * ty_n + ty) * tx_n + tx; the entropy window is the ball of integer voxel
// offsets dx^2 + dy^2 + dz^2 <= r^2.
//
//   k3_assign   nearest tile (exact double-precision argmin over the 3x3x3 neighbourhood of the
//               per-axis guess, lowest index on ties), key 2*beta+psi, label check, per-chunk key
//               histogram; the scan of the histogram into sort offsets and work items, and the
//               final reduction, are the plane encoder's (encode.hip)
//   k3_scatter  stable counting sort of the tile-local coordinates (and their rounding
//               residuals) by key
//   k3_encode   per (work item of one memory's sorted points, block of bins): sum of
//               exp(2 pi i t), t in revolutions, two points per step; a work item whose phases
//               could exceed kWidePhaseRev forms and wraps them in double precision
//   k3_classify_tiled  radii <= kClassify3TiledRadius: per 8x8x8 block, -Q ln Q with
//               Q = (P / max P)^2 of the block and its halo into LDS, ball sums there, softmax
//               difference tanh((H1 - H0)/2), threshold
//   k3_entropy, k3_classify  larger radii: the same in two passes through a scratch buffer
// The similarity of every voxel is the same GEMM as for maps: its rows are the volume's joint
// (z, y) rows, with a cached table of exp(i (Theta_y y + Theta_z z)) as the row operand
// (decode.hip).
#include "internal.h"

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

// One point per thread, blocks of kAssignChunk points; hist[key][chunk] = the chunk's count,
// added with one LDS atomic per key and wavefront.
__global__ __launch_bounds__(kAssignChunk) void k3_assign(const float* __restrict__ xyz,
                                                          const uint8_t* __restrict__ label, int64_t n,
                                                          Layout3Dev L, int nkeys, int nchunks, int key_bits,
                                                          int* __restrict__ key_out, int* __restrict__ hist,
                                                          unsigned long long* __restrict__ n_bad) {
    extern __shared__ int sh_hist[];
    for (int k = threadIdx.x; k < nkeys; k += blockDim.x) sh_hist[k] = 0;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kAssignChunk + threadIdx.x;
    int k = -1;
    if (i < n) {
        const unsigned l = label[i];
        if (l <= 1u) k = 2 * nearest_tile3(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], L) + (int)l;
        if (k < 0) atomicAdd(n_bad, 1ull);
        key_out[i] = k;
    }
    const int lane = threadIdx.x & 63;
    const uint64_t same = same_value_lanes(k < 0 ? (unsigned)nkeys : (unsigned)k, key_bits);
    if (k >= 0 && (same & ((1ull << lane) - 1ull)) == 0) atomicAdd(&sh_hist[k], __popcll(same));
    __syncthreads();
    for (int k = threadIdx.x; k < nkeys; k += blockDim.x) hist[(size_t)k * nchunks + blockIdx.x] = sh_hist[k];
}

// Stable counting-sort scatter, one block of WAVES wavefronts per chunk of kAssignChunk points;
// wave w takes the chunk's w-th part.  Each wave starts every key at the chunk's base plus the
// counts of the earlier waves; within a round of 64 lanes, a point's rank among equal keys comes
// from ballots over the key's bits.  The destination receives the tile-local coordinates,
// formed in double precision and split into fp32 value and residual.
template <int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k3_scatter(const float* __restrict__ xyz, const int* __restrict__ key,
                                                         int64_t n, Layout3Dev L, int nkeys, int nchunks,
                                                         int key_bits, const int* __restrict__ base,
                                                         float4* __restrict__ sorted,
                                                         float4* __restrict__ sorted_lo) {
    extern __shared__ int run[];   // [WAVES][nkeys]
    constexpr int Q = kAssignChunk / WAVES, R = Q / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t q0 = (int64_t)blockIdx.x * kAssignChunk + (int64_t)wave * Q;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int kk[R];
    uint64_t same[R];   // lanes of the round with this lane's key
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = q0 + r * 64 + lane;
        kk[r] = (i < n) ? key[i] : -1;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) same[r] = same_value_lanes(kk[r] < 0 ? (unsigned)nkeys : (unsigned)kk[r], key_bits);
    for (int k = threadIdx.x; k < WAVES * nkeys; k += blockDim.x) run[k] = 0;
    __syncthreads();
    int* my = run + wave * nkeys;
#pragma unroll
    for (int r = 0; r < R; ++r)   // one atomic per key and round
        if (kk[r] >= 0 && (same[r] & lt_mask) == 0) atomicAdd(&my[kk[r]], __popcll(same[r]));
    __syncthreads();
    for (int k = threadIdx.x; k < nkeys; k += blockDim.x) {
        int acc = base[(size_t)k * nchunks + blockIdx.x];
        for (int w = 0; w < WAVES; ++w) {
            const int c = run[w * nkeys + k];
            run[w * nkeys + k] = acc;
            acc += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int k = kk[r];
        if (k >= 0) {
            const int64_t i = q0 + r * 64 + lane;
            const int dest = my[k] + __popcll(same[r] & lt_mask);
            const int b = k >> 1;
            const int tx = b % L.tx, ty = (b / L.tx) % L.ty, tz = b / (L.tx * L.ty);
            const double lx = (double)xyz[3 * i] - L.cx[tx], ly = (double)xyz[3 * i + 1] - L.cy[ty],
                         lz = (double)xyz[3 * i + 2] - L.cz[tz];
            const float fx = (float)lx, fy = (float)ly, fz = (float)lz;
            sorted[dest] = make_float4(fx, fy, fz, 0.f);
            sorted_lo[dest] = make_float4((float)(lx - (double)fx), (float)(ly - (double)fy), (float)(lz - (double)fz), 0.f);
            if ((same[r] & lt_mask) == 0) my[k] += __popcll(same[r]);
        }
        __syncthreads();
    }
}

// Partial spectrum of one work item (consecutive sorted points of one memory) for one block of
// bins; thread t owns bins b0 + t + j kEncodeThreads, j < BPT.  Consecutive points go in pairs:
//   exp(i a) + exp(i b) = 2 cos((a - b) / 2) exp(i (a + b) / 2),
// three hardware sine/cosine evaluations per two points, with the pair's mid-point and
// half-difference formed once in LDS for all bins.
template <int BPT>
__global__ __launch_bounds__(kEncodeThreads) void k3_encode(const float4* __restrict__ sorted,
                                                            const float4* __restrict__ sorted_lo,
                                                            const EChunk* __restrict__ table,
                                                            const int* __restrict__ meta,
                                                            const float4* __restrict__ rev,
                                                            const double* __restrict__ rev_d, float4 max_rev,
                                                            int halfp, float2* __restrict__ partial) {
    const int c = blockIdx.x;
    if (c >= meta[0]) return;
    const EChunk e = table[c];
    const int b0 = blockIdx.y * (kEncodeThreads * BPT) + threadIdx.x;
    const float4* __restrict__ p = sorted + e.start;
    __shared__ float sh_max[kEncodeThreads / 64];
    __shared__ float4 sh_mid[kEncodeChunk / 2], sh_hd[kEncodeChunk / 2];

    // largest phase (revolutions) any bin can reach on the work item's points
    float bound = 0.f;
    for (int q = threadIdx.x; q < e.len; q += kEncodeThreads) {
        const float4 v = p[q];
        bound = fmaxf(bound, fabsf(v.x) * max_rev.x + fabsf(v.y) * max_rev.y + fabsf(v.z) * max_rev.z);
    }
    for (int off = 32; off > 0; off >>= 1) bound = fmaxf(bound, __shfl_xor(bound, off));
    if ((threadIdx.x & 63) == 0) sh_max[threadIdx.x >> 6] = bound;
    __syncthreads();
    float wmax = 0.f;
#pragma unroll
    for (int w = 0; w < kEncodeThreads / 64; ++w) wmax = fmaxf(wmax, sh_max[w]);

    float re[BPT], im[BPT];
#pragma unroll
    for (int j = 0; j < BPT; ++j) re[j] = im[j] = 0.f;
    if (wmax <= kWidePhaseRev) {
        float ax[BPT], ay[BPT], az[BPT];
#pragma unroll
        for (int j = 0; j < BPT; ++j) {
            const int k = b0 + j * kEncodeThreads;
            const float4 t = (k < halfp) ? rev[k] : make_float4(0.f, 0.f, 0.f, 0.f);
            ax[j] = t.x;
            ay[j] = t.y;
            az[j] = t.z;
        }
        const int npairs = e.len >> 1;
        for (int q = threadIdx.x; q < npairs; q += kEncodeThreads) {
            const float4 a = p[2 * q], b = p[2 * q + 1];
            sh_mid[q] = make_float4(0.5f * (a.x + b.x), 0.5f * (a.y + b.y), 0.5f * (a.z + b.z), 0.f);
            sh_hd[q] = make_float4(0.5f * (a.x - b.x), 0.5f * (a.y - b.y), 0.5f * (a.z - b.z), 0.f);
        }
        __syncthreads();
#pragma unroll 2
        for (int q = 0; q < npairs; ++q) {
            const float4 m = sh_mid[q], d = sh_hd[q];
#pragma unroll
            for (int j = 0; j < BPT; ++j) {
                const float tm = __builtin_fmaf(ax[j], m.x, __builtin_fmaf(ay[j], m.y, az[j] * m.z));
                const float td = __builtin_fmaf(ax[j], d.x, __builtin_fmaf(ay[j], d.y, az[j] * d.z));
                const float cd = __builtin_amdgcn_cosf(td);
                re[j] = __builtin_fmaf(cd, __builtin_amdgcn_cosf(tm), re[j]);
                im[j] = __builtin_fmaf(cd, __builtin_amdgcn_sinf(tm), im[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < BPT; ++j) {
            re[j] *= 2.f;
            im[j] *= 2.f;
        }
        if (e.len & 1) {
            const float4 a = p[e.len - 1];
#pragma unroll
            for (int j = 0; j < BPT; ++j) {
                const float t = __builtin_fmaf(ax[j], a.x, __builtin_fmaf(ay[j], a.y, az[j] * a.z));
                re[j] += __builtin_amdgcn_cosf(t);
                im[j] += __builtin_amdgcn_sinf(t);
            }
        }
    } else {
        // large arguments: phase formed and wrapped to [-1/2, 1/2] revolutions in double
        // precision from the double-float local coordinates
        const float4* __restrict__ plo = sorted_lo + e.start;
        double ax[BPT], ay[BPT], az[BPT];
#pragma unroll
        for (int j = 0; j < BPT; ++j) {
            const int k = min(b0 + j * kEncodeThreads, halfp - 1);
            ax[j] = rev_d[3 * k];
            ay[j] = rev_d[3 * k + 1];
            az[j] = rev_d[3 * k + 2];
        }
        for (int q = 0; q < e.len; ++q) {
            const float4 a = p[q], al = plo[q];
            const double x = (double)a.x + (double)al.x, y = (double)a.y + (double)al.y,
                         z = (double)a.z + (double)al.z;
#pragma unroll
            for (int j = 0; j < BPT; ++j) {
                const double t = ax[j] * x + ay[j] * y + az[j] * z;
                const float r = (float)(t - rint(t));
                re[j] += __builtin_amdgcn_cosf(r);
                im[j] += __builtin_amdgcn_sinf(r);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
        const int k = b0 + j * kEncodeThreads;
        if (k < halfp) partial[(size_t)c * halfp + k] = make_float2(re[j], im[j]);
    }
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
    Layout3Dev L{V.cx, V.cy, V.cz, V.tx, V.ty, V.tz, V.x0, V.y0, V.z0, V.wx, V.wy, V.wz};
    hipLaunchKernelGGL(k3_assign, dim3(p.nchunks), dim3(kAssignChunk), nkeys * sizeof(int), s, xyz, label, n, L,
                       nkeys, p.nchunks, key_bits_for(nkeys), w.key, w.hist, w.n_bad);
    launch_key_scan(w.hist, p.nchunks, nkeys, p.echunk, w.table, w.meta, nullptr, s);
    if (4 * nkeys * (int)sizeof(int) <= 65536)
        hipLaunchKernelGGL(k3_scatter<4>, dim3(p.nchunks), dim3(256), 4 * nkeys * sizeof(int), s, xyz, w.key, n, L,
                           nkeys, p.nchunks, key_bits_for(nkeys), w.hist, w.sorted, w.sorted_lo);
    else
        hipLaunchKernelGGL(k3_scatter<1>, dim3(p.nchunks), dim3(64), nkeys * sizeof(int), s, xyz, w.key, n, L,
                           nkeys, p.nchunks, key_bits_for(nkeys), w.hist, w.sorted, w.sorted_lo);
    const dim3 eg(p.max_echunks, p.binblocks);
    const hipEvent_t e0 = profile_start(kStageEncode), e1 = profile_stop(kStageEncode);
    static_assert(kEncodeBpt == 2, "instantiations below");
    if (p.bpt == 1)
        hipExtLaunchKernelGGL(k3_encode<1>, eg, dim3(kEncodeThreads), 0, s, e0, e1, 0, w.sorted, w.sorted_lo, w.table,
                              w.meta, rev, rev_d, max_rev, halfp, w.partial);
    else
        hipExtLaunchKernelGGL(k3_encode<2>, eg, dim3(kEncodeThreads), 0, s, e0, e1, 0, w.sorted, w.sorted_lo, w.table,
                              w.meta, rev, rev_d, max_rev, halfp, w.partial);
    launch_key_reduce(w.partial, w.meta, nkeys, half, halfp, omega, s);
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
