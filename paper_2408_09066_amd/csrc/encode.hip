// Encoding and bundling (Sec. III-B "Encoding Point Clouds", Algorithm 1) on gfx950.
//
// A point gamma_i with class psi_i is fractionally bound (2-D encoding equation) into the
// spectrum exp(i*Theta[k].gamma_i) and added (eq. bundling) to memory 2*beta+psi_i of its
// nearest tile beta.  Memories are kept in tile-local coordinates,
//   Omega_local[key][k] = sum_i exp(i*Theta[k].(gamma_i - mu_beta)),
// which is exp(-i*Theta[k].mu_beta) times the paper's memory; the decode queries cells in
// the same local frame, so the factor cancels exactly in every similarity, while the phases
// stay small enough for single precision.
//
// Pipeline (all on the stream, no host synchronisation):
//   k_assign   nearest tile (exact double-precision argmin, lowest index on ties), key,
//              label check, per-chunk key histogram
//   k_scan     per-key totals and exclusive bases, encode work table
//   k_scatter  stable counting sort of the local coordinates by key (four wavefronts per chunk)
//   k_encode   per (work item, block of bins): sum of exp(2*pi*i*t) with t in revolutions,
//              hardware v_sin/v_cos, two points per step:
//                exp(i a) + exp(i b) = 2 cos((a-b)/2) exp(i (a+b)/2)
//   k_reduce   fixed-order sum of the work items' partial spectra into the memories
#include "internal.h"

namespace vsaogm {
namespace {

__device__ inline int nearest_tile(double x, double y, const LayoutDev& L) {
    // Guess by the per-axis floor, then evaluate the exact squared distances of the 3x3
    // neighbourhood in increasing tile order (row-major), keeping the first strict minimum.
    double gx = fmin(fmax((x - L.x0) * L.inv_wx, -1.0), (double)L.tiles_x);
    double gy = fmin(fmax((y - L.y0) * L.inv_wy, -1.0), (double)L.tiles_y);
    int ex = (int)floor(gx), ey = (int)floor(gy);
    int i0 = max(ex - 1, 0), i1 = min(ex + 1, L.tiles_x - 1);
    int j0 = max(ey - 1, 0), j1 = min(ey + 1, L.tiles_y - 1);
    int best = -1;
    double bd = INFINITY;
    for (int j = j0; j <= j1; ++j) {
        double dy = __dsub_rn(y, L.cy[j]);
        double dy2 = __dmul_rn(dy, dy);
        for (int i = i0; i <= i1; ++i) {
            double dx = __dsub_rn(x, L.cx[i]);
            double d2 = __dadd_rn(__dmul_rn(dx, dx), dy2);
            if (d2 < bd) {
                bd = d2;
                best = j * L.tiles_x + i;
            }
        }
    }
    return best;
}

// One point per thread; blocks of kAssignChunk points.  hist is key-major:
// hist[key][chunk] = number of the chunk's points with that key.  The lanes of a wavefront
// holding one key add their count with one LDS atomic (a chunk's points share few keys).
__global__ __launch_bounds__(kAssignChunk) void k_assign(const float2* __restrict__ xy,
                                                         const uint8_t* __restrict__ label,
                                                         int64_t n, LayoutDev L, int nkeys,
                                                         int nchunks, int key_bits, int* __restrict__ key_out,
                                                         int* __restrict__ hist,
                                                         unsigned long long* __restrict__ n_bad) {
    extern __shared__ int sh_hist[];
    for (int k = threadIdx.x; k < nkeys; k += blockDim.x) sh_hist[k] = 0;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kAssignChunk + threadIdx.x;
    int key = -1;
    if (i < n) {
        const float2 p = xy[i];
        const unsigned l = label[i];
        if (l <= 1u) {
            const int b = nearest_tile((double)p.x, (double)p.y, L);
            if (b >= 0) key = 2 * b + (int)l;
        }
        if (key < 0) atomicAdd(n_bad, 1ull);
        key_out[i] = key;
    }
    const int lane = threadIdx.x & 63;
    const uint64_t same = same_value_lanes(key < 0 ? (unsigned)nkeys : (unsigned)key, key_bits);
    if (key >= 0 && (same & ((1ull << lane) - 1ull)) == 0) atomicAdd(&sh_hist[key], __popcll(same));
    __syncthreads();
    for (int k = threadIdx.x; k < nkeys; k += blockDim.x)
        hist[(size_t)k * nchunks + blockIdx.x] = sh_hist[k];
}

// Exclusive scan across a block of kScanThreads threads; returns the block total in *total.
constexpr int kScanThreads = 1024;
constexpr int kScanGroup = 16;     // histogram entries per thread and pass
static_assert(kScanGroup <= kHistPad && kScanGroup % 4 == 0, "aligned group reads stay in the padding");
__device__ int block_scan_excl(int v, int* sh_w, int* total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int x = v;
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) sh_w[wv] = x;
    __syncthreads();
    if (wv == 0) {
        int t = (lane < kScanThreads / 64) ? sh_w[lane] : 0;
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(t, off);
            if (lane >= off) t += y;
        }
        if (lane < kScanThreads / 64) sh_w[lane] = t;
    }
    __syncthreads();
    const int before = (wv > 0) ? sh_w[wv - 1] : 0;
    *total = sh_w[kScanThreads / 64 - 1];
    __syncthreads();
    return before + x - v;
}

// One block.  The key-major histogram becomes, by one flat exclusive scan, the destination
// base of every (key, chunk) -- the stable counting sort's offsets.  Then per key: point
// count, encode work items and their table.
__global__ __launch_bounds__(kScanThreads) void k_scan(int* __restrict__ hist, int nchunks,
                                                       int nkeys, int echunk,
                                                       EChunk* __restrict__ table,
                                                       int* __restrict__ meta,
                                                       unsigned* __restrict__ version) {
    __shared__ int sh_w[kScanThreads / 64];
    extern __shared__ int key_start[];   // [nkeys]
    const int64_t N = (int64_t)nkeys * nchunks;
    // coalesced passes of kScanThreads * kScanGroup entries (one aligned group per thread; the
    // histogram buffer is padded so the last group stays in bounds); the next pass's group is
    // loaded before the current pass is scanned
    constexpr int G = kScanGroup;
    constexpr int64_t PASS = (int64_t)kScanThreads * G;
    typedef int i32x4 __attribute__((ext_vector_type(4)));
    auto load_group = [&](int64_t j, i32x4 (&dst)[G / 4]) {
        const i32x4* src = reinterpret_cast<const i32x4*>(hist + min(j, N - 1) / G * G);
#pragma unroll
        for (int u = 0; u < G / 4; ++u) dst[u] = src[u];
    };
    int carry = 0;
    i32x4 nxt[G / 4];
    load_group((int64_t)threadIdx.x * G, nxt);
    for (int64_t base = 0; base < N; base += PASS) {
        const int64_t j0 = base + (int64_t)threadIdx.x * G;
        int v[G];
#pragma unroll
        for (int u = 0; u < G; ++u) v[u] = (j0 + u < N) ? nxt[u / 4][u % 4] : 0;
        if (base + PASS < N) load_group(j0 + PASS, nxt);
        int sum = 0;
#pragma unroll
        for (int u = 0; u < G; ++u) sum += v[u];
        int total;
        int run = carry + block_scan_excl(sum, sh_w, &total);
        if (j0 + G <= N) {
            i32x4* dst = reinterpret_cast<i32x4*>(hist + j0);
#pragma unroll
            for (int q = 0; q < G / 4; ++q) {
                i32x4 out;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    out[u] = run;
                    run += v[4 * q + u];
                }
                dst[q] = out;
            }
        } else {
#pragma unroll
            for (int u = 0; u < G; ++u) {
                if (j0 + u < N) hist[j0 + u] = run;
                run += v[u];
            }
        }
        carry += total;
    }
    __syncthreads();  // the bases written above are visible to the whole block
    for (int k = threadIdx.x; k < nkeys; k += kScanThreads) key_start[k] = hist[(int64_t)k * nchunks];
    __syncthreads();
    const int n_valid = carry;
    // per-key counts and work items (keys in slices of kScanThreads, scanned in order)
    int ec_carry = 0;
    for (int k0 = 0; k0 < nkeys; k0 += kScanThreads) {
        const int k = k0 + threadIdx.x;
        int start = 0, cnt = 0, ne = 0;
        if (k < nkeys) {
            start = key_start[k];
            const int next = (k + 1 < nkeys) ? key_start[k + 1] : n_valid;
            cnt = next - start;
            ne = (cnt + echunk - 1) / echunk;
        }
        int total;
        const int e0 = ec_carry + block_scan_excl(ne, sh_w, &total);
        if (k < nkeys) {
            meta[1 + k] = e0;
            meta[1 + nkeys + k] = ne;
            meta[1 + 2 * nkeys + k] = cnt;
            if (version && cnt > 0) version[k] += 1u;  // the memory changes: decodes of it are stale
        }
        ec_carry += total;
    }
    if (threadIdx.x == 0) meta[0] = ec_carry;
    __syncthreads();  // meta's first-item offsets are visible to the whole block
    // the work table, one entry per thread: its key is the last whose first item is <= the entry
    // (keys without items share their successor's offset and are passed over)
    const int* e_first = meta + 1;
    for (int idx = threadIdx.x; idx < ec_carry; idx += kScanThreads) {
        int lo = 0, hi = nkeys;   // e_first[lo] <= idx < e_first[hi] (e_first[nkeys] taken as +inf)
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (e_first[mid] <= idx) lo = mid;
            else hi = mid;
        }
        const int j = idx - e_first[lo];
        EChunk e;
        e.key = lo;
        e.start = key_start[lo] + j * echunk;
        e.len = min(echunk, meta[1 + 2 * nkeys + lo] - j * echunk);
        e.pad = 0;
        table[idx] = e;
    }
}

// Stable counting-sort scatter: one block of WAVES wavefronts per chunk of kAssignChunk points,
// wave w taking the chunk's w-th part in order (four waves; one when the per-wave key tables
// would not fit the LDS of a workgroup).  The waves' key counts give each wave its
// own running base per key (the chunk's base plus the counts of the earlier quarters); within a
// wave, a point's slot is its key's running base plus the number of earlier lanes of the same
// round with the same key (lanes are matched bit by bit with ballots).
template <int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_scatter(const float2* __restrict__ xy,
                                                const int* __restrict__ key, int64_t n,
                                                LayoutDev L, int nkeys, int nchunks, int key_bits,
                                                const int* __restrict__ base,
                                                float2* __restrict__ sorted,
                                                float2* __restrict__ sorted_lo) {
    extern __shared__ int run[];  // [WAVES][nkeys]
    constexpr int Q = kAssignChunk / WAVES;           // points per wave
    constexpr int R = Q / 64;                         // rounds per wave
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t q0 = (int64_t)blockIdx.x * kAssignChunk + (int64_t)wave * Q;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int kk[R];
    float2 pp[R];
    uint64_t same[R];   // lanes of the round with this lane's key
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = q0 + r * 64 + lane;
        kk[r] = (i < n) ? key[i] : -1;
        pp[r] = (i < n) ? xy[i] : make_float2(0.f, 0.f);
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
    for (int k = threadIdx.x; k < nkeys; k += blockDim.x) {  // counts -> per-wave bases
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
            const int rank = __popcll(same[r] & lt_mask);
            const int dest = my[k] + rank;
            const int beta = k >> 1;
            const int tx = beta % L.tiles_x, ty = beta / L.tiles_x;
            const double lx = (double)pp[r].x - L.cx[tx];
            const double ly = (double)pp[r].y - L.cy[ty];
            const float fx = (float)lx, fy = (float)ly;
            sorted[dest] = make_float2(fx, fy);
            sorted_lo[dest] = make_float2((float)(lx - (double)fx), (float)(ly - (double)fy));
            if ((same[r] & lt_mask) == 0) my[k] += __popcll(same[r]);
        }
        __syncthreads();
    }
}

// Partial spectra of one work item for one block of bins.  Thread t owns bins
// b0 + t + j*256, j < BPT; the points are read as wave-uniform (scalar) loads.
template <int BPT>
__global__ __launch_bounds__(kEncodeThreads) void k_encode(
    const float2* __restrict__ sorted, const float2* __restrict__ sorted_lo,
    const EChunk* __restrict__ table, const int* __restrict__ meta,
    const float2* __restrict__ rev, const double2* __restrict__ rev_d, float max_rev_x,
    float max_rev_y, int halfp, float2* __restrict__ partial) {
    const int c = blockIdx.x;
    if (c >= meta[0]) return;
    const EChunk e = table[c];
    const int b0 = blockIdx.y * (kEncodeThreads * BPT) + threadIdx.x;
    const float2* __restrict__ p = sorted + e.start;

    // Largest phase (revolutions) any bin can reach on this work item's points.
    __shared__ float sh_max[kEncodeThreads / 64];
    __shared__ float4 sh_pair[kEncodeChunk / 2];
    float bound = 0.f;
    for (int q = threadIdx.x; q < e.len; q += kEncodeThreads) {
        float2 v = p[q];
        bound = fmaxf(bound, fabsf(v.x) * max_rev_x + fabsf(v.y) * max_rev_y);
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
        float ax[BPT], ay[BPT];
#pragma unroll
        for (int j = 0; j < BPT; ++j) {
            const int k = b0 + j * kEncodeThreads;
            float2 t = (k < halfp) ? rev[k] : make_float2(0.f, 0.f);
            ax[j] = t.x;
            ay[j] = t.y;
        }
        // pair mid-points and half-differences, formed once per pair for all bins
        const int npairs = e.len >> 1;
        for (int q = threadIdx.x; q < npairs; q += kEncodeThreads) {
            const float2 a = p[2 * q], b = p[2 * q + 1];
            sh_pair[q] = make_float4(0.5f * (a.x + b.x), 0.5f * (a.y + b.y), 0.5f * (a.x - b.x),
                                     0.5f * (a.y - b.y));
        }
        __syncthreads();
#pragma unroll 2
        for (int q = 0; q < npairs; ++q) {
            const float4 pq = sh_pair[q];
            const float mx = pq.x, my = pq.y, dx = pq.z, dy = pq.w;
#pragma unroll
            for (int j = 0; j < BPT; ++j) {
                const float tm = __builtin_fmaf(ax[j], mx, ay[j] * my);
                const float td = __builtin_fmaf(ax[j], dx, ay[j] * dy);
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
            const float2 a = p[e.len - 1];
#pragma unroll
            for (int j = 0; j < BPT; ++j) {
                const float t = __builtin_fmaf(ax[j], a.x, ay[j] * a.y);
                re[j] += __builtin_amdgcn_cosf(t);
                im[j] += __builtin_amdgcn_sinf(t);
            }
        }
    } else {
        // Large arguments: the phase is formed and wrapped to [-1/2, 1/2] revolutions in
        // double precision, from the double-float local coordinates.
        double ax[BPT], ay[BPT];
#pragma unroll
        for (int j = 0; j < BPT; ++j) {
            const int k = b0 + j * kEncodeThreads;
            double2 t = (k < halfp) ? rev_d[k] : make_double2(0.0, 0.0);
            ax[j] = t.x;
            ay[j] = t.y;
        }
        const float2* __restrict__ plo = sorted_lo + e.start;
        for (int q = 0; q < e.len; ++q) {
            const float2 a = p[q], al = plo[q];
            const double x = (double)a.x + (double)al.x, y = (double)a.y + (double)al.y;
#pragma unroll
            for (int j = 0; j < BPT; ++j) {
                const double t = __fma_rn(ax[j], x, ay[j] * y);
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

// omega[key][k] += sum over the key's work items.  Four groups of 64 threads per block of 64
// bins: group g sums the items g, g + 4, g + 8, ... in order, eight loads in flight, and the four
// group sums are added in a fixed order (deterministic).
__global__ __launch_bounds__(256) void k_reduce(const float2* __restrict__ partial,
                                                const int* __restrict__ meta, int nkeys, int half,
                                                int halfp, float2* __restrict__ omega) {
    __shared__ float2 sh[4][64];
    const int key = blockIdx.y;
    const int g = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int k = blockIdx.x * 64 + lane;
    const int e0 = meta[1 + key], ne = meta[1 + nkeys + key];
    if (ne == 0) return;   // uniform over the block
    float sr = 0.f, si = 0.f;
    if (k < half) {
        const float2* p = partial + (size_t)e0 * halfp + k;
        int c = g;
        for (; c + 28 < ne; c += 32) {
            float2 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = p[(size_t)(c + 4 * u) * halfp];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                sr += v[u].x;
                si += v[u].y;
            }
        }
        for (; c < ne; c += 4) {
            const float2 v = p[(size_t)c * halfp];
            sr += v.x;
            si += v.y;
        }
    }
    sh[g][lane] = make_float2(sr, si);
    __syncthreads();
    if (g == 0 && k < half) {
        const float2 a = sh[0][lane], b = sh[1][lane], c = sh[2][lane], d = sh[3][lane];
        float2* o = omega + (size_t)key * halfp + k;
        const float2 w = *o;
        *o = make_float2(w.x + ((a.x + b.x) + (c.x + d.x)), w.y + ((a.y + b.y) + (c.y + d.y)));
    }
}

// scale[key] = 1 / ||w|| with ||w||^2 = (2/D) sum_{k < D/2} |Omega_k|^2 (Parseval over the
// conjugate-symmetric spectrum; bins 0 and D/2 both equal the point count), 0 for an empty
// memory (eq. vector-normalization); omega_s[key] = conj(Omega[key]) * scale[key].
constexpr int kNormThreads = 1024;
__global__ __launch_bounds__(kNormThreads) void k_norm(const float2* __restrict__ omega, int half,
                                              int halfp, int D, float* __restrict__ scale,
                                              float2* __restrict__ omega_s,
                                              unsigned* __restrict__ hmax_u) {
    const int key = blockIdx.x;
    // the following similarity GEMM folds its class maxima into hmax_u[0..1]; they start from
    // zero here
    if (key == 0 && threadIdx.x < 2) hmax_u[threadIdx.x] = 0u;
    const float2* w = omega + (size_t)key * halfp;
    double s = 0.0;
    for (int k = threadIdx.x; k < half; k += kNormThreads) {
        double re = w[k].x, im = w[k].y;
        s += re * re + im * im;
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    __shared__ double sh[kNormThreads / 64];
    __shared__ float sh_inv;
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < kNormThreads / 64; ++i) t += sh[i];
        double nrm = sqrt(2.0 * t / (double)D);
        const float inv = (nrm > 0.0) ? (float)(1.0 / nrm) : 0.f;
        scale[key] = inv;
        sh_inv = inv;
    }
    __syncthreads();
    // conj(Omega) / ||w|| for the similarity GEMM (padding bins stay zero)
    const float inv = sh_inv;
    float2* o = omega_s + (size_t)key * halfp;
    for (int k = threadIdx.x; k < halfp; k += kNormThreads) o[k] = make_float2(w[k].x * inv, -w[k].y * inv);
}

// Paper-frame export: out[key][k] = exp(i*Theta[k].mu_beta) * Omega_local[key][k] for
// k < D/2, and out[key][D/2] = Omega_local[key][0] (the point count; Theta[D/2] = 0).
__global__ __launch_bounds__(256) void k_export(const float2* __restrict__ omega,
                                                const double* __restrict__ theta_rad,
                                                LayoutDev L, int half, int halfp,
                                                float* __restrict__ out) {
    const int key = blockIdx.y;
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k > half) return;
    const int beta = key >> 1;
    const double mx = L.cx[beta % L.tiles_x], my = L.cy[beta / L.tiles_x];
    const float2* w = omega + (size_t)key * halfp;
    float* o = out + ((size_t)key * (half + 1) + k) * 2;
    if (k == half) {
        o[0] = w[0].x;
        o[1] = w[0].y;
        return;
    }
    double ph = theta_rad[2 * k] * mx + theta_rad[2 * k + 1] * my;
    double s, c;
    sincos(ph, &s, &c);
    double re = w[k].x, im = w[k].y;
    o[0] = (float)(c * re - s * im);
    o[1] = (float)(s * re + c * im);
}

__global__ __launch_bounds__(256) void k_bump(unsigned* __restrict__ version, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) version[i] += 1u;
}

__global__ __launch_bounds__(256) void k_add(float2* __restrict__ dst,
                                             const float2* __restrict__ src, size_t n) {
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        float2 a = dst[i], b = src[i];
        dst[i] = make_float2(a.x + b.x, a.y + b.y);
    }
}

int bits_for(int v) {
    int b = 0;
    while ((1 << b) <= v) ++b;
    return b;
}

}  // namespace

EncodePlan encode_plan(int64_t n, int halfp, int nkeys) {
    EncodePlan p;
    p.nchunks = (int)((n + kAssignChunk - 1) / kAssignChunk);
    p.bpt = 1;
    while (p.bpt < kEncodeBpt && kEncodeThreads * p.bpt < halfp) p.bpt *= 2;
    p.binblocks = (halfp + kEncodeThreads * p.bpt - 1) / (kEncodeThreads * p.bpt);
    int64_t ec = (n * p.binblocks + 1023) / 1024;
    ec = ec < 64 ? 64 : (ec > kEncodeChunk ? kEncodeChunk : ec);
    ec += ec & 1;
    p.echunk = (int)ec;
    p.max_echunks = (int)((n + ec - 1) / ec) + nkeys;
    return p;
}

hipError_t launch_encode(const float* xy, const uint8_t* label, int64_t n, const LayoutDev& L,
                         int nkeys, const float2* theta_rev, const double* theta_rev_d,
                         float max_rev_x, float max_rev_y, int half, int halfp,
                         const EncodeWork& w, float2* omega, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const EncodePlan p = encode_plan(n, halfp, nkeys);
    const float2* xy2 = reinterpret_cast<const float2*>(xy);
    hipLaunchKernelGGL(k_assign, dim3(p.nchunks), dim3(kAssignChunk), nkeys * sizeof(int), s, xy2,
                       label, n, L, nkeys, p.nchunks, bits_for(nkeys), w.key, w.hist, w.n_bad);
    launch_key_scan(w.hist, p.nchunks, nkeys, p.echunk, w.table, w.meta, w.version, s);
    if (4 * nkeys * (int)sizeof(int) <= 65536)
        hipLaunchKernelGGL(k_scatter<4>, dim3(p.nchunks), dim3(256), 4 * nkeys * sizeof(int), s, xy2, w.key,
                           n, L, nkeys, p.nchunks, bits_for(nkeys), w.hist, w.sorted, w.sorted_lo);
    else
        hipLaunchKernelGGL(k_scatter<1>, dim3(p.nchunks), dim3(64), nkeys * sizeof(int), s, xy2, w.key,
                           n, L, nkeys, p.nchunks, bits_for(nkeys), w.hist, w.sorted, w.sorted_lo);
    const double2* rev_d = reinterpret_cast<const double2*>(theta_rev_d);
    const dim3 eg(p.max_echunks, p.binblocks);
    const hipEvent_t e0 = profile_start(kStageEncode), e1 = profile_stop(kStageEncode);
    static_assert(kEncodeBpt == 2, "instantiations below");
    if (p.bpt == 1)
        hipExtLaunchKernelGGL(k_encode<1>, eg, dim3(kEncodeThreads), 0, s, e0, e1, 0, w.sorted, w.sorted_lo, w.table,
                              w.meta, theta_rev, rev_d, max_rev_x, max_rev_y, halfp, w.partial);
    else
        hipExtLaunchKernelGGL(k_encode<2>, eg, dim3(kEncodeThreads), 0, s, e0, e1, 0, w.sorted, w.sorted_lo, w.table,
                              w.meta, theta_rev, rev_d, max_rev_x, max_rev_y, halfp, w.partial);
    launch_key_reduce(w.partial, w.meta, nkeys, half, halfp, omega, s);
    return hipGetLastError();
}

void launch_key_scan(int* hist, int nchunks, int nkeys, int echunk, EChunk* table, int* meta, unsigned* version,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), nkeys * sizeof(int), s, hist, nchunks, nkeys, echunk,
                       table, meta, version);
}

void launch_key_reduce(const float2* partial, const int* meta, int nkeys, int half, int halfp, float2* omega,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3((half + 63) / 64, nkeys), dim3(256), 0, s, partial, meta, nkeys, half,
                       halfp, omega);
}

hipError_t launch_norm(const float2* omega, int nkeys, int half, int halfp, int D, float* scale,
                       float2* omega_s, unsigned* hmax_u, hipStream_t s) {
    hipLaunchKernelGGL(k_norm, dim3(nkeys), dim3(kNormThreads), 0, s, omega, half, halfp, D, scale, omega_s,
                       hmax_u);
    return hipGetLastError();
}

hipError_t launch_memories_export(const float2* omega, const double* theta_rad, const LayoutDev& L,
                                  int nkeys, int half, int halfp, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_export, dim3((half + 1 + 255) / 256, nkeys), dim3(256), 0, s, omega,
                       theta_rad, L, half, halfp, out);
    return hipGetLastError();
}

hipError_t launch_bump_versions(unsigned* version, int nkeys, hipStream_t s) {
    hipLaunchKernelGGL(k_bump, dim3((nkeys + 255) / 256), dim3(256), 0, s, version, nkeys);
    return hipGetLastError();
}

hipError_t launch_add(float2* dst, const float2* src, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dst, src, n);
    return hipGetLastError();
}

}  // namespace vsaogm
