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
// Pipeline (all on the stream, no host synchronisation; the bodies of k_assign, k_scatter and
// k_encode are bundle.h's, shared with volumes, on PlaneGeom):
//   k_assign   nearest tile (exact double-precision argmin, lowest index on ties), key,
//              label check, per-chunk key histogram
//   k_scan     per-key totals and exclusive bases, encode work table
//   k_scatter  stable counting sort of the local coordinates by key (four wavefronts per chunk)
//   k_encode   per (work item, block of bins): sum of exp(2*pi*i*t) with t in revolutions,
//              hardware v_sin/v_cos, two points per step:
//                exp(i a) + exp(i b) = 2 cos((a-b)/2) exp(i (a+b)/2)
//   k_reduce   fixed-order sum of the work items' partial spectra into the memories
#include "bundle.h"

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
        double dy = __dsub_rn(y, as_global(L.cy)[j]);
        double dy2 = __dmul_rn(dy, dy);
        for (int i = i0; i <= i1; ++i) {
            double dx = __dsub_rn(x, as_global(L.cx)[i]);
            double d2 = __dadd_rn(__dmul_rn(dx, dx), dy2);
            if (d2 < bd) {
                bd = d2;
                best = j * L.tiles_x + i;
            }
        }
    }
    return best;
}

// The plane: points (x, y), tiles numbered beta = ty * tiles_x + tx, pairs kept in LDS as
// (mid-point x, y, half-difference x, y).
struct PlaneGeom {
    using Src = float2;
    using Pt = float2;
    using Rev = float2;
    using RevD = double2;
    using Pair = float4;
    __device__ static float2 src0() { return make_float2(0.f, 0.f); }
    __device__ static float2 load(const EncodeReq& q, int64_t i) { return as_global(q.xy)[i]; }
    __device__ static int nearest(const EncodeReq& q, float2 p) { return nearest_tile((double)p.x, (double)p.y, q.L); }
    __device__ static void local(const EncodeReq& q, int beta, float2 s, float2& h, float2& l) {
        const int tx = beta % q.L.tiles_x, ty = beta / q.L.tiles_x;
        const double lx = (double)s.x - as_global(q.L.cx)[tx];
        const double ly = (double)s.y - as_global(q.L.cy)[ty];
        const float fx = (float)lx, fy = (float)ly;
        h = make_float2(fx, fy);
        l = make_float2((float)(lx - (double)fx), (float)(ly - (double)fy));
    }
    __device__ static float reach(float2 v, float2 m) { return fabsf(v.x) * m.x + fabsf(v.y) * m.y; }
    __device__ static float4 pair(float2 a, float2 b) {
        return make_float4(0.5f * (a.x + b.x), 0.5f * (a.y + b.y), 0.5f * (a.x - b.x), 0.5f * (a.y - b.y));
    }
    __device__ static float mid(float2 r, float4 pr) { return __builtin_fmaf(r.x, pr.x, r.y * pr.y); }
    __device__ static float half(float2 r, float4 pr) { return __builtin_fmaf(r.x, pr.z, r.y * pr.w); }
    __device__ static float phase(float2 r, float2 p) { return __builtin_fmaf(r.x, p.x, r.y * p.y); }
    __device__ static double wide(double2 r, float2 h, float2 l) {
        const double x = (double)h.x + (double)l.x, y = (double)h.y + (double)l.y;
        return __fma_rn(r.x, x, r.y * y);
    }
    __device__ static float2 rev0() { return make_float2(0.f, 0.f); }
    __device__ static float2 rev(const EncodeReq& q, int k) { return as_global(q.rev)[k]; }
    __device__ static double2 rev_d0() { return make_double2(0.0, 0.0); }
    __device__ static double2 rev_d(const EncodeReq& q, int k) { return as_global(q.rev_d)[k]; }
    __device__ static float2 max_rev(const EncodeReq& q) { return make_float2(q.max_rev_x, q.max_rev_y); }
};

__global__ __launch_bounds__(kAssignChunk) void k_assign(EncodeReq q) {
    extern __shared__ int sh_hist[];
    assign_points<PlaneGeom>(q, blockIdx.x, sh_hist);
}
__global__ __launch_bounds__(kAssignChunk) void k_assign_b(const EncodeReq* __restrict__ qs, const int* __restrict__ b0,
                                                           int nq) {
    extern __shared__ int sh_hist[];
    const int r = batch_job(b0, nq, blockIdx.x);
    assign_points<PlaneGeom>(qs[r], blockIdx.x - b0[r], sh_hist);
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
__device__ inline void scan_body(const EncodeReq& q, int* key_start /* LDS [nkeys] */) {
    __shared__ int sh_w[kScanThreads / 64];
    gmem_rw<int>* __restrict__ hist = as_global_rw(q.hist);
    const int nchunks = q.nchunks, nkeys = q.nkeys, echunk = q.echunk;
    gmem_rw<EChunk>* __restrict__ table = as_global_rw(q.table);
    gmem_rw<int>* __restrict__ meta = as_global_rw(q.meta);
    gmem_rw<unsigned>* __restrict__ version = q.version ? as_global_rw(q.version) : nullptr;
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
__global__ __launch_bounds__(kScanThreads) void k_scan(EncodeReq q) {
    extern __shared__ int key_start[];
    scan_body(q, key_start);
}
__global__ __launch_bounds__(kScanThreads) void k_scan_b(const EncodeReq* __restrict__ qs, const int* __restrict__ b0,
                                                         int nq) {
    extern __shared__ int key_start[];
    scan_body(qs[batch_job(b0, nq, blockIdx.x)], key_start);
}

template <int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_scatter(EncodeReq q) {
    extern __shared__ int run[];
    scatter_points<WAVES, PlaneGeom>(q, blockIdx.x, run);
}
template <int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_scatter_b(const EncodeReq* __restrict__ qs,
                                                          const int* __restrict__ b0, int nq) {
    extern __shared__ int run[];
    const int r = batch_job(b0, nq, blockIdx.x);
    scatter_points<WAVES, PlaneGeom>(qs[r], blockIdx.x - b0[r], run);
}

template <int BPT>
__global__ __launch_bounds__(kEncodeThreads) void k_encode(EncodeReq q) {
    encode_points<BPT, PlaneGeom>(q, blockIdx.x);
}
template <int BPT>
__global__ __launch_bounds__(kEncodeThreads) void k_encode_b(const EncodeReq* __restrict__ qs,
                                                             const int* __restrict__ b0, int nq) {
    const int r = batch_job(b0, nq, blockIdx.x);
    encode_points<BPT, PlaneGeom>(qs[r], blockIdx.x - b0[r]);
}

// omega[key][k] += sum over the key's work items.  Four groups of 64 threads per block of 64
// bins: group g sums the items g, g + 4, g + 8, ... in order, eight loads in flight, and the four
// group sums are added in a fixed order (deterministic).
// Blocks are numbered bin block fastest: block bid is bins 64 * (bid % ceil(half / 64)) .. of key
// bid / ceil(half / 64).
__device__ inline void reduce_body(const EncodeReq& q, int bid) {
    gmem<float2>* __restrict__ partial = as_global(q.partial);
    gmem<int>* __restrict__ meta = as_global(q.meta);
    const int nkeys = q.nkeys, half = q.half, halfp = q.halfp;
    gmem_rw<float2>* __restrict__ omega = as_global_rw(q.omega);
    __shared__ float2 sh[4][64];
    const int bblocks = (half + 63) / 64;
    const int key = bid / bblocks;
    const int g = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int k = (bid % bblocks) * 64 + lane;
    const int e0 = meta[1 + key], ne = meta[1 + nkeys + key];
    if (ne == 0 || (ne == 1 && q.direct_single)) return;   // uniform over the block (one work item: the encode added it)
    float sr = 0.f, si = 0.f;
    if (k < half) {
        gmem<float2>* p = partial + (size_t)e0 * halfp + k;
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
        gmem_rw<float2>* o = omega + (size_t)key * halfp + k;
        const float2 w = *o;
        *o = make_float2(w.x + ((a.x + b.x) + (c.x + d.x)), w.y + ((a.y + b.y) + (c.y + d.y)));
    }
}
__global__ __launch_bounds__(256) void k_reduce(EncodeReq q) { reduce_body(q, blockIdx.x); }
__global__ __launch_bounds__(256) void k_reduce_b(const EncodeReq* __restrict__ qs, const int* __restrict__ b0,
                                                  int nq) {
    const int r = batch_job(b0, nq, blockIdx.x);
    reduce_body(qs[r], blockIdx.x - b0[r]);
}

// scale[key] = 1 / ||w|| with ||w||^2 = (2/D) sum_{k < D/2} |Omega_k|^2 (Parseval over the
// conjugate-symmetric spectrum; bins 0 and D/2 both equal the point count), 0 for an empty
// memory (eq. vector-normalization); omega_s[key] = conj(Omega[key]) * scale[key].
constexpr int kNormThreads = 1024;
__device__ inline void norm_body(const EncodeReq& q, int key) {
    gmem<float2>* __restrict__ omega = as_global(q.omega);
    const int half = q.half, halfp = q.halfp, D = q.D;
    gmem_rw<float>* __restrict__ scale = as_global_rw(q.scale);
    gmem_rw<float2>* __restrict__ omega_s = as_global_rw(q.omega_s);
    gmem_rw<unsigned>* __restrict__ hmax_u = as_global_rw(q.hmax_u);
    // the following similarity GEMM folds its class maxima into hmax_u[0..1]; they start from
    // zero here
    if (key == 0 && threadIdx.x < 2) hmax_u[threadIdx.x] = 0u;
    gmem<float2>* w = omega + (size_t)key * halfp;
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
    gmem_rw<float2>* o = omega_s + (size_t)key * halfp;
    for (int k = threadIdx.x; k < halfp; k += kNormThreads) o[k] = make_float2(w[k].x * inv, -w[k].y * inv);
}
__global__ __launch_bounds__(kNormThreads) void k_norm(EncodeReq q) { norm_body(q, blockIdx.x); }
__global__ __launch_bounds__(kNormThreads) void k_norm_b(const EncodeReq* __restrict__ qs, const int* __restrict__ b0,
                                                         int nq) {
    const int r = batch_job(b0, nq, blockIdx.x);
    norm_body(qs[r], blockIdx.x - b0[r]);
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

// Algorithm 3 over several agents in one pass: dst[i] += src[0][i], then src[1][i], ... in
// source order, the additions (and so the rounding) of that many pairwise k_add launches.
struct FuseSources {
    const float2* p[kFuseSources];
};
__global__ __launch_bounds__(256) void k_add_many(float2* __restrict__ dst, FuseSources src, int nsrc, size_t n) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float2 a = dst[i];
    for (int j = 0; j < nsrc; ++j) {
        const float2 b = as_global(src.p[j])[i];
        a = make_float2(a.x + b.x, a.y + b.y);
    }
    dst[i] = a;
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

// The request of one map's encode chain (everything but the spectra-side fields of a norm).
EncodeReq encode_req(const float* xy, const uint8_t* label, int64_t n, const LayoutDev& L, int nkeys,
                     const float2* theta_rev, const double* theta_rev_d, float max_rev_x, float max_rev_y,
                     int half, int halfp, const EncodeWork& w, float2* omega) {
    const EncodePlan p = encode_plan(n, halfp, nkeys);
    EncodeReq q{};
    q.xy = reinterpret_cast<const float2*>(xy);
    q.label = label;
    q.n = n;
    q.L = L;
    q.nkeys = nkeys;
    q.key_bits = bits_for(nkeys);
    q.nchunks = p.nchunks;
    q.echunk = p.echunk;
    q.max_echunks = p.max_echunks;
    q.binblocks = p.binblocks;
    q.bpt = p.bpt;
    q.key = w.key;
    q.hist = w.hist;
    q.table = w.table;
    q.meta = w.meta;
    q.sorted = w.sorted;
    q.sorted_lo = w.sorted_lo;
    q.partial = w.partial;
    q.n_bad = w.n_bad;
    q.version = w.version;
    q.rev = theta_rev;
    q.rev_d = reinterpret_cast<const double2*>(theta_rev_d);
    q.max_rev_x = max_rev_x;
    q.max_rev_y = max_rev_y;
    q.half = half;
    q.halfp = halfp;
    q.direct_single = 1;
    q.omega = omega;
    return q;
}

hipError_t launch_encode(const float* xy, const uint8_t* label, int64_t n, const LayoutDev& L,
                         int nkeys, const float2* theta_rev, const double* theta_rev_d,
                         float max_rev_x, float max_rev_y, int half, int halfp,
                         const EncodeWork& w, float2* omega, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const EncodeReq q = encode_req(xy, label, n, L, nkeys, theta_rev, theta_rev_d, max_rev_x, max_rev_y, half,
                                   halfp, w, omega);
    hipLaunchKernelGGL(k_assign, dim3(q.nchunks), dim3(kAssignChunk), nkeys * sizeof(int), s, q);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), nkeys * sizeof(int), s, q);
    if (4 * nkeys * (int)sizeof(int) <= 65536)
        hipLaunchKernelGGL(k_scatter<4>, dim3(q.nchunks), dim3(256), 4 * nkeys * sizeof(int), s, q);
    else
        hipLaunchKernelGGL(k_scatter<1>, dim3(q.nchunks), dim3(64), nkeys * sizeof(int), s, q);
    const dim3 eg((unsigned)q.max_echunks * q.binblocks);
    const hipEvent_t e0 = profile_start(kStageEncode), e1 = profile_stop(kStageEncode);
    static_assert(kEncodeBpt == 2, "instantiations below");
    if (q.bpt == 1)
        hipExtLaunchKernelGGL(k_encode<1>, eg, dim3(kEncodeThreads), 0, s, e0, e1, 0, q);
    else
        hipExtLaunchKernelGGL(k_encode<2>, eg, dim3(kEncodeThreads), 0, s, e0, e1, 0, q);
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)((half + 63) / 64 * nkeys)), dim3(256), 0, s, q);
    return hipGetLastError();
}

void launch_key_scan(int* hist, int nchunks, int nkeys, int echunk, EChunk* table, int* meta, unsigned* version,
                     hipStream_t s) {
    EncodeReq q{};
    q.hist = hist;
    q.nchunks = nchunks;
    q.nkeys = nkeys;
    q.echunk = echunk;
    q.table = table;
    q.meta = meta;
    q.version = version;
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), nkeys * sizeof(int), s, q);
}

void launch_key_reduce(const float2* partial, const int* meta, int nkeys, int half, int halfp, int direct_single,
                       float2* omega, hipStream_t s) {
    EncodeReq q{};
    q.direct_single = direct_single;
    q.partial = const_cast<float2*>(partial);
    q.meta = const_cast<int*>(meta);
    q.nkeys = nkeys;
    q.half = half;
    q.halfp = halfp;
    q.omega = omega;
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)((half + 63) / 64 * nkeys)), dim3(256), 0, s, q);
}

hipError_t launch_norm(const float2* omega, int nkeys, int half, int halfp, int D, float* scale,
                       float2* omega_s, unsigned* hmax_u, hipStream_t s) {
    EncodeReq q{};
    q.omega = const_cast<float2*>(omega);
    q.half = half;
    q.halfp = halfp;
    q.D = D;
    q.scale = scale;
    q.omega_s = omega_s;
    q.hmax_u = hmax_u;
    hipLaunchKernelGGL(k_norm, dim3(nkeys), dim3(kNormThreads), 0, s, q);
    return hipGetLastError();
}

hipError_t launch_encode_batch(const EncodeBatch& b, hipStream_t s) {
    const int nq = b.nreq;
    auto b0 = [&](int stage) { return b.block0 + (size_t)stage * (nq + 1); };
    if (b.blocks[0] > 0) {
        hipLaunchKernelGGL(k_assign_b, dim3(b.blocks[0]), dim3(kAssignChunk), b.max_keys * sizeof(int), s, b.reqs,
                           b0(0), nq);
        hipLaunchKernelGGL(k_scan_b, dim3(b.blocks[1]), dim3(kScanThreads), b.max_keys * sizeof(int), s, b.reqs,
                           b0(1), nq);
        if (4 * b.max_keys * (int)sizeof(int) <= 65536)
            hipLaunchKernelGGL(k_scatter_b<4>, dim3(b.blocks[2]), dim3(256), 4 * b.max_keys * sizeof(int), s, b.reqs,
                               b0(2), nq);
        else
            hipLaunchKernelGGL(k_scatter_b<1>, dim3(b.blocks[2]), dim3(64), b.max_keys * sizeof(int), s, b.reqs,
                               b0(2), nq);
        const hipEvent_t e0 = profile_start(kStageEncode), e1 = profile_stop(kStageEncode);
        if (b.bpt == 1)
            hipExtLaunchKernelGGL(k_encode_b<1>, dim3(b.blocks[3]), dim3(kEncodeThreads), 0, s, e0, e1, 0, b.reqs,
                                  b0(3), nq);
        else
            hipExtLaunchKernelGGL(k_encode_b<2>, dim3(b.blocks[3]), dim3(kEncodeThreads), 0, s, e0, e1, 0, b.reqs,
                                  b0(3), nq);
        hipLaunchKernelGGL(k_reduce_b, dim3(b.blocks[4]), dim3(256), 0, s, b.reqs, b0(4), nq);
    }
    if (b.blocks[5] > 0) hipLaunchKernelGGL(k_norm_b, dim3(b.blocks[5]), dim3(kNormThreads), 0, s, b.reqs, b0(5), nq);
    return hipGetLastError();
}

void encode_batch_blocks(const EncodeReq& q, int out[kEncodeStages]) {
    const bool enc = q.n > 0;
    out[0] = enc ? q.nchunks : 0;
    out[1] = enc ? 1 : 0;
    out[2] = enc ? q.nchunks : 0;
    out[3] = enc ? q.max_echunks * q.binblocks : 0;
    out[4] = enc ? (q.half + 63) / 64 * q.nkeys : 0;
    out[5] = q.nkeys;
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

hipError_t launch_add_many(float2* dst, const float2* const* srcs, int nsrc, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    for (int j0 = 0; j0 < nsrc; j0 += kFuseSources) {   // chunks in source order
        FuseSources f{};
        const int m = std::min(kFuseSources, nsrc - j0);
        for (int j = 0; j < m; ++j) f.p[j] = srcs[j0 + j];
        hipLaunchKernelGGL(k_add_many, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dst, f, m, n);
    }
    return hipGetLastError();
}

hipError_t launch_add(float2* dst, const float2* src, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dst, src, n);
    return hipGetLastError();
}

}  // namespace vsaogm
