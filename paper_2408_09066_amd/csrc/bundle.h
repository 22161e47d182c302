// Device bodies of the encode pipeline (Sec. III-B, Algorithm 1) that maps and volumes share:
// the key histogram of the tile assignment, the stable counting-sort scatter of the tile-local
// coordinates, and the partial spectra of one work item.  The volume is the method with a third
// axis (the 3-D mapping named in Sec. V); only the geometry differs.
//
// The bodies are templated on
//   G  the geometry (PlaneGeom in encode.hip, VolumeGeom in volume.hip), which supplies
//        Src              a point as the caller stores it
//        Pt               tile-local coordinates in fp32; their rounding residuals have this type
//        Rev, RevD        a bin's rates Theta[k] / (2 pi), revolutions per unit length, fp32/fp64
//        Pair             a pair's mid-point and half-difference as kept in LDS
//        load(q, i)       point i
//        nearest(q, s)    its tile: exact argmin of the squared distance to the tile centres,
//                         lowest index on ties; -1 when there is none
//        local(q, beta, s, h, l)   s minus tile beta's centre in double precision, split into
//                         the fp32 value h and residual l
//        reach(p, m)      sum over the axes of |p| m: with m the largest |rate| per axis, a bound
//                         on p's phase over all bins
//        pair(a, b)       ((a + b) / 2, (a - b) / 2)
//        mid(r, pr), half(r, pr)   phase of the pair's mid-point / half-difference
//        phase(r, p)      phase of one point
//        wide(r, h, l)    phase in double precision from the double-float coordinates h + l
//        rev(q, k), rev_d(q, k), rev0(), rev_d0()   bin k's rates (k < halfp), zero rates
//        max_rev(q)       largest |rate| per axis over the bins
//   Q  the request: the encode's buffers under EncodeReq's member names (label, n, key, hist,
//      table, meta, sorted, sorted_lo, partial, omega, ...), plus what G reads.
#pragma once
#include "internal.h"

namespace vsaogm {

// One point per thread; blocks of kAssignChunk points.  hist is key-major:
// hist[key][chunk] = number of the chunk's points with that key.  The lanes of a wavefront
// holding one key add their count with one LDS atomic (a chunk's points share few keys).
template <class G, class Q>
__device__ inline void assign_points(const Q& q, int bid, int* sh_hist) {
    for (int k = threadIdx.x; k < q.nkeys; k += blockDim.x) sh_hist[k] = 0;
    __syncthreads();
    const int64_t i = (int64_t)bid * kAssignChunk + threadIdx.x;
    int key = -1;
    if (i < q.n) {
        const typename G::Src p = G::load(q, i);
        const unsigned l = as_global(q.label)[i];
        if (l <= 1u) {
            const int b = G::nearest(q, p);
            if (b >= 0) key = 2 * b + (int)l;
        }
        if (key < 0) atomicAdd(as_global_rw(q.n_bad), 1ull);
        as_global_rw(q.key)[i] = key;
    }
    const int lane = threadIdx.x & 63;
    const uint64_t same = same_value_lanes(key < 0 ? (unsigned)q.nkeys : (unsigned)key, q.key_bits);
    if (key >= 0 && (same & ((1ull << lane) - 1ull)) == 0) atomicAdd(&sh_hist[key], __popcll(same));
    __syncthreads();
    for (int k = threadIdx.x; k < q.nkeys; k += blockDim.x)
        as_global_rw(q.hist)[(size_t)k * q.nchunks + bid] = sh_hist[k];
}

// Stable counting-sort scatter: one block of WAVES wavefronts per chunk of kAssignChunk points,
// wave w taking the chunk's w-th part in order (four waves; one when the per-wave key tables
// would not fit the LDS of a workgroup).  The waves' key counts give each wave its own running
// base per key (the chunk's base plus the counts of the earlier parts); within a wave, a point's
// slot is its key's running base plus the number of earlier lanes of the same round with the
// same key (lanes are matched bit by bit with ballots).  The slot receives the point's
// tile-local coordinates and their rounding residuals.
template <int WAVES, class G, class Q>
__device__ inline void scatter_points(const Q& q, int bid, int* run /* LDS [WAVES][nkeys] */) {
    auto* __restrict__ key = as_global(q.key);
    const int64_t n = q.n;
    const int nkeys = q.nkeys, nchunks = q.nchunks, key_bits = q.key_bits;
    auto* __restrict__ base = as_global(q.hist);
    auto* __restrict__ sorted = as_global_rw(q.sorted);
    auto* __restrict__ sorted_lo = as_global_rw(q.sorted_lo);
    constexpr int QW = kAssignChunk / WAVES;          // points per wave
    constexpr int R = QW / 64;                        // rounds per wave
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t q0 = (int64_t)bid * kAssignChunk + (int64_t)wave * QW;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int kk[R];
    typename G::Src pp[R];
    uint64_t same[R];   // lanes of the round with this lane's key
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = q0 + r * 64 + lane;
        kk[r] = (i < n) ? key[i] : -1;
        pp[r] = G::src0();
        if (i < n) pp[r] = G::load(q, i);
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
        int acc = base[(size_t)k * nchunks + bid];
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
            typename G::Pt h, l;
            G::local(q, k >> 1, pp[r], h, l);
            sorted[dest] = h;
            sorted_lo[dest] = l;
            if ((same[r] & lt_mask) == 0) my[k] += __popcll(same[r]);
        }
        __syncthreads();
    }
}

// Partial spectrum of one work item (consecutive sorted points of one memory) for one block of
// bins: thread t owns bins b0 + t + j*kEncodeThreads, j < BPT; the points are read as
// wave-uniform loads.  Blocks are numbered work item fastest: block bid is work item
// bid % max_echunks of bin block bid / max_echunks.
//
// Consecutive points go in pairs,
//   exp(i a) + exp(i b) = 2 cos((a - b) / 2) exp(i (a + b) / 2),
// three hardware sine/cosine evaluations per two points (phases in revolutions), with each
// pair's mid-point and half-difference formed once in LDS for all bins.  A work item whose
// phases could exceed kWidePhaseRev forms and wraps every phase to [-1/2, 1/2] revolutions in
// double precision instead.
template <int BPT, class G, class Q>
__device__ inline void encode_points(const Q& q, int bid) {
    using Pt = typename G::Pt;
    using Rev = typename G::Rev;
    using RevD = typename G::RevD;
    using Pair = typename G::Pair;
    auto* __restrict__ sorted = as_global(q.sorted);
    auto* __restrict__ sorted_lo = as_global(q.sorted_lo);
    const Rev max_rev = G::max_rev(q);
    const int halfp = q.halfp;
    gmem_rw<float2>* __restrict__ partial = as_global_rw(q.partial);
    const int c = bid % q.max_echunks;
    if (c >= as_global(q.meta)[0]) return;
    const EChunk e = as_global(q.table)[c];
    // the only work item of its memory: its sums go straight into the memory (below)
    const bool alone = q.direct_single && as_global(q.meta)[1 + q.nkeys + e.key] == 1;
    const int b0 = (bid / q.max_echunks) * (kEncodeThreads * BPT) + threadIdx.x;
    auto* __restrict__ p = sorted + e.start;

    // Largest phase (revolutions) any bin can reach on this work item's points.
    __shared__ float sh_max[kEncodeThreads / 64];
    __shared__ Pair sh_pair[kEncodeChunk / 2];
    float bound = 0.f;
    for (int u = threadIdx.x; u < e.len; u += kEncodeThreads) bound = fmaxf(bound, G::reach(p[u], max_rev));
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
        Rev a[BPT];
#pragma unroll
        for (int j = 0; j < BPT; ++j) {
            const int k = b0 + j * kEncodeThreads;
            a[j] = G::rev0();
            if (k < halfp) a[j] = G::rev(q, k);
        }
        const int npairs = e.len >> 1;
        for (int u = threadIdx.x; u < npairs; u += kEncodeThreads) sh_pair[u] = G::pair(p[2 * u], p[2 * u + 1]);
        __syncthreads();
#pragma unroll 2
        for (int u = 0; u < npairs; ++u) {
            const Pair pr = sh_pair[u];
#pragma unroll
            for (int j = 0; j < BPT; ++j) {
                const float tm = G::mid(a[j], pr);
                const float td = G::half(a[j], pr);
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
            const Pt pl = p[e.len - 1];
#pragma unroll
            for (int j = 0; j < BPT; ++j) {
                const float t = G::phase(a[j], pl);
                re[j] += __builtin_amdgcn_cosf(t);
                im[j] += __builtin_amdgcn_sinf(t);
            }
        }
    } else {
        RevD a[BPT];
#pragma unroll
        for (int j = 0; j < BPT; ++j) {
            const int k = b0 + j * kEncodeThreads;
            a[j] = G::rev_d0();
            if (k < halfp) a[j] = G::rev_d(q, k);
        }
        auto* __restrict__ plo = sorted_lo + e.start;
        for (int u = 0; u < e.len; ++u) {
            const Pt h = p[u], l = plo[u];
#pragma unroll
            for (int j = 0; j < BPT; ++j) {
                const double t = G::wide(a[j], h, l);
                const float r = (float)(t - rint(t));
                re[j] += __builtin_amdgcn_cosf(r);
                im[j] += __builtin_amdgcn_sinf(r);
            }
        }
    }
    if (alone) {
        // what the reduction would add for one work item: w + (0 + s), bins below half only
        gmem_rw<float2>* __restrict__ w = as_global_rw(q.omega) + (size_t)e.key * halfp;
#pragma unroll
        for (int j = 0; j < BPT; ++j) {
            const int k = b0 + j * kEncodeThreads;
            if (k < q.half) {
                const float2 o = w[k];
                w[k] = make_float2(o.x + (0.f + re[j]), o.y + (0.f + im[j]));
            }
        }
        return;
    }
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
        const int k = b0 + j * kEncodeThreads;
        if (k < halfp) partial[(size_t)c * halfp + k] = make_float2(re[j], im[j]);
    }
}

}  // namespace vsaogm
