// Decoding: similarity of every grid cell with the normalised memories of its tile
// (Sec. III-B eqs. vector-normalization and loc-query) on gfx950 matrix cores.
//
// The location vector of cell c = (x, y) has the spectrum exp(i*Theta[k].c), which factors
// per axis: exp(i*Theta_x[k]*x) * exp(i*Theta_y[k]*y).  In tile-local coordinates, and
// using the conjugate symmetry of the spectra, the similarity of cell (row y, column x)
// of tile beta with memory key = 2*beta+psi is
//   P[psi][y][x] = scale[key] * sum_{k < D/2} Re( conj(Omega[key][k]) Ex[x][k] Ey[y][k] )
// with scale = 2 / (D ||w||).  Written over real and imaginary parts this is a real
// contraction of length D:
//   L[y][2k] = Re Ey[y][k],           L[y][2k+1] = Im Ey[y][k]
//   R[x][2k] = Re(conj(Om) Ex[x][k]), R[x][2k+1] = -Im(conj(Om) Ex[x][k])
//   P = scale * L . R^T
// so every tile is a dense GEMM (rows x columns x D) run on MFMA.  The per-axis tables Ex,
// Ey (the paper's precomputed location vectors, factored) are built once per grid in double
// precision; the memory factor conj(Omega) is applied to R while it is staged into LDS.
// The GEMM epilogue applies the scale, stores the heatmap and folds each class's maximum
// into an order-preserving unsigned atomic (the maximum of eq. non-linearities).
#include "internal.h"

namespace vsaogm {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

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

// Monotone map float -> unsigned so that unsigned max = float max.
__device__ inline unsigned order_key(float f) {
    unsigned u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float order_value(unsigned u) {
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

__global__ void k_hmax_init(unsigned* hmax_u) {
    if (threadIdx.x < 2) hmax_u[threadIdx.x] = 0u;
}
__global__ void k_hmax_final(const unsigned* hmax_u, float* hmax) {
    if (threadIdx.x < 2) hmax[threadIdx.x] = order_value(hmax_u[threadIdx.x]);
}

constexpr int TM = 64, TN = 64;   // cells per block (rows x columns)
constexpr int KB = 16;            // complex bins per K step (32 reals)
constexpr int LDA = 2 * KB + 4;   // padded LDS row (floats)

// FP32 operands, MFMA v_mfma_f32_16x16x4_f32.  256 threads = 4 waves in a 2 x 2 layout,
// each wave a 32 x 32 block of both classes.  Within a K step lane group g = lane/16 owns
// reals 8g..8g+7 and feeds them to eight MFMAs (the order of a sum is immaterial).
__global__ __launch_bounds__(256) void k_decode_f32(const DTile* __restrict__ tiles,
                                                    const float2* __restrict__ ex,
                                                    const float2* __restrict__ ey,
                                                    const float2* __restrict__ omega,
                                                    const float* __restrict__ scale, int halfp,
                                                    int nx, int ny, float* __restrict__ heat,
                                                    unsigned* __restrict__ hmax_u) {
    __shared__ float As[TM * LDA];
    __shared__ float Bs[2 * TN * LDA];
    const DTile t = tiles[blockIdx.x];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int g = lane >> 4, i16 = lane & 15;

    // staging assignment: two float4 (= 2 complex bins each) of L and of Ex per thread
    int lrow[2], lpart[2];
    const float2* ey_p[2];
    const float2* ex_p[2];
    const float2* om_p[2][2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int idx = tid + 256 * s;
        lrow[s] = idx >> 3;
        lpart[s] = idx & 7;
        const int gr = min(t.r0 + lrow[s], t.rend - 1);
        const int gc = min(t.c0 + lrow[s], t.cend - 1);
        ey_p[s] = ey + (size_t)gr * halfp + 2 * lpart[s];
        ex_p[s] = ex + (size_t)gc * halfp + 2 * lpart[s];
        om_p[s][0] = omega + (size_t)(2 * t.beta) * halfp + 2 * lpart[s];
        om_p[s][1] = omega + (size_t)(2 * t.beta + 1) * halfp + 2 * lpart[s];
    }

    float4 rl[2], rx[2], ro[2][2];
    auto gload = [&](int kb) {
        const int off = kb * KB;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            rl[s] = *reinterpret_cast<const float4*>(ey_p[s] + off);
            rx[s] = *reinterpret_cast<const float4*>(ex_p[s] + off);
            ro[s][0] = *reinterpret_cast<const float4*>(om_p[s][0] + off);
            ro[s][1] = *reinterpret_cast<const float4*>(om_p[s][1] + off);
        }
    };

    v4f acc[2][2][2];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[p][a][b] = v4f{0.f, 0.f, 0.f, 0.f};

    const int nk = halfp / KB;
    gload(0);
    for (int kb = 0; kb < nk; ++kb) {
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            *reinterpret_cast<float4*>(&As[lrow[s] * LDA + 4 * lpart[s]]) = rl[s];
            const float4 e = rx[s];
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                const float4 o = ro[s][p];
                float4 r;
                r.x = o.x * e.x + o.y * e.y;
                r.y = o.y * e.x - o.x * e.y;
                r.z = o.z * e.z + o.w * e.w;
                r.w = o.w * e.z - o.z * e.w;
                *reinterpret_cast<float4*>(&Bs[(p * TN + lrow[s]) * LDA + 4 * lpart[s]]) = r;
            }
        }
        __syncthreads();
        if (kb + 1 < nk) gload(kb + 1);

        float a[2][8], b[2][2][8];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            const float* src = &As[(wm * 32 + rb * 16 + i16) * LDA + 8 * g];
            const float4 u = *reinterpret_cast<const float4*>(src);
            const float4 v = *reinterpret_cast<const float4*>(src + 4);
            a[rb][0] = u.x; a[rb][1] = u.y; a[rb][2] = u.z; a[rb][3] = u.w;
            a[rb][4] = v.x; a[rb][5] = v.y; a[rb][6] = v.z; a[rb][7] = v.w;
        }
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                const float* src = &Bs[(p * TN + wn * 32 + cb * 16 + i16) * LDA + 8 * g];
                const float4 u = *reinterpret_cast<const float4*>(src);
                const float4 v = *reinterpret_cast<const float4*>(src + 4);
                b[p][cb][0] = u.x; b[p][cb][1] = u.y; b[p][cb][2] = u.z; b[p][cb][3] = u.w;
                b[p][cb][4] = v.x; b[p][cb][5] = v.y; b[p][cb][6] = v.z; b[p][cb][7] = v.w;
            }
#pragma unroll
        for (int s = 0; s < 8; ++s)
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb)
                        acc[p][rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                            a[rb][s], b[p][cb][s], acc[p][rb][cb], 0, 0, 0);
    }

    // epilogue: scale, store, per-class maximum
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const float sc = scale[2 * t.beta + p];
        float mx = -INFINITY;
        float* out = heat + (size_t)p * nx * ny;
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int row = t.r0 + wm * 32 + rb * 16 + 4 * g + j;
                    const int col = t.c0 + wn * 32 + cb * 16 + i16;
                    if (row < t.rend && col < t.cend) {
                        const float v = acc[p][rb][cb][j] * sc;
                        out[(size_t)row * nx + col] = v;
                        mx = fmaxf(mx, v);
                    }
                }
        for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
        if (lane == 0 && mx > -INFINITY) atomicMax(hmax_u + p, order_key(mx));
    }
}

}  // namespace

hipError_t launch_table_f32(const double* theta_rad, int axis, const double* local, int ncells,
                            int half, int halfp, float2* tab, hipStream_t s) {
    hipLaunchKernelGGL(k_table_f32, dim3((halfp + 255) / 256, ncells), dim3(256), 0, s, theta_rad,
                       axis, local, half, halfp, tab);
    return hipGetLastError();
}

hipError_t launch_decode(int precision, const DTile* tiles, int ntiles, const void* ex_hi,
                         const void* ex_lo, const void* ey_hi, const void* ey_lo,
                         const float2* omega, const float* scale, int halfp, int nx, int ny,
                         float* heat, unsigned* hmax_u, float* hmax, hipStream_t s) {
    (void)ex_lo;
    (void)ey_lo;
    if (precision != 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_hmax_init, dim3(1), dim3(64), 0, s, hmax_u);
    profile_begin(kStageDecode, s);
    hipLaunchKernelGGL(k_decode_f32, dim3(ntiles), dim3(256), 0, s, tiles,
                       static_cast<const float2*>(ex_hi), static_cast<const float2*>(ey_hi),
                       omega, scale, halfp, nx, ny, heat, hmax_u);
    profile_end(kStageDecode, s);
    hipLaunchKernelGGL(k_hmax_final, dim3(1), dim3(64), 0, s, hmax_u, hmax);
    return hipGetLastError();
}

}  // namespace vsaogm
