// Sparse coding (step 1 of the DL iteration, Alg. 1): OMP with fixed
// sparsity s, computed Batch-OMP style from G = D D^T and A0 = Y D^T, one
// wavefront per signal.
//
// Per signal the wave keeps the correlations alpha = D^T r of its current
// residual in registers (n/64 per lane).  Each step:
//   1. j = argmax over unselected atoms of |alpha_j| (ties: lowest index);
//   2. the new Cholesky row of G_II: w_t = u_t[j] (t < k) and
//      delta^2 = G_jj - |w|^2; pivots below `pivot_fp64` are recomputed in
//      FP64 from the G entries (forward substitution with L);
//   3. u_k = (G[j,:] - sum_t w_t u_t) / delta, which equals D^T q_k for the
//      orthonormalised new direction q_k;
//   4. c_k = alpha_j / delta (the coefficient of y on q_k) and
//      alpha -= c_k u_k (the residual loses its q_k component).
// After the last step the coefficients solve L^T x = c (L is the Cholesky
// factor of G_II, since D_I = Q L^T).  This is the same arithmetic as
// Batch-OMP's alpha = A0 - G_I (G_II^{-1} A0_I) rearranged so that every
// step costs one pass over n values instead of a triangular solve.
//
// The u_t rows live in registers (SMAX x NPL per lane); the wave's Cholesky
// factor, support and coefficients live in LDS.
#include "dl_internal.h"

namespace dlk {
namespace {

__device__ inline float readlane_f(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// NPL values per lane held as one vector value, so that picking element c
// (uniform across the wave) stays in registers.
template <int NPL>
struct VecT {
    typedef float type __attribute__((ext_vector_type(NPL)));
};
template <>
struct VecT<1> {
    typedef float type;
};

template <int NPL>
__device__ inline float pick(const typename VecT<NPL>::type &v, int c)
{
    if constexpr (NPL == 1)
        return v;
    else
        return v[c];
}

template <int NPL>
__device__ inline void put(typename VecT<NPL>::type &v, int c, float x)
{
    if constexpr (NPL == 1)
        v = x;
    else
        v[c] = x;
}

__device__ inline float wave_sum(float v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_xor(v, off);
    return v;
}

constexpr int kWaves = 4;  // signals (waves) per workgroup

// Order this wave's LDS stores before its later LDS loads from other lanes.
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int NPL, int SMAX>
__global__ __launch_bounds__(256) void omp_kernel(OmpArgs a)
{
    __shared__ float sL[kWaves][SMAX * SMAX];
    __shared__ float sC[kWaves][SMAX];
    __shared__ float sX[kWaves][SMAX];
    __shared__ int sI[kWaves][SMAX];
    __shared__ float sG[kWaves][SMAX];
    __shared__ double sW[kWaves][SMAX];
    __shared__ double sD2[kWaves];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int i = blockIdx.x * kWaves + wave;
    if (i >= a.m)
        return;  // no workgroup barrier follows: waves are independent
    const int n = a.n, p = a.p, s = a.s;
    float *L = sL[wave];

    // signal norm (for the orthogonality stop rule) and the residual epilogue
    constexpr int PR = 4;  // p <= 256: at most 4 coordinates per lane
    float yv[PR];
    float ysq = 0.f;
#pragma unroll
    for (int r = 0; r < PR; ++r) {
        const int q = lane + 64 * r;
        yv[r] = q < p ? a.Y[(size_t)i * p + q] : 0.f;
        ysq += yv[r] * yv[r];
    }
    const float ynorm = sqrtf(wave_sum(ysq));

    typedef typename VecT<NPL>::type vec;
    vec alpha;
    vec u[SMAX];
    unsigned selmask = 0;
#pragma unroll
    for (int c = 0; c < NPL; ++c) {
        const int atom = c * 64 + lane;
        put<NPL>(alpha, c, atom < n ? a.A0[(size_t)i * n + atom] : 0.f);
    }
    if (!isfinite(ynorm) && lane == 0)
        atomicAdd(&a.ctl->nonfinite, 1ull);

    int k = 0;
    for (; k < s; ++k) {
        // 1. masked argmax, lowest index on ties
        float best = -1.f;
        int bidx = 0x7fffffff;
#pragma unroll
        for (int c = 0; c < NPL; ++c) {
            const int atom = c * 64 + lane;
            const float v = fabsf(pick<NPL>(alpha, c));
            if (atom < n && !((selmask >> c) & 1u) && v > best) {
                best = v;
                bidx = atom;
            }
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const float ov = __shfl_xor(best, off);
            const int oi = __shfl_xor(bidx, off);
            if (ov > best || (ov == best && oi < bidx)) {
                best = ov;
                bidx = oi;
            }
        }
        best = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(best)));
        const int j = __builtin_amdgcn_readfirstlane(bidx);
        if (!(best > a.tol_corr * ynorm) || j >= n)
            break;
        const int cj = j >> 6, lj = j & 63;

        // 2. Cholesky row of G_II for the new atom
        vec g;
#pragma unroll
        for (int c = 0; c < NPL; ++c) {
            const int atom = c * 64 + lane;
            put<NPL>(g, c, atom < n ? a.G[(size_t)j * n + atom] : 0.f);
        }
        const float gjj = readlane_f(pick<NPL>(g, cj), lj);
        float w[SMAX];
        float d2 = gjj;
#pragma unroll
        for (int t = 0; t < SMAX; ++t) {
            w[t] = 0.f;
            if (t < k) {
                w[t] = readlane_f(pick<NPL>(u[t], cj), lj);
                d2 -= w[t] * w[t];
            }
        }
        if (d2 < a.pivot_fp64) {
            // recompute w = L^{-1} G[I, j] and the pivot in FP64 (rare path:
            // lane t fetches G[j][I_t], lane 0 does the substitution)
            if (lane < k)
                sG[wave][lane] = a.G[(size_t)j * n + sI[wave][lane]];
            wave_lds_sync();
            if (lane == 0) {
                double d2_64 = (double)gjj;
                for (int t = 0; t < k; ++t) {
                    double acc = (double)sG[wave][t];
                    for (int r = 0; r < t; ++r)
                        acc -= (double)L[t * SMAX + r] * sW[wave][r];
                    sW[wave][t] = acc / (double)L[t * SMAX + t];
                    d2_64 -= sW[wave][t] * sW[wave][t];
                }
                sD2[wave] = d2_64;
                atomicAdd(&a.ctl->fp64_pivot_recomputes, 1ull);
            }
            wave_lds_sync();
            const double d2_64 = sD2[wave];
            if (!(d2_64 > (double)a.tol_pivot * (double)gjj))
                break;
#pragma unroll
            for (int t = 0; t < SMAX; ++t)
                if (t < k)
                    w[t] = (float)sW[wave][t];
            d2 = (float)d2_64;
        }
        const float delta = sqrtf(d2);
        const float inv = 1.0f / delta;

        // 3. u_k = (G[j,:] - sum_t w_t u_t) / delta
        vec unew = g;
#pragma unroll
        for (int t = 0; t < SMAX; ++t)
            if (t < k)
                unew -= w[t] * u[t];
        unew *= inv;
#pragma unroll
        for (int t = 0; t < SMAX; ++t)
            if (t == k)
                u[t] = unew;

        // 4. coefficient on q_k and the correlation update
        const float ck = readlane_f(pick<NPL>(alpha, cj), lj) * inv;
        alpha -= ck * unew;
        if (lane == lj)
            selmask |= 1u << cj;
        if (lane < SMAX) {
            float lv = 0.f;
#pragma unroll
            for (int t = 0; t < SMAX; ++t)
                if (t == lane)
                    lv = w[t];
            if (lane < k)
                L[k * SMAX + lane] = lv;
            if (lane == k)
                L[k * SMAX + k] = delta;
        }
        if (lane == 0) {
            sI[wave][k] = j;
            sC[wave][k] = ck;
        }
        wave_lds_sync();
    }
    if (k < s && lane == 0)
        atomicAdd(&a.ctl->early_stops, 1ull);

    // coefficients: L^T x = c (back substitution; uniform scalar work)
    if (lane == 0) {
        for (int r = k - 1; r >= 0; --r) {
            float acc = sC[wave][r];
            for (int t = r + 1; t < k; ++t)
                acc -= L[t * SMAX + r] * sX[wave][t];
            sX[wave][r] = acc / L[r * SMAX + r];
        }
    }
    wave_lds_sync();

    if (lane < s) {
        const bool on = lane < k;
        a.idx[(size_t)i * s + lane] = on ? sI[wave][lane] : -1;
        a.val[(size_t)i * s + lane] = on ? sX[wave][lane] : 0.f;
    }
    // residual e = y - D_I x with the dictionary used for coding
    if (a.E) {
        float e[PR];
#pragma unroll
        for (int r = 0; r < PR; ++r)
            e[r] = yv[r];
        for (int t = 0; t < k; ++t) {
            const float x = sX[wave][t];
            const float *d = a.D + (size_t)sI[wave][t] * p;
#pragma unroll
            for (int r = 0; r < PR; ++r) {
                const int q = lane + 64 * r;
                if (q < p)
                    e[r] -= d[q] * x;
            }
        }
#pragma unroll
        for (int r = 0; r < PR; ++r) {
            const int q = lane + 64 * r;
            if (q < p)
                a.E[(size_t)i * p + q] = e[r];
        }
    }
}

template <int NPL, int SMAX>
hipError_t launch_omp_t(const OmpArgs &a, hipStream_t st)
{
    const int blocks = (a.m + kWaves - 1) / kWaves;
    hipLaunchKernelGGL((omp_kernel<NPL, SMAX>), dim3(blocks), dim3(64 * kWaves), 0, st, a);
    return hipGetLastError();
}

template <int NPL>
hipError_t launch_omp_s(const OmpArgs &a, hipStream_t st)
{
    if (a.s <= 4)
        return launch_omp_t<NPL, 4>(a, st);
    if (a.s <= 8)
        return launch_omp_t<NPL, 8>(a, st);
    if (a.s <= 12)
        return launch_omp_t<NPL, 12>(a, st);
    return launch_omp_t<NPL, 16>(a, st);
}

}  // namespace

hipError_t launch_omp(const OmpArgs &a, hipStream_t st)
{
    const int npl = (a.n + 63) / 64;
    if (npl <= 1)
        return launch_omp_s<1>(a, st);
    if (npl <= 2)
        return launch_omp_s<2>(a, st);
    if (npl <= 4)
        return launch_omp_s<4>(a, st);
    if (npl <= 8)
        return launch_omp_s<8>(a, st);
    return launch_omp_s<16>(a, st);
}

}  // namespace dlk
