// Sparse coding (step 1 of the DL iteration, Alg. 1): OMP with fixed
// sparsity s, computed Batch-OMP style from G = D D^T and A0 = Y D^T.
//
// A signal is handled by a group of LPS lanes of a wavefront (64/LPS signals
// per wave); lane l of the group owns atoms [l*NPL, (l+1)*NPL).  The group
// keeps the correlations alpha = D^T r of the signal's current residual in
// registers.  Each step k:
//   1. j = argmax over unselected atoms of |alpha_j| (ties: lowest index),
//      reduced over the group with DPP moves;
//   2. the new Cholesky row of G_II: w_t = u_t[j] (t < k) and
//      delta^2 = G_jj - |w|^2; pivots below `pivot_fp64` are recomputed in
//      FP64 from the G entries by forward substitution with L;
//   3. u_k = (G[j,:] - sum_t w_t u_t) / delta, which equals D^T q_k for the
//      orthonormalised new direction q_k;
//   4. c_k = alpha_j / delta (the coefficient of y on q_k) and
//      alpha -= c_k u_k (the residual loses its q_k component).
// The coefficients then solve L^T x = c (D_I = Q L^T with L the Cholesky
// factor of G_II).  This is Batch-OMP's alpha = A0 - G_I (G_II^{-1} A0_I)
// rearranged so that a step is one pass over the n correlations and needs no
// triangular solve.  The last step needs neither u_k nor the alpha update.
//
// u_t live in registers ((SMAX-1) x NPL per lane); L, c, the support and x
// live in LDS, one small block per signal.  G and A0 rows have leading
// dimension ldn (a multiple of 4, so rows load as float4).
#include "dl_internal.h"

namespace dlk {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;  // waves per workgroup

__device__ inline float bits_f(int v) { return __int_as_float(v); }
__device__ inline int f_bits(float v) { return __float_as_int(v); }

// Order this wave's LDS stores before its later LDS loads from other lanes.
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int CTRL>
__device__ inline int dpp(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

// Combine (value, index) pairs: larger value wins, lower index on ties.
__device__ inline void take_better(float &v, int &ix, float ov, int oi)
{
    if (ov > v || (ov == v && oi < ix)) {
        v = ov;
        ix = oi;
    }
}

// All-reduce of (max value, lowest index) over groups of LPS lanes.
template <int LPS>
__device__ inline void group_argmax(float &v, int &ix)
{
    if constexpr (LPS >= 2)
        take_better(v, ix, bits_f(dpp<0xB1>(f_bits(v))), dpp<0xB1>(ix));      // lane ^ 1
    if constexpr (LPS >= 4)
        take_better(v, ix, bits_f(dpp<0x4E>(f_bits(v))), dpp<0x4E>(ix));      // lane ^ 2
    if constexpr (LPS >= 8)
        take_better(v, ix, bits_f(dpp<0x141>(f_bits(v))), dpp<0x141>(ix));    // half-row mirror
    if constexpr (LPS >= 16)
        take_better(v, ix, bits_f(dpp<0x140>(f_bits(v))), dpp<0x140>(ix));    // row mirror
    if constexpr (LPS >= 32)
        take_better(v, ix, __shfl_xor(v, 16), __shfl_xor(ix, 16));
    if constexpr (LPS >= 64)
        take_better(v, ix, __shfl_xor(v, 32), __shfl_xor(ix, 32));
}

template <int LPS>
__device__ inline float group_sum(float v)
{
    if constexpr (LPS >= 2)
        v += bits_f(dpp<0xB1>(f_bits(v)));
    if constexpr (LPS >= 4)
        v += bits_f(dpp<0x4E>(f_bits(v)));
    if constexpr (LPS >= 8)
        v += bits_f(dpp<0x141>(f_bits(v)));
    if constexpr (LPS >= 16)
        v += bits_f(dpp<0x140>(f_bits(v)));
    if constexpr (LPS >= 32)
        v += __shfl_xor(v, 16);
    if constexpr (LPS >= 64)
        v += __shfl_xor(v, 32);
    return v;
}

// A lane's NPL values are one vector value (not an array), so that selecting
// element c (which may differ between groups) stays a compare/select chain on
// registers and never becomes an indexed access to a private memory copy.
template <int NPL>
using vec_t = float __attribute__((ext_vector_type(NPL)));

template <int NPL>
__device__ inline float select(const vec_t<NPL> &v, int c)
{
    float r = v[0];
#pragma unroll
    for (int q = 1; q < NPL; ++q)
        r = (c == q) ? v[q] : r;
    return r;
}

// Broadcast of element c of lane `src` (same for the whole group) to the group.
template <int LPS, int NPL>
__device__ inline float group_fetch(const vec_t<NPL> &v, int c, int src_lane)
{
    return __shfl(select<NPL>(v, c), src_lane, 64);
}

template <int LPS, int NPL, int SMAX>
__global__ __launch_bounds__(64 * kWaves) void omp_kernel(OmpArgs a)
{
    constexpr int GPW = 64 / LPS;        // signals per wave
    constexpr int US = SMAX > 1 ? SMAX - 1 : 1;  // stored u vectors
    __shared__ float sL[kWaves][GPW][SMAX * SMAX];
    __shared__ float sC[kWaves][GPW][SMAX];
    __shared__ float sX[kWaves][GPW][SMAX];
    __shared__ int sI[kWaves][GPW][SMAX];
    __shared__ float sG[kWaves][GPW][SMAX];
    __shared__ double sW[kWaves][GPW][SMAX];
    __shared__ double sD2[kWaves][GPW];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int grp = lane / LPS;          // signal slot of this lane in the wave
    const int l = lane % LPS;            // lane within the group
    const int base = lane - l;           // first lane of the group
    const int wave_sig0 = (blockIdx.x * kWaves + wave) * GPW;
    if (wave_sig0 >= a.m)
        return;  // whole wave leaves together; no workgroup barrier follows
    const int i = wave_sig0 + grp;
    const bool valid = i < a.m;
    const int n = a.n, p = a.p, s = a.s, ldn = a.ldn;
    float *L = sL[wave][grp];

    // ||y|| for the orthogonality stop rule
    float ysq = 0.f;
    if (valid)
        for (int q = 4 * l; q < p; q += 4 * LPS) {
            const f32x4 y = *reinterpret_cast<const f32x4 *>(a.Y + (size_t)i * p + q);
            ysq += y[0] * y[0] + y[1] * y[1] + y[2] * y[2] + y[3] * y[3];
        }
    const float ynorm = sqrtf(group_sum<LPS>(ysq));
    const float thr = a.tol_corr * ynorm;

    // correlations of y; atoms beyond n are marked as taken
    vec_t<NPL> alpha;
    unsigned taken = 0;
    const int a_first = l * NPL;
#pragma unroll
    for (int c4 = 0; c4 < NPL / 4; ++c4) {
        const int at = a_first + 4 * c4;
        f32x4 v = {0.f, 0.f, 0.f, 0.f};
        if (valid && at < ldn)
            v = *reinterpret_cast<const f32x4 *>(a.A0 + (size_t)i * ldn + at);
#pragma unroll
        for (int r = 0; r < 4; ++r)
            alpha[4 * c4 + r] = v[r];
    }
#pragma unroll
    for (int c = 0; c < NPL; ++c)
        if (a_first + c >= n)
            taken |= 1u << c;

    vec_t<NPL> u[US];
    bool active = valid && isfinite(ynorm);
    if (valid && !isfinite(ynorm) && l == 0)
        atomicAdd(&a.ctl->nonfinite, 1ull);
    int kg = 0;  // atoms selected for this lane's signal

    for (int k = 0; k < s; ++k) {
        if (!__any(active))
            break;
        // 1. masked argmax over the group, lowest index on ties
        float best = -1.f;
        int bidx = 0x7fffffff;
#pragma unroll
        for (int c = 0; c < NPL; ++c) {
            const float v = fabsf(alpha[c]);
            if (!((taken >> c) & 1u) && v > best) {
                best = v;
                bidx = a_first + c;
            }
        }
        group_argmax<LPS>(best, bidx);
        bool ok = active && best > thr && bidx < n;
        const int j = ok ? bidx : 0;
        const int cj = j % NPL, lj = base + j / NPL;

        // 2. Cholesky row of G_II for the new atom
        vec_t<NPL> g;
#pragma unroll
        for (int c4 = 0; c4 < NPL / 4; ++c4) {
            const int at = a_first + 4 * c4;
            f32x4 v = {0.f, 0.f, 0.f, 0.f};
            if (ok && at < ldn)
                v = *reinterpret_cast<const f32x4 *>(a.G + (size_t)j * ldn + at);
#pragma unroll
            for (int r = 0; r < 4; ++r)
                g[4 * c4 + r] = v[r];
        }
        const float gjj = group_fetch<LPS, NPL>(g, cj, lj);
        float w[US];
        float d2 = gjj;
#pragma unroll
        for (int t = 0; t < US; ++t) {
            w[t] = 0.f;
            if (t < k) {
                w[t] = group_fetch<LPS, NPL>(u[t], cj, lj);
                d2 -= w[t] * w[t];
            }
        }
        const bool need64 = ok && d2 < a.pivot_fp64;
        if (__any(need64)) {
            // rare: w = L^{-1} G[I, j] and the pivot in FP64 (lane t of the
            // group fetches G[j][I_t]; the group's first lane substitutes)
            for (int t = l; t < k; t += LPS)
                if (need64)
                    sG[wave][grp][t] = a.G[(size_t)j * ldn + sI[wave][grp][t]];
            wave_lds_sync();
            if (need64 && l == 0) {
                double d2_64 = (double)gjj;
                for (int t = 0; t < k; ++t) {
                    double acc = (double)sG[wave][grp][t];
                    for (int r = 0; r < t; ++r)
                        acc -= (double)L[t * SMAX + r] * sW[wave][grp][r];
                    sW[wave][grp][t] = acc / (double)L[t * SMAX + t];
                    d2_64 -= sW[wave][grp][t] * sW[wave][grp][t];
                }
                sD2[wave][grp] = d2_64;
                atomicAdd(&a.ctl->fp64_pivot_recomputes, 1ull);
            }
            wave_lds_sync();
            if (need64) {
                const double d2_64 = sD2[wave][grp];
                if (!(d2_64 > (double)a.tol_pivot * (double)gjj)) {
                    ok = false;
                } else {
#pragma unroll
                    for (int t = 0; t < US; ++t)
                        if (t < k)
                            w[t] = (float)sW[wave][grp][t];
                    d2 = (float)d2_64;
                }
            }
        }
        if (!ok)
            active = false;
        const float delta = sqrtf(d2);
        const float inv = 1.0f / delta;
        // 4. coefficient of y on q_k
        const float ck = group_fetch<LPS, NPL>(alpha, cj, lj) * inv;
        if (ok && k + 1 < s) {
            // 3. u_k and the correlation update (not needed after the last step)
            vec_t<NPL> unew = g;
#pragma unroll
            for (int t = 0; t < US; ++t)
                if (t < k)
                    unew -= w[t] * u[t];
            unew *= inv;
            alpha -= ck * unew;
#pragma unroll
            for (int t = 0; t < US; ++t)
                if (t == k)
                    u[t] = unew;
        }
        if (ok) {
            if (lane == lj)
                taken |= 1u << cj;
            // row k of L, and the support / coefficient bookkeeping
            for (int t = l; t < k; t += LPS) {
                float wt = w[0];
#pragma unroll
                for (int q = 1; q < US; ++q)
                    wt = (t == q) ? w[q] : wt;
                L[k * SMAX + t] = wt;
            }
            if (l == 0) {
                L[k * SMAX + k] = delta;
                sI[wave][grp][k] = j;
                sC[wave][grp][k] = ck;
            }
            kg = k + 1;
        }
        wave_lds_sync();
    }
    if (valid && l == 0 && kg < s)
        atomicAdd(&a.ctl->early_stops, 1ull);

    // coefficients: L^T x = c (back substitution, the group's first lane)
    if (valid && l == 0) {
        for (int r = kg - 1; r >= 0; --r) {
            float acc = sC[wave][grp][r];
            for (int t = r + 1; t < kg; ++t)
                acc -= L[t * SMAX + r] * sX[wave][grp][t];
            sX[wave][grp][r] = acc / L[r * SMAX + r];
        }
    }
    wave_lds_sync();
    if (!valid)
        return;
    for (int t = l; t < s; t += LPS) {
        const bool on = t < kg;
        a.idx[(size_t)i * s + t] = on ? sI[wave][grp][t] : -1;
        a.val[(size_t)i * s + t] = on ? sX[wave][grp][t] : 0.f;
    }
    // residual e = y - D_I x with the dictionary used for coding
    if (a.E) {
        for (int q = 4 * l; q < p; q += 4 * LPS) {
            f32x4 e = *reinterpret_cast<const f32x4 *>(a.Y + (size_t)i * p + q);
            for (int t = 0; t < kg; ++t) {
                const f32x4 d =
                    *reinterpret_cast<const f32x4 *>(a.D + (size_t)sI[wave][grp][t] * p + q);
                e -= d * sX[wave][grp][t];
            }
            *reinterpret_cast<f32x4 *>(a.E + (size_t)i * p + q) = e;
        }
    }
}

template <int LPS, int NPL, int SMAX>
hipError_t launch_omp_t(const OmpArgs &a, hipStream_t st)
{
    constexpr int sig_per_block = kWaves * (64 / LPS);
    const int blocks = (a.m + sig_per_block - 1) / sig_per_block;
    prof_begin(DL_K_OMP, st);
    hipLaunchKernelGGL((omp_kernel<LPS, NPL, SMAX>), dim3(blocks), dim3(64 * kWaves), 0, st, a);
    prof_end(DL_K_OMP, st);
    return hipGetLastError();
}

template <int LPS, int NPL>
hipError_t launch_omp_s(const OmpArgs &a, hipStream_t st)
{
    if (a.s <= 4)
        return launch_omp_t<LPS, NPL, 4>(a, st);
    if (a.s <= 6)
        return launch_omp_t<LPS, NPL, 6>(a, st);
    if (a.s <= 8)
        return launch_omp_t<LPS, NPL, 8>(a, st);
    if (a.s <= 12)
        return launch_omp_t<LPS, NPL, 12>(a, st);
    return launch_omp_t<LPS, NPL, 16>(a, st);
}

}  // namespace

// Default lanes per signal for n atoms at `npl` atoms per lane (4..64).
int omp_lanes_per_signal(int n, int npl)
{
    int lps = 4;
    while (lps * npl < n && lps < 64)
        lps <<= 1;
    return lps;
}

bool omp_config_ok(int n, int lps, int npl)
{
    const bool lps_ok = lps == 4 || lps == 8 || lps == 16 || lps == 32 || lps == 64;
    const bool npl_ok = npl == 16 || (npl == 8 && lps >= 8);
    return lps_ok && npl_ok && lps * npl >= n;
}

hipError_t launch_omp(const OmpArgs &a, hipStream_t st)
{
    const int npl = a.atoms_per_lane > 0 ? a.atoms_per_lane : 16;
    const int lps = a.lanes_per_signal > 0 ? a.lanes_per_signal : omp_lanes_per_signal(a.n, npl);
    if (!omp_config_ok(a.n, lps, npl))
        return hipErrorInvalidValue;
    if (npl == 8) {
        switch (lps) {
        case 8: return launch_omp_s<8, 8>(a, st);
        case 16: return launch_omp_s<16, 8>(a, st);
        case 32: return launch_omp_s<32, 8>(a, st);
        case 64: return launch_omp_s<64, 8>(a, st);
        default: return hipErrorInvalidValue;
        }
    }
    switch (lps) {
    case 4: return launch_omp_s<4, 16>(a, st);
    case 8: return launch_omp_s<8, 16>(a, st);
    case 16: return launch_omp_s<16, 16>(a, st);
    case 32: return launch_omp_s<32, 16>(a, st);
    case 64: return launch_omp_s<64, 16>(a, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace dlk
