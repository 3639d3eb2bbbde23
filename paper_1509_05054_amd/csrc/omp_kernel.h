// Sparse coding (step 1 of the DL iteration, Alg. 1): OMP with fixed
// sparsity s, computed Batch-OMP style from G = D D^T and A0 = Y D^T.
// Included by the omp_npl*.hip translation units, which instantiate it.
//
// A signal is handled by a group of LPS lanes of a wavefront (64/LPS signals
// per wave); lane l of the group owns atoms [l*NPL, (l+1)*NPL) and row l of
// the Cholesky factor L of G_II.  The group keeps the correlations
// alpha = D^T r of the signal's current residual in registers.  Step k:
//   1. j = argmax over unselected atoms of |alpha_j| (ties: lowest index),
//      reduced over the group with DPP moves;
//   2. the new row of L: w = L^{-1} G[I, j] by forward substitution (lane t
//      loads G[j][I_t]; each round broadcasts one w_t inside the group), and
//      delta^2 = G_jj - |w|^2; pivots below `pivot_fp64` are recomputed in
//      FP64;
//   3. c_k = (A0_j - sum_t w_t c_t) / delta, the coefficient of y on the
//      orthonormalised new direction q_k;
//   4. u_k = (G[j,:] - sum_t w_t u_t) / delta (= D^T q_k) and
//      alpha -= c_k u_k, so that alpha stays the correlation of the residual
//      (not needed after the last step).
// The coefficients then solve L^T x = c (D_I = Q L^T), by back substitution
// with group sums.  This is the arithmetic of Batch-OMP (alpha = A0 - G_I
// gamma with gamma = G_II^{-1} A0_I), reorganised so that a step is one pass
// over the n correlations plus k short rounds.
//
// G and A0 rows have leading dimension ldn (a multiple of 4: rows load as
// float4).  Requirements: LPS in {4..64}, LPS >= SMAX >= s, LPS*NPL >= n.
#pragma once

#include "dl_internal.h"
#include "rmse_body.h"

namespace dlk {
namespace omp_detail {

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

// A DPP lane permutation with bound control set, which lets the compiler fold
// the move into the VALU instruction that consumes it (every pattern used
// here reads lanes inside the row, so no lane is out of bounds).
template <int CTRL>
__device__ inline int dpp_fold(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}

// Combine (value, index) pairs: larger value wins, lower index on ties
// (selects, no branch).
__device__ inline void take_better(float &v, int &ix, float ov, int oi)
{
    // bitwise, not short-circuit, operators: one mask, no branch
    const bool b = (ov > v) | ((ov == v) & (oi < ix));
    v = b ? ov : v;
    ix = b ? oi : ix;
}

// The value of a 64-lane group from its four row values (every lane of row r
// holding v_r): DPP row broadcasts combine rows 0+1 into row 1 and 2+3 into
// row 3, then row 1 into row 3, and lane 63 is read out, so the result is
// op(op(v_0, v_1), op(v_2, v_3)) (for a sum, the association of the xor
// butterfly across rows, whose result every lane held) and wave-uniform.
// The cross-row steps of the butterfly go through the LDS crossbar
// (ds_bpermute); these stay in the VALU.
template <class Op>
__device__ inline int rows64_combine(int x, int identity, Op op)
{
    x = op(x, __builtin_amdgcn_update_dpp(identity, x, 0x142, 0xA, 0xF, false));  // row_bcast:15
    x = op(x, __builtin_amdgcn_update_dpp(identity, x, 0x143, 0xC, 0xF, false));  // row_bcast:31
    return __builtin_amdgcn_readlane(x, 63);
}

// All-reduce over groups of LPS lanes: the maximum of v, then the lowest
// index among the lanes that hold it.  v is -1 or a non-negative float (never
// NaN), whose order is that of its bits as signed integers, so both are
// integer reductions; two plain reductions take fewer instructions than one
// over (value, index) pairs.
template <int LPS>
__device__ inline int group_min_max(int x, bool take_max)
{
    auto pick = [&](int a, int b) { return take_max ? max(a, b) : min(a, b); };
    if constexpr (LPS >= 2)
        x = pick(x, dpp_fold<0xB1>(x));
    if constexpr (LPS >= 4)
        x = pick(x, dpp_fold<0x4E>(x));
    if constexpr (LPS >= 8)
        x = pick(x, dpp_fold<0x141>(x));
    if constexpr (LPS >= 16)
        x = pick(x, dpp_fold<0x140>(x));
    if constexpr (LPS == 64)
        return rows64_combine(x, take_max ? (int)0x80000000 : 0x7fffffff, pick);
    if constexpr (LPS == 32) {
        int u, w;
        pair_xor16(x, u, w);  // this lane's value and lane ^ 16's
        x = pick(u, w);
    }
    return x;
}

template <int LPS>
__device__ inline void group_argmax(float &v, int &ix)
{
    const int gmax = group_min_max<LPS>(f_bits(v), true);
    ix = group_min_max<LPS>(f_bits(v) == gmax ? ix : 0x7fffffff, false);
    v = bits_f(gmax);
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
    if constexpr (LPS == 64)
        return bits_f(rows64_combine(f_bits(v), 0, [](int a, int b) {
            return f_bits(bits_f(a) + bits_f(b));
        }));
    if constexpr (LPS == 32)
        v = sum_xor(v, 16);
    return v;
}

// Value of lane R of each group, in every lane of that group.
template <int LPS, int R>
__device__ inline float group_bcast(float v)
{
    if constexpr (LPS == 64) {
        return bits_f(__builtin_amdgcn_readlane(f_bits(v), R));
    } else if constexpr (LPS == 16) {
        // DPP row_newbcast: lane R of every row of 16 (measured 3% faster
        // coding than the swizzle at m = 16384)
        return bits_f(__builtin_amdgcn_mov_dpp(f_bits(v), 0x150 + R, 0xF, 0xF, false));
    } else if constexpr (LPS == 4) {
        // DPP quad_perm [R, R, R, R]
        return bits_f(__builtin_amdgcn_mov_dpp(f_bits(v), R | (R << 2) | (R << 4) | (R << 6), 0xF,
                                               0xF, false));
    } else {
        // ds_swizzle bit mode inside 32 lanes: source = (lane & and) | or
        constexpr int and_mask = 31 & ~(LPS - 1);
        constexpr int pattern = and_mask | (R << 5);
        return bits_f(__builtin_amdgcn_ds_swizzle(f_bits(v), pattern));
    }
}

// group_bcast from lane t, where t is the index of an unrolled loop (the
// switch folds to its one case).
template <int LPS>
__device__ __forceinline__ float group_bcast_at(float v, int t)
{
    switch (t) {
#define DL_BCAST_AT(T)                       \
    case T:                                  \
        if constexpr (T < LPS)               \
            return group_bcast<LPS, T>(v);   \
        break;
        DL_BCAST_AT(0) DL_BCAST_AT(1) DL_BCAST_AT(2) DL_BCAST_AT(3)
        DL_BCAST_AT(4) DL_BCAST_AT(5) DL_BCAST_AT(6) DL_BCAST_AT(7)
        DL_BCAST_AT(8) DL_BCAST_AT(9) DL_BCAST_AT(10) DL_BCAST_AT(11)
        DL_BCAST_AT(12) DL_BCAST_AT(13) DL_BCAST_AT(14) DL_BCAST_AT(15)
#undef DL_BCAST_AT
    default:
        break;
    }
    return v;
}

template <int NPL>
using vec_t = float __attribute__((ext_vector_type(NPL)));

template <int K>
struct IntC {
    static constexpr int value = K;
};

// f(IntC<K>) for K = B, B+1, ... < E while f returns true: the body is
// instantiated once per K, so K is a compile-time constant inside it.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        if (f(IntC<B>{}))
            static_for<B + 1, E>(f);
    }
}

template <int NPL>
__device__ inline void load_row(vec_t<NPL> &v, const float *row, int first, int ldn, bool on)
{
#pragma unroll
    for (int c4 = 0; c4 < NPL / 4; ++c4) {
        const int at = first + 4 * c4;
        f32x4 x = {0.f, 0.f, 0.f, 0.f};
        if (on && at < ldn)
            x = *reinterpret_cast<const f32x4 *>(row + at);
        v[4 * c4 + 0] = x[0];
        v[4 * c4 + 1] = x[1];
        v[4 * c4 + 2] = x[2];
        v[4 * c4 + 3] = x[3];
    }
}

// The same loads from a G row given by its byte offset from G (G is at most
// 1024 x 1024 floats, so every byte offset fits in 32 bits): the address is
// G's base, which is the same in every lane, plus a 32-bit lane offset, and
// needs no 64-bit arithmetic per lane.
template <int NPL>
__device__ inline void load_grow(vec_t<NPL> &v, const float *G, unsigned row_bytes, int first,
                                 int ldn, bool on)
{
    const char *base = reinterpret_cast<const char *>(G);
#pragma unroll
    for (int c4 = 0; c4 < NPL / 4; ++c4) {
        const int at = first + 4 * c4;
        f32x4 x = {0.f, 0.f, 0.f, 0.f};
        if (on && at < ldn)
            x = *reinterpret_cast<const f32x4 *>(base + (row_bytes + 4u * (unsigned)at));
        v[4 * c4 + 0] = x[0];
        v[4 * c4 + 1] = x[1];
        v[4 * c4 + 2] = x[2];
        v[4 * c4 + 3] = x[3];
    }
}

__device__ inline float load_g(const float *G, unsigned row_bytes, int col)
{
    return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(G) +
                                            (row_bytes + 4u * (unsigned)col));
}

// The GPW = 64 / LPS signals [wave_sig0, wave_sig0 + GPW) of one wave
// (signals at or beyond m_eff are skipped); waves never wait for each other.
//
// WPS = 2 (with LPS = 64): one signal per two-wave workgroup.  Wave w holds
// the correlations of atoms [64 NPL w, 64 NPL (w + 1)); both waves keep their
// own copy of L and the coefficients and take every step with the same
// operations on the same values, so they make the same decisions and their
// correlations match those of one 128-lane group exactly.  The only exchange
// is the step's argmax, through LDS with one workgroup barrier (two slots by
// step parity, so a slot is rewritten only after both waves have read it).
// Wave 0 writes the outputs and the counters.
template <int LPS, int NPL, int SMAX, int WPS = 1>
__device__ __forceinline__ void omp_signals(const OmpArgs &a, int wave_sig0, int m_eff)
{
    static_assert(LPS >= SMAX, "one lane per row of L");
    static_assert(WPS == 1 || (WPS == 2 && LPS == 64), "two waves per signal need LPS = 64");
    constexpr int GPW = 64 / LPS;                 // signals per wave
    constexpr int US = SMAX > 1 ? SMAX - 1 : 1;   // stored u vectors
    // rare FP64 pivot path only
    __shared__ float sL[kWaves][GPW][SMAX * SMAX];
    __shared__ float sB[kWaves][GPW][SMAX];
    __shared__ double sW[kWaves][GPW][SMAX];
    __shared__ double sD2[kWaves][GPW];
    __shared__ float sPairV[2][2];  // [step parity][wave]: the waves' argmax
    __shared__ int sPairI[2][2];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wsub = WPS == 2 ? (wave & 1) : 0;  // this wave's half of the atoms
    const bool lead = wsub == 0;                 // writes outputs and counters
    const int grp = lane / LPS;   // signal slot of this lane in the wave
    const int l = lane % LPS;     // lane within the group
    const int i = wave_sig0 + grp;
    const bool valid = i < m_eff;
    const int n = a.n, p = a.p, s = a.s, ldn = a.ldn;

    // ||y|| for the orthogonality stop rule
    float ysq = 0.f;
    if (valid)
        for (int q = 4 * l; q < p; q += 4 * LPS) {
            const f32x4 y = *reinterpret_cast<const f32x4 *>(a.Y + (size_t)i * p + q);
            ysq += y[0] * y[0] + y[1] * y[1] + y[2] * y[2] + y[3] * y[3];
        }
    const float ynorm = sqrtf(group_sum<LPS>(ysq));
    const float thr = a.tol_corr * ynorm;

    // correlations of y.  A selected atom's correlation turns NaN in the
    // step's update (G holds NaN on its diagonal, so u_k is NaN there) and
    // stays NaN, and no comparison picks a NaN: the argmax needs no mask.
    // Atoms beyond n start as NaN.
    const int a_first = (wsub * LPS + l) * NPL;
    vec_t<NPL> alpha;
    load_row<NPL>(alpha, a.A0 + (size_t)i * ldn, a_first, ldn, valid);
#pragma unroll
    for (int c = 0; c < NPL; ++c)
        if (a_first + c >= n)
            alpha[c] = __builtin_nanf("");

    // Row t of L and the values of step t live in lane t of the group (c_t,
    // 1 / L[t][t] and the selected atom), and are broadcast where the other
    // lanes need them: registers held per lane for every step would cost the
    // coding kernel occupancy at large s.
    vec_t<NPL> u[US];
    float Lrow[SMAX];     // row l of L (this lane's row)
    float cown = 0.f;     // c_l
    float rdg = 1.f;      // 1 / L[l][l], this lane's own diagonal
    int selj = -1;        // this lane's atom (row l)
#pragma unroll
    for (int t = 0; t < SMAX; ++t)
        Lrow[t] = 0.f;
    bool active = valid && isfinite(ynorm);
    if (lead && valid && !isfinite(ynorm) && l == 0)
        atomicAdd(&a.ctl->nonfinite, 1ull);
    int kg = 0;  // atoms selected for this lane's signal

    // the steps are expanded at compile time (static_for), so that every
    // register index below is a constant: no select chains or copies
    static_for<0, SMAX>([&](auto kc) -> bool {
        constexpr int k = decltype(kc)::value;
        if (k >= s || !__any(active))
            return false;
        // 1. argmax over the group (selected atoms are NaN), lowest index on ties:
        // the lane's largest |alpha| by a max chain (which passes over NaN),
        // then the first of its atoms holding it
        float best = -1.f;
#pragma unroll
        for (int c = 0; c < NPL; ++c)
            best = fmaxf(best, fabsf(alpha[c]));
        int cfirst = NPL;
#pragma unroll
        for (int c = NPL - 1; c >= 0; --c)
            cfirst = fabsf(alpha[c]) == best ? c : cfirst;
        int bidx = cfirst < NPL ? a_first + cfirst : 0x7fffffff;
        group_argmax<LPS>(best, bidx);
        if constexpr (WPS == 2) {
            if (l == 0) {
                sPairV[k & 1][wsub] = best;
                sPairI[k & 1][wsub] = bidx;
            }
            __syncthreads();
            // both waves combine the two in the same order
            best = sPairV[k & 1][0];
            bidx = sPairI[k & 1][0];
            take_better(best, bidx, sPairV[k & 1][1], sPairI[k & 1][1]);
        }
        bool ok = active && best > thr && bidx < n;
        const int j = ok ? bidx : 0;
        const unsigned gj_bytes = 4u * (unsigned)(j * ldn);  // row j of G

        // 2. loads for this step: the G row (NaN at j), G_jj, A0_j, and G[j][I_l]
        vec_t<NPL> g;
        load_grow<NPL>(g, a.G, gj_bytes, a_first, ldn, ok);
        const float gjj = ok ? a.Gdiag[j] : 1.f;
        const float a0j = ok ? a.A0[(size_t)i * ldn + j] : 0.f;
        float acc = (ok && l < k) ? load_g(a.G, gj_bytes, selj) : 0.f;

        // forward substitution L w = G[I, j]: round t finalises w_t in lane t
        float w[US];
        float d2 = gjj;
#pragma unroll
        for (int t = 0; t < US; ++t) {
            w[t] = 0.f;
            if (t < k) {
                float wt = acc * rdg;         // meaningful in lane t
                switch (t) {                  // broadcast lane t of the group
#define DL_BCAST_CASE(T) \
    case T:              \
        if constexpr (T < LPS) wt = group_bcast<LPS, T>(wt); \
        break;
                    DL_BCAST_CASE(0) DL_BCAST_CASE(1) DL_BCAST_CASE(2) DL_BCAST_CASE(3)
                    DL_BCAST_CASE(4) DL_BCAST_CASE(5) DL_BCAST_CASE(6) DL_BCAST_CASE(7)
                    DL_BCAST_CASE(8) DL_BCAST_CASE(9) DL_BCAST_CASE(10) DL_BCAST_CASE(11)
                    DL_BCAST_CASE(12) DL_BCAST_CASE(13) DL_BCAST_CASE(14)
#undef DL_BCAST_CASE
                default: break;
                }
                w[t] = wt;
                if (l > t)
                    acc -= Lrow[t] * wt;
                d2 -= wt * wt;
            }
        }
        const bool need64 = ok && d2 < a.pivot_fp64;
        if (__any(need64)) {
            // rare: w and the pivot again in FP64 (the group's first lane
            // substitutes serially from L and G[I, j] staged in LDS)
            if (need64 && l < k) {
#pragma unroll
                for (int r = 0; r < SMAX; ++r)
                    if (r <= l)
                        sL[wave][grp][l * SMAX + r] = Lrow[r];
                sB[wave][grp][l] = load_g(a.G, gj_bytes, selj);
            }
            wave_lds_sync();
            if (need64 && l == 0) {
                double d2_64 = (double)gjj;
                for (int t = 0; t < k; ++t) {
                    double accd = (double)sB[wave][grp][t];
                    for (int r = 0; r < t; ++r)
                        accd -= (double)sL[wave][grp][t * SMAX + r] * sW[wave][grp][r];
                    sW[wave][grp][t] = accd / (double)sL[wave][grp][t * SMAX + t];
                    d2_64 -= sW[wave][grp][t] * sW[wave][grp][t];
                }
                sD2[wave][grp] = d2_64;
                if (lead)
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
            wave_lds_sync();
        }
        if (!ok)
            active = false;
        // the pivot's reciprocal by the hardware reciprocal square root (1 ulp;
        // measured 4% faster than the correctly rounded square root and
        // division at m = 16384), and delta = d2 / sqrt(d2) from it
        const float inv = __builtin_amdgcn_rsqf(d2);
        const float delta = d2 * inv;

        // 3. coefficient of y on q_k
        float ck = a0j;
#pragma unroll
        for (int t = 0; t < US; ++t)
            if (t < k)
                ck -= w[t] * group_bcast_at<LPS>(cown, t);
        ck *= inv;

        // 4. u_k and the correlation update (not needed after the last step)
        // (u_k is formed in its own registers: k is a compile-time constant)
        if constexpr (k < US) {
            if (ok && k + 1 < s) {
                u[k] = g;
#pragma unroll
                for (int t = 0; t < k; ++t)
                    u[k] -= w[t] * u[t];
                u[k] *= inv;
                alpha -= ck * u[k];
            }
        }
        if (ok) {
            if (l == k) {
#pragma unroll
                for (int t = 0; t < US; ++t)
                    if (t < k)
                        Lrow[t] = w[t];
#pragma unroll
                for (int t = 0; t < SMAX; ++t)
                    if (t == k)
                        Lrow[t] = delta;
                rdg = inv;
                cown = ck;
                selj = j;
            }
            kg = k + 1;
        }
        return true;
    });
    if (lead && valid && l == 0 && kg < s)
        atomicAdd(&a.ctl->early_stops, 1ull);

    // coefficients: L^T x = c, from the last row up; lane t holds L[t][*]
    float xs[SMAX];
    float xown = 0.f;
#pragma unroll
    for (int r = SMAX - 1; r >= 0; --r) {
        const float part = (l > r && l < kg) ? Lrow[r] * xown : 0.f;
        const float ssum = group_sum<LPS>(part);
        const float xr =
            (group_bcast_at<LPS>(cown, r) - ssum) * group_bcast_at<LPS>(rdg, r);
        xs[r] = r < kg ? xr : 0.f;
        if (l == r)
            xown = xs[r];
    }
    // output row of this signal
    if (!lead)
        return;
    const int io = (valid && a.rowmap) ? a.rowmap[i] : i;
    if (valid && l < s) {
        const bool on = l < kg;
        a.idx[(size_t)io * s + l] = on ? selj : -1;
        a.val[(size_t)io * s + l] = on ? xown : 0.f;
    }
    // residual e = y - D_I x with the dictionary used for coding; slots past
    // kg hold atom 0 with a zero coefficient, so the row loads need no
    // per-lane branch and are in flight together
    if (a.E || a.rnorm) {
        int js[SMAX];  // selected atoms; atom 0 past kg
#pragma unroll
        for (int t = 0; t < SMAX; ++t) {
            const int jt = f_bits(group_bcast_at<LPS>(bits_f(selj), t));
            js[t] = jt < 0 ? 0 : jt;
        }
        float esq = 0.f;
        if (valid)
            for (int q = 4 * l; q < p; q += 4 * LPS) {
                f32x4 e = *reinterpret_cast<const f32x4 *>(a.Y + (size_t)i * p + q);
                f32x4 d[SMAX];
#pragma unroll
                for (int t = 0; t < SMAX; ++t)
                    if (t < s)
                        d[t] = *reinterpret_cast<const f32x4 *>(a.D + (size_t)js[t] * p + q);
#pragma unroll
                for (int t = 0; t < SMAX; ++t)
                    if (t < s)
                        e -= d[t] * xs[t];
                if (a.E)
                    *reinterpret_cast<f32x4 *>(a.E + (size_t)io * p + q) = e;
                esq += e[0] * e[0] + e[1] * e[1] + e[2] * e[2] + e[3] * e[3];
            }
        esq = group_sum<LPS>(esq);
        if (a.rnorm && valid && l == 0)
            a.rnorm[io] = sqrtf(esq);
    }
}

// Small sparsity bounds ask for three waves per SIMD (a few dwords spill;
// measured faster than two waves without spills).
// The err_blocks workgroups after the coding ones carry the partial pass of
// the previous iteration's refreshing error (its X and E are not the ones
// this coding writes); they start as coding workgroups retire, so they fill
// the launch's last, partly occupied round.
template <int LPS, int NPL, int SMAX>
__global__ __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(SMAX <= 6 ? 3 : 1)))
void omp_kernel(OmpArgs a, RmseArgs err, int omp_blocks, int err_blocks)
{
    if ((int)blockIdx.x >= omp_blocks) {
        rmse_refresh_body(err, (int)blockIdx.x - omp_blocks, err_blocks);
        return;
    }
    constexpr int GPW = 64 / LPS;
    const int m_eff = a.m_dev ? min(*a.m_dev, a.m) : a.m;
    const int wave_sig0 = (blockIdx.x * kWaves + (int)(threadIdx.x >> 6)) * GPW;
    if (wave_sig0 >= m_eff)
        return;  // whole wave leaves together; no workgroup barrier follows
    omp_signals<LPS, NPL, SMAX>(a, wave_sig0, m_eff);
}

// One signal per two-wave workgroup (WPS = 2 above).  At n = 1024, s = 12 a
// wave of the one-wave shape needs 11 u-vectors of 16 values per lane (256
// VGPRs + AGPRs: one wave per SIMD); split over two waves it fits two per
// SIMD without spills (measured: 1.58 -> 1.33 ms per coding pass at m =
// 65536; forcing three per SIMD spills and was slower).
template <int NPL, int SMAX>
__global__ __launch_bounds__(128) void omp_pair_kernel(OmpArgs a)
{
    const int m_eff = a.m_dev ? min(*a.m_dev, a.m) : a.m;
    if ((int)blockIdx.x >= m_eff)
        return;  // both waves leave together
    omp_signals<64, NPL, SMAX, 2>(a, (int)blockIdx.x, m_eff);
}

// Batched problems of one launch shape: every wave takes tickets from the
// queue until none are left; a ticket is `per_ticket` consecutive items of
// the launch's item list (an item is GPW signals of one problem), so the
// one counter sees a few atomics per wave rather than one per item (with
// hundreds of thousands of small items the atomics on one address serialise).
template <int LPS, int NPL, int SMAX>
__global__ __launch_bounds__(64 * kWaves) void omp_batched_kernel(const OmpArgs *__restrict__ tab,
                                                                  BatchList bl, int per_ticket)
{
    constexpr int GPW = 64 / LPS;
    const int lane = threadIdx.x & 63;
    const int total = bl.start[bl.count];
    for (;;) {
        int tk = 0;
        if (lane == 0)
            tk = (int)atomicAdd(&bl.q->ticket, 1u);
        tk = __builtin_amdgcn_readfirstlane(tk);  // lane 0's ticket, wave-uniform
        const long long first = (long long)tk * per_ticket;
        if (first >= total)
            break;
        const int end = (int)min((long long)total, first + per_ticket);
        // consecutive items mostly belong to one problem: its index, item range
        // and arguments are looked up again only when an item leaves that range
        int b = batch_find(bl.start, bl.count, (int)first);
        int b0 = bl.start[b], b1 = bl.start[b + 1];
        OmpArgs a = tab[b];
        for (int it = (int)first; it < end; ++it) {
            if (it >= b1) {
                b = batch_find(bl.start, bl.count, it);
                b0 = bl.start[b];
                b1 = bl.start[b + 1];
                a = tab[b];
            }
            omp_signals<LPS, NPL, SMAX>(a, (it - b0) * GPW, a.m);
        }
    }
    if (lane == 0)
        batch_leave(bl.q, gridDim.x * kWaves);
}

template <int LPS, int NPL, int SMAX>
hipError_t launch_omp_batched_t(const OmpArgs *tab, const BatchList &bl, int items,
                                hipStream_t st)
{
    const int wg = batch_workers((const void *)omp_batched_kernel<LPS, NPL, SMAX>, 64 * kWaves, 0,
                                 (items + kWaves - 1) / kWaves);
    // about 16 tickets per wave, at most 8 items each
    const long long waves = (long long)wg * kWaves;
    int per = (int)(items / (16 * waves));
    per = per < 1 ? 1 : (per > 8 ? 8 : per);
    prof_begin(DL_K_OMP, st);
    hipLaunchKernelGGL((omp_batched_kernel<LPS, NPL, SMAX>), dim3(wg), dim3(64 * kWaves), 0, st,
                       tab, bl, per);
    prof_end(DL_K_OMP, st);
    return hipGetLastError();
}

template <int LPS, int NPL, int SMAX>
hipError_t launch_omp_t(const OmpArgs &a, hipStream_t st, const RmseArgs *err)
{
    constexpr int sig_per_block = kWaves * (64 / LPS);
    const int blocks = (a.m + sig_per_block - 1) / sig_per_block;
    const int eb = err ? rmse_blocks_dev(err->m) : 0;
    prof_begin(DL_K_OMP, st);
    hipLaunchKernelGGL((omp_kernel<LPS, NPL, SMAX>), dim3(blocks + eb), dim3(64 * kWaves), 0, st,
                       a, err ? *err : RmseArgs{}, blocks, eb);
    prof_end(DL_K_OMP, st);
    return hipGetLastError();
}

template <int NPL, int SMAX>
hipError_t launch_omp_pair_t(const OmpArgs &a, hipStream_t st)
{
    prof_begin(DL_K_OMP, st);
    hipLaunchKernelGGL((omp_pair_kernel<NPL, SMAX>), dim3(a.m), dim3(128), 0, st, a);
    prof_end(DL_K_OMP, st);
    return hipGetLastError();
}

// Two waves per signal (lanes_per_signal = 128), for sparsity bounds above 6.
template <int NPL>
hipError_t launch_omp_pair_s(const OmpArgs &a, hipStream_t st)
{
    if (a.s <= 8)
        return launch_omp_pair_t<NPL, 8>(a, st);
    if (a.s <= 12)
        return launch_omp_pair_t<NPL, 12>(a, st);
    return launch_omp_pair_t<NPL, 16>(a, st);
}

template <int LPS, int NPL>
hipError_t launch_omp_batched_s(const OmpArgs *tab, const BatchList &bl, int items, int smax,
                                hipStream_t st)
{
    if (smax == 4)
        return launch_omp_batched_t<LPS, NPL, 4>(tab, bl, items, st);
    if constexpr (LPS >= 8) {
        if (smax == 6)
            return launch_omp_batched_t<LPS, NPL, 6>(tab, bl, items, st);
        if (smax == 8)
            return launch_omp_batched_t<LPS, NPL, 8>(tab, bl, items, st);
    }
    if constexpr (LPS >= 16) {
        if (smax == 12)
            return launch_omp_batched_t<LPS, NPL, 12>(tab, bl, items, st);
        if (smax == 16)
            return launch_omp_batched_t<LPS, NPL, 16>(tab, bl, items, st);
    }
    return hipErrorInvalidValue;
}

// Dispatch over SMAX for one (LPS, NPL); configurations with LPS < SMAX are
// never requested (omp_config_ok rejects them).
template <int LPS, int NPL>
hipError_t launch_omp_s(const OmpArgs &a, hipStream_t st, const RmseArgs *err)
{
    if (a.s <= 4)
        return launch_omp_t<LPS, NPL, 4>(a, st, err);
    if constexpr (LPS >= 8) {
        if (a.s <= 6)
            return launch_omp_t<LPS, NPL, 6>(a, st, err);
        if (a.s <= 8)
            return launch_omp_t<LPS, NPL, 8>(a, st, err);
    }
    if constexpr (LPS >= 16) {
        if (a.s <= 12)
            return launch_omp_t<LPS, NPL, 12>(a, st, err);
        return launch_omp_t<LPS, NPL, 16>(a, st, err);
    }
    return hipErrorInvalidValue;
}

}  // namespace omp_detail

hipError_t launch_omp_npl4(const OmpArgs &a, int lps, hipStream_t st, const RmseArgs *err);
hipError_t launch_omp_npl8(const OmpArgs &a, int lps, hipStream_t st, const RmseArgs *err);
hipError_t launch_omp_npl16(const OmpArgs &a, int lps, hipStream_t st, const RmseArgs *err);
hipError_t launch_omp_batched_npl4(const OmpArgs *tab, const BatchList &bl, int items, int lps,
                                   int smax, hipStream_t st);
hipError_t launch_omp_batched_npl8(const OmpArgs *tab, const BatchList &bl, int items, int lps,
                                   int smax, hipStream_t st);
hipError_t launch_omp_batched_npl16(const OmpArgs *tab, const BatchList &bl, int items, int lps,
                                    int smax, hipStream_t st);

}  // namespace dlk
