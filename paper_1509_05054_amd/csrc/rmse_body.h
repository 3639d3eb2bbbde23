// Device bodies of the error ||Y - D X||_F^2 (FP64 reduction), shared by the
// error launches and by the launches that carry the error of the previous
// iteration alongside their own work (the products and the CSR scan).
#pragma once
#include "dl_internal.h"

namespace dlk {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline f32x4 load4(const float *base, int q, int p)
{
    if (q < p)
        return *reinterpret_cast<const f32x4 *>(base + q);
    return f32x4{0.f, 0.f, 0.f, 0.f};
}

// Lanes per user row: a power of two >= p/4, each lane owning a float4.
__device__ inline int lanes_per_user(int p)
{
    int l = 1;
    while (4 * l < p)
        l <<= 1;
    return l;
}

// Partials: one workgroup per block of kRmseSignals signals;
// the block's X rows are staged in LDS, each lane group forms residual rows 4
// coordinates per lane with its atom rows loaded four at a time (branch-free,
// so the loads are in flight together), squares are summed in FP64 and the
// block's sum is stored.  Final: one workgroup sums the block partials in
// block order.  The launch boundary orders the two, so no workgroup needs a
// device-scope fence (which writes the L2 back on a multi-XCD GPU).
// Workgroups of the partials launch: one per kRmseSignals signals, at most
// kRmseMaxBlocks (each then strides over several signal blocks), so the final
// one-workgroup sum stays short.
constexpr int kRmseMaxBlocks = 1024;
__host__ __device__ inline int rmse_blocks_dev(int m)
{
    const int b = (m + kRmseSignals - 1) / kRmseSignals;
    return b < kRmseMaxBlocks ? b : kRmseMaxBlocks;
}

// Sum over groups of lpu consecutive lanes (lpu a power of two, every lane
// gets its group's sum), in the association of the xor butterfly: inside a
// row of 16 lanes by DPP (xor 1 and xor 2 by quad permutes; the half-row and
// row mirrors then pair the same quads and the same half-rows as xor 4 and
// xor 8, and addition commutes, so every lane gets the same bits), across
// rows by shuffles.  All lanes of a group must be active.
template <int CTRL, int ROWS = 0xF>
__device__ inline float dpp_mov_f(float x)
{
    return __int_as_float(
        __builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROWS, 0xF, false));
}

__device__ inline float lanes_sum(float v, int lpu)
{
    if (lpu >= 2)
        v += dpp_mov_f<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    if (lpu >= 4)
        v += dpp_mov_f<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    if (lpu >= 8)
        v += dpp_mov_f<0x141>(v);  // row_half_mirror
    if (lpu >= 16)
        v += dpp_mov_f<0x140>(v);  // row_mirror
    for (int off = 16; off < lpu; off <<= 1)
        v = sum_xor(v, off);
    return v;
}

// Sum over the wave, the same in every lane: the row sums as in lanes_sum,
// then rows 0 + 1 into row 1 and 2 + 3 into row 3 by DPP row broadcasts, row
// 1 into row 3, and lane 63 read out, (r0 + r1) + (r2 + r3).  No LDS
// crossbar operation.
__device__ inline float wave_sum_f32(float v)
{
    v = lanes_sum(v, 16);
    v += dpp_mov_f<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_mov_f<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ inline double wave_sum_f64(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_xor(v, off);
    return v;
}

// Sum of v over the workgroup (256 threads), in a fixed order; every thread
// gets the result.
__device__ inline double block_sum_f64(double v, double *red4)
{
    v = wave_sum_f64(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0)
        red4[wave] = v;
    __syncthreads();
    return ((red4[0] + red4[1]) + red4[2]) + red4[3];
}

__device__ inline void rmse_body(const RmseArgs &a, int blk, int nblk)
{
    __shared__ double red4[4];
    __shared__ int sIdx[kRmseSignals * 16];
    __shared__ float sVal[kRmseSignals * 16];
    const int p = a.p, s = a.s, n = a.n;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lpu = lanes_per_user(p);
    const int upw = 64 / lpu;
    const int sub = lane / lpu;
    const int q = 4 * (lane % lpu);
    double acc = 0.0;
    const int nsb = (a.m + kRmseSignals - 1) / kRmseSignals;
    for (int sb = blk; sb < nsb; sb += nblk) {
        const int i0 = sb * kRmseSignals;
        const int nsig = min(kRmseSignals, a.m - i0);
        __syncthreads();  // the previous signal block's rows are no longer read
        for (int r = threadIdx.x; r < nsig * s; r += blockDim.x) {
            int j = a.idx[(size_t)i0 * s + r];
            float x = a.val[(size_t)i0 * s + r];
            if (j < 0 || j >= n) {
                j = 0;  // unused slot: row 0 with a zero coefficient
                x = 0.f;
            }
            sIdx[r] = j;
            sVal[r] = x;
        }
        __syncthreads();
        // a lane group's signals il0, il0 + G, il0 + 2G, ... (G groups in the
        // block) are formed together, so all their loads are in flight at once
        constexpr int RU = 4;
        const int G = 4 * upw;
        if (q < p) {
            for (int il0 = wave * upw + sub; il0 < nsig; il0 += G * RU) {
                f32x4 e[RU];
    #pragma unroll
                for (int u = 0; u < RU; ++u) {
                    const int il = il0 + u * G;
                    e[u] = il < nsig ? *reinterpret_cast<const f32x4 *>(a.Y + (size_t)(i0 + il) * p + q)
                                     : f32x4{0.f, 0.f, 0.f, 0.f};
                }
                for (int t0 = 0; t0 < s; t0 += 4) {
                    f32x4 d[RU][4];
                    float x[RU][4];
    #pragma unroll
                    for (int u = 0; u < RU; ++u) {
                        const int il = il0 + u * G < nsig ? il0 + u * G : il0;
    #pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int t = t0 + v < s ? t0 + v : t0;
                            x[u][v] = (t0 + v < s && il0 + u * G < nsig) ? sVal[il * s + t] : 0.f;
                            d[u][v] = *reinterpret_cast<const f32x4 *>(a.D + (size_t)sIdx[il * s + t] * p + q);
                        }
                    }
    #pragma unroll
                    for (int u = 0; u < RU; ++u)
    #pragma unroll
                        for (int v = 0; v < 4; ++v)
                            e[u] -= d[u][v] * x[u][v];
                }
    #pragma unroll
                for (int u = 0; u < RU; ++u)
    #pragma unroll
                    for (int r = 0; r < 4; ++r)
                        acc += (double)e[u][r] * (double)e[u][r];
            }
        }
    }
    const double tot_blk = block_sum_f64(acc, red4);
    if (threadIdx.x == 0)
        a.partial[blk] = tot_blk;
}

// The refreshed coefficients and residual rows of the RU signals [ilc[u]] of
// a lane group in a staged signal block (slots in sIdx/sVal/sCos, rows of y
// and of the coding residual e in ey/eo), their squares added to acc.
template <int RU>
__device__ inline void refresh_rows(const RmseArgs &a, int i0, const bool (&on)[RU],
                                    const int (&ilc)[RU], f32x4 (&ey)[RU], const f32x4 (&eo)[RU],
                                    const int *sIdx, const float *sVal, const float *sCos,
                                    int lpu, int q, int lane, double &acc)
{
    const int p = a.p, s = a.s;
    // TS slots at a time: all their atom rows are loaded before any is used,
    // so the loads are in flight together (the stores of x' between them
    // would otherwise order each slot's loads after the previous slot's
    // store)
    constexpr int TS = 4;
    for (int t0 = 0; t0 < s; t0 += TS) {
        f32x4 dn[RU][TS];
        float x[RU][TS], cj[RU][TS];
#pragma unroll
        for (int u = 0; u < RU; ++u)
#pragma unroll
            for (int v = 0; v < TS; ++v) {
                const int t = t0 + v < s ? t0 + v : t0;
                const int r = ilc[u] * s + t;
                const int j = sIdx[r];
                x[u][v] = on[u] ? sVal[r] : 0.f;
                cj[u][v] = on[u] ? sCos[r] : __builtin_nanf("");
                dn[u][v] = load4(a.D + (size_t)j * p, q, p);
            }
#pragma unroll
        for (int v = 0; v < TS; ++v) {
            if (t0 + v >= s)
                break;  // uniform over the workgroup
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                float part = eo[u][0] * dn[u][v][0] + eo[u][1] * dn[u][v][1] +
                             eo[u][2] * dn[u][v][2] + eo[u][3] * dn[u][v][3];
                part = lanes_sum(part, lpu);
                const bool keep = cj[u][v] != cj[u][v];  // NaN: kept
                const float xn = keep ? x[u][v] : part + x[u][v] * cj[u][v];
                if (on[u] && (lane % lpu) == 0)
                    a.valn[(size_t)(i0 + ilc[u]) * s + t0 + v] = xn;
                ey[u] -= dn[u][v] * xn;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < RU; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            acc += (double)ey[u][r] * (double)ey[u][r];
}

// The same partials with the coefficient refresh of the atom update (all
// atoms in one group): per slot, x' = (e + d x)^T d' formed as
// e^T d' + x (d^T d') with pass 2's operations and order (so the same bits;
// d^T d' is pass 2's per-atom atom_cos), stored to valn, and the residual row
// y - sum_t d'_t x'_t formed as above.  Two signals per lane group in flight
// (each slot needs its new atom row).  Every lane of a group runs the loop
// (zero rows past p), since x' is reduced over the group.
__device__ inline void rmse_refresh_body(const RmseArgs &a, int blk, int nblk)
{
    __shared__ double red4[4];
    __shared__ int sIdx[kRmseSignals * 16];
    __shared__ float sVal[kRmseSignals * 16];
    // per slot: d^T d' of an atom whose coefficient is refreshed, NaN for a
    // slot that keeps its coefficient (one array: the carrying launches'
    // LDS budgets count it)
    __shared__ float sCos[kRmseSignals * 16];
    const int p = a.p, s = a.s, n = a.n;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lpu = lanes_per_user(p);
    const int upw = 64 / lpu;
    const int sub = lane / lpu;
    const int q = 4 * (lane % lpu);
    const f32x4 zero = f32x4{0.f, 0.f, 0.f, 0.f};
    double acc = 0.0;
    const int nsb = (a.m + kRmseSignals - 1) / kRmseSignals;
    for (int sb = blk; sb < nsb; sb += nblk) {
        const int i0 = sb * kRmseSignals;
        const int nsig = min(kRmseSignals, a.m - i0);
        __syncthreads();  // the previous signal block's rows are no longer read
        for (int r = threadIdx.x; r < nsig * s; r += blockDim.x) {
            int j = a.idx[(size_t)i0 * s + r];
            float x = a.val_old[(size_t)i0 * s + r];
            float cj = __builtin_nanf("");
            if (j < 0 || j >= n) {
                j = 0;  // unused slot: row 0, coefficient 0 (kept)
                x = 0.f;
            } else if (a.rule == DL_RULE_AKSVD && a.atom_state[j] == 0) {
                cj = a.atom_cos[j];  // NaN only if d' is not finite: kept then
            }
            sIdx[r] = j;
            sVal[r] = x;
            sCos[r] = cj;
        }
        __syncthreads();
        constexpr int RU = 2;  // measured: 4 in flight was 6% slower at c2
        const int G = 4 * upw;
        for (int il0 = wave * upw + sub; il0 < nsig; il0 += G * RU) {
            f32x4 ey[RU], eo[RU];
            bool on[RU];
            int ilc[RU];
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                const int il = il0 + u * G;
                on[u] = il < nsig;
                ilc[u] = on[u] ? il : il0;
                ey[u] = on[u] ? load4(a.Y + (size_t)(i0 + il) * p, q, p) : zero;
                eo[u] = on[u] ? load4(a.E + (size_t)(i0 + il) * p, q, p) : zero;
            }
            refresh_rows<RU>(a, i0, on, ilc, ey, eo, sIdx, sVal, sCos, lpu, q, lane, acc);
        }
    }
    const double tot_blk = block_sum_f64(acc, red4);
    if (threadIdx.x == 0)
        a.partial[blk] = tot_blk;
}

// The refreshing partials of the error launch of its own, software
// pipelined over the signal blocks of a workgroup: the next block's slots
// and its rows of y and e are loaded while the current block is computed, and
// d^T d' of every atom comes from a table staged in LDS once, so a block
// waits on its atom rows only.  The arithmetic, the assignment of signals to
// lanes and the order of every sum are those of rmse_refresh_body (the same
// bits).  Requires p <= 64 (one pass of the lane groups covers a block) and
// n <= kRmseCosTab.
constexpr int kRmseCosTab = 2048;
__device__ inline void rmse_refresh_body_pf(const RmseArgs &a, int blk, int nblk)
{
    __shared__ double red4[4];
    __shared__ int sIdx[kRmseSignals * 16];
    __shared__ float sVal[kRmseSignals * 16];
    __shared__ float sCos[kRmseSignals * 16];
    __shared__ float sTab[kRmseCosTab];
    constexpr int RU = 2;
    constexpr int CPT = kRmseSignals * 16 / 256;  // staged slots per thread
    const int s = a.s, n = a.n, p = a.p;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lpu = lanes_per_user(p);
    const int upw = 64 / lpu;
    const int sub = lane / lpu;
    const int q = 4 * (lane % lpu);
    const int G = 4 * upw;
    const int il0 = wave * upw + sub;  // G * RU >= kRmseSignals: one pass per block
    const f32x4 zero = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int j = threadIdx.x; j < n; j += blockDim.x)
        sTab[j] = (a.rule == DL_RULE_AKSVD && a.atom_state[j] == 0) ? a.atom_cos[j]
                                                                     : __builtin_nanf("");
    double acc = 0.0;
    const int nsb = (a.m + kRmseSignals - 1) / kRmseSignals;
    int pj[CPT];
    float px[CPT];
    f32x4 py[RU], pe[RU];
    auto prefetch = [&](int sb) {
        const int i0 = sb * kRmseSignals;
        const int nsig = min(kRmseSignals, a.m - i0);
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int r = (int)threadIdx.x + 256 * c;
            pj[c] = -1;
            px[c] = 0.f;
            if (r < nsig * s) {
                pj[c] = a.idx[(size_t)i0 * s + r];
                px[c] = a.val_old[(size_t)i0 * s + r];
            }
        }
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int il = il0 + u * G;
            py[u] = il < nsig ? load4(a.Y + (size_t)(i0 + il) * p, q, p) : zero;
            pe[u] = il < nsig ? load4(a.E + (size_t)(i0 + il) * p, q, p) : zero;
        }
    };
    if (blk < nsb)
        prefetch(blk);
    for (int sb = blk; sb < nsb; sb += nblk) {
        const int i0 = sb * kRmseSignals;
        const int nsig = min(kRmseSignals, a.m - i0);
        __syncthreads();  // the previous block's slots are no longer read (and sTab is staged)
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int r = (int)threadIdx.x + 256 * c;
            if (r < nsig * s) {
                int j = pj[c];
                float x = px[c];
                float cj = __builtin_nanf("");
                if (j < 0 || j >= n) {
                    j = 0;  // unused slot: row 0, coefficient 0 (kept)
                    x = 0.f;
                } else {
                    cj = sTab[j];
                }
                sIdx[r] = j;
                sVal[r] = x;
                sCos[r] = cj;
            }
        }
        __syncthreads();
        f32x4 ey[RU], eo[RU];
        bool on[RU];
        int ilc[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int il = il0 + u * G;
            on[u] = il < nsig;
            ilc[u] = on[u] ? il : il0;
            ey[u] = py[u];
            eo[u] = pe[u];
        }
        if (sb + nblk < nsb)
            prefetch(sb + nblk);
        if (il0 < nsig)
            refresh_rows<RU>(a, i0, on, ilc, ey, eo, sIdx, sVal, sCos, lpu, q, lane, acc);
    }
    const double tot_blk = block_sum_f64(acc, red4);
    if (threadIdx.x == 0)
        a.partial[blk] = tot_blk;
}

// Sum of the nblk block partials in block order, and the error.
// The first 256 threads of the workgroup take part (a larger workgroup's
// other waves only pass the barriers), so the sum has the same bits in every
// launch that runs it.
__device__ inline void rmse_final_body(const RmseArgs &a, int nblk)
{
    __shared__ double red4[4];
    double v = 0.0;
    if (threadIdx.x < 256)
        for (int b = threadIdx.x; b < nblk; b += 256)
            v += a.partial[b];
    v = wave_sum_f64(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0 && threadIdx.x < 256)
        red4[threadIdx.x >> 6] = v;
    __syncthreads();
    const double tot = ((red4[0] + red4[1]) + red4[2]) + red4[3];
    if (threadIdx.x == 0) {
        a.out[0] = sqrt(tot / ((double)a.p * (double)a.m));
        if (!isfinite(tot))
            atomicAdd(&a.ctl->nonfinite, 1ull);
    }
}

}  // namespace
}  // namespace dlk
