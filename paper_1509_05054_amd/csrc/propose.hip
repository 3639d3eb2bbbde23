// Learned support proposal, per signal: the 2s candidate atoms with the
// largest logits, least squares restricted to them, backward elimination to
// s atoms, and the fallback test against the reference OMP residual.
#include "dl_internal.h"

namespace dlk {
namespace {

template <int CTRL>
__device__ inline int dpp(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

__device__ inline void take_better(float &v, int &ix, float ov, int oi)
{
    if (ov > v || (ov == v && oi < ix)) {
        v = ov;
        ix = oi;
    }
}

template <int LPS>
__device__ inline void group_argmax(float &v, int &ix)
{
    if constexpr (LPS >= 2)
        take_better(v, ix, __int_as_float(dpp<0xB1>(__float_as_int(v))), dpp<0xB1>(ix));
    if constexpr (LPS >= 4)
        take_better(v, ix, __int_as_float(dpp<0x4E>(__float_as_int(v))), dpp<0x4E>(ix));
    if constexpr (LPS >= 8)
        take_better(v, ix, __int_as_float(dpp<0x141>(__float_as_int(v))), dpp<0x141>(ix));
    if constexpr (LPS >= 16)
        take_better(v, ix, __int_as_float(dpp<0x140>(__float_as_int(v))), dpp<0x140>(ix));
    if constexpr (LPS >= 32)
        take_better(v, ix, __shfl_xor(v, 16), __shfl_xor(ix, 16));
    if constexpr (LPS >= 64)
        take_better(v, ix, __shfl_xor(v, 32), __shfl_xor(ix, 32));
}

// k rounds of a masked group argmax; a group of LPS lanes holds one row,
// 16 consecutive entries per lane.
template <int LPS>
__global__ __launch_bounds__(256) void topk_kernel(const float *__restrict__ Z, int rows, int cols,
                                                   int k, int32_t *__restrict__ out)
{
    constexpr int NPL = 16;
    const int lane = threadIdx.x & 63;
    const int l = lane % LPS;
    const int row = (blockIdx.x * 256 + threadIdx.x) / LPS;
    const int wave_row0 = (blockIdx.x * 256 + (threadIdx.x & ~63)) / LPS;
    if (wave_row0 >= rows)
        return;  // whole wave
    const bool valid = row < rows;
    float v[NPL];
    unsigned taken = 0;
#pragma unroll
    for (int c = 0; c < NPL; ++c) {
        const int col = l * NPL + c;
        const bool on = valid && col < cols;
        v[c] = on ? Z[(size_t)row * cols + col] : 0.f;
        if (!on || !(v[c] == v[c]))
            taken |= 1u << c;  // outside the row, or NaN: never chosen
    }
    for (int t = 0; t < k; ++t) {
        float best = -INFINITY;
        int bidx = 0x7fffffff;
#pragma unroll
        for (int c = 0; c < NPL; ++c)
            if (!((taken >> c) & 1u) && (v[c] > best || bidx == 0x7fffffff)) {
                best = v[c];
                bidx = l * NPL + c;
            }
        group_argmax<LPS>(best, bidx);
        if (valid && l == 0)
            out[(size_t)row * k + t] = bidx < cols ? bidx : -1;
        if (bidx / NPL == l && bidx < cols)
            taken |= 1u << (bidx % NPL);
    }
}

}  // namespace

hipError_t launch_topk(const float *logits, int rows, int cols, int k, int32_t *out, hipStream_t st)
{
    int lps = 4;
    while (lps * 16 < cols)
        lps <<= 1;
    const int rows_per_block = 256 / lps;
    const dim3 grid((rows + rows_per_block - 1) / rows_per_block);
    prof_begin(DL_K_PROPOSE, st);
    switch (lps) {
    case 4: hipLaunchKernelGGL(topk_kernel<4>, grid, dim3(256), 0, st, logits, rows, cols, k, out); break;
    case 8: hipLaunchKernelGGL(topk_kernel<8>, grid, dim3(256), 0, st, logits, rows, cols, k, out); break;
    case 16: hipLaunchKernelGGL(topk_kernel<16>, grid, dim3(256), 0, st, logits, rows, cols, k, out); break;
    case 32: hipLaunchKernelGGL(topk_kernel<32>, grid, dim3(256), 0, st, logits, rows, cols, k, out); break;
    default: hipLaunchKernelGGL(topk_kernel<64>, grid, dim3(256), 0, st, logits, rows, cols, k, out); break;
    }
    prof_end(DL_K_PROPOSE, st);
    return hipGetLastError();
}

}  // namespace dlk

namespace dlk {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Lower-triangle storage index of entry (r, q), r >= q.
__host__ __device__ constexpr int tri(int r, int q) { return r * (r + 1) / 2 + q; }

// Cholesky factor of the masked K2 x K2 matrix (entries of dead atoms replaced
// by those of the identity), with reciprocal diagonals; ok becomes false on a
// non-positive pivot (that pivot is then taken as 1).
template <int K2>
__device__ inline void masked_cholesky(const float *Gc, const bool *alive, float *L, float *rd,
                                       bool &ok)
{
#pragma unroll
    for (int r = 0; r < K2; ++r)
#pragma unroll
        for (int q = 0; q <= r; ++q) {
            float acc = (alive[r] && alive[q]) ? Gc[tri(r, q)] : (r == q ? 1.f : 0.f);
#pragma unroll
            for (int t = 0; t < q; ++t)
                acc -= L[tri(r, t)] * L[tri(q, t)];
            if (r == q) {
                if (!(acc > 0.f)) {
                    ok = false;
                    acc = 1.f;
                }
                // hardware square root and reciprocal (1 ulp): the pruning's
                // decisions are checked for validity, not bit for bit
                L[tri(r, r)] = __builtin_amdgcn_sqrtf(acc);
                rd[r] = __builtin_amdgcn_rcpf(L[tri(r, r)]);
            } else {
                L[tri(r, q)] = acc * rd[q];
            }
        }
}

// Sum over the groups of LPU consecutive lanes (every lane gets its group's
// sum): DPP moves inside rows of 16 lanes, shuffles across rows.
template <int LPU>
__device__ inline float lane_group_sum(float v)
{
    if constexpr (LPU >= 2)
        v += __int_as_float(dpp<0xB1>(__float_as_int(v)));   // lane ^ 1
    if constexpr (LPU >= 4)
        v += __int_as_float(dpp<0x4E>(__float_as_int(v)));   // lane ^ 2
    if constexpr (LPU >= 8)
        v += __int_as_float(dpp<0x141>(__float_as_int(v)));  // half-row mirror
    if constexpr (LPU >= 16)
        v += __int_as_float(dpp<0x140>(__float_as_int(v)));  // row mirror
    if constexpr (LPU >= 32)
        v += __shfl_xor(v, 16);
    if constexpr (LPU >= 64)
        v += __shfl_xor(v, 32);
    return v;
}

// The learned coding, a block of kPruneBlock signals at a time per
// workgroup (persistent over the blocks), in three phases:
//  1. (LPU lanes per signal, one float4 of the signal per lane, so the loads
//     of y and of the candidate atoms are whole row segments) the
//     correlations b_t = d_{c_t}^T y of the K2 candidates, to LDS.  When the
//     dictionary fits (n p <= kPruneLdsFloats) it is staged in LDS once per
//     workgroup, and the candidate rows of phases 1 and 3 are read from there:
//     every signal reads K2 rows, which from L2 would be 3 KB per signal;
//  2. (one thread per signal) least squares on the candidates and backward
//     elimination to s atoms: drop the atom with the smallest
//     c_j^2 / [(G_C)^{-1}]_jj (ties: lower atom index) until s remain.  The
//     inverse W = (G_C)^{-1} is formed once from the Cholesky factor of the
//     Gram entries G_C; each removal of atom j then updates it and the
//     solution in O(K2^2):
//         W <- W - W e_j e_j^T W / W_jj,   c <- c - W e_j c_j / W_jj,
//     which are the inverse and the least-squares solution of the remaining
//     set (the removed row and column become zero), so the survivors'
//     coefficients are their least-squares solution without a refit.
//     Runtime indices select with masks, so no register array is indexed by
//     a run-time value;
//  3. (LPU lanes per signal again) the residual e = y - D_S x, written to E,
//     and the fallback test: the signal goes back to OMP when
//     ||e|| > (1 + margin) * rref.  A block's rejected signals are gathered
//     in LDS and take consecutive places of the fallback list with one
//     atomic per block (one per signal or per wave serialises on the single
//     counter when most signals fall back); the list order decides only
//     where OMP codes a signal, not its result.
constexpr int kPruneBlock = 512;        // signals per block (8 waves)
constexpr int kPruneLdsFloats = 16384;  // dictionaries up to 64 KB are staged in LDS
constexpr int kPruneSlots = 32;         // LDS floats per signal: b, then (atom, x) pairs
constexpr int RU = 4;                   // signals per lane group in flight in phases 1 and 3

template <int K2, int LPU, bool DLDS>
__global__ __launch_bounds__(kPruneBlock) __attribute__((amdgpu_waves_per_eu(2)))
void ls_prune_kernel(ProposeArgs a)
{
    static_assert(2 * K2 <= kPruneSlots, "LDS slots per signal");
    constexpr int NT = K2 * (K2 + 1) / 2;
    constexpr int GPW = 64 / LPU;          // signals per wave in phases 1 and 3
    constexpr int NW = kPruneBlock / 64;   // waves per workgroup
    __shared__ float sD[DLDS ? kPruneLdsFloats : 1];
    __shared__ float sBX[kPruneBlock * kPruneSlots];
    __shared__ int sOk[kPruneBlock];
    __shared__ int sFb[kPruneBlock];
    __shared__ int sFbCount, sFbBase;
    const int p = a.p, s = a.s, n = a.n, ldn = a.ldn;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (DLDS) {
        for (int e = 4 * tid; e < n * p; e += 4 * kPruneBlock)
            *reinterpret_cast<f32x4 *>(sD + e) = *reinterpret_cast<const f32x4 *>(a.D + e);
    }
    const float *Dr = DLDS ? sD : a.D;  // rows of the dictionary for phases 1 and 3
    const int g = lane / LPU, l = lane % LPU, q = 4 * l;
    const f32x4 zero = f32x4{0.f, 0.f, 0.f, 0.f};
    const int nblocks = (a.m + kPruneBlock - 1) / kPruneBlock;
    for (int blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {
        const int i0 = blk * kPruneBlock;
        const int nsig = min(kPruneBlock, a.m - i0);
        if (tid == 0)
            sFbCount = 0;
        __syncthreads();  // the dictionary is staged; the previous block is done

        // ---- phase 1: candidate correlations (RU signals per lane group at
        // a time, so that their loads of y are in flight together)
        for (int il0 = wave * GPW; il0 < kPruneBlock; il0 += NW * GPW * RU) {
            f32x4 y[RU];
            int cc[RU][K2];
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                const int il = il0 + u * NW * GPW + g;
                const bool on = il < nsig;
                y[u] = (on && q < p)
                           ? *reinterpret_cast<const f32x4 *>(a.Y + (size_t)(i0 + il) * p + q)
                           : zero;
#pragma unroll
                for (int t = 0; t < K2; ++t) {
                    const int c = on ? a.cand[(size_t)(i0 + il) * K2 + t] : -1;
                    cc[u][t] = (c >= 0 && c < n) ? c : -1;
                }
            }
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                const int il = il0 + u * NW * GPW + g;
                float part[K2];
#pragma unroll
                for (int t = 0; t < K2; ++t) {
                    const int c = cc[u][t];
                    const f32x4 d = (c >= 0 && q < p)
                                        ? *reinterpret_cast<const f32x4 *>(Dr + (size_t)c * p + q)
                                        : zero;
                    part[t] = d[0] * y[u][0] + d[1] * y[u][1] + d[2] * y[u][2] + d[3] * y[u][3];
                }
#pragma unroll
                for (int t = 0; t < K2; ++t)
                    part[t] = lane_group_sum<LPU>(part[t]);
                if (il < nsig && l == 0)
#pragma unroll
                    for (int t = 0; t < K2; ++t)
                        sBX[il * kPruneSlots + t] = part[t];
            }
        }
        __syncthreads();

        // ---- phase 2: least squares and backward elimination, one thread per signal
        if (tid < nsig) {
            const int i = i0 + tid;
            int c[K2];
            bool alive[K2];
            float b[K2];
#pragma unroll
            for (int t = 0; t < K2; ++t) {
                c[t] = a.cand[(size_t)i * K2 + t];
                alive[t] = c[t] >= 0 && c[t] < n;
                if (!alive[t])
                    c[t] = 0;
                b[t] = alive[t] ? sBX[tid * kPruneSlots + t] : 0.f;
            }
            float Gc[NT];
#pragma unroll
            for (int r = 0; r < K2; ++r)
#pragma unroll
                for (int qq = 0; qq <= r; ++qq)
                    Gc[tri(r, qq)] = c[r] == c[qq] ? a.Gdiag[c[r]]  // G holds NaN there
                                                   : a.G[(size_t)c[r] * ldn + c[qq]];
            int kept = 0;
#pragma unroll
            for (int t = 0; t < K2; ++t)
                kept += alive[t] ? 1 : 0;
            bool ok = true;
            float x[K2];
            float W[NT];
            {
                // W = L^{-T} L^{-1}: first M = L^{-1} (lower), then W_rq = sum_t M_tr M_tq
                float L[NT], rd[K2];
                masked_cholesky<K2>(Gc, alive, L, rd, ok);
                float Mi[NT];
#pragma unroll
                for (int qq = 0; qq < K2; ++qq) {
                    Mi[tri(qq, qq)] = rd[qq];
#pragma unroll
                    for (int r = qq + 1; r < K2; ++r) {
                        float acc = 0.f;
#pragma unroll
                        for (int t = qq; t < r; ++t)
                            acc += L[tri(r, t)] * Mi[tri(t, qq)];
                        Mi[tri(r, qq)] = -acc * rd[r];
                    }
                }
#pragma unroll
                for (int r = 0; r < K2; ++r)
#pragma unroll
                    for (int qq = 0; qq <= r; ++qq) {
                        float acc = 0.f;
#pragma unroll
                        for (int t = r; t < K2; ++t)
                            acc += Mi[tri(t, r)] * Mi[tri(t, qq)];
                        W[tri(r, qq)] = acc;
                    }
            }
#pragma unroll
            for (int r = 0; r < K2; ++r) {
                float acc = 0.f;
#pragma unroll
                for (int qq = 0; qq < K2; ++qq)
                    acc += W[r >= qq ? tri(r, qq) : tri(qq, r)] * b[qq];
                x[r] = acc;
            }
            while (kept > s) {
                // the removal that raises the residual least
                float best = INFINITY;
                int batom = 0x7fffffff;
#pragma unroll
                for (int j = 0; j < K2; ++j) {
                    const float cost = x[j] * x[j] * __builtin_amdgcn_rcpf(W[tri(j, j)]);
                    const bool better =
                        alive[j] & ((cost < best) | ((cost == best) & (c[j] < batom)));
                    best = better ? cost : best;
                    batom = better ? c[j] : batom;
                }
                bool oh[K2];
                float wjj = 1.f, xj = 0.f;
#pragma unroll
                for (int j = 0; j < K2; ++j) {
                    oh[j] = alive[j] && c[j] == batom;
                    wjj = oh[j] ? W[tri(j, j)] : wjj;
                    xj = oh[j] ? x[j] : xj;
                }
                // column j of W (by mask), then the rank-one downdate
                float col[K2];
#pragma unroll
                for (int r = 0; r < K2; ++r) {
                    float v = 0.f;
#pragma unroll
                    for (int j = 0; j < K2; ++j)
                        v = oh[j] ? W[r >= j ? tri(r, j) : tri(j, r)] : v;
                    col[r] = v;
                }
                const float inv = __builtin_amdgcn_rcpf(wjj);
                const float f = xj * inv;
#pragma unroll
                for (int r = 0; r < K2; ++r) {
                    x[r] -= col[r] * f;
                    const float cr = col[r] * inv;
#pragma unroll
                    for (int qq = 0; qq <= r; ++qq)
                        W[tri(r, qq)] -= cr * col[qq];
                }
#pragma unroll
                for (int j = 0; j < K2; ++j)
                    alive[j] = alive[j] && !oh[j];
                --kept;
            }
            // outputs in candidate order; the survivors' (atom, coefficient)
            // pairs also go to this signal's LDS slots for phase 3
            float *mine = sBX + tid * kPruneSlots;
            int slot = 0;
#pragma unroll
            for (int t = 0; t < K2; ++t)
                if (alive[t] && slot < s) {
                    a.idx[(size_t)i * s + slot] = c[t];
                    a.val[(size_t)i * s + slot] = x[t];
                    mine[2 * slot] = __int_as_float(c[t]);
                    mine[2 * slot + 1] = x[t];
                    ++slot;
                }
            for (int t = slot; t < s; ++t) {
                a.idx[(size_t)i * s + t] = -1;
                a.val[(size_t)i * s + t] = 0.f;
                mine[2 * t] = __int_as_float(0);
                mine[2 * t + 1] = 0.f;
            }
            sOk[tid] = ok ? 1 : 0;
        }
        __syncthreads();

        // ---- phase 3: residual rows and the fallback test (RU signals per
        // lane group at a time)
        for (int il0 = wave * GPW; il0 < kPruneBlock; il0 += NW * GPW * RU) {
            f32x4 e[RU];
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                const int il = il0 + u * NW * GPW + g;
                const bool on = il < nsig;
                e[u] = (on && q < p)
                           ? *reinterpret_cast<const f32x4 *>(a.Y + (size_t)(i0 + il) * p + q)
                           : zero;
            }
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                const int il = il0 + u * NW * GPW + g;
                const bool on = il < nsig;
                const int i = i0 + (on ? il : 0);
                const float *mine = sBX + (on ? il : 0) * kPruneSlots;
                for (int t = 0; t < s; ++t) {
                    const int c = on ? __float_as_int(mine[2 * t]) : 0;
                    const float xv = on ? mine[2 * t + 1] : 0.f;
                    if (q < p)
                        e[u] -= *reinterpret_cast<const f32x4 *>(Dr + (size_t)c * p + q) * xv;
                }
                if (on && q < p)
                    *reinterpret_cast<f32x4 *>(a.E + (size_t)i * p + q) = e[u];
                const float enorm = sqrtf(lane_group_sum<LPU>(
                    e[u][0] * e[u][0] + e[u][1] * e[u][1] + e[u][2] * e[u][2] + e[u][3] * e[u][3]));
                if (on && l == 0 && (!sOk[il] || !(enorm <= (1.f + a.margin) * a.rref[i])))
                    sFb[atomicAdd(&sFbCount, 1)] = i;
            }
        }
        __syncthreads();
        const int cnt = sFbCount;
        if (tid == 0 && cnt > 0) {
            sFbBase = atomicAdd(a.fb_count, cnt);
            atomicAdd(&a.ctl->fallbacks, (unsigned long long)cnt);
        }
        __syncthreads();
        for (int k = tid; k < cnt; k += kPruneBlock)
            a.fb_list[sFbBase + k] = sFb[k];
    }
}

// rows[k] = src[list[k]] for k < *count (p floats per row)
__global__ void gather_list_kernel(const float *__restrict__ src, int p,
                                   const int32_t *__restrict__ list,
                                   const int32_t *__restrict__ count, int cap,
                                   float *__restrict__ rows)
{
    const int nrows = min(*count, cap);
    const size_t total = (size_t)nrows * (p / 4);
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(e / (p / 4)), q = 4 * (int)(e % (p / 4));
        *reinterpret_cast<f32x4 *>(rows + (size_t)k * p + q) =
            *reinterpret_cast<const f32x4 *>(src + (size_t)list[k] * p + q);
    }
}

}  // namespace

template <int K2, bool DLDS>
hipError_t launch_ls_prune_k(const ProposeArgs &a, hipStream_t st)
{
    int lpu = 1;
    while (4 * lpu < a.p)
        lpu <<= 1;
    const int blocks = (a.m + kPruneBlock - 1) / kPruneBlock;
    const void *kern;
    switch (lpu) {
    case 1:
    case 2:
    case 4: kern = (const void *)ls_prune_kernel<K2, 4, DLDS>; break;
    case 8: kern = (const void *)ls_prune_kernel<K2, 8, DLDS>; break;
    case 16: kern = (const void *)ls_prune_kernel<K2, 16, DLDS>; break;
    case 32: kern = (const void *)ls_prune_kernel<K2, 32, DLDS>; break;
    default: kern = (const void *)ls_prune_kernel<K2, 64, DLDS>; break;
    }
    // persistent workgroups: each stages the dictionary once and then codes
    // block after block
    const dim3 grid(batch_workers(kern, kPruneBlock, 0, blocks));
    switch (lpu) {
    case 1:
    case 2:
    case 4: hipLaunchKernelGGL((ls_prune_kernel<K2, 4, DLDS>), grid, dim3(kPruneBlock), 0, st, a); break;
    case 8: hipLaunchKernelGGL((ls_prune_kernel<K2, 8, DLDS>), grid, dim3(kPruneBlock), 0, st, a); break;
    case 16: hipLaunchKernelGGL((ls_prune_kernel<K2, 16, DLDS>), grid, dim3(kPruneBlock), 0, st, a); break;
    case 32: hipLaunchKernelGGL((ls_prune_kernel<K2, 32, DLDS>), grid, dim3(kPruneBlock), 0, st, a); break;
    default: hipLaunchKernelGGL((ls_prune_kernel<K2, 64, DLDS>), grid, dim3(kPruneBlock), 0, st, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_ls_prune(const ProposeArgs &a, int k2, hipStream_t st)
{
    if ((k2 != 8 && k2 != 12 && k2 != 16) || a.s > k2 || a.p > 256 || a.p % 4 != 0)
        return hipErrorInvalidValue;
    const bool in_lds = (long long)a.n * a.p <= kPruneLdsFloats;
    prof_begin(DL_K_PROPOSE, st);
    hipError_t e;
    if (k2 == 8)
        e = in_lds ? launch_ls_prune_k<8, true>(a, st) : launch_ls_prune_k<8, false>(a, st);
    else if (k2 == 12)
        e = in_lds ? launch_ls_prune_k<12, true>(a, st) : launch_ls_prune_k<12, false>(a, st);
    else
        e = in_lds ? launch_ls_prune_k<16, true>(a, st) : launch_ls_prune_k<16, false>(a, st);
    prof_end(DL_K_PROPOSE, st);
    return e;
}

hipError_t launch_gather_list(const float *src, int p, const int32_t *list, const int32_t *count,
                              int cap, float *rows, hipStream_t st)
{
    size_t blocks = ((size_t)cap * (p / 4) + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    if (blocks < 1)
        blocks = 1;
    prof_begin(DL_K_PROPOSE, st);
    hipLaunchKernelGGL(gather_list_kernel, dim3((unsigned)blocks), dim3(256), 0, st, src, p, list,
                       count, cap, rows);
    prof_end(DL_K_PROPOSE, st);
    return hipGetLastError();
}

}  // namespace dlk
