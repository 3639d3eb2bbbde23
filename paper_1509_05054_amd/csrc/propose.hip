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
                L[tri(r, r)] = sqrtf(acc);
                rd[r] = 1.0f / L[tri(r, r)];
            } else {
                L[tri(r, q)] = acc * rd[q];
            }
        }
}

// One thread per signal.  K2 candidates: correlations b = D_C^T y and Gram
// entries G_C from the atoms' Gram matrix; least squares on the candidates;
// backward elimination to s atoms: drop the atom with the smallest
// c_j^2 / [(G_C)^{-1}]_jj (ties: lower atom index) until s remain.
// The inverse W = (G_C)^{-1} is formed once from the Cholesky factor; each
// removal of atom j then updates it and the solution in O(K2^2):
//     W <- W - W e_j e_j^T W / W_jj,   c <- c - W e_j c_j / W_jj,
// which are the inverse and the least-squares solution of the remaining set
// (the removed row and column become zero).  The survivors' coefficients are
// finally refitted by a fresh Cholesky solve.  Runtime indices select with
// masks, so no register array is indexed by a run-time value.  The residual
// e = y - D_S x is formed explicitly; the signal goes back to OMP when
// ||e|| > (1 + margin) * rref.
template <int K2>
__global__ __launch_bounds__(256) void ls_prune_kernel(ProposeArgs a)
{
    constexpr int NT = K2 * (K2 + 1) / 2;
    const int i0 = blockIdx.x * blockDim.x + threadIdx.x;
    if (blockIdx.x * blockDim.x + (threadIdx.x & ~63) >= a.m)
        return;  // the whole wave (the fallback list below is filled per wave)
    const bool valid = i0 < a.m;
    const int i = valid ? i0 : a.m - 1;  // lanes past the end redo the last signal, store nothing
    const int p = a.p, s = a.s, n = a.n, ldn = a.ldn;
    int c[K2];
    bool alive[K2];
#pragma unroll
    for (int t = 0; t < K2; ++t) {
        c[t] = a.cand[(size_t)i * K2 + t];
        alive[t] = c[t] >= 0 && c[t] < n;
        if (!alive[t])
            c[t] = 0;
    }
    // correlations with the candidates
    float b[K2];
#pragma unroll
    for (int t = 0; t < K2; ++t)
        b[t] = 0.f;
    for (int q = 0; q < p; q += 4) {
        const f32x4 y = *reinterpret_cast<const f32x4 *>(a.Y + (size_t)i * p + q);
#pragma unroll
        for (int t = 0; t < K2; ++t) {
            const f32x4 d = *reinterpret_cast<const f32x4 *>(a.D + (size_t)c[t] * p + q);
            b[t] += d[0] * y[0] + d[1] * y[1] + d[2] * y[2] + d[3] * y[3];
        }
    }
#pragma unroll
    for (int t = 0; t < K2; ++t)
        if (!alive[t])
            b[t] = 0.f;
    // Gram entries (lower triangle)
    float Gc[NT];
#pragma unroll
    for (int r = 0; r < K2; ++r)
#pragma unroll
        for (int q = 0; q <= r; ++q)
            Gc[tri(r, q)] = a.G[(size_t)c[r] * ldn + c[q]];

    int kept = 0;
#pragma unroll
    for (int t = 0; t < K2; ++t)
        kept += alive[t] ? 1 : 0;
    bool ok = true;
    float x[K2];
    if (kept > s) {
        // W = L^{-T} L^{-1}: first M = L^{-1} (lower), then W_rq = sum_t M_tr M_tq
        float L[NT], rd[K2];
        masked_cholesky<K2>(Gc, alive, L, rd, ok);
        float Mi[NT];
#pragma unroll
        for (int q = 0; q < K2; ++q) {
            Mi[tri(q, q)] = rd[q];
#pragma unroll
            for (int r = q + 1; r < K2; ++r) {
                float acc = 0.f;
#pragma unroll
                for (int t = q; t < r; ++t)
                    acc += L[tri(r, t)] * Mi[tri(t, q)];
                Mi[tri(r, q)] = -acc * rd[r];
            }
        }
        float W[NT];
#pragma unroll
        for (int r = 0; r < K2; ++r)
#pragma unroll
            for (int q = 0; q <= r; ++q) {
                float acc = 0.f;
#pragma unroll
                for (int t = r; t < K2; ++t)
                    acc += Mi[tri(t, r)] * Mi[tri(t, q)];
                W[tri(r, q)] = acc;
            }
#pragma unroll
        for (int r = 0; r < K2; ++r) {
            float acc = 0.f;
#pragma unroll
            for (int q = 0; q < K2; ++q)
                acc += W[r >= q ? tri(r, q) : tri(q, r)] * b[q];
            x[r] = acc;
        }
        while (kept > s) {
            // the removal that raises the residual least
            float best = INFINITY;
            int batom = 0x7fffffff;
            bool oh[K2];
#pragma unroll
            for (int j = 0; j < K2; ++j) {
                const float cost = x[j] * x[j] / W[tri(j, j)];
                const bool better = alive[j] && (cost < best || (cost == best && c[j] < batom));
                best = better ? cost : best;
                batom = better ? c[j] : batom;
            }
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
            const float inv = 1.0f / wjj;
            const float f = xj * inv;
#pragma unroll
            for (int r = 0; r < K2; ++r) {
                x[r] -= col[r] * f;
                const float cr = col[r] * inv;
#pragma unroll
                for (int q = 0; q <= r; ++q)
                    W[tri(r, q)] -= cr * col[q];
            }
#pragma unroll
            for (int j = 0; j < K2; ++j)
                alive[j] = alive[j] && !oh[j];
            --kept;
        }
    }
    {
        // least squares on the survivors: a fresh masked Cholesky solve
        float L[NT], rd[K2];
        masked_cholesky<K2>(Gc, alive, L, rd, ok);
        float z[K2];
#pragma unroll
        for (int r = 0; r < K2; ++r) {
            float acc = alive[r] ? b[r] : 0.f;
#pragma unroll
            for (int t = 0; t < r; ++t)
                acc -= L[tri(r, t)] * z[t];
            z[r] = acc * rd[r];
        }
#pragma unroll
        for (int r = K2 - 1; r >= 0; --r) {
            float acc = z[r];
#pragma unroll
            for (int t = r + 1; t < K2; ++t)
                acc -= L[tri(t, r)] * x[t];
            x[r] = acc * rd[r];
        }
    }

    // explicit residual and the fallback test
    float enorm2 = 0.f;
    for (int q = 0; q < p; q += 4) {
        f32x4 e = *reinterpret_cast<const f32x4 *>(a.Y + (size_t)i * p + q);
#pragma unroll
        for (int t = 0; t < K2; ++t)
            if (alive[t])
                e -= *reinterpret_cast<const f32x4 *>(a.D + (size_t)c[t] * p + q) * x[t];
        if (valid)
            *reinterpret_cast<f32x4 *>(a.E + (size_t)i * p + q) = e;
        enorm2 += e[0] * e[0] + e[1] * e[1] + e[2] * e[2] + e[3] * e[3];
    }
    if (valid) {
        int slot = 0;
#pragma unroll
        for (int t = 0; t < K2; ++t)
            if (alive[t] && slot < s) {
                a.idx[(size_t)i * s + slot] = c[t];
                a.val[(size_t)i * s + slot] = x[t];
                ++slot;
            }
        for (int t = slot; t < s; ++t) {
            a.idx[(size_t)i * s + t] = -1;
            a.val[(size_t)i * s + t] = 0.f;
        }
    }
    // The rejected signals of the wave take consecutive places of the
    // fallback list: one atomic per wave (a per-signal atomic on the one
    // counter serialises most of the launch when most signals fall back).
    // The list order only decides where OMP codes a signal, not its result.
    const float enorm = sqrtf(enorm2);
    const bool fb = valid && (!ok || !(enorm <= (1.f + a.margin) * a.rref[i]));
    const unsigned long long mask = __ballot(fb);
    const int lane = threadIdx.x & 63;
    const int cnt = __popcll(mask);
    int base = 0;
    if (lane == 0 && cnt > 0) {
        base = atomicAdd(a.fb_count, cnt);
        atomicAdd(&a.ctl->fallbacks, (unsigned long long)cnt);
    }
    base = __shfl(base, 0);
    if (fb)
        a.fb_list[base + __popcll(mask & ((1ull << lane) - 1ull))] = i;
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

hipError_t launch_ls_prune(const ProposeArgs &a, int k2, hipStream_t st)
{
    const dim3 grid((a.m + 255) / 256);
    prof_begin(DL_K_PROPOSE, st);
    if (k2 == 8)
        hipLaunchKernelGGL(ls_prune_kernel<8>, grid, dim3(256), 0, st, a);
    else if (k2 == 12)
        hipLaunchKernelGGL(ls_prune_kernel<12>, grid, dim3(256), 0, st, a);
    else if (k2 == 16)
        hipLaunchKernelGGL(ls_prune_kernel<16>, grid, dim3(256), 0, st, a);
    else {
        prof_end(DL_K_PROPOSE, st);
        return hipErrorInvalidValue;
    }
    prof_end(DL_K_PROPOSE, st);
    return hipGetLastError();
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
