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

// One thread per signal.  K2 candidates: correlations b = D_C^T y and Gram
// entries G_C from the atoms' Gram matrix; least squares on the candidates;
// backward elimination to s atoms: each round refits on the surviving set and
// drops the atom with the smallest c_j^2 / [(G_C)^{-1}]_jj (ties: lower atom
// index).  Eliminated atoms are masked (their rows and columns of G_C become
// those of the identity), so no array is ever indexed by a run-time value.
// The residual e = y - D_S x is formed explicitly; the signal goes back to
// OMP when ||e|| > (1 + margin) * rref.
template <int K2>
__global__ __launch_bounds__(256) void ls_prune_kernel(ProposeArgs a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.m)
        return;
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
    // Gram entries (lower triangle)
    float Gc[K2 * (K2 + 1) / 2];
#pragma unroll
    for (int r = 0; r < K2; ++r)
#pragma unroll
        for (int q = 0; q <= r; ++q)
            Gc[r * (r + 1) / 2 + q] = a.G[(size_t)c[r] * ldn + c[q]];

    int kept = 0;
#pragma unroll
    for (int t = 0; t < K2; ++t)
        kept += alive[t] ? 1 : 0;
    float x[K2];
    bool ok = true;
    for (int round = 0;; ++round) {
        // Cholesky of the masked G_C
        float L[K2 * (K2 + 1) / 2];
#pragma unroll
        for (int r = 0; r < K2; ++r)
#pragma unroll
            for (int q = 0; q <= r; ++q) {
                float acc = (alive[r] && alive[q]) ? Gc[r * (r + 1) / 2 + q] : (r == q ? 1.f : 0.f);
#pragma unroll
                for (int t = 0; t < q; ++t)
                    acc -= L[r * (r + 1) / 2 + t] * L[q * (q + 1) / 2 + t];
                if (r == q) {
                    if (!(acc > 0.f)) {
                        ok = false;
                        acc = 1.f;
                    }
                    L[r * (r + 1) / 2 + r] = sqrtf(acc);
                } else {
                    L[r * (r + 1) / 2 + q] = acc / L[q * (q + 1) / 2 + q];
                }
            }
        // x = G_C^{-1} b (masked entries of b are 0)
        float z[K2];
#pragma unroll
        for (int r = 0; r < K2; ++r) {
            float acc = alive[r] ? b[r] : 0.f;
#pragma unroll
            for (int t = 0; t < r; ++t)
                acc -= L[r * (r + 1) / 2 + t] * z[t];
            z[r] = acc / L[r * (r + 1) / 2 + r];
        }
#pragma unroll
        for (int r = K2 - 1; r >= 0; --r) {
            float acc = z[r];
#pragma unroll
            for (int t = r + 1; t < K2; ++t)
                acc -= L[t * (t + 1) / 2 + r] * x[t];
            x[r] = acc / L[r * (r + 1) / 2 + r];
        }
        if (kept <= s)
            break;
        // removal costs: [(G_C)^{-1}]_jj = || L^{-1} e_j ||^2
        float best = INFINITY;
        int bj = -1, batom = 0x7fffffff;
#pragma unroll
        for (int j = 0; j < K2; ++j) {
            float w[K2];
            float dj = 0.f;
#pragma unroll
            for (int r = j; r < K2; ++r) {
                float acc = r == j ? 1.f : 0.f;
#pragma unroll
                for (int t = j; t < r; ++t)
                    acc -= L[r * (r + 1) / 2 + t] * w[t];
                w[r] = acc / L[r * (r + 1) / 2 + r];
                dj += w[r] * w[r];
            }
            const float cost = x[j] * x[j] / dj;
            if (alive[j] && (cost < best || (cost == best && c[j] < batom))) {
                best = cost;
                bj = j;
                batom = c[j];
            }
        }
#pragma unroll
        for (int j = 0; j < K2; ++j)
            if (j == bj)
                alive[j] = false;
        --kept;
    }

    // explicit residual and the fallback test
    float enorm2 = 0.f;
    for (int q = 0; q < p; q += 4) {
        f32x4 e = *reinterpret_cast<const f32x4 *>(a.Y + (size_t)i * p + q);
#pragma unroll
        for (int t = 0; t < K2; ++t)
            if (alive[t])
                e -= *reinterpret_cast<const f32x4 *>(a.D + (size_t)c[t] * p + q) * x[t];
        *reinterpret_cast<f32x4 *>(a.E + (size_t)i * p + q) = e;
        enorm2 += e[0] * e[0] + e[1] * e[1] + e[2] * e[2] + e[3] * e[3];
    }
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
    const float enorm = sqrtf(enorm2);
    if (!ok || !(enorm <= (1.f + a.margin) * a.rref[i])) {
        const int pos = atomicAdd(a.fb_count, 1);
        a.fb_list[pos] = i;
        atomicAdd(&a.ctl->fallbacks, 1ull);
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
