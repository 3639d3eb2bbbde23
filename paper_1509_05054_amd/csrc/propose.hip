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
