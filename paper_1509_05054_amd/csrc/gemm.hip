// Dense products of the coding stage on the matrix cores (MFMA):
//   G  = D D^T   [n][n]  (Gram matrix of the atoms)
//   A0 = Y D^T   [m][n]  (correlations D^T y of every signal)
// Both are "NT" products C[M][N] = A[M][K] B[N][K]^T of row-major operands
// whose K dimension (the signal size p) is contiguous, so each lane loads
// short contiguous K-slices straight from global memory (the operands are
// small and L2-resident: D is at most 1 MiB) and no LDS staging is needed.
//
// MFMA layout used (16x16 output tile, wave64): lane l supplies row l%16 of
// the A-tile and column l%16 of the B-tile over a K-slice chosen by l/16, and
// receives C[4*(l/16) + r][l%16], r = 0..3.  Which K indices a lane group
// holds is irrelevant to the product as long as A and B use the same choice,
// so every lane loads 4 (FP32) or 8 (BF16) consecutive K values at once.
#include "dl_internal.h"

namespace dlk {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

constexpr int kWaveM = 32;  // rows of C per wave (2 MFMA tiles)
constexpr int kWaveN = 32;  // cols of C per wave (2 MFMA tiles)
constexpr int kBlockM = 64; // 2 x 2 waves per workgroup
constexpr int kBlockN = 64;

__device__ inline void store_tile(float *C, int M, int N, int row0, int col0, const f32x4 &acc,
                                  int lane)
{
    const int col = col0 + (lane & 15);
    const int rbase = row0 + 4 * (lane >> 4);
    if (col >= N)
        return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = rbase + r;
        if (row < M)
            C[(size_t)row * N + col] = acc[r];
    }
}

__global__ __launch_bounds__(256) void gemm_nt_f32_kernel(const float *__restrict__ A,
                                                          const float *__restrict__ B,
                                                          float *__restrict__ C, int M, int N,
                                                          int K)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int row0 = blockIdx.y * kBlockM + (wave >> 1) * kWaveM;
    const int col0 = blockIdx.x * kBlockN + (wave & 1) * kWaveN;
    const int r = lane & 15;
    const int kq = 4 * (lane >> 4);  // this lane's K offset inside a 16-wide K step

    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
            acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int arow[2] = {row0 + r, row0 + 16 + r};
    const int brow[2] = {col0 + r, col0 + 16 + r};

    for (int k0 = 0; k0 < K; k0 += 16) {
        const int k = k0 + kq;
        f32x4 av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            av[a] = f32x4{0.f, 0.f, 0.f, 0.f};
            if (arow[a] < M && k < K)
                av[a] = *reinterpret_cast<const f32x4 *>(A + (size_t)arow[a] * K + k);
            bv[a] = f32x4{0.f, 0.f, 0.f, 0.f};
            if (brow[a] < N && k < K)
                bv[a] = *reinterpret_cast<const f32x4 *>(B + (size_t)brow[a] * K + k);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a][q], bv[b][q],
                                                                      acc[a][b], 0, 0, 0);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
            store_tile(C, M, N, row0 + 16 * a, col0 + 16 * b, acc[a][b], lane);
}

__global__ __launch_bounds__(256) void gemm_nt_bf16_kernel(const uint16_t *__restrict__ A,
                                                           const uint16_t *__restrict__ B,
                                                           float *__restrict__ C, int M, int N,
                                                           int K)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int row0 = blockIdx.y * kBlockM + (wave >> 1) * kWaveM;
    const int col0 = blockIdx.x * kBlockN + (wave & 1) * kWaveN;
    const int r = lane & 15;
    const int kq = 8 * (lane >> 4);  // 8 consecutive K values per lane in a 32-wide K step

    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
            acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int arow[2] = {row0 + r, row0 + 16 + r};
    const int brow[2] = {col0 + r, col0 + 16 + r};

    for (int k0 = 0; k0 < K; k0 += 32) {
        const int k = k0 + kq;
        u16x8 av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            // K % 4 == 0: load 8 values as two halves so a tail of 4 is exact
            av[a] = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
            bv[a] = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
            if (arow[a] < M) {
                const uint16_t *pa = A + (size_t)arow[a] * K + k;
                if (k + 8 <= K) {
                    av[a] = *reinterpret_cast<const u16x8 *>(pa);
                } else if (k + 4 <= K) {
                    const uint2 h = *reinterpret_cast<const uint2 *>(pa);
                    av[a][0] = h.x & 0xffff; av[a][1] = h.x >> 16;
                    av[a][2] = h.y & 0xffff; av[a][3] = h.y >> 16;
                }
            }
            if (brow[a] < N) {
                const uint16_t *pb = B + (size_t)brow[a] * K + k;
                if (k + 8 <= K) {
                    bv[a] = *reinterpret_cast<const u16x8 *>(pb);
                } else if (k + 4 <= K) {
                    const uint2 h = *reinterpret_cast<const uint2 *>(pb);
                    bv[a][0] = h.x & 0xffff; bv[a][1] = h.x >> 16;
                    bv[a][2] = h.y & 0xffff; bv[a][3] = h.y >> 16;
                }
            }
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    __builtin_bit_cast(bf16x8, av[a]), __builtin_bit_cast(bf16x8, bv[b]),
                    acc[a][b], 0, 0, 0);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
            store_tile(C, M, N, row0 + 16 * a, col0 + 16 * b, acc[a][b], lane);
}

// Round-to-nearest-even FP32 -> BF16 on the bit pattern (NaN kept quiet).
__device__ inline uint16_t to_bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu))
        return (uint16_t)((u >> 16) | 0x0040u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__global__ void cast_bf16_kernel(const float *__restrict__ x, uint16_t *__restrict__ y,
                                 size_t count)
{
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < count;
         k += (size_t)gridDim.x * blockDim.x)
        y[k] = to_bf16_rne(x[k]);
}

}  // namespace

hipError_t launch_gemm_nt_f32(const float *A, const float *B, float *C, int M, int N, int K,
                              hipStream_t st)
{
    dim3 grid((N + kBlockN - 1) / kBlockN, (M + kBlockM - 1) / kBlockM);
    hipLaunchKernelGGL(gemm_nt_f32_kernel, grid, dim3(256), 0, st, A, B, C, M, N, K);
    return hipGetLastError();
}

hipError_t launch_gemm_nt_bf16(const uint16_t *A, const uint16_t *B, float *C, int M, int N,
                               int K, hipStream_t st)
{
    dim3 grid((N + kBlockN - 1) / kBlockN, (M + kBlockM - 1) / kBlockM);
    hipLaunchKernelGGL(gemm_nt_bf16_kernel, grid, dim3(256), 0, st, A, B, C, M, N, K);
    return hipGetLastError();
}

hipError_t launch_cast_bf16(const float *x, uint16_t *y, size_t count, hipStream_t st)
{
    if (count == 0)
        return hipSuccess;
    size_t blocks = (count + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    hipLaunchKernelGGL(cast_bf16_kernel, dim3((unsigned)blocks), dim3(256), 0, st, x, y, count);
    return hipGetLastError();
}

}  // namespace dlk
