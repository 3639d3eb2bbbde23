// Support-proposal network: in -> H -> H -> out with ReLU, BF16 storage of
// weights and activations, FP32 accumulation on the BF16 matrix cores, FP32
// master weights and Adam state.  Trained with a multi-label loss (mean binary
// cross-entropy on the logits, positives weighted by w_pos) on (signal, OMP
// support) pairs.  The network sees each signal scaled to unit norm: the OMP
// support depends only on the signal's direction.
//
// Every product is an "NT" GEMM C[M][N] = A[M][K] B[N][K]^T with both operands
// K-contiguous BF16; the backward pass gets K-contiguous operands because the
// forward epilogues also write transposed copies of the activations, and the
// weights are kept transposed in BF16 as well:
//   forward   H1 = relu(X W1^T + b1), H2 = relu(H1 W2^T + b2), Z = H2 W3^T + b3
//   loss      dZ = (sigmoid(Z) (1 - T) - (1 - sigmoid(Z)) T w_pos) / (B * out)
//   backward  dA2 = (dZ W3) . [H2 > 0]     A = dZ,   B = W3^T
//             dW3 = dZ^T H2                A = dZ^T, B = H2^T   (split over K)
//             dA1 = (dA2 W2) . [H1 > 0]    A = dA2,  B = W2^T
//             dW2 = dA2^T H1,  dW1 = dA1^T X
//   biases    row sums of dZ^T, dA2^T, dA1^T
#include "dl_internal.h"

namespace dlk {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kTM = 2, kTN = 4;           // 16x16 tiles per wave (M, N)
constexpr int kBM = 2 * 16 * kTM;         // 64 rows per workgroup
constexpr int kBN = 2 * 16 * kTN;         // 128 cols per workgroup

__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu))
        return (uint16_t)((u >> 16) | 0x0040u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__global__ __launch_bounds__(256) void mlp_gemm_kernel(MlpGemm g)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int row0 = blockIdx.y * kBM + (wave >> 1) * 16 * kTM;
    const int col0 = blockIdx.x * kBN + (wave & 1) * 16 * kTN;
    const int r = lane & 15;
    const int kq = 8 * (lane >> 4);
    // K range of this split (a multiple of 32 long)
    const int kper = ((g.K + gridDim.z - 1) / gridDim.z + 31) & ~31;
    const int kb = blockIdx.z * kper;
    const int ke = min(g.K, kb + kper);

    f32x4 acc[kTM][kTN];
#pragma unroll
    for (int a = 0; a < kTM; ++a)
#pragma unroll
        for (int b = 0; b < kTN; ++b)
            acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = kb; k0 < ke; k0 += 32) {
        const int k = k0 + kq;
        uint4 av[kTM], bv[kTN];
#pragma unroll
        for (int a = 0; a < kTM; ++a) {
            const int row = row0 + 16 * a + r;
            av[a] = make_uint4(0, 0, 0, 0);
            if (row < g.M && k < ke)
                av[a] = *reinterpret_cast<const uint4 *>(g.A + (size_t)row * g.lda + k);
        }
#pragma unroll
        for (int b = 0; b < kTN; ++b) {
            const int col = col0 + 16 * b + r;
            bv[b] = make_uint4(0, 0, 0, 0);
            if (col < g.N && k < ke)
                bv[b] = *reinterpret_cast<const uint4 *>(g.B + (size_t)col * g.ldb + k);
        }
#pragma unroll
        for (int a = 0; a < kTM; ++a)
#pragma unroll
            for (int b = 0; b < kTN; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    __builtin_bit_cast(bf16x8, av[a]), __builtin_bit_cast(bf16x8, bv[b]), acc[a][b],
                    0, 0, 0);
    }

    // epilogue: lane holds C[rb + 0..3][col] of each tile
#pragma unroll
    for (int a = 0; a < kTM; ++a)
#pragma unroll
        for (int b = 0; b < kTN; ++b) {
            const int col = col0 + 16 * b + (lane & 15);
            const int rb = row0 + 16 * a + 4 * (lane >> 4);
            if (col >= g.N)
                continue;
            float v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                v[q] = acc[a][b][q];
                if (g.bias)
                    v[q] += g.bias[col];
            }
            if (g.epi == kEpiF32) {
                float *C = g.Cf + (size_t)blockIdx.z * g.split_stride;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (rb + q < g.M)
                        C[(size_t)(rb + q) * g.ldcf + col] = v[q];
                continue;
            }
            uint16_t h[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                float x = v[q];
                if (g.epi == kEpiBiasRelu)
                    x = fmaxf(x, 0.f);
                else if (rb + q < g.M && !(bf2f(g.mask[(size_t)(rb + q) * g.ldmask + col]) > 0.f))
                    x = 0.f;  // ReLU backward: the forward activation was 0
                h[q] = f2bf(x);
            }
            if (g.Cb)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (rb + q < g.M)
                        g.Cb[(size_t)(rb + q) * g.ldcb + col] = h[q];
            if (g.Ct) {
                uint16_t *t = g.Ct + (size_t)col * g.ldct + rb;
                if (rb + 3 < g.M) {
                    uint2 pk;
                    pk.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
                    pk.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
                    *reinterpret_cast<uint2 *>(t) = pk;
                } else {
                    for (int q = 0; q < 4; ++q)
                        if (rb + q < g.M)
                            t[q] = h[q];
                }
            }
        }
}

// out[e] = sum over splits of part[s * stride + e], in split order
__global__ void sum_splits_kernel(const float *__restrict__ part, float *__restrict__ out,
                                  size_t count, int splits, size_t stride)
{
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (size_t)gridDim.x * blockDim.x) {
        float acc = 0.f;
        for (int s = 0; s < splits; ++s)
            acc += part[(size_t)s * stride + e];
        out[e] = acc;
    }
}

// out[r] = sum_c X[r][c] for a BF16 matrix X[rows][cols] (cols % 8 == 0): one
// workgroup per row, 16-byte loads (8 values per lane per load), the lane
// partials summed in a fixed order (wave shuffles, then the four waves).
__global__ __launch_bounds__(256) void rowsum_bf16_kernel(const uint16_t *__restrict__ X,
                                                          float *__restrict__ out, int rows,
                                                          int cols)
{
    __shared__ float red[4];
    const int row = blockIdx.x;
    const uint16_t *x = X + (size_t)row * cols;
    float acc = 0.f;
    for (int c = 8 * threadIdx.x; c < cols; c += 8 * 256) {
        const uint4 v = *reinterpret_cast<const uint4 *>(x + c);
        acc += bf2f(v.x & 0xffff) + bf2f(v.x >> 16) + bf2f(v.y & 0xffff) + bf2f(v.y >> 16) +
               bf2f(v.z & 0xffff) + bf2f(v.z >> 16) + bf2f(v.w & 0xffff) + bf2f(v.w >> 16);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0)
        out[row] = ((red[0] + red[1]) + red[2]) + red[3];
}

// 1 / ||row|| in FP32 for one wave's row (0 for a zero row); every lane gets it.
__device__ inline float inv_row_norm(const float *__restrict__ row, int p, int lane)
{
    float ss = 0.f;
    for (int q = lane; q < p; q += 64)
        ss += row[q] * row[q];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        ss += __shfl_xor(ss, off);
    return ss > 0.f ? 1.0f / sqrtf(ss) : 0.f;
}

// Minibatch: unit-norm X rows (BF16) and their transpose from the chosen
// pairs, one wave per row; pair id q names signal q % m and label row q of
// `hist`.
__global__ __launch_bounds__(256) void gather_batch_kernel(const float *__restrict__ Y, int m,
                                                           int p,
                                                           const int32_t *__restrict__ pairs,
                                                           int B, uint16_t *__restrict__ Xb,
                                                           uint16_t *__restrict__ Xbt)
{
    const int lane = threadIdx.x & 63;
    const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= B)
        return;
    const int sig = (int)((unsigned)pairs[b] % (unsigned)m);
    const float *row = Y + (size_t)sig * p;
    const float inv = inv_row_norm(row, p, lane);
    for (int q = lane; q < p; q += 64) {
        const uint16_t h = f2bf(row[q] * inv);
        Xb[(size_t)b * p + q] = h;
        if (Xbt)
            Xbt[(size_t)q * B + b] = h;
    }
}

// Consecutive FP32 rows -> unit-norm BF16 rows (inference input), one wave
// per row.
__global__ __launch_bounds__(256) void gather_rows_kernel(const float *__restrict__ X, int rows,
                                                          int cols, uint16_t *__restrict__ Xb)
{
    const int lane = threadIdx.x & 63;
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= rows)
        return;
    const float *row = X + (size_t)r * cols;
    const float inv = inv_row_norm(row, cols, lane);
    for (int q = lane; q < cols; q += 64)
        Xb[(size_t)r * cols + q] = f2bf(row[q] * inv);
}

// Loss and its gradient w.r.t. the logits, one wave per minibatch row.
__global__ __launch_bounds__(256) void bce_kernel(const float *__restrict__ Z, int out_dim,
                                                  const int32_t *__restrict__ hist, int s,
                                                  const int32_t *__restrict__ pairs, int B,
                                                  uint16_t *__restrict__ dZ,
                                                  uint16_t *__restrict__ dZt,
                                                  double *__restrict__ loss_rows, float w_pos)
{
    const int lane = threadIdx.x & 63;
    const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= B)
        return;
    const int32_t *lab = hist + (size_t)pairs[b] * s;
    const float scale = 1.0f / ((float)B * (float)out_dim);
    double l = 0.0;
    for (int c = lane; c < out_dim; c += 64) {
        bool t = false;
        for (int q = 0; q < s; ++q)
            t |= lab[q] == c;
        const float z = Z[(size_t)b * out_dim + c];
        const float sig = 1.0f / (1.0f + expf(-z));
        const float d = (t ? -(1.0f - sig) * w_pos : sig) * scale;
        const uint16_t h = f2bf(d);
        dZ[(size_t)b * out_dim + c] = h;
        dZt[(size_t)c * B + b] = h;
        // positives: w_pos softplus(-z); negatives: softplus(z) (stable forms)
        const float sp = log1pf(expf(-fabsf(z)));
        l += t ? (double)w_pos * (double)(fmaxf(-z, 0.f) + sp) : (double)(fmaxf(z, 0.f) + sp);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        l += __shfl_xor(l, off);
    if (lane == 0)
        loss_rows[b] = l;
}

// Adam on FP32 master weights; refreshes the BF16 copy (and its transpose).
__global__ void adam_kernel(float *__restrict__ w, const float *__restrict__ g,
                            float *__restrict__ m1, float *__restrict__ m2, size_t count,
                            int rows, int cols, uint16_t *__restrict__ wb,
                            uint16_t *__restrict__ wbt, AdamHyper h, int do_step)
{
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (size_t)gridDim.x * blockDim.x) {
        float x = w[e];
        if (do_step) {
            const float gr = g[e];
            const float a = h.beta1 * m1[e] + (1.f - h.beta1) * gr;
            const float v = h.beta2 * m2[e] + (1.f - h.beta2) * gr * gr;
            m1[e] = a;
            m2[e] = v;
            const float mh = a / h.bc1;
            const float vh = v / h.bc2;
            x -= h.lr * mh / (sqrtf(vh) + h.eps);
            w[e] = x;
        }
        const uint16_t hb = f2bf(x);
        if (wb)
            wb[e] = hb;
        if (wbt) {
            const int rr = (int)(e / cols), cc = (int)(e % cols);
            wbt[(size_t)cc * rows + rr] = hb;
        }
    }
}

unsigned grid1(size_t items, unsigned cap)
{
    size_t b = (items + 255) / 256;
    if (b < 1)
        b = 1;
    return (unsigned)(b > cap ? cap : b);
}

}  // namespace

hipError_t launch_mlp_gemm(const MlpGemm &g, int splits, hipStream_t st)
{
    dim3 grid((g.N + kBN - 1) / kBN, (g.M + kBM - 1) / kBM, splits);
    prof_begin(DL_K_MLP, st);
    hipLaunchKernelGGL(mlp_gemm_kernel, grid, dim3(256), 0, st, g);
    prof_end(DL_K_MLP, st);
    return hipGetLastError();
}

hipError_t launch_sum_splits(const float *part, float *out, size_t count, int splits,
                             size_t stride, hipStream_t st)
{
    prof_begin(DL_K_MLP, st);
    hipLaunchKernelGGL(sum_splits_kernel, dim3(grid1(count, 2048)), dim3(256), 0, st, part, out,
                       count, splits, stride);
    prof_end(DL_K_MLP, st);
    return hipGetLastError();
}

hipError_t launch_rowsum_bf16(const uint16_t *X, float *out, int rows, int cols, hipStream_t st)
{
    if (cols % 8 != 0)
        return hipErrorInvalidValue;  // every caller passes the batch size, a multiple of 32
    prof_begin(DL_K_MLP, st);
    hipLaunchKernelGGL(rowsum_bf16_kernel, dim3(rows), dim3(256), 0, st, X, out, rows, cols);
    prof_end(DL_K_MLP, st);
    return hipGetLastError();
}

hipError_t launch_gather_batch(const float *Y, int m, int p, const int32_t *pairs, int B,
                               uint16_t *Xb, uint16_t *Xbt, hipStream_t st)
{
    prof_begin(DL_K_MLP, st);
    hipLaunchKernelGGL(gather_batch_kernel, dim3((B + 3) / 4), dim3(256), 0, st, Y, m, p, pairs,
                       B, Xb, Xbt);
    prof_end(DL_K_MLP, st);
    return hipGetLastError();
}

hipError_t launch_gather_rows(const float *X, int rows, int cols, uint16_t *Xb, hipStream_t st)
{
    prof_begin(DL_K_MLP, st);
    hipLaunchKernelGGL(gather_rows_kernel, dim3((rows + 3) / 4), dim3(256), 0, st, X, rows, cols,
                       Xb);
    prof_end(DL_K_MLP, st);
    return hipGetLastError();
}

hipError_t launch_bce(const float *Z, int out_dim, const int32_t *hist, int s,
                      const int32_t *pairs, int B, uint16_t *dZ, uint16_t *dZt, double *loss_rows,
                      float w_pos, hipStream_t st)
{
    prof_begin(DL_K_MLP, st);
    hipLaunchKernelGGL(bce_kernel, dim3((B + 3) / 4), dim3(256), 0, st, Z, out_dim, hist, s,
                       pairs, B, dZ, dZt, loss_rows, w_pos);
    prof_end(DL_K_MLP, st);
    return hipGetLastError();
}

hipError_t launch_adam(float *w, const float *g, float *m1, float *m2, int rows, int cols,
                       uint16_t *wb, uint16_t *wbt, const AdamHyper &h, int do_step,
                       hipStream_t st)
{
    const size_t count = (size_t)rows * cols;
    prof_begin(DL_K_MLP, st);
    hipLaunchKernelGGL(adam_kernel, dim3(grid1(count, 4096)), dim3(256), 0, st, w, g, m1, m2,
                       count, rows, cols, wb, wbt, h, do_step);
    prof_end(DL_K_MLP, st);
    return hipGetLastError();
}

}  // namespace dlk
