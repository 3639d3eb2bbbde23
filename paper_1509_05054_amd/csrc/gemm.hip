// Dense products of the coding stage on the matrix cores (MFMA):
//   G  = D D^T   [n][n]  (Gram matrix of the atoms)
//   A0 = Y D^T   [m][n]  (correlations D^T y of every signal)
// Both are "NT" products C[M][N] = A[M][K] B[N][K]^T of row-major operands
// whose K dimension (the signal size p) is contiguous.  Workgroup tiles of
// 128 rows stage row segments of the operands in LDS (coalesced loads, see
// gemm_f32_tile) and feed the MFMAs from there.
//
// MFMA layout used (16x16 output tile, wave64): lane l supplies row l%16 of
// the A-tile and column l%16 of the B-tile over a K-slice chosen by l/16, and
// receives C[4*(l/16) + r][l%16], r = 0..3.  Which K indices a lane group
// holds is irrelevant to the product as long as A and B use the same choice,
// so every lane loads 4 (FP32) or 8 (BF16) consecutive K values at once.
#include "dl_internal.h"
#include "rmse_body.h"

namespace dlk {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

constexpr int kTN = 4;                // 16x16 MFMA tiles per wave along N
constexpr int kBlockN = 2 * 16 * kTN;

// The workgroup's tile is written through LDS so that global stores cover
// whole contiguous row segments (the MFMA output layout gives each store
// instruction four 64-byte pieces of different rows).  acc[a][b] holds the
// 16x16 tile (a, b) of the calling wave; rows/cols are relative to the
// workgroup tile at (brow0, bcol0) of height BM.
constexpr int kStageLd = kBlockN + 4;

template <int TM, int BM>
__device__ inline void store_block(float *C, int M, int N, int ldc, int brow0, int bcol0,
                                   const f32x4 (&acc)[TM][kTN], float *sC, float *diag)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wr = (wave >> 1) * 16 * TM, wc = (wave & 1) * 16 * kTN;
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < kTN; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                sC[(wr + 16 * a + 4 * (lane >> 4) + r) * kStageLd + wc + 16 * b + (lane & 15)] =
                    acc[a][b][r];
    __syncthreads();
    if (diag) {  // a Gram tile: its diagonal entries go to diag, NaN to C
        const int d0 = max(brow0, bcol0);
        const int d1 = min(min(brow0 + BM, bcol0 + kBlockN), min(M, N));
        for (int r = d0 + (int)threadIdx.x; r < d1; r += (int)blockDim.x) {
            float *e = sC + (r - brow0) * kStageLd + (r - bcol0);
            diag[r] = *e;
            *e = __builtin_nanf("");
        }
        __syncthreads();
    }
    // 32 lanes per row, 4 columns each: 8 rows per pass of the workgroup;
    // 16-byte stores when C and its row stride allow them
    const bool vec_ok = (ldc % 4) == 0 && ((uintptr_t)C % 16) == 0;
    const int cc = 4 * (threadIdx.x & 31);
    const int col = bcol0 + cc;
#pragma unroll
    for (int r0 = 0; r0 < BM; r0 += 8) {
        const int rr = r0 + (int)(threadIdx.x >> 5);
        const int row = brow0 + rr;
        if (row >= M || col >= N)
            continue;
        const f32x4 v = *reinterpret_cast<const f32x4 *>(sC + rr * kStageLd + cc);
        float *dst = C + (size_t)row * ldc + col;
        if (vec_ok && col + 3 < N) {
            *reinterpret_cast<f32x4 *>(dst) = v;
        } else {
            for (int q = 0; q < 4 && col + q < N; ++q)
                dst[q] = v[q];
        }
    }
    __syncthreads();  // sC is reused by the next tile of a persistent workgroup
}

// The grid is one-dimensional (row tiles may exceed the 65535 limit of the
// y dimension): workgroup t < tiles computes tile (t % tiles_x, t / tiles_x)
// of the grid of output tiles, row-major as a two-dimensional launch would
// order them.  The err_blocks workgroups after the tiles carry the partial
// pass of an error with the coefficient refresh (measured: faster behind the
// tiles than ahead of them).
// Returns the tile index, or -1 for the error workgroups after running their
// share.
__device__ inline int error_blocks(int tiles, const RmseArgs &err, int err_blocks)
{
    const int w = (int)blockIdx.x;
    if (w < tiles)
        return w;
    if (w - tiles < err_blocks)
        rmse_refresh_body(err, w - tiles, err_blocks);
    return -1;
}

// Which of the (up to two) problems of a grouped launch this workgroup
// computes, and its tile origin.
template <class P>
__device__ inline bool pick_problem(const P &p0, const P &p1, int tiles_y0, int tiles_x, int tile,
                                    P &out, int &row0, int &col0, int block_m)
{
    const int by = tile / tiles_x;
    const int bx = tile % tiles_x;
    out = by < tiles_y0 ? p0 : p1;
    if (out.M_dev) {
        const int md = *out.M_dev;
        out.M = md < out.M ? md : out.M;
    }
    const int ty = by < tiles_y0 ? by : by - tiles_y0;
    row0 = ty * block_m;
    col0 = bx * kBlockN;
    return col0 < out.N && row0 < out.M;
}

// Operand tiles are staged in LDS, one K block at a time (double-buffered):
// the global loads are row segments, 8 lanes per 128 bytes (a lane-per-row
// load straight into the MFMA layout touches 16 rows per instruction; for the
// tall products that measured 20-35% slower), and each lane then reads its
// MFMA operands with 16-byte LDS loads.  The next block's global loads are issued before the
// current block's MFMAs.  LDS rows are padded by 16 bytes.
constexpr int kLdF32 = 32 + 4;  // floats per LDS row of a 32-wide FP32 K block
constexpr int kLdBf = 64 + 8;   // bf16 values per LDS row of a 64-wide BF16 K block

// One (32 TM) x kBlockN tile of C at (brow0, bcol0), by a 256-thread
// workgroup; every element is summed in the same K order for any TM.
template <int TM>
__device__ inline void gemm_f32_tile(const GemmF32 &P, int brow0, int bcol0)
{
    constexpr int BM = 32 * TM;
    constexpr int SA = BM * kLdF32;                 // A rows of a stage
    constexpr int STAGE = SA + kBlockN * kLdF32;    // + B rows
    constexpr int NA = BM * 8 / 256, NB = kBlockN * 8 / 256;  // float4 loads per thread
    constexpr int LDS = 2 * STAGE > BM * kStageLd ? 2 * STAGE : BM * kStageLd;
    __shared__ float lds[LDS];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wr = (wave >> 1) * 16 * TM, wc = (wave & 1) * 16 * kTN;
    const int r = lane & 15;
    const int kq = 4 * (lane >> 4);  // this lane's K offset inside a 16-wide K step
    const int M = P.M, N = P.N, K = P.K;

    f32x4 acc[TM][kTN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < kTN; ++b)
            acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

    f32x4 ra[NA], rb[NB];
    auto gload = [&](int k0) {
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int f = threadIdx.x + 256 * i;
            const int row = brow0 + f / 8, k = k0 + 4 * (f % 8);
            ra[i] = f32x4{0.f, 0.f, 0.f, 0.f};
            if (row < M && k < K)
                ra[i] = *reinterpret_cast<const f32x4 *>(P.A + (size_t)row * K + k);
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int f = threadIdx.x + 256 * i;
            const int col = bcol0 + f / 8, k = k0 + 4 * (f % 8);
            rb[i] = f32x4{0.f, 0.f, 0.f, 0.f};
            if (col < N && k < K)
                rb[i] = *reinterpret_cast<const f32x4 *>(P.B + (size_t)col * K + k);
        }
    };
    const int nk = (K + 31) / 32;
    gload(0);
    for (int kb = 0; kb < nk; ++kb) {
        // stage kb & 1 was last read two blocks ago, before the barrier below
        // of the previous block
        float *st = lds + (kb & 1) * STAGE;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int f = threadIdx.x + 256 * i;
            *reinterpret_cast<f32x4 *>(st + (f / 8) * kLdF32 + 4 * (f % 8)) = ra[i];
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int f = threadIdx.x + 256 * i;
            *reinterpret_cast<f32x4 *>(st + SA + (f / 8) * kLdF32 + 4 * (f % 8)) = rb[i];
        }
        __syncthreads();
        if (kb + 1 < nk)
            gload(32 * (kb + 1));
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            f32x4 av[TM], bv[kTN];
#pragma unroll
            for (int a = 0; a < TM; ++a)
                av[a] = *reinterpret_cast<const f32x4 *>(st + (wr + 16 * a + r) * kLdF32 + 16 * h + kq);
#pragma unroll
            for (int b = 0; b < kTN; ++b)
                bv[b] = *reinterpret_cast<const f32x4 *>(st + SA + (wc + 16 * b + r) * kLdF32 +
                                                         16 * h + kq);
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int a = 0; a < TM; ++a)
#pragma unroll
                    for (int b = 0; b < kTN; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a][q], bv[b][q],
                                                                          acc[a][b], 0, 0, 0);
        }
    }
    __syncthreads();  // the output stage overwrites the operand stages
    store_block<TM, BM>(P.C, M, N, P.ldc, brow0, bcol0, acc, lds, P.diag);
}

// Workgroup tiles of 128 rows (TM = 4) for the batched products and the
// large single-problem ones (measured: faster than 64-row tiles that load
// their operands straight into the MFMA layout, at m = 262144 and for the
// batched problems); small single problems take 32-row tiles (below).
constexpr int kF32TM = 4;
constexpr int kF32M = 32 * kF32TM;

template <int TM>
__global__ __launch_bounds__(256) void gemm_nt_f32_kernel(GemmF32 p0, GemmF32 p1, int tiles_y0,
                                                          int tiles_x, int tiles, RmseArgs err,
                                                          int err_blocks)
{
    const int tile = error_blocks(tiles, err, err_blocks);
    if (tile < 0)
        return;
    GemmF32 P;
    int brow0, bcol0;
    if (pick_problem(p0, p1, tiles_y0, tiles_x, tile, P, brow0, bcol0, 32 * TM))
        gemm_f32_tile<TM>(P, brow0, bcol0);
}

__host__ __device__ inline int gemm_tiles(const GemmF32 &P)
{
    return ((P.M + kF32M - 1) / kF32M) * ((P.N + kBlockN - 1) / kBlockN);
}

// Batched problems: the items of problem b are the tiles of its Gram matrix,
// then those of its correlations, row-major over the tile grid.  Items past
// all tiles, when etab is set, are the error partials of another iteration
// (list el, the blocks of each problem's partial pass).
__global__ __launch_bounds__(256) void gemm_batched_kernel(const GemmPair *__restrict__ tab,
                                                           BatchList bl,
                                                           const RmseArgs *__restrict__ etab,
                                                           BatchList el, int per)
{
    __shared__ int slot;
    const int tiles = bl.start[bl.count];
    const int total = tiles + (etab ? el.start[el.count] : 0);
    BatchCursor cur;
    BatchOwner own, eown;
    GemmF32 G, C;
    int tg = 0;
    RmseArgs ea;
    while (batch_advance(bl.q, total, per, cur, &slot)) {
        const int it = cur.it;
        if (it >= tiles) {
            const int e = it - tiles;
            if (batch_owner(el.start, el.count, e, eown))
                ea = etab[eown.b];
            rmse_body(ea, e - eown.b0, eown.b1 - eown.b0);
            continue;
        }
        if (batch_owner(bl.start, bl.count, it, own)) {
            G = tab[own.b].g;
            C = tab[own.b].c;
            tg = gemm_tiles(G);
        }
        int t = it - own.b0;
        const GemmF32 &P = t < tg ? G : C;
        if (t >= tg)
            t -= tg;
        const int tx = (P.N + kBlockN - 1) / kBlockN;
        gemm_f32_tile<kF32TM>(P, (t / tx) * kF32M, (t % tx) * kBlockN);
    }
    if (threadIdx.x == 0)
        batch_leave(bl.q, gridDim.x);
}

// 8 consecutive BF16 values (K % 4 == 0: a tail of 4 is loaded exactly).
__device__ inline u16x8 load_bf16x8(const uint16_t *ptr, int k, int K)
{
    u16x8 v = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
    if (k + 8 <= K) {
        const uint2 lo = *reinterpret_cast<const uint2 *>(ptr);
        const uint2 hi = *reinterpret_cast<const uint2 *>(ptr + 4);
        v[0] = lo.x & 0xffff; v[1] = lo.x >> 16; v[2] = lo.y & 0xffff; v[3] = lo.y >> 16;
        v[4] = hi.x & 0xffff; v[5] = hi.x >> 16; v[6] = hi.y & 0xffff; v[7] = hi.y >> 16;
    } else if (k + 4 <= K) {
        const uint2 lo = *reinterpret_cast<const uint2 *>(ptr);
        v[0] = lo.x & 0xffff; v[1] = lo.x >> 16; v[2] = lo.y & 0xffff; v[3] = lo.y >> 16;
    }
    return v;
}

template <int TM>
__global__ __launch_bounds__(256) void gemm_nt_bf16_kernel(GemmBF16 p0, GemmBF16 p1, int tiles_y0,
                                                           int tiles_x, int tiles, RmseArgs err,
                                                           int err_blocks)
{
    const int tile = error_blocks(tiles, err, err_blocks);
    if (tile < 0)
        return;
    constexpr int kTM = TM;
    GemmBF16 P;
    int brow0, bcol0;
    if (!pick_problem(p0, p1, tiles_y0, tiles_x, tile, P, brow0, bcol0, 32 * TM))
        return;
    constexpr int BM = 32 * TM;
    constexpr int SA = BM * kLdBf;                // A rows of a stage (bf16 values)
    constexpr int STAGE = SA + kBlockN * kLdBf;   // + B rows
    constexpr int NA = BM * 8 / 256, NB = kBlockN * 8 / 256;  // 16-byte loads per thread
    constexpr int LDS = STAGE > BM * kStageLd ? STAGE : BM * kStageLd;  // floats (2 stages)
    __shared__ float lds[LDS];
    uint16_t *ops = reinterpret_cast<uint16_t *>(lds);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wr = (wave >> 1) * 16 * kTM, wc = (wave & 1) * 16 * kTN;
    const int r = lane & 15;
    const int kq = 8 * (lane >> 4);  // 8 consecutive K values per lane in a 32-wide K step
    const int M = P.M, N = P.N, K = P.K;

    f32x4 acc[kTM][kTN];
#pragma unroll
    for (int a = 0; a < kTM; ++a)
#pragma unroll
        for (int b = 0; b < kTN; ++b)
            acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

    u16x8 ra[NA], rb[NB];
    const u16x8 zero8 = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
    auto gload = [&](int k0) {
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int f = threadIdx.x + 256 * i;
            const int row = brow0 + f / 8, k = k0 + 8 * (f % 8);
            ra[i] = row < M ? load_bf16x8(P.A + (size_t)row * K + k, k, K) : zero8;
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int f = threadIdx.x + 256 * i;
            const int col = bcol0 + f / 8, k = k0 + 8 * (f % 8);
            rb[i] = col < N ? load_bf16x8(P.B + (size_t)col * K + k, k, K) : zero8;
        }
    };
    // 64-wide K blocks staged as for the FP32 tile (two 32-wide MFMA steps each)
    const int nk = (K + 63) / 64;
    gload(0);
    for (int kb = 0; kb < nk; ++kb) {
        uint16_t *st = ops + (kb & 1) * STAGE;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int f = threadIdx.x + 256 * i;
            *reinterpret_cast<u16x8 *>(st + (f / 8) * kLdBf + 8 * (f % 8)) = ra[i];
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int f = threadIdx.x + 256 * i;
            *reinterpret_cast<u16x8 *>(st + SA + (f / 8) * kLdBf + 8 * (f % 8)) = rb[i];
        }
        __syncthreads();
        if (kb + 1 < nk)
            gload(64 * (kb + 1));
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            u16x8 av[kTM], bv[kTN];
#pragma unroll
            for (int a = 0; a < kTM; ++a)
                av[a] = *reinterpret_cast<const u16x8 *>(st + (wr + 16 * a + r) * kLdBf + 32 * h + kq);
#pragma unroll
            for (int b = 0; b < kTN; ++b)
                bv[b] = *reinterpret_cast<const u16x8 *>(st + SA + (wc + 16 * b + r) * kLdBf +
                                                         32 * h + kq);
#pragma unroll
            for (int a = 0; a < kTM; ++a)
#pragma unroll
                for (int b = 0; b < kTN; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        __builtin_bit_cast(bf16x8, av[a]), __builtin_bit_cast(bf16x8, bv[b]),
                        acc[a][b], 0, 0, 0);
        }
    }
    __syncthreads();  // the output stage overwrites the operand stages
    store_block<TM, BM>(P.C, M, N, P.ldc, brow0, bcol0, acc, lds, P.diag);
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

template <class P, class Kern>
hipError_t launch_grouped(Kern kern, const P &p0, const P *p1, int kid, hipStream_t st,
                          int block_m, const RmseArgs *err)
{
    const int ty0 = (p0.M + block_m - 1) / block_m;
    const int ty1 = p1 ? (p1->M + block_m - 1) / block_m : 0;
    int tx = (p0.N + kBlockN - 1) / kBlockN;
    if (p1)
        tx = tx > (p1->N + kBlockN - 1) / kBlockN ? tx : (p1->N + kBlockN - 1) / kBlockN;
    const int eb = err ? rmse_blocks_dev(err->m) : 0;
    const long long tiles = (long long)tx * (ty0 + ty1);
    if (tiles + eb > 0x7fffffffll)
        return hipErrorInvalidConfiguration;
    prof_begin(kid, st);
    hipLaunchKernelGGL(kern, dim3((unsigned)(tiles + eb)), dim3(256), 0, st, p0, p1 ? *p1 : p0,
                       ty0, tx, (int)tiles, err ? *err : RmseArgs{}, eb);
    prof_end(kid, st);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm_nt_f32(const GemmF32 &p0, const GemmF32 *p1, int kid, hipStream_t st,
                              const RmseArgs *err)
{
    // 32-row tiles while 128-row tiles would give fewer than four per CU
    // (measured at p = 64, n = 256: m = 16384 products 17.1 -> 14.9 us; at
    // m = 262144 the 128-row tiles stay faster, 123 vs 143 us); every element
    // is summed in the same order either way
    const long long rows = (long long)p0.M + (p1 ? p1->M : 0);
    const long long tiles128 = ((rows + 127) / 128) * ((p0.N + kBlockN - 1) / kBlockN);
    if (tiles128 < 1024)
        return launch_grouped(gemm_nt_f32_kernel<1>, p0, p1, kid, st, 32, err);
    return launch_grouped(gemm_nt_f32_kernel<4>, p0, p1, kid, st, 128, err);
}

hipError_t launch_gemm_nt_bf16(const GemmBF16 &p0, const GemmBF16 *p1, int kid, hipStream_t st,
                               const RmseArgs *err)
{
    return launch_grouped(gemm_nt_bf16_kernel<4>, p0, p1, kid, st, 128, err);
}

int gemm_pair_items(const GemmPair &pp) { return gemm_tiles(pp.g) + gemm_tiles(pp.c); }

hipError_t launch_batched_gemm(const GemmPair *tab, const BatchList &bl, int items,
                               hipStream_t st, const RmseArgs *etab, const BatchList &el,
                               int eitems)
{
    const int wg = batch_workers((const void *)gemm_batched_kernel, 256, 0,
                                 items + (etab ? eitems : 0));
    prof_begin(DL_K_CORR, st);
    hipLaunchKernelGGL(gemm_batched_kernel, dim3(wg), dim3(256), 0, st, tab, bl, etab, el,
                       batch_per_ticket(items + (etab ? eitems : 0), wg));
    prof_end(DL_K_CORR, st);
    return hipGetLastError();
}

hipError_t launch_cast_bf16(const float *x, uint16_t *y, size_t count, hipStream_t st)
{
    if (count == 0)
        return hipSuccess;
    size_t blocks = (count + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    prof_begin(DL_K_MISC, st);
    hipLaunchKernelGGL(cast_bf16_kernel, dim3((unsigned)blocks), dim3(256), 0, st, x, y, count);
    prof_end(DL_K_MISC, st);
    return hipGetLastError();
}

}  // namespace dlk
