// Users of every atom (the set I_j of Sec. 3): a deterministic, stable
// counting-sort transpose of the ELL representation X into CSR by atom.
//
//   count   : one workgroup per block of kCsrBlock signals.  Each wave walks
//             its 64 signals' entries in (signal, slot) order, 64 at a time;
//             entries of one atom inside a 64-entry chunk are ranked with a
//             ballot loop, and per-wave running counts (LDS) rank them across
//             chunks.  Result: per-block atom counts and, per entry, its rank
//             among the block's uses of that atom.
//   scan    : one workgroup; per atom, totals over blocks, an exclusive scan
//             over atoms (row_ptr, and chunk_ptr for the update's chunks of
//             kChunk users), then the per-(block, atom) start offsets.
//   scatter : one thread per entry: users[offset(block, atom) + rank] = entry.
// Entries of an atom end up in increasing (signal, slot) order, so the
// result is unique and the atom update's summation order is fixed.
#include "dl_internal.h"

namespace dlk {
namespace {

constexpr int kWavesPerBlock = kCsrBlock / 64;

__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(kCsrBlock) void csr_count_kernel(const int32_t *__restrict__ idx,
                                                              int32_t *__restrict__ blkcnt,
                                                              int32_t *__restrict__ lrank, int n,
                                                              int m, int s)
{
    extern __shared__ int32_t wcnt[];  // [kWavesPerBlock][n]
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int b = blockIdx.x;
    for (int t = threadIdx.x; t < kWavesPerBlock * n; t += blockDim.x)
        wcnt[t] = 0;
    __syncthreads();

    int32_t *mycnt = wcnt + wave * n;
    const int sig0 = b * kCsrBlock + wave * 64;
    const unsigned long long lt = (1ull << lane) - 1ull;
    for (int c = 0; c < s; ++c) {
        const int e = 64 * c + lane;  // entry inside this wave's 64 x s block
        const int i = sig0 + e / s;
        const int t = e % s;
        int atom = i < m ? idx[(size_t)i * s + t] : -1;
        if (atom >= n)
            atom = -1;  // out-of-range indices are treated as unused slots
        unsigned long long pending = __ballot(atom >= 0);
        int myrank = 0, mycount = 0;
        bool last = false;
        while (pending) {
            const int leader = __ffsll((long long)pending) - 1;
            const int la = __builtin_amdgcn_readlane(atom, leader);
            const unsigned long long mm = __ballot(atom == la);
            if (atom == la) {
                myrank = __popcll(mm & lt);
                mycount = __popcll(mm);
                last = lane == 63 - __clzll((long long)mm);
            }
            pending &= ~mm;
        }
        int base = 0;
        if (atom >= 0) {
            base = mycnt[atom];
            lrank[(size_t)i * s + t] = base + myrank;
        }
        wave_lds_sync();
        if (atom >= 0 && last)
            mycnt[atom] = base + mycount;
        wave_lds_sync();
    }
    __syncthreads();
    // block totals, and per-wave counts -> exclusive prefix over waves
    for (int a = threadIdx.x; a < n; a += blockDim.x) {
        int run = 0;
        for (int w = 0; w < kWavesPerBlock; ++w) {
            const int v = wcnt[w * n + a];
            wcnt[w * n + a] = run;
            run += v;
        }
        blkcnt[(size_t)b * n + a] = run;
    }
    __syncthreads();
    for (int c = 0; c < s; ++c) {
        const int e = 64 * c + lane;
        const int i = sig0 + e / s;
        const int t = e % s;
        if (i < m) {
            const int atom = idx[(size_t)i * s + t];
            if (atom >= 0 && atom < n)
                lrank[(size_t)i * s + t] += mycnt[atom];
        }
    }
}

// Exclusive scan of one value per thread over a 1024-thread workgroup;
// returns the exclusive prefix and writes the workgroup total to *total.
__device__ int block_exclusive_scan(int v, int *sh /*[16]*/, int *total)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off);
        if (lane >= off)
            x += y;
    }
    if (lane == 63)
        sh[wave] = x;
    __syncthreads();
    int wbase = 0, tot = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
        const int t = sh[w];
        if (w < wave)
            wbase += t;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return wbase + x - v;
}

__global__ __launch_bounds__(1024) void csr_scan_kernel(int32_t *__restrict__ blkcnt,
                                                        int32_t *__restrict__ row_ptr,
                                                        int32_t *__restrict__ chunk_ptr, int n,
                                                        int nb)
{
    __shared__ int sh[16];
    int carry_u = 0, carry_c = 0;
    for (int a0 = 0; a0 < n; a0 += blockDim.x) {
        const int a = a0 + threadIdx.x;
        int tot = 0;
        if (a < n)
            for (int b = 0; b < nb; ++b)
                tot += blkcnt[(size_t)b * n + a];
        const int chunks = (tot + kChunk - 1) / kChunk;
        int tu, tc;
        const int pu = block_exclusive_scan(tot, sh, &tu) + carry_u;
        const int pc = block_exclusive_scan(chunks, sh, &tc) + carry_c;
        if (a < n) {
            row_ptr[a] = pu;
            chunk_ptr[a] = pc;
            int run = pu;
            for (int b = 0; b < nb; ++b) {
                const int v = blkcnt[(size_t)b * n + a];
                blkcnt[(size_t)b * n + a] = run;
                run += v;
            }
        }
        carry_u += tu;
        carry_c += tc;
    }
    if (threadIdx.x == 0) {
        row_ptr[n] = carry_u;
        chunk_ptr[n] = carry_c;
    }
}

__global__ void csr_scatter_kernel(const int32_t *__restrict__ idx,
                                   const int32_t *__restrict__ blkoff,
                                   const int32_t *__restrict__ lrank, int32_t *__restrict__ users,
                                   float *__restrict__ val_pad, int n, int m, int s)
{
    const size_t total = (size_t)m * s;
    for (size_t pos = (size_t)blockIdx.x * blockDim.x + threadIdx.x; pos < total;
         pos += (size_t)gridDim.x * blockDim.x) {
        const int atom = idx[pos];
        if (atom < 0 || atom >= n) {
            if (val_pad)
                val_pad[pos] = 0.f;
            continue;
        }
        const int b = (int)(pos / s) / kCsrBlock;
        users[blkoff[(size_t)b * n + atom] + lrank[pos]] = (int32_t)pos;
    }
}

}  // namespace

int csr_blocks(int m) { return (m + kCsrBlock - 1) / kCsrBlock; }

hipError_t launch_csr(const CsrArgs &a, hipStream_t st)
{
    const int nb = csr_blocks(a.m);
    const size_t shmem = sizeof(int32_t) * kWavesPerBlock * a.n;
    hipLaunchKernelGGL(csr_count_kernel, dim3(nb), dim3(kCsrBlock), shmem, st, a.idx, a.blkcnt,
                       a.lrank, a.n, a.m, a.s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(csr_scan_kernel, dim3(1), dim3(1024), 0, st, a.blkcnt, a.row_ptr,
                       a.chunk_ptr, a.n, nb);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const size_t total = (size_t)a.m * a.s;
    size_t blocks = (total + 255) / 256;
    if (blocks > 8192)
        blocks = 8192;
    hipLaunchKernelGGL(csr_scatter_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a.idx,
                       a.blkcnt, a.lrank, a.users, a.val_pad, a.n, a.m, a.s);
    return hipGetLastError();
}

}  // namespace dlk
