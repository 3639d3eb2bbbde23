// Users of every atom (the set I_j of Sec. 3): a deterministic, stable
// counting-sort transpose of the ELL representation X into CSR by atom.
//
//   count   : one workgroup per block of kCsrBlock signals, one wave per 64
//             signals.  A wave walks its entries in (signal, slot) order, 64
//             at a time; each lane sets its bit in an LDS bit mask of its
//             atom, so its rank among the chunk's uses of that atom is the
//             popcount of the lower bits, and per-wave running counts rank
//             the chunks.  Result: per-(atom, block) counts and, per entry,
//             its rank among the block's uses of the atom.
//   scan    : one wave per atom scans its per-block counts into offsets and
//             its total.
//   scatter : every workgroup scans the atom totals into atom offsets in LDS
//             (the first also writes row_ptr and chunk_ptr, the update's
//             chunks of the update's chunk size); one thread per entry:
//             users[row offset + block offset + rank] = entry.
// Entries of an atom end up in increasing (signal, slot) order, so the
// result is unique and the atom update's summation order is fixed.
#include "dl_internal.h"
#include "rmse_body.h"

namespace dlk {
namespace {

constexpr int kWavesPerBlock = kCsrBlock / 64;

__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Signal block b of the count pass; smem holds kWavesPerBlock * n 64-bit
// masks and as many counters.
__device__ inline void csr_count_body(const int32_t *__restrict__ idx, int32_t *__restrict__ blkcnt,
                                      int32_t *__restrict__ lrank, int n, int m, int s, int nb,
                                      int b, unsigned long long *smem)
{
    unsigned long long *masks = smem;                                  // [waves][n]
    int32_t *wcnt = reinterpret_cast<int32_t *>(smem + kWavesPerBlock * n);  // [waves][n]
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    for (int t = threadIdx.x; t < kWavesPerBlock * n; t += blockDim.x) {
        masks[t] = 0ull;
        wcnt[t] = 0;
    }
    __syncthreads();

    unsigned long long *mymask = masks + wave * n;
    int32_t *mycnt = wcnt + wave * n;
    // the wave's 64 signals hold 64 s consecutive slots; this lane's slot c
    // is slot 64 c + lane of them, loaded once and kept in registers with its
    // rank among the wave's users of the same atom
    constexpr int kMaxS = 16;
    const size_t pos0 = ((size_t)b * kCsrBlock + wave * 64) * s + lane;
    const size_t ms = (size_t)m * s;
    int atoms[kMaxS], rk[kMaxS];
#pragma unroll
    for (int c = 0; c < kMaxS; ++c) {
        atoms[c] = -1;
        rk[c] = 0;
        if (c < s && pos0 + 64 * c < ms) {
            const int atom = idx[pos0 + 64 * c];
            atoms[c] = atom < n ? atom : -1;  // out-of-range indices are unused slots
        }
    }
    const unsigned long long bit = 1ull << lane;
    const unsigned long long lower = bit - 1ull;
#pragma unroll
    for (int c = 0; c < kMaxS; ++c) {
        if (c >= s)
            break;
        const int atom = atoms[c];
        if (atom >= 0)
            atomicOr(&mymask[atom], bit);
        wave_lds_sync();
        unsigned long long mm = 0;
        int base = 0;
        if (atom >= 0) {
            mm = mymask[atom];
            base = mycnt[atom];
            rk[c] = base + __popcll(mm & lower);
        }
        wave_lds_sync();
        if (atom >= 0 && lane == 63 - __clzll((long long)mm)) {
            mycnt[atom] = base + __popcll(mm);
            mymask[atom] = 0ull;
        }
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
        blkcnt[(size_t)a * nb + b] = run;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kMaxS; ++c)
        if (c < s && atoms[c] >= 0)
            lrank[pos0 + 64 * c] = rk[c] + mycnt[atoms[c]];
}

__global__ __launch_bounds__(kCsrBlock) void csr_count_kernel(const int32_t *__restrict__ idx,
                                                              int32_t *__restrict__ blkcnt,
                                                              int32_t *__restrict__ lrank, int n,
                                                              int m, int s, int nb)
{
    extern __shared__ unsigned long long smem[];
    csr_count_body(idx, blkcnt, lrank, n, m, s, nb, blockIdx.x, smem);
}

__device__ inline int wave_inclusive_scan(int x)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off);
        if (lane >= off)
            x += y;
    }
    return x;
}

// Per atom (one wave each): per-block counts -> offsets inside the atom's
// user list, and the atom total.  Item blk covers atoms 4 blk .. 4 blk + 3.
__device__ inline void csr_scan_body(int32_t *__restrict__ blkcnt, int32_t *__restrict__ tot,
                                     int n, int nb, int blk)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int a = blk * 4 + wave;
    if (a >= n)
        return;
    int carry = 0;
    for (int b0 = 0; b0 < nb; b0 += 64) {
        const int b = b0 + lane;
        const int v = b < nb ? blkcnt[(size_t)a * nb + b] : 0;
        const int x = wave_inclusive_scan(v);
        if (b < nb)
            blkcnt[(size_t)a * nb + b] = carry + x - v;
        carry += __shfl(x, 63);
    }
    if (lane == 0)
        tot[a] = carry;
}

// Exclusive scan of the atom totals into sRow[0..n] (users) and, when
// chunk_ptr is given, of their chunk counts (chunk users per chunk) into
// chunk_ptr, and sRow into row_ptr; 256 threads, thread t owning atoms
// [t*per, (t+1)*per).
__device__ inline void csr_prefix_block(const int32_t *__restrict__ tot, int n, int32_t *sRow,
                                        int32_t *__restrict__ row_ptr,
                                        int32_t *__restrict__ chunk_ptr, int chunk)
{
    __shared__ int sh[2][4];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int per = (n + 255) / 256;
    const int a0 = threadIdx.x * per;
    int su = 0, sc = 0;
    for (int q = 0; q < per; ++q) {
        const int aa = a0 + q;
        if (aa < n) {
            const int v = tot[aa];
            su += v;
            sc += (v + chunk - 1) / chunk;
        }
    }
    const int xu = wave_inclusive_scan(su);
    const int xc = wave_inclusive_scan(sc);
    __syncthreads();  // sh and sRow of a previous item are no longer read
    if (lane == 63) {
        sh[0][wave] = xu;
        sh[1][wave] = xc;
    }
    __syncthreads();
    int bu = 0, bc = 0, tu = 0, tc = 0;
    for (int w = 0; w < 4; ++w) {
        if (w < wave) {
            bu += sh[0][w];
            bc += sh[1][w];
        }
        tu += sh[0][w];
        tc += sh[1][w];
    }
    int ru = bu + xu - su, rc = bc + xc - sc;
    for (int q = 0; q < per; ++q) {
        const int aa = a0 + q;
        if (aa < n) {
            const int v = tot[aa];
            sRow[aa] = ru;
            if (chunk_ptr) {
                row_ptr[aa] = ru;
                chunk_ptr[aa] = rc;
            }
            ru += v;
            rc += (v + chunk - 1) / chunk;
        }
    }
    if (threadIdx.x == 0) {
        sRow[n] = tu;
        if (chunk_ptr) {
            row_ptr[n] = tu;
            chunk_ptr[n] = tc;
        }
    }
    __syncthreads();
}

// The last workgroup, when err_blocks > 0, sums the partials of an error
// (independent of the scan).
__global__ __launch_bounds__(256) void csr_scan_kernel(int32_t *__restrict__ blkcnt,
                                                       int32_t *__restrict__ tot, int n, int nb,
                                                       RmseArgs err, int err_blocks)
{
    if (err_blocks > 0 && blockIdx.x == gridDim.x - 1) {
        rmse_final_body(err, err_blocks);
        return;
    }
    csr_scan_body(blkcnt, tot, n, nb, blockIdx.x);
}


// Scatter (workgroup of 256 threads): the atom offsets are scanned from the
// atom totals by every workgroup (n <= 1024, cheap), and item 0 also writes
// row_ptr and chunk_ptr for the atom update.
__device__ inline void csr_scatter_body(const int32_t *__restrict__ idx,
                                        const int32_t *__restrict__ blkoff,
                                        const int32_t *__restrict__ tot,
                                        int32_t *__restrict__ row_ptr,
                                        int32_t *__restrict__ chunk_ptr,
                                        const int32_t *__restrict__ lrank,
                                        int32_t *__restrict__ users, int2 *__restrict__ uent,
                                        const float *__restrict__ val,
                                        float *__restrict__ val_pad, int n, int m, int s, int nb,
                                        int chunk, int blk, int nblk)
{
    __shared__ int32_t sRow[1025];
    csr_prefix_block(tot, n, sRow, row_ptr, blk == 0 ? chunk_ptr : nullptr, chunk);
    const size_t total = (size_t)m * s;
    for (size_t pos = (size_t)blk * blockDim.x + threadIdx.x; pos < total;
         pos += (size_t)nblk * blockDim.x) {
        const int atom = idx[pos];
        if (atom < 0 || atom >= n) {
            if (val_pad)
                val_pad[pos] = 0.f;
            continue;
        }
        const int b = (int)(pos / s) / kCsrBlock;
        const int u = sRow[atom] + blkoff[(size_t)atom * nb + b] + lrank[pos];
        if (users)
            users[u] = (int32_t)pos;
        if (uent)
            uent[u] = make_int2((int)pos, __float_as_int(val[pos]));
    }
}

__global__ __launch_bounds__(256) void csr_scatter_kernel(
    const int32_t *__restrict__ idx, const int32_t *__restrict__ blkoff,
    const int32_t *__restrict__ tot, int32_t *__restrict__ row_ptr,
    int32_t *__restrict__ chunk_ptr, const int32_t *__restrict__ lrank,
    int32_t *__restrict__ users, int2 *__restrict__ uent, const float *__restrict__ val,
    float *__restrict__ val_pad, int n, int m, int s, int nb, int chunk)
{
    csr_scatter_body(idx, blkoff, tot, row_ptr, chunk_ptr, lrank, users, uent, val, val_pad, n,
                     m, s, nb, chunk, blockIdx.x, gridDim.x);
}

// ---- batched problems: one launch per pass over every problem's items ----
__device__ inline int csr_nb(int m) { return (m + kCsrBlock - 1) / kCsrBlock; }

__global__ __launch_bounds__(kCsrBlock) void csr_count_batched(const CsrArgs *__restrict__ tab,
                                                               BatchList bl, int per)
{
    extern __shared__ unsigned long long smem[];
    __shared__ int slot;
    const int total = bl.start[bl.count];
    BatchCursor cur;
    BatchOwner own;
    CsrArgs a;
    while (batch_advance(bl.q, total, per, cur, &slot)) {
        if (batch_owner(bl.start, bl.count, cur.it, own))
            a = tab[own.b];
        csr_count_body(a.idx, a.blkcnt, a.lrank, a.n, a.m, a.s, csr_nb(a.m), cur.it - own.b0,
                       smem);
    }
    if (threadIdx.x == 0)
        batch_leave(bl.q, gridDim.x);
}

// Items past the scans, when etab is set, are the final sums of another
// iteration's errors (list el, one item per problem), stored to out[k].
__global__ __launch_bounds__(256) void csr_scan_batched(const CsrArgs *__restrict__ tab,
                                                        BatchList bl,
                                                        const RmseArgs *__restrict__ etab,
                                                        BatchList el, int k, int per)
{
    __shared__ int slot;
    const int scans = bl.start[bl.count];
    const int total = scans + (etab ? el.start[el.count] : 0);
    BatchCursor cur;
    BatchOwner own;
    CsrArgs a;
    while (batch_advance(bl.q, total, per, cur, &slot)) {
        const int it = cur.it;
        if (it >= scans) {
            RmseArgs e = etab[batch_find(el.start, el.count, it - scans)];
            e.out += k;
            rmse_final_body(e, rmse_blocks_dev(e.m));
            continue;
        }
        if (batch_owner(bl.start, bl.count, it, own))
            a = tab[own.b];
        csr_scan_body(a.blkcnt, a.tot, a.n, csr_nb(a.m), it - own.b0);
    }
    if (threadIdx.x == 0)
        batch_leave(bl.q, gridDim.x);
}

__global__ __launch_bounds__(256) void csr_scatter_batched(const CsrArgs *__restrict__ tab,
                                                           BatchList bl, int per)
{
    __shared__ int slot;
    const int total = bl.start[bl.count];
    BatchCursor cur;
    BatchOwner own;
    CsrArgs a;
    while (batch_advance(bl.q, total, per, cur, &slot)) {
        if (batch_owner(bl.start, bl.count, cur.it, own))
            a = tab[own.b];
        csr_scatter_body(a.idx, a.blkcnt, a.tot, a.row_ptr, a.chunk_ptr, a.lrank, a.users,
                         a.uent, a.val, a.val_pad, a.n, a.m, a.s, csr_nb(a.m), a.chunk,
                         cur.it - own.b0, own.b1 - own.b0);
    }
    if (threadIdx.x == 0)
        batch_leave(bl.q, gridDim.x);
}

}  // namespace

int csr_blocks(int m) { return (m + kCsrBlock - 1) / kCsrBlock; }

// Items: count = signal blocks, scan = atom quads, scatter = blocks of 256 entries.
hipError_t launch_batched_csr(const CsrArgs *tab, const BatchList &count_list, int count_items,
                              const BatchList &scan_list, int scan_items,
                              const BatchList &scatter_list, int scatter_items, int max_n,
                              hipStream_t st, const RmseArgs *etab, const BatchList &el, int k)
{
    const size_t shmem = (sizeof(unsigned long long) + sizeof(int32_t)) * kWavesPerBlock * max_n;
    int wg = batch_workers((const void *)csr_count_batched, kCsrBlock, shmem, count_items);
    prof_begin(DL_K_CSR_COUNT, st);
    hipLaunchKernelGGL(csr_count_batched, dim3(wg), dim3(kCsrBlock), shmem, st, tab, count_list,
                       batch_per_ticket(count_items, wg));
    prof_end(DL_K_CSR_COUNT, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    wg = batch_workers((const void *)csr_scan_batched, 256, 0,
                       scan_items + (etab ? el.count : 0));
    prof_begin(DL_K_CSR_SCAN, st);
    hipLaunchKernelGGL(csr_scan_batched, dim3(wg), dim3(256), 0, st, tab, scan_list, etab, el,
                       k, batch_per_ticket(scan_items + (etab ? el.count : 0), wg));
    prof_end(DL_K_CSR_SCAN, st);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    wg = batch_workers((const void *)csr_scatter_batched, 256, 0, scatter_items);
    prof_begin(DL_K_CSR_SCATTER, st);
    hipLaunchKernelGGL(csr_scatter_batched, dim3(wg), dim3(256), 0, st, tab, scatter_list,
                       batch_per_ticket(scatter_items, wg));
    prof_end(DL_K_CSR_SCATTER, st);
    return hipGetLastError();
}

hipError_t launch_csr(const CsrArgs &a, hipStream_t st, const RmseArgs *err)
{
    const int nb = csr_blocks(a.m);
    const size_t shmem = (sizeof(unsigned long long) + sizeof(int32_t)) * kWavesPerBlock * a.n;
    prof_begin(DL_K_CSR_COUNT, st);
    hipLaunchKernelGGL(csr_count_kernel, dim3(nb), dim3(kCsrBlock), shmem, st, a.idx, a.blkcnt,
                       a.lrank, a.n, a.m, a.s, nb);
    prof_end(DL_K_CSR_COUNT, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    prof_begin(DL_K_CSR_SCAN, st);
    const int eb = err ? rmse_blocks_dev(err->m) : 0;
    hipLaunchKernelGGL(csr_scan_kernel, dim3((a.n + 3) / 4 + (err ? 1 : 0)), dim3(256), 0, st,
                       a.blkcnt, a.tot, a.n, nb, err ? *err : RmseArgs{}, eb);
    prof_end(DL_K_CSR_SCAN, st);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const size_t total = (size_t)a.m * a.s;
    size_t blocks = (total + 255) / 256;
    if (blocks > 8192)
        blocks = 8192;
    prof_begin(DL_K_CSR_SCATTER, st);
    hipLaunchKernelGGL(csr_scatter_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a.idx,
                       a.blkcnt, a.tot, a.row_ptr, a.chunk_ptr, a.lrank, a.users, a.uent, a.val,
                       a.val_pad, a.n, a.m, a.s, nb, a.chunk);
    prof_end(DL_K_CSR_SCATTER, st);
    return hipGetLastError();
}

}  // namespace dlk
