// Atom-update stage (step 2 of the DL iteration): the group loop of Alg. 2
// with the AK-SVD rule of eq. (5) (or SGK, eq. 6), and the error.
//
// For group l (atoms [a0, a1)), every atom j of the group reads the same
// group-start dictionary, representations and error E (the rule of eq. 2):
//   pass 1 : g_j = F x_j^T = sum_{i in I_j} (e_i + d_j x_ji) x_ji   (eq. 3)
//            over chunks of kChunk users, one workgroup per chunk, partial
//            sums written per chunk (no float atomics);
//   pass 2 : per chunk, g_j summed over the atom's chunks in chunk order and
//            d_j' = g_j / ||g_j|| (eq. 5, first line; SGK's least-squares
//            atom has the same direction), written to the next dictionary Dn
//            by the atom's first chunk; then the AK-SVD refresh
//            x_ji' = (e_i + d_j x_ji)^T d_j' (eq. 5, second line) to valn;
//   E      : for group sizes below n, E is brought up to date for the next
//            group: e_i += d_j x_ji - d_j' x_ji' over the group's atoms that
//            signal i uses (the incremental error update the paper mentions
//            in Sec. 3), one signal at a time, so no two writers meet.
//
// Lane mapping of the per-user work: a user's p-vector is split over LPU
// lanes (LPU = power of two >= p/4), each lane owning 4 consecutive
// coordinates (float4), so one wave handles 64/LPU users at once.
#include "dl_internal.h"
#include "rmse_body.h"

namespace dlk {
namespace {



// Atom of global chunk gc among atoms [a0, a1): chunk_ptr[j] <= gc < chunk_ptr[j+1].
__device__ inline int chunk_atom(const int32_t *chunk_ptr, int a0, int a1, int gc)
{
    int lo = a0, hi = a1 - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (chunk_ptr[mid] <= gc)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// ---- pass 1: partial F x^T per chunk ------------------------------------
// The chunk's ELL positions and coefficients are staged in LDS first, so the
// residual rows of several users are in flight at once.
__device__ inline void pass1_body(const UpdateArgs &a, int a0, int a1, int blk, int nblk)
{
    __shared__ f32x4 red[4][64];
    __shared__ int sPos[kChunk];
    __shared__ float sX[kChunk];
    const int p = a.p, s = a.s;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lpu = lanes_per_user(p);
    const int upw = 64 / lpu;       // users per wave step
    const int sub = lane / lpu;     // user slot of this lane
    const int q = 4 * (lane % lpu); // first coordinate of this lane
    const int cbase = a.chunk_ptr[a0];
    const int nch = a.chunk_ptr[a1] - cbase;
    for (int c = blk; c < nch; c += nblk) {
        const int gc = cbase + c;
        const int j = chunk_atom(a.chunk_ptr, a0, a1, gc);
        const int u0 = a.row_ptr[j] + (gc - a.chunk_ptr[j]) * a.chunk;
        const int cnt = min(a.chunk, a.row_ptr[j + 1] - u0);
        for (int r = threadIdx.x; r < cnt; r += blockDim.x) {
            const int2 ue = a.uent[u0 + r];
            sPos[r] = ue.x;
            sX[r] = __int_as_float(ue.y);
        }
        __syncthreads();
        const f32x4 d = load4(a.D + (size_t)j * p, q, p);
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        const int stride = 4 * upw;
        // the residual rows of U users per lane are loaded before any is
        // used (in flight together); they are summed in user order
        constexpr int U = 8;
        for (int rb = wave * upw + sub; rb < cnt; rb += stride * U) {
            f32x4 e[U];
            float x[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int r = rb + u * stride;
                const bool on = r < cnt;
                x[u] = on ? sX[r] : 0.f;
                e[u] = on ? load4(a.E + (size_t)(sPos[r] / s) * p, q, p)
                          : f32x4{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (rb + u * stride < cnt)
                    acc += (e[u] + d * x[u]) * x[u];
        }
        // sum over the user slots of the wave (lanes with the same q)
        for (int off = lpu; off < 64; off <<= 1) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                acc[r] = off >= 16 ? sum_xor(acc[r], off) : acc[r] + __shfl_xor(acc[r], off);
        }
        red[wave][lane] = acc;
        __syncthreads();
        if (wave == 0 && lane < lpu && q < p) {
            const f32x4 t = red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
            *reinterpret_cast<f32x4 *>(a.partial + (size_t)gc * p + q) = t;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void pass1_kernel(UpdateArgs a, int a0, int a1)
{
    pass1_body(a, a0, a1, blockIdx.x, gridDim.x);
}

template <int CTRL, bool BC>
__device__ inline int dpp_i(int x)
{
    return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, BC);
}

// Integer sum over the wave (every lane gets it): within rows by DPP, across
// rows by reading one lane of each row.  Integer addition is exact, so the
// order is free.
__device__ inline int wave_sum_i32(int x)
{
    x += dpp_i<0xB1, false>(x);   // quad_perm [1, 0, 3, 2]
    x += dpp_i<0x4E, false>(x);   // quad_perm [2, 3, 0, 1]
    x += dpp_i<0x141, false>(x);  // row_half_mirror
    x += dpp_i<0x140, false>(x);  // row_mirror
    return __builtin_amdgcn_readlane(x, 0) + __builtin_amdgcn_readlane(x, 16) +
           __builtin_amdgcn_readlane(x, 32) + __builtin_amdgcn_readlane(x, 48);
}

// Inclusive prefix sum over the wave's lanes: a scan inside each row of 16 by
// DPP row shifts (lanes shifted in from outside the row read 0), then the
// totals of the earlier rows.
__device__ inline int wave_scan_i32(int x)
{
    x += dpp_i<0x111, true>(x);  // row_shr:1
    x += dpp_i<0x112, true>(x);  // row_shr:2
    x += dpp_i<0x114, true>(x);  // row_shr:4
    x += dpp_i<0x118, true>(x);  // row_shr:8
    const int t0 = __builtin_amdgcn_readlane(x, 15);
    const int t1 = __builtin_amdgcn_readlane(x, 31);
    const int t2 = __builtin_amdgcn_readlane(x, 47);
    const int row = (int)(threadIdx.x & 63) >> 4;
    return x + (row >= 1 ? t0 : 0) + (row >= 2 ? t1 : 0) + (row >= 3 ? t2 : 0);
}

__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---- pass 1 by signal blocks (all atoms in one group) ---------------------
// Item (signal block b, atom range r): the range holds one atom per lane
// group of the workgroup (256 / LPU atoms).  The block's entries (signal,
// slot) are split over the four waves in contiguous runs, loaded into
// registers at once.  Each wave counts its entries of the range's atoms per
// atom, and compacts them, in order, into its own run of an LDS list (ballot
// and bit count); the counts give every (atom, wave) pair a place in the
// atoms' lists, and each wave ranks its compacted entries in order (LDS bit
// masks per atom, as in the CSR count) and writes them there, so every
// atom's list holds its users of the block in (signal, slot) order.  Each
// lane group then sums g_jb = sum (e_i + d_j x_ji) x_ji over its atom's list
// in that order, with the residual rows of U users per lane loaded before
// any is used, and stores g_jb and the block's user count.  Pass 2 sums an
// atom's block sums in block order.  Items are numbered so that the ranges
// of one signal block share a blockIdx residue mod 8: they run on one XCD,
// whose L2 then serves the block's entries and residual rows to all of them.
__device__ inline void gsum_item(int it, int nr, int nsb, int &b, int &r)
{
    const int g = it / (8 * nr), w = it - g * 8 * nr;
    const int nl = min(8, nsb - 8 * g);  // blocks in this group of eight
    b = 8 * g + w % nl;
    r = w / nl;
}

constexpr int kGsumRows = 8;  // residual rows in flight per lane

// W waves per workgroup (64 W threads): 64 W / LPU atoms per range, at most
// 64 (the caller keeps W <= LPU).  The sums do not depend on W or on the
// ranges, only on the signal blocks.
template <int W>
__device__ inline void gsum_body(const UpdateArgs &a, int a0, int a1, int blk, int nblk)
{
    __shared__ unsigned short pool[kGsumPool];  // the atoms' lists (entries of the block)
    __shared__ unsigned short ce[kGsumPool];    // each wave's entries of the range's atoms
    __shared__ unsigned char ck[kGsumPool];     // and their atoms within the range
    __shared__ int wcnt[W][64];
    __shared__ unsigned long long wmask[W][64];
    __shared__ int seg0[64], segn[64];
    __shared__ int wbase[W];
    const int p = a.p, s = a.s;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lpu = lanes_per_user(p);
    const int R = 64 * W / lpu;  // atoms per range
    const int nr = (a1 - a0 + R - 1) / R;
    const int B = a.sig_block, nsb = a.nsb;
    const int grp = threadIdx.x / lpu;  // atom of this lane group within the range
    const int q = 4 * (lane % lpu);
    const unsigned long long bit = 1ull << lane;
    const unsigned long long lower = bit - 1ull;
    // signal of entry e: floor((e + 1/2) / s) in FP32 is exact for entries
    // below 2^13 (an error under 1e-3 against a distance of at least 1/(2s)
    // from the next integer)
    const float inv_s = 1.0f / (float)s;
    for (int it = blk; it < nr * nsb; it += nblk) {
        int b, r;
        gsum_item(it, nr, nsb, b, r);
        const int lo = a0 + r * R;
        const int rr = min(R, a1 - lo);
        const int i0 = b * B;
        const int len = (min(a.m, i0 + B) - i0) * s;
        const size_t e0 = (size_t)i0 * s;
        const int per = ((len + 64 * W - 1) / (64 * W)) * 64;  // entries per wave
        const int w0 = min(len, wave * per), w1 = min(len, w0 + per);
        // this lane's entries w0 + lane + 64 c, as atoms of the range (-1:
        // another atom or an unused slot), all loaded before any is used
        constexpr int kPer = kGsumPool / (64 * W);
        int kk[kPer];
#pragma unroll
        for (int c = 0; c < kPer; ++c) {
            const int e = w0 + lane + 64 * c;
            int k = -1;
            if (e < w1) {
                k = a.idx[e0 + e] - lo;
                if ((unsigned)k >= (unsigned)rr)
                    k = -1;
            }
            kk[c] = k;
        }
        __syncthreads();  // the previous item's lists are no longer read
        for (int t = threadIdx.x; t < W * 64; t += blockDim.x) {
            (&wcnt[0][0])[t] = 0;
            (&wmask[0][0])[t] = 0ull;
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < kPer; ++c)
            if (kk[c] >= 0)
                atomicAdd(&wcnt[wave][kk[c]], 1);
        __syncthreads();
        if (wave == 0) {
            int v[W];
            int tot = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) {
                v[w] = lane < rr ? wcnt[w][lane] : 0;
                tot += v[w];
            }
            const int x = wave_scan_i32(tot);
            const int ex = x - tot;
            seg0[lane] = ex;
            segn[lane] = tot;
            // per (wave, atom) offsets, and each wave's compacted run after
            // the earlier waves' runs
            int run = ex, before = 0, wb = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) {
                wcnt[w][lane] = run;
                run += v[w];
                const int tw = wave_sum_i32(v[w]);
                wb = lane == w ? before : wb;
                before += tw;
            }
            if (lane < W)
                wbase[lane] = wb;
        }
        __syncthreads();
        // compaction of the wave's entries of the range's atoms, in order
        const int cb0 = wbase[wave];
        int cb = cb0;
#pragma unroll
        for (int c = 0; c < kPer; ++c) {
            if (w0 + 64 * c >= w1)
                break;  // uniform over the wave
            const unsigned long long m = __ballot(kk[c] >= 0);
            if (kk[c] >= 0) {
                const int pos = cb + __popcll(m & lower);
                ce[pos] = (unsigned short)(w0 + lane + 64 * c);
                ck[pos] = (unsigned char)kk[c];
            }
            cb += __popcll(m);
        }
        wave_lds_sync();
        // ranks among the wave's compacted entries of each atom, in order
        for (int cbase = cb0; cbase < cb; cbase += 64) {
            const int ci = cbase + lane;
            const int k = ci < cb ? (int)ck[ci] : -1;
            const int e = ci < cb ? (int)ce[ci] : 0;
            if (k >= 0)
                atomicOr(&wmask[wave][k], bit);
            wave_lds_sync();
            unsigned long long mm = 0;
            int base = 0;
            if (k >= 0) {
                mm = wmask[wave][k];
                base = wcnt[wave][k];
                pool[base + __popcll(mm & lower)] = (unsigned short)e;
            }
            wave_lds_sync();
            if (k >= 0 && lane == 63 - __clzll((long long)mm)) {
                wcnt[wave][k] = base + __popcll(mm);
                wmask[wave][k] = 0ull;
            }
            wave_lds_sync();
        }
        __syncthreads();
        if (grp < rr) {
            const int j = lo + grp;
            const int u0 = seg0[grp], cnt = segn[grp];
            const f32x4 d = load4(a.D + (size_t)j * p, q, p);
            const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
            f32x4 acc = zero;
            constexpr int U = kGsumRows;
            for (int ub = 0; ub < cnt; ub += U) {
                f32x4 er[U];
                float x[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const bool on = ub + u < cnt;
                    const int e = on ? (int)pool[u0 + ub + u] : 0;
                    const int il = (int)(((float)e + 0.5f) * inv_s);
                    x[u] = on ? a.val[e0 + e] : 0.f;
                    er[u] = on ? load4(a.E + (size_t)(i0 + il) * p, q, p) : zero;
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (ub + u < cnt)
                        acc += (er[u] + d * x[u]) * x[u];
            }
            const size_t row = (size_t)(j - a0) * nsb + b;
            if (q < p)
                *reinterpret_cast<f32x4 *>(a.partial + row * p + q) = acc;
            if (lane % lpu == 0)
                a.bcnt[row] = cnt;
        }
    }
}

// The optional last workgroup sums a carried error's partials.
template <int W>
__global__ __launch_bounds__(64 * W) void gsum_kernel(UpdateArgs a, int a0, int a1, RmseArgs err,
                                                      int eb)
{
    if (eb > 0 && blockIdx.x == gridDim.x - 1) {
        rmse_final_body(err, eb);
        return;
    }
    gsum_body<W>(a, a0, a1, blockIdx.x, gridDim.x - (eb > 0 ? 1 : 0));
}

// ---- pass 2: d_j' and the AK-SVD representation refresh ------------------
// Every chunk of atom j sums the atom's chunk partials in chunk order (so
// every chunk gets the same bits), normalises (d_j' = g_j / ||g_j||, eq. 5
// first line; SGK's least-squares atom has the same direction) and refreshes
// its users x_ji' = (e_i + d_j x_ji)^T d_j' (eq. 5, second line).  The first
// chunk of the atom writes d_j' to Dn and the atom's state.  Atoms without
// users keep d_j; the items after the chunks handle them.
__device__ inline float block_sum_f32(float v, float *red4)
{
    v = wave_sum_f32(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        red4[threadIdx.x >> 6] = v;
    __syncthreads();
    return ((red4[0] + red4[1]) + red4[2]) + red4[3];
}

// Sum of cnt rows (stride p) from src, in row order, loads sixteen at a time.
__device__ inline float sum_rows(const float *src, int cnt, int p)
{
    float g = 0.f;
    int c = 0;
    for (; c + 16 <= cnt; c += 16) {
        float v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u)
            v[u] = src[(size_t)(c + u) * p];
#pragma unroll
        for (int u = 0; u < 16; ++u)
            g += v[u];
    }
    for (; c < cnt; ++c)
        g += src[(size_t)c * p];
    return g;
}

// g_j, coordinate t = threadIdx.x < p (workgroup-wide: every thread calls
// it): the atom's partials summed in order, those of its user chunks
// [c0, c1), or, with pass 1 by signal blocks, its block sums: the workgroup
// splits them into W contiguous runs (W = 256 / P, P the power of two >= p),
// sums each run in block order, and adds the run sums in run order.
__device__ inline float atom_g(const UpdateArgs &a, int j, int a0, int c0, int c1, int t)
{
    const int p = a.p;
    if (!a.sig_block)
        return t < p ? sum_rows(a.partial + (size_t)c0 * p + t, c1 - c0, p) : 0.f;
    __shared__ float sg[256];
    int P = 1;
    while (P < p)
        P <<= 1;
    const int W = 256 / P;
    const int tc = threadIdx.x % P, part = threadIdx.x / P;
    const int per = (a.nsb + W - 1) / W;
    const int b0 = min(a.nsb, part * per), b1 = min(a.nsb, b0 + per);
    const float g = tc < p ? sum_rows(a.partial + ((size_t)(j - a0) * a.nsb + b0) * p + tc,
                                      b1 - b0, p)
                           : 0.f;
    __syncthreads();  // sg of the previous atom is no longer read
    sg[threadIdx.x] = g;
    __syncthreads();
    float r = 0.f;
    if (t < p)
        for (int w = 0; w < W; ++w)
            r += sg[w * P + t];
    return r;
}

// x' = (e + d x)^T d', formed as e^T d' + x (d^T d') with cj = d^T d' (the
// same value with one atom row per user instead of two), for the chunk's
// users staged in sPos/sX; every lane of
// the wave runs the same trip count (shuffles below), and the residual rows
// of U users per lane are loaded before any of them is used, so their loads
// are in flight together.
template <int U>
__device__ inline void pass2_refresh(const UpdateArgs &a, float cj, f32x4 dn, const int *sPos,
                                     const float *sX, int cnt, int wave, int lane, int lpu,
                                     int upw, int sub, int q)
{
    const int p = a.p, s = a.s;
    const int stride = 4 * upw;
    for (int rb = wave * upw; rb < cnt; rb += stride * U) {
        f32x4 e[U];
        float x[U];
        int pos[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = rb + u * stride + sub;
            const bool on = r < cnt;
            pos[u] = on ? sPos[r] : -1;
            x[u] = on ? sX[r] : 0.f;
            e[u] = on ? load4(a.E + (size_t)(pos[u] / s) * p, q, p) : f32x4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            float part = e[u][0] * dn[0] + e[u][1] * dn[1] + e[u][2] * dn[2] + e[u][3] * dn[3];
            part = lanes_sum(part, lpu);
            if (pos[u] >= 0 && (lane % lpu) == 0)
                a.valn[pos[u]] = part + x[u] * cj;
        }
    }
}

// U: residual rows in flight per lane in the refresh (a template parameter,
// so that each choice is a kernel with its own register allocation), or 0:
// 8 for signal sizes up to 64, else 4, chosen in the kernel.  Short signals
// use U = 0 (measured 2% faster for pass 2 at p = 64 than U = 8, with the
// same registers), long ones U = 4.
template <int U>
__device__ inline void pass2_body(const UpdateArgs &a, int a0, int a1, int blk, int nblk)
{
    __shared__ int sPos[kChunk];
    __shared__ float sX[kChunk];
    __shared__ float sDn[256];
    __shared__ float red4[4];
    const int p = a.p;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lpu = lanes_per_user(p);
    const int upw = 64 / lpu;
    const int sub = lane / lpu;
    const int q = 4 * (lane % lpu);
    const int t = threadIdx.x;  // coordinate of d_j' owned by this thread
    if (a.no_refresh) {
        // d' only (the error pass refreshes X): item blk takes atoms blk,
        // blk + nblk, ... of the group, each summing its chunk partials in
        // chunk order; atoms without users keep d_j
        for (int j = a0 + blk; j < a1; j += nblk) {
            int c0 = 0, c1 = 0;
            if (a.sig_block) {  // users counted per signal block
                int used = 0;
                for (int bb = t; bb < a.nsb; bb += blockDim.x)
                    used |= a.bcnt[(size_t)(j - a0) * a.nsb + bb];
                c1 = __syncthreads_or(used) ? 1 : 0;
            } else {
                c0 = a.chunk_ptr[j];
                c1 = a.chunk_ptr[j + 1];
            }
            if (c0 == c1) {  // uniform
                for (int k = t; k < p; k += blockDim.x)
                    a.Dn[(size_t)j * p + k] = a.D[(size_t)j * p + k];
                if (t == 0) {
                    a.atom_state[j] = 1;
                    atomicAdd(&a.ctl->unused_atoms, 1ull);
                }
                continue;
            }
            const float g = atom_g(a, j, a0, c0, c1, t);
            const float sq = block_sum_f32(g * g, red4);
            const int state = sq > 0.f ? 0 : 2;
            const float inv = state == 0 ? 1.0f / sqrtf(sq) : 0.f;
            const float dt = t < p ? a.D[(size_t)j * p + t] : 0.f;
            const float dnt = state == 0 ? g * inv : dt;
            if (t < p)
                a.Dn[(size_t)j * p + t] = dnt;
            const float cj = block_sum_f32(dt * dnt, red4);  // d^T d' for the refresh
            if (t == 0) {
                a.atom_cos[j] = cj;
                a.atom_state[j] = state;
                if (state == 2) {
                    atomicAdd(&a.ctl->zero_updates, 1ull);
                    if (!(sq == 0.f))
                        atomicAdd(&a.ctl->nonfinite, 1ull);
                }
            }
        }
        return;
    }
    const int cbase = a.chunk_ptr[a0];
    const int nch = a.chunk_ptr[a1] - cbase;
    for (int c = blk; c < nch; c += nblk) {
        const int gc = cbase + c;
        const int j = chunk_atom(a.chunk_ptr, a0, a1, gc);
        const int c0 = a.chunk_ptr[j], c1 = a.chunk_ptr[j + 1];
        if (a.no_refresh && gc != c0)
            continue;  // only the atom's first chunk forms d' (uniform branch)
        const int u0 = a.row_ptr[j] + (gc - c0) * a.chunk;
        const int cnt = min(a.chunk, a.row_ptr[j + 1] - u0);
        const float g = atom_g(a, j, a0, c0, c1, t);
        const float sq = block_sum_f32(g * g, red4);
        const int state = sq > 0.f ? 0 : 2;  // 2: F x^T = 0 (or not finite): unchanged
        const float inv = state == 0 ? 1.0f / sqrtf(sq) : 0.f;
        const float dt = t < p ? a.D[(size_t)j * p + t] : 0.f;
        const float dnt = state == 0 ? g * inv : dt;
        if (t < p) {
            sDn[t] = dnt;
            if (gc == c0)
                a.Dn[(size_t)j * p + t] = dnt;
        }
        const float cj = block_sum_f32(dt * dnt, red4);  // d^T d' for the refresh
        if (gc == c0 && t == 0) {
            a.atom_cos[j] = cj;
            a.atom_state[j] = state;
            if (state == 2) {
                atomicAdd(&a.ctl->zero_updates, 1ull);
                if (!(sq == 0.f))
                    atomicAdd(&a.ctl->nonfinite, 1ull);
            }
        }
        if (a.no_refresh)
            continue;  // the error pass refreshes X
        // kept: other rules, atoms not updated, and (as in the error pass's
        // refresh) a d^T d' that is not a number
        const bool keep = a.rule != DL_RULE_AKSVD || state != 0 || cj != cj;
        for (int r = threadIdx.x; r < cnt; r += blockDim.x) {
            const int2 ue = a.uent[u0 + r];
            sPos[r] = ue.x;
            sX[r] = __int_as_float(ue.y);
        }
        __syncthreads();
        if (keep) {
            for (int r = threadIdx.x; r < cnt; r += blockDim.x)
                a.valn[sPos[r]] = sX[r];
        } else {
            const f32x4 dn = q < p ? *reinterpret_cast<const f32x4 *>(sDn + q)
                                   : f32x4{0.f, 0.f, 0.f, 0.f};
            if (U > 0)
                pass2_refresh<(U > 0 ? U : 4)>(a, cj, dn, sPos, sX, cnt, wave, lane, lpu, upw,
                                                sub, q);
            else if (lpu <= 16)
                pass2_refresh<8>(a, cj, dn, sPos, sX, cnt, wave, lane, lpu, upw, sub, q);
            else
                pass2_refresh<4>(a, cj, dn, sPos, sX, cnt, wave, lane, lpu, upw, sub, q);
        }
        __syncthreads();
    }
    // atoms without users: d_j unchanged (one wave per atom)
    for (int qd = blk; qd < (a1 - a0 + 3) / 4; qd += nblk) {
        const int j = a0 + 4 * qd + wave;
        if (j >= a1 || a.chunk_ptr[j + 1] != a.chunk_ptr[j])
            continue;
        for (int k = lane; k < p; k += 64)
            a.Dn[(size_t)j * p + k] = a.D[(size_t)j * p + k];
        if (lane == 0) {
            a.atom_state[j] = 1;
            atomicAdd(&a.ctl->unused_atoms, 1ull);
        }
    }
}

template <int U>
__global__ __launch_bounds__(256) void pass2_kernel(UpdateArgs a, int a0, int a1)
{
    pass2_body<U>(a, a0, a1, blockIdx.x, gridDim.x);
}

// ---- incremental error update after a group (group sizes below n) -------
// One lane group per entry of the group's CSR range; the entry that holds the
// signal's first slot inside the group applies all of that signal's changes.
__global__ __launch_bounds__(256) void eupdate_kernel(UpdateArgs a, int a0, int a1)
{
    const int p = a.p, s = a.s;
    const int lane = threadIdx.x & 63;
    const int lpu = lanes_per_user(p);
    const int upw = 64 / lpu;
    const int sub = lane / lpu;
    const int q = 4 * (lane % lpu);
    const int e0 = a.row_ptr[a0], e1 = a.row_ptr[a1];
    const int wpg = blockDim.x >> 6;
    const int wid = blockIdx.x * wpg + (threadIdx.x >> 6);
    const int nw = gridDim.x * wpg;
    for (int base = e0 + wid * upw; base < e1; base += nw * upw) {
        const int u = base + sub;
        if (u >= e1)
            continue;
        const int pos = a.uent[u].x;
        const int i = pos / s;
        const int t0 = pos - i * s;
        const int32_t *row = a.idx + (size_t)i * s;
        bool first = true;
        for (int t = 0; t < t0; ++t) {
            const int jt = row[t];
            if (jt >= a0 && jt < a1)
                first = false;
        }
        if (!first || q >= p)
            continue;
        f32x4 e = *reinterpret_cast<const f32x4 *>(a.E + (size_t)i * p + q);
        for (int t = t0; t < s; ++t) {
            const int jt = row[t];
            if (jt < a0 || jt >= a1)
                continue;
            const float xo = a.val[(size_t)i * s + t];
            const float xn = a.valn[(size_t)i * s + t];
            const f32x4 dold = *reinterpret_cast<const f32x4 *>(a.D + (size_t)jt * p + q);
            const f32x4 dnew = *reinterpret_cast<const f32x4 *>(a.Dn + (size_t)jt * p + q);
            e += dold * xo - dnew * xn;
        }
        *reinterpret_cast<f32x4 *>(a.E + (size_t)i * p + q) = e;
    }
}

template <bool REFRESH>
__global__ __launch_bounds__(256) void rmse_kernel(RmseArgs a)
{
    if constexpr (REFRESH)
        rmse_refresh_body(a, blockIdx.x, gridDim.x);
    else
        rmse_body(a, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(256) void rmse_pf_kernel(RmseArgs a)
{
    rmse_refresh_body_pf(a, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(256) void rmse_final_kernel(RmseArgs a, int nblk)
{
    rmse_final_body(a, nblk);
}

__global__ __launch_bounds__(256) void residual_kernel(const float *__restrict__ Y,
                                                       const float *__restrict__ D,
                                                       const int32_t *__restrict__ idx,
                                                       const float *__restrict__ val,
                                                       float *__restrict__ E, int p, int n, int m,
                                                       int s)
{
    const int lane = threadIdx.x & 63;
    const int lpu = lanes_per_user(p);
    const int upw = 64 / lpu;
    const int sub = lane / lpu;
    const int q = 4 * (lane % lpu);
    const int wid = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int nw = gridDim.x * 4;
    for (int i = wid * upw + sub; i < m; i += nw * upw) {
        if (q >= p)
            continue;
        f32x4 e = *reinterpret_cast<const f32x4 *>(Y + (size_t)i * p + q);
        for (int t = 0; t < s; ++t) {
            const int j = idx[(size_t)i * s + t];
            if (j < 0 || j >= n)
                continue;
            e -= *reinterpret_cast<const f32x4 *>(D + (size_t)j * p + q) * val[(size_t)i * s + t];
        }
        *reinterpret_cast<f32x4 *>(E + (size_t)i * p + q) = e;
    }
}

__device__ inline void normalize_body(float *D, int n, int p, Control *ctl, int blk)
{
    const int lane = threadIdx.x & 63;
    const int j = blk * 4 + (threadIdx.x >> 6);
    if (j >= n)
        return;
    float v[4];
    float sq = 0.f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int q = lane + 64 * r;
        v[r] = q < p ? D[(size_t)j * p + q] : 0.f;
        sq += v[r] * v[r];
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        sq += __shfl_xor(sq, off);
    if (!isfinite(sq) && lane == 0)
        atomicAdd(&ctl->nonfinite, 1ull);
    // zero atoms stay zero; atoms already of unit norm (to FP32 rounding) are
    // left bit-for-bit as they are, so a run resumed from a saved dictionary
    // continues exactly
    if (!(sq > 0.f) || fabsf(sq - 1.0f) <= 4e-7f)
        return;
    const float inv = 1.0f / sqrtf(sq);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int q = lane + 64 * r;
        if (q < p)
            D[(size_t)j * p + q] = v[r] * inv;
    }
}

__global__ __launch_bounds__(256) void normalize_kernel(float *D, int n, int p, Control *ctl)
{
    normalize_body(D, n, p, ctl, blockIdx.x);
}

// ---- batched problems (one group per problem: atoms [0, n)) --------------
// Items: pass 1 = chunk slots, or (signal block, atom range) pairs with pass
// 1 by signal blocks; pass 2 = chunk slots (an upper bound of the chunks; the
// excess leaves at once, and pass 2's slots also cover the atom quads of its
// unused-atom step), error = signal blocks,
// normalisation = atom quads.
template <int STAGE>
__global__ __launch_bounds__(256) void update_batched(const UpdateArgs *__restrict__ tab,
                                                      BatchList bl, int per)
{
    __shared__ int slot;
    const int total = bl.start[bl.count];
    BatchCursor cur;
    BatchOwner own;
    UpdateArgs a;
    while (batch_advance(bl.q, total, per, cur, &slot)) {
        if (batch_owner(bl.start, bl.count, cur.it, own))
            a = tab[own.b];
        const int t = cur.it - own.b0, nt = own.b1 - own.b0;
        if (STAGE == 0) {
            if (a.sig_block)
                gsum_body<4>(a, 0, a.n, t, nt);
            else
                pass1_body(a, 0, a.n, t, nt);
        } else
            pass2_body<4>(a, 0, a.n, t, nt);
    }
    if (threadIdx.x == 0)
        batch_leave(bl.q, gridDim.x);
}

// Block partials of every problem; the error of iteration k then goes to
// out[k] of every problem (rmse_final_batched).
__global__ __launch_bounds__(256) void rmse_batched(const RmseArgs *__restrict__ tab, BatchList bl,
                                                    int per)
{
    __shared__ int slot;
    const int total = bl.start[bl.count];
    BatchCursor cur;
    BatchOwner own;
    RmseArgs a;
    while (batch_advance(bl.q, total, per, cur, &slot)) {
        if (batch_owner(bl.start, bl.count, cur.it, own))
            a = tab[own.b];
        rmse_body(a, cur.it - own.b0, own.b1 - own.b0);
    }
    if (threadIdx.x == 0)
        batch_leave(bl.q, gridDim.x);
}

// One item per problem: its block partials in block order.
__global__ __launch_bounds__(256) void rmse_final_batched(const RmseArgs *__restrict__ tab,
                                                          BatchList bl, int k)
{
    __shared__ int slot;
    const int total = bl.start[bl.count];
    for (;;) {
        const int it = batch_next_item(bl.q, &slot);
        if (it >= total)
            break;
        const int b = batch_find(bl.start, bl.count, it);
        RmseArgs a = tab[b];
        a.out += k;
        rmse_final_body(a, rmse_blocks_dev(a.m));
    }
    if (threadIdx.x == 0)
        batch_leave(bl.q, gridDim.x);
}

__global__ __launch_bounds__(256) void normalize_batched(const NormArgs *__restrict__ tab,
                                                         BatchList bl, int per)
{
    __shared__ int slot;
    const int total = bl.start[bl.count];
    BatchCursor cur;
    BatchOwner own;
    NormArgs a;
    while (batch_advance(bl.q, total, per, cur, &slot)) {
        if (batch_owner(bl.start, bl.count, cur.it, own))
            a = tab[own.b];
        normalize_body(a.D, a.n, a.p, a.ctl, cur.it - own.b0);
    }
    if (threadIdx.x == 0)
        batch_leave(bl.q, gridDim.x);
}

__global__ void copy_kernel(const uint32_t *__restrict__ src, uint32_t *__restrict__ dst,
                            size_t words)
{
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < words;
         k += (size_t)gridDim.x * blockDim.x)
        dst[k] = src[k];
}

__global__ void zero_kernel(uint32_t *__restrict__ dst, size_t words)
{
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < words;
         k += (size_t)gridDim.x * blockDim.x)
        dst[k] = 0u;
}

unsigned grid_for(size_t items, unsigned cap)
{
    size_t b = (items + 255) / 256;
    if (b < 1)
        b = 1;
    return (unsigned)(b > cap ? cap : b);
}

}  // namespace

int rmse_blocks(int m) { return rmse_blocks_dev(m); }

// Deferred (carried by the next iteration's launches) up to 16384 signals:
// measured faster there, and slower at 262144, where the partial workgroups
// each stride over many blocks and form a tail behind the product tiles.
bool error_defer_ok(int m) { return m <= 16384; }

int chunk_users(const dl_params &prm) { return prm.group_size >= prm.n ? kChunk : kChunk / 2; }

int max_chunks(const dl_params &prm)
{
    const long long ms = (long long)prm.m * prm.s;
    const int ch = chunk_users(prm);
    return (int)((ms + ch - 1) / ch) + prm.n;
}

static int host_lanes_per_user(int p)
{
    int l = 1;
    while (4 * l < p)
        l <<= 1;
    return l;
}

int gsum_block(const dl_params &prm)
{
    if (prm.group_size < prm.n || prm.p < 16)
        return 0;
    const int R = 256 / host_lanes_per_user(prm.p);
    if ((prm.n + R - 1) / R > 32)
        return 0;
    // about kGsumBlocks blocks, in multiples of 64 signals, within the pool
    int B = (prm.m + kGsumBlocks - 1) / kGsumBlocks;
    B = (B + 63) / 64 * 64;
    const int cap = kGsumPool / prm.s / 64 * 64;
    return B < cap ? B : cap;
}

int gsum_signal_blocks(const dl_params &prm)
{
    const int B = gsum_block(prm);
    return B ? (prm.m + B - 1) / B : 0;
}

int gsum_items(const dl_params &prm)
{
    const int R = 256 / host_lanes_per_user(prm.p);
    return gsum_signal_blocks(prm) * ((prm.n + R - 1) / R);
}

// Waves per workgroup of a single problem's pass 1 by signal blocks: the most
// (up to 16, and at most LPU, so that a range holds at most 64 atoms) whose
// items still number at least kGsumMinItems (measured at p = 64, n = 256:
// m = 16384 takes 8, 336 -> 345 M signals*iters/s against 4, where 16 gave
// 340 M; m = 262144 takes 16, 547 -> 578 M).
constexpr int kGsumMinItems = 512;
static int gsum_waves(int p, int n, int nsb)
{
    const int lpu = host_lanes_per_user(p);
    int w = 4;
    for (int c = 8; c <= 16 && c <= lpu; c *= 2) {
        const int R = 64 * c / lpu;
        if ((long long)nsb * ((n + R - 1) / R) >= kGsumMinItems)
            w = c;
    }
    return w;
}

hipError_t launch_update(const UpdateArgs &a, hipStream_t st, const RmseArgs *err)
{
    const int gs = a.group_size >= a.n ? a.n : a.group_size;
    for (int a0 = 0; a0 < a.n; a0 += gs) {
        const int a1 = a0 + gs < a.n ? a0 + gs : a.n;
        // upper bound of the group's chunks: each atom has at most m users
        const long long users_ub = (long long)a.m * (a1 - a0) < (long long)a.m * a.s
                                       ? (long long)a.m * (a1 - a0)
                                       : (long long)a.m * a.s;
        long long chunks_ub = (users_ub + a.chunk - 1) / a.chunk + (a1 - a0);
        if (chunks_ub > a.max_chunks)
            chunks_ub = a.max_chunks;
        const unsigned grid = (unsigned)(chunks_ub > 2048 ? 2048 : (chunks_ub < 1 ? 1 : chunks_ub));
        prof_begin(DL_K_UPD_PASS1, st);
        if (a.sig_block) {
            // one group (a0 = 0, a1 = n); at most 4096 workgroups, a multiple
            // of 8 when the items are more, so an item keeps its XCD
            const int W = gsum_waves(a.p, a1 - a0, a.nsb);
            const int R = 64 * W / host_lanes_per_user(a.p);
            const int items = a.nsb * ((a1 - a0 + R - 1) / R);
            const int g1 = items < 4096 ? items : 4096;
            const int eb = err ? rmse_blocks_dev(err->m) : 0;
            const dim3 grid(g1 + (err ? 1 : 0));
            const RmseArgs e = err ? *err : RmseArgs{};
            if (W == 16)
                hipLaunchKernelGGL(gsum_kernel<16>, grid, dim3(1024), 0, st, a, a0, a1, e, eb);
            else if (W == 8)
                hipLaunchKernelGGL(gsum_kernel<8>, grid, dim3(512), 0, st, a, a0, a1, e, eb);
            else
                hipLaunchKernelGGL(gsum_kernel<4>, grid, dim3(256), 0, st, a, a0, a1, e, eb);
        } else {
            hipLaunchKernelGGL(pass1_kernel, dim3(grid), dim3(256), 0, st, a, a0, a1);
        }
        prof_end(DL_K_UPD_PASS1, st);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
        prof_begin(DL_K_UPD_PASS2, st);
        // residual rows in flight per lane: 8 for short signals, 4 for long
        // ones (measured: 8 is 5% faster at p = 64 and 20% slower at p = 256,
        // where the 8-row kernel holds more registers)
        // with the refresh in the error pass, pass 2 takes one item per atom
        const unsigned g2 = a.no_refresh ? (unsigned)(a1 - a0 < 2048 ? a1 - a0 : 2048) : grid;
        if (a.p <= 64)
            hipLaunchKernelGGL(pass2_kernel<0>, dim3(g2), dim3(256), 0, st, a, a0, a1);
        else
            hipLaunchKernelGGL(pass2_kernel<4>, dim3(g2), dim3(256), 0, st, a, a0, a1);
        prof_end(DL_K_UPD_PASS2, st);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
        if (a1 < a.n) {
            const unsigned eg = grid_for((size_t)users_ub * 16, 2048);
            prof_begin(DL_K_UPD_EUPDATE, st);
            hipLaunchKernelGGL(eupdate_kernel, dim3(eg), dim3(256), 0, st, a, a0, a1);
            prof_end(DL_K_UPD_EUPDATE, st);
            if ((e = hipGetLastError()) != hipSuccess)
                return e;
        }
    }
    return hipSuccess;
}

hipError_t launch_batched_update(const UpdateArgs *tab, const BatchList &pass1_list,
                                 int pass1_items, const BatchList &chunk_list, int chunk_items,
                                 hipStream_t st)
{
    int wg = batch_workers((const void *)update_batched<0>, 256, 0, pass1_items);
    prof_begin(DL_K_UPD_PASS1, st);
    hipLaunchKernelGGL(update_batched<0>, dim3(wg), dim3(256), 0, st, tab, pass1_list,
                       batch_per_ticket(pass1_items, wg));
    prof_end(DL_K_UPD_PASS1, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    wg = batch_workers((const void *)update_batched<2>, 256, 0, chunk_items);
    prof_begin(DL_K_UPD_PASS2, st);
    hipLaunchKernelGGL(update_batched<2>, dim3(wg), dim3(256), 0, st, tab, chunk_list,
                       batch_per_ticket(chunk_items, wg));
    prof_end(DL_K_UPD_PASS2, st);
    return hipGetLastError();
}

hipError_t launch_batched_rmse(const RmseArgs *tab, const BatchList &bl, int items,
                               const BatchList &final_list, int k, hipStream_t st)
{
    int wg = batch_workers((const void *)rmse_batched, 256, 0, items);
    prof_begin(DL_K_RMSE, st);
    hipLaunchKernelGGL(rmse_batched, dim3(wg), dim3(256), 0, st, tab, bl,
                       batch_per_ticket(items, wg));
    prof_end(DL_K_RMSE, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    wg = batch_workers((const void *)rmse_final_batched, 256, 0, final_list.count);
    prof_begin(DL_K_RMSE, st);
    hipLaunchKernelGGL(rmse_final_batched, dim3(wg), dim3(256), 0, st, tab, final_list, k);
    prof_end(DL_K_RMSE, st);
    return hipGetLastError();
}

hipError_t launch_batched_normalize(const NormArgs *tab, const BatchList &bl, int items,
                                    hipStream_t st)
{
    const int wg = batch_workers((const void *)normalize_batched, 256, 0, items);
    prof_begin(DL_K_MISC, st);
    hipLaunchKernelGGL(normalize_batched, dim3(wg), dim3(256), 0, st, tab, bl,
                       batch_per_ticket(items, wg));
    prof_end(DL_K_MISC, st);
    return hipGetLastError();
}

hipError_t launch_rmse(const RmseArgs &a, hipStream_t st)
{
    const int nb = rmse_blocks(a.m);
    prof_begin(DL_K_RMSE, st);
    if (a.refresh && a.p <= 64 && a.n <= kRmseCosTab)
        hipLaunchKernelGGL(rmse_pf_kernel, dim3(nb), dim3(256), 0, st, a);
    else if (a.refresh)
        hipLaunchKernelGGL(rmse_kernel<true>, dim3(nb), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(rmse_kernel<false>, dim3(nb), dim3(256), 0, st, a);
    prof_end(DL_K_RMSE, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    prof_begin(DL_K_RMSE, st);
    hipLaunchKernelGGL(rmse_final_kernel, dim3(1), dim3(256), 0, st, a, nb);
    prof_end(DL_K_RMSE, st);
    return hipGetLastError();
}

hipError_t launch_rmse_unprofiled(const RmseArgs &a, hipStream_t st)
{
    const int nb = rmse_blocks(a.m);
    hipLaunchKernelGGL(rmse_kernel<false>, dim3(nb), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(rmse_final_kernel, dim3(1), dim3(256), 0, st, a, nb);
    return hipGetLastError();
}

hipError_t launch_residual(const float *Y, const float *D, const int32_t *idx, const float *val,
                           float *E, int p, int n, int m, int s, hipStream_t st)
{
    prof_begin(DL_K_MISC, st);
    hipLaunchKernelGGL(residual_kernel, dim3(grid_for((size_t)m * 16, 4096)), dim3(256), 0, st, Y,
                       D, idx, val, E, p, n, m, s);
    prof_end(DL_K_MISC, st);
    return hipGetLastError();
}

hipError_t launch_normalize_rows(float *D, int n, int p, Control *ctl, hipStream_t st)
{
    prof_begin(DL_K_MISC, st);
    hipLaunchKernelGGL(normalize_kernel, dim3((n + 3) / 4), dim3(256), 0, st, D, n, p, ctl);
    prof_end(DL_K_MISC, st);
    return hipGetLastError();
}

hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t st)
{
    const size_t words = bytes / 4;  // every buffer here is a multiple of 4 bytes
    if (words == 0)
        return hipSuccess;
    prof_begin(DL_K_MISC, st);
    hipLaunchKernelGGL(copy_kernel, dim3(grid_for(words, 4096)), dim3(256), 0, st,
                       (const uint32_t *)src, (uint32_t *)dst, words);
    prof_end(DL_K_MISC, st);
    return hipGetLastError();
}

hipError_t launch_zero(void *dst, size_t bytes, hipStream_t st)
{
    const size_t words = bytes / 4;
    if (words == 0)
        return hipSuccess;
    prof_begin(DL_K_MISC, st);
    hipLaunchKernelGGL(zero_kernel, dim3(grid_for(words, 4096)), dim3(256), 0, st,
                       (uint32_t *)dst, words);
    prof_end(DL_K_MISC, st);
    return hipGetLastError();
}

}  // namespace dlk
