// Internal declarations shared by the HIP translation units of the library.
// Nothing here is part of the C ABI (include/dl.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/dl.h"

namespace dlk {

// Users of one atom are processed in chunks of this many (atom update).
constexpr int kChunk = 256;  // most users per chunk of the atom update
// Signals per block of the CSR transpose (one workgroup each).
constexpr int kCsrBlock = 256;
// Signals per workgroup of the FP64 error reduction.
// Signals per block of the error's partial pass (measured: 32 is 5% faster
// than 16 end to end; 64 enlarges the error body's LDS, which also counts in
// the product launches that carry it, and cost the 128-row GEMM tiles a
// workgroup per CU).
constexpr int kRmseSignals = 32;
// Pass 1 by signal blocks (all atoms in one group): the entries (signals x
// slots) of one signal block are ranked in LDS, at most this many (a
// multiple of 256, below 2^13).
constexpr int kGsumPool = 7168;
// Signal blocks aimed at by pass 1 by signal blocks (the blocks are made no
// larger than the pool allows).
constexpr int kGsumBlocks = 64;

// Device-side counters and control words at the start of the workspace.
struct Control {
    unsigned long long fp64_pivot_recomputes;
    unsigned long long early_stops;
    unsigned long long unused_atoms;
    unsigned long long zero_updates;
    unsigned long long nonfinite;
    unsigned long long fallbacks;
    unsigned int pad[16];
};

// Byte offsets of the workspace regions (each 256-byte aligned).
struct Layout {
    size_t control;
    size_t G;          // [n][n] float, NaN on the diagonal (the coding's copy)
    size_t Gdiag;      // [n] float, the diagonal of G
    size_t A0;         // [m][n] float, D^T y per signal
    size_t E;          // [m][p] float, residual
    size_t Dn;         // [n][p] float, next dictionary
    size_t val_ws;     // [m][s] float, OMP coefficients before the update
    size_t valn;       // [m][s] float, refreshed coefficients (dl_jau_update)
    size_t blkcnt;     // [n][nb] int, per-(atom, block) counts, then offsets
    size_t lrank;      // [m*s] int, rank of an entry among its block's uses of the atom
    size_t atom_tot;   // [n] int, users per atom
    size_t row_ptr;    // [n+1] int
    size_t chunk_ptr;  // [n+1] int
    size_t uent;       // [m*s] int2: (ELL position, coefficient bits) of every user, in user order
    size_t atom_state; // [n] int: 0 updated, 1 no users, 2 zero F x^T
    size_t atom_cos;   // [n] float: d_j^T d_j' of the updated atoms
    size_t partial;    // [max(max_chunks, n * nsb)][p] float
    size_t bcnt;       // [n][nsb] int: users per (atom, signal block) of pass 1 by signal blocks
    size_t rmse_part;  // [rmse_blocks(m)] double
    size_t idx_prev;   // [m][s] int, previous coding (NSGK rule, or a carried error)
    size_t val_prev;   // [m][s] float, previous coding (NSGK rule, or a carried error)
    size_t E2;         // [m][p] float, the previous iteration's residual (carried error only)
    size_t Dbf;        // [n][p] bf16 (precision variant)
    size_t Ybf;        // [m][p] bf16 (precision variant)
    size_t total;
};

Layout layout_for(const dl_params &prm);
bool params_ok(const dl_params *prm);
int csr_blocks(int m);
int max_chunks(const dl_params &prm);
// Users per chunk of the atom update: kChunk with all atoms in one group;
// half that with smaller groups, whose atoms have fewer users each (measured
// at group size 16, m = 16384: 39.6 -> 47.3 M signals*iters/s; with one
// group the larger chunks stay faster, 282 vs 279 M, and at m = 262144
// 483 vs 468 M).
int chunk_users(const dl_params &prm);
// Signals per block of pass 1 by signal blocks, or 0 when pass 1 goes over
// chunks of each atom's user list.  Used with all atoms in one group, when an
// item's atom range (one atom per lane group of a workgroup) covers at least
// a thirty-second of the atoms: each item then ranks its block's entries for
// its own atoms without a global user list.
int gsum_block(const dl_params &prm);
// Signal blocks of that pass (0 when it is not used).
int gsum_signal_blocks(const dl_params &prm);
// Work items of that pass: (signal block, atom range) pairs.
int gsum_items(const dl_params &prm);
int rmse_blocks(int m);

// Optional per-kernel timing (dl_profile_enable): bracket a launch.
void prof_begin(int kernel, hipStream_t st);
void prof_end(int kernel, hipStream_t st);

// ---- launchers (return hipSuccess or the launch error) -------------------
// C[M][N] (row stride ldc) = A[M][K] * B[N][K]^T on MFMA with FP32
// accumulation; K % 4 == 0.  Up to two independent problems share a launch.
// diag (optional, Gram matrices only): the diagonal C_ii is stored there and
// C_ii itself is set to NaN.  The coding reads G rows with the selected atom's
// own entry NaN: its correlation then turns NaN in the step's update and stays
// so, which no comparison selects again, so the argmax needs no mask.
struct GemmF32 {
    const float *A, *B;
    float *C;
    int M, N, K, ldc;
    const int32_t *M_dev;  // optional: rows read on the device (<= M)
    float *diag = nullptr;
};
struct GemmBF16 {  // BF16 inputs as uint16 bit patterns
    const uint16_t *A, *B;
    float *C;
    int M, N, K, ldc;
    const int32_t *M_dev;
    float *diag = nullptr;
};
struct RmseArgs;
// err: optional error partials (rmse_blocks(err->m) workgroups of the
// error's partial pass) run by extra workgroups of the same launch.
hipError_t launch_gemm_nt_f32(const GemmF32 &p0, const GemmF32 *p1, int kid, hipStream_t st,
                              const RmseArgs *err = nullptr);
hipError_t launch_gemm_nt_bf16(const GemmBF16 &p0, const GemmBF16 *p1, int kid, hipStream_t st,
                               const RmseArgs *err = nullptr);
// Round FP32 to BF16 (nearest even).
hipError_t launch_cast_bf16(const float *x, uint16_t *y, size_t count, hipStream_t st);

struct OmpArgs {
    const float *A0;   // [m][n]
    const float *G;    // [n][n], NaN on the diagonal
    const float *Gdiag;  // [n] the diagonal of G
    const float *Y;    // [m][p]
    const float *D;    // [n][p]
    int32_t *idx;      // [m][s]
    float *val;        // [m][s]
    float *E;          // [m][p] residual, may be null
    Control *ctl;
    int p, n, m, s;
    int ldn;               // leading dimension of G and A0 rows (multiple of 4, >= n)
    const int32_t *m_dev;  // optional: signal count read on the device (<= m)
    const int32_t *rowmap; // optional: output row of compact signal i
    float *rnorm;          // optional: ||y - D x|| per output row
    int lanes_per_signal;  // 4..64, or 0 for the default
    int atoms_per_lane;    // 8 or 16, or 0 for the default (16)
    float pivot_fp64, tol_corr, tol_pivot;
};
// err: optional error partials (rmse_blocks(err->m) workgroups of the
// refreshing error pass) run by extra workgroups behind the coding ones;
// only shapes of one wave per signal group take them (omp_carries_error).
hipError_t launch_omp(const OmpArgs &a, hipStream_t st, const RmseArgs *err = nullptr);
bool omp_carries_error(int n, int s, int lps_req, int npl_req);
int omp_lanes_per_signal(int n, int npl, int s);
bool omp_config_ok(int n, int s, int lps, int npl);
// Leading dimension used for G and A0 rows.
inline int padded_n(int n) { return (n + 3) & ~3; }

// The values of this lane and of lane ^ 16 (permlane16_swap: rows 2r and
// 2r + 1 trade places) or lane ^ 32 (permlane32_swap: the wave's halves trade
// places), as the pair (x, y) in an order that depends on the lane.  A sum
// x + y or a max/min of the pair is the same in both lanes of a pair (both
// commute), so one VALU instruction replaces a shuffle through the LDS
// crossbar.
__device__ inline void pair_xor16(int v, int &x, int &y)
{
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    x = (int)r[0];
    y = (int)r[1];
}
__device__ inline void pair_xor32(int v, int &x, int &y)
{
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    x = (int)r[0];
    y = (int)r[1];
}
__device__ inline float sum_xor(float v, int off)  // off: 16 or 32
{
    int x, y;
    if (off == 16)
        pair_xor16(__float_as_int(v), x, y);
    else
        pair_xor32(__float_as_int(v), x, y);
    return __int_as_float(x) + __int_as_float(y);
}

struct CsrArgs {
    const int32_t *idx;  // [m][s]
    int32_t *blkcnt;     // [n][nb] per-(atom, block) counts, then offsets
    int32_t *tot;        // [n] users per atom
    Control *ctl;
    int32_t *lrank;      // [m*s]
    int32_t *row_ptr;    // [n+1]
    int32_t *chunk_ptr;  // [n+1]
    int32_t *users;      // optional: ELL positions of the users [m*s]
    int2 *uent;          // optional: (position, coefficient bits) of the users [m*s]
    const float *val;    // coefficients [m][s] (with uent)
    float *val_pad;      // optional: zero written at padding slots
    int n, m, s;
    int chunk = kChunk;  // users per chunk of the atom update (chunk_ptr)
};
// err: optional error whose partials are complete; its final sum runs as one
// extra workgroup of the scan launch.
hipError_t launch_csr(const CsrArgs &a, hipStream_t st, const RmseArgs *err = nullptr);

struct UpdateArgs {
    const float *Y;       // [m][p]
    const float *D;       // [n][p] dictionary at the start of the sweep
    float *Dn;            // [n][p] next dictionary
    const int32_t *idx;   // [m][s]
    const float *val;     // [m][s] coefficients at the start of the sweep
    float *valn;          // [m][s] refreshed coefficients
    float *E;             // [m][p] residual with the current D, X (kept up to date across groups)
    const int32_t *row_ptr, *chunk_ptr;
    const int2 *uent;     // [m*s] (ELL position, val there) of every user, in user order
    int32_t *atom_state;
    float *atom_cos;      // [n] d_j^T d_j' (the refresh's x term)
    float *partial;
    Control *ctl;
    int p, n, m, s, group_size, rule, max_chunks;
    int no_refresh;  // 1: pass 2 only forms d' (the error pass refreshes X)
    int chunk;       // users per chunk (chunk_users, at most kChunk)
    // pass 1 by signal blocks (gsum_block): signals per block, or 0 for pass 1
    // over chunks of users; nsb blocks; bcnt [n][nsb] users per (atom, block),
    // partial [n][nsb][p] the block sums
    int sig_block, nsb;
    int32_t *bcnt;
};
// err: optional error whose partials are complete; with pass 1 by signal
// blocks and no refresh in pass 2 (no user lists built) its final sum runs
// as one extra workgroup of pass 1's launch.
hipError_t launch_update(const UpdateArgs &a, hipStream_t st, const RmseArgs *err = nullptr);

struct RmseArgs {
    const float *Y, *D;
    const int32_t *idx;
    const float *val;
    double *partial;  // [rmse_blocks(m)] block partials
    double *out;      // one double
    Control *ctl;
    int p, n, m, s;
    // Optional refresh (all atoms in one group, D the updated dictionary):
    // with refresh set, the pass also forms the refreshed coefficients
    // x' = (e + d x)^T d' (eq. 5, second line) as e^T d' + x (d^T d'), from
    // the coefficients val_old, the residual E and atom_cos = d^T d' per atom
    // (pass 2's), writes them to valn, and measures the error with them.
    // Atoms whose atom_state is not 0, and the SGK rule, keep their
    // coefficients.
    int refresh = 0;
    const float *E = nullptr, *val_old = nullptr;
    const int32_t *atom_state = nullptr;
    const float *atom_cos = nullptr;
    float *valn = nullptr;
    int rule = 0;
};
hipError_t launch_rmse(const RmseArgs &a, hipStream_t st);
// The same two launches without the optional per-launch timing (which may
// create events): for the entry point that allocates nothing.
hipError_t launch_rmse_unprofiled(const RmseArgs &a, hipStream_t st);
// Most error partials any launch uses (rmse_blocks(m) never exceeds it).
constexpr int kRmseMaxPartials = 1024;
// Whether an error over m signals is one signal block per partial workgroup
// (the sizes at which it is carried by the next iteration's launches).
bool error_defer_ok(int m);
// Whether dl_iterate carries each iteration's error into the next one's
// launches (all atoms in one group, error_defer_ok); the coding then keeps
// two sets of X and E buffers, alternating between iterations.
bool error_carried(const dl_params &prm);

// E = Y - D X (one signal per lane group).
hipError_t launch_residual(const float *Y, const float *D, const int32_t *idx, const float *val,
                           float *E, int p, int n, int m, int s, hipStream_t st);
hipError_t launch_normalize_rows(float *D, int n, int p, Control *ctl, hipStream_t st);
hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t st);
hipError_t launch_zero(void *dst, size_t bytes, hipStream_t st);

// ---- proposal network (mlp.hip) -------------------------------------------
constexpr int kEpiF32 = 0;       // C (fp32) = acc (+ bias)
constexpr int kEpiBiasRelu = 1;  // C, C^T (bf16) = relu(acc + bias)
constexpr int kEpiReluMask = 2;  // C, C^T (bf16) = acc where mask > 0, else 0
struct MlpGemm {
    const uint16_t *A;  // [M][lda] bf16, K-contiguous
    const uint16_t *B;  // [N][ldb] bf16, K-contiguous
    int lda, ldb, M, N, K;  // K % 8 == 0, lda/ldb % 8 == 0
    int epi;
    const float *bias;      // [N] or null (only with a single K split)
    const uint16_t *mask;   // [M][ldmask] (kEpiReluMask)
    int ldmask;
    float *Cf;              // kEpiF32 output; split s writes Cf + s * split_stride
    int ldcf;
    size_t split_stride;
    uint16_t *Cb;           // bf16 output [M][ldcb] or null
    int ldcb;
    uint16_t *Ct;           // bf16 transposed output [N][ldct] or null
    int ldct;
};
struct AdamHyper {
    float lr, beta1, beta2, eps, bc1, bc2;  // bc = 1 - beta^t
};
hipError_t launch_mlp_gemm(const MlpGemm &g, int splits, hipStream_t st);
hipError_t launch_sum_splits(const float *part, float *out, size_t count, int splits,
                             size_t stride, hipStream_t st);
hipError_t launch_rowsum_bf16(const uint16_t *X, float *out, int rows, int cols, hipStream_t st);
hipError_t launch_gather_batch(const float *Y, int m, int p, const int32_t *pairs, int B,
                               uint16_t *Xb, uint16_t *Xbt, hipStream_t st);
hipError_t launch_gather_rows(const float *X, int rows, int cols, uint16_t *Xb, hipStream_t st);
hipError_t launch_bce(const float *Z, int out_dim, const int32_t *hist, int s,
                      const int32_t *pairs, int B, uint16_t *dZ, uint16_t *dZt, double *loss_rows,
                      float w_pos, hipStream_t st);
hipError_t launch_adam(float *w, const float *g, float *m1, float *m2, int rows, int cols,
                       uint16_t *wb, uint16_t *wbt, const AdamHyper &h, int do_step,
                       hipStream_t st);
hipError_t launch_topk(const float *logits, int rows, int cols, int k, int32_t *out,
                       hipStream_t st);

struct ProposeArgs {
    const float *Y, *D, *G;    // [m][p], [n][p], [n][ldn] (NaN on the diagonal)
    const float *Gdiag;        // [n] the diagonal of G
    const int32_t *cand;       // [m][k2]
    const float *rref;         // [m] reference OMP residual norms
    int32_t *idx;              // [m][s]
    float *val;                // [m][s]
    float *E;                  // [m][p]
    int32_t *fb_list;          // [m] signals handed back to OMP
    int32_t *fb_count;         // one int (zeroed before the launch)
    Control *ctl;
    int p, n, m, s, ldn;
    float margin;
};
hipError_t launch_ls_prune(const ProposeArgs &a, int k2, hipStream_t st);
hipError_t launch_gather_list(const float *src, int p, const int32_t *list, const int32_t *count,
                              int cap, float *rows, hipStream_t st);

// ---- batched problems (batch_api.hip) ---------------------------------------
// A batched launch runs one stage for many independent problems.  Problem b
// owns the work items [start[b], start[b+1]) of the launch; persistent
// workgroups (or, for OMP, waves) take items from a device ticket counter
// until none are left.  The last worker to leave resets the counters, so one
// queue serves every launch of a stream in turn.
struct BatchQueue {
    unsigned int ticket;
    unsigned int exited;
    unsigned int pad[62];
};
struct BatchList {
    const int32_t *start;  // [count + 1] item prefix sums
    int count;
    BatchQueue *q;
};

// Problem owning item `it` (start is non-decreasing, start[0] = 0).
__device__ inline int batch_find(const int32_t *start, int count, int it)
{
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= it)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Workgroup-wide: the next item of a batched launch (every thread gets it);
// `slot` is a shared int of the calling kernel.
__device__ inline int batch_next_item(BatchQueue *q, int *slot)
{
    __syncthreads();  // everyone has read the previous item
    if (threadIdx.x == 0)
        *slot = (int)atomicAdd(&q->ticket, 1u);
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(*slot);
}

// Workgroup-wide cursor over a batched launch's items: a ticket is `per`
// consecutive items, so the one counter sees a few atomics per workgroup
// rather than one per item.  Every call begins with a workgroup barrier (the
// previous item's shared memory is no longer read); it returns false when
// no item is left.
struct BatchCursor {
    int it = 0, end = 0;
};
__device__ inline bool batch_advance(BatchQueue *q, int total, int per, BatchCursor &c, int *slot)
{
    if (c.it + 1 < c.end) {
        __syncthreads();
        ++c.it;
        return true;
    }
    const int tk = batch_next_item(q, slot);
    const long long first = (long long)tk * per;
    if (first >= total)
        return false;
    c.it = (int)first;
    c.end = (int)(first + per < total ? first + per : total);
    return true;
}

// The problem owning item `it` of a list, looked up again only when `it`
// leaves the cached problem's item range [b0, b1).  Returns true when the
// problem changed (its arguments must be reloaded).
struct BatchOwner {
    int b = -1, b0 = 0, b1 = 0;
};
__device__ inline bool batch_owner(const int32_t *start, int count, int it, BatchOwner &o)
{
    if (o.b >= 0 && it >= o.b0 && it < o.b1)
        return false;
    o.b = batch_find(start, count, it);
    o.b0 = start[o.b];
    o.b1 = start[o.b + 1];
    return true;
}

// Items per ticket for a launch of `workers` workgroups: about eight tickets
// per workgroup, at most 16 items each.
inline int batch_per_ticket(int items, int workers)
{
    long long per = (long long)items / (8ll * (workers > 0 ? workers : 1));
    return per < 1 ? 1 : (per > 16 ? 16 : (int)per);
}

// Called once by every worker after its last item; `workers` is the number
// of workers in the launch.  Only the counters are shared (results reach the
// next launch through the launch boundary), so no fence is needed.
__device__ inline void batch_leave(BatchQueue *q, unsigned workers)
{
    const unsigned prev = atomicAdd(&q->exited, 1u);
    if (prev == workers - 1) {
        atomicExch(&q->ticket, 0u);
        atomicExch(&q->exited, 0u);
    }
}

struct NormArgs {
    float *D;
    int n, p;
    Control *ctl;
};
// Gram and correlation products of one problem (single-problem tiles).
struct GemmPair {
    GemmF32 g, c;
};
int batch_workers(const void *kernel, int block, size_t lds, int items);
int gemm_pair_items(const GemmPair &pp);
// etab/el/eitems: optional error partials of another iteration (the blocks
// of each problem's partial pass), run as extra items of the same launch.
hipError_t launch_batched_gemm(const GemmPair *tab, const BatchList &bl, int items,
                               hipStream_t st, const RmseArgs *etab = nullptr,
                               const BatchList &el = BatchList{}, int eitems = 0);
hipError_t launch_batched_omp(const OmpArgs *tab, const BatchList &bl, int items, int lps,
                              int npl, int smax, hipStream_t st);
hipError_t launch_batched_csr(const CsrArgs *tab, const BatchList &count_list, int count_items,
                              const BatchList &scan_list, int scan_items,
                              const BatchList &scatter_list, int scatter_items, int max_n,
                              hipStream_t st, const RmseArgs *etab = nullptr,
                              const BatchList &el = BatchList{}, int k = 0);
hipError_t launch_batched_update(const UpdateArgs *tab, const BatchList &pass1_list,
                                 int pass1_items, const BatchList &chunk_list, int chunk_items,
                                 hipStream_t st);
hipError_t launch_batched_rmse(const RmseArgs *tab, const BatchList &bl, int items,
                               const BatchList &final_list, int k, hipStream_t st);
hipError_t launch_batched_normalize(const NormArgs *tab, const BatchList &bl, int items,
                                    hipStream_t st);
int omp_smax(int s);
int omp_default_npl(int n, int s);
int omp_signals_per_item(int lps);

}  // namespace dlk
