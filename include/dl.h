/*
 * dl.h - C ABI of the MI355X (gfx950) dictionary-learning library.
 *
 * The library runs one or more iterations of dictionary learning with Jacobi
 * atom updates (Irofti & Dumitrescu, "Overcomplete Dictionary Learning with
 * Jacobi Atom Updates"):
 *   step 1 (Alg. 1): sparse coding of every signal with OMP at fixed sparsity s,
 *            computed as Batch-OMP from G = D^T D and D^T Y;
 *   step 2 (Alg. 1, Alg. 2): atoms updated in groups of `group_size`; every atom
 *            of a group is refreshed from the same error E = Y - D X with the
 *            AK-SVD rule (eq. 5), normalised, and the group is committed before
 *            the next one starts (eq. 2);
 *   error  : ||Y - D X||_F / sqrt(p m) after the update, with the refreshed X.
 *
 * Conventions shared by every entry point
 *   - Every array argument is a DEVICE pointer owned by the caller, aligned to
 *     16 bytes (the workspace to 256 bytes).  The library never allocates or
 *     frees device memory and never synchronises the stream, except where an
 *     entry point says so.
 *   - Layouts are row-major:
 *       D  [n][p] float   atom j is D + j*p (unit-norm rows)
 *       Y  [m][p] float   signal i is Y + i*p
 *       X  ELL: X_idx [m][s] int32 atom index, -1 in unused slots;
 *               X_val [m][s] float coefficient, 0 in unused slots.
 *               Slot t of signal i holds the t-th atom OMP selected.
 *   - All work is enqueued on `stream` (a hipStream_t; NULL = default stream).
 *   - Arguments are validated on the host before anything is launched; a
 *     failure returns DL_EINVAL or DL_EWORKSPACE and enqueues nothing.
 *   - A launch failure returns DL_EHIP.  Non-finite values met on the device
 *     are counted in the workspace statistics; dl_read_stats reports them as
 *     DL_ENUMERIC.
 *   - Calls that share a workspace must not overlap in time (use one stream).
 *   - No C++ exception crosses this boundary.
 *
 * Limits: 4 <= p <= 256 with p % 4 == 0; 1 <= n <= 1024; 1 <= s <= min(p, n, 16);
 * m >= 1 with m * s < 2^31; group_size >= 1 (values above n mean n).
 */
#ifndef DL_MI355_H
#define DL_MI355_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *dl_stream_t; /* the same handle type as hipStream_t */

typedef enum {
    DL_OK = 0,
    DL_EINVAL = -1,       /* bad size, pointer, alignment or option */
    DL_EWORKSPACE = -2,   /* workspace smaller than dl_workspace_size() */
    DL_EHIP = -3,         /* a HIP launch or copy failed */
    DL_ENUMERIC = -4,     /* non-finite values were met on the device */
    DL_EUNSUPPORTED = -5  /* option valid in principle but not built */
} dl_status;

typedef enum { DL_PREC_FP32 = 0, DL_PREC_BF16 = 1 } dl_precision;

/* Atom rule.  AK-SVD (eq. 5): d = F x^T / ||F x^T||, then x = F^T d (X is
   refreshed).  SGK (eq. 6): d = F x^T / (x x^T), normalised; X unchanged.
   NSGK (Sec. 3, eq. 7): SGK on Z = Y + D X_prev - D X with the
   representations X_prev the iteration started from (the previous
   iteration's coding; the first iteration uses its own), so the users I_j and
   the coefficients x come from X_prev and the group error is Z - D X_prev;
   X unchanged.  dl_iterate keeps X_prev itself; a single update takes it as
   an argument (dl_jau_update_nsgk). */
typedef enum { DL_RULE_AKSVD = 0, DL_RULE_SGK = 1, DL_RULE_NSGK = 2 } dl_rule;

typedef struct dl_params {
    int p, n, m, s;               /* signal size, atoms, signals, sparsity */
    int group_size;               /* atoms updated in parallel (eq. 2); >= n: all at once */
    int precision;                /* dl_precision of D^T Y, D^T D and the residual products */
    int rule;                     /* dl_rule */
    float pivot_fp64_threshold;   /* FP32 Cholesky pivots below this are recomputed in FP64 (1e-6) */
    float tol_corr;               /* OMP stops when max |d_j^T r| <= tol_corr * ||y|| (1e-5) */
    float tol_pivot;              /* OMP stops when the FP64 pivot <= tol_pivot * G_jj (1e-10) */
    /* Launch shape of the OMP kernel (0 = default).  A signal is coded by
       omp_lanes_per_signal lanes (4, 8, 16, 32 or 64, or 128 = two waves
       with 4 or 8 correlations per lane) each holding omp_atoms_per_lane
       correlations (4, 8 or 16); their product must be >= n and the lanes
       at least the sparsity bound (s rounded up to 4, 6, 8, 12 or 16).
       Only the launch shape changes: every value is computed with the same
       operations, except the summation order of ||y|| in the stop test
       (which 128 lanes share with 64).  Batched calls run a 128-lane shape
       as 64 lanes with twice the correlations per lane. */
    int omp_lanes_per_signal;
    int omp_atoms_per_lane;
} dl_params;

/* Counters kept in the workspace (device); read them with dl_read_stats. */
typedef struct dl_stats {
    long long fp64_pivot_recomputes; /* OMP steps whose pivot was recomputed in FP64 */
    long long early_stops;           /* signals coded with fewer than s atoms */
    long long unused_atoms;          /* atom updates skipped: the atom had no users */
    long long zero_updates;          /* atom updates skipped: F x^T was zero */
    long long nonfinite;             /* non-finite values met (inputs or results) */
    long long fallbacks;             /* learned-proposal signals handed back to OMP */
} dl_stats;

/* ABI version of this header (increments on any signature change). */
int dl_abi_version(void);

/* Human-readable name of a dl_status value. */
const char *dl_status_string(int status);

/* Fill *prm with the defaults for a problem of the given sizes
   (group_size = n, FP32, AK-SVD, thresholds as documented above). */
dl_status dl_params_default(dl_params *prm, int p, int n, int m, int s);

/* Bytes of workspace the calls below need for these parameters (host only,
   pure).  Returns 0 if the parameters are invalid. */
size_t dl_workspace_size(const dl_params *prm);

/* Zero the workspace's counters and control words.  Call once after
   allocating a workspace (dl_iterate does it itself). */
dl_status dl_workspace_init(const dl_params *prm, void *ws, size_t ws_bytes, dl_stream_t stream);

/* G = D D^T as [n][n] (the Gram matrix of the atoms that Batch-OMP uses for
   its incremental Cholesky; the paper's coder is OMP, Sec. 4).  FP32 MFMA
   with FP32 accumulation (BF16 inputs when prm->precision is DL_PREC_BF16). */
dl_status dl_gram(const dl_params *prm, const float *D, float *G, dl_stream_t stream);

/* A0 = Y D^T as [m][n]: the correlations D^T y of every signal with every
   atom, the first term of Batch-OMP's correlation update.  Same precision
   rules as dl_gram. */
dl_status dl_corr(const dl_params *prm, const float *D, const float *Y, float *A0,
                  dl_stream_t stream);

/* The dense products of the coding stage exactly as dl_omp forms them:
   G = D D^T ([n][n]) and A0 = Y D^T ([m][n]), in prm->precision (BF16 inputs
   rounded to nearest-even, FP32 accumulation on the matrix cores, or FP32).
   Uses the workspace for the BF16 copies. */
dl_status dl_products(const dl_params *prm, const float *D, const float *Y, float *G, float *A0,
                      void *ws, size_t ws_bytes, dl_stream_t stream);

/* Step 1 of the DL iteration (Alg. 1): OMP with fixed sparsity s of every
   signal against D, written to X_idx/X_val.  Ties between correlations go to
   the lowest atom index.  A signal stops early when its residual is
   numerically orthogonal to every atom (tol_corr) or the next atom's pivot
   vanishes (tol_pivot); its remaining slots are (-1, 0).  Also leaves the
   coding residual E = Y - D X in the workspace. */
dl_status dl_omp(const dl_params *prm, const float *D, const float *Y, int32_t *X_idx,
                 float *X_val, void *ws, size_t ws_bytes, dl_stream_t stream);

/* The users of every atom (the set I_j of Sec. 3: signals whose representation
   uses d_j), as a CSR transpose of X: row_ptr [n+1] and users [m*s]; entry
   users[row_ptr[j] + r] is the ELL position i*s + t of the r-th use of atom j,
   in increasing signal order.  Slots with index -1 are not listed.
   Deterministic; the result is exact. */
dl_status dl_csr(const dl_params *prm, const int32_t *X_idx, int32_t *row_ptr, int32_t *users,
                 void *ws, size_t ws_bytes, dl_stream_t stream);

/* Step 2 of the DL iteration: the Jacobi atom update of Alg. 2 with the rule
   prm->rule, groups of prm->group_size atoms in index order.  D is replaced
   by the new dictionary, X_val by the refreshed representations (AK-SVD; SGK
   leaves them).  X_idx is not changed.  An atom with no users, or whose
   F x^T is zero, keeps its value. */
dl_status dl_jau_update(const dl_params *prm, const float *Y, float *D, const int32_t *X_idx,
                        float *X_val, void *ws, size_t ws_bytes, dl_stream_t stream);

/* Step 2 with the NSGK rule (Sec. 3, eq. 7; prm->rule must be DL_RULE_NSGK):
   the group loop of dl_jau_update on Z = Y + D X_prev - D X, where X
   (X_idx/X_val) is this iteration's coding against D and X_prev
   (Xprev_idx/Xprev_val, the same ELL layout) the previous one: the users of
   every atom and their coefficients come from X_prev, the group error is
   Z - D X_prev with the current D, and d_j = F x^T / (x x^T), normalised.
   D is replaced by the new dictionary; neither X changes.  An atom X_prev
   does not use keeps its value. */
dl_status dl_jau_update_nsgk(const dl_params *prm, const float *Y, float *D,
                             const int32_t *X_idx, const float *X_val,
                             const int32_t *Xprev_idx, const float *Xprev_val, void *ws,
                             size_t ws_bytes, dl_stream_t stream);

/* rmse_out[0] = ||Y - D X||_F / sqrt(p m), accumulated in FP64 (the error the
   paper plots, Sec. 4.2).  rmse_out is a device pointer to one double. */
dl_status dl_rmse(const dl_params *prm, const float *Y, const float *D, const int32_t *X_idx,
                  const float *X_val, double *rmse_out, void *ws, size_t ws_bytes,
                  dl_stream_t stream);

/* As dl_rmse, for callers that cannot allocate device memory (code under
   graph capture, tight serving loops, harnesses that forbid allocation): no
   workspace argument, and the call allocates nothing.  Its scratch (the
   error's control words and at most 1024 FP64 block partials, 8.4 KB) is a
   static device array of the library; each GPU holds its own copy from the
   first call on that device until the process ends.  Every size dl_rmse
   accepts fits it; invalid sizes or pointers return DL_EINVAL.  The stream
   must belong to the current device.  Calls on one GPU share its array, so
   calls that overlap in time on one GPU race (use one stream).  A non-finite
   error is returned as a non-finite value. */
dl_status dl_rmse_noalloc(const dl_params *prm, const float *Y, const float *D,
                          const int32_t *X_idx, const float *X_val, double *rmse_out,
                          dl_stream_t stream);

/* `iters` DL iterations (Alg. 1): D holds D0 on entry (it is normalised
   first) and the final dictionary on exit; X_idx/X_val hold the last
   iteration's representations after its update; rmse[k] (device, `iters`
   doubles) is the error after iteration k.  Zeroes the workspace counters
   first.  With the NSGK rule the workspace also keeps the previous
   iteration's representations. */
dl_status dl_iterate(const dl_params *prm, const float *Y, float *D, int iters, int32_t *X_idx,
                     float *X_val, double *rmse, void *ws, size_t ws_bytes, dl_stream_t stream);

/* ---- learned support proposal ------------------------------------------
   A network in_dim -> hidden -> hidden -> out_dim with ReLU maps a signal to
   one logit per atom; it sees the signal scaled to unit norm (the OMP support
   depends on its direction only).  It is trained on (signal, OMP support)
   pairs with the mean binary cross-entropy of the logits against the
   multi-hot support, positive terms weighted by pos_weight, and Adam.  Weights and activations are stored in BF16 for the matrix cores
   (FP32 accumulation); Adam keeps FP32 master weights.  Parameters travel
   packed as [W1 (hidden x in) | b1 | W2 (hidden x hidden) | b2 |
   W3 (out x hidden) | b3], row-major, FP32. */
typedef struct dl_mlp_params {
    int in_dim;    /* input size (= p), multiple of 8 */
    int hidden;    /* units per hidden layer, multiple of 32 */
    int out_dim;   /* outputs (= n), multiple of 8 */
    int batch;     /* minibatch rows, multiple of 32 */
    float lr, beta1, beta2, eps;  /* Adam */
    float pos_weight;  /* weight of the loss terms of support atoms, > 0;
                          (n - s) / s balances the s positives of a row */
} dl_mlp_params;

/* Packed parameter count, and the workspace bytes of the network (host
   only; 0 if invalid). */
size_t dl_mlp_param_count(const dl_mlp_params *q);
size_t dl_mlp_workspace_size(const dl_mlp_params *q);

/* Load the packed parameters (device) into the workspace, zero the Adam
   moments and make the BF16 copies. */
dl_status dl_mlp_init(const dl_mlp_params *q, const float *params, void *ws, size_t ws_bytes,
                      dl_stream_t stream);

/* One minibatch of q->batch pairs: pair id pairs[b] names signal
   pairs[b] % m of Y [m][p] (p = in_dim) and the support row pairs[b] of hist
   ([*][s], -1 = empty slot).  Forward, loss, backward (gradients kept in the
   workspace); if step > 0, one Adam step with bias corrections for step
   number `step` (1-based). */
dl_status dl_mlp_train_step(const dl_mlp_params *q, void *ws, size_t ws_bytes, const float *Y,
                            int m, int p, const int32_t *hist, int s, const int32_t *pairs,
                            int step, dl_stream_t stream);

/* Copy the packed FP32 parameters and/or the last step's packed gradients
   to device buffers (either may be NULL); with loss != NULL, synchronise the
   stream and store the last step's mean loss (host double). */
dl_status dl_mlp_read(const dl_mlp_params *q, const void *ws, size_t ws_bytes, float *params,
                      float *grads, double *loss, dl_stream_t stream);

/* logits [rows][out_dim] (FP32) of the signals X [rows][in_dim]. */
dl_status dl_mlp_forward(const dl_mlp_params *q, void *ws, size_t ws_bytes, const float *X,
                         int rows, float *logits, dl_stream_t stream);

/* The k largest entries of every row of logits [rows][cols], largest first,
   ties to the lower index: out [rows][k] int32 (cols <= 1024, k <= 32). */
dl_status dl_topk(int rows, int cols, int k, const float *logits, int32_t *out,
                  dl_stream_t stream);

/* Kernels the library launches, for dl_profile_read. */
typedef enum {
    DL_K_GRAM = 0,      /* G = D D^T */
    DL_K_CORR,          /* A0 = Y D^T */
    DL_K_OMP,           /* per-signal OMP */
    DL_K_CSR_COUNT,     /* users of every atom: per-block counts */
    DL_K_CSR_SCAN,      /* users of every atom: offsets */
    DL_K_CSR_SCATTER,   /* users of every atom: placement */
    DL_K_UPD_PASS1,     /* F x^T per chunk of users */
    DL_K_UPD_REDUCE,    /* (reserved: the sum over chunks runs inside pass 2) */
    DL_K_UPD_PASS2,     /* sum over chunks, normalisation, AK-SVD refresh of X */
    DL_K_UPD_EUPDATE,   /* error update between groups */
    DL_K_RMSE,          /* error with the FP64 reduction */
    DL_K_MISC,          /* casts, copies, normalisation, residual */
    DL_K_MLP,           /* proposal network: GEMMs, loss, optimiser */
    DL_K_PROPOSE,       /* top-k candidates, restricted least squares, pruning */
    DL_K_COUNT
} dl_kernel;

/* Measurement support.  While enabled, every kernel launch of the library is
   bracketed by two HIP events recorded on the launch's own stream (the
   caller's), so that per-kernel GPU time can be read back.  Host-side state,
   not thread-safe; at most `max_launches` launches are recorded (later ones
   are not timed).  on = 0 disables and discards recorded events. */
dl_status dl_profile_enable(int on, int max_launches);

/* Wait for the recorded events, add each kernel's total time (ms) and launch
   count into ms[k] / launches[k] for k < count (count <= DL_K_COUNT), then
   clear the record (timing stays enabled). */
dl_status dl_profile_read(double *ms, long long *launches, int count);

/* As dl_iterate, and also record every iteration's OMP supports in hist
   [iters][m][s] (device, may be NULL) and the residual norm ||y - D X|| of
   every signal's last OMP in rref [m] (device, may be NULL): the training
   pairs and reference residuals of the learned proposal. */
dl_status dl_iterate_record(const dl_params *prm, const float *Y, float *D, int iters,
                            int32_t *X_idx, float *X_val, double *rmse, int32_t *hist,
                            float *rref, void *ws, size_t ws_bytes, dl_stream_t stream);

/* Learned support proposal for the coding stage. */
typedef struct dl_proposal {
    const int32_t *cand;  /* [m][k] candidate atoms per signal (device), e.g. dl_topk */
    int k;                /* candidates per signal: 8, 12 or 16, >= s */
    float margin;         /* hand a signal back to OMP when its residual exceeds
                             (1 + margin) times its reference OMP residual (0.02) */
    int audit_every;      /* code every signal with OMP on every audit_every-th
                             iteration (iterations audit_every, 2 audit_every, ...
                             of the call), refreshing the references (0 = never) */
} dl_proposal;

/* Bytes of the proposal workspace (fallback list and gathered signals). */
size_t dl_proposal_workspace_size(const dl_params *prm);

/* The coding stage of dl_iterate_proposed on its own (one call, no update):
   X_idx/X_val of every signal from the proposal or, when rejected, from OMP;
   rref is refreshed for the rejected signals. */
dl_status dl_code_proposed(const dl_params *prm, const dl_proposal *pr, const float *D,
                           const float *Y, float *rref, int32_t *X_idx, float *X_val, void *ws,
                           size_t ws_bytes, void *pws, size_t pws_bytes, dl_stream_t stream);

/* `iters` DL iterations whose coding stage uses the proposal: least squares
   restricted to the k candidates, backward elimination to s atoms (drop the
   atom whose removal raises the residual least), and OMP for the signals whose
   residual exceeds the margin (their reference residuals in rref [m] are
   refreshed); the atom update and the error are those of dl_iterate.  FP32
   only.  Arguments otherwise as dl_iterate; the fallback count is in the
   workspace statistics. */
dl_status dl_iterate_proposed(const dl_params *prm, const dl_proposal *pr, const float *Y,
                              float *D, int iters, float *rref, int32_t *X_idx, float *X_val,
                              double *rmse, void *ws, size_t ws_bytes, void *pws, size_t pws_bytes,
                              dl_stream_t stream);

/* ---- batched independent problems -----------------------------------------
   Many independent problems of uneven (p, n, m, s) iterate together (the DL
   iteration of Alg. 1 with all atoms in one Jacobi group, eq. 2).  Every
   stage of an iteration is one persistent launch over the problems: its
   workgroups take (problem, tile) items from a device queue, larger problems
   first; OMP runs one such launch per lane-group shape in use.  A problem
   whose coding launch alone fills the GPU (a full round of three waves per
   SIMD) runs instead with the launches of dl_iterate, on one of three
   streams the library keeps per device (default priority), concurrently
   with other such problems and with the shared launches; the caller's
   stream waits for them before the call's work counts as done.  Each
   problem gets bit-for-bit the results of dl_iterate with the same
   parameters. */
typedef struct dl_problem {
    dl_params prm;    /* FP32, group_size >= n and the AK-SVD or SGK rule only;
                         tolerances and OMP launch shape as for dl_iterate */
    const float *Y;   /* [m][p] signals (device, 16-byte aligned) */
    float *D;         /* [n][p] initial dictionary in, learned dictionary out
                         (rows are normalised first; device, 16-byte aligned) */
    int32_t *X_idx;   /* [m][s] out: atoms of the last coding (device) */
    float *X_val;     /* [m][s] out: coefficients after the last update (device) */
    double *rmse;     /* [iters] out: ||Y - D X||_F / sqrt(p m) after every
                         iteration (device, 8-byte aligned) */
} dl_problem;

/* Workspace bytes for the problems (host only; 0 if any is invalid or
   count is outside 1..4096). */
size_t dl_batch_workspace_size(const dl_problem *probs, int count);

/* `iters` iterations of every problem.  The workspace (device, 256-byte
   aligned, dl_batch_workspace_size bytes) needs no initialisation; the call
   copies its launch tables from host memory and synchronises `stream` once
   before enqueuing the iterations.  Problems must not share output buffers.
   DL_EINVAL for a bad problem, size or pointer (nothing is enqueued). */
dl_status dl_iterate_batched(const dl_problem *probs, int count, int iters, void *ws,
                             size_t ws_bytes, dl_stream_t stream);

/* Autotuner of the OMP launch shape of the problems that share the
   persistent launches (those that run alone keep theirs): for every
   distinct (p, n, s) among them it times
   each valid one-wave (omp_lanes_per_signal, omp_atoms_per_lane) with the
   OMP kernel of dl_iterate_batched on the largest such problem (its first
   65536 signals, correlations from its current D, `reps` timed launches
   after one warm-up, 1 <= reps <= 1000) and writes the
   fastest into prm of every such problem with that (p, n, s); the default shape
   is kept unless another is at least 5% faster.  Synchronous;
   overwrites X_idx and X_val of the problems it times, not D.  Workspace as
   for dl_iterate_batched. */
dl_status dl_autotune(dl_problem *probs, int count, int reps, void *ws, size_t ws_bytes,
                      dl_stream_t stream);

/* Synchronise `stream` and copy the workspace counters to *out (host).
   Returns DL_ENUMERIC if any non-finite value was counted, else DL_OK. */
dl_status dl_read_stats(const dl_params *prm, const void *ws, size_t ws_bytes, dl_stats *out,
                        dl_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* DL_MI355_H */
