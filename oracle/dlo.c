/*
 * FP64 CPU oracle for one dictionary-learning iteration with Jacobi atom
 * updates (Irofti & Dumitrescu, "Overcomplete Dictionary Learning with Jacobi
 * Atom Updates").
 *
 * TEST INFRASTRUCTURE ONLY.  It is the slow, plain, obviously correct
 * statement of what the GPU path computes.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it; the product path
 * never calls it and shares no code, header or table with it.
 *
 * Layouts (row-major):
 *   D   [n][p]  atom j is D + j*p
 *   Y   [m][p]  signal i is Y + i*p
 *   X   ELL     idx[m][s] (int32, -1 = unused slot), val[m][s] (double, 0 in
 *               unused slots); slot t holds the t-th atom selected for signal i.
 *
 * Readings of points the paper leaves open (listed in the design notes):
 *   - OMP ties go to the lowest atom index; selected atoms are excluded.
 *   - OMP stops early when every correlation of the residual is at most
 *     tol_corr * ||y|| (residual numerically orthogonal to all atoms, so y = 0
 *     gives an empty support) or when the new atom's Cholesky pivot is at most
 *     tol_pivot times its squared norm (atom in the span of the support).
 *   - An atom with no users, or whose F x^T is zero, keeps its value.
 *   - Group g covers atoms [g*gs, min((g+1)*gs, n)); groups run in index order.
 *   - The error is measured after the atom update, with the refreshed X.
 *   - P-NSGK: the group error is E = Z - D X^(k-1) with Z of eq. (7), the users
 *     I_j are those of X^(k-1); the first iteration, which has no earlier
 *     representation, takes X^(k-1) = X^(k) (then Z = Y and it is P-SGK).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define DLO_RULE_AKSVD 0
#define DLO_RULE_SGK 1
#define DLO_RULE_NSGK 2

static double dot(const double *a, const double *b, int p)
{
    double acc = 0.0;
    for (int k = 0; k < p; ++k)
        acc += a[k] * b[k];
    return acc;
}

/* Cholesky factor L (lower, row-major k x k) of the symmetric matrix A.
   Returns 0 on success, -1 if a pivot is not positive. */
static int cholesky(int k, const double *A, double *L)
{
    memset(L, 0, sizeof(double) * (size_t)k * k);
    for (int r = 0; r < k; ++r) {
        for (int c = 0; c <= r; ++c) {
            double acc = A[r * k + c];
            for (int t = 0; t < c; ++t)
                acc -= L[r * k + t] * L[c * k + t];
            if (r == c) {
                if (!(acc > 0.0))
                    return -1;
                L[r * k + r] = sqrt(acc);
            } else {
                L[r * k + c] = acc / L[c * k + c];
            }
        }
    }
    return 0;
}

/* Solve L z = b (forward substitution). */
static void solve_lower(int k, const double *L, const double *b, double *z)
{
    for (int r = 0; r < k; ++r) {
        double acc = b[r];
        for (int t = 0; t < r; ++t)
            acc -= L[r * k + t] * z[t];
        z[r] = acc / L[r * k + r];
    }
}

/* Solve L^T x = z (back substitution). */
static void solve_upper_t(int k, const double *L, const double *z, double *x)
{
    for (int r = k - 1; r >= 0; --r) {
        double acc = z[r];
        for (int t = r + 1; t < k; ++t)
            acc -= L[t * k + r] * x[t];
        x[r] = acc / L[r * k + r];
    }
}

/*
 * Orthogonal Matching Pursuit for one signal (Pati, Rezaiifar &
 * Krishnaprasad, the coder the paper runs in step 1 of its DL iteration,
 * with the fixed sparsity target s).  At every step: correlate the residual
 * with all atoms, add the atom of largest |correlation|, refit the
 * coefficients on the enlarged support by least squares (normal equations,
 * Cholesky), recompute the residual.
 * Returns 1 if it stopped before s atoms, 0 otherwise.
 */
int dlo_omp_signal(int p, int n, int s, const double *D, const double *y,
                   double tol_corr, double tol_pivot, int32_t *idx, double *val)
{
    int *sel = (int *)malloc(sizeof(int) * (size_t)s);
    char *used = (char *)calloc((size_t)n, 1);
    double *r = (double *)malloc(sizeof(double) * (size_t)p);
    double *A = (double *)malloc(sizeof(double) * (size_t)s * s);
    double *L = (double *)malloc(sizeof(double) * (size_t)s * s);
    double *b = (double *)malloc(sizeof(double) * (size_t)s);
    double *z = (double *)malloc(sizeof(double) * (size_t)s);
    double *x = (double *)calloc((size_t)s, sizeof(double));
    int k = 0;
    const double ynorm = sqrt(dot(y, y, p));
    memcpy(r, y, sizeof(double) * (size_t)p);

    while (k < s) {
        /* correlations of the residual with every atom not yet selected */
        int best = -1;
        double bestv = -1.0;
        for (int j = 0; j < n; ++j) {
            if (used[j])
                continue;
            double c = fabs(dot(D + (size_t)j * p, r, p));
            if (c > bestv) { /* strict: ties keep the lowest index */
                bestv = c;
                best = j;
            }
        }
        if (best < 0 || bestv <= tol_corr * ynorm)
            break;
        /* Gram matrix of the enlarged support and its Cholesky factor */
        int kk = k + 1;
        sel[k] = best;
        for (int a = 0; a < kk; ++a)
            for (int c = 0; c < kk; ++c)
                A[a * kk + c] = dot(D + (size_t)sel[a] * p, D + (size_t)sel[c] * p, p);
        if (cholesky(kk, A, L) != 0)
            break;
        double pivot = L[k * kk + k] * L[k * kk + k];
        if (pivot <= tol_pivot * A[k * kk + k])
            break;
        used[best] = 1;
        k = kk;
        /* least squares on the support: (D_I^T D_I) x = D_I^T y */
        for (int a = 0; a < k; ++a)
            b[a] = dot(D + (size_t)sel[a] * p, y, p);
        solve_lower(k, L, b, z);
        solve_upper_t(k, L, z, x);
        /* residual r = y - D_I x */
        for (int q = 0; q < p; ++q) {
            double acc = y[q];
            for (int a = 0; a < k; ++a)
                acc -= D[(size_t)sel[a] * p + q] * x[a];
            r[q] = acc;
        }
    }
    for (int t = 0; t < s; ++t) {
        idx[t] = t < k ? sel[t] : -1;
        val[t] = t < k ? x[t] : 0.0;
    }
    free(sel);
    free(used);
    free(r);
    free(A);
    free(L);
    free(b);
    free(z);
    free(x);
    return k < s;
}

/* OMP for all m signals.  Returns the number of signals that stopped early. */
long dlo_omp(int p, int n, int m, int s, const double *D, const double *Y,
             double tol_corr, double tol_pivot, int32_t *idx, double *val)
{
    long early = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : early)
    for (int i = 0; i < m; ++i)
        early += dlo_omp_signal(p, n, s, D, Y + (size_t)i * p, tol_corr, tol_pivot,
                                idx + (size_t)i * s, val + (size_t)i * s);
    return early;
}

/* E = Y - D X for all signals (the representation error of eq. (1)). */
void dlo_residual(int p, int m, int s, const double *Y, const double *D,
                  const int32_t *idx, const double *val, double *E)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < m; ++i) {
        double *e = E + (size_t)i * p;
        memcpy(e, Y + (size_t)i * p, sizeof(double) * (size_t)p);
        for (int t = 0; t < s; ++t) {
            int j = idx[(size_t)i * s + t];
            if (j < 0)
                continue;
            double x = val[(size_t)i * s + t];
            for (int q = 0; q < p; ++q)
                e[q] -= D[(size_t)j * p + q] * x;
        }
    }
}

/* ||Y - D X||_F / sqrt(p m). */
double dlo_rmse(int p, int m, int s, const double *Y, const double *D,
                const int32_t *idx, const double *val)
{
    double *E = (double *)malloc(sizeof(double) * (size_t)m * p);
    dlo_residual(p, m, s, Y, D, idx, val, E);
    double acc = 0.0;
    for (size_t k = 0; k < (size_t)m * p; ++k)
        acc += E[k] * E[k];
    free(E);
    return sqrt(acc / ((double)p * (double)m));
}

/*
 * Atom-update stage of one DL iteration with Jacobi atom updates: the group
 * loop of the paper's P-SGK algorithm (Alg. 2), with the atom rule chosen by
 * `rule`:
 *   AK-SVD (eq. 5): d_j = F x^T / ||F x^T||, then x_{j,I_j} = F^T d_j;
 *   SGK    (eq. 6): d_j = F x^T / (x x^T), then normalised; X unchanged.
 * For every group, E = Y - D X is recomputed from the current D and X (step
 * 2); every atom of the group reads the same group-start D, X and E (the
 * rule of eq. (2)); the group's new atoms and representations are committed
 * before the next group starts.  F = E_{I_j} + d_j x_{j,I_j} (eq. 3).
 * Only atoms [first_atom, end_atom) are visited (the whole sweep is [0, n));
 * the groups start at first_atom.
 * Returns the number of atom updates skipped because the atom had no users.
 */
long dlo_jau_update_range(int p, int n, int m, int s, const double *Y, double *D,
                          const int32_t *idx, double *val, int group_size, int rule,
                          int first_atom, int end_atom)
{
    double *E = (double *)malloc(sizeof(double) * (size_t)m * p);
    double *Dn = (double *)malloc(sizeof(double) * (size_t)n * p);
    double *valn = (double *)malloc(sizeof(double) * (size_t)m * s);
    long unused = 0;
    memcpy(Dn, D, sizeof(double) * (size_t)n * p);
    memcpy(valn, val, sizeof(double) * (size_t)m * s);

    for (int a0 = first_atom; a0 < end_atom; a0 += group_size) {
        int a1 = a0 + group_size < end_atom ? a0 + group_size : end_atom;
        dlo_residual(p, m, s, Y, D, idx, val, E);
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : unused)
        for (int j = a0; j < a1; ++j) {
            const double *dj = D + (size_t)j * p;
            double *g = (double *)calloc((size_t)p, sizeof(double));
            double *f = (double *)malloc(sizeof(double) * (size_t)p);
            double xx = 0.0;
            long users = 0;
            /* g = F x^T with F = E_{I_j} + d_j x_{j,I_j} */
            for (size_t e = 0; e < (size_t)m * s; ++e) {
                if (idx[e] != j)
                    continue;
                size_t i = e / (size_t)s;
                double x = val[e];
                for (int q = 0; q < p; ++q)
                    g[q] += (E[i * p + q] + dj[q] * x) * x;
                xx += x * x;
                ++users;
            }
            if (users == 0) {
                ++unused;
            } else {
                double gn = sqrt(dot(g, g, p));
                if (gn > 0.0) {
                    double *dn = Dn + (size_t)j * p;
                    if (rule == DLO_RULE_SGK) {
                        /* least-squares atom (eq. 6), then normalisation */
                        for (int q = 0; q < p; ++q)
                            dn[q] = g[q] / xx;
                        double dnn = sqrt(dot(dn, dn, p));
                        for (int q = 0; q < p; ++q)
                            dn[q] /= dnn;
                    } else {
                        /* one power-method step (eq. 5) */
                        for (int q = 0; q < p; ++q)
                            dn[q] = g[q] / gn;
                        for (size_t e = 0; e < (size_t)m * s; ++e) {
                            if (idx[e] != j)
                                continue;
                            size_t i = e / (size_t)s;
                            for (int q = 0; q < p; ++q)
                                f[q] = E[i * p + q] + dj[q] * val[e];
                            valn[e] = dot(f, dn, p);
                        }
                    }
                }
            }
            free(g);
            free(f);
        }
        /* commit the group */
        memcpy(D + (size_t)a0 * p, Dn + (size_t)a0 * p, sizeof(double) * (size_t)(a1 - a0) * p);
        for (size_t e = 0; e < (size_t)m * s; ++e)
            if (idx[e] >= a0 && idx[e] < a1)
                val[e] = valn[e];
    }
    free(E);
    free(Dn);
    free(valn);
    return unused;
}

/*
 * Atom-update stage of P-NSGK (Sec. 3): the P-SGK group loop applied to the
 * modified signals of eq. (7),
 *     Z = Y + D^(k) X^(k-1) - D^(k) X^(k),
 * with the representations X^(k-1) that the iteration started from in place
 * of X^(k) (ELL idx_prev/val_prev; X^(k) is idx/val).  D holds D^(k) on entry.
 * For every group the error is E = Z - D X^(k-1) with the current D (step 2
 * of Alg. 2 with Y replaced by Z and X by X^(k-1)), every atom of the group
 * reads the same group-start D and E (eq. 2), I_j are the signals whose
 * X^(k-1) uses d_j, F = E_{I_j} + d_j x_{j,I_j} (eq. 3) and
 * d_j = F x^T / (x x^T) (eq. 6), then normalised.  Neither X is changed.
 * Only atoms [first_atom, end_atom) are visited.  Returns the number of atom
 * updates skipped because the atom had no users in X^(k-1).
 */
long dlo_nsgk_update_range(int p, int n, int m, int s, const double *Y, double *D,
                           const int32_t *idx, const double *val, const int32_t *idx_prev,
                           const double *val_prev, int group_size, int first_atom,
                           int end_atom)
{
    double *Dk = (double *)malloc(sizeof(double) * (size_t)n * p);
    double *Z = (double *)malloc(sizeof(double) * (size_t)m * p);
    double *E = (double *)malloc(sizeof(double) * (size_t)m * p);
    double *Dn = (double *)malloc(sizeof(double) * (size_t)n * p);
    long unused = 0;
    memcpy(Dk, D, sizeof(double) * (size_t)n * p);
    memcpy(Dn, D, sizeof(double) * (size_t)n * p);

    /* Z = (Y - D^(k) X^(k)) + D^(k) X^(k-1) */
    dlo_residual(p, m, s, Y, Dk, idx, val, Z);
    for (int i = 0; i < m; ++i)
        for (int t = 0; t < s; ++t) {
            int j = idx_prev[(size_t)i * s + t];
            if (j < 0)
                continue;
            double x = val_prev[(size_t)i * s + t];
            for (int q = 0; q < p; ++q)
                Z[(size_t)i * p + q] += Dk[(size_t)j * p + q] * x;
        }

    for (int a0 = first_atom; a0 < end_atom; a0 += group_size) {
        int a1 = a0 + group_size < end_atom ? a0 + group_size : end_atom;
        dlo_residual(p, m, s, Z, D, idx_prev, val_prev, E);
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : unused)
        for (int j = a0; j < a1; ++j) {
            const double *dj = D + (size_t)j * p;
            double *g = (double *)calloc((size_t)p, sizeof(double));
            double xx = 0.0;
            long users = 0;
            for (size_t e = 0; e < (size_t)m * s; ++e) {
                if (idx_prev[e] != j)
                    continue;
                size_t i = e / (size_t)s;
                double x = val_prev[e];
                for (int q = 0; q < p; ++q)
                    g[q] += (E[i * p + q] + dj[q] * x) * x;
                xx += x * x;
                ++users;
            }
            if (users == 0) {
                ++unused;
            } else if (sqrt(dot(g, g, p)) > 0.0) {
                double *dn = Dn + (size_t)j * p;
                for (int q = 0; q < p; ++q)
                    dn[q] = g[q] / xx;
                double dnn = sqrt(dot(dn, dn, p));
                for (int q = 0; q < p; ++q)
                    dn[q] /= dnn;
            }
            free(g);
        }
        memcpy(D + (size_t)a0 * p, Dn + (size_t)a0 * p, sizeof(double) * (size_t)(a1 - a0) * p);
    }
    free(Dk);
    free(Z);
    free(E);
    free(Dn);
    return unused;
}

long dlo_jau_update(int p, int n, int m, int s, const double *Y, double *D,
                    const int32_t *idx, double *val, int group_size, int rule)
{
    return dlo_jau_update_range(p, n, m, s, Y, D, idx, val, group_size, rule, 0, n);
}

/* Scale every atom to unit norm (the constraint of the DL problem); zero atoms stay zero. */
void dlo_normalize(int p, int n, double *D)
{
    for (int j = 0; j < n; ++j) {
        double nr = sqrt(dot(D + (size_t)j * p, D + (size_t)j * p, p));
        if (nr > 0.0)
            for (int q = 0; q < p; ++q)
                D[(size_t)j * p + q] /= nr;
    }
}

/*
 * `iters` DL iterations (the paper's Alg. 1): sparse coding with OMP, then
 * the Jacobi atom update, then the error with the updated D and X.  D holds
 * D0 on entry (normalised first) and the final dictionary on exit; idx/val
 * hold the representations of the last iteration after its update;
 * rmse[k] is the error after iteration k.
 */
void dlo_iterate(int p, int n, int m, int s, const double *Y, double *D, int iters,
                 int group_size, int rule, double tol_corr, double tol_pivot,
                 int32_t *idx, double *val, double *rmse)
{
    /* P-NSGK keeps the representations the iteration started from; the first
       iteration has none before it and starts from its own X^(0) (so Z = Y). */
    int32_t *idx_prev = NULL;
    double *val_prev = NULL;
    if (rule == DLO_RULE_NSGK) {
        idx_prev = (int32_t *)malloc(sizeof(int32_t) * (size_t)m * s);
        val_prev = (double *)malloc(sizeof(double) * (size_t)m * s);
    }
    dlo_normalize(p, n, D);
    for (int k = 0; k < iters; ++k) {
        dlo_omp(p, n, m, s, D, Y, tol_corr, tol_pivot, idx, val);
        if (rule == DLO_RULE_NSGK) {
            if (k == 0) {
                memcpy(idx_prev, idx, sizeof(int32_t) * (size_t)m * s);
                memcpy(val_prev, val, sizeof(double) * (size_t)m * s);
            }
            dlo_nsgk_update_range(p, n, m, s, Y, D, idx, val, idx_prev, val_prev, group_size,
                                  0, n);
            memcpy(idx_prev, idx, sizeof(int32_t) * (size_t)m * s);
            memcpy(val_prev, val, sizeof(double) * (size_t)m * s);
        } else {
            dlo_jau_update(p, n, m, s, Y, D, idx, val, group_size, rule);
        }
        rmse[k] = dlo_rmse(p, m, s, Y, D, idx, val);
    }
    free(idx_prev);
    free(val_prev);
}

/* Threads the oracle's parallel loops use. */
int dlo_max_threads(void) { return omp_get_max_threads(); }

/* Set the number of threads of the following parallel loops (for timing). */
void dlo_set_threads(int threads) { omp_set_num_threads(threads > 0 ? threads : 1); }
