// C ABI of the library (include/dl.h): argument validation, workspace
// layout and the launch order of one DL iteration (Alg. 1):
//   Gram G = D D^T, correlations A0 = Y D^T, OMP (+ residual E),
//   users of every atom (CSR), group atom update, error.
#include <string.h>

#include "dl_internal.h"

namespace dlk {

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool error_carried(const dl_params &prm) { return prm.group_size >= prm.n && error_defer_ok(prm.m); }

Layout layout_for(const dl_params &prm)
{
    const size_t p = prm.p, n = prm.n, m = prm.m, s = prm.s;
    const size_t nb = (size_t)csr_blocks(prm.m);
    Layout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += align256(bytes);
        return at;
    };
    L.control = take(sizeof(Control));
    const size_t ldn = (size_t)padded_n(prm.n);
    L.G = take(sizeof(float) * n * ldn);
    L.Gdiag = take(sizeof(float) * n);
    L.A0 = take(sizeof(float) * m * ldn);
    L.E = take(sizeof(float) * m * p);
    L.Dn = take(sizeof(float) * n * p);
    L.val_ws = take(sizeof(float) * m * s);
    L.valn = take(sizeof(float) * m * s);
    L.blkcnt = take(sizeof(int32_t) * nb * n);
    L.lrank = take(sizeof(int32_t) * m * s);
    L.atom_tot = take(sizeof(int32_t) * n);
    L.row_ptr = take(sizeof(int32_t) * (n + 1));
    L.chunk_ptr = take(sizeof(int32_t) * (n + 1));
    L.uent = take(sizeof(int2) * m * s);
    L.atom_state = take(sizeof(int32_t) * n);
    L.atom_cos = take(sizeof(float) * n);
    const size_t nsb = (size_t)gsum_signal_blocks(prm);
    const size_t chunks = (size_t)max_chunks(prm);
    L.partial = take(sizeof(float) * (chunks > n * nsb ? chunks : n * nsb) * p);
    L.bcnt = take(sizeof(int32_t) * (nsb ? n * nsb : 1));
    L.rmse_part = take(sizeof(double) * (size_t)rmse_blocks(prm.m));
    if (prm.rule == DL_RULE_NSGK || error_carried(prm)) {
        L.idx_prev = take(sizeof(int32_t) * m * s);
        L.val_prev = take(sizeof(float) * m * s);
    } else {
        L.idx_prev = L.val_prev = 0;
    }
    L.E2 = error_carried(prm) ? take(sizeof(float) * m * p) : 0;
    if (prm.precision == DL_PREC_BF16) {
        L.Dbf = take(sizeof(uint16_t) * n * p);
        L.Ybf = take(sizeof(uint16_t) * m * p);
    } else {
        L.Dbf = L.Ybf = 0;
    }
    L.total = off;
    return L;
}

}  // namespace dlk

using namespace dlk;

namespace {

bool valid_params(const dl_params *prm)
{
    if (!prm)
        return false;
    const dl_params &q = *prm;
    if (q.p < 4 || q.p > 256 || q.p % 4 != 0)
        return false;
    if (q.n < 1 || q.n > 1024 || q.m < 1)
        return false;
    if (q.s < 1 || q.s > 16 || q.s > q.p || q.s > q.n)
        return false;
    if ((long long)q.m * q.s >= (1ll << 31) || (long long)q.m * q.n >= (1ll << 40))
        return false;
    if (q.group_size < 1)
        return false;
    if (q.precision != DL_PREC_FP32 && q.precision != DL_PREC_BF16)
        return false;
    if (q.precision == DL_PREC_BF16 && q.p % 8 != 0)
        return false;
    if (q.rule != DL_RULE_AKSVD && q.rule != DL_RULE_SGK && q.rule != DL_RULE_NSGK)
        return false;
    if (!(q.pivot_fp64_threshold >= 0.f) || !(q.tol_corr >= 0.f) || !(q.tol_pivot >= 0.f))
        return false;
    if (q.omp_lanes_per_signal != 0 || q.omp_atoms_per_lane != 0) {
        const int npl = q.omp_atoms_per_lane ? q.omp_atoms_per_lane : 16;
        const int lps = q.omp_lanes_per_signal ? q.omp_lanes_per_signal
                                               : omp_lanes_per_signal(q.n, npl, q.s);
        if (!omp_config_ok(q.n, q.s, lps, npl))
            return false;
    }
    return true;
}

bool aligned(const void *ptr, size_t a) { return ptr && ((uintptr_t)ptr % a) == 0; }

}  // namespace

bool dlk::params_ok(const dl_params *prm) { return valid_params(prm); }

namespace {

struct Ws {
    char *base;
    Layout L;
    template <class T>
    T *at(size_t off) const { return reinterpret_cast<T *>(base + off); }
    Control *ctl() const { return at<Control>(L.control); }
};

dl_status check_ws(const dl_params *prm, const void *ws, size_t ws_bytes, Ws *out)
{
    if (!aligned(ws, 256))
        return DL_EINVAL;
    const Layout L = layout_for(*prm);
    if (ws_bytes < L.total)
        return DL_EWORKSPACE;
    out->base = (char *)ws;
    out->L = L;
    return DL_OK;
}

#define DL_TRY(expr)                               \
    do {                                           \
        if ((expr) != hipSuccess)                  \
            return DL_EHIP;                        \
    } while (0)

// G and A0 for the coding stage in one launch, in the precision the
// parameters ask for; rows of G and A0 have stride ldn.
// prev_err: optional error partials of the previous iteration, computed by
// extra workgroups of the grouped launch (independent of the products).
// Gdiag (the coding's copy of G only): G's diagonal goes there and NaN to G's
// diagonal.
dl_status products(const dl_params &prm, const float *D, const float *Y, float *G, float *A0,
                   const Ws *ws, hipStream_t st, int ldn, const int32_t *m_dev = nullptr,
                   const RmseArgs *prev_err = nullptr, float *Gdiag = nullptr)
{
    if (prev_err && (!(G && A0) || !prev_err->refresh))
        return DL_EINVAL;  // the launch carries only the refreshing error pass
    if (prm.precision == DL_PREC_BF16) {
        uint16_t *Dbf = ws->at<uint16_t>(ws->L.Dbf);
        uint16_t *Ybf = ws->at<uint16_t>(ws->L.Ybf);
        DL_TRY(launch_cast_bf16(D, Dbf, (size_t)prm.n * prm.p, st));
        DL_TRY(launch_cast_bf16(Y, Ybf, (size_t)prm.m * prm.p, st));
        const GemmBF16 g{Dbf, Dbf, G, prm.n, prm.n, prm.p, ldn, nullptr, Gdiag};
        const GemmBF16 c{Ybf, Dbf, A0, prm.m, prm.n, prm.p, ldn, m_dev};
        if (G && A0)
            DL_TRY(launch_gemm_nt_bf16(g, &c, DL_K_CORR, st, prev_err));
        else if (G)
            DL_TRY(launch_gemm_nt_bf16(g, nullptr, DL_K_GRAM, st));
        else if (A0)
            DL_TRY(launch_gemm_nt_bf16(c, nullptr, DL_K_CORR, st));
    } else {
        const GemmF32 g{D, D, G, prm.n, prm.n, prm.p, ldn, nullptr, Gdiag};
        const GemmF32 c{Y, D, A0, prm.m, prm.n, prm.p, ldn, m_dev};
        if (G && A0)
            DL_TRY(launch_gemm_nt_f32(g, &c, DL_K_CORR, st, prev_err));
        else if (G)
            DL_TRY(launch_gemm_nt_f32(g, nullptr, DL_K_GRAM, st));
        else if (A0)
            DL_TRY(launch_gemm_nt_f32(c, nullptr, DL_K_CORR, st));
    }
    return DL_OK;
}

struct OmpExtra {
    const float *Y = nullptr;      // compact signals (default: the caller's Y)
    const int32_t *m_dev = nullptr;
    const int32_t *rowmap = nullptr;
    float *rnorm = nullptr;
    float *E = nullptr;            // residual rows (default: the workspace's E)
    bool products = true;          // form G and A0 here
    // error partials carried by the coding launch (one wave per signal
    // group), else by the products launch; the coding must not write what
    // the error reads (X, E)
    const RmseArgs *prev_err = nullptr;
};

dl_status run_omp(const dl_params &prm, const float *D, const float *Y, int32_t *idx, float *val,
                  const Ws &ws, hipStream_t st, const OmpExtra &x = OmpExtra())
{
    float *G = ws.at<float>(ws.L.G);
    float *A0 = ws.at<float>(ws.L.A0);
    const float *Yin = x.Y ? x.Y : Y;
    const bool err_in_coding =
        x.prev_err && omp_carries_error(prm.n, prm.s, prm.omp_lanes_per_signal,
                                        prm.omp_atoms_per_lane);
    if (x.products) {
        dl_status rc = products(prm, D, Yin, G, A0, &ws, st, padded_n(prm.n), nullptr,
                                err_in_coding ? nullptr : x.prev_err, ws.at<float>(ws.L.Gdiag));
        if (rc != DL_OK)
            return rc;
    }
    if (x.prev_err && !x.products)
        return DL_EINVAL;
    OmpArgs a;
    a.A0 = A0;
    a.G = G;
    a.Gdiag = ws.at<float>(ws.L.Gdiag);
    a.Y = Yin;
    a.D = D;
    a.idx = idx;
    a.val = val;
    a.E = x.E ? x.E : ws.at<float>(ws.L.E);
    a.ctl = ws.ctl();
    a.p = prm.p;
    a.n = prm.n;
    a.m = prm.m;
    a.s = prm.s;
    a.ldn = padded_n(prm.n);
    a.m_dev = x.m_dev;
    a.rowmap = x.rowmap;
    a.rnorm = x.rnorm;
    a.lanes_per_signal = prm.omp_lanes_per_signal;
    a.atoms_per_lane = prm.omp_atoms_per_lane;
    a.pivot_fp64 = prm.pivot_fp64_threshold;
    a.tol_corr = prm.tol_corr;
    a.tol_pivot = prm.tol_pivot;
    DL_TRY(launch_omp(a, st, err_in_coding ? x.prev_err : nullptr));
    return DL_OK;
}

// prev_err: optional error whose partials are complete; its final sum is
// carried by the scan launch (by pass 1's launch when no user lists are
// built).
// The users are written as positions (users) or as (position, val there)
// pairs (uent); either may be null.
dl_status run_csr(const dl_params &prm, const int32_t *idx, int32_t *row_ptr, int32_t *users,
                  int2 *uent, const float *val, float *val_pad, const Ws &ws, hipStream_t st,
                  const RmseArgs *prev_err = nullptr)
{
    CsrArgs c;
    c.idx = idx;
    c.blkcnt = ws.at<int32_t>(ws.L.blkcnt);
    c.tot = ws.at<int32_t>(ws.L.atom_tot);
    c.ctl = ws.ctl();
    c.lrank = ws.at<int32_t>(ws.L.lrank);
    c.row_ptr = row_ptr;
    c.chunk_ptr = ws.at<int32_t>(ws.L.chunk_ptr);
    c.users = users;
    c.uent = uent;
    c.val = val;
    c.val_pad = val_pad;
    c.n = prm.n;
    c.m = prm.m;
    c.s = prm.s;
    c.chunk = chunk_users(prm);
    DL_TRY(launch_csr(c, st, prev_err));
    return DL_OK;
}

// One atom-update sweep reading (D, val) and writing (Dn, valn); E must hold
// Y - D X on entry.
// error_refreshes: the error pass that follows forms valn (all atoms in one
// group only); pass 2 then only forms Dn and the atom states.
dl_status run_update(const dl_params &prm, const float *Y, const float *D, float *Dn,
                     const int32_t *idx, const float *val, float *valn, const Ws &ws,
                     hipStream_t st, const RmseArgs *prev_err = nullptr,
                     bool error_refreshes = false, float *E = nullptr)
{
    int32_t *row_ptr = ws.at<int32_t>(ws.L.row_ptr);
    int2 *uent = ws.at<int2>(ws.L.uent);
    // pass 1 by signal blocks needs no user lists; pass 2 needs them only to
    // refresh X itself
    const int sig_block = gsum_block(prm);
    const bool lists = !(sig_block && error_refreshes);
    if (lists) {
        dl_status rc = run_csr(prm, idx, row_ptr, nullptr, uent, val, valn, ws, st, prev_err);
        if (rc != DL_OK)
            return rc;
    }
    UpdateArgs u;
    u.Y = Y;
    u.D = D;
    u.Dn = Dn;
    u.idx = idx;
    u.val = val;
    u.valn = valn;
    u.E = E ? E : ws.at<float>(ws.L.E);
    u.row_ptr = row_ptr;
    u.chunk_ptr = ws.at<int32_t>(ws.L.chunk_ptr);
    u.uent = uent;
    u.atom_state = ws.at<int32_t>(ws.L.atom_state);
    u.atom_cos = ws.at<float>(ws.L.atom_cos);
    u.partial = ws.at<float>(ws.L.partial);
    u.ctl = ws.ctl();
    u.p = prm.p;
    u.n = prm.n;
    u.m = prm.m;
    u.s = prm.s;
    u.group_size = prm.group_size;
    u.rule = prm.rule;
    u.max_chunks = max_chunks(prm);
    u.no_refresh = error_refreshes ? 1 : 0;
    u.chunk = chunk_users(prm);
    u.sig_block = sig_block;
    u.nsb = gsum_signal_blocks(prm);
    u.bcnt = ws.at<int32_t>(ws.L.bcnt);
    DL_TRY(launch_update(u, st, lists ? nullptr : prev_err));
    return DL_OK;
}

RmseArgs rmse_args(const dl_params &prm, const float *Y, const float *D, const int32_t *idx,
                   const float *val, double *out, const Ws &ws)
{
    RmseArgs r;
    r.Y = Y;
    r.D = D;
    r.idx = idx;
    r.val = val;
    r.partial = ws.at<double>(ws.L.rmse_part);
    r.out = out;
    r.ctl = ws.ctl();
    r.p = prm.p;
    r.n = prm.n;
    r.m = prm.m;
    r.s = prm.s;
    return r;
}

// The error pass also forms the refreshed coefficients valn from the
// coefficients val_old, the residual E and pass 2's d^T d' per atom (all
// atoms in one group, after an update with error_refreshes).
void add_refresh(RmseArgs &r, const dl_params &prm, const float *val_old, float *valn,
                 const Ws &ws, const float *E = nullptr)
{
    r.refresh = 1;
    r.E = E ? E : ws.at<float>(ws.L.E);
    r.val_old = val_old;
    r.atom_state = ws.at<int32_t>(ws.L.atom_state);
    r.atom_cos = ws.at<float>(ws.L.atom_cos);
    r.valn = valn;
    r.rule = prm.rule;
}

dl_status run_rmse(const dl_params &prm, const float *Y, const float *D, const int32_t *idx,
                   const float *val, double *out, const Ws &ws, hipStream_t st)
{
    DL_TRY(launch_rmse(rmse_args(prm, Y, D, idx, val, out, ws), st));
    return DL_OK;
}

}  // namespace

extern "C" {

int dl_abi_version(void) { return 1; }

const char *dl_status_string(int status)
{
    switch (status) {
    case DL_OK: return "DL_OK";
    case DL_EINVAL: return "DL_EINVAL: invalid argument";
    case DL_EWORKSPACE: return "DL_EWORKSPACE: workspace too small";
    case DL_EHIP: return "DL_EHIP: HIP launch or copy failed";
    case DL_ENUMERIC: return "DL_ENUMERIC: non-finite values met on the device";
    case DL_EUNSUPPORTED: return "DL_EUNSUPPORTED: option not built";
    default: return "unknown dl_status";
    }
}

dl_status dl_params_default(dl_params *prm, int p, int n, int m, int s)
{
    if (!prm)
        return DL_EINVAL;
    memset(prm, 0, sizeof(*prm));
    prm->p = p;
    prm->n = n;
    prm->m = m;
    prm->s = s;
    prm->group_size = n;
    prm->precision = DL_PREC_FP32;
    prm->rule = DL_RULE_AKSVD;
    prm->pivot_fp64_threshold = 1e-6f;
    prm->tol_corr = 1e-5f;
    prm->tol_pivot = 1e-10f;
    return valid_params(prm) ? DL_OK : DL_EINVAL;
}

size_t dl_workspace_size(const dl_params *prm)
{
    if (!valid_params(prm))
        return 0;
    return layout_for(*prm).total;
}

dl_status dl_workspace_init(const dl_params *prm, void *ws, size_t ws_bytes, dl_stream_t stream)
{
    if (!valid_params(prm))
        return DL_EINVAL;
    Ws w;
    dl_status rc = check_ws(prm, ws, ws_bytes, &w);
    if (rc != DL_OK)
        return rc;
    DL_TRY(launch_zero(w.ctl(), sizeof(Control), (hipStream_t)stream));
    return DL_OK;
}

dl_status dl_gram(const dl_params *prm, const float *D, float *G, dl_stream_t stream)
{
    if (!valid_params(prm) || !aligned(D, 16) || !aligned(G, 16))
        return DL_EINVAL;
    if (prm->precision != DL_PREC_FP32)
        return DL_EUNSUPPORTED;  // the BF16 product needs the workspace: use dl_omp
    const GemmF32 g{D, D, G, prm->n, prm->n, prm->p, prm->n};
    DL_TRY(launch_gemm_nt_f32(g, nullptr, DL_K_GRAM, (hipStream_t)stream));
    return DL_OK;
}

dl_status dl_corr(const dl_params *prm, const float *D, const float *Y, float *A0,
                  dl_stream_t stream)
{
    if (!valid_params(prm) || !aligned(D, 16) || !aligned(Y, 16) || !aligned(A0, 16))
        return DL_EINVAL;
    if (prm->precision != DL_PREC_FP32)
        return DL_EUNSUPPORTED;
    const GemmF32 c{Y, D, A0, prm->m, prm->n, prm->p, prm->n};
    DL_TRY(launch_gemm_nt_f32(c, nullptr, DL_K_CORR, (hipStream_t)stream));
    return DL_OK;
}

dl_status dl_products(const dl_params *prm, const float *D, const float *Y, float *G, float *A0,
                      void *ws, size_t ws_bytes, dl_stream_t stream)
{
    if (!valid_params(prm) || !aligned(D, 16) || !aligned(Y, 16) || !aligned(G, 4) ||
        !aligned(A0, 4))
        return DL_EINVAL;
    Ws w;
    dl_status rc = check_ws(prm, ws, ws_bytes, &w);
    if (rc != DL_OK)
        return rc;
    return products(*prm, D, Y, G, A0, &w, (hipStream_t)stream, prm->n);
}

dl_status dl_omp(const dl_params *prm, const float *D, const float *Y, int32_t *X_idx,
                 float *X_val, void *ws, size_t ws_bytes, dl_stream_t stream)
{
    if (!valid_params(prm) || !aligned(D, 16) || !aligned(Y, 16) || !aligned(X_idx, 4) ||
        !aligned(X_val, 4))
        return DL_EINVAL;
    Ws w;
    dl_status rc = check_ws(prm, ws, ws_bytes, &w);
    if (rc != DL_OK)
        return rc;
    return run_omp(*prm, D, Y, X_idx, X_val, w, (hipStream_t)stream);
}

dl_status dl_csr(const dl_params *prm, const int32_t *X_idx, int32_t *row_ptr, int32_t *users,
                 void *ws, size_t ws_bytes, dl_stream_t stream)
{
    if (!valid_params(prm) || !aligned(X_idx, 4) || !aligned(row_ptr, 4) || !aligned(users, 4))
        return DL_EINVAL;
    Ws w;
    dl_status rc = check_ws(prm, ws, ws_bytes, &w);
    if (rc != DL_OK)
        return rc;
    return run_csr(*prm, X_idx, row_ptr, users, nullptr, nullptr, nullptr, w,
                   (hipStream_t)stream);
}

dl_status dl_jau_update(const dl_params *prm, const float *Y, float *D, const int32_t *X_idx,
                        float *X_val, void *ws, size_t ws_bytes, dl_stream_t stream)
{
    if (!valid_params(prm) || !aligned(Y, 16) || !aligned(D, 16) || !aligned(X_idx, 4) ||
        !aligned(X_val, 4))
        return DL_EINVAL;
    Ws w;
    dl_status rc = check_ws(prm, ws, ws_bytes, &w);
    if (rc != DL_OK)
        return rc;
    if (prm->rule == DL_RULE_NSGK)
        return DL_EINVAL;  // the previous representations are needed: dl_jau_update_nsgk
    hipStream_t st = (hipStream_t)stream;
    const dl_params &q = *prm;
    float *E = w.at<float>(w.L.E);
    float *Dn = w.at<float>(w.L.Dn);
    float *valn = w.at<float>(w.L.valn);
    // E = Y - D X of the given representations (the first group's error)
    DL_TRY(launch_residual(Y, D, X_idx, X_val, E, q.p, q.n, q.m, q.s, st));
    rc = run_update(q, Y, D, Dn, X_idx, X_val, valn, w, st);
    if (rc != DL_OK)
        return rc;
    DL_TRY(launch_copy(Dn, D, sizeof(float) * (size_t)q.n * q.p, st));
    DL_TRY(launch_copy(valn, X_val, sizeof(float) * (size_t)q.m * q.s, st));
    return DL_OK;
}

dl_status dl_jau_update_nsgk(const dl_params *prm, const float *Y, float *D,
                             const int32_t *X_idx, const float *X_val,
                             const int32_t *Xprev_idx, const float *Xprev_val, void *ws,
                             size_t ws_bytes, dl_stream_t stream)
{
    if (!valid_params(prm) || prm->rule != DL_RULE_NSGK || !aligned(Y, 16) || !aligned(D, 16) ||
        !aligned(X_idx, 4) || !aligned(X_val, 4) || !aligned(Xprev_idx, 4) ||
        !aligned(Xprev_val, 4))
        return DL_EINVAL;
    Ws w;
    dl_status rc = check_ws(prm, ws, ws_bytes, &w);
    if (rc != DL_OK)
        return rc;
    hipStream_t st = (hipStream_t)stream;
    const dl_params &q = *prm;
    float *E = w.at<float>(w.L.E);
    float *Dn = w.at<float>(w.L.Dn);
    float *valn = w.at<float>(w.L.valn);
    // The first group's error Z - D X_prev = Y - D X (eq. 7); the users and
    // coefficients come from X_prev, whose coefficients the update keeps (the
    // kernels treat every rule but AK-SVD alike), and later groups keep E equal
    // to Z - D X_prev with the current D.
    DL_TRY(launch_residual(Y, D, X_idx, X_val, E, q.p, q.n, q.m, q.s, st));
    rc = run_update(q, Y, D, Dn, Xprev_idx, Xprev_val, valn, w, st);
    if (rc != DL_OK)
        return rc;
    DL_TRY(launch_copy(Dn, D, sizeof(float) * (size_t)q.n * q.p, st));
    return DL_OK;
}

dl_status dl_rmse(const dl_params *prm, const float *Y, const float *D, const int32_t *X_idx,
                  const float *X_val, double *rmse_out, void *ws, size_t ws_bytes,
                  dl_stream_t stream)
{
    if (!valid_params(prm) || !aligned(Y, 16) || !aligned(D, 16) || !aligned(X_idx, 4) ||
        !aligned(X_val, 4) || !aligned(rmse_out, 8))
        return DL_EINVAL;
    Ws w;
    dl_status rc = check_ws(prm, ws, ws_bytes, &w);
    if (rc != DL_OK)
        return rc;
    return run_rmse(*prm, Y, D, X_idx, X_val, rmse_out, w, (hipStream_t)stream);
}

static dl_status iterate_impl(const dl_params *prm, const float *Y, float *D, int iters,
                              int32_t *X_idx, float *X_val, double *rmse, int32_t *hist,
                              float *rref, void *ws, size_t ws_bytes, dl_stream_t stream)
{
    if (!valid_params(prm) || iters < 0 || !aligned(Y, 16) || !aligned(D, 16) ||
        !aligned(X_idx, 4) || !aligned(X_val, 4) || (iters > 0 && !aligned(rmse, 8)))
        return DL_EINVAL;
    Ws w;
    dl_status rc = check_ws(prm, ws, ws_bytes, &w);
    if (rc != DL_OK)
        return rc;
    hipStream_t st = (hipStream_t)stream;
    const dl_params &q = *prm;
    DL_TRY(launch_zero(w.ctl(), sizeof(Control), st));
    DL_TRY(launch_normalize_rows(D, q.n, q.p, w.ctl(), st));
    float *Dws = w.at<float>(w.L.Dn);
    float *val_ws = w.at<float>(w.L.val_ws);
    // the dictionary alternates between the caller's buffer and the workspace
    float *Dcur = D, *Dnext = Dws;
    const size_t ms = (size_t)q.m * q.s;
    // The error of iteration k needs only its outputs (Dn, X), the residual
    // E and the dictionary its coding used; nothing before iteration k+1's
    // update overwrites them when X and E alternate between two buffers.
    // For signal counts whose error partials take one signal block per
    // workgroup (latency-bound sizes), its partials run as extra workgroups
    // of k+1's coding launch (behind the coding workgroups, in its last,
    // partly occupied round; the two-wave coding shapes carry them in the
    // products launch instead) and its final sum in k+1's CSR scan launch:
    // two launches fewer per iteration, with the same bodies and block
    // decomposition as the error launches, so the same bits.  Larger counts
    // (each partial workgroup striding over several blocks) keep the error
    // launches, which measured faster there.  The last iteration's deferred
    // error runs on its own.  With all atoms in one group the refreshed X is
    // read only by the error and returned: the error pass forms it (pass 2
    // only forms d'), reading the residual E, the coefficients and the
    // dictionary the coding used.  The carried error needs that refresh, so
    // it is used at group size n only.
    const bool one_group = q.group_size >= q.n;
    const bool defer = error_carried(q);
    // NSGK updates with the previous iteration's coding (eq. 7) and keeps X:
    // the codings alternate between the caller's X and the workspace's
    // previous-coding buffers, arranged so that the last one lands in X.
    // A carried error runs in the next iteration's coding launch (shapes of
    // one wave per signal group) while that coding writes its own X and E,
    // so the codings and residuals alternate between two buffers as well.
    const bool nsgk = q.rule == DL_RULE_NSGK;
    const bool alt = nsgk || defer;
    int32_t *idx_buf[2] = {X_idx, alt ? w.at<int32_t>(w.L.idx_prev) : nullptr};
    float *val_buf[2] = {nsgk ? X_val : val_ws, alt ? w.at<float>(w.L.val_prev) : nullptr};
    float *E_buf[2] = {w.at<float>(w.L.E), defer ? w.at<float>(w.L.E2) : nullptr};
    RmseArgs prev{};
    bool pending = false;
    for (int k = 0; k < iters; ++k) {
        const int cb = (iters - 1 - k) & 1;
        int32_t *idx_k = alt ? idx_buf[cb] : X_idx;
        float *val_k = alt ? val_buf[cb] : val_ws;
        float *E_k = defer ? E_buf[cb] : E_buf[0];
        OmpExtra x;
        x.rnorm = rref;
        x.E = E_k;
        x.prev_err = pending ? &prev : nullptr;
        rc = run_omp(q, Dcur, Y, idx_k, val_k, w, st, x);
        if (rc != DL_OK)
            return rc;
        if (hist)
            DL_TRY(launch_copy(idx_k, hist + (size_t)k * ms, 4 * ms, st));
        if (nsgk) {
            // the users and coefficients of the previous coding (the first
            // iteration's own); the update's kept coefficients go to scratch
            const int32_t *idx_p = k == 0 ? idx_k : idx_buf[cb ^ 1];
            const float *val_p = k == 0 ? val_k : val_buf[cb ^ 1];
            rc = run_update(q, Y, Dcur, Dnext, idx_p, val_p, w.at<float>(w.L.valn), w, st,
                            pending ? &prev : nullptr, one_group, E_k);
        } else {
            rc = run_update(q, Y, Dcur, Dnext, idx_k, val_k, X_val, w, st,
                            pending ? &prev : nullptr, one_group, E_k);
        }
        if (rc != DL_OK)
            return rc;
        float *xout = nsgk ? val_k : X_val;
        prev = rmse_args(q, Y, Dnext, idx_k, xout, rmse + k, w);
        if (one_group)
            add_refresh(prev, q, val_k, xout, w, E_k);
        pending = defer;
        if (!defer)
            DL_TRY(launch_rmse(prev, st));
        float *t = Dcur;
        Dcur = Dnext;
        Dnext = t;
    }
    if (pending)
        DL_TRY(launch_rmse(prev, st));
    if (Dcur != D)
        DL_TRY(launch_copy(Dcur, D, sizeof(float) * (size_t)q.n * q.p, st));
    return DL_OK;
}

dl_status dl_iterate(const dl_params *prm, const float *Y, float *D, int iters, int32_t *X_idx,
                     float *X_val, double *rmse, void *ws, size_t ws_bytes, dl_stream_t stream)
{
    return iterate_impl(prm, Y, D, iters, X_idx, X_val, rmse, nullptr, nullptr, ws, ws_bytes,
                        stream);
}

dl_status dl_iterate_record(const dl_params *prm, const float *Y, float *D, int iters,
                            int32_t *X_idx, float *X_val, double *rmse, int32_t *hist,
                            float *rref, void *ws, size_t ws_bytes, dl_stream_t stream)
{
    if ((hist && !aligned(hist, 4)) || (rref && !aligned(rref, 4)))
        return DL_EINVAL;
    return iterate_impl(prm, Y, D, iters, X_idx, X_val, rmse, hist, rref, ws, ws_bytes, stream);
}

// Coding stage with the proposal: Gram matrix, restricted least squares and
// pruning for every signal, OMP for the rejected ones.
static dl_status code_proposed(const dl_params &q, const dl_proposal &pr, const float *D,
                               const float *Y, float *rref, int32_t *X_idx, float *val,
                               const Ws &w, void *pws, hipStream_t st)
{
    int32_t *fb_count = (int32_t *)pws;
    int32_t *fb_list = (int32_t *)((char *)pws + align256(sizeof(int32_t) * 64));
    float *Y_fb = (float *)((char *)fb_list + align256(sizeof(int32_t) * (size_t)q.m));
    float *G = w.at<float>(w.L.G);
    dl_status rc = products(q, D, Y, G, nullptr, &w, st, padded_n(q.n), nullptr, nullptr,
                            w.at<float>(w.L.Gdiag));
    if (rc != DL_OK)
        return rc;
    DL_TRY(launch_zero(fb_count, 4, st));
    ProposeArgs a;
    a.Y = Y;
    a.D = D;
    a.G = G;
    a.Gdiag = w.at<float>(w.L.Gdiag);
    a.cand = pr.cand;
    a.rref = rref;
    a.idx = X_idx;
    a.val = val;
    a.E = w.at<float>(w.L.E);
    a.fb_list = fb_list;
    a.fb_count = fb_count;
    a.ctl = w.ctl();
    a.p = q.p;
    a.n = q.n;
    a.m = q.m;
    a.s = q.s;
    a.ldn = padded_n(q.n);
    a.margin = pr.margin;
    DL_TRY(launch_ls_prune(a, pr.k, st));
    // the rejected signals are coded by OMP
    DL_TRY(launch_gather_list(Y, q.p, fb_list, fb_count, q.m, Y_fb, st));
    rc = products(q, D, Y_fb, nullptr, w.at<float>(w.L.A0), &w, st, padded_n(q.n), fb_count);
    if (rc != DL_OK)
        return rc;
    OmpExtra x;
    x.Y = Y_fb;
    x.m_dev = fb_count;
    x.rowmap = fb_list;
    x.rnorm = rref;
    x.products = false;
    return run_omp(q, D, Y, X_idx, val, w, st, x);
}

static bool proposal_ok(const dl_params *prm, const dl_proposal *pr, const void *pws,
                        size_t pws_bytes)
{
    return pr && aligned(pr->cand, 4) && (pr->k == 8 || pr->k == 12 || pr->k == 16) &&
           pr->k >= prm->s && pr->margin >= 0.f && pr->audit_every >= 0 &&
           prm->precision == DL_PREC_FP32 && prm->rule != DL_RULE_NSGK && aligned(pws, 256);
}

dl_status dl_code_proposed(const dl_params *prm, const dl_proposal *pr, const float *D,
                           const float *Y, float *rref, int32_t *X_idx, float *X_val, void *ws,
                           size_t ws_bytes, void *pws, size_t pws_bytes, dl_stream_t stream)
{
    if (!valid_params(prm) || !proposal_ok(prm, pr, pws, pws_bytes) || !aligned(D, 16) ||
        !aligned(Y, 16) || !aligned(rref, 4) || !aligned(X_idx, 4) || !aligned(X_val, 4))
        return DL_EINVAL;
    if (pws_bytes < dl_proposal_workspace_size(prm))
        return DL_EWORKSPACE;
    Ws w;
    dl_status rc = check_ws(prm, ws, ws_bytes, &w);
    if (rc != DL_OK)
        return rc;
    return code_proposed(*prm, *pr, D, Y, rref, X_idx, X_val, w, pws, (hipStream_t)stream);
}

size_t dl_proposal_workspace_size(const dl_params *prm)
{
    if (!valid_params(prm))
        return 0;
    const size_t m = prm->m, p = prm->p;
    return align256(sizeof(int32_t) * 64) + align256(sizeof(int32_t) * m) +
           align256(sizeof(float) * m * p);
}

dl_status dl_iterate_proposed(const dl_params *prm, const dl_proposal *pr, const float *Y,
                              float *D, int iters, float *rref, int32_t *X_idx, float *X_val,
                              double *rmse, void *ws, size_t ws_bytes, void *pws, size_t pws_bytes,
                              dl_stream_t stream)
{
    if (!valid_params(prm) || !proposal_ok(prm, pr, pws, pws_bytes) || iters < 0 ||
        !aligned(Y, 16) || !aligned(D, 16) || !aligned(X_idx, 4) || !aligned(X_val, 4) ||
        !aligned(rref, 4) || (iters > 0 && !aligned(rmse, 8)))
        return DL_EINVAL;
    if (pws_bytes < dl_proposal_workspace_size(prm))
        return DL_EWORKSPACE;
    Ws w;
    dl_status rc = check_ws(prm, ws, ws_bytes, &w);
    if (rc != DL_OK)
        return rc;
    hipStream_t st = (hipStream_t)stream;
    const dl_params &q = *prm;
    DL_TRY(launch_zero(w.ctl(), sizeof(Control), st));
    DL_TRY(launch_normalize_rows(D, q.n, q.p, w.ctl(), st));
    float *Dws = w.at<float>(w.L.Dn);
    float *val_ws = w.at<float>(w.L.val_ws);
    float *Dcur = D, *Dnext = Dws;
    for (int k = 0; k < iters; ++k) {
        const bool audit = pr->audit_every > 0 && (k + 1) % pr->audit_every == 0;
        if (audit) {
            OmpExtra x;
            x.rnorm = rref;
            rc = run_omp(q, Dcur, Y, X_idx, val_ws, w, st, x);
            if (rc != DL_OK)
                return rc;
        } else {
            rc = code_proposed(q, *pr, Dcur, Y, rref, X_idx, val_ws, w, pws, st);
            if (rc != DL_OK)
                return rc;
        }
        // all atoms in one group: the error pass refreshes X (as in iterate_impl)
        const bool one_group = q.group_size >= q.n;
        rc = run_update(q, Y, Dcur, Dnext, X_idx, val_ws, X_val, w, st, nullptr, one_group);
        if (rc != DL_OK)
            return rc;
        RmseArgs ra = rmse_args(q, Y, Dnext, X_idx, X_val, rmse + k, w);
        if (one_group)
            add_refresh(ra, q, val_ws, X_val, w);
        DL_TRY(launch_rmse(ra, st));
        float *t = Dcur;
        Dcur = Dnext;
        Dnext = t;
    }
    if (Dcur != D)
        DL_TRY(launch_copy(Dcur, D, sizeof(float) * (size_t)q.n * q.p, st));
    return DL_OK;
}

dl_status dl_read_stats(const dl_params *prm, const void *ws, size_t ws_bytes, dl_stats *out,
                        dl_stream_t stream)
{
    if (!valid_params(prm) || !out)
        return DL_EINVAL;
    Ws w;
    dl_status rc = check_ws(prm, ws, ws_bytes, &w);
    if (rc != DL_OK)
        return rc;
    Control c;
    DL_TRY(hipMemcpyAsync(&c, w.ctl(), sizeof(Control), hipMemcpyDeviceToHost,
                          (hipStream_t)stream));
    DL_TRY(hipStreamSynchronize((hipStream_t)stream));
    out->fp64_pivot_recomputes = (long long)c.fp64_pivot_recomputes;
    out->early_stops = (long long)c.early_stops;
    out->unused_atoms = (long long)c.unused_atoms;
    out->zero_updates = (long long)c.zero_updates;
    out->nonfinite = (long long)c.nonfinite;
    out->fallbacks = (long long)c.fallbacks;
    return c.nonfinite ? DL_ENUMERIC : DL_OK;
}

}  // extern "C"
