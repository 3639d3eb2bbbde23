// C ABI of the support-proposal network (include/dl.h, dl_mlp_*): workspace
// layout, one training step (gather, forward, loss, backward, Adam) and
// batched inference.
#include <string.h>

#include "dl_internal.h"

namespace dlk {
namespace {

constexpr int kSplits = 8;  // K splits of the weight-gradient GEMMs (K = batch)

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct MlpLayout {
    size_t P;  // packed parameter count
    size_t oW1, ob1, oW2, ob2, oW3, ob3;  // offsets (floats) inside a packed vector
    size_t params, m1, m2, grads, part;
    size_t W1b, W2b, W3b, W2tb, W3tb;
    size_t Xb, Xbt, H1, H1t, H2, H2t, Z, dZ, dZt, dA2, dA2t, dA1t, loss;
    size_t total;
};

bool mlp_valid(const dl_mlp_params *q)
{
    return q && q->in_dim >= 8 && q->in_dim % 8 == 0 && q->hidden >= 32 && q->hidden % 32 == 0 &&
           q->out_dim >= 1 && q->out_dim % 8 == 0 && q->batch >= 32 && q->batch % 32 == 0 &&
           q->lr > 0.f && q->beta1 >= 0.f && q->beta1 < 1.f && q->beta2 >= 0.f &&
           q->beta2 < 1.f && q->eps > 0.f && q->pos_weight > 0.f;
}

MlpLayout mlp_layout(const dl_mlp_params &q)
{
    const size_t I = q.in_dim, H = q.hidden, O = q.out_dim, B = q.batch;
    MlpLayout L;
    L.oW1 = 0;
    L.ob1 = L.oW1 + H * I;
    L.oW2 = L.ob1 + H;
    L.ob2 = L.oW2 + H * H;
    L.oW3 = L.ob2 + H;
    L.ob3 = L.oW3 + O * H;
    L.P = L.ob3 + O;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += al256(bytes);
        return at;
    };
    L.params = take(4 * L.P);
    L.m1 = take(4 * L.P);
    L.m2 = take(4 * L.P);
    L.grads = take(4 * L.P);
    size_t big = H * H;
    if (O * H > big)
        big = O * H;
    if (H * I > big)
        big = H * I;
    L.part = take(4 * big * kSplits);
    L.W1b = take(2 * H * I);
    L.W2b = take(2 * H * H);
    L.W3b = take(2 * O * H);
    L.W2tb = take(2 * H * H);
    L.W3tb = take(2 * H * O);
    L.Xb = take(2 * B * I);
    L.Xbt = take(2 * I * B);
    L.H1 = take(2 * B * H);
    L.H1t = take(2 * H * B);
    L.H2 = take(2 * B * H);
    L.H2t = take(2 * H * B);
    L.Z = take(4 * B * O);
    L.dZ = take(2 * B * O);
    L.dZt = take(2 * O * B);
    L.dA2 = take(2 * B * H);
    L.dA2t = take(2 * H * B);
    L.dA1t = take(2 * H * B);
    L.loss = take(8 * B);
    L.total = off;
    return L;
}

struct MWs {
    char *base;
    MlpLayout L;
    template <class T>
    T *at(size_t off) const { return reinterpret_cast<T *>(base + off); }
    float *P(size_t region, size_t elem) const { return at<float>(region) + elem; }
};

dl_status check_mws(const dl_mlp_params *q, const void *ws, size_t bytes, MWs *w)
{
    if (!mlp_valid(q))
        return DL_EINVAL;
    if (!ws || ((uintptr_t)ws % 256) != 0)
        return DL_EINVAL;
    w->L = mlp_layout(*q);
    if (bytes < w->L.total)
        return DL_EWORKSPACE;
    w->base = (char *)ws;
    return DL_OK;
}

#define MLP_TRY(expr)              \
    do {                           \
        if ((expr) != hipSuccess)  \
            return DL_EHIP;        \
    } while (0)

MlpGemm gemm(const uint16_t *A, int lda, const uint16_t *B, int ldb, int M, int N, int K, int epi)
{
    MlpGemm g;
    memset(&g, 0, sizeof(g));
    g.A = A;
    g.lda = lda;
    g.B = B;
    g.ldb = ldb;
    g.M = M;
    g.N = N;
    g.K = K;
    g.epi = epi;
    return g;
}

// Forward of `rows` (<= batch) rows already in Xb: H1, H2 (and their
// transposes when `keep_t`), logits Z (fp32, row stride ldz).
dl_status forward_rows(const dl_mlp_params &q, const MWs &w, int rows, float *Z, int ldz,
                       bool keep_t, hipStream_t st)
{
    const int I = q.in_dim, H = q.hidden, O = q.out_dim, B = q.batch;
    const MlpLayout &L = w.L;
    MlpGemm g1 = gemm(w.at<uint16_t>(L.Xb), I, w.at<uint16_t>(L.W1b), I, rows, H, I, kEpiBiasRelu);
    g1.bias = w.P(L.params, L.ob1);
    g1.Cb = w.at<uint16_t>(L.H1);
    g1.ldcb = H;
    g1.Ct = keep_t ? w.at<uint16_t>(L.H1t) : nullptr;
    g1.ldct = B;
    MLP_TRY(launch_mlp_gemm(g1, 1, st));
    MlpGemm g2 = gemm(w.at<uint16_t>(L.H1), H, w.at<uint16_t>(L.W2b), H, rows, H, H, kEpiBiasRelu);
    g2.bias = w.P(L.params, L.ob2);
    g2.Cb = w.at<uint16_t>(L.H2);
    g2.ldcb = H;
    g2.Ct = keep_t ? w.at<uint16_t>(L.H2t) : nullptr;
    g2.ldct = B;
    MLP_TRY(launch_mlp_gemm(g2, 1, st));
    MlpGemm g3 = gemm(w.at<uint16_t>(L.H2), H, w.at<uint16_t>(L.W3b), H, rows, O, H, kEpiF32);
    g3.bias = w.P(L.params, L.ob3);
    g3.Cf = Z;
    g3.ldcf = ldz;
    MLP_TRY(launch_mlp_gemm(g3, 1, st));
    return DL_OK;
}

// dW[M][N] = A[M][B] Bm[N][B]^T summed over the batch, split over K.
dl_status weight_grad(const dl_mlp_params &q, const MWs &w, const uint16_t *A, const uint16_t *Bm,
                      int M, int N, float *out, hipStream_t st)
{
    const int B = q.batch;
    MlpGemm g = gemm(A, B, Bm, B, M, N, B, kEpiF32);
    g.Cf = w.at<float>(w.L.part);
    g.ldcf = N;
    g.split_stride = (size_t)M * N;
    MLP_TRY(launch_mlp_gemm(g, kSplits, st));
    MLP_TRY(launch_sum_splits(w.at<float>(w.L.part), out, (size_t)M * N, kSplits, (size_t)M * N,
                              st));
    return DL_OK;
}

dl_status refresh_bf16(const dl_mlp_params &q, const MWs &w, const AdamHyper &h, int do_step,
                       hipStream_t st)
{
    const int I = q.in_dim, H = q.hidden, O = q.out_dim;
    const MlpLayout &L = w.L;
    float *p = w.at<float>(L.params), *g = w.at<float>(L.grads);
    float *m1 = w.at<float>(L.m1), *m2 = w.at<float>(L.m2);
    struct Arr {
        size_t off;
        int rows, cols;
        uint16_t *wb, *wbt;
    } arrs[6] = {
        {L.oW1, H, I, w.at<uint16_t>(L.W1b), nullptr},
        {L.ob1, 1, H, nullptr, nullptr},
        {L.oW2, H, H, w.at<uint16_t>(L.W2b), w.at<uint16_t>(L.W2tb)},
        {L.ob2, 1, H, nullptr, nullptr},
        {L.oW3, O, H, w.at<uint16_t>(L.W3b), w.at<uint16_t>(L.W3tb)},
        {L.ob3, 1, O, nullptr, nullptr},
    };
    for (const Arr &a : arrs)
        MLP_TRY(launch_adam(p + a.off, g + a.off, m1 + a.off, m2 + a.off, a.rows, a.cols, a.wb,
                            a.wbt, h, do_step, st));
    return DL_OK;
}

}  // namespace
}  // namespace dlk

using namespace dlk;

extern "C" {

size_t dl_mlp_param_count(const dl_mlp_params *q)
{
    if (!mlp_valid(q))
        return 0;
    return mlp_layout(*q).P;
}

size_t dl_mlp_workspace_size(const dl_mlp_params *q)
{
    if (!mlp_valid(q))
        return 0;
    return mlp_layout(*q).total;
}

dl_status dl_mlp_init(const dl_mlp_params *q, const float *params, void *ws, size_t ws_bytes,
                      dl_stream_t stream)
{
    MWs w;
    dl_status rc = check_mws(q, ws, ws_bytes, &w);
    if (rc != DL_OK)
        return rc;
    if (!params || ((uintptr_t)params % 4) != 0)
        return DL_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const MlpLayout &L = w.L;
    MLP_TRY(launch_copy(params, w.at<float>(L.params), 4 * L.P, st));
    MLP_TRY(launch_zero(w.at<float>(L.m1), 4 * L.P, st));
    MLP_TRY(launch_zero(w.at<float>(L.m2), 4 * L.P, st));
    MLP_TRY(launch_zero(w.at<float>(L.grads), 4 * L.P, st));
    AdamHyper h{q->lr, q->beta1, q->beta2, q->eps, 1.f, 1.f};
    return refresh_bf16(*q, w, h, 0, st);
}

dl_status dl_mlp_train_step(const dl_mlp_params *q, void *ws, size_t ws_bytes, const float *Y,
                            int m, int p, const int32_t *hist, int s, const int32_t *pairs,
                            int step, dl_stream_t stream)
{
    MWs w;
    dl_status rc = check_mws(q, ws, ws_bytes, &w);
    if (rc != DL_OK)
        return rc;
    if (!Y || !hist || !pairs || m < 1 || p != q->in_dim || s < 1 || step < 0 ||
        ((uintptr_t)Y % 4) != 0)
        return DL_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const int I = q->in_dim, H = q->hidden, O = q->out_dim, B = q->batch;
    const MlpLayout &L = w.L;
    MLP_TRY(launch_gather_batch(Y, m, p, pairs, B, w.at<uint16_t>(L.Xb), w.at<uint16_t>(L.Xbt), st));
    rc = forward_rows(*q, w, B, w.at<float>(L.Z), O, true, st);
    if (rc != DL_OK)
        return rc;
    MLP_TRY(launch_bce(w.at<float>(L.Z), O, hist, s, pairs, B, w.at<uint16_t>(L.dZ),
                       w.at<uint16_t>(L.dZt), w.at<double>(L.loss), q->pos_weight, st));
    float *gr = w.at<float>(L.grads);
    // layer 3
    rc = weight_grad(*q, w, w.at<uint16_t>(L.dZt), w.at<uint16_t>(L.H2t), O, H, gr + L.oW3, st);
    if (rc != DL_OK)
        return rc;
    MLP_TRY(launch_rowsum_bf16(w.at<uint16_t>(L.dZt), gr + L.ob3, O, B, st));
    MlpGemm d2 = gemm(w.at<uint16_t>(L.dZ), O, w.at<uint16_t>(L.W3tb), O, B, H, O, kEpiReluMask);
    d2.mask = w.at<uint16_t>(L.H2);
    d2.ldmask = H;
    d2.Cb = w.at<uint16_t>(L.dA2);
    d2.ldcb = H;
    d2.Ct = w.at<uint16_t>(L.dA2t);
    d2.ldct = B;
    MLP_TRY(launch_mlp_gemm(d2, 1, st));
    // layer 2
    rc = weight_grad(*q, w, w.at<uint16_t>(L.dA2t), w.at<uint16_t>(L.H1t), H, H, gr + L.oW2, st);
    if (rc != DL_OK)
        return rc;
    MLP_TRY(launch_rowsum_bf16(w.at<uint16_t>(L.dA2t), gr + L.ob2, H, B, st));
    MlpGemm d1 = gemm(w.at<uint16_t>(L.dA2), H, w.at<uint16_t>(L.W2tb), H, B, H, H, kEpiReluMask);
    d1.mask = w.at<uint16_t>(L.H1);
    d1.ldmask = H;
    d1.Ct = w.at<uint16_t>(L.dA1t);
    d1.ldct = B;
    MLP_TRY(launch_mlp_gemm(d1, 1, st));
    // layer 1
    rc = weight_grad(*q, w, w.at<uint16_t>(L.dA1t), w.at<uint16_t>(L.Xbt), H, I, gr + L.oW1, st);
    if (rc != DL_OK)
        return rc;
    MLP_TRY(launch_rowsum_bf16(w.at<uint16_t>(L.dA1t), gr + L.ob1, H, B, st));
    if (step > 0) {
        AdamHyper h{q->lr, q->beta1, q->beta2, q->eps,
                    1.f - powf(q->beta1, (float)step), 1.f - powf(q->beta2, (float)step)};
        return refresh_bf16(*q, w, h, 1, st);
    }
    return DL_OK;
}

dl_status dl_mlp_read(const dl_mlp_params *q, const void *ws, size_t ws_bytes, float *params,
                      float *grads, double *loss, dl_stream_t stream)
{
    MWs w;
    dl_status rc = check_mws(q, ws, ws_bytes, &w);
    if (rc != DL_OK)
        return rc;
    hipStream_t st = (hipStream_t)stream;
    const MlpLayout &L = w.L;
    if (params)
        MLP_TRY(launch_copy(w.at<float>(L.params), params, 4 * L.P, st));
    if (grads)
        MLP_TRY(launch_copy(w.at<float>(L.grads), grads, 4 * L.P, st));
    if (loss) {
        // host-side sum of the per-row losses of the last training step
        const int B = q->batch;
        double *rows = new double[B];
        if (hipMemcpyAsync(rows, w.at<double>(L.loss), 8 * (size_t)B, hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            delete[] rows;
            return DL_EHIP;
        }
        double acc = 0.0;
        for (int b = 0; b < B; ++b)
            acc += rows[b];
        delete[] rows;
        *loss = acc / ((double)B * (double)q->out_dim);
    }
    return DL_OK;
}

dl_status dl_mlp_forward(const dl_mlp_params *q, void *ws, size_t ws_bytes, const float *X,
                         int rows, float *logits, dl_stream_t stream)
{
    MWs w;
    dl_status rc = check_mws(q, ws, ws_bytes, &w);
    if (rc != DL_OK)
        return rc;
    if (!X || !logits || rows < 0 || ((uintptr_t)X % 4) != 0 || ((uintptr_t)logits % 4) != 0)
        return DL_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const int B = q->batch, O = q->out_dim, I = q->in_dim;
    for (int r0 = 0; r0 < rows; r0 += B) {
        const int nr = rows - r0 < B ? rows - r0 : B;
        MLP_TRY(launch_gather_rows(X + (size_t)r0 * I, nr, I, w.at<uint16_t>(w.L.Xb), st));
        rc = forward_rows(*q, w, nr, logits + (size_t)r0 * O, O, false, st);
        if (rc != DL_OK)
            return rc;
    }
    return DL_OK;
}

dl_status dl_topk(int rows, int cols, int k, const float *logits, int32_t *out, dl_stream_t stream)
{
    if (rows < 0 || cols < 1 || cols > 1024 || k < 1 || k > 32 || k > cols || !logits || !out)
        return DL_EINVAL;
    if (rows == 0)
        return DL_OK;
    MLP_TRY(launch_topk(logits, rows, cols, k, out, (hipStream_t)stream));
    return DL_OK;
}

}  // extern "C"
