// Batched independent problems (include/dl.h, "batched problems"): tables of
// per-problem stage arguments, the work lists of the persistent launches,
// the launch order of an iteration, and the OMP launch-shape autotuner.
//
// Every stage of Alg. 1 runs for all problems in one launch whose workers
// take (problem, item) pairs from a device queue; problems are ordered by
// decreasing size so the largest items start first.  OMP is templated on its
// lane-group shape, so it runs one such launch per shape in use.  The stage
// bodies are those of the single-problem path, and every reduction keeps its
// order, so a batched problem gives bit-for-bit the single-problem results.
#include <string.h>

#include <algorithm>
#include <mutex>
#include <numeric>
#include <unordered_map>
#include <vector>

#include "dl_internal.h"

namespace dlk {

static std::mutex g_occ_mu;

// Compute units of the current device (queried once; 256 if the query fails).
static int device_cus_locked()
{
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                hipSuccess ||
            cus <= 0)
            cus = 256;
    }
    return cus;
}

int batch_workers(const void *kernel, int block, size_t lds, int items)
{
    static std::unordered_map<const void *, int> per_cu;
    int occ = 0, cus = 0;
    {
        std::lock_guard<std::mutex> lock(g_occ_mu);
        cus = device_cus_locked();
        auto it = per_cu.find(kernel);
        if (it != per_cu.end() && lds == 0) {
            occ = it->second;
        } else {
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, block, lds) !=
                    hipSuccess ||
                occ <= 0)
                occ = 1;
            if (lds == 0)
                per_cu[kernel] = occ;
        }
    }
    long long w = (long long)occ * cus;
    if (w > items)
        w = items;
    return w < 1 ? 1 : (int)w;
}

}  // namespace dlk

using namespace dlk;

namespace {

constexpr int kMaxProblems = 4096;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool problem_ok(const dl_problem &pb)
{
    const dl_params &q = pb.prm;
    if (!params_ok(&q) || q.precision != DL_PREC_FP32 || q.group_size < q.n ||
        q.rule == DL_RULE_NSGK)
        return false;
    auto al = [](const void *ptr, size_t a) { return ptr && ((uintptr_t)ptr % a) == 0; };
    return al(pb.Y, 16) && al(pb.D, 16) && al(pb.X_idx, 4) && al(pb.X_val, 4);
}

struct OmpShape {
    int lps, npl, smax;
    bool operator==(const OmpShape &o) const
    {
        return lps == o.lps && npl == o.npl && smax == o.smax;
    }
};

OmpShape shape_of(const dl_params &q)
{
    OmpShape sh;
    sh.npl = q.omp_atoms_per_lane > 0 ? q.omp_atoms_per_lane : omp_default_npl(q.n, q.s);
    sh.lps = q.omp_lanes_per_signal > 0 ? q.omp_lanes_per_signal
                                        : omp_lanes_per_signal(q.n, sh.npl, q.s);
    sh.smax = omp_smax(q.s);
    if (sh.lps == 128) {  // the batched OMP runs one wave per signal: the same values
        sh.lps = 64;
        sh.npl *= 2;
    }
    return sh;
}

// A problem whose coding launch alone holds a full round of waves (three per
// SIMD) runs with its own single-problem launches, on one of the side
// streams beside other such problems: sharing the persistent launches would
// only add queue tickets and argument lookups to work that fills the GPU,
// and the single-problem path has the launch shapes sized for it (two waves
// per signal for large n and s, the error carried in the coding launch).
// The smaller problems share the persistent launches on the caller's stream
// (measured on 64 uneven problems: persistent launches for all of them ran
// at 71 M signals*iters/s, one dl_iterate after another at 77 M).
// Work of one coding pass (flop), to balance the side streams.
double coding_work(const dl_params &q)
{
    return (double)q.m * ((double)q.n * (q.s * q.s + 3.0 * q.s) + 2.0 * q.p * q.n);
}

bool runs_alone(const dl_params &q)
{
    int cus;
    {
        std::lock_guard<std::mutex> lock(g_occ_mu);
        cus = device_cus_locked();
    }
    // decided on the default launch shape, so that a shape the autotuner
    // writes does not move a problem between the two groups
    const int npl = omp_default_npl(q.n, q.s);
    const int lps = omp_lanes_per_signal(q.n, npl, q.s);
    const long long waves = lps > 64 ? 2ll * q.m : ((long long)q.m * lps + 63) / 64;
    return waves >= 3ll * 4 * cus;
}

// Streams of the library for the problems that run alone: their iterations
// are independent, so up to kSideStreams of them run at once, and the small
// launches of one (CSR, update, error) overlap the others' work.  Created
// once per device with the default priority, never destroyed.
constexpr int kSideStreams = 3;

hipError_t side_streams(hipStream_t *out)
{
    static std::mutex mu;
    static std::unordered_map<int, std::vector<hipStream_t>> by_dev;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    std::lock_guard<std::mutex> lock(mu);
    std::vector<hipStream_t> &v = by_dev[dev];
    while ((int)v.size() < kSideStreams) {
        hipStream_t sd;
        if ((e = hipStreamCreateWithFlags(&sd, hipStreamNonBlocking)) != hipSuccess)
            return e;
        v.push_back(sd);
    }
    for (int i = 0; i < kSideStreams; ++i)
        out[i] = v[i];
    return hipSuccess;
}

// Byte offsets of the batch workspace: queue, controls, tables and work
// lists, then every problem's own single-problem workspace.
struct BatchLayout {
    size_t queue, ctl, gemm, omp, csr, upd, rmse, norm, lists, probs_begin, total;
    std::vector<size_t> prob;  // workspace offset of every problem (input order)
    int lists_len;             // int32 entries of the work lists
};

BatchLayout batch_layout(const dl_problem *probs, int count)
{
    BatchLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += align256(bytes);
        return at;
    };
    const size_t c = (size_t)count;
    L.queue = take(sizeof(BatchQueue));
    L.ctl = take(sizeof(Control) * c);
    L.gemm = take(sizeof(GemmPair) * 2 * c);
    L.omp = take(sizeof(OmpArgs) * 2 * c);
    L.csr = take(sizeof(CsrArgs) * c);
    L.upd = take(sizeof(UpdateArgs) * 2 * c);
    L.rmse = take(sizeof(RmseArgs) * 2 * c);
    L.norm = take(sizeof(NormArgs) * c);
    // 8 stage lists of count + 1 entries, and at most count shape lists of
    // (problems in the shape + 1) entries
    L.lists_len = (int)(9 * (c + 1) + 2 * c);
    L.lists = take(sizeof(int32_t) * (size_t)L.lists_len);
    L.probs_begin = off;
    L.prob.resize(c);
    for (int b = 0; b < count; ++b)
        L.prob[b] = take(layout_for(probs[b].prm).total);
    L.total = off;
    return L;
}

struct Plan {
    // host images of the device tables
    std::vector<GemmPair> gemm;   // [2][count], sorted order
    std::vector<OmpArgs> omp;     // [2][count], shape order
    std::vector<CsrArgs> csr;     // [count], sorted order
    std::vector<UpdateArgs> upd;  // [2][count]
    std::vector<RmseArgs> rmse;   // [2][count]
    std::vector<NormArgs> norm;   // [count]
    std::vector<int32_t> lists;
    // per stage: offset of its list in `lists` and its item total
    int l_gemm, l_count, l_quad, l_scatter, l_pass1, l_chunk, l_rmse, l_one;
    int n_gemm, n_count, n_quad, n_scatter, n_pass1, n_chunk, n_rmse, n_one;
    struct Shape {
        OmpShape sh;
        int first, num;  // problems [first, first + num) of the OMP table
        int list, items;
    };
    std::vector<Shape> shapes;
    int max_n;
};

// Both parities of the per-problem arguments: in iteration k the dictionary
// is read from buffer k % 2 (0 = the caller's D, 1 = the workspace's Dn) and
// the update writes the other one.
void build_plan(const dl_problem *probs, const std::vector<int> &members, char *base,
                const BatchLayout &L, Plan &P)
{
    const int count = (int)members.size();
    std::vector<int> order(members);
    auto size_key = [&](int b) {
        const dl_params &q = probs[b].prm;
        return (long long)q.n * q.s * 1024 + q.p;
    };
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return size_key(x) > size_key(y); });
    Control *ctl = reinterpret_cast<Control *>(base + L.ctl);
    P.gemm.resize(2 * count);
    P.omp.resize(2 * count);
    P.csr.resize(count);
    P.upd.resize(2 * count);
    P.rmse.resize(2 * count);
    P.norm.resize(count);
    P.max_n = 0;
    std::vector<int> it_gemm(count), it_count(count), it_quad(count), it_scatter(count),
        it_pass1(count), it_chunk(count), it_rmse(count);
    for (int r = 0; r < count; ++r) {
        const int b = order[r];
        const dl_problem &pb = probs[b];
        const dl_params &q = pb.prm;
        const Layout W = layout_for(q);
        char *wb = base + L.prob[b];
        auto f = [&](size_t o) { return reinterpret_cast<float *>(wb + o); };
        auto i32 = [&](size_t o) { return reinterpret_cast<int32_t *>(wb + o); };
        const int ldn = padded_n(q.n);
        float *Dbuf[2] = {pb.D, f(W.Dn)};
        Control *c = ctl + b;
        for (int par = 0; par < 2; ++par) {
            const float *Dc = Dbuf[par];
            float *Dx = Dbuf[par ^ 1];
            GemmPair gp;
            gp.g = GemmF32{Dc, Dc, f(W.G), q.n, q.n, q.p, ldn, nullptr, f(W.Gdiag)};
            gp.c = GemmF32{pb.Y, Dc, f(W.A0), q.m, q.n, q.p, ldn, nullptr};
            P.gemm[par * count + r] = gp;
            UpdateArgs u;
            memset(&u, 0, sizeof(u));
            u.Y = pb.Y;
            u.D = Dc;
            u.Dn = Dx;
            u.idx = pb.X_idx;
            u.val = f(W.val_ws);
            u.valn = pb.X_val;
            u.E = f(W.E);
            u.row_ptr = i32(W.row_ptr);
            u.chunk_ptr = i32(W.chunk_ptr);
            u.uent = reinterpret_cast<const int2 *>(wb + W.uent);
            u.atom_state = i32(W.atom_state);
            u.atom_cos = f(W.atom_cos);
            u.partial = f(W.partial);
            u.ctl = c;
            u.p = q.p;
            u.n = q.n;
            u.m = q.m;
            u.s = q.s;
            u.group_size = q.n;
            u.rule = q.rule;
            u.max_chunks = max_chunks(q);
            u.chunk = chunk_users(q);
            u.sig_block = gsum_block(q);
            u.nsb = gsum_signal_blocks(q);
            u.bcnt = i32(W.bcnt);
            P.upd[par * count + r] = u;
            RmseArgs rm;
            rm.Y = pb.Y;
            rm.D = Dx;  // the error after the update
            rm.idx = pb.X_idx;
            rm.val = pb.X_val;
            rm.partial = reinterpret_cast<double *>(wb + W.rmse_part);
            rm.out = pb.rmse;
            rm.ctl = c;
            rm.p = q.p;
            rm.n = q.n;
            rm.m = q.m;
            rm.s = q.s;
            P.rmse[par * count + r] = rm;
        }
        CsrArgs cs;
        cs.idx = pb.X_idx;
        cs.blkcnt = i32(W.blkcnt);
        cs.tot = i32(W.atom_tot);
        cs.ctl = c;
        cs.lrank = i32(W.lrank);
        cs.row_ptr = i32(W.row_ptr);
        cs.chunk_ptr = i32(W.chunk_ptr);
        cs.users = nullptr;
        cs.uent = reinterpret_cast<int2 *>(wb + W.uent);
        cs.val = f(W.val_ws);
        cs.val_pad = pb.X_val;
        cs.n = q.n;
        cs.m = q.m;
        cs.s = q.s;
        cs.chunk = chunk_users(q);
        P.csr[r] = cs;
        P.norm[r] = NormArgs{pb.D, q.n, q.p, c};
        it_gemm[r] = gemm_pair_items(P.gemm[r]);
        it_count[r] = csr_blocks(q.m);
        it_quad[r] = (q.n + 3) / 4;
        it_scatter[r] = (int)(((long long)q.m * q.s + 255) / 256);
        it_chunk[r] = max_chunks(q);
        it_pass1[r] = gsum_block(q) ? gsum_items(q) : it_chunk[r];
        it_rmse[r] = rmse_blocks(q.m);
        P.max_n = std::max(P.max_n, q.n);
    }
    P.lists.clear();
    auto add_list = [&](const std::vector<int> &items, int &at, int &total) {
        at = (int)P.lists.size();
        int run = 0;
        P.lists.push_back(0);
        for (int v : items) {
            run += v;
            P.lists.push_back(run);
        }
        total = run;
    };
    add_list(it_gemm, P.l_gemm, P.n_gemm);
    add_list(it_count, P.l_count, P.n_count);
    add_list(it_quad, P.l_quad, P.n_quad);
    add_list(it_scatter, P.l_scatter, P.n_scatter);
    add_list(it_pass1, P.l_pass1, P.n_pass1);
    add_list(it_chunk, P.l_chunk, P.n_chunk);
    add_list(it_rmse, P.l_rmse, P.n_rmse);
    add_list(std::vector<int>(count, 1), P.l_one, P.n_one);

    // OMP: problems grouped by launch shape (shapes of larger groups first)
    P.shapes.clear();
    std::vector<int> shape_of_rank(count);
    for (int r = 0; r < count; ++r) {
        const OmpShape sh = shape_of(probs[order[r]].prm);
        int k = 0;
        while (k < (int)P.shapes.size() && !(P.shapes[k].sh == sh))
            ++k;
        if (k == (int)P.shapes.size())
            P.shapes.push_back(Plan::Shape{sh, 0, 0, 0, 0});
        shape_of_rank[r] = k;
    }
    int next = 0;
    for (size_t k = 0; k < P.shapes.size(); ++k) {
        Plan::Shape &S = P.shapes[k];
        S.first = next;
        std::vector<int> items;
        for (int r = 0; r < count; ++r) {
            if (shape_of_rank[r] != (int)k)
                continue;
            const int b = order[r];
            for (int par = 0; par < 2; ++par) {
                const UpdateArgs &u = P.upd[par * count + r];
                const GemmPair &gp = P.gemm[par * count + r];
                OmpArgs a;
                memset(&a, 0, sizeof(a));
                a.A0 = gp.c.C;
                a.G = gp.g.C;
                a.Gdiag = gp.g.diag;
                a.Y = probs[b].Y;
                a.D = u.D;
                a.idx = probs[b].X_idx;
                a.val = const_cast<float *>(u.val);  // the workspace coefficients
                a.E = u.E;
                a.ctl = u.ctl;
                a.p = u.p;
                a.n = u.n;
                a.m = u.m;
                a.s = u.s;
                a.ldn = padded_n(u.n);
                a.lanes_per_signal = S.sh.lps;
                a.atoms_per_lane = S.sh.npl;
                a.pivot_fp64 = probs[b].prm.pivot_fp64_threshold;
                a.tol_corr = probs[b].prm.tol_corr;
                a.tol_pivot = probs[b].prm.tol_pivot;
                P.omp[par * count + next] = a;
            }
            const int gpw = omp_signals_per_item(S.sh.lps);
            items.push_back((probs[b].prm.m + gpw - 1) / gpw);
            ++next;
        }
        S.num = next - S.first;
        add_list(items, S.list, S.items);
    }
}

}  // namespace

#define DL_TRY(expr)                               \
    do {                                           \
        if ((expr) != hipSuccess)                  \
            return DL_EHIP;                        \
    } while (0)

// The caller's stream waits for everything enqueued on the side streams.
hipError_t join_side_streams(hipStream_t st)
{
    hipStream_t side[kSideStreams];
    hipError_t e = side_streams(side);
    for (int i = 0; i < kSideStreams && e == hipSuccess; ++i) {
        hipEvent_t done;
        if ((e = hipEventCreateWithFlags(&done, hipEventDisableTiming)) != hipSuccess)
            break;
        e = hipEventRecord(done, side[i]);
        if (e == hipSuccess)
            e = hipStreamWaitEvent(st, done, 0);
        hipEventDestroy(done);
    }
    return e;
}

// The problems of `shared` iterate together in persistent launches on st.
dl_status iterate_shared(const dl_problem *probs, const std::vector<int> &shared, int iters,
                         char *base, const BatchLayout &L, hipStream_t st)
{
    Plan P;
    build_plan(probs, shared, base, L, P);
    const int count = (int)shared.size();
    const size_t c = (size_t)count;
    DL_TRY(hipMemcpyAsync(base + L.gemm, P.gemm.data(), sizeof(GemmPair) * 2 * c,
                          hipMemcpyHostToDevice, st));
    DL_TRY(hipMemcpyAsync(base + L.omp, P.omp.data(), sizeof(OmpArgs) * 2 * c,
                          hipMemcpyHostToDevice, st));
    DL_TRY(hipMemcpyAsync(base + L.csr, P.csr.data(), sizeof(CsrArgs) * c, hipMemcpyHostToDevice,
                          st));
    DL_TRY(hipMemcpyAsync(base + L.upd, P.upd.data(), sizeof(UpdateArgs) * 2 * c,
                          hipMemcpyHostToDevice, st));
    DL_TRY(hipMemcpyAsync(base + L.rmse, P.rmse.data(), sizeof(RmseArgs) * 2 * c,
                          hipMemcpyHostToDevice, st));
    DL_TRY(hipMemcpyAsync(base + L.norm, P.norm.data(), sizeof(NormArgs) * c,
                          hipMemcpyHostToDevice, st));
    DL_TRY(hipMemcpyAsync(base + L.lists, P.lists.data(), sizeof(int32_t) * P.lists.size(),
                          hipMemcpyHostToDevice, st));
    // the host images are released on return
    DL_TRY(hipStreamSynchronize(st));
    DL_TRY(launch_zero(base + L.queue, L.gemm - L.queue, st));  // queue and controls

    BatchQueue *q = reinterpret_cast<BatchQueue *>(base + L.queue);
    const int32_t *lists = reinterpret_cast<const int32_t *>(base + L.lists);
    auto list = [&](int at, int num) { return BatchList{lists + at, num, q}; };
    const GemmPair *gemm = reinterpret_cast<const GemmPair *>(base + L.gemm);
    const OmpArgs *omp = reinterpret_cast<const OmpArgs *>(base + L.omp);
    const CsrArgs *csr = reinterpret_cast<const CsrArgs *>(base + L.csr);
    const UpdateArgs *upd = reinterpret_cast<const UpdateArgs *>(base + L.upd);
    const RmseArgs *rmse = reinterpret_cast<const RmseArgs *>(base + L.rmse);
    const NormArgs *norm = reinterpret_cast<const NormArgs *>(base + L.norm);

    DL_TRY(launch_batched_normalize(norm, list(P.l_quad, count), P.n_quad, st));
    // As in the single-problem iteration, the error of iteration k is carried
    // by iteration k+1's launches (partials with the products, final sums
    // with the CSR scans); the last one runs on its own.  Same bodies and
    // block decompositions, so every problem gets the same bits either way.
    for (int k = 0; k < iters; ++k) {
        const size_t par = (size_t)(k & 1) * c;
        const RmseArgs *prev = k > 0 ? rmse + (size_t)((k - 1) & 1) * c : nullptr;
        DL_TRY(launch_batched_gemm(gemm + par, list(P.l_gemm, count), P.n_gemm, st, prev,
                                   list(P.l_rmse, count), P.n_rmse));
        for (const Plan::Shape &S : P.shapes)
            DL_TRY(launch_batched_omp(omp + par + S.first, list(S.list, S.num), S.items, S.sh.lps,
                                      S.sh.npl, S.sh.smax, st));
        DL_TRY(launch_batched_csr(csr, list(P.l_count, count), P.n_count, list(P.l_quad, count),
                                  P.n_quad, list(P.l_scatter, count), P.n_scatter, P.max_n, st,
                                  prev, list(P.l_one, count), k - 1));
        DL_TRY(launch_batched_update(upd + par, list(P.l_pass1, count), P.n_pass1,
                                     list(P.l_chunk, count), P.n_chunk, st));
    }
    if (iters > 0)
        DL_TRY(launch_batched_rmse(rmse + (size_t)((iters - 1) & 1) * c, list(P.l_rmse, count),
                                   P.n_rmse, list(P.l_one, count), iters - 1, st));
    if (iters % 2 == 1)
        for (int b : shared) {
            const dl_params &pq = probs[b].prm;
            const Layout W = layout_for(pq);
            DL_TRY(launch_copy(base + L.prob[b] + W.Dn, probs[b].D,
                               sizeof(float) * (size_t)pq.n * pq.p, st));
        }
    return DL_OK;
}

extern "C" {

size_t dl_batch_workspace_size(const dl_problem *probs, int count)
{
    if (!probs || count < 1 || count > kMaxProblems)
        return 0;
    for (int b = 0; b < count; ++b) {
        const dl_params &q = probs[b].prm;
        if (!params_ok(&q) || q.precision != DL_PREC_FP32 || q.group_size < q.n ||
            q.rule == DL_RULE_NSGK)
            return 0;
    }
    return batch_layout(probs, count).total;
}

dl_status dl_iterate_batched(const dl_problem *probs, int count, int iters, void *ws,
                             size_t ws_bytes, dl_stream_t stream)
{
    if (!probs || count < 1 || count > kMaxProblems || iters < 0 || !ws ||
        ((uintptr_t)ws % 256) != 0)
        return DL_EINVAL;
    for (int b = 0; b < count; ++b)
        if (!problem_ok(probs[b]) ||
            (iters > 0 && (!probs[b].rmse || ((uintptr_t)probs[b].rmse % 8) != 0)))
            return DL_EINVAL;
    const BatchLayout L = batch_layout(probs, count);
    if (ws_bytes < L.total)
        return DL_EWORKSPACE;
    char *base = (char *)ws;
    hipStream_t st = (hipStream_t)stream;
    std::vector<int> shared, alone;
    for (int b = 0; b < count; ++b)
        (runs_alone(probs[b].prm) ? alone : shared).push_back(b);
    if (!alone.empty()) {
        // the problems that run alone go to the side streams, largest first,
        // each to the stream with the least work so far; the side streams
        // start after the caller's earlier work and the caller's stream
        // waits for them at the end of the call
        std::sort(alone.begin(), alone.end(), [&](int x, int y) {
            return coding_work(probs[x].prm) > coding_work(probs[y].prm);
        });
        hipStream_t side[kSideStreams];
        DL_TRY(side_streams(side));
        hipEvent_t ev;
        DL_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        hipError_t e = hipEventRecord(ev, st);
        for (int i = 0; i < kSideStreams && e == hipSuccess; ++i)
            e = hipStreamWaitEvent(side[i], ev, 0);
        hipEventDestroy(ev);
        DL_TRY(e);
        double load[kSideStreams] = {0.0};
        dl_status rc = DL_OK;
        for (int b : alone) {
            int i = 0;
            for (int j = 1; j < kSideStreams; ++j)
                if (load[j] < load[i])
                    i = j;
            load[i] += coding_work(probs[b].prm);
            const dl_problem &pb = probs[b];
            rc = dl_iterate(&pb.prm, pb.Y, pb.D, iters, pb.X_idx, pb.X_val, pb.rmse,
                            base + L.prob[b], layout_for(pb.prm).total, side[i]);
            if (rc != DL_OK)
                break;
        }
        if (rc != DL_OK) {
            join_side_streams(st);
            return rc;
        }
    }
    dl_status rc = shared.empty() ? DL_OK : iterate_shared(probs, shared, iters, base, L, st);
    if (!alone.empty() && join_side_streams(st) != hipSuccess && rc == DL_OK)
        rc = DL_EHIP;
    return rc;
}

dl_status dl_autotune(dl_problem *probs, int count, int reps, void *ws, size_t ws_bytes,
                      dl_stream_t stream)
{
    if (!probs || count < 1 || count > kMaxProblems || reps < 1 || reps > 1000 || !ws ||
        ((uintptr_t)ws % 256) != 0)
        return DL_EINVAL;
    for (int b = 0; b < count; ++b)
        if (!problem_ok(probs[b]))
            return DL_EINVAL;
    const BatchLayout L = batch_layout(probs, count);
    if (ws_bytes < L.total)
        return DL_EWORKSPACE;
    char *base = (char *)ws;
    hipStream_t st = (hipStream_t)stream;
    DL_TRY(launch_zero(base + L.queue, L.gemm - L.queue, st));
    Control *ctl = reinterpret_cast<Control *>(base + L.ctl);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess)
        return DL_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return DL_EHIP;
    }
    dl_status rc = DL_OK;
    // problems that run alone keep their shape (the single-problem launches)
    std::vector<bool> done(count, false);
    for (int b = 0; b < count; ++b)
        done[b] = runs_alone(probs[b].prm);
    for (int b0 = 0; b0 < count && rc == DL_OK; ++b0) {
        if (done[b0])
            continue;
        const dl_params &k0 = probs[b0].prm;
        auto same = [&](int b) {
            const dl_params &q = probs[b].prm;
            return !done[b] && q.p == k0.p && q.n == k0.n && q.s == k0.s;
        };
        int rep = b0;  // the largest problem of this (p, n, s)
        for (int b = b0; b < count; ++b)
            if (same(b) && probs[b].prm.m > probs[rep].prm.m)
                rep = b;
        const dl_problem &pb = probs[rep];
        const dl_params &q = pb.prm;
        const Layout W = layout_for(q);
        char *wb = base + L.prob[rep];
        float *G = reinterpret_cast<float *>(wb + W.G);
        float *A0 = reinterpret_cast<float *>(wb + W.A0);
        const int ldn = padded_n(q.n);
        const GemmF32 g{pb.D, pb.D, G, q.n, q.n, q.p, ldn, nullptr,
                        reinterpret_cast<float *>(wb + W.Gdiag)};
        const GemmF32 cr{pb.Y, pb.D, A0, q.m, q.n, q.p, ldn, nullptr};
        if (launch_gemm_nt_f32(g, &cr, DL_K_CORR, st) != hipSuccess) {
            rc = DL_EHIP;
            break;
        }
        OmpArgs a;
        memset(&a, 0, sizeof(a));
        a.A0 = A0;
        a.G = G;
        a.Gdiag = g.diag;
        a.Y = pb.Y;
        a.D = pb.D;
        a.idx = pb.X_idx;
        a.val = pb.X_val;
        a.E = reinterpret_cast<float *>(wb + W.E);
        a.ctl = ctl + rep;
        a.p = q.p;
        a.n = q.n;
        a.m = std::min(q.m, 65536);
        a.s = q.s;
        a.ldn = ldn;
        a.pivot_fp64 = q.pivot_fp64_threshold;
        a.tol_corr = q.tol_corr;
        a.tol_pivot = q.tol_pivot;
        // candidates are timed with the batched OMP kernel (the one the shape
        // is for) on a batch of this one problem: its argument table and item
        // list go to the start of the workspace's OMP table and list regions
        // (iterate_batched rewrites both)
        OmpArgs *tab = reinterpret_cast<OmpArgs *>(base + L.omp);
        int32_t *lst = reinterpret_cast<int32_t *>(base + L.lists);
        BatchQueue *queue = reinterpret_cast<BatchQueue *>(base + L.queue);
        if (hipMemcpyAsync(tab, &a, sizeof(OmpArgs), hipMemcpyHostToDevice, st) != hipSuccess) {
            rc = DL_EHIP;
            break;
        }
        float best_ms = -1.f, default_ms = -1.f;
        int best_lps = 0, best_npl = 0;
        dl_params dq = q;
        dq.omp_lanes_per_signal = 0;
        dq.omp_atoms_per_lane = 0;
        const OmpShape def = shape_of(dq);
        for (int npl : {4, 8, 16})
            for (int lps : {4, 8, 16, 32, 64}) {
                if (!omp_config_ok(q.n, q.s, lps, npl) || rc != DL_OK)
                    continue;
                const int gpw = omp_signals_per_item(lps);
                const int items = (a.m + gpw - 1) / gpw;
                const int32_t start[2] = {0, items};  // alive until the event wait below
                const BatchList one{lst, 1, queue};
                const int smax = omp_smax(q.s);
                float ms = 0.f;
                if (hipMemcpyAsync(lst, start, sizeof(start), hipMemcpyHostToDevice, st) !=
                        hipSuccess ||
                    launch_batched_omp(tab, one, items, lps, npl, smax, st) != hipSuccess ||
                    hipEventRecord(e0, st) != hipSuccess) {
                    rc = DL_EHIP;
                    hipStreamSynchronize(st);  // the copy reads `start`
                    break;
                }
                for (int r = 0; r < reps && rc == DL_OK; ++r)
                    if (launch_batched_omp(tab, one, items, lps, npl, smax, st) != hipSuccess)
                        rc = DL_EHIP;
                if (rc != DL_OK || hipEventRecord(e1, st) != hipSuccess ||
                    hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                    rc = DL_EHIP;
                    hipStreamSynchronize(st);
                    break;
                }
                if (lps == def.lps && npl == def.npl)
                    default_ms = ms;
                if (best_ms < 0.f || ms < best_ms) {
                    best_ms = ms;
                    best_lps = lps;
                    best_npl = npl;
                }
            }
        // keep the default shape unless another is clearly faster (timing
        // noise, and the shapes behave alike inside the batched launches)
        if (default_ms > 0.f && best_ms > 0.95f * default_ms) {
            best_lps = def.lps;
            best_npl = def.npl;
        }
        for (int b = b0; b < count; ++b)
            if (same(b)) {
                done[b] = true;
                if (best_lps > 0) {
                    probs[b].prm.omp_lanes_per_signal = best_lps;
                    probs[b].prm.omp_atoms_per_lane = best_npl;
                }
            }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return rc;
}

}  // extern "C"
