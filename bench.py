"""Throughput of dictionary learning with Jacobi atom updates on one MI355X.

Headline: a step is one call of dl_iterate on the patch workload, 50 DL
iterations of Batch-OMP coding (p=64, n=256, s=6) of m=16384 zero-mean 8x8
patches, each followed by the Jacobi AK-SVD update of all atoms at once and
the error.  The dictionary is reset to the same D0 before every step, so every
step does the same work.  Inputs are generated once (seeded, synthetic) and
are resident in HBM before the timed region starts.

Prints one JSON line:
  value          signals * iterations per second over the timed steps
  roofline       the dominant kernel's algorithmic work per launch (the
                 method's own flops and bytes, not the design's
                 intermediates) over its average launch time, measured with
                 HIP events on the launch stream, against the MI355X peak of
                 the resource that binds it
  path_roofline  the headline value against the roofline of a whole
                 iteration, 1 / max(bytes / HBM, MFMA flop / peak,
                 VALU flop / peak) per signal-iteration
  oracle         the GPU run against the FP64 CPU oracle on the same inputs
  cpu_baseline   the FP64 CPU oracle on the same workload, on the host's cores
  rows           the other measured configurations (unless --rows none):
                 group16    the headline workload with groups of 16 atoms
                 group_sizes the headline workload over group sizes 1, 2, 4,
                            ..., n (Gauss-Seidel to Jacobi)
                 precision  BF16 products, p=256 n=1024 s=12 m=65536, 30 iters
                 learned    plain vs learned support proposal, p=64 n=256 s=6
                            m=262144: 10 plain iterations, training, then the
                            30 steady-state iterations timed on both paths
                 batched    64 uneven problems, 20 iterations, one persistent
                            launch per stage, default and autotuned OMP shapes,
                            against the problems run one after another; and
                            200 small problems the same way
                 fig7       (not in the default list) the execution-time sweeps
                            of the paper's timing experiment, 200 iterations,
                            groups of n and of 1
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12          # bytes/s
PEAK_FP32_MFMA = 157.3e12  # flop/s, dense
PEAK_BF16_MFMA = 2.5e15
# FP32 vector ALU: 256 CUs x 4 SIMDs x 16 lanes x 2 flop (FMA) x 2 (packed
# FP32) x 2.4 GHz.  The library is built without packed FP32 instructions,
# so half of it is the ceiling it can reach.
PEAK_FP32_VALU = 157.3e12
PEAK_FP32_VALU_UNPACKED = PEAK_FP32_VALU / 2


# ------------------------------------------------------------------ models
def path_work(p, n, m, s):
    """The method's own work per signal-iteration: what it must move or compute
    (Y, X and D), not the design's intermediates (the correlations A0 and the
    residual E are not counted).
      bytes: Y read by the coding (4p) and by the update (4p); X written (8s),
             read (8s) and its values rewritten (4s)
      MFMA:  D^T y (2pn) plus the Gram matrix amortised over the signals
      VALU:  the OMP loop n(s^2 + 3s) + s^3, plus the residual, the
             accumulation of F x^T and the X refresh (2ps each)"""
    return {"bytes": 8.0 * p + 20.0 * s,
            "mfma_flop": 2.0 * p * n + 2.0 * p * n * n / m,
            "valu_flop": float(n * (s * s + 3 * s) + s ** 3 + 6 * p * s)}


def path_roofline(p, n, m, s, value, precision="fp32"):
    w = path_work(p, n, m, s)
    pk_mfma = PEAK_BF16_MFMA if precision == "bf16" else PEAK_FP32_MFMA
    t = {"hbm": w["bytes"] / PEAK_HBM, "mfma": w["mfma_flop"] / pk_mfma,
         "alu": w["valu_flop"] / PEAK_FP32_VALU}
    bound = max(t, key=t.get)
    roof = 1.0 / t[bound]
    t_unpacked = dict(t, alu=w["valu_flop"] / PEAK_FP32_VALU_UNPACKED)
    roof_unpacked = 1.0 / max(t_unpacked.values())
    return {"per_signal_iter": w, "bound": bound, "roofline_value": roof,
            "frac": value / roof, "unit": "signals*iters/s",
            "roofline_value_unpacked_valu": roof_unpacked,
            "frac_unpacked_valu": value / roof_unpacked}


def kernel_work(p, n, m, s, group_size):
    """Algorithmic work of one launch of each kernel: dict of flop on the
    vector ALU ("valu"), flop on the matrix cores ("mfma") and bytes the
    method must move ("bytes") -- the per-signal figures of path_work split
    over the kernels that do them."""
    ngroups = math.ceil(n / min(group_size, n))
    pairs = float(m * s)
    return {
        "gram": {"mfma": 2.0 * p * n * n, "bytes": 4.0 * n * p},
        # A0 = Y D^T and the Gram matrix in one launch: Y read once (4p per
        # signal), the products on the matrix cores
        "corr": {"mfma": 2.0 * p * n * (m + n), "bytes": 4.0 * p * (m + n)},
        # OMP: n(s^2 + 3s) + s^3 per signal; X written (8s)
        "omp": {"valu": float(m * (n * (s * s + 3 * s) + s ** 3)), "bytes": 8.0 * m * s},
        # F x^T: 2p per (signal, slot) pair; X read (8 per pair)
        "upd_pass1": {"valu": 2.0 * p * pairs / ngroups, "bytes": 8.0 * pairs / ngroups},
        # d' and, with groups, the refresh x' = f^T d' (2p per pair; 4 bytes)
        "upd_pass2": {"valu": (2.0 * p * pairs / ngroups) if ngroups > 1 else 0.0,
                      "bytes": (4.0 * pairs / ngroups) if ngroups > 1 else 4.0 * n * p},
        # error with the refresh (all atoms in one group): Y read by the
        # update (4p), the residual (2ps) and the refresh (2ps), X rewritten (4s)
        "rmse": {"valu": 4.0 * p * s * m, "bytes": m * (4.0 * p + 12.0 * s)},
        "csr_count": {"bytes": 4.0 * pairs},
        "csr_scatter": {"bytes": 8.0 * pairs},
        # learned coding: y (4p), 2s candidates (8s), X out (8s)
        "propose": {"bytes": float(m * (4 * p + 16 * s))},
    }


def kernel_roofline(prof, work_totals, precision):
    """Dominant kernel (largest total time) of a profiled run; its achieved
    rate against the peak of each resource it uses, and the binding one (the
    largest fraction).  prof: kernel -> (ms, launches); work_totals: kernel ->
    work summed over the run's launches."""
    timed = {k: v for k, v in prof.items() if v[1] > 0 and k in work_totals}
    dom = max(timed, key=lambda k: timed[k][0])
    ms, launches = timed[dom]
    sec = ms / 1e3
    w = work_totals[dom]
    pk_mfma = PEAK_BF16_MFMA if precision == "bf16" else PEAK_FP32_MFMA
    res = {}
    if w.get("valu"):
        a = w["valu"] / sec / 1e12
        res["alu"] = {"achieved": a, "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s",
                      "frac": a / (PEAK_FP32_VALU / 1e12),
                      "frac_unpacked": a / (PEAK_FP32_VALU_UNPACKED / 1e12)}
    if w.get("mfma"):
        a = w["mfma"] / sec / 1e12
        res["mfma"] = {"achieved": a, "peak": pk_mfma / 1e12, "unit": "TFLOP/s",
                       "frac": a / (pk_mfma / 1e12)}
    if w.get("bytes"):
        a = w["bytes"] / sec / 1e9
        res["hbm"] = {"achieved": a, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                      "frac": a / (PEAK_HBM / 1e9)}
    bound = max(res, key=lambda r: res[r]["frac"])
    out = {"bound": bound, "kernel": dom}
    out.update({k: res[bound][k] for k in ("achieved", "peak", "unit", "frac")})
    if bound == "alu":
        out["frac_unpacked_valu"] = res["alu"]["frac_unpacked"]
    out["avg_launch_us"] = ms * 1e3 / launches
    out["launches"] = launches
    out["other_resources"] = {k: v for k, v in res.items() if k != bound}
    return dom, out


def work_totals(models, launches_of):
    """Per-launch work times the launches each kernel had."""
    return {k: {r: a * launches_of.get(k, 0) for r, a in w.items()} for k, w in models.items()}


def source_digest(paths):
    h = hashlib.sha256()
    for pth in paths:
        with open(pth, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(kernel, workload, digest):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if they
    were taken on the current kernel source; else None."""
    fn = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(fn):
        return None
    with open(fn) as f:
        rec = json.load(f)
    if rec.get("source_digest") != digest:
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, iters_sample, m_sample, min_seconds=10.0):
    """FP64 oracle (as it stands) on the first m_sample signals for
    iters_sample iterations on all the process's threads, repeated until
    min_seconds have passed; then the same on one thread over a smaller
    sample.  Returns the baseline record and the oracle's last run (D, idx,
    val, rmse), which the oracle comparison reuses."""
    import oracle
    Y = w.Y[:m_sample]
    threads = len(os.sched_getaffinity(0))
    oracle.set_threads(threads)
    runs = 0
    last = None
    t0 = time.perf_counter()
    while True:
        last = oracle.iterate(Y, w.D0, w.s, iters_sample, w.n)
        runs += 1
        dt = time.perf_counter() - t0
        if dt >= min_seconds:
            break
    # one thread: 2048 signals, 20 iterations (about a second or two)
    m1, it1 = min(2048, m_sample), min(20, iters_sample)
    oracle.set_threads(1)
    t1 = time.perf_counter()
    oracle.iterate(w.Y[:m1], w.D0, w.s, it1, w.n)
    dt1 = time.perf_counter() - t1
    oracle.set_threads(threads)
    rec = {
        "value": runs * m_sample * iters_sample / dt,
        "unit": "signals*iters/s",
        "cores": oracle.max_threads(),
        "kind": "oracle",
        "cpu_model": cpu_model(),
        "sample": f"{m_sample} of the {w.m} signals, {iters_sample} of the {w.iters} "
                  f"iterations, group size n, run {runs} times ({dt:.1f} s), "
                  f"{oracle.max_threads()} OpenMP threads",
        "value_1thread": m1 * it1 / dt1,
        "sample_1thread": f"first {m1} signals, {it1} iterations, one thread ({dt1:.1f} s)",
    }
    return rec, last


class Gpu:
    """Timing helpers on the current stream (the one every call launches on)."""

    def __init__(self):
        import torch
        from paper_1509_05054_amd import dl
        self.torch, self.dl = torch, dl
        self.stream = torch.cuda.current_stream()

    def time_ms(self, fn):
        t = self.torch
        t.cuda.synchronize()
        e0 = t.cuda.Event(enable_timing=True)
        e1 = t.cuda.Event(enable_timing=True)
        e0.record(self.stream)
        fn()
        e1.record(self.stream)
        t.cuda.synchronize()
        return e0.elapsed_time(e1)

    def profile(self, fn):
        self.dl.profile_enable(True, 1 << 20)
        fn()
        self.torch.cuda.synchronize()
        prof = self.dl.profile_read()
        self.dl.profile_enable(False)
        return prof

    def dev(self, a, dtype=None):
        t = self.torch
        return t.from_numpy(a).to("cuda:0", dtype=dtype or t.float32).contiguous()

    # one-call helpers on fresh workspaces (parity checks, not timed)
    def omp(self, D, Y, s, **kw):
        dl, torch = self.dl, self.torch
        m, p = Y.shape
        prm = dl.Params(p, D.shape[0], m, s, **kw)
        ws = dl.workspace(prm)
        idx = torch.empty((m, s), dtype=torch.int32, device="cuda:0")
        val = torch.empty((m, s), device="cuda:0")
        dl.omp(prm, self.dev(D), self.dev(Y), idx, val, ws)
        return idx.cpu().numpy(), val.cpu().numpy()

    def update_rmse(self, Y, D, idx, val, gs):
        """dl_jau_update then dl_rmse of the result."""
        dl, torch = self.dl, self.torch
        m, p = Y.shape
        prm = dl.Params(p, D.shape[0], m, idx.shape[1], group_size=gs)
        ws = dl.workspace(prm)
        Yg, Dg, vg = self.dev(Y), self.dev(D), self.dev(val.astype("float32"))
        ig = self.dev(idx, torch.int32)
        dl.jau_update(prm, Yg, Dg, ig, vg, ws)
        out = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        dl.rmse(prm, Yg, Dg, ig, vg, out, ws)
        return float(out.item())


def support_agreement(a, b):
    import numpy as np
    sa = [frozenset(int(j) for j in row if j >= 0) for row in a]
    sb = [frozenset(int(j) for j in row if j >= 0) for row in b]
    return float(np.mean([x == y for x, y in zip(sa, sb)]))


def teacher_forced(g, D, Y, s, gs, bf16=False):
    """One iteration from the same dictionary D on both sides: the GPU's
    coding against the oracle's (support agreement), and the GPU's update and
    error of the oracle's representation against the oracle's (relative RMSE
    difference); with bf16, the GPU codes with BF16 products and the oracle
    both exactly and with D and Y rounded to BF16."""
    import numpy as np
    import oracle
    D32 = np.ascontiguousarray(D, dtype=np.float32)
    kw = {"precision": g.dl.PREC_BF16} if bf16 else {}
    ig, _ = g.omp(D32, Y, s, **kw)
    ir, vr, _ = oracle.omp(D32, Y, s)
    out = {"signals": int(Y.shape[0]), "support_agreement": support_agreement(ig, ir)}
    if bf16:
        from oracle.bf16 import round_bf16
        ib, _, _ = oracle.omp(round_bf16(D32), round_bf16(np.ascontiguousarray(Y)), s)
        out["support_agreement_vs_bf16_emulation"] = support_agreement(ig, ib)
    Dn, vn, _ = oracle.jau_update(Y, D32, ir, vr.astype(np.float32), gs)
    rr = oracle.rmse(Y, Dn, ir, vn)
    rg = g.update_rmse(Y, D32, ir, vr.astype(np.float32), gs)
    out.update({"rmse_oracle": rr, "rmse_gpu": rg, "rmse_rel": abs(rg - rr) / rr})
    return out


# ------------------------------------------------------------------ rows
def row_group_size(g, w, gs, steps=2):
    """The headline workload with groups of gs atoms (eq. 2)."""
    dl, torch = g.dl, g.torch
    prm = dl.Params(w.p, w.n, w.m, w.s, group_size=gs)
    Y, D0 = g.dev(w.Y), g.dev(w.D0)
    D = D0.clone()
    idx = torch.empty((w.m, w.s), dtype=torch.int32, device="cuda:0")
    val = torch.empty((w.m, w.s), device="cuda:0")
    r = torch.empty(w.iters, dtype=torch.float64, device="cuda:0")
    ws = dl.workspace(prm)

    def step():
        D.copy_(D0)
        dl.iterate(prm, Y, D, w.iters, idx, val, r, ws)

    step()
    ms = g.time_ms(lambda: [step() for _ in range(steps)]) / steps
    return {"group_size": gs, "value": w.m * w.iters / (ms / 1e3), "ms_per_step": ms,
            "final_rmse": float(r[-1].item()), "D_final": D.cpu().numpy()}


def row_group16(g, w, with_oracle):
    rec = row_group_size(g, w, 16, steps=3)
    Df = rec.pop("D_final")
    prof = g.profile(lambda: row_group_size(g, w, 16, steps=1))
    rec["kernels_ms_per_call"] = {k: round(v[0] / 2, 3) for k, v in prof.items() if v[1]}
    rec["workload"] = w.name
    rec["unit"] = "signals*iters/s"
    if with_oracle:
        rec["oracle_teacher_forced_final_D"] = teacher_forced(g, Df, w.Y, w.s, 16)
    return rec


def row_group_sizes(g, w):
    """Group sizes 1, 2, 4, ..., n on the headline workload: from the
    sequential (Gauss-Seidel) sweep to the fully parallel one."""
    out = []
    gs = 1
    while True:
        r = row_group_size(g, w, gs, steps=1)
        r.pop("D_final")
        out.append(r)
        if gs >= w.n:
            break
        gs = min(2 * gs, w.n)
    by = {r["group_size"]: r["value"] for r in out}
    return {"workload": w.name, "iters": w.iters, "unit": "signals*iters/s", "points": out,
            "jacobi_over_gauss_seidel": by[w.n] / by[1]}


def row_fig7(g):
    """The three execution-time sweeps of the paper's timing experiment
    (200 iterations of 8x8 patches): s = 4..12 (n = 128, m = 8192),
    n = 128..512 (m = 12288, s = 6), m = 4096..16384 (n = 256, s = 10), each
    with all atoms in one group and with groups of one atom."""
    from paper_1509_05054_amd import synth
    dl, torch = g.dl, g.torch
    iters = 200
    imgs = synth.synthetic_images(8, 512, 707)
    pool = synth.image_patches(imgs, 8, 16384, 708)
    sweeps = {"s": [(128, 8192, s) for s in range(4, 13, 2)],
              "n": [(n, 12288, 6) for n in range(128, 513, 64)],
              "m": [(256, m, 10) for m in range(4096, 16385, 1024)]}
    out = {}
    for axis, pts in sweeps.items():
        rows = []
        for n, m, s in pts:
            Y = pool[:m]
            D0 = synth.initial_dictionary(Y, n, 709)
            rec = {"n": n, "m": m, "s": s}
            for gs in (n, 1):
                prm = dl.Params(64, n, m, s, group_size=gs)
                ws = dl.workspace(prm)
                Yd, D = g.dev(Y), g.dev(D0)
                idx = torch.empty((m, s), dtype=torch.int32, device="cuda:0")
                val = torch.empty((m, s), device="cuda:0")
                r = torch.empty(iters, dtype=torch.float64, device="cuda:0")
                dl.iterate(prm, Yd, D.clone(), 2, idx, val, r, ws)  # warm-up
                ms = g.time_ms(lambda: dl.iterate(prm, Yd, D, iters, idx, val, r, ws))
                rec[f"ms_group_{'n' if gs == n else '1'}"] = ms
                rec[f"rmse_group_{'n' if gs == n else '1'}"] = float(r[-1].item())
            rec["speedup_jacobi_over_gauss_seidel"] = rec["ms_group_1"] / rec["ms_group_n"]
            rows.append(rec)
            print(json.dumps({"fig7": axis, **rec}), file=sys.stderr, flush=True)
        out[axis] = rows
    return {"iters": iters, "sweeps": out}


def row_precision(g, steps, with_oracle):
    dl, torch = g.dl, g.torch
    from paper_1509_05054_amd import synth
    w = synth.workload("patches_p256_n1024_s12_m65536")
    iters = w.iters
    prm = dl.Params(w.p, w.n, w.m, w.s, precision=dl.PREC_BF16)
    Y, D0 = g.dev(w.Y), g.dev(w.D0)
    D = D0.clone()
    idx = torch.empty((w.m, w.s), dtype=torch.int32, device="cuda:0")
    val = torch.empty((w.m, w.s), device="cuda:0")
    r = torch.empty(iters, dtype=torch.float64, device="cuda:0")
    ws = dl.workspace(prm)

    def step():
        D.copy_(D0)
        dl.iterate(prm, Y, D, iters, idx, val, r, ws)

    step()
    ms = g.time_ms(lambda: [step() for _ in range(steps)]) / steps
    prof = g.profile(step)
    models = kernel_work(w.p, w.n, w.m, w.s, w.n)
    dom, rl = kernel_roofline(prof, work_totals(models, {k: v[1] for k, v in prof.items()}),
                              "bf16")
    rh = r.cpu().numpy()
    value = w.m * iters / (ms / 1e3)
    rec = {"workload": "patches_p256_n1024_s12_m65536",
           "precision": "bf16 products (Gram, correlations), fp32 coding loop and update",
           "value": value, "unit": "signals*iters/s", "ms_per_step": ms,
           "iters_per_step": iters, "roofline": rl,
           "path_roofline": path_roofline(w.p, w.n, w.m, w.s, value, "bf16"),
           "kernels_ms_per_step": {k: round(v[0], 3) for k, v in prof.items() if v[1]},
           "rmse_first_last": [float(rh[0]), float(rh[-1])]}
    if with_oracle:
        import numpy as np
        import oracle
        sample = 4096
        Ys = w.Y[:sample]
        rec["oracle_teacher_forced"] = {
            "sample": f"first {sample} of {w.m} signals",
            "at_D0": teacher_forced(g, oracle.normalize(w.D0), Ys, w.s, w.n, bf16=True),
            "at_final_D": teacher_forced(g, D.cpu().numpy().astype(np.float64), Ys, w.s, w.n,
                                         bf16=True)}
    return rec


def row_learned(g, with_oracle):
    dl, torch = g.dl, g.torch
    import numpy as np
    from paper_1509_05054_amd import synth
    w = synth.workload("patches_p64_n256_s6_m262144")
    p, n, s, m = w.p, w.n, w.s, w.m
    warm, steady, hidden = 10, 30, 512
    prm = dl.Params(p, n, m, s)
    Y = g.dev(w.Y)
    D = g.dev(w.D0)
    idx = torch.empty((m, s), dtype=torch.int32, device="cuda:0")
    val = torch.empty((m, s), device="cuda:0")
    ws = dl.workspace(prm)
    r1 = torch.empty(warm, dtype=torch.float64, device="cuda:0")
    hist = torch.empty((warm * m, s), dtype=torch.int32, device="cuda:0")
    rref = torch.empty(m, device="cuda:0")
    t_record = g.time_ms(lambda: dl.iterate_record(prm, Y, D, warm, idx, val, r1, hist, rref, ws))
    D10 = D.clone()

    # training: equal-weight pairs of all recorded iterations, 5 epochs
    q = dl.MlpParams(p, hidden, n, batch=4096, lr=3e-3, pos_weight=(n - s) / s)
    vec = synth.mlp_params((p, hidden, hidden, n), 4041)
    mws = dl.mlp_workspace(q, g.dev(vec))
    rng = np.random.default_rng(4041)
    epochs = 5
    order = np.concatenate([rng.permutation(warm * m) for _ in range(epochs)]).astype(np.int32)
    order_d = g.dev(order, torch.int32)
    nsteps = len(order) // q.batch

    def train():
        for t in range(nsteps):
            dl.mlp_train_step(q, mws, Y, hist, order_d[t * q.batch:(t + 1) * q.batch], step=t + 1)

    t_train = g.time_ms(train)
    loss = dl.mlp_read(q, mws, want_loss=True)
    logits = torch.empty((m, n), device="cuda:0")
    cand = torch.empty((m, 2 * s), dtype=torch.int32, device="cuda:0")

    def infer():
        dl.mlp_forward(q, mws, Y, logits)
        dl.topk(logits, 2 * s, cand)

    t_infer = g.time_ms(infer)
    last = hist[(warm - 1) * m:].cpu().numpy()
    cn = cand.cpu().numpy()

    def recall_of(c):
        return float(np.mean([len(set(a) & set(b[b >= 0])) / max(1, int((b >= 0).sum()))
                              for a, b in zip(c[:20000], last[:20000])]))

    recall = recall_of(cn)
    # the method without the network: the 2s largest |D^T y| at D10
    corr = torch.empty((m, n), device="cuda:0")
    dl.corr(prm, D10, Y, corr)
    cand_corr = torch.empty((m, 2 * s), dtype=torch.int32, device="cuda:0")
    dl.topk(corr.abs(), 2 * s, cand_corr)
    recall_corr = recall_of(cand_corr.cpu().numpy())
    # planted candidates: the last OMP support plus random other atoms (what a
    # network of perfect recall would propose), to separate kernel cost from recall
    keys = np.random.default_rng(4042).random((m, n))
    rows_ix = np.repeat(np.arange(m), s)
    flat = last.reshape(-1)
    on = flat >= 0
    keys[rows_ix[on], flat[on]] = 2.0  # the support atoms rank first
    planted = np.argsort(-keys, axis=1, kind="stable")[:, :2 * s].astype(np.int32)
    del keys
    cand_planted = g.dev(planted, torch.int32)

    # the steady-state iterations, from the same D10, on each path
    pws = dl.proposal_workspace(prm)
    wsl = dl.workspace(prm)

    def run_learned(cands):
        Dl, rr = D10.clone(), rref.clone()
        rl = torch.empty(steady, dtype=torch.float64, device="cuda:0")
        t = g.time_ms(lambda: dl.iterate_proposed(prm, cands, 0.02, 10, Y, Dl, steady, rr, idx,
                                                  val, rl, wsl, pws))
        fb = dl.read_stats(prm, wsl)["fallbacks"]
        return t, rl.cpu().numpy(), fb / (m * steady)

    t_learned, rl_h, fb_l = run_learned(cand)
    t_corr, rc_h, fb_c = run_learned(cand_corr)
    t_planted, rpl_h, fb_p = run_learned(cand_planted)
    Dp = D10.clone()
    rp = torch.empty(steady, dtype=torch.float64, device="cuda:0")
    t_plain = g.time_ms(lambda: dl.iterate(prm, Y, Dp, steady, idx, val, rp, ws))
    # per-kernel split of the learned iterations
    Dl2, rr2 = D10.clone(), rref.clone()
    rl2 = torch.empty(steady, dtype=torch.float64, device="cuda:0")
    prof = g.profile(lambda: dl.iterate_proposed(prm, cand, 0.02, 10, Y, Dl2, steady, rr2, idx,
                                                 val, rl2, wsl, pws))
    rp_h = rp.cpu().numpy()
    v_l = m * steady / (t_learned / 1e3)
    v_p = m * steady / (t_plain / 1e3)
    gain_ms = (t_plain - t_learned) / steady

    def eq(rx):
        return bool(abs(rx[-1] - rp_h[-1]) <= 0.01 * rp_h[-1])

    rec = {
        "workload": "patches_p64_n256_s6_m262144",
        "iterations": f"{warm} plain (recorded) + {steady} timed on each path",
        "plain_value": v_p, "learned_value": v_l, "unit": "signals*iters/s",
        "learned_over_plain": v_l / v_p,
        "rmse_final_plain": float(rp_h[-1]), "rmse_final_learned": float(rl_h[-1]),
        "equal_rmse_within_1pct": eq(rl_h),
        "fallback_fraction": fb_l,
        "audits": "every 10th learned iteration (3 of 30)",
        "candidate_recall_vs_last_omp": recall,
        "without_network_top2s_correlations": {
            "candidate_recall_vs_last_omp": recall_corr, "fallback_fraction": fb_c,
            "over_plain": t_plain / t_corr, "rmse_final": float(rc_h[-1]),
            "equal_rmse_within_1pct": eq(rc_h)},
        "planted_candidates_perfect_recall": {
            "fallback_fraction": fb_p, "over_plain": t_plain / t_planted,
            "rmse_final": float(rpl_h[-1]), "equal_rmse_within_1pct": eq(rpl_h)},
        "train": {"pairs": warm * m, "epochs": epochs, "steps": nsteps, "batch": q.batch,
                  "ms": t_train, "final_batch_loss": loss},
        "record_10_plain_ms": t_record, "inference_ms": t_infer,
        "break_even_iters": ((t_train + t_infer) / gain_ms) if gain_ms > 0 else None,
        "learned_kernels_ms": {k: round(v[0], 3) for k, v in prof.items() if v[1]},
        "path_roofline_plain": path_roofline(p, n, m, s, v_p),
    }
    if with_oracle:
        sample = 16384
        rec["oracle_teacher_forced_plain_final_D"] = dict(
            teacher_forced(g, Dp.cpu().numpy().astype(np.float64), w.Y[:sample], s, n),
            sample=f"first {sample} of {m} signals")
    return rec


def row_batched(g, steps, with_oracle):
    dl, torch = g.dl, g.torch
    import numpy as np
    from paper_1509_05054_amd import synth
    specs = synth.batched_problems(64, seed=505)
    iters = 20
    probs = []
    for q in specs:
        prm = dl.Params(q["p"], q["n"], q["m"], q["s"])
        probs.append(dl.Problem(prm, g.dev(q["Y"]), g.dev(q["D0"]),
                                torch.empty((q["m"], q["s"]), dtype=torch.int32, device="cuda:0"),
                                torch.empty((q["m"], q["s"]), device="cuda:0"),
                                torch.empty(iters, dtype=torch.float64, device="cuda:0")))
    D0s = [pb.D.clone() for pb in probs]
    ws = dl.batch_workspace(probs)
    total = sum(q["m"] for q in specs) * iters

    def reset():
        for pb, d0 in zip(probs, D0s):
            pb.D.copy_(d0)

    def batched():
        reset()
        dl.iterate_batched(probs, iters, ws)

    batched()
    t_default = g.time_ms(lambda: [batched() for _ in range(steps)]) / steps
    # one problem after another through dl_iterate (default shapes)
    single_ws = [dl.workspace(pb.prm) for pb in probs]

    def sequential():
        reset()
        for pb, w1 in zip(probs, single_ws):
            dl.iterate(pb.prm, pb.Y, pb.D, iters, pb.X_idx, pb.X_val, pb.rmse, w1)

    sequential()
    t_seq = g.time_ms(lambda: [sequential() for _ in range(steps)]) / steps
    reset()
    t0 = time.perf_counter()
    shapes = dl.autotune(probs, ws, reps=3)
    t_tune = time.perf_counter() - t0
    batched()
    t_tuned = g.time_ms(lambda: [batched() for _ in range(steps)]) / steps
    prof = g.profile(batched)
    prof_seq = g.profile(sequential)
    # algorithmic totals of one batched call: per-problem work summed
    totals = {}
    for q in specs:
        for k, wk in kernel_work(q["p"], q["n"], q["m"], q["s"], q["n"]).items():
            acc = totals.setdefault(k, {})
            for r, a in wk.items():
                acc[r] = acc.get(r, 0.0) + a * iters
    dom, rl = kernel_roofline(prof, totals, "fp32")
    r_final = np.array([float(pb.rmse[-1].item()) for pb in probs])
    rec_oracle = None
    if with_oracle:
        # teacher-forced iteration at each of 8 problems' final dictionaries
        # (first 2048 signals of each)
        chk = []
        for b in range(0, 64, 8):
            q = specs[b]
            t = teacher_forced(g, probs[b].D.cpu().numpy().astype(np.float64), q["Y"][:2048],
                               q["s"], q["n"])
            chk.append(dict(t, problem=b, p=q["p"], n=q["n"], s=q["s"]))
        rec_oracle = {"problems": chk,
                      "min_support_agreement": min(c["support_agreement"] for c in chk),
                      "max_rmse_rel": max(c["rmse_rel"] for c in chk)}

    # many small problems (the shape of the dictionary-recovery experiment,
    # p=20 n=50 m=1500 s=3..5), where one launch per stage matters most
    small = []
    for b in range(200):
        sb = 3 + b % 3
        Ys, _, _, _ = synth.recovery_problem(20, 50, sb, 1500, 0.0, seed=9000 + b, snr_db=20)
        D0s_ = synth.initial_dictionary(Ys, 50, seed=9500 + b)
        small.append(dl.Problem(dl.Params(20, 50, 1500, sb), g.dev(Ys), g.dev(D0s_),
                                torch.empty((1500, sb), dtype=torch.int32, device="cuda:0"),
                                torch.empty((1500, sb), device="cuda:0"),
                                torch.empty(iters, dtype=torch.float64, device="cuda:0")))
    small_D0 = [pb.D.clone() for pb in small]
    small_ws = dl.batch_workspace(small)
    small_single = [dl.workspace(pb.prm) for pb in small]

    def small_reset():
        for pb, d0 in zip(small, small_D0):
            pb.D.copy_(d0)

    def small_batched():
        small_reset()
        dl.iterate_batched(small, iters, small_ws)

    def small_sequential():
        small_reset()
        for pb, w1 in zip(small, small_single):
            dl.iterate(pb.prm, pb.Y, pb.D, iters, pb.X_idx, pb.X_val, pb.rmse, w1)

    small_batched()
    small_sequential()
    t_sb = g.time_ms(lambda: [small_batched() for _ in range(steps)]) / steps
    t_ss = g.time_ms(lambda: [small_sequential() for _ in range(steps)]) / steps
    small_total = 200 * 1500 * iters
    return {
        "workload": "64 uneven problems: p in {16,36,64,144,256}, n in {2p,4p}, s in 3..16, "
                    "m log-uniform 2k..64k (seed 505)",
        "signals_total": int(sum(q["m"] for q in specs)), "iters": iters,
        "value_default_shapes": total / (t_default / 1e3),
        "value_autotuned": total / (t_tuned / 1e3),
        "value_sequential_single_calls": total / (t_seq / 1e3),
        "unit": "signals*iters/s", "ms_batched_tuned": t_tuned, "ms_batched_default": t_default,
        "ms_sequential": t_seq, "autotune_s": t_tune,
        "omp_shapes_tuned": sorted(set((q["p"], q["n"], q["s"], lps, npl)
                                       for q, (lps, npl) in zip(specs, shapes))),
        "roofline": rl, "rmse_final_mean": float(r_final.mean()),
        "oracle_teacher_forced_final_D": rec_oracle,
        "kernels_ms": {k: round(v[0], 3) for k, v in prof.items() if v[1]},
        "kernels_ms_sequential": {k: round(v[0], 3) for k, v in prof_seq.items() if v[1]},
        "small_problems": {
            "workload": "200 problems p=20 n=50 m=1500 s=3..5, 20 iterations",
            "value_batched": small_total / (t_sb / 1e3),
            "value_sequential_single_calls": small_total / (t_ss / 1e3),
            "batched_over_sequential": t_ss / t_sb, "ms_batched": t_sb, "ms_sequential": t_ss},
    }


def headline_oracle(g, w, gpu_rmse, last):
    """The headline run against the oracle's run of the same workload (its
    CPU-baseline run): the free-running error trajectories, and one
    teacher-forced iteration at the oracle's final dictionary."""
    import numpy as np
    Dr, ir, vr, rr = last
    rel = np.abs(gpu_rmse - rr) / rr
    return {"free_running": {"rmse_gpu_first_last": [float(gpu_rmse[0]), float(gpu_rmse[-1])],
                             "rmse_oracle_first_last": [float(rr[0]), float(rr[-1])],
                             "rel_first": float(rel[0]), "rel_final": float(rel[-1]),
                             "rel_max": float(rel.max())},
            "teacher_forced_at_oracle_final_D": teacher_forced(g, Dr, w.Y, w.s, w.n)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="patches_p64_n256_s6_m16384")
    ap.add_argument("--group-size", type=int, default=0, help="0 = all atoms (n)")
    ap.add_argument("--iters", type=int, default=0, help="0 = the workload's iteration count")
    ap.add_argument("--cpu-sample", type=int, default=0, help="signals in the CPU sample (0 = all)")
    ap.add_argument("--cpu-iters", type=int, default=0, help="0 = all the workload's iterations")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the CPU baseline and every comparison with the oracle")
    ap.add_argument("--precision", choices=["fp32", "bf16"], default=None,
                    help="products' precision (default: the workload's own)")
    ap.add_argument("--rows", default="group16,group_sizes,precision,learned,batched",
                    help="extra configurations to measure (comma list, or 'none')")
    ap.add_argument("--kernels-only", action="store_true",
                    help="run the warm-up and timed steps only (for profilers)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one plain 256 MiB read + 256 MiB write elementwise kernel, "
                         "the reference for scaling HBM counters")
    ap.add_argument("--row-only", default=None,
                    help="measure only this row and print it")
    ap.add_argument("--omp-only", action="store_true",
                    help="run the coding stage (dl_omp) twice on the workload and stop (for "
                         "counter profiles of the OMP kernel)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the design of the signal-sharded version is in DESIGN.md).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1509_05054_amd import dl, synth

    g = Gpu()
    with_oracle = not args.no_cpu
    if args.calibrate_copy:
        a = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.mul(a, 2.0, out=b)
        torch.cuda.synchronize()
        del a, b
    w = synth.workload(args.workload)
    if args.row_only:
        fn = {"precision": lambda: row_precision(g, 2, with_oracle),
              "learned": lambda: row_learned(g, with_oracle),
              "batched": lambda: row_batched(g, 2, with_oracle),
              "group16": lambda: row_group16(g, w, with_oracle),
              "group_sizes": lambda: row_group_sizes(g, w),
              "fig7": lambda: row_fig7(g)}[args.row_only]
        print(json.dumps({args.row_only: fn()}))
        return
    if args.omp_only:
        prec = args.precision or ("bf16" if args.workload.startswith("patches_p256") else "fp32")
        prm = dl.Params(w.p, w.n, w.m, w.s,
                        precision=dl.PREC_BF16 if prec == "bf16" else dl.PREC_FP32)
        ws = dl.workspace(prm)
        Yd, Dd = g.dev(w.Y), g.dev(w.D0)
        idx = torch.empty((w.m, w.s), dtype=torch.int32, device="cuda:0")
        val = torch.empty((w.m, w.s), device="cuda:0")
        for _ in range(2):
            dl.omp(prm, Dd, Yd, idx, val, ws)
        torch.cuda.synchronize()
        print(json.dumps({"workload": args.workload, "omp_runs": 2}))
        return
    iters = args.iters or w.iters
    gs = args.group_size or w.n
    precision = args.precision or ("bf16" if args.workload.startswith("patches_p256") else "fp32")
    prm = dl.Params(w.p, w.n, w.m, w.s, group_size=gs,
                    precision=dl.PREC_BF16 if precision == "bf16" else dl.PREC_FP32)
    Y = g.dev(w.Y)
    D0 = g.dev(w.D0)
    D = D0.clone()
    idx = torch.empty((w.m, w.s), dtype=torch.int32, device="cuda:0")
    val = torch.empty((w.m, w.s), dtype=torch.float32, device="cuda:0")
    rmse = torch.empty(iters, dtype=torch.float64, device="cuda:0")
    ws = dl.workspace(prm)

    def step():
        D.copy_(D0)
        dl.iterate(prm, Y, D, iters, idx, val, rmse, ws)

    for _ in range(args.warmup):
        step()
    t0 = time.perf_counter()
    gpu_ms = g.time_ms(lambda: [step() for _ in range(args.steps)])
    wall = time.perf_counter() - t0
    if args.kernels_only:
        print(json.dumps({"workload": args.workload, "ms_per_step": gpu_ms / args.steps}))
        return
    ms_per_step = gpu_ms / args.steps
    value = w.m * iters * args.steps / (gpu_ms / 1e3)
    stats = dl.read_stats(prm, ws)
    rmse_h = rmse.cpu().numpy()

    # per-kernel times: the same steps again with HIP events around every launch
    prof = g.profile(lambda: [step() for _ in range(args.steps)])
    models = kernel_work(w.p, w.n, w.m, w.s, gs)
    dominant, rl = kernel_roofline(prof, work_totals(models, {k: v[1] for k, v in prof.items()}),
                                   precision)
    csrc = os.path.join(ROOT, "paper_1509_05054_amd", "csrc")
    digest = source_digest(sorted(os.path.join(csrc, f) for f in os.listdir(csrc)))
    rl["traffic"] = read_traffic(dominant, args.workload, digest)

    out = {
        "metric": f"signals*iters/s for OMP+JAU (p{w.p} n{w.n} s{w.s})",
        "value": value,
        "unit": "signals*iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if precision == "fp32" else "bf16+f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "p": w.p, "n": w.n, "s": w.s, "m": w.m,
                   "iters_per_step": iters, "group_size": gs, "precision": precision,
                   "rule": "aksvd"},
        "roofline": rl,
        "path_roofline": path_roofline(w.p, w.n, w.m, w.s, value, precision),
        "kernels_us_per_step": {k: round(v[0] * 1e3 / args.steps, 2)
                                for k, v in prof.items() if v[1]},
        "wall_s": wall,
        "final_rmse": float(rmse_h[-1]),
        "stats": stats,
    }
    cpu_rec, last = (None, None)
    if with_oracle:
        full = (args.cpu_sample in (0, w.m)) and (args.cpu_iters in (0, iters)) and gs == w.n
        cpu_rec, last = cpu_baseline(w, args.cpu_iters or iters, min(args.cpu_sample or w.m, w.m))
        if full and precision == "fp32":
            out["oracle"] = headline_oracle(g, w, rmse_h, last)
    rows = {}
    for name in [r for r in args.rows.split(",") if r and r != "none"]:
        t1 = time.perf_counter()
        try:
            if name == "precision":
                rows[name] = row_precision(g, 2, with_oracle)
            elif name == "learned":
                rows[name] = row_learned(g, with_oracle)
            elif name == "batched":
                rows[name] = row_batched(g, 2, with_oracle)
            elif name == "group16":
                rows[name] = row_group16(g, w, with_oracle)
            elif name == "group_sizes":
                rows[name] = row_group_sizes(g, w)
            elif name == "fig7":
                rows[name] = row_fig7(g)
            else:
                rows[name] = {"error": "unknown row"}
        except Exception as e:  # a failed row must not hide the headline
            rows[name] = {"error": f"{type(e).__name__}: {e}"}
        rows[name]["row_wall_s"] = round(time.perf_counter() - t1, 1)
        print(f"[bench] row {name} done in {rows[name]['row_wall_s']} s", file=sys.stderr,
              flush=True)
        torch.cuda.empty_cache()
    out["rows"] = rows
    out["cpu_baseline"] = cpu_rec
    print(json.dumps(out))


if __name__ == "__main__":
    main()
