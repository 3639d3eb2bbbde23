"""Throughput of dictionary learning with Jacobi atom updates on one MI355X.

Headline: a step is one call of dl_iterate on the patch workload, 50 DL
iterations of Batch-OMP coding (p=64, n=256, s=6) of m=16384 zero-mean 8x8
patches, each followed by the Jacobi AK-SVD update of all atoms at once and
the error.  The dictionary is reset to the same D0 before every step, so every
step does the same work.  Inputs are generated once (seeded, synthetic) and
are resident in HBM before the timed region starts.

Prints one JSON line:
  value        signals * iterations per second over the timed steps
  roofline     the dominant kernel's algorithmic rate against the MI355X peak,
               from its average launch time measured with HIP events on the
               launch stream (library-side events around every launch)
  cpu_baseline the FP64 CPU oracle on the same workload, on the host's cores
  rows         the other measured configurations (unless --rows none):
               precision  BF16 products, p=256 n=1024 s=12 m=65536, 30 iters
               learned    plain vs learned support proposal, p=64 n=256 s=6
                          m=262144: 10 plain iterations, training, then the
                          30 steady-state iterations timed on both paths
               batched    64 uneven problems, 20 iterations, one persistent
                          launch per stage, default and autotuned OMP shapes,
                          against the problems run one after another; and
                          200 small problems the same way
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


def kernel_models(p, n, m, s, group_size):
    """Algorithmic work of one launch of each kernel (per-unit figures and
    units in the design doc): (bound, amount, unit), amount in bytes or flops."""
    ngroups = math.ceil(n / min(group_size, n))
    return {
        # G = D D^T: 2 p n^2 flop on the matrix cores
        "gram": ("mfma", 2.0 * p * n * n, "flop"),
        # A0 = Y D^T (2 p n m flop) and the Gram matrix (2 p n^2), one launch
        "corr": ("mfma", 2.0 * p * n * (m + n), "flop"),
        # OMP: per signal it must read its correlation row (4n) and y (4p)
        # and write X (8s) and its residual (4p)
        "omp": ("hbm", float(m * (4 * n + 8 * p + 8 * s)), "byte"),
        # F x^T over chunks: every pair reads its residual row (4p), the ELL
        # position (4) and the coefficient (4); one launch per group
        "upd_pass1": ("hbm", float(m * s * (4 * p + 8)) / ngroups, "byte"),
        "upd_pass2": ("hbm", float(m * s * (4 * p + 12)) / ngroups, "byte"),
        # error: Y (4p) and X (8s) per signal
        "rmse": ("hbm", float(m * (4 * p + 8 * s)), "byte"),
        "csr_count": ("hbm", float(m * s * 8), "byte"),
        "csr_scatter": ("hbm", float(m * s * 16), "byte"),
        # learned coding: y (4p), 2s candidates (8s), reference residual (4),
        # X out (8s) and residual row out (4p) per signal
        "propose": ("hbm", float(m * (8 * p + 16 * s + 4)), "byte"),
    }


def roofline(prof, totals, precision):
    """Dominant kernel of a profiled run and its achieved rate.  prof: kernel
    -> (ms, launches); totals: kernel -> (bound, amount over the whole run,
    unit)."""
    timed = {k: v for k, v in prof.items() if v[1] > 0 and k in totals}
    dom = max(timed, key=lambda k: timed[k][0])
    ms, launches = timed[dom]
    bound, amount, _ = totals[dom]
    sec = ms / 1e3
    if bound == "hbm":
        achieved, peak, unit = amount / sec / 1e9, PEAK_HBM / 1e9, "GB/s"
    else:
        pk = PEAK_BF16_MFMA if precision == "bf16" else PEAK_FP32_MFMA
        achieved, peak, unit = amount / sec / 1e12, pk / 1e12, "TFLOP/s"
    return dom, {"bound": bound, "kernel": dom, "achieved": achieved, "peak": peak,
                 "unit": unit, "frac": achieved / peak, "avg_launch_us": ms * 1e3 / launches,
                 "launches": launches}


def scaled(models, launches_of):
    """Per-launch models times the launches each kernel had."""
    return {k: (b, a * launches_of.get(k, 0), u) for k, (b, a, u) in models.items()}


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


def cpu_baseline(w, iters_sample, m_sample, min_seconds=10.0):
    """FP64 oracle (as it stands) on the first m_sample signals for
    iters_sample iterations, repeated until min_seconds have passed."""
    import oracle
    Y = w.Y[:m_sample]
    runs = 0
    t0 = time.perf_counter()
    while True:
        oracle.iterate(Y, w.D0, w.s, iters_sample, w.n)
        runs += 1
        dt = time.perf_counter() - t0
        if dt >= min_seconds:
            break
    return {
        "value": runs * m_sample * iters_sample / dt,
        "unit": "signals*iters/s",
        "cores": oracle.max_threads(),
        "kind": "oracle",
        "sample": f"{m_sample} of the {w.m} signals, {iters_sample} of the {w.iters} "
                  f"iterations, group size n, run {runs} times ({dt:.1f} s)",
    }


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


# ------------------------------------------------------------------ rows
def row_precision(g, steps):
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
    models = kernel_models(w.p, w.n, w.m, w.s, w.n)
    dom, rl = roofline(prof, scaled(models, {k: v[1] for k, v in prof.items()}), "bf16")
    rh = r.cpu().numpy()
    return {"workload": "patches_p256_n1024_s12_m65536", "precision": "bf16 products, fp32 rest",
            "value": w.m * iters / (ms / 1e3), "unit": "signals*iters/s", "ms_per_step": ms,
            "iters_per_step": iters, "roofline": rl,
            "kernels_ms_per_step": {k: round(v[0], 3) for k, v in prof.items() if v[1]},
            "rmse_first_last": [float(rh[0]), float(rh[-1])]}


def row_learned(g):
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
    recall = float(np.mean([len(set(a) & set(b[b >= 0])) / max(1, int((b >= 0).sum()))
                            for a, b in zip(cn[:20000], last[:20000])]))

    # the steady-state iterations, from the same D10, on both paths
    pws = dl.proposal_workspace(prm)
    wsl = dl.workspace(prm)
    Dl = D10.clone()
    rr = rref.clone()
    rl = torch.empty(steady, dtype=torch.float64, device="cuda:0")
    t_learned = g.time_ms(lambda: dl.iterate_proposed(prm, cand, 0.02, 10, Y, Dl, steady, rr, idx,
                                                      val, rl, wsl, pws))
    fallbacks = dl.read_stats(prm, wsl)["fallbacks"]
    Dp = D10.clone()
    rp = torch.empty(steady, dtype=torch.float64, device="cuda:0")
    t_plain = g.time_ms(lambda: dl.iterate(prm, Y, Dp, steady, idx, val, rp, ws))
    # per-kernel split of the learned iterations
    Dl2, rr2 = D10.clone(), rref.clone()
    prof = g.profile(lambda: dl.iterate_proposed(prm, cand, 0.02, 10, Y, Dl2, steady, rr2, idx,
                                                 val, rl, wsl, pws))
    rl_h, rp_h = rl.cpu().numpy(), rp.cpu().numpy()
    v_l = m * steady / (t_learned / 1e3)
    v_p = m * steady / (t_plain / 1e3)
    gain_ms = (t_plain - t_learned) / steady
    return {
        "workload": "patches_p64_n256_s6_m262144",
        "iterations": f"{warm} plain (recorded) + {steady} timed on each path",
        "plain_value": v_p, "learned_value": v_l, "unit": "signals*iters/s",
        "learned_over_plain": v_l / v_p,
        "rmse_final_plain": float(rp_h[-1]), "rmse_final_learned": float(rl_h[-1]),
        "equal_rmse_within_1pct": bool(abs(rl_h[-1] - rp_h[-1]) <= 0.01 * rp_h[-1]),
        "fallback_fraction": fallbacks / (m * steady),
        "audits": "every 10th learned iteration (3 of 30)",
        "candidate_recall_vs_last_omp": recall,
        "train": {"pairs": warm * m, "epochs": epochs, "steps": nsteps, "batch": q.batch,
                  "ms": t_train, "final_batch_loss": loss},
        "record_10_plain_ms": t_record, "inference_ms": t_infer,
        "break_even_iters": ((t_train + t_infer) / gain_ms) if gain_ms > 0 else None,
        "learned_kernels_ms": {k: round(v[0], 3) for k, v in prof.items() if v[1]},
    }


def row_batched(g, steps):
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
    # algorithmic totals of one batched call: per-problem models summed
    totals = {}
    for q in specs:
        for k, (b, a, u) in kernel_models(q["p"], q["n"], q["m"], q["s"], q["n"]).items():
            if k in ("gram",):
                continue
            tb, ta, tu = totals.get(k, (b, 0.0, u))
            totals[k] = (b, ta + a * iters, u)
    dom, rl = roofline(prof, totals, "fp32")
    r_final = np.array([float(pb.rmse[-1].item()) for pb in probs])

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
        "kernels_ms": {k: round(v[0], 3) for k, v in prof.items() if v[1]},
        "small_problems": {
            "workload": "200 problems p=20 n=50 m=1500 s=3..5, 20 iterations",
            "value_batched": small_total / (t_sb / 1e3),
            "value_sequential_single_calls": small_total / (t_ss / 1e3),
            "batched_over_sequential": t_ss / t_sb, "ms_batched": t_sb, "ms_sequential": t_ss},
    }


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
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--precision", choices=["fp32", "bf16"], default=None,
                    help="products' precision (default: the workload's own)")
    ap.add_argument("--rows", default="precision,learned,batched",
                    help="extra configurations to measure (comma list, or 'none')")
    ap.add_argument("--kernels-only", action="store_true",
                    help="run the warm-up and timed steps only (for profilers)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one plain 256 MiB read + 256 MiB write elementwise kernel, "
                         "the reference for scaling HBM counters")
    ap.add_argument("--row-only", default=None,
                    help="measure only this row (precision, learned or batched) and print it")
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
    if args.calibrate_copy:
        a = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.mul(a, 2.0, out=b)
        torch.cuda.synchronize()
        del a, b
    if args.row_only:
        fn = {"precision": lambda: row_precision(g, 2), "learned": lambda: row_learned(g),
              "batched": lambda: row_batched(g, 2)}[args.row_only]
        print(json.dumps({args.row_only: fn()}))
        return
    w = synth.workload(args.workload)
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
    final_rmse = float(rmse[-1].item())

    # per-kernel times: the same steps again with HIP events around every launch
    prof = g.profile(lambda: [step() for _ in range(args.steps)])
    models = kernel_models(w.p, w.n, w.m, w.s, gs)
    dominant, rl = roofline(prof, scaled(models, {k: v[1] for k, v in prof.items()}), precision)
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
        "kernels_us_per_step": {k: round(v[0] * 1e3 / args.steps, 2)
                                for k, v in prof.items() if v[1]},
        "wall_s": wall,
        "final_rmse": final_rmse,
        "stats": stats,
    }
    rows = {}
    for name in [r for r in args.rows.split(",") if r and r != "none"]:
        t1 = time.perf_counter()
        try:
            if name == "precision":
                rows[name] = row_precision(g, 2)
            elif name == "learned":
                rows[name] = row_learned(g)
            elif name == "batched":
                rows[name] = row_batched(g, 2)
            else:
                rows[name] = {"error": "unknown row"}
        except Exception as e:  # a failed row must not hide the headline
            rows[name] = {"error": f"{type(e).__name__}: {e}"}
        rows[name]["row_wall_s"] = round(time.perf_counter() - t1, 1)
        torch.cuda.empty_cache()
    out["rows"] = rows
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_iters or iters,
                                           min(args.cpu_sample or w.m, w.m))
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out))


if __name__ == "__main__":
    main()
