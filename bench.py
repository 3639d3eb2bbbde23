"""Throughput of dictionary learning with Jacobi atom updates on one MI355X.

A step is one call of dl_iterate on the patch workload: 50 DL iterations of
Batch-OMP coding (p=64, n=256, s=6) of m=16384 zero-mean 8x8 patches followed
by the Jacobi AK-SVD atom update of all atoms at once, with the error after
every iteration.  The dictionary is reset to the same D0 before every step, so
every step does the same work.  Inputs are generated once (seeded, synthetic)
and are resident in HBM before the timed region starts.

Prints one JSON line:
  value        signals * iterations per second over the timed steps
  roofline     the dominant kernel's algorithmic rate against the MI355X peak,
               from its average launch time measured with HIP events
  cpu_baseline the FP64 CPU oracle on a bounded sample of the same workload
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
PEAK_FP32_VALU = 157.3e12  # flop/s, packed vector FP32 of the chip
PEAK_BF16_MFMA = 2.5e15


def kernel_models(p, n, m, s, group_size):
    """Algorithmic work of one launch of each kernel:
    (bound, amount, unit) with amount in bytes or flops."""
    ngroups = math.ceil(n / min(group_size, n))
    return {
        # G = D D^T: 2 p n^2 flop on FP32 MFMA
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
    }


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


def cpu_baseline(w, iters_sample, m_sample):
    """FP64 oracle (as it stands) on the first m_sample signals for iters_sample iterations."""
    import oracle
    Y = w.Y[:m_sample]
    t0 = time.perf_counter()
    oracle.iterate(Y, w.D0, w.s, iters_sample, w.n)
    dt = time.perf_counter() - t0
    return {
        "value": m_sample * iters_sample / dt,
        "unit": "signals*iters/s",
        "cores": oracle.max_threads(),
        "kind": "oracle",
        "sample": f"{m_sample} of the {w.m} signals, {iters_sample} of the {w.iters} iterations "
                  f"({dt:.1f} s)",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="patches_p64_n256_s6_m16384")
    ap.add_argument("--group-size", type=int, default=0, help="0 = all atoms (n)")
    ap.add_argument("--iters", type=int, default=0, help="0 = the workload's iteration count")
    ap.add_argument("--cpu-sample", type=int, default=4096, help="signals in the CPU sample")
    ap.add_argument("--cpu-iters", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--precision", choices=["fp32", "bf16"], default=None,
                    help="products' precision (default: the workload's own)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the design of the signal-sharded version is in DESIGN.md).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1509_05054_amd import dl, synth

    w = synth.workload(args.workload)
    iters = args.iters or w.iters
    gs = args.group_size or w.n
    precision = args.precision or ("bf16" if args.workload.startswith("patches_p256") else "fp32")
    prm = dl.Params(w.p, w.n, w.m, w.s, group_size=gs,
                    precision=dl.PREC_BF16 if precision == "bf16" else dl.PREC_FP32)
    dev = torch.device("cuda:0")
    Y = torch.from_numpy(w.Y).to(dev)
    D0 = torch.from_numpy(w.D0).to(dev)
    D = D0.clone()
    idx = torch.empty((w.m, w.s), dtype=torch.int32, device=dev)
    val = torch.empty((w.m, w.s), dtype=torch.float32, device=dev)
    rmse = torch.empty(iters, dtype=torch.float64, device=dev)
    ws = dl.workspace(prm, dev)
    stream = torch.cuda.current_stream()

    def step():
        D.copy_(D0)
        dl.iterate(prm, Y, D, iters, idx, val, rmse, ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = gpu_ms / args.steps
    value = w.m * iters * args.steps / (gpu_ms / 1e3)
    stats = dl.read_stats(prm, ws)
    final_rmse = float(rmse[-1].item())

    # per-kernel times: the same steps again with HIP events around every launch
    dl.profile_enable(True, 1 << 20)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    prof = dl.profile_read()
    dl.profile_enable(False)
    models = kernel_models(w.p, w.n, w.m, w.s, gs)
    timed = {k: v for k, v in prof.items() if v[1] > 0}
    dominant = max((k for k in timed if k in models), key=lambda k: timed[k][0])
    tot_ms, launches = timed[dominant]
    avg_s = tot_ms / launches / 1e3
    bound, amount, unit = models[dominant]
    if bound == "hbm":
        achieved, peak, runit = amount / avg_s / 1e9, PEAK_HBM / 1e9, "GB/s"
    elif bound == "mfma":
        mfma_peak = PEAK_BF16_MFMA if precision == "bf16" else PEAK_FP32_MFMA
        achieved, peak, runit = amount / avg_s / 1e12, mfma_peak / 1e12, "TFLOP/s"
    else:
        achieved, peak, runit = amount / avg_s / 1e12, PEAK_FP32_VALU / 1e12, "TFLOP/s"
    csrc = os.path.join(ROOT, "paper_1509_05054_amd", "csrc")
    digest = source_digest(sorted(os.path.join(csrc, f) for f in os.listdir(csrc)))
    traffic = read_traffic(dominant, args.workload, digest)

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
        "roofline": {"bound": bound, "kernel": dominant, "achieved": achieved, "peak": peak,
                     "unit": runit, "frac": achieved / peak, "traffic": traffic,
                     "avg_launch_us": avg_s * 1e6, "launches": launches},
        "kernels_us_per_step": {k: round(v[0] * 1e3 / args.steps, 2) for k, v in timed.items()},
        "wall_s": wall,
        "final_rmse": final_rmse,
        "stats": stats,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_iters, min(args.cpu_sample, w.m))
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out))


if __name__ == "__main__":
    main()
