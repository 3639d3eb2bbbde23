"""The dictionary-recovery experiment of Sec. 4.1 (Table 1) on the GPU: all
600 runs (3 sparsities x 4 noise levels x 50 runs, p = 20, n = 50, m = 1500,
9 s^2 iterations, all atoms in one Jacobi group) go through the batched
launch, one call per sparsity.  The printed percentages pin whole trajectories
of the GPU iteration statistically: the average over 50 runs must fall within
a band of the paper's figure.

At full parallelism PAK-SVD's atoms equal P-SGK's (Sec. 4.1), so the P-SGK
row of the table is the reference.  A true atom counts as recovered when some
learned atom has 1 - |d_true^T d| < 0.01 (the criterion of the K-SVD paper the
experiment follows).
"""
import json
import math
import os

import numpy as np
import pytest
import torch

from paper_1509_05054_amd import dl, synth

from gpu_util import dev, host, note

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1_recovery.json")))
SNRS = [10, 20, 30, math.inf]
RUNS = 50


def _recovered(D_true, D):
    C = np.abs(D_true.astype(np.float64) @ D.astype(np.float64).T)
    return float(np.mean(1.0 - C.max(axis=1) < 0.01)) * 100.0


def test_table1_recovery_through_the_batched_launch():
    results = {}
    for s in (3, 4, 5):
        iters = 9 * s * s
        note(f"table 1 recovery s={s}: {len(SNRS) * RUNS} problems, {iters} iterations")
        probs, truths = [], []
        for col, snr in enumerate(SNRS):
            for run in range(RUNS):
                Y, Dt, _, _ = synth.recovery_problem(20, 50, s, 1500, 0.0, seed=1000 * s + run,
                                                     snr_db=snr)
                D0 = synth.initial_dictionary(Y, 50, seed=7000 + run)
                prm = dl.Params(20, 50, 1500, s)
                probs.append(dl.Problem(prm, dev(Y), dev(D0),
                                        torch.empty((1500, s), dtype=torch.int32, device="cuda"),
                                        torch.empty((1500, s), device="cuda"),
                                        torch.empty(iters, dtype=torch.float64, device="cuda")))
                truths.append((col, Dt))
        dl.iterate_batched(probs, iters, dl.batch_workspace(probs))
        torch.cuda.synchronize()
        per_cell = {c: [] for c in range(len(SNRS))}
        for (col, Dt), pb in zip(truths, probs):
            per_cell[col].append(_recovered(Dt, host(pb.D)))
            assert np.all(np.isfinite(host(pb.rmse)))
        for col in per_cell:
            v = np.array(per_cell[col])
            results[(s, col)] = (float(v.mean()), float(v.std(ddof=1) / math.sqrt(len(v))))
    lines = []
    bad = []
    for (s, col), (got, se) in sorted(results.items()):
        want = GOLDEN["P-SGK"][str(s)][col]
        lines.append(f"s={s} snr={SNRS[col]}: gpu {got:.2f} (se {se:.2f})  paper {want:.2f}")
        # the paper's figure is itself a 50-run mean: allow 3 points, or three
        # standard errors of ours where the spread between runs is large
        if abs(got - want) > max(3.0, 3.0 * se):
            bad.append(lines[-1])
    print("\n".join(lines))
    assert not bad, bad
