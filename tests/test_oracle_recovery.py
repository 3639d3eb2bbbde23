"""Statistical pin of whole DL iterations against the paper's printed numbers:
the dictionary-recovery experiment of Sec. 4.1 (Table 1).

The paper averages 50 runs; a handful of runs is used here, so the bar is a
band around the printed percentage.  Recovery follows the K-SVD paper's
criterion that the paper refers to: a true atom counts as recovered when some
learned atom has 1 - |d_true^T d| < 0.01.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_1509_05054_amd import synth

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1_recovery.json")))


def _recovered(D_true, D):
    C = np.abs(D_true.astype(np.float64) @ D.T)
    return float(np.mean(1.0 - C.max(axis=1) < 0.01)) * 100.0


def _run(s, snr, runs, group_size=50):
    out = []
    for run in range(runs):
        Y, Dt, _, _ = synth.recovery_problem(20, 50, s, 1500, 0.0, seed=1000 * s + run, snr_db=snr)
        D0 = synth.initial_dictionary(Y, 50, seed=7000 + run)
        D, _, _, _ = oracle.iterate(Y, D0, s, 9 * s * s, group_size=group_size)
        out.append(_recovered(Dt, D))
    return float(np.mean(out))


@pytest.mark.parametrize("s,snr,col", [(3, math.inf, 3), (4, 20, 1)])
def test_full_jacobi_recovery_matches_table1(s, snr, col):
    want = GOLDEN["P-SGK"][str(s)][col]
    got = _run(s, snr, runs=6)
    assert abs(got - want) <= 6.0, (got, want)


def test_recovery_collapses_at_low_snr_and_s5():
    """Table 1's distinctive cell: at SNR 10 dB and s = 5 only about 12% of
    the atoms are recovered, against over 90% at 20 dB."""
    want = GOLDEN["P-SGK"]["5"][0]
    got = _run(5, 10, runs=3)
    assert want < 25 and got < 25, got
