"""Precision variant: D^T Y and D^T D on BF16 matrix cores with FP32
accumulation, FP32 Cholesky (FP64 pivot recompute), FP64 error.

Parity is checked against the oracle fed BF16-rounded inputs (quantisation
emulated, so only kernel error remains), and the error against the exact FP64
oracle is measured and bounded (that difference is the quantisation's).
"""
import numpy as np
import pytest
import torch

import oracle
from oracle.bf16 import round_bf16
from paper_1509_05054_amd import dl, synth

from gpu_util import dev, disagreements_are_near_ties, host, note, support_agreement

pytestmark = pytest.mark.gpu


def _patches(p, n, m, seed):
    imgs = synth.synthetic_images(2, 256, seed)
    pool = synth.image_patches(imgs, int(round(np.sqrt(p))), m + 2 * n, seed + 1)
    return pool[:m], synth.initial_dictionary(pool[m:], n, seed + 2)


@pytest.mark.parametrize("p,n,m", [(256, 1024, 700), (64, 256, 1000), (144, 288, 333)])
def test_bf16_products_equal_fp32_sums_of_rounded_inputs(p, n, m):
    note(f"bf16 products p={p} n={n} m={m}")
    Y, D = _patches(p, n, m, seed=p + n)
    prm = dl.Params(p, n, m, 4, precision=dl.PREC_BF16)
    ws = dl.workspace(prm)
    G = torch.empty((n, n), device="cuda")
    A0 = torch.empty((m, n), device="cuda")
    dl.products(prm, dev(D), dev(Y), G, A0, ws)
    Db = round_bf16(D).astype(np.float64)
    Yb = round_bf16(Y).astype(np.float64)
    # products of BF16 values are exact in FP32; only the FP32 accumulation differs
    nd, ny = np.linalg.norm(Db, axis=1), np.linalg.norm(Yb, axis=1)
    eg = np.abs(host(G) - Db @ Db.T) / np.outer(nd, nd)
    ea = np.abs(host(A0) - Yb @ Db.T) / np.maximum(np.outer(ny, nd), 1e-30)
    assert eg.max() < 2e-6 and ea.max() < 2e-6, (eg.max(), ea.max())
    # and they are not the FP32 products: the rounding really happened
    D64, Y64 = D.astype(np.float64), Y.astype(np.float64)
    assert np.abs(host(A0) - Y64 @ D64.T).max() > 1e-5 * ny.max()


def test_bf16_omp_matches_emulated_oracle():
    note("bf16 omp p256 n1024 s12")
    p, n, s, m = 256, 1024, 12, 600
    Y, D = _patches(p, n, m, seed=31)
    prm = dl.Params(p, n, m, s, precision=dl.PREC_BF16)
    ws = dl.workspace(prm)
    idx = torch.empty((m, s), dtype=torch.int32, device="cuda")
    val = torch.empty((m, s), device="cuda")
    dl.omp(prm, dev(D), dev(Y), idx, val, ws)
    ig, vg = host(idx), host(val)
    Db, Yb = round_bf16(D), round_bf16(Y)
    ir, vr, _ = oracle.omp(Db, Yb, s)
    agree = support_agreement(ig, ir)
    assert agree >= 0.995, agree
    assert not disagreements_are_near_ties(Db, Yb, ig, ir)
    same = np.all(ig == ir, axis=1)
    yn = np.linalg.norm(Yb.astype(np.float64), axis=1, keepdims=True)
    assert (np.abs(vg[same] - vr[same]) / yn[same]).max() < 1e-4


def test_bf16_iterate_error_against_fp64_oracle():
    """16x16 patches, n=1024, s=12 (the precision workload's shapes) on a
    subset of signals: the RMSE trajectory follows the BF16-emulated oracle
    tightly and the exact FP64 oracle within the quantisation's effect."""
    note("bf16 iterate p256 n1024 s12 m4096")
    w = synth.workload("patches_p256_n1024_s12_m65536", m=4096)
    iters = 3
    prm = dl.Params(w.p, w.n, w.m, w.s, precision=dl.PREC_BF16)
    ws = dl.workspace(prm)
    D = dev(w.D0)
    idx = torch.empty((w.m, w.s), dtype=torch.int32, device="cuda")
    val = torch.empty((w.m, w.s), device="cuda")
    r = torch.empty(iters, dtype=torch.float64, device="cuda")
    dl.iterate(prm, dev(w.Y), D, iters, idx, val, r, ws)
    rg = host(r)
    _, _, _, re = oracle.iterate_bf16(w.Y, w.D0, w.s, iters, w.n)
    _, _, _, rx = oracle.iterate(w.Y, w.D0, w.s, iters, w.n)
    rel_emul = np.abs(rg - re) / re
    rel_exact = np.abs(rg - rx) / rx
    print(f"bf16 rmse gpu={rg} emulated={re} fp64={rx} rel_emul={rel_emul} rel_exact={rel_exact}")
    assert rel_emul[0] < 1e-4, rel_emul
    assert rel_emul.max() < 2e-3, rel_emul
    assert rel_exact.max() < 2e-2, rel_exact


def test_bf16_precision_workload_full_size_one_iteration():
    """The precision workload at its full size (65,536 signals, p=256,
    n=1024, s=12), one iteration teacher-forced: the BF16 coding at D0
    against the oracle fed the same BF16-rounded D and Y (supports, near-tie
    validity of every disagreement, coefficients), then the FP32 atom update
    from the oracle's coding against the FP64 update."""
    note("bf16 precision workload full size, one iteration")
    w = synth.workload("patches_p256_n1024_s12_m65536")
    p, n, m, s = w.p, w.n, w.m, w.s
    assert m == 65536
    prm = dl.Params(p, n, m, s, precision=dl.PREC_BF16)
    ws = dl.workspace(prm)
    idx = torch.empty((m, s), dtype=torch.int32, device="cuda")
    val = torch.empty((m, s), device="cuda")
    dl.omp(prm, dev(w.D0), dev(w.Y), idx, val, ws)
    ig, vg = host(idx), host(val)
    Db, Yb = round_bf16(w.D0), round_bf16(w.Y)
    ir, vr, _ = oracle.omp(Db, Yb, s)
    agree = support_agreement(ig, ir)
    print(f"full-size BF16 coding: support agreement {agree:.5f}")
    assert agree >= 0.995, agree
    assert not disagreements_are_near_ties(Db, Yb, ig, ir)
    same = np.all(ig == ir, axis=1)
    yn = np.linalg.norm(Yb.astype(np.float64), axis=1, keepdims=True)
    assert (np.abs(vg[same] - vr[same]) / yn[same]).max() < 1e-4
    # the update (FP32 residual products) from the oracle's coding
    v32 = vr.astype(np.float32)
    Dr, vnr, unused = oracle.jau_update(w.Y, w.D0, ir, v32, n)
    prm32 = dl.Params(p, n, m, s)
    ws32 = dl.workspace(prm32)
    Dg = dev(w.D0)
    vng = dev(v32)
    dl.jau_update(prm32, dev(w.Y), Dg, dev(ir, torch.int32), vng, ws32)
    st = dl.read_stats(prm32, ws32)
    assert st["unused_atoms"] == unused
    assert np.abs(host(Dg).astype(np.float64) - Dr).max() < 1e-4
    ynf = np.linalg.norm(w.Y.astype(np.float64), axis=1, keepdims=True)
    assert (np.abs(host(vng).astype(np.float64) - vnr) / ynf).max() < 1e-4
