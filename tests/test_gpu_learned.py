"""Proposal network on the GPU (BF16 storage, FP32 accumulation) against the
FP64 oracle: forward, gradients, the optimiser step, top-k."""
import numpy as np
import pytest
import torch

import oracle
from oracle import learned
from oracle.bf16 import round_bf16
from paper_1509_05054_amd import dl, synth

from gpu_util import dev, host, note

pytestmark = pytest.mark.gpu

SIZES = (64, 512, 512, 256)


def _net(batch=256, seed=5):
    q = dl.MlpParams(64, 512, 256, batch=batch)
    vec = synth.mlp_params(SIZES, seed)
    assert vec.size == dl.mlp_param_count(q)
    ws = dl.mlp_workspace(q, dev(vec))
    return q, vec, ws


def _data(m=2048, seed=1):
    w = synth.workload("patches_p64_n256_s6_m16384", m=m)
    idx, val, _ = oracle.omp(w.D0, w.Y, w.s)
    return w, idx


def test_forward_matches_bf16_emulated_oracle():
    note("mlp forward")
    q, vec, ws = _net()
    w, _ = _data(1000)
    logits = torch.empty((w.m, 256), device="cuda")
    dl.mlp_forward(q, ws, dev(w.Y), logits)
    _, Zr = learned.forward(synth.unpack_mlp(vec, SIZES), w.Y, emulate_bf16=True)
    Zg = host(logits)
    err = np.abs(Zg - Zr).max() / np.abs(Zr).max()
    assert err < 2e-2, err
    # rows are independent of their batch position (1000 rows = 4 batches)
    assert np.corrcoef(Zg.ravel(), Zr.ravel())[0, 1] > 0.9999


def test_gradients_match_fp64_oracle():
    note("mlp gradients")
    B = 256
    q, vec, ws = _net(batch=B)
    w, idx = _data(1024)
    pairs = np.random.default_rng(3).permutation(w.m)[:B].astype(np.int32)
    dl.mlp_train_step(q, ws, dev(w.Y), dev(idx, torch.int32), dev(pairs, torch.int32), step=0)
    grads = torch.empty(vec.size, device="cuda")
    loss = dl.mlp_read(q, ws, grads=grads, want_loss=True)
    g = host(grads)
    params = synth.unpack_mlp(vec.astype(np.float64), SIZES)
    X = w.Y[pairs]
    T = learned.targets(idx[pairs], 256)
    A, Z = learned.forward(params, X, emulate_bf16=True)
    ref = learned.backward(params, A, Z, T)
    assert abs(loss - learned.bce_loss(Z, T)) / learned.bce_loss(Z, T) < 1e-3
    off = 0
    for (W, b), (gW, gb) in zip(params, ref):
        for arr, gr in ((W, gW), (b, gb)):
            got = g[off:off + arr.size].reshape(arr.shape)
            off += arr.size
            rel = np.linalg.norm(got - gr) / np.linalg.norm(gr)
            cos = float((got.ravel() @ gr.ravel()) / (np.linalg.norm(got) * np.linalg.norm(gr)))
            assert rel < 2e-2 and cos > 0.999, (arr.shape, rel, cos)


def test_adam_step_and_loss_decrease():
    note("mlp adam + training")
    B = 512
    q, vec, ws = _net(batch=B)
    w, idx = _data(4096)
    rng = np.random.default_rng(4)
    Yd, hd = dev(w.Y), dev(idx, torch.int32)
    pairs0 = dev(rng.permutation(w.m)[:B].astype(np.int32), torch.int32)
    dl.mlp_train_step(q, ws, Yd, hd, pairs0, step=0)
    g0 = torch.empty(vec.size, device="cuda")
    dl.mlp_read(q, ws, grads=g0)
    # the same batch with step 1: the first Adam step moves every weight by lr*g/(|g|+eps)
    dl.mlp_train_step(q, ws, Yd, hd, pairs0, step=1)
    p1 = torch.empty(vec.size, device="cuda")
    dl.mlp_read(q, ws, params=p1)
    g = host(g0).astype(np.float64)
    want = vec - 1e-3 * g / (np.abs(g) + 1e-8)
    np.testing.assert_allclose(host(p1), want, rtol=1e-5, atol=1e-7)
    losses = []
    for t in range(2, 60):
        pairs = dev(rng.permutation(w.m)[:B].astype(np.int32), torch.int32)
        dl.mlp_train_step(q, ws, Yd, hd, pairs, step=t)
        if t % 10 == 1:
            losses.append(dl.mlp_read(q, ws, want_loss=True))
    assert losses[-1] < 0.8 * losses[0], losses


@pytest.mark.parametrize("cols,k", [(256, 12), (1024, 24), (40, 5)])
def test_topk_exact(cols, k):
    note(f"topk cols={cols} k={k}")
    rng = np.random.default_rng(cols)
    Z = rng.standard_normal((777, cols)).astype(np.float32)
    Z[3, :10] = 1.5  # ties: the lower index goes first
    out = torch.empty((777, k), dtype=torch.int32, device="cuda")
    dl.topk(dev(Z), k, out)
    np.testing.assert_array_equal(host(out), learned.top_candidates(Z, k))
