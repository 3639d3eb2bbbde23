"""Helpers shared by the GPU parity tests: device transfer, calls through the
C-ABI binding, and the comparison rules against the FP64 oracle."""
import sys

import numpy as np
import torch

from paper_1509_05054_amd import dl


def note(msg):
    """Name the case before a GPU step (flushed, so it survives a crash)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype).contiguous()


def host(t):
    return t.detach().cpu().numpy()


def gpu_omp(D, Y, s, **kw):
    m, p = Y.shape
    n = D.shape[0]
    prm = dl.Params(p, n, m, s, **kw)
    ws = dl.workspace(prm)
    Dg, Yg = dev(D), dev(Y)
    idx = torch.empty((m, s), dtype=torch.int32, device="cuda")
    val = torch.empty((m, s), dtype=torch.float32, device="cuda")
    dl.omp(prm, Dg, Yg, idx, val, ws)
    stats = dl.read_stats(prm, ws)
    return host(idx), host(val), stats


def gpu_update(Y, D, idx, val, group_size, rule=dl.RULE_AKSVD):
    m, p = Y.shape
    n = D.shape[0]
    s = idx.shape[1]
    prm = dl.Params(p, n, m, s, group_size=group_size, rule=rule)
    ws = dl.workspace(prm)
    Dg = dev(D)
    vg = dev(val)
    dl.jau_update(prm, dev(Y), Dg, dev(idx, torch.int32), vg, ws)
    stats = dl.read_stats(prm, ws)
    return host(Dg).astype(np.float64), host(vg).astype(np.float64), stats


def gpu_rmse(Y, D, idx, val):
    m, p = Y.shape
    n = D.shape[0]
    s = idx.shape[1]
    prm = dl.Params(p, n, m, s)
    ws = dl.workspace(prm)
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    dl.rmse(prm, dev(Y), dev(D), dev(idx, torch.int32), dev(val), out, ws)
    return float(host(out)[0])


def support_sets(idx):
    return [frozenset(int(j) for j in row if j >= 0) for row in idx]


def support_agreement(idx_a, idx_b):
    a, b = support_sets(idx_a), support_sets(idx_b)
    return float(np.mean([x == y for x, y in zip(a, b)]))


def disagreements_are_near_ties(D, Y, idx_gpu, idx_ref, rel=2e-4):
    """For every signal whose support differs, the first differing pick must
    be a near tie: with the common prefix's least-squares residual r (FP64),
    |d_gpu^T r| >= |d_ref^T r| - rel * ||y||.  Returns the offending rows."""
    D = np.asarray(D, dtype=np.float64)
    bad = []
    for i in np.nonzero([set(a) != set(b) for a, b in zip(idx_gpu, idx_ref)])[0]:
        y = np.asarray(Y[i], dtype=np.float64)
        g, r_ = list(idx_gpu[i]), list(idx_ref[i])
        t = 0
        while t < len(g) and g[t] == r_[t]:
            t += 1
        if t == len(g):
            continue
        if g[t] < 0 or r_[t] < 0:
            # one side stopped early: the other's correlation must be negligible
            res = y - D[g[:t]].T @ np.linalg.lstsq(D[g[:t]].T, y, rcond=None)[0] if t else y
            other = r_[t] if g[t] < 0 else g[t]
            if abs(D[other] @ res) > 1e-3 * np.linalg.norm(y):
                bad.append(int(i))
            continue
        pre = g[:t]
        res = y - D[pre].T @ np.linalg.lstsq(D[pre].T, y, rcond=None)[0] if t else y
        cg, cr = abs(D[g[t]] @ res), abs(D[r_[t]] @ res)
        if cg < cr - rel * np.linalg.norm(y):
            bad.append(int(i))
    return bad
