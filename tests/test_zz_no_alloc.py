"""The error entry point that allocates nothing (static device scratch)
against dl_rmse with a caller workspace: the same kernels and block
decomposition, so the same bits, on two calls in a row (the second smaller,
so it reuses the scratch the first left behind), and the oracle's value."""
import numpy as np
import pytest
import torch

import oracle
from paper_1509_05054_amd import dl

from gpu_util import dev, host, note

pytestmark = pytest.mark.gpu


def _problem(p, n, s, m, seed):
    rng = np.random.default_rng(seed)
    Y = rng.standard_normal((m, p)).astype(np.float32)
    D = rng.standard_normal((n, p))
    D = (D / np.linalg.norm(D, axis=1, keepdims=True)).astype(np.float32)
    idx = np.stack([rng.choice(n, size=s, replace=False) for _ in range(m)]).astype(np.int32)
    val = rng.standard_normal((m, s)).astype(np.float32)
    idx[::5, -1] = -1  # unused slots
    val[::5, -1] = 0.0
    return Y, D, idx, val


@pytest.mark.parametrize("first,second", [((64, 256, 6, 40001), (64, 256, 6, 3001)),
                                          ((256, 1024, 12, 5000), (16, 32, 3, 77))])
def test_rmse_noalloc_matches_workspace_entry_point(first, second):
    for k, (p, n, s, m) in enumerate((first, second)):
        note(f"rmse_noalloc call {k} p={p} n={n} s={s} m={m}")
        Y, D, idx, val = _problem(p, n, s, m, seed=100 * k + m)
        prm = dl.Params(p, n, m, s)
        Yg, Dg, ig, vg = dev(Y), dev(D), dev(idx, torch.int32), dev(val)
        out_ws = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
        out_na = torch.full((1,), -2.0, dtype=torch.float64, device="cuda")
        ws = dl.workspace(prm)
        dl.rmse(prm, Yg, Dg, ig, vg, out_ws, ws)
        dl.rmse_noalloc(prm, Yg, Dg, ig, vg, out_na)
        torch.cuda.synchronize()
        a, b = float(host(out_ws)[0]), float(host(out_na)[0])
        assert a == b, (k, a, b)
        rr = oracle.rmse(Y, D, idx, val)
        assert abs(b - rr) / rr < 1e-6, (k, b, rr)
