"""Batched independent problems of uneven (p, n, m, s): every stage of an
iteration runs as one persistent launch over all problems.  Each problem must
get bit-for-bit what the single-problem iteration gives it (the same stage
bodies, the same reduction orders), which the single-problem parity tests tie
to the FP64 oracle; the first iteration is also checked against the oracle
directly, and the autotuner's choices must be valid launch shapes."""
import numpy as np
import pytest
import torch

import oracle
from paper_1509_05054_amd import dl, synth

from gpu_util import dev, host, note, support_agreement

pytestmark = pytest.mark.gpu


def _problems(specs, iters, shapes=None):
    out = []
    for k, q in enumerate(specs):
        prm = dl.Params(q["p"], q["n"], q["m"], q["s"])
        if shapes is not None:
            prm.omp_lanes_per_signal, prm.omp_atoms_per_lane = shapes[k]
        out.append(dl.Problem(
            prm, dev(q["Y"]), dev(q["D0"]),
            torch.empty((q["m"], q["s"]), dtype=torch.int32, device="cuda"),
            torch.empty((q["m"], q["s"]), device="cuda"),
            torch.full((max(iters, 1),), -1.0, dtype=torch.float64, device="cuda")))
    return out


def _single(q, iters, prm):
    ws = dl.workspace(prm)
    D = dev(q["D0"])
    idx = torch.empty((q["m"], q["s"]), dtype=torch.int32, device="cuda")
    val = torch.empty((q["m"], q["s"]), device="cuda")
    r = torch.full((max(iters, 1),), -1.0, dtype=torch.float64, device="cuda")
    dl.iterate(prm, dev(q["Y"]), D, iters, idx, val, r, ws)
    return host(D), host(idx), host(val), host(r)


def _assert_same_as_single(specs, probs, iters, which=None):
    torch.cuda.synchronize()
    for k in (range(len(specs)) if which is None else which):
        q, pb = specs[k], probs[k]
        D, idx, val, r = _single(q, iters, pb.prm)
        tag = (k, q["p"], q["n"], q["s"], q["m"])
        np.testing.assert_array_equal(host(pb.D), D, err_msg=str(tag))
        if iters > 0:
            np.testing.assert_array_equal(host(pb.X_idx), idx, err_msg=str(tag))
            np.testing.assert_array_equal(host(pb.X_val), val, err_msg=str(tag))
            np.testing.assert_array_equal(host(pb.rmse)[:iters], r[:iters], err_msg=str(tag))


def _tiny(p, n, m, s, seed):
    rng = np.random.default_rng(seed)
    Y = rng.standard_normal((m, p)).astype(np.float32)
    D0 = rng.standard_normal((n, p)).astype(np.float32)
    return dict(p=p, n=n, m=m, s=s, Y=Y, D0=D0)


@pytest.mark.parametrize("iters", [3, 4])
def test_batched_equals_single_problem_bitwise(iters):
    specs = synth.batched_problems(12, seed=505, m_scale=0.05)
    note(f"batched 12 small problems iters={iters}")
    probs = _problems(specs, iters)
    ws = dl.batch_workspace(probs)
    dl.iterate_batched(probs, iters, ws)
    _assert_same_as_single(specs, probs, iters)


def test_batched_edge_cases():
    """Signal counts below one item, a single problem, equal problems, and
    zero iterations (the dictionary is only normalised)."""
    specs = [_tiny(16, 32, 7, 3, 1), _tiny(4, 4, 1, 1, 2), _tiny(256, 1024, 300, 16, 3),
             _tiny(36, 72, 65, 5, 4), _tiny(36, 72, 65, 5, 4)]
    note("batched edge cases")
    for iters in (0, 1, 2):
        probs = _problems(specs, iters)
        ws = dl.batch_workspace(probs)
        dl.iterate_batched(probs, iters, ws)
        _assert_same_as_single(specs, probs, iters)
        if iters == 0:
            for q, pb in zip(specs, probs):
                np.testing.assert_allclose(np.linalg.norm(host(pb.D), axis=1), 1.0, atol=1e-6)
                assert host(pb.rmse)[0] == -1.0  # untouched
    one = _problems(specs[2:3], 2)
    dl.iterate_batched(one, 2, dl.batch_workspace(one))
    _assert_same_as_single(specs[2:3], one, 2)
    # the workspace can be reused for another call without re-initialisation
    again = _problems(specs[2:3], 2)
    ws = dl.batch_workspace(again)
    dl.iterate_batched(again, 2, ws)
    dl.iterate_batched(_problems(specs[2:3], 2), 2, ws)
    _assert_same_as_single(specs[2:3], again, 2)


def test_batched_first_iteration_matches_oracle():
    specs = synth.batched_problems(6, seed=506, m_scale=0.04)
    note("batched vs oracle, first iteration")
    probs = _problems(specs, 1)
    dl.iterate_batched(probs, 1, dl.batch_workspace(probs))
    torch.cuda.synchronize()
    for q, pb in zip(specs, probs):
        D = oracle.normalize(q["D0"]).astype(np.float32)
        ir, _, _ = oracle.omp(D, q["Y"], q["s"])
        agree = support_agreement(host(pb.X_idx), ir)
        assert agree >= 0.995, (q["p"], q["n"], q["s"], agree)
        _, _, _, rr = oracle.iterate(q["Y"], q["D0"], q["s"], 1, q["n"])
        rg = host(pb.rmse)[0]
        # relative bar, with a floor at FP32 rounding of the signal scale for
        # problems the dictionary represents exactly (m <= n: D0 holds Y)
        floor = 1e-6 * np.sqrt(np.mean(q["Y"].astype(np.float64) ** 2))
        assert abs(rg - rr[0]) < 1e-4 * rr[0] + floor, (q["p"], q["n"], q["s"], rg, rr[0])


def test_autotuner_picks_valid_shapes_and_keeps_results():
    specs = synth.batched_problems(8, seed=507, m_scale=0.1)
    note("autotune + batched with tuned shapes")
    probs = _problems(specs, 2)
    ws = dl.batch_workspace(probs)
    shapes = dl.autotune(probs, ws, reps=2)
    for q, (lps, npl) in zip(specs, shapes):
        if (lps, npl) == (0, 0):
            continue  # a problem that runs alone keeps the default shape
        assert lps in (4, 8, 16, 32, 64) and npl in (4, 8, 16), (lps, npl)
        assert lps * npl >= q["n"] and lps >= min(16, max(4, q["s"])), (q["n"], q["s"], lps)
    # the tuner left D alone: run the tuned batch and compare with the
    # single-problem path under the same shapes
    probs = _problems(specs, 2, shapes)
    dl.iterate_batched(probs, 2, ws)
    _assert_same_as_single(specs, probs, 2)


def test_batched_mixed_alone_and_shared():
    """Problems whose coding fills the GPU (they run with the single-problem
    launches on the library's side streams, concurrently) next to problems
    that share the persistent launches, in one call with an odd iteration
    count: every problem bit for bit as dl_iterate gives it."""
    specs = [_tiny(64, 256, 20000, 6, 11), _tiny(64, 256, 3000, 6, 12),
             _tiny(256, 1024, 2000, 12, 13), _tiny(36, 72, 2500, 5, 14),
             _tiny(64, 256, 13000, 6, 15), _tiny(16, 32, 40, 3, 16)]
    note("batched mix of problems that run alone and problems that share launches")
    probs = _problems(specs, 3)
    ws = dl.batch_workspace(probs)
    dl.iterate_batched(probs, 3, ws)
    _assert_same_as_single(specs, probs, 3)
    shapes = dl.autotune(probs, ws, reps=1)
    assert shapes[0] == (0, 0) and shapes[2] == (0, 0) and shapes[4] == (0, 0), shapes


def test_batched_orders_on_the_callers_stream():
    """The problems that run alone go to the library's own streams; the call
    still orders like one launch sequence on the caller's stream: it starts
    after the caller's earlier work there (here the copy of the initial
    dictionaries, behind a long kernel) and later work on that stream sees its
    results, with only that stream synchronised."""
    specs = [_tiny(64, 256, 20000, 6, 21), _tiny(64, 256, 3000, 6, 22),
             _tiny(64, 256, 14000, 6, 23)]
    note("batched call ordered on a caller's stream")
    probs = _problems(specs, 2)
    ws = dl.batch_workspace(probs)
    side = torch.cuda.Stream()
    D0s = [dev(q["D0"]) for q in specs]
    for pb in probs:
        pb.D.fill_(float("nan"))
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        big = torch.randn(4096, 4096, device="cuda")
        for _ in range(4):
            big = big @ big.T / 4096.0  # keeps the stream busy before the copies
        for pb, d0 in zip(probs, D0s):
            pb.D.copy_(d0)
        dl.iterate_batched(probs, 2, ws, stream=side)
        outs = [(pb.D.clone(), pb.X_idx.clone(), pb.X_val.clone(), pb.rmse.clone())
                for pb in probs]
    side.synchronize()
    for k, q in enumerate(specs):
        D, idx, val, r = _single(q, 2, probs[k].prm)
        np.testing.assert_array_equal(host(outs[k][0]), D, err_msg=str(k))
        np.testing.assert_array_equal(host(outs[k][1]), idx, err_msg=str(k))
        np.testing.assert_array_equal(host(outs[k][2]), val, err_msg=str(k))
        np.testing.assert_array_equal(host(outs[k][3])[:2], r[:2], err_msg=str(k))


def test_full_batch_of_uneven_problems():
    """The 64-problem batch at full size for two iterations; a spread of its
    problems is checked bit-for-bit against the single-problem path."""
    specs = synth.batched_problems(64, seed=505)
    note("batched 64 full-size problems")
    probs = _problems(specs, 2)
    ws = dl.batch_workspace(probs)
    dl.iterate_batched(probs, 2, ws)
    order = np.argsort([q["n"] * q["s"] for q in specs])
    which = sorted(set(int(order[k]) for k in (0, 1, 16, 32, 48, 62, 63)))
    _assert_same_as_single(specs, probs, 2, which)
    r = np.array([host(pb.rmse)[:2] for pb in probs])
    assert np.all(np.isfinite(r)) and np.all(r > 0)
