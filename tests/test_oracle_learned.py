"""Pins of the learned-proposal oracle: gradients by central finite
differences, Adam's closed-form first step, the removal-cost identity of
backward elimination, brute force over candidate subsets, top-k order."""
import itertools

import numpy as np
import pytest

from oracle import learned


def _small_params(rng, sizes=(6, 9, 7, 5)):
    return [(rng.standard_normal((o, i)) * np.sqrt(2.0 / i), rng.standard_normal(o) * 0.1)
            for i, o in zip(sizes[:-1], sizes[1:])]


@pytest.mark.parametrize("pos_weight", [1.0, 3.5])
def test_mlp_gradients_match_central_differences(pos_weight):
    rng = np.random.default_rng(0)
    params = _small_params(rng)
    X = rng.standard_normal((11, 6))
    T = (rng.random((11, 5)) < 0.3).astype(float)
    A, Z = learned.forward(params, X)
    grads = learned.backward(params, A, Z, T, pos_weight)
    h = 1e-6
    for li, (W, b) in enumerate(params):
        for arr, g in ((W, grads[li][0]), (b, grads[li][1])):
            num = np.zeros_like(arr)
            it = np.nditer(arr, flags=["multi_index"])
            for _ in it:
                ix = it.multi_index
                old = arr[ix]
                arr[ix] = old + h
                lp = learned.bce_loss(learned.forward(params, X)[1], T, pos_weight)
                arr[ix] = old - h
                lm = learned.bce_loss(learned.forward(params, X)[1], T, pos_weight)
                arr[ix] = old
                num[ix] = (lp - lm) / (2 * h)
            rel = np.linalg.norm(num - g) / max(np.linalg.norm(num), 1e-12)
            assert rel < 1e-6, (li, rel)


def test_bce_loss_closed_forms():
    Z = np.array([[0.0, 2.0], [-3.0, 1.5]])
    T = np.array([[1.0, 0.0], [0.0, 1.0]])
    # -log sigmoid(z) for positives, -log(1 - sigmoid(z)) for negatives
    terms = [np.log(2), np.log1p(np.exp(2.0)), np.log1p(np.exp(-3.0)), np.log1p(np.exp(-1.5))]
    assert abs(learned.bce_loss(Z, T) - np.mean(terms)) < 1e-12
    w = 4.0
    weighted = [w * terms[0], terms[1], terms[2], w * terms[3]]
    assert abs(learned.bce_loss(Z, T, w) - np.mean(weighted)) < 1e-12


def test_network_input_is_unit_norm_direction():
    Y = np.array([[3.0, 4.0], [0.0, 0.0]])
    np.testing.assert_allclose(learned.network_input(Y), [[0.6, 0.8], [0.0, 0.0]])


def test_adam_first_step_is_signed_learning_rate():
    """After one step the bias-corrected moments are g and g^2, so every
    parameter moves by lr * g / (|g| + eps)."""
    rng = np.random.default_rng(1)
    params = _small_params(rng)
    grads = [(rng.standard_normal(W.shape), rng.standard_normal(b.shape)) for W, b in params]
    new, _ = learned.adam_step(params, grads, learned.adam_init(params), t=1, lr=1e-3)
    for (W, b), (Wn, bn), (gW, gb) in zip(params, new, grads):
        np.testing.assert_allclose(W - Wn, 1e-3 * gW / (np.abs(gW) + 1e-8), rtol=1e-12)
        np.testing.assert_allclose(b - bn, 1e-3 * gb / (np.abs(gb) + 1e-8), rtol=1e-12)


def test_adam_constant_gradient_moves_by_signed_learning_rate_every_step():
    """With the same gradient g at every step the moments are m_t = (1 - b1^t) g
    and v_t = (1 - b2^t) g^2, so the bias-corrected moments are g and g^2 at
    every t and each step moves by lr * g / (|g| + eps).  Dividing by
    (1 - b) instead of (1 - b^t) breaks this from the second step on."""
    rng = np.random.default_rng(7)
    params = _small_params(rng)
    grads = [(rng.standard_normal(W.shape), rng.standard_normal(b.shape)) for W, b in params]
    state = learned.adam_init(params)
    cur = params
    steps = 5
    for t in range(1, steps + 1):
        cur, state = learned.adam_step(cur, grads, state, t=t, lr=2e-3)
    for (W, b), (Wn, bn), (gW, gb) in zip(params, cur, grads):
        np.testing.assert_allclose(W - Wn, steps * 2e-3 * gW / (np.abs(gW) + 1e-8), rtol=1e-9)
        np.testing.assert_allclose(b - bn, steps * 2e-3 * gb / (np.abs(gb) + 1e-8), rtol=1e-9)


def test_adam_two_steps_hand_computed():
    """Scalar weight 1, gradients 1 then -2, lr 0.1, b1 0.9, b2 0.999, eps 0.
    By hand: step 1 gives m = 0.1, v = 0.001, corrected 1 and 1, so w = 0.9.
    Step 2: m = 0.09 - 0.2 = -0.11 and v = 0.000999 + 0.004 = 0.004999;
    corrected by 1 - 0.81 = 0.19 and 1 - 0.998001 = 0.001999 they are -11/19
    and 4999/1999, so w = 0.9 + 0.1 (11/19) / sqrt(4999/1999) = 0.93661035..."""
    p0 = [(np.array([[1.0]]), np.array([0.0]))]
    g1 = [(np.array([[1.0]]), np.array([0.0]))]
    g2 = [(np.array([[-2.0]]), np.array([0.0]))]
    st = learned.adam_init(p0)
    p1, st = learned.adam_step(p0, g1, st, t=1, lr=0.1, eps=0.0)
    assert abs(p1[0][0][0, 0] - 0.9) < 1e-15
    p2, st = learned.adam_step(p1, g2, st, t=2, lr=0.1, eps=0.0)
    assert abs(p2[0][0][0, 0] - 0.9366103527035843) < 1e-13
    mW, vW, _, _ = st[0]
    assert abs(mW[0, 0] + 0.11) < 1e-15 and abs(vW[0, 0] - 0.004999) < 1e-15


def test_removal_cost_equals_explicit_refit():
    """Dropping atom j from a least-squares fit raises ||r||^2 by exactly
    c_j^2 / [(D_C^T D_C)^{-1}]_jj."""
    rng = np.random.default_rng(2)
    D = rng.standard_normal((30, 16))
    y = rng.standard_normal(16)
    C = list(rng.choice(30, size=8, replace=False))
    A = D[C]
    Gi = np.linalg.inv(A @ A.T)
    c = Gi @ (A @ y)
    r2 = np.sum((y - A.T @ c) ** 2)
    for q in range(len(C)):
        keep = [C[t] for t in range(len(C)) if t != q]
        x, *_ = np.linalg.lstsq(D[keep].T, y, rcond=None)
        r2q = np.sum((y - D[keep].T @ x) ** 2)
        assert abs((r2q - r2) - c[q] ** 2 / Gi[q, q]) < 1e-10


def test_pruning_never_beats_bruteforce_and_often_matches():
    rng = np.random.default_rng(3)
    D = rng.standard_normal((40, 16))
    D /= np.linalg.norm(D, axis=1, keepdims=True)
    exact = 0
    for trial in range(40):
        y = rng.standard_normal(16)
        cand = rng.choice(40, size=12, replace=False)
        sup, c, rn = learned.restricted_ls_prune(D, y, cand, 6)
        assert len(sup) == 6 and set(sup) <= set(cand)
        best = min(np.linalg.norm(y - D[list(S)].T @ np.linalg.lstsq(D[list(S)].T, y, rcond=None)[0])
                   for S in itertools.combinations(cand, 6))
        assert rn >= best - 1e-12
        exact += rn <= best + 1e-12
        np.testing.assert_allclose(c, np.linalg.lstsq(D[sup].T, y, rcond=None)[0], rtol=1e-9,
                                   atol=1e-12)
    assert exact >= 10  # greedy elimination finds the optimum in a fair share of cases


def test_pruning_recovers_a_planted_support():
    rng = np.random.default_rng(4)
    D = rng.standard_normal((50, 32))
    D /= np.linalg.norm(D, axis=1, keepdims=True)
    true = rng.choice(50, size=6, replace=False)
    y = rng.standard_normal(6) @ D[true]
    others = [j for j in range(50) if j not in true][:6]
    sup, c, rn = learned.restricted_ls_prune(D, y, np.concatenate([others, true]), 6)
    assert set(sup) == set(true) and rn < 1e-10


def test_top_candidates_order_and_ties():
    Z = np.array([[0.1, 0.5, 0.5, -1.0, 0.7]])
    np.testing.assert_array_equal(learned.top_candidates(Z, 3), [[4, 1, 2]])


def test_fallback_margin():
    assert learned.needs_fallback(1.021, 1.0) and not learned.needs_fallback(1.019, 1.0)
