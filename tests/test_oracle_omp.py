"""Pins of the oracle's OMP (step 1 of the DL iteration, Alg. 1) against facts
that do not depend on the oracle itself: brute-force enumeration, the
coherence-based exact-recovery guarantee, and special cases with closed forms.
"""
import itertools

import numpy as np
import pytest
import scipy.linalg

import oracle


def _lstsq_residual(D, y, support):
    A = D[list(support)].T  # p x k
    x, *_ = np.linalg.lstsq(A, y, rcond=None)
    return y - A @ x, x


def _unit_rows(A):
    return A / np.linalg.norm(A, axis=1, keepdims=True)


@pytest.mark.parametrize("p,n,s,seed", [(8, 16, 2, 1), (8, 16, 3, 2), (6, 12, 4, 3)])
def test_omp_greedy_steps_match_bruteforce_lstsq(p, n, s, seed):
    """Every OMP pick is the argmax of |d_j^T r| with r the least-squares
    residual (numpy lstsq, an SVD-based solver) of the previous picks; the final
    coefficients are the least-squares fit on the chosen support; the residual
    is never below the best residual over all C(n, s) supports."""
    rng = np.random.default_rng(seed)
    D = _unit_rows(rng.standard_normal((n, p)))
    Y = rng.standard_normal((300, p))
    idx, val, early = oracle.omp(D, Y, s)
    assert early == 0
    supports = list(itertools.combinations(range(n), s))
    for i in range(Y.shape[0]):
        y = Y[i]
        sel = list(idx[i])
        assert len(set(sel)) == s and min(sel) >= 0
        for t in range(s):
            r, _ = _lstsq_residual(D, y, sel[:t]) if t else (y.copy(), None)
            c = np.abs(D @ r)
            c[sel[:t]] = -1
            assert sel[t] == int(np.argmax(c)), (i, t)
        r, x = _lstsq_residual(D, y, sel)
        np.testing.assert_allclose(val[i], x, rtol=1e-9, atol=1e-11)
        best = min(np.linalg.norm(_lstsq_residual(D, y, S)[0]) for S in supports)
        assert np.linalg.norm(r) >= best - 1e-12


def test_omp_reaches_bruteforce_optimum_on_exact_instances():
    """Noiseless 2-sparse signals over a well-conditioned dictionary: the
    brute-force optimum is zero error and OMP attains it with the true support."""
    rng = np.random.default_rng(7)
    p, n, s = 8, 12, 2
    D = _unit_rows(rng.standard_normal((n, p)))
    hits = 0
    for trial in range(200):
        sup = rng.choice(n, size=s, replace=False)
        coef = rng.standard_normal(s)
        y = coef @ D[sup]
        idx, val, _ = oracle.omp(D, y[None, :], s)
        r, _ = _lstsq_residual(D, y, idx[0])
        if set(idx[0]) == set(sup):
            hits += 1
            assert np.linalg.norm(r) < 1e-12
    # exact-recovery is not guaranteed at this coherence; most instances succeed
    assert hits >= 150


@pytest.mark.parametrize("p,s", [(16, 1), (16, 2), (64, 2), (64, 4)])
def test_omp_exact_recovery_low_coherence(p, s):
    """D = [I | H/sqrt(p)] has coherence 1/sqrt(p); OMP recovers every
    s-sparse signal exactly when s < (1 + sqrt(p)) / 2 (Tropp 2004, Donoho-Elad)."""
    assert s < (1 + np.sqrt(p)) / 2
    H = scipy.linalg.hadamard(p).astype(np.float64) / np.sqrt(p)
    D = np.vstack([np.eye(p), H])  # rows are atoms, n = 2p
    n = 2 * p
    rng = np.random.default_rng(p * 10 + s)
    m = 400
    idx_true = np.array([rng.choice(n, size=s, replace=False) for _ in range(m)])
    val_true = rng.standard_normal((m, s))
    Y = np.einsum("ms,msp->mp", val_true, D[idx_true])
    idx, val, early = oracle.omp(D, Y, s)
    assert early == 0
    for i in range(m):
        got = dict(zip(idx[i], val[i]))
        want = dict(zip(idx_true[i], val_true[i]))
        assert set(got) == set(want)
        for j in want:
            assert abs(got[j] - want[j]) < 1e-12


def test_omp_s1_is_max_correlation():
    rng = np.random.default_rng(11)
    D = _unit_rows(rng.standard_normal((40, 10)))
    Y = rng.standard_normal((100, 10))
    idx, val, _ = oracle.omp(D, Y, 1)
    c = Y @ D.T
    j = np.argmax(np.abs(c), axis=1)
    np.testing.assert_array_equal(idx[:, 0], j)
    np.testing.assert_allclose(val[:, 0], c[np.arange(100), j], rtol=1e-12)


def test_omp_orthonormal_dictionary_is_hard_thresholding():
    """n = p orthonormal atoms: OMP keeps the s largest |D^T y| with x = D^T y."""
    rng = np.random.default_rng(12)
    p, s = 12, 4
    Q, _ = np.linalg.qr(rng.standard_normal((p, p)))
    D = Q.T
    Y = rng.standard_normal((200, p))
    idx, val, _ = oracle.omp(D, Y, s)
    c = Y @ D.T
    for i in range(200):
        order = np.argsort(-np.abs(c[i]), kind="stable")[:s]
        np.testing.assert_array_equal(idx[i], order)
        np.testing.assert_allclose(val[i], c[i, order], rtol=1e-10, atol=1e-12)


def test_omp_signal_equal_to_atom_stops_after_one():
    rng = np.random.default_rng(13)
    D = _unit_rows(rng.standard_normal((30, 16)))
    j = 17
    idx, val, early = oracle.omp(D, D[j][None, :], 4)
    assert early == 1
    assert idx[0, 0] == j and abs(val[0, 0] - 1.0) < 1e-12
    assert list(idx[0, 1:]) == [-1, -1, -1] and list(val[0, 1:]) == [0, 0, 0]


def test_omp_zero_signal_gives_empty_support():
    rng = np.random.default_rng(14)
    D = _unit_rows(rng.standard_normal((30, 16)))
    idx, val, early = oracle.omp(D, np.zeros((1, 16)), 3)
    assert early == 1 and list(idx[0]) == [-1] * 3 and list(val[0]) == [0] * 3


def test_omp_ties_and_duplicate_atoms():
    """Duplicate atoms give an exact correlation tie: the lower index wins and
    the duplicate is then rejected by the pivot test (it lies in the span)."""
    rng = np.random.default_rng(15)
    D = _unit_rows(rng.standard_normal((10, 8)))
    D[7] = D[3]
    y = 2.0 * D[3] + 1e-3 * D[5]
    idx, val, _ = oracle.omp(D, y[None, :], 3)
    assert idx[0, 0] == 3
    assert 7 not in set(idx[0])


def test_omp_selection_order_and_padding_layout():
    rng = np.random.default_rng(16)
    D = _unit_rows(rng.standard_normal((20, 10)))
    Y = rng.standard_normal((50, 10))
    idx, val, _ = oracle.omp(D, Y, 5)
    c0 = np.abs(Y @ D.T)
    # slot 0 is the first (largest-correlation) pick
    np.testing.assert_array_equal(idx[:, 0], np.argmax(c0, axis=1))
