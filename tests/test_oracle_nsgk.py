"""Pins of the oracle's P-NSGK atom update (Sec. 3, eq. 7): the P-SGK group
loop run on Z = Y + D^(k) X^(k-1) - D^(k) X^(k) with the representations
X^(k-1) the iteration started from.  Each pin comes from the paper or the
mathematics, not from the oracle's own code: the reduction to SGK when the
representations repeat, a closed form at full parallelism, a separately
written sequential (Gauss-Seidel) NSGK, the exact fixed point, and the P-NSGK
row of Table 1."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_1509_05054_amd import synth

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1_recovery.json")))


def _unit_rows(A):
    return A / np.linalg.norm(A, axis=1, keepdims=True)


def _dense_X(idx, val, n):
    m, s = idx.shape
    X = np.zeros((n, m))
    for i in range(m):
        for t in range(s):
            if idx[i, t] >= 0:
                X[idx[i, t], i] = val[i, t]
    return X


def _two_codings(p=12, n=24, s=3, m=400, seed=0):
    """Signals, D^(k), X^(k) (OMP against D^(k)) and X^(k-1) (OMP against a
    perturbed dictionary, as the previous iteration's coding would be)."""
    rng = np.random.default_rng(seed)
    D = _unit_rows(rng.standard_normal((n, p)))
    Y = rng.standard_normal((m, p))
    idx, val, _ = oracle.omp(D, Y, s)
    Dprev = _unit_rows(D + 0.3 * rng.standard_normal((n, p)))
    idx_p, val_p, _ = oracle.omp(Dprev, Y, s)
    return Y, D, idx, val, idx_p, val_p


@pytest.mark.parametrize("gs", [1, 5, 24])
def test_repeated_representations_reduce_to_sgk(gs):
    """With X^(k-1) = X^(k), eq. 7 gives Z = Y and the update is P-SGK's."""
    Y, D, idx, val, _, _ = _two_codings(seed=1)
    Dn, unused = oracle.nsgk_update(Y, D, idx, val, idx, val, gs)
    Ds, vs, unused_s = oracle.jau_update(Y, D, idx, val, gs, rule=oracle.RULE_SGK)
    np.testing.assert_allclose(Dn, Ds, atol=1e-12)
    assert unused == unused_s


def test_full_parallel_closed_form():
    """At group size n every atom reads E = Z - D^(k) X^(k-1) = Y - D^(k) X^(k),
    so d_j' = normalise(E x_j^T + d_j ||x_j||^2) with x_j the j-th row of
    X^(k-1); atoms X^(k-1) does not use keep their value."""
    Y, D, idx, val, idx_p, val_p = _two_codings(seed=2)
    n = D.shape[0]
    X = _dense_X(idx, val, n)
    Xp = _dense_X(idx_p, val_p, n)
    E = Y.T - D.T @ X                       # p x m
    G = (E @ Xp.T).T + D * (Xp * Xp).sum(axis=1, keepdims=True)
    used = np.abs(Xp).sum(axis=1) > 0
    want = D.copy()
    want[used] = _unit_rows(G[used])
    Dn, unused = oracle.nsgk_update(Y, D, idx, val, idx_p, val_p, n)
    assert unused == int((~used).sum())
    np.testing.assert_allclose(Dn, want, atol=1e-12)


def _sequential_nsgk(Y, D, idx, val, idx_p, val_p):
    """Gauss-Seidel NSGK written independently from dense matrices: Z from
    eq. 7, then one atom at a time the residual R = Z - D X^(k-1) is kept up
    to date after each atom instead of being recomputed."""
    D = D.copy()
    n = D.shape[0]
    X = _dense_X(idx, val, n)
    Xp = _dense_X(idx_p, val_p, n)
    Z = Y.T + D.T @ Xp - D.T @ X
    R = Z - D.T @ Xp
    for j in range(n):
        I = np.nonzero(Xp[j])[0]
        if I.size == 0:
            continue
        x = Xp[j, I]
        F = R[:, I] + np.outer(D[j], x)
        g = F @ x / (x @ x)
        if np.linalg.norm(g) == 0:
            continue
        d = g / np.linalg.norm(g)
        R[:, I] = F - np.outer(d, x)
        D[j] = d
    return D


def test_group_size_one_is_sequential_nsgk():
    Y, D, idx, val, idx_p, val_p = _two_codings(seed=3)
    Dn, _ = oracle.nsgk_update(Y, D, idx, val, idx_p, val_p, 1)
    np.testing.assert_allclose(Dn, _sequential_nsgk(Y, D, idx, val, idx_p, val_p), atol=1e-11)


def test_groups_see_committed_atoms_of_earlier_groups():
    """A sweep in groups equals running the groups one call at a time, each
    call starting from the dictionary the previous one returned (eq. 2) and
    from the same D^(k) in Z: here checked through the two halves of a sweep
    against a dense recomputation of E for the second half."""
    Y, D, idx, val, idx_p, val_p = _two_codings(seed=4)
    n = D.shape[0]
    Dfull, _ = oracle.nsgk_update(Y, D, idx, val, idx_p, val_p, n // 2)
    X = _dense_X(idx, val, n)
    Xp = _dense_X(idx_p, val_p, n)
    Z = Y.T + D.T @ Xp - D.T @ X
    Dh = D.copy()
    for a0 in (0, n // 2):
        E = Z - Dh.T @ Xp           # the group's error with the current D
        new = Dh.copy()
        for j in range(a0, a0 + n // 2):
            I = np.nonzero(Xp[j])[0]
            if I.size == 0:
                continue
            x = Xp[j, I]
            g = (E[:, I] + np.outer(Dh[j], x)) @ x / (x @ x)
            new[j] = g / np.linalg.norm(g)
        Dh = new
    np.testing.assert_allclose(Dfull, Dh, atol=1e-11)


def test_exact_representation_is_a_fixed_point():
    """Y = D X exactly with X^(k-1) = X^(k): Z = Y, F = d_j x_j, nothing moves."""
    rng = np.random.default_rng(6)
    p, n, s, m = 10, 20, 3, 300
    D = _unit_rows(rng.standard_normal((n, p)))
    idx = np.array([rng.choice(n, size=s, replace=False) for _ in range(m)], dtype=np.int32)
    val = rng.standard_normal((m, s))
    Y = np.einsum("ms,msp->mp", val, D[idx])
    for gs in (1, 4, n):
        Dn, _ = oracle.nsgk_update(Y, D, idx, val, idx, val, gs)
        np.testing.assert_allclose(Dn, D, atol=1e-12)


def test_updated_atoms_have_unit_norm_and_unused_keep_their_value():
    Y, D, idx, val, idx_p, val_p = _two_codings(seed=7)
    n = D.shape[0]
    idx_p = idx_p.copy()
    idx_p[idx_p == 5] = -1  # atom 5 unused in X^(k-1) (still used in X^(k))
    Dn, unused = oracle.nsgk_update(Y, D, idx, val, idx_p, val_p, 7)
    assert unused >= 1
    np.testing.assert_array_equal(Dn[5], D[5])
    np.testing.assert_allclose(np.linalg.norm(Dn, axis=1), 1.0, atol=1e-12)


def test_iterate_first_iteration_is_sgk():
    """The first iteration has no earlier representation; it uses its own, so
    its dictionary equals P-SGK's."""
    w = synth.workload("patches_p64_n256_s6_m16384", m=1500)
    Dn, _, _, rn = oracle.iterate(w.Y, w.D0, w.s, 1, w.n, rule=oracle.RULE_NSGK)
    Ds, _, _, rs = oracle.iterate(w.Y, w.D0, w.s, 1, w.n, rule=oracle.RULE_SGK)
    np.testing.assert_allclose(Dn, Ds, atol=1e-12)
    assert abs(rn[0] - rs[0]) < 1e-14


def _recovered(D_true, D):
    C = np.abs(D_true.astype(np.float64) @ D.T)
    return float(np.mean(1.0 - C.max(axis=1) < 0.01)) * 100.0


@pytest.mark.parametrize("s,snr,col", [(3, math.inf, 3), (4, 20, 1)])
def test_full_parallel_nsgk_recovery_matches_table1(s, snr, col):
    """The P-NSGK row of Table 1 (Sec. 4.1), on 6 of the paper's 50 runs."""
    want = GOLDEN["P-NSGK"][str(s)][col]
    got = []
    for run in range(6):
        Y, Dt, _, _ = synth.recovery_problem(20, 50, s, 1500, 0.0, seed=1000 * s + run, snr_db=snr)
        D0 = synth.initial_dictionary(Y, 50, seed=7000 + run)
        D, _, _, _ = oracle.iterate(Y, D0, s, 9 * s * s, 50, rule=oracle.RULE_NSGK)
        got.append(_recovered(Dt, D))
    assert abs(float(np.mean(got)) - want) <= 6.0, (np.mean(got), want)
