"""Pins of the oracle's Jacobi atom update (the group loop of Alg. 2 with the
AK-SVD rule of eq. (5)) and of its error, against facts that come from the
paper and from the mathematics rather than from the oracle's own code.
"""
import numpy as np
import pytest

import oracle
from paper_1509_05054_amd import synth


def _unit_rows(A):
    return A / np.linalg.norm(A, axis=1, keepdims=True)


def _problem(p=12, n=24, s=3, m=400, seed=0):
    rng = np.random.default_rng(seed)
    D = _unit_rows(rng.standard_normal((n, p)))
    Y = rng.standard_normal((m, p))
    idx, val, _ = oracle.omp(D, Y, s)
    return Y, D, idx, val


def _dense_X(idx, val, n):
    m, s = idx.shape
    X = np.zeros((n, m))
    for i in range(m):
        for t in range(s):
            if idx[i, t] >= 0:
                X[idx[i, t], i] = val[i, t]
    return X


def test_full_jacobi_matches_closed_form():
    """At group size n every atom sees the same E, so g_j = (E X^T)_j + d_j (X X^T)_jj,
    i.e. D'^T = colnormalize(Y^T X^T - D^T (X X^T - Diag(X X^T))) (eqs. 3 and 5),
    and x'_ji = f_i^T d'_j with f_i = y_i - sum_{k != j} d_k x_ki."""
    Y, D, idx, val = _problem(seed=1)
    n = D.shape[0]
    X = _dense_X(idx, val, n)  # n x m
    XXt = X @ X.T
    G = X @ Y - (XXt - np.diag(np.diag(XXt))) @ D  # rows = unnormalised atoms
    used = np.abs(X).sum(axis=1) > 0
    Dcf = D.copy()
    Dcf[used] = G[used] / np.linalg.norm(G[used], axis=1, keepdims=True)
    Dn, valn, unused = oracle.jau_update(Y, D, idx, val, group_size=n)
    assert unused == int((~used).sum())
    np.testing.assert_allclose(Dn, Dcf, rtol=0, atol=1e-12)
    m, s = idx.shape
    for i in range(m):
        for t in range(s):
            j = idx[i, t]
            f = Y[i] - sum(D[idx[i, u]] * val[i, u] for u in range(s) if u != t)
            assert abs(valn[i, t] - f @ Dcf[j]) < 1e-12


def test_full_jacobi_aksvd_atoms_equal_sgk_atoms():
    """At full parallelism the AK-SVD and SGK atoms have the same direction (Sec. 3)."""
    Y, D, idx, val = _problem(seed=2)
    n = D.shape[0]
    Da, va, _ = oracle.jau_update(Y, D, idx, val, n, rule=oracle.RULE_AKSVD)
    Ds, vs, _ = oracle.jau_update(Y, D, idx, val, n, rule=oracle.RULE_SGK)
    np.testing.assert_allclose(Da, Ds, atol=1e-12)
    np.testing.assert_array_equal(vs, val)  # SGK leaves X alone


def _sequential_aksvd(Y, D, idx, val):
    """Gauss-Seidel AK-SVD written independently: keeps E up to date after each
    atom instead of recomputing it, and finds users through a dense X."""
    D = D.copy()
    n = D.shape[0]
    X = _dense_X(idx, val, n)
    E = Y.T - D.T @ X  # p x m
    for j in range(n):
        I = np.nonzero(X[j])[0]
        if I.size == 0:
            continue
        F = E[:, I] + np.outer(D[j], X[j, I])
        g = F @ X[j, I]
        if np.linalg.norm(g) == 0:
            continue
        d = g / np.linalg.norm(g)
        x = F.T @ d
        E[:, I] = F - np.outer(d, x)
        D[j] = d
        X[j, I] = x
    valn = val.copy()
    m, s = idx.shape
    for i in range(m):
        for t in range(s):
            if idx[i, t] >= 0:
                valn[i, t] = X[idx[i, t], i]
    return D, valn


def test_group_size_one_is_sequential_aksvd():
    """Group size 1 is the usual sequential (Gauss-Seidel) form (Sec. 2)."""
    Y, D, idx, val = _problem(seed=3)
    Dn, vn, _ = oracle.jau_update(Y, D, idx, val, group_size=1)
    Ds, vs = _sequential_aksvd(Y, D, idx, val)
    np.testing.assert_allclose(Dn, Ds, atol=1e-11)
    np.testing.assert_allclose(vn, vs, atol=1e-11)


@pytest.mark.parametrize("gs", [1, 5, 7, 24])
def test_updated_atoms_have_unit_norm(gs):
    Y, D, idx, val = _problem(seed=4)
    Dn, _, _ = oracle.jau_update(Y, D, idx, val, group_size=gs)
    np.testing.assert_allclose(np.linalg.norm(Dn, axis=1), 1.0, atol=1e-12)


def test_single_atom_update_never_increases_error():
    """With X fixed, d' = F x^T / ||F x^T|| minimises ||F - d x^T|| over unit d,
    then x' = F^T d' minimises over x: one atom's update cannot raise ||E||_F."""
    Y, D, idx, val = _problem(seed=5)
    n = D.shape[0]
    for j in range(n):
        before = oracle.rmse(Y, D, idx, val)
        Dn, vn, _ = oracle.jau_update(Y, D, idx, val, group_size=1, atoms=(j, j + 1))
        after = oracle.rmse(Y, Dn, idx, vn)
        assert after <= before + 1e-14
        D, val = Dn, vn


def test_exact_representation_is_a_fixed_point():
    """If Y = D X exactly, F = d_j x_j, so g = d_j ||x_j||^2 and nothing moves."""
    rng = np.random.default_rng(6)
    p, n, s, m = 10, 20, 3, 300
    D = _unit_rows(rng.standard_normal((n, p)))
    idx = np.array([rng.choice(n, size=s, replace=False) for _ in range(m)], dtype=np.int32)
    val = rng.standard_normal((m, s))
    Y = np.einsum("ms,msp->mp", val, D[idx])
    for gs in (1, 4, n):
        Dn, vn, _ = oracle.jau_update(Y, D, idx, val, group_size=gs)
        np.testing.assert_allclose(Dn, D, atol=1e-12)
        np.testing.assert_allclose(vn, val, atol=1e-12)


def test_single_user_atom_closed_form():
    """I_j = {i}: d' = sign(x) f/||f||, x' = sign(x) ||f|| with f = e_i + d_j x_ji."""
    rng = np.random.default_rng(8)
    p, n, s, m = 8, 6, 2, 5
    D = _unit_rows(rng.standard_normal((n, p)))
    Y = rng.standard_normal((m, p))
    idx = np.array([[0, 1], [0, 2], [1, 2], [3, 4], [0, 5]], dtype=np.int32)  # atom 3 -> signal 3 only
    val = rng.standard_normal((m, s))
    val[3, 0] = -0.7
    Dn, vn, _ = oracle.jau_update(Y, D, idx, val, group_size=n)
    f = Y[3] - D[4] * val[3, 1]
    sgn = np.sign(val[3, 0])
    np.testing.assert_allclose(Dn[3], sgn * f / np.linalg.norm(f), atol=1e-13)
    assert abs(vn[3, 0] - sgn * np.linalg.norm(f)) < 1e-12


def test_unused_atom_unchanged():
    rng = np.random.default_rng(9)
    p, n, s, m = 8, 10, 2, 50
    D = _unit_rows(rng.standard_normal((n, p)))
    Y = rng.standard_normal((m, p))
    idx = rng.integers(0, n - 1, size=(m, s)).astype(np.int32)  # atom n-1 never used
    idx[:, 1] = np.where(idx[:, 1] == idx[:, 0], (idx[:, 0] + 1) % (n - 1), idx[:, 1])
    val = rng.standard_normal((m, s))
    Dn, _, unused = oracle.jau_update(Y, D, idx, val, group_size=3)
    assert unused >= 1
    np.testing.assert_array_equal(Dn[n - 1], D[n - 1])


def test_full_jacobi_permutation_equivariance():
    Y, D, idx, val = _problem(seed=10)
    n = D.shape[0]
    perm = np.random.default_rng(10).permutation(n)  # new label of old atom j is inv[j]
    inv = np.argsort(perm)
    Dp = D[perm]
    idxp = np.where(idx >= 0, inv[np.maximum(idx, 0)], -1).astype(np.int32)
    Dn, vn, _ = oracle.jau_update(Y, D, idx, val, n)
    Dpn, vpn, _ = oracle.jau_update(Y, Dp, idxp, val, n)
    np.testing.assert_allclose(Dpn, Dn[perm], atol=1e-12)
    np.testing.assert_allclose(vpn, vn, atol=1e-12)


def test_padding_slots_are_ignored():
    """Slots with index -1 carry no atom: adding them changes nothing."""
    Y, D, idx, val = _problem(s=2, seed=11)
    m = idx.shape[0]
    idx3 = np.hstack([idx, -np.ones((m, 1), dtype=np.int32)])
    val3 = np.hstack([val, np.zeros((m, 1))])
    Dn, vn, _ = oracle.jau_update(Y, D, idx, val, 5)
    Dn3, vn3, _ = oracle.jau_update(Y, D, idx3, val3, 5)
    np.testing.assert_allclose(Dn3, Dn, atol=0)
    np.testing.assert_allclose(vn3[:, :2], vn, atol=0)
    assert (vn3[:, 2] == 0).all()


def test_rmse_is_frobenius_norm():
    Y, D, idx, val = _problem(seed=12)
    X = _dense_X(idx, val, D.shape[0])
    E = Y.T - D.T @ X
    want = np.linalg.norm(E) / np.sqrt(E.size)
    assert abs(oracle.rmse(Y, D, idx, val) - want) < 1e-14
    np.testing.assert_allclose(oracle.residual(Y, D, idx, val), E.T, atol=1e-13)


def test_iterate_decreases_error_on_patches():
    """A short DL run on synthetic patches: the error after 5 iterations is
    below the first iteration's (the paper's curves descend, Sec. 4.2)."""
    w = synth.workload("patches_p64_n256_s6_m16384", m=2048)
    D, idx, val, r = oracle.iterate(w.Y, w.D0, w.s, 5, group_size=w.n)
    assert r[-1] < r[0]
    np.testing.assert_allclose(np.linalg.norm(D, axis=1), 1.0, atol=1e-12)
    assert abs(r[-1] - oracle.rmse(w.Y, D, idx, val)) < 1e-15
