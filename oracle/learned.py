"""FP64 oracle for the learned support proposal (test infrastructure only).

The proposal network maps a signal's direction y / ||y|| (p = 64; the OMP
support of y does not depend on its scale) to one logit per atom (n = 256)
through two ReLU hidden layers of 512 units; it is trained with a multi-label
loss (mean binary cross-entropy on the logits, targets = the atoms OMP chose,
positives weighted by pos_weight, e.g. (n - s) / s to balance the s positives
against the n - s negatives) and Adam.  A proposal keeps the 2s atoms with the largest logits; least
squares restricted to them is pruned greedily (backward elimination) to s
atoms; the signal goes back to OMP when the pruned residual exceeds the
reference OMP residual by more than a stated margin.

Plain numpy in float64, one function per step; random draws (initial weights,
minibatch order) are inputs, not drawn here.
"""
from __future__ import annotations

import numpy as np

from .bf16 import round_bf16

SIZES = (64, 512, 512, 256)


# --------------------------------------------------------------- network
def network_input(Y):
    """Rows of Y scaled to unit norm (zero rows stay zero)."""
    Y = np.asarray(Y, np.float64)
    nrm = np.linalg.norm(Y, axis=1, keepdims=True)
    return Y / np.where(nrm > 0, nrm, 1.0)


def forward(params, X, emulate_bf16=False):
    """params = [(W1, b1), (W2, b2), (W3, b3)], W_l of shape [out][in].
    Returns (hidden activations [A0=X, A1, A2], logits Z).  With
    emulate_bf16 the weights, the input and the hidden activations are
    rounded to BF16 where the GPU stores them in BF16."""
    r = (lambda a: round_bf16(np.asarray(a, np.float32)).astype(np.float64)) if emulate_bf16 \
        else (lambda a: np.asarray(a, np.float64))
    A = [r(X)]
    for li, (W, b) in enumerate(params):
        z = A[-1] @ r(W).T + np.asarray(b, np.float64)
        if li < len(params) - 1:
            A.append(r(np.maximum(z, 0.0)))
        else:
            return A, z
    raise AssertionError


def targets(idx, n):
    """Multi-hot targets [B][n] from ELL supports (-1 = empty slot)."""
    T = np.zeros((idx.shape[0], n))
    for i, row in enumerate(idx):
        for j in row:
            if j >= 0:
                T[i, j] = 1.0
    return T


def bce_loss(Z, T, pos_weight=1.0):
    """Mean over all entries of the binary cross-entropy of sigmoid(Z) vs T
    with positives weighted: w t softplus(-z) + (1 - t) softplus(z)."""
    return float(np.mean(pos_weight * T * np.logaddexp(0.0, -Z) + (1 - T) * np.logaddexp(0.0, Z)))


def backward(params, A, Z, T, pos_weight=1.0):
    """Gradients of bce_loss w.r.t. every (W, b), by the chain rule."""
    n_el = Z.size
    sig = 1.0 / (1.0 + np.exp(-Z))
    dZ = (sig * (1 - T) - (1 - sig) * T * pos_weight) / n_el
    grads = [None] * len(params)
    d = dZ
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        grads[li] = (d.T @ A[li], d.sum(axis=0))
        if li > 0:
            d = (d @ np.asarray(W, np.float64)) * (A[li] > 0)
    return grads


def adam_step(params, grads, state, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) on every array; state holds (m, v) per
    array and t is the 1-based step number.  Returns new params and state."""
    new_params, new_state = [], []
    for (W, b), (gW, gb), (mW, vW, mb, vb) in zip(params, grads, state):
        out = []
        for w, g, m, v in ((W, gW, mW, vW), (b, gb, mb, vb)):
            m = b1 * m + (1 - b1) * g
            v = b2 * v + (1 - b2) * g * g
            mh = m / (1 - b1 ** t)
            vh = v / (1 - b2 ** t)
            out.append((w - lr * mh / (np.sqrt(vh) + eps), m, v))
        (Wn, mWn, vWn), (bn, mbn, vbn) = out
        new_params.append((Wn, bn))
        new_state.append((mWn, vWn, mbn, vbn))
    return new_params, new_state


def adam_init(params):
    return [(np.zeros_like(W, dtype=np.float64), np.zeros_like(W, dtype=np.float64),
             np.zeros_like(b, dtype=np.float64), np.zeros_like(b, dtype=np.float64))
            for W, b in params]


# --------------------------------------------------------------- proposal
def top_candidates(Z, k):
    """Indices of the k largest logits per row, largest first; ties go to the
    lower atom index."""
    out = np.empty((Z.shape[0], k), dtype=np.int32)
    cols = np.arange(Z.shape[1])
    for i, z in enumerate(Z):
        order = np.lexsort((cols, -z))  # primary: -z ascending, secondary: index
        out[i] = order[:k]
    return out


def restricted_ls_prune(D, y, cand, s):
    """Least squares of y on the candidate atoms, then backward elimination to
    s atoms: repeatedly drop the atom whose removal raises the residual the
    least (c_j^2 / [(D_C^T D_C)^{-1}]_jj, ties: lower atom index) and refit.
    Returns (support in candidate order, coefficients, residual norm)."""
    D = np.asarray(D, np.float64)
    y = np.asarray(y, np.float64)
    C = [int(j) for j in cand]
    while True:
        A = D[C]
        Gi = np.linalg.inv(A @ A.T)
        c = Gi @ (A @ y)
        if len(C) <= s:
            r = y - A.T @ c
            return np.array(C, dtype=np.int32), c, float(np.linalg.norm(r))
        cost = c * c / np.diag(Gi)
        best = min(range(len(C)), key=lambda q: (cost[q], C[q]))
        C.pop(best)


def needs_fallback(res_norm, ref_norm, margin=0.02):
    """The proposal is rejected when its residual exceeds the reference OMP
    residual by more than the margin (relative)."""
    return res_norm > (1.0 + margin) * ref_norm
