"""FP64 reference of the learned support proposal (test infrastructure only).

Network (same flat parameter layout as the library): x = vec(Y)/||Y||_F;
h1 = gelu(W1 x + b1); h2 = gelu(W2 h1 + b2); z = W3 h2 + b3 (one logit per atom);
loss = mean over batch and atoms of the sigmoid cross-entropy with the multi-hot
support label, in its stable form max(z,0) - z*y + log(1 + exp(-|z|)).
gelu is the exact form z * Phi(z).  Proposal: the s largest logits (ties: smallest
index), least squares on them.

Pinned by tests/test_oracle_mlp.py: central finite differences of the loss, the closed
form sigmoid(z) - y of the logit gradient, and least squares against numpy lstsq.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SQRT2 = math.sqrt(2.0)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / SQRT2))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / SQRT2)) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def layout(M, H, A):
    """Offsets of W1 (H x M), b1, W2 (H x H), b2, W3 (A x H), b3 in the flat vector."""
    sizes = [H * M, H, H * H, H, A * H, A]
    off = np.cumsum([0] + sizes)
    return off, int(off[-1])


def unpack(params, M, H, A):
    off, n = layout(M, H, A)
    assert params.size == n
    p = np.asarray(params, np.float64)
    W1 = p[off[0]:off[1]].reshape(H, M)
    b1 = p[off[1]:off[2]]
    W2 = p[off[2]:off[3]].reshape(H, H)
    b2 = p[off[3]:off[4]]
    W3 = p[off[4]:off[5]].reshape(A, H)
    b3 = p[off[5]:off[6]]
    return W1, b1, W2, b2, W3, b3


def inputs(Y):
    """Y (N, m1, m2) math shape -> x (N, m1*m2) = column-major vec(Y)/||Y||_F."""
    v = np.stack([y.flatten("F") for y in np.asarray(Y, np.float64)])
    n = np.linalg.norm(v, axis=1, keepdims=True)
    return np.where(n > 0, v / np.where(n > 0, n, 1.0), 0.0)


def labels(supp, A):
    N = supp.shape[0]
    y = np.zeros((N, A))
    for k in range(N):
        for a in supp[k]:
            if a >= 0:
                y[k, a] = 1.0
    return y


def forward(params, x, M, H, A):
    W1, b1, W2, b2, W3, b3 = unpack(params, M, H, A)
    z1 = x @ W1.T + b1
    h1 = gelu(z1)
    z2 = h1 @ W2.T + b2
    h2 = gelu(z2)
    z3 = h2 @ W3.T + b3
    return z3, (x, z1, h1, z2, h2)


def loss_and_grad(params, x, y, M, H, A):
    """Mean BCE-with-logits loss and its gradient w.r.t. the flat parameters."""
    W1, b1, W2, b2, W3, b3 = unpack(params, M, H, A)
    z3, (x, z1, h1, z2, h2) = forward(params, x, M, H, A)
    B = x.shape[0]
    loss = np.mean(np.maximum(z3, 0) - z3 * y + np.log1p(np.exp(-np.abs(z3))))
    dz3 = (1.0 / (1.0 + np.exp(-z3)) - y) / (B * A)
    gW3 = dz3.T @ h2
    gb3 = dz3.sum(0)
    dz2 = (dz3 @ W3) * gelu_grad(z2)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2) * gelu_grad(z1)
    gW1 = dz1.T @ x
    gb1 = dz1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return float(loss), g


def top_s(z, s):
    """Indices of the s largest entries of each row, in decreasing order (ties: smallest index)."""
    return np.argsort(-z, axis=1, kind="stable")[:, :s]


def least_squares_on_support(Y, d1, d2, supp):
    """Coefficients and squared residual of LS on the given atoms (explicit Kronecker columns)."""
    K = np.kron(d2, d1)
    N = len(Y)
    coef = np.zeros(supp.shape)
    res2 = np.zeros(N)
    for k in range(N):
        yv = np.asarray(Y[k], np.float64).flatten("F")
        S = list(supp[k])
        x, *_ = np.linalg.lstsq(K[:, S], yv, rcond=None)
        coef[k] = x
        res2[k] = float(np.sum((yv - K[:, S] @ x) ** 2))
    return coef, res2
