"""FP64 oracle of the learned block preconditioner's network (test
infrastructure: only tests/, the smoke check and the CPU baseline use it).

The network maps the normalised diagonal block A^ = A / s (s = max |A_ij|),
given as vec() of the column-major b x b matrix, to M ~ A^^-1 (same layout):

    h1 = relu(W1 x + b1),  h2 = relu(W2 h1 + b2),  y = W3 h2 + b3,

and is trained on L = (1/B) sum_n ||A^_n M_n - I||_F^2.  The paper defines the
Jacobian blocks (eq. "jacobian_rhs") but no learned preconditioner: this is
the plain definition of the network and loss used by the library, written
with numpy matmuls in float64, and its gradient by reverse-mode chain rule.
Pinned by central finite differences (tests/test_oracle_mlp.py).

Parameter vector: [W1 (H x b^2), b1 (H), W2 (H x H), b2 (H), W3 (b^2 x H), b3 (b^2)].
"""
from __future__ import annotations

import numpy as np


def n_params(b: int, H: int) -> int:
    n = b * b
    return H * n + H + H * H + H + n * H + n


def unpack(p, b: int, H: int):
    n = b * b
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + H * n].reshape(H, n); o += H * n
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + n * H].reshape(n, H); o += n * H
    b3 = p[o:o + n]; o += n
    assert o == p.size
    return W1, b1, W2, b2, W3, b3


def mat(v, b: int):
    """vec() of a column-major b x b matrix -> the matrix."""
    return np.asarray(v, dtype=np.float64).reshape(b, b).T


def forward(p, X, b: int, H: int):
    """Network outputs Y [B][b^2] for inputs X [B][b^2] (float64)."""
    W1, b1, W2, b2, W3, b3 = unpack(p, b, H)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.maximum(X @ W1.T + b1, 0.0)
    h2 = np.maximum(h1 @ W2.T + b2, 0.0)
    return h2 @ W3.T + b3


def residual_norms(X, Y, b: int):
    """||A^_n M_n - I||_F for each sample."""
    out = np.empty(len(X))
    for i in range(len(X)):
        E = mat(X[i], b) @ mat(Y[i], b) - np.eye(b)
        out[i] = np.sqrt(np.sum(E * E))
    return out


def loss_grad(p, X, b: int, H: int):
    """L = (1/B) sum_n ||A^_n M_n - I||_F^2 and dL/dp (flat, float64)."""
    W1, b1, W2, b2, W3, b3 = unpack(p, b, H)
    X = np.asarray(X, dtype=np.float64)
    B = len(X)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    Y = h2 @ W3.T + b3
    L = 0.0
    dY = np.empty_like(Y)
    for i in range(B):
        A = mat(X[i], b)
        E = A @ mat(Y[i], b) - np.eye(b)
        L += np.sum(E * E)
        dM = (2.0 / B) * (A.T @ E)            # dL/dM_n
        dY[i] = dM.T.reshape(-1)               # back to column-major vec()
    L /= B
    gW3 = dY.T @ h2
    gb3 = dY.sum(axis=0)
    dz2 = (dY @ W3) * (z2 > 0)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return L, g


def loss(p, X, b: int, H: int) -> float:
    Y = forward(p, X, b, H)
    r = residual_norms(X, Y, b)
    return float(np.mean(r * r))
