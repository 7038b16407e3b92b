"""Pins of the FP64 network oracle (CPU): gradients against central finite
differences, the loss against its definition at a known exact inverse, and
the layout convention of vec() against numpy's column-major order."""
import numpy as np

from oracle import mlp as OM


def _case(b=4, H=6, B=3, seed=0):
    rng = np.random.default_rng(seed)
    p = rng.normal(size=OM.n_params(b, H)) * 0.4
    A = rng.normal(size=(B, b, b)) + 2.0 * np.eye(b)
    A /= np.max(np.abs(A), axis=(1, 2), keepdims=True)
    X = np.stack([a.T.reshape(-1) for a in A])        # column-major vec()
    return p, X, b, H


def test_vec_is_column_major():
    A = np.arange(9.0).reshape(3, 3)
    assert np.array_equal(OM.mat(A.reshape(-1, order="F"), 3), A)


def test_gradient_matches_central_differences():
    p, X, b, H = _case()
    L, g = OM.loss_grad(p, X, b, H)
    assert abs(L - OM.loss(p, X, b, H)) <= 1e-12 * abs(L)
    h = 1e-6
    rng = np.random.default_rng(1)
    idx = rng.choice(p.size, 60, replace=False)
    for i in idx:
        e = np.zeros_like(p); e[i] = h
        fd = (OM.loss(p + e, X, b, H) - OM.loss(p - e, X, b, H)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_exact_inverse_in_the_output_bias_gives_zero_loss():
    """With W3 = 0 the network outputs b3; b3 = vec(A^-1) is a stationary
    point of zero loss for a single sample."""
    p, X, b, H = _case(B=1)
    W1, b1, W2, b2, W3, b3 = OM.unpack(p, b, H)
    q = p.copy()
    n = b * b
    o3 = q.size - n - n * H
    q[o3:o3 + n * H] = 0.0
    q[-n:] = np.linalg.inv(OM.mat(X[0], b)).T.reshape(-1)
    L, g = OM.loss_grad(q, X, b, H)
    assert L <= 1e-26 and np.max(np.abs(g)) <= 1e-12


def test_relu_inactive_layer_has_zero_gradient():
    """Biases driving every hidden unit negative switch the hidden layers off:
    only the output bias then carries gradient."""
    p, X, b, H = _case()
    W1, b1, W2, b2, W3, b3 = OM.unpack(p, b, H)
    q = p.copy()
    n = b * b
    q[H * n:H * n + H] = -1e3                          # b1
    q[H * n + H + H * H:H * n + 2 * H + H * H] = -1e3  # b2
    L, g = OM.loss_grad(q, X, b, H)
    assert np.all(g[:H * n + H + H * H + H + n * H] == 0.0)
    assert np.max(np.abs(g[-n:])) > 0.0
