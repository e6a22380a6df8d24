"""FP64 reference of the learned-shift MLP (test infrastructure only: used by
the tests to check the HIP forward, gradient and in-solver inference; never
called by the library).

Network and loss as declared with dashsvd_mlp_init: x (D) -> relu(W1 x + b1)
-> relu(W2 . + b2) -> W3 . + b3 = o (2); c = 1/2 + (c_max - 1/2) sigmoid(o_0);
L = mean_b [(c_b - c*_b)^2 + lambda (o_1,b - log N*_b)^2], lambda = 0.1.
Parameters are one vector: W1 (H x D), b1, W2 (H x H), b2, W3 (2 x H), b3.
The learned shift is our design (the paper's shift rule is fixed), so this
reference is pinned by finite differences of its own loss in the tests."""
import numpy as np

LAMBDA = 0.1


def unpack(P, D, H):
    P = np.asarray(P, dtype=np.float64)
    o = 0
    W1 = P[o:o + H * D].reshape(H, D); o += H * D
    b1 = P[o:o + H]; o += H
    W2 = P[o:o + H * H].reshape(H, H); o += H * H
    b2 = P[o:o + H]; o += H
    W3 = P[o:o + 2 * H].reshape(2, H); o += 2 * H
    b3 = P[o:o + 2]; o += 2
    assert o == P.shape[0]
    return W1, b1, W2, b2, W3, b3


def forward(P, X, D, H):
    W1, b1, W2, b2, W3, b3 = unpack(P, D, H)
    X = np.asarray(X, dtype=np.float64)
    a1 = np.maximum(X @ W1.T + b1, 0.0)
    a2 = np.maximum(a1 @ W2.T + b2, 0.0)
    return a1, a2, a2 @ W3.T + b3


def outputs(P, X, D, H, c_max):
    o = forward(P, X, D, H)[2]
    c = 0.5 + (c_max - 0.5) / (1.0 + np.exp(-o[:, 0]))
    return np.stack([c, o[:, 1]], axis=1)


def loss(P, X, Y, D, H, c_max):
    o = forward(P, X, D, H)[2]
    c = 0.5 + (c_max - 0.5) / (1.0 + np.exp(-o[:, 0]))
    Y = np.asarray(Y, dtype=np.float64)
    return float(np.mean((c - Y[:, 0]) ** 2 + LAMBDA * (o[:, 1] - Y[:, 1]) ** 2))


def grad(P, X, Y, D, H, c_max):
    """Analytic gradient of loss() (chain rule through the three layers)."""
    W1, b1, W2, b2, W3, b3 = unpack(P, D, H)
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    B = X.shape[0]
    a1, a2, o = forward(P, X, D, H)
    sg = 1.0 / (1.0 + np.exp(-o[:, 0]))
    c = 0.5 + (c_max - 0.5) * sg
    do = np.zeros_like(o)
    do[:, 0] = 2.0 * (c - Y[:, 0]) * (c_max - 0.5) * sg * (1.0 - sg) / B
    do[:, 1] = 2.0 * LAMBDA * (o[:, 1] - Y[:, 1]) / B
    gW3 = do.T @ a2
    gb3 = do.sum(axis=0)
    da2 = (do @ W3) * (a2 > 0)
    gW2 = da2.T @ a1
    gb2 = da2.sum(axis=0)
    da1 = (da2 @ W2) * (a1 > 0)
    gW1 = da1.T @ X
    gb1 = da1.sum(axis=0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
