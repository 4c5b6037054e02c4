"""FP64 CPU reference of the near-field surrogate network (test
infrastructure): forward pass and exact gradients of the training loss, written
from the definitions, used to check the GPU training kernels.

Network: y = W3 s(W2 s(W1 x + b1) + b2) + b3, s(z) = z / (1 + exp(-z)) (SiLU),
x in R^18, y in R^2.  Loss over a batch of n samples with targets t:
    L0 = mean (y0 - t)^2
    L1 = mean (y1 - g)^2,  g = (log10(scale |y0 - t| / rho^4 + 1e-12) - mu) / sig
(rho: norm of the mean of features 9..17, the target centroid in the source
frame)
with g treated as a constant (no gradient flows through it); the total loss
is L0 + lam * L1.  Weights are packed W1[H][18] b1[H] W2[H][H] b2[H] W3[2][H]
b3[2].
"""
import numpy as np


def unpack(w, H):
    w = np.asarray(w, dtype=np.float64)
    o = 0
    out = []
    for shape in ((H, 18), (H,), (H, H), (H,), (2, H), (2,)):
        size = int(np.prod(shape))
        out.append(w[o:o + size].reshape(shape))
        o += size
    assert o == len(w)
    return out


def pack(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(w, H, X):
    W1, b1, W2, b2, W3, b3 = unpack(w, H)
    z1 = X @ W1.T + b1
    h1 = silu(z1)
    z2 = h1 @ W2.T + b2
    h2 = silu(z2)
    y = h2 @ W3.T + b3
    return y, (z1, h1, z2, h2)


def rho4(X):
    c = (X[:, 9:12] + X[:, 12:15] + X[:, 15:18]) / 3.0
    r2 = (c ** 2).sum(1)
    return r2 * r2


def loss_and_grad(w, H, X, t, lam, mu, sig, scale):
    X = np.asarray(X, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    n = len(t)
    W1, b1, W2, b2, W3, b3 = unpack(w, H)
    y, (z1, h1, z2, h2) = forward(w, H, X)
    e0 = y[:, 0] - t
    g = (np.log10(scale * np.abs(e0) / rho4(X) + 1e-12) - mu) / sig
    e1 = y[:, 1] - g
    L0 = np.mean(e0 ** 2)
    L1 = np.mean(e1 ** 2)
    dy = np.stack([2 * e0 / n, 2 * lam * e1 / n], 1)
    dW3 = dy.T @ h2
    db3 = dy.sum(0)
    dz2 = (dy @ W3) * dsilu(z2)
    dW2 = dz2.T @ h1
    db2 = dz2.sum(0)
    dz1 = (dz2 @ W2) * dsilu(z1)
    dW1 = dz1.T @ X
    db1 = dz1.sum(0)
    return (L0, L1), pack([dW1, db1, dW2, db2, dW3, db3])


def total_loss(w, H, X, t, lam, mu, sig, scale, g_fixed):
    """L0 + lam * L1 with the calibration target held at g_fixed (for finite
    differences of the gradient, which treats g as a constant)."""
    y, _ = forward(w, H, X)
    return np.mean((y[:, 0] - t) ** 2) + lam * np.mean((y[:, 1] - g_fixed) ** 2)
