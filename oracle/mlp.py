"""Float64 two-layer MLP used to check the learned PP controller (test oracle).

The paper's PP-CP-ALS leaves the PP phase with a fixed threshold on
||dA^(i)|| / ||A^(i)|| (Algorithm 3) and names other switching schemes as future work
(Section 6).  The controller regresses the relative error of the PP right-hand side
on the per-mode relative changes, the sweep index and the fit; this module is the
plain float64 reference of that network, its loss, its gradients and its optimiser.

Network (d inputs, H hidden units, one output):
    h = tanh(W1 x + b1),  y = W2 . h + b2
Loss over a batch of B samples with targets t:
    L = (1/B) sum_b (y_b - t_b)^2
Optimiser: Adam (Kingma & Ba, 2015) with bias correction,
    m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
    p <- p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Flat parameter layout (shared with the device kernels through the C ABI, not
through code): [W1 (H x d, row-major), b1 (H), W2 (H), b2 (1)].

Features of a PP iterate (all float64): log10(rho_i + 1e-12) for each mode i,
log1p(sweep index), -log10(1 - fit + 1e-16).  Label: log10 of
max_n ||M~^(n) - M^(n)||_F / ||M^(n)||_F at the same iterate.
"""
from __future__ import annotations

import numpy as np


def n_params(d, H):
    return H * d + 2 * H + 1


def unpack(p, d, H):
    p = np.asarray(p, dtype=np.float64)
    W1 = p[: H * d].reshape(H, d)
    b1 = p[H * d: H * d + H]
    W2 = p[H * d + H: H * d + 2 * H]
    b2 = p[H * d + 2 * H]
    return W1, b1, W2, b2


def pack(W1, b1, W2, b2):
    return np.concatenate([np.ravel(W1), np.ravel(b1), np.ravel(W2), np.atleast_1d(b2)]).astype(np.float64)


def forward(p, X, d, H):
    """Returns (y, h) for inputs X of shape B x d."""
    W1, b1, W2, b2 = unpack(p, d, H)
    X = np.asarray(X, dtype=np.float64)
    h = np.tanh(X @ W1.T + b1)
    y = h @ W2 + b2
    return y, h


def loss(p, X, t, d, H):
    y, _ = forward(p, X, d, H)
    r = y - np.asarray(t, dtype=np.float64)
    return float(np.mean(r * r))


def loss_and_grad(p, X, t, d, H):
    """MSE loss and its gradient with respect to the flat parameters (chain rule
    through the output layer and tanh, whose derivative is 1 - h^2)."""
    W1, b1, W2, b2 = unpack(p, d, H)
    X = np.asarray(X, dtype=np.float64)
    y, h = forward(p, X, d, H)
    B = X.shape[0]
    r = y - np.asarray(t, dtype=np.float64)
    L = float(np.mean(r * r))
    dy = 2.0 * r / B                      # dL/dy_b
    gW2 = h.T @ dy                        # sum_b dy_b h_bj
    gb2 = float(np.sum(dy))
    dz = np.outer(dy, W2) * (1.0 - h * h)  # dL/d(pre-activation)
    gW1 = dz.T @ X
    gb1 = np.sum(dz, axis=0)
    return L, pack(gW1, gb1, gW2, gb2)


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1).  Returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    p = p - lr * mhat / (np.sqrt(vhat) + eps)
    return p, m, v


def features(rel_change, sweep, fit):
    """Controller input for one PP iterate."""
    rc = [np.log10(float(r) + 1e-12) for r in rel_change]
    return np.array(rc + [np.log1p(float(sweep)), -np.log10(1.0 - float(fit) + 1e-16)])


def label(Mt, M):
    """log10 of the largest relative right-hand-side error over the modes."""
    e = max(np.linalg.norm(a - b) / np.linalg.norm(b) for a, b in zip(Mt, M))
    return float(np.log10(e))
