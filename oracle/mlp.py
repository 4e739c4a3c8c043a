"""Oracle of the learned bound / mu predictor: a two-layer perceptron, its
loss gradient and the Adam update, in plain NumPy float64.

TEST INFRASTRUCTURE (see the package header).

The predictor itself is not part of the paper.  It serves the paper's remark
that a good initial guess of the eigenvalue bounds avoids recomputing the
polynomials after a failed penalty check (Sec. "Determination of the
eigenvalue bounds and polynomial degree") and that a good bound guess saves
the expensive bound search (Sec. "Scaling with spectral properties").

Network (sizes N_IN -> N_HID -> N_OUT):
    h = tanh(W1 x + b1),   y = W2 h + b2
Loss over a batch of B rows (targets t):
    L = 1 / (2 B) * sum_b sum_o (y_bo - t_bo)^2
Flat parameter layout (row-major): W1 [N_HID][N_IN], b1 [N_HID],
W2 [N_OUT][N_HID], b2 [N_OUT].
Adam (Kingma and Ba, 2015) with bias correction, step t = 1, 2, ...:
    m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
    p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)

Pins: tests/test_oracle_mlp.py (central differences, closed forms of special
parameter values, the first Adam step).
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT = 64, 128, 3


def n_params(n_in: int = N_IN, n_hid: int = N_HID, n_out: int = N_OUT) -> int:
    return n_hid * n_in + n_hid + n_out * n_hid + n_out


def unpack(p: np.ndarray, n_in: int = N_IN, n_hid: int = N_HID, n_out: int = N_OUT):
    o = 0
    W1 = p[o:o + n_hid * n_in].reshape(n_hid, n_in)
    o += n_hid * n_in
    b1 = p[o:o + n_hid]
    o += n_hid
    W2 = p[o:o + n_out * n_hid].reshape(n_out, n_hid)
    o += n_out * n_hid
    b2 = p[o:o + n_out]
    return W1, b1, W2, b2


def forward(p, X, n_in=N_IN, n_hid=N_HID, n_out=N_OUT):
    """Returns (hidden activations [B, n_hid], outputs [B, n_out])."""
    W1, b1, W2, b2 = unpack(np.asarray(p, dtype=np.float64), n_in, n_hid, n_out)
    X = np.asarray(X, dtype=np.float64)
    Hh = np.tanh(X @ W1.T + b1)
    return Hh, Hh @ W2.T + b2


def loss(p, X, T, **kw):
    _, Y = forward(p, X, **kw)
    return 0.5 * np.sum((Y - T) ** 2) / X.shape[0]


def loss_grad(p, X, T, n_in=N_IN, n_hid=N_HID, n_out=N_OUT):
    """Gradient of `loss` by the chain rule, flat in the parameter layout."""
    W1, b1, W2, b2 = unpack(np.asarray(p, dtype=np.float64), n_in, n_hid, n_out)
    X = np.asarray(X, dtype=np.float64)
    B = X.shape[0]
    Hh, Y = forward(p, X, n_in, n_hid, n_out)
    dY = (Y - T) / B                      # dL/dy
    gW2 = dY.T @ Hh                       # [n_out, n_hid]
    gb2 = dY.sum(axis=0)
    dH = (dY @ W2) * (1.0 - Hh * Hh)      # through tanh
    gW1 = dH.T @ X                        # [n_hid, n_in]
    gb1 = dH.sum(axis=0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2])


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (returns new p, m, v; inputs are not modified)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
