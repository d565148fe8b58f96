"""Learned proposal network, FP64 reference.

Test infrastructure only.

A multilayer perceptron maps the normalised voxel signature x = Z_v/||Z_v||
(interleaved re/im for complex dictionaries, the real part for real ones)
to standardised parameters u_p = (f_p(theta_p) - mean_p)/std_p with f_p = ln
for positive parameters spanning a wide range (T1, T2) and identity
otherwise (df, B1):
    a1 = W1 x + b1, h1 = gelu(a1); a2 = W2 h1 + b2, h2 = gelu(a2); y = W3 h2 + b3
with gelu(a) = a Phi(a) = a (1 + erf(a / sqrt 2)) / 2 (exact form), weights
stored [out][in].  Loss: mean over batch and outputs of (y - u)^2.  Adam
(Kingma and Ba, 2015): m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
w <- w - lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).

The network is an extension beyond the paper (which compares cover-tree and
KD-tree searches): its proposal only seeds an exact local matched filter,
and the exhaustive filter remains the fallback.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def gelu(a):
    return 0.5 * a * (1.0 + erf(a / math.sqrt(2.0)))


def gelu_grad(a):
    return 0.5 * (1.0 + erf(a / math.sqrt(2.0))) + a * np.exp(-0.5 * a * a) / math.sqrt(2.0 * math.pi)


def forward(params, X):
    """params: dict W1 [H][I], b1 [H], W2 [H][H], b2, W3 [P][H], b3 [P];
    X: [B][I].  Returns y [B][P] and the cache for backward."""
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ params["W1"].T + params["b1"]
    h1 = gelu(a1)
    a2 = h1 @ params["W2"].T + params["b2"]
    h2 = gelu(a2)
    y = h2 @ params["W3"].T + params["b3"]
    return y, (X, a1, h1, a2, h2)


def forward_bf16(params, X, round_hidden=True):
    """Inference form with BF16 operands: X, W1 and W2 rounded to the nearest
    BF16 (ties to even); a BF16 x BF16 product is exact, sums are taken in
    FP64 here; h1 is rounded to BF16 after its GELU (round_hidden), h2 and
    the output layer stay in full precision (W3, b1, b2, b3 unrounded)."""
    from oracle.quant import bf16_round
    r = lambda a: bf16_round(np.asarray(a, dtype=np.float32)).astype(np.float64)
    a1 = r(X) @ r(params["W1"]).T + params["b1"]
    h1 = gelu(a1)
    if round_hidden:
        h1 = r(h1)
    a2 = h1 @ r(params["W2"]).T + params["b2"]
    h2 = gelu(a2)
    return h2 @ np.asarray(params["W3"], dtype=np.float64).T + params["b3"]


def loss_and_grads(params, X, T):
    """MSE loss (mean over B*P) and its gradients w.r.t. every parameter."""
    y, (X, a1, h1, a2, h2) = forward(params, X)
    T = np.asarray(T, dtype=np.float64)
    B, P = y.shape
    r = y - T
    loss = float(np.sum(r * r) / (B * P))
    dy = 2.0 * r / (B * P)
    g = {}
    g["W3"] = dy.T @ h2
    g["b3"] = dy.sum(axis=0)
    dh2 = dy @ params["W3"]
    da2 = dh2 * gelu_grad(a2)
    g["W2"] = da2.T @ h1
    g["b2"] = da2.sum(axis=0)
    dh1 = da2 @ params["W2"]
    da1 = dh1 * gelu_grad(a1)
    g["W1"] = da1.T @ X
    g["b1"] = da1.sum(axis=0)
    return loss, g


NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def adam_step(params, grads, state, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t >= 1; state holds m and v per parameter."""
    out = {}
    for k in NAMES:
        m = b1 * state["m"][k] + (1.0 - b1) * grads[k]
        v = b2 * state["v"][k] + (1.0 - b2) * grads[k] ** 2
        state["m"][k], state["v"][k] = m, v
        mh = m / (1.0 - b1 ** t)
        vh = v / (1.0 - b2 ** t)
        out[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
    return out


def standardise(params_table, log_mask):
    """Per-parameter transform f_p and its mean/std over the table rows."""
    f = np.where(np.asarray(log_mask)[None, :], np.log(np.maximum(params_table, 1e-300)), params_table)
    mean = f.mean(axis=0)
    std = f.std(axis=0)
    std = np.where(std > 0, std, 1.0)
    return (f - mean) / std, mean, std


def nearest_cells(u, mean, std, log_mask, axes):
    """Proposal -> nearest grid index per parameter, the distance measured in
    the transformed space (ties to the lower index)."""
    u = np.asarray(u, dtype=np.float64)
    cells = np.zeros(u.shape, dtype=np.int64)
    for p, ax in enumerate(axes):
        val = u[:, p] * std[p] + mean[p]
        fa = np.log(ax) if log_mask[p] else np.asarray(ax, dtype=np.float64)
        dist = np.abs(val[:, None] - fa[None, :])
        cells[:, p] = np.argmin(dist, axis=1)
    return cells
