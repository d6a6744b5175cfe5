"""FP64 NumPy oracle of the learned demapper network — TEST INFRASTRUCTURE ONLY.

Network: features (y_1..y_D, (SNR_dB - 7.5)/7.5) -> Linear(D+1, H) -> GELU -> Linear(H, H)
-> GELU -> Linear(H, m), the m outputs being LLR estimates in nats.  GELU is the tanh form
0.5 x (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3))).  The training loss is the soft binary
cross-entropy between sigma(output) and the exact bit posterior sigma(lambda_exact),
averaged over samples and bits: softplus(o) - sigma(lambda) o (+ a term without o).
The optimiser is Adam (beta1 0.9, beta2 0.999, eps 1e-8) on FP32 master weights.

Weights are given as a dict of float64 arrays: W1 (D+1, H), b1 (H), W2 (H, H), b2 (H),
W3 (H, m), b3 (m) — row-major, y = x @ W + b.  Pure NumPy, written for reading.
"""
from __future__ import annotations

import math

import numpy as np

GELU_C = math.sqrt(2.0 / math.pi)
GELU_A = 0.044715
SNR_CENTER = 7.5
SNR_SCALE = 7.5


def features(y, snr_db):
    """Network input: the received coordinates and the normalised SNR in dB."""
    y = np.asarray(y, dtype=np.float64)
    s = np.broadcast_to(np.asarray(snr_db, dtype=np.float64), (y.shape[0],))
    return np.concatenate([y, ((s - SNR_CENTER) / SNR_SCALE)[:, None]], axis=1)


def gelu(x):
    return 0.5 * x * (1.0 + np.tanh(GELU_C * (x + GELU_A * x ** 3)))


def gelu_grad(x):
    u = GELU_C * (x + GELU_A * x ** 3)
    t = np.tanh(u)
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * GELU_C * (1.0 + 3.0 * GELU_A * x * x)


def forward(w, X):
    """Returns (outputs, cache) for inputs X (B, D+1)."""
    h1 = X @ w["W1"] + w["b1"]
    a1 = gelu(h1)
    h2 = a1 @ w["W2"] + w["b2"]
    a2 = gelu(h2)
    out = a2 @ w["W3"] + w["b3"]
    return out, (X, h1, a1, h2, a2)


def sigmoid(x):
    return 0.5 * (1.0 + np.tanh(0.5 * x))


def softplus(x):
    return np.maximum(x, 0.0) + np.log1p(np.exp(-np.abs(x)))


def loss(out, llr_target):
    """Mean soft-BCE: softplus(o) - sigma(lambda) o - [softplus(lambda) - sigma(lambda) lambda]
    (the bracket makes the minimum 0; it carries no gradient)."""
    p = sigmoid(llr_target)
    per = softplus(out) - p * out - (softplus(llr_target) - p * llr_target)
    return float(np.mean(per))


def backward(w, cache, out, llr_target):
    """Gradients of `loss` with respect to every weight (same keys as w)."""
    X, h1, a1, h2, a2 = cache
    B, m = out.shape
    d_out = (sigmoid(out) - sigmoid(llr_target)) / (B * m)
    g = {"W3": a2.T @ d_out, "b3": d_out.sum(axis=0)}
    d_h2 = (d_out @ w["W3"].T) * gelu_grad(h2)
    g["W2"] = a1.T @ d_h2
    g["b2"] = d_h2.sum(axis=0)
    d_h1 = (d_h2 @ w["W2"].T) * gelu_grad(h1)
    g["W1"] = X.T @ d_h1
    g["b1"] = d_h1.sum(axis=0)
    return g


def adam_step(w, g, state, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update in place (state holds the first and second moments, step starts at 1)."""
    for k in w:
        m_ = state.setdefault("m_" + k, np.zeros_like(w[k]))
        v_ = state.setdefault("v_" + k, np.zeros_like(w[k]))
        m_ *= beta1
        m_ += (1.0 - beta1) * g[k]
        v_ *= beta2
        v_ += (1.0 - beta2) * g[k] * g[k]
        mhat = m_ / (1.0 - beta1 ** step)
        vhat = v_ / (1.0 - beta2 ** step)
        w[k] -= lr * mhat / (np.sqrt(vhat) + eps)


# ---- storage rounding of the mixed-precision network (BF16 operands, FP32 accumulation) ----

def bf16_round(x):
    """Round to the nearest BF16 value (ties to even), via FP32, returned as float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16x2_round(x):
    """A value carried as two BF16 words: hi = bf16(x), lo = bf16(x - hi) (the difference taken
    in FP32), returned as hi + lo in float64 (about 16 significant bits)."""
    x32 = np.asarray(x, dtype=np.float64).astype(np.float32)
    hi = bf16_round(x32)
    lo = bf16_round((x32 - hi.astype(np.float32)).astype(np.float32))
    return hi + lo


def identity(x):
    return np.asarray(x, dtype=np.float64)


def forward_stored(w, X, rnd=bf16_round, b1=None, rnd_act=None):
    """Forward pass where every stored operand is rounded: the weights and the inputs by `rnd`,
    the two hidden activations after GELU by `rnd_act` (default: `rnd`); accumulation and biases
    in full precision.  `b1` overrides the first-layer bias (e.g. its BF16 hi + lo pair).
    Returns (out, cache)."""
    ra = rnd if rnd_act is None else rnd_act
    Xr = rnd(X)
    h1 = Xr @ rnd(w["W1"]) + (w["b1"] if b1 is None else b1)
    a1 = ra(gelu(h1))
    h2 = a1 @ rnd(w["W2"]) + w["b2"]
    a2 = ra(gelu(h2))
    out = a2 @ rnd(w["W3"]) + w["b3"]
    return out, (Xr, h1, a1, h2, a2)


def backward_stored(w, cache, out, llr_target, rnd=bf16_round, rnd_act=None):
    """Gradients of `loss` with the weights rounded by `rnd` as in forward_stored and the stored
    back-propagated deltas (output delta, two hidden deltas) rounded by `rnd_act` (default `rnd`)."""
    ra = rnd if rnd_act is None else rnd_act
    X, h1, a1, h2, a2 = cache
    B, m = out.shape
    d_out = ra((sigmoid(out) - sigmoid(llr_target)) / (B * m))
    g = {"W3": a2.T @ d_out, "b3": d_out.sum(axis=0)}
    d_h2 = ra((d_out @ rnd(w["W3"]).T) * gelu_grad(h2))
    g["W2"] = a1.T @ d_h2
    g["b2"] = d_h2.sum(axis=0)
    d_h1 = ra((d_h2 @ rnd(w["W2"]).T) * gelu_grad(h1))
    g["W1"] = X.T @ d_h1
    g["b1"] = d_h1.sum(axis=0)
    return g
