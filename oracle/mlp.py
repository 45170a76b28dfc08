"""FP64 reference of the surrogate network used to gate RM synthesis -- test
infrastructure only.

The network maps the Q/U spectrum of one line of sight to (phi_hat / phi_scale,
detection logit):

    x  = [w Q | w U] / rms,   rms = sqrt(mean of the squares of the 2 nchan inputs)
    h1 = relu(W1 x + b1)
    h2 = relu(W2 h1 + b2)
    o  = W3 h2 + b3                       o[0] = phi_hat / phi_scale, o[1] = logit

    loss = mean over the batch of
           BCE(sigmoid(o[1]), det) + det * (o[0] - phi / phi_scale)^2

and Adam (Kingma & Ba 2015) updates FP32 master weights.  `round16`, when set,
rounds to IEEE half precision at the points where the GPU kernels feed its
16-bit matrix units (the inputs x and h of every layer and the weights), so
that the two sides take identical precision decisions; all arithmetic here is
FP64 otherwise.
"""
from __future__ import annotations

import numpy as np


def _r16(a, on):
    return a.astype(np.float16).astype(np.float64) if on else np.asarray(a, dtype=np.float64)


def normalise(Q, U, w=None):
    """x = [w Q | w U] / rms per row (rows of all zeros stay zero)."""
    Q = np.asarray(Q, np.float64)
    U = np.asarray(U, np.float64)
    if w is not None:
        w = np.asarray(w, np.float64)
        Q = Q * w
        U = U * w
    x = np.concatenate([Q, U], axis=1)
    rms = np.sqrt(np.mean(x * x, axis=1, keepdims=True))
    return np.where(rms > 0, x / np.where(rms > 0, rms, 1.0), 0.0)


def forward(params, x, round16=False):
    W1, b1, W2, b2, W3, b3 = (np.asarray(p, np.float64) for p in params)
    x16 = _r16(x, round16)
    z1 = x16 @ _r16(W1, round16).T + b1
    h1 = np.maximum(z1, 0.0)
    h1_16 = _r16(h1, round16)
    z2 = h1_16 @ _r16(W2, round16).T + b2
    h2 = np.maximum(z2, 0.0)
    h2_16 = _r16(h2, round16)
    o = h2_16 @ _r16(W3, round16).T + b3
    cache = dict(x16=x16, z1=z1, h1_16=h1_16, z2=z2, h2_16=h2_16)
    return o, cache


def loss_and_grad_out(o, phi_label, det_label, phi_scale):
    """Mean loss and dL/do for a batch."""
    o = np.asarray(o, np.float64)
    t = np.asarray(phi_label, np.float64) / phi_scale
    d = np.asarray(det_label, np.float64)
    B = o.shape[0]
    s = o[:, 1]
    # BCE(sigmoid(s), d) = softplus(s) - d s, written stably.
    bce = np.maximum(s, 0.0) + np.log1p(np.exp(-np.abs(s))) - d * s
    err = o[:, 0] - t
    loss = float(np.mean(bce + d * err * err))
    g = np.zeros_like(o)
    e = np.exp(-np.abs(s))
    sig = np.where(s >= 0, 1.0 / (1.0 + e), e / (1.0 + e))
    g[:, 1] = (sig - d) / B
    g[:, 0] = 2.0 * d * err / B
    return loss, g


def backward(params, cache, g_out, round16=False, dz_scale=1.0):
    """Gradients of the mean loss w.r.t. (W1, b1, W2, b2, W3, b3).

    With round16 the back-propagated dz are rounded to half as dz_scale * dz
    (the GPU rounds the gradient of the batch sum, dz_scale = batch size) and
    scaled back exactly afterwards."""
    W1, b1, W2, b2, W3, b3 = (np.asarray(p, np.float64) for p in params)

    def r16s(a):
        return _r16(a * dz_scale, round16) / dz_scale if round16 else a

    gW3 = g_out.T @ cache["h2_16"]
    gb3 = g_out.sum(axis=0)
    gh2 = g_out @ _r16(W3, round16)
    gz2 = gh2 * (cache["z2"] > 0)
    gz2_16 = r16s(gz2)
    gW2 = gz2_16.T @ cache["h1_16"]
    gb2 = gz2.sum(axis=0)
    gh1 = gz2_16 @ _r16(W2, round16)
    gz1 = gh1 * (cache["z1"] > 0)
    gz1_16 = r16s(gz1)
    gW1 = gz1_16.T @ cache["x16"]
    gb1 = gz1.sum(axis=0)
    return [gW1, gb1, gW2, gb2, gW3, gb3]


def adam_update(params, grads, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (bias-corrected), in place on lists of arrays."""
    bc1 = 1.0 - beta1 ** step
    bc2 = 1.0 - beta2 ** step
    for p, g, mi, vi in zip(params, grads, m, v):
        mi *= beta1
        mi += (1.0 - beta1) * g
        vi *= beta2
        vi += (1.0 - beta2) * g * g
        p -= lr * (mi / bc1) / (np.sqrt(vi / bc2) + eps)


def init_params(nin, h1, h2, rng):
    """He-normal weights, zero biases (float64)."""
    W1 = rng.standard_normal((h1, nin)) * np.sqrt(2.0 / nin)
    W2 = rng.standard_normal((h2, h1)) * np.sqrt(2.0 / h1)
    W3 = rng.standard_normal((2, h2)) * np.sqrt(1.0 / h2)
    return [W1, np.zeros(h1), W2, np.zeros(h2), W3, np.zeros(2)]
