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
rounds the network's 16-bit inputs to IEEE half precision: the normalised
spectrum x and the weight matrices (the survey's FP16 operands).  Values the
network forms inside (h1, h2, the back-propagated dz) are never rounded here:
`error_bound` gives, element by element, how far an evaluation that rounds
them to half and accumulates in FP32 can move from this FP64 network.
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
    z2 = h1 @ _r16(W2, round16).T + b2
    h2 = np.maximum(z2, 0.0)
    o = h2 @ _r16(W3, round16).T + b3
    cache = dict(x16=x16, z1=z1, h1=h1, z2=z2, h2=h2)
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


def backward(params, cache, g_out, round16=False):
    """Gradients of the mean loss w.r.t. (W1, b1, W2, b2, W3, b3); with
    round16 the weight matrices enter as their half roundings (as in
    `forward`)."""
    W1, b1, W2, b2, W3, b3 = (np.asarray(p, np.float64) for p in params)
    gW3 = g_out.T @ cache["h2"]
    gb3 = g_out.sum(axis=0)
    gh2 = g_out @ _r16(W3, round16)
    gz2 = gh2 * (cache["z2"] > 0)
    gW2 = gz2.T @ cache["h1"]
    gb2 = gz2.sum(axis=0)
    gh1 = gz2 @ _r16(W2, round16)
    gz1 = gh1 * (cache["z1"] > 0)
    gW1 = gz1.T @ cache["x16"]
    gb1 = gz1.sum(axis=0)
    return [gW1, gb1, gW2, gb2, gW3, gb3]


def error_bound(params, x, phi_label, det_label, phi_scale, u=2.0 ** -11, ua=2.0 ** -25,
                acc=2.0 ** -24, lam=6.0):
    """Elementwise error bar for the outputs o and mean-loss gradients of
    `forward`/`backward` with round16 (x and the weights rounded to half)
    against the same network evaluated with

      * x, h1, h2 rounded to half from a value within FP32 accumulation
        error (relative u, absolute ua below half's normal range),
      * the back-propagated dz of both hidden layers rounded to half at the
        scale of the batch-SUM gradient (relative u, absolute ua / batch),
        the bias gradients summing the unrounded dz,
      * every dot product accumulated in FP32 (relative acc per addition),
      * ReLU masks taken from its own pre-activations (where |z| is within its
        error bar the mask may differ, and the whole term it admits or
        removes then counts as error).

    Probabilistic rounding-error analysis (Higham & Mary, SIAM J. Sci.
    Comput. 41, 2019): each rounding is an independent error uniform within
    +-u|v| (variance u^2 v^2 / 3); the variances propagate through each
    layer's products (a sum of independent errors adds their variances:
    var(sum a_i e_i) = sum a_i^2 var(e_i)), ReLU is 1-Lipschitz, the sigmoid's
    slope is at most 1/4; the bar is lam standard deviations.  A worst-case
    bound (|A||B| in place of the squares) holds always but lies 100-300 times
    above the errors a real evaluation makes, too far to be a useful bar.
    Returns (bar on o [B][2], [bars on gW1, gb1, gW2, gb2, gW3, gb3])."""
    W1, b1, W2, b2, W3, b3 = (np.asarray(p, np.float64) for p in params)
    W1, W2, W3 = (_r16(W, True) for W in (W1, W2, W3))
    q1, q2, q3 = W1 * W1, W2 * W2, W3 * W3
    x16 = _r16(x, True)
    B, nin = x16.shape
    nh1, nh2 = W1.shape[0], W2.shape[0]
    z1 = x16 @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    o = h2 @ W3.T + b3
    r3 = u * u / 3.0          # variance of one half rounding, relative
    a3 = acc * acc / 3.0      # variance of one FP32 rounding, relative

    def rnd(v, var, absolute):                     # rounding of v to half
        return var + r3 * v * v + absolute * absolute / 3.0

    def accum(n, terms2):                          # n FP32 additions of terms with these squares
        return a3 * n * terms2

    v_x = rnd(x16, a3 * x16 * x16, ua)             # FP32 normalisation, then half
    v_z1 = v_x @ q1.T + accum(nin + 1, (x16 * x16) @ q1.T + b1 * b1)
    v_h1 = rnd(h1, v_z1, ua)
    v_z2 = v_h1 @ q2.T + accum(nh1 + 1, (h1 * h1) @ q2.T + b2 * b2)
    v_h2 = rnd(h2, v_z2, ua)
    v_o = v_h2 @ q3.T + accum(nh2 + 1, (h2 * h2) @ q3.T + b3 * b3)

    d = np.asarray(det_label, np.float64)
    t = np.asarray(phi_label, np.float64) / phi_scale
    s = o[:, 1]
    ex = np.exp(-np.abs(s))
    sig = np.where(s >= 0, 1.0 / (1.0 + ex), ex / (1.0 + ex))
    g = np.stack([2.0 * d * (o[:, 0] - t), sig - d], axis=1) / B
    g2 = g * g
    v_g = np.stack([4.0 * d * v_o[:, 0] + a3 * 4 * (o[:, 0] ** 2 + t * t),
                    v_o[:, 1] / 16.0 + a3 * 16], axis=1) / (B * B)

    v_W3 = v_g.T @ (h2 * h2 + v_h2) + g2.T @ v_h2 + accum(B, g2.T @ (h2 * h2))
    v_b3 = v_g.sum(axis=0) + accum(B, g2.sum(axis=0))

    def hidden(gh, v_gh, z, v_z):                  # ReLU' mask, possibly flipped
        m = z > 0
        flip = np.abs(z) <= lam * np.sqrt(v_z)
        gz = gh * m
        v_gz = np.where(m, v_gh, 0.0) + np.where(flip, gh * gh + v_gh, 0.0)
        return gz, v_gz

    gh2 = g @ W3
    v_gh2 = v_g @ q3 + accum(2, g2 @ q3)
    gz2, v_gz2 = hidden(gh2, v_gh2, z2, v_z2)
    v_gz2r = rnd(gz2, v_gz2, ua / B)
    v_W2 = v_gz2r.T @ (h1 * h1 + v_h1) + (gz2 * gz2).T @ v_h1 + accum(B, (gz2 * gz2).T @ (h1 * h1))
    v_b2 = v_gz2.sum(axis=0) + accum(B, (gz2 * gz2).sum(axis=0))

    gh1 = gz2 @ W2
    v_gh1 = v_gz2r @ q2 + accum(nh2, (gz2 * gz2) @ q2)
    gz1, v_gz1 = hidden(gh1, v_gh1, z1, v_z1)
    v_gz1r = rnd(gz1, v_gz1, ua / B)
    v_W1 = v_gz1r.T @ (x16 * x16 + v_x) + (gz1 * gz1).T @ v_x + accum(B, (gz1 * gz1).T @ (x16 * x16))
    v_b1 = v_gz1.sum(axis=0) + accum(B, (gz1 * gz1).sum(axis=0))
    bar = [lam * np.sqrt(v) for v in (v_W1, v_b1, v_W2, v_b2, v_W3, v_b3)]
    return lam * np.sqrt(v_o), bar


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
