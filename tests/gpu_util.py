"""Helpers shared by the GPU parity tests: tolerances and marshalling (the
method's arithmetic is the oracle's)."""
import sys

import numpy as np

import oracle

PREC_TOL = {  # per-LOS bound on max_k |F_gpu - F_oracle| / max_k |F_oracle|
    "fp32": 1e-5,
    "bf16x3": 1e-5,
    "fp16x3": 1e-5,
}

# Bound for grids too short for max_k |F| to be representative (a handful of
# phi): the error relative to max(max_k |F|, K sqrt(sum w^2 |P|^2)).  FP32 keeps
# 1e-5; the bfloat16 hi+lo split carries 16 significand bits per operand, so
# one product is off by at most ~3 x 2^-16 of its size (two split residuals
# and the dropped lo*lo term).
SCALE_TOL = {
    "fp32": 1e-5,
    "bf16x3": 3 * 2.0 ** -16,
    "fp16x3": 1e-5,   # 11-bit halves: split residuals 2^-22, below FP32 rounding effects
}


def note(msg: str):
    """Print what names the case before a GPU step, flushed."""
    print(msg, flush=True)
    sys.stdout.flush()


def dev32(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def fit_bar(Fq, Fu, phi, idx, dy):
    """Largest change of the parabola's vertex (phi, amp) when each of the
    three amplitudes around idx moves by up to dy[l] (corners of the box),
    doubled.  Rows whose peak sits at a grid end only move amp (by dy)."""
    Fq, Fu = np.asarray(Fq, np.float64), np.asarray(Fu, np.float64)
    rows = np.arange(len(idx))
    nphi = Fq.shape[1]
    k = np.clip(idx, 1, nphi - 2)
    y = [np.hypot(Fq[rows, k + d], Fu[rows, k + d]) for d in (-1, 0, 1)]
    x = [phi[k + d] for d in (-1, 0, 1)]
    p0, a0 = oracle.peak_fit(y[0], y[1], y[2], *x)
    dp, da = np.zeros(len(idx)), np.zeros(len(idx))
    for s0 in (-1, 1):
        for s1 in (-1, 1):
            for s2 in (-1, 1):
                p, a = oracle.peak_fit(y[0] + s0 * dy, y[1] + s1 * dy, y[2] + s2 * dy, *x)
                dp = np.maximum(dp, np.abs(p - p0))
                da = np.maximum(da, np.abs(a - a0))
    edge = (idx == 0) | (idx == nphi - 1)
    return np.where(edge, 0.0, 2 * dp), np.where(edge, 2 * dy, 2 * da)
