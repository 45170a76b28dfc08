"""Helpers shared by the GPU parity tests (no arithmetic of the method here)."""
import sys

import numpy as np

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
