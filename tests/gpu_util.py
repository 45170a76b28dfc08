"""Helpers shared by the GPU parity tests (no arithmetic of the method here)."""
import sys

import numpy as np

PREC_TOL = {  # per-LOS bound on max_k |F_gpu - F_oracle| / max_k |F_oracle|
    "fp32": 1e-5,
    "bf16x3": 1e-5,
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
