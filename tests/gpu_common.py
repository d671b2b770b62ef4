"""Helpers shared by the GPU tests (no method arithmetic here)."""
import sys

import numpy as np


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_err(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.abs(x - ref).max() / max(np.abs(ref).max(), 1e-300))


def to_dev(x, dtype):
    import torch
    return torch.tensor(np.asarray(x), dtype=dtype, device="cuda")


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy()
