"""Shared helpers of the GPU tests: device copies of generator inputs and error metrics."""
import math

import numpy as np


def dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def rel_rms(a, ref):
    return math.sqrt(float(((a - ref) ** 2).sum()) / float((ref ** 2).sum()))


def rel_max(a, ref):
    num = np.linalg.norm(a - ref, axis=1)
    den = np.linalg.norm(ref, axis=1)
    ok = den > 0
    return float((num[ok] / den[ok]).max()) if ok.any() else 0.0


def u64(t):
    return t.cpu().numpy().view(np.uint64)
