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


def mix64(x):
    """Interaction-set checksum mixer, vectorised: the SplitMix64 finalizer of x + golden gamma
    (pinned against the generator's published outputs in tests/test_mix64_kat.py)."""
    with np.errstate(over="ignore"):
        z = np.asarray(x).astype(np.uint64) + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))
