"""Shared helpers of the GPU parity tests (no method arithmetic)."""
import numpy as np

RTOL_APPLY = 1e-12     # one operator / preconditioner apply, FP64 (rounding order only)
RTOL_SOLVE = 1e-10     # FP64 solution against the oracle solution


def rand_vec(ndof, seed):
    return np.random.default_rng(seed).standard_normal(ndof)


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300)


def to_dev(x):
    import torch
    return torch.tensor(np.asarray(x, float), dtype=torch.float64, device="cuda")


def to_host(t):
    return t.detach().cpu().numpy()
