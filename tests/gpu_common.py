"""Shared helpers of the GPU parity tests (no method arithmetic)."""
import numpy as np

RTOL_APPLY = 1e-12     # one operator / preconditioner apply, FP64 (rounding order only)
RTOL_SOLVE = 1e-10     # FP64 solution against the oracle solution
RTOL_MIXED = 1e-8      # mixed-precision solution (float operator, FP64 replacement) against FP64
# one apply of the float operator: every output is a chain of about five
# contractions of at most 2W+1 <= 25 float terms (float unit roundoff 6e-8)
# on data rounded to float, and X cancels up to two digits on random input
RTOL_FP32_APPLY = 1e-4


def rand_vec(ndof, seed):
    return np.random.default_rng(seed).standard_normal(ndof)


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300)


def to_dev(x):
    import torch
    return torch.tensor(np.asarray(x, float), dtype=torch.float64, device="cuda")


def to_host(t):
    return t.detach().cpu().numpy()
