"""Shared helpers of the GPU parity tests (inputs, tolerances, comparisons)."""
import numpy as np

import oracle
from paper_2108_04315_amd import synth

# Tolerances stated for the hot path: FP32 operator applications 1e-5 rel-L2,
# FP32 SCG image after the fixed pass count 1e-4, 16-bit storage 1e-2.
TOL_OP = 1e-5
TOL_SCG = 1e-4
TOL_LOWP = 1e-2


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def psnr(a, b, peak=1.0) -> float:
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    return float("inf") if mse == 0 else 10 * np.log10(peak * peak / mse)


def problem(L, s, sigma, P=None, noise=("poisson", 1e4), jitter=0.05, n_iter=10,
            seeds=(0, 1, 2), Lw=None):
    """Inputs drawn by the generator, clean frames from the oracle's forward."""
    return synth.make_problem(oracle.forward, L=L, s=s, sigma=sigma, P=P, noise=noise,
                              jitter=jitter, n_iter=n_iter, seeds=seeds, Lw=Lw)


def to_dev(a, dtype=None):
    import torch
    dtype = dtype or torch.float32
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda").to(dtype)


def to_np(t):
    import torch
    return t.detach().to(torch.float64).cpu().numpy()
