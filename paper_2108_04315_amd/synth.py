"""Seeded synthetic inputs for multi-image super-resolution of CT projections.

This module draws the inputs that both the GPU path and the CPU checker
consume: ground-truth phantoms, per-frame subpixel shifts, the 1-D Gaussian PSF
taps, additive noise and the bicubic initial guess.  It holds none of the
observation model or the SCG arithmetic: clean low-resolution frames are made
by a forward operator that the caller passes in (``forward_fn``).

Workload shapes follow the paper's experiments (Sec. 4 and Table "runtime"):
x2 upscaling from 4 frames shifted by half a detector pixel (the detector moves
right, down, left, up; Sec. 3.2 "Real-Time MISR for CT"), x3 with 9 frames on a
1/3-pixel grid (Table "natural"), piecewise-constant disks and bar patterns
standing in for the aluminium cylinder and QRM bar phantoms, which are not
available here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "phantom", "frame_shifts", "psf_size", "psf_taps", "add_gaussian_noise",
    "add_poisson_noise", "bicubic_upsample", "Problem", "make_problem",
    "CONFIGS", "batch_specs", "serving_requests",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def phantom(H: int, W: int, seed: int) -> np.ndarray:
    """Piecewise-constant HR test image in [0, 1], float64, shape (H, W).

    20 disks (centre uniform in the image, radius uniform in
    [0.02, 0.12] * min(H, W), intensity uniform in [0.2, 1]; later disks
    overwrite earlier ones), then 3 groups of 5 bars of intensity 1 whose bar
    width is 1, 2 or 3 times max(1, H // 512) pixels with gap equal to width,
    horizontal or vertical by coin flip.
    """
    rng = _rng(seed)
    img = np.zeros((H, W), dtype=np.float64)
    m = min(H, W)
    for _ in range(20):
        cy = rng.uniform(0, H)
        cx = rng.uniform(0, W)
        r = rng.uniform(0.02, 0.12) * m
        val = rng.uniform(0.2, 1.0)
        y0, y1 = max(0, int(cy - r) - 1), min(H, int(cy + r) + 2)
        x0, x1 = max(0, int(cx - r) - 1), min(W, int(cx + r) + 2)
        if y0 >= y1 or x0 >= x1:
            continue
        yy = (np.arange(y0, y1) + 0.5 - cy)[:, None]
        xx = (np.arange(x0, x1) + 0.5 - cx)[None, :]
        mask = yy * yy + xx * xx <= r * r
        img[y0:y1, x0:x1][mask] = val
    unit = max(1, H // 512)
    for _ in range(3):
        width = int(rng.integers(1, 4)) * unit
        vertical = bool(rng.integers(0, 2))
        length = max(1, int(rng.uniform(0.05, 0.2) * m))
        span = 10 * width
        oy = int(rng.integers(0, max(1, H - (length if vertical else span))))
        ox = int(rng.integers(0, max(1, W - (span if vertical else length))))
        for b in range(5):
            off = 2 * b * width
            if vertical:
                img[oy:oy + length, ox + off:ox + off + width] = 1.0
            else:
                img[oy + off:oy + off + width, ox:ox + length] = 1.0
    np.clip(img, 0.0, 1.0, out=img)
    return img


def frame_shifts(s: int, K: int | None = None, jitter: float = 0.0,
                 seed: int = 0) -> np.ndarray:
    """Per-frame subpixel shifts in LR pixels, shape (K, 2) as (dx, dy).

    s = 2 follows the detector movement order of the paper (reference, then
    right, down, left by half a pixel): (0,0), (1/2,0), (1/2,1/2), (0,1/2).
    Other s use the s x s grid {0, 1/s, ..., (s-1)/s}^2 in row-major order
    (dy outer).  Frame 0 is the reference and never jittered; frames k >= 1
    get independent uniform jitter in [-jitter, +jitter] on both axes.
    """
    if K is None:
        K = s * s
    if s == 2:
        grid = [(0.0, 0.0), (0.5, 0.0), (0.5, 0.5), (0.0, 0.5)]
    else:
        grid = [(dx / s, dy / s) for dy in range(s) for dx in range(s)]
    out = np.array([grid[k % len(grid)] for k in range(K)], dtype=np.float64)
    if jitter > 0 and K > 1:
        rng = _rng(seed)
        out[1:] += rng.uniform(-jitter, jitter, size=(K - 1, 2))
    return out


def psf_size(sigma: float) -> int:
    """Odd PSF support 2*ceil(3*sigma)+1 (5 for sigma 0.6, 7 for 0.8 and 1.0)."""
    return 2 * int(math.ceil(3.0 * sigma - 1e-12)) + 1


def psf_taps(sigma: float, P: int | None = None) -> np.ndarray:
    """Point-sampled 1-D Gaussian taps, normalised to sum 1 (float64, length P).

    The 2-D PSF is the outer product of these taps with themselves.
    """
    if P is None:
        P = psf_size(sigma)
    if P % 2 != 1:
        raise ValueError("PSF size must be odd")
    a = np.arange(P, dtype=np.float64) - (P - 1) / 2
    h = np.exp(-(a * a) / (2.0 * sigma * sigma))
    return h / h.sum()


def add_gaussian_noise(clean: np.ndarray, sigma: float, seed: int) -> np.ndarray:
    rng = _rng(seed)
    return clean + rng.normal(0.0, sigma, size=clean.shape)


def add_poisson_noise(clean: np.ndarray, mean_counts: float, seed: int) -> np.ndarray:
    """Poisson-like noise: scale to ``mean_counts`` mean, draw Poisson, rescale."""
    rng = _rng(seed)
    mean = float(np.mean(clean))
    n0 = mean_counts / mean if mean > 0 else mean_counts
    lam = np.maximum(clean, 0.0) * n0
    return rng.poisson(lam).astype(np.float64) / n0


def _keys_weights(t: np.ndarray, a: float = -0.5) -> np.ndarray:
    """Keys cubic convolution weights for the 4 taps at offsets -1, 0, 1, 2."""
    out = np.empty(t.shape + (4,), dtype=np.float64)
    for j, off in enumerate((-1.0, 0.0, 1.0, 2.0)):
        d = np.abs(t - off)
        w = np.where(d <= 1.0, (a + 2) * d**3 - (a + 3) * d**2 + 1.0,
                     np.where(d < 2.0, a * d**3 - 5 * a * d**2 + 8 * a * d - 4 * a, 0.0))
        out[..., j] = w
    return out


def _cubic_axis(img: np.ndarray, s: int, axis: int) -> np.ndarray:
    n = img.shape[axis]
    u = np.arange(n * s, dtype=np.float64)
    c = (u + 0.5) / s - 0.5
    base = np.floor(c).astype(np.int64)
    w = _keys_weights(c - base)
    out = None
    for j in range(4):
        idx = np.clip(base - 1 + j, 0, n - 1)
        term = np.take(img, idx, axis=axis)
        shape = [1, 1]
        shape[axis] = n * s
        term = term * w[:, j].reshape(shape)
        out = term if out is None else out + term
    return out


def bicubic_upsample(lr: np.ndarray, s: int) -> np.ndarray:
    """Keys bicubic (a = -0.5) upsampling by s with pixel-centre alignment.

    HR sample u sits at LR coordinate (u + 1/2)/s - 1/2; taps outside the
    frame are clamped to the edge.  Float64 in, float64 out.
    """
    return _cubic_axis(_cubic_axis(np.asarray(lr, dtype=np.float64), s, 0), s, 1)


@dataclass
class Problem:
    """One projection's inputs. ``y`` has shape (K, H//s, W//s)."""
    H: int
    W: int
    s: int
    shifts: np.ndarray
    psf: np.ndarray
    x_gt: np.ndarray
    y: np.ndarray
    x0: np.ndarray
    n_iter: int
    lambda_reg: float = 0.01
    alpha_btv: float = 0.4
    eps: float = 1e-3
    btv_w: int = 3
    meta: dict = field(default_factory=dict)

    @property
    def K(self) -> int:
        return self.shifts.shape[0]


# Configurations: the recipe of each workload.  "jitter" in LR pixels.
CONFIGS = {
    "plain128": dict(L=64, s=2, sigma=0.6, P=5, noise=("gauss", 0.01), jitter=0.0,
                     n_iter=50, seeds=(0, 0, 1)),
    "plain2048": dict(L=1024, s=2, sigma=0.8, P=7, noise=("poisson", 1e4), jitter=0.05,
                      n_iter=100, seeds=(0, 1, 2)),
    "precision6144": dict(L=2048, s=3, sigma=1.0, P=7, noise=("poisson", 1e4), jitter=0.05,
                          n_iter=100, seeds=(0, 1, 2)),
}


def make_problem(forward_fn, L: int, s: int, sigma: float, P: int | None = None,
                 noise=("poisson", 1e4), jitter: float = 0.05, n_iter: int = 100,
                 seeds=(0, 1, 2), Lw: int | None = None, **kw) -> Problem:
    """Build one projection's inputs.

    ``forward_fn(x_gt, shifts, psf, s)`` must return the clean frames
    (K, H//s, W//s) as float64; the caller chooses which implementation.
    """
    Lw = L if Lw is None else Lw
    H, W = s * L, s * Lw
    ph_seed, jit_seed, noise_seed = seeds
    x_gt = phantom(H, W, ph_seed)
    shifts = frame_shifts(s, s * s, jitter, jit_seed)
    psf = psf_taps(sigma, P)
    clean = np.asarray(forward_fn(x_gt, shifts, psf, s), dtype=np.float64)
    kind, level = noise
    if kind == "gauss":
        y = add_gaussian_noise(clean, level, noise_seed)
    elif kind == "poisson":
        y = add_poisson_noise(clean, level, noise_seed)
    elif kind == "none":
        y = clean.copy()
    else:
        raise ValueError(kind)
    x0 = bicubic_upsample(y[0], s)
    return Problem(H=H, W=W, s=s, shifts=shifts, psf=psf, x_gt=x_gt, y=y, x0=x0,
                   n_iter=n_iter, meta=dict(kw, L=L, sigma=sigma, noise=noise,
                                            jitter=jitter, seeds=seeds), **{
                       k: v for k, v in kw.items()
                       if k in ("lambda_reg", "alpha_btv", "eps", "btv_w")})


def batch_specs(n: int = 64, base_seed: int = 1000):
    """Size/scale draws for the batched workload: projection i uses seed base+i.

    LR side uniform in {512, 768, 1024, 1536, 2048}, scale uniform in {2, 3},
    K = s^2 frames, PSF sigma 0.8, Poisson noise, jitter 0.05, 60 iterations.
    """
    out = []
    for i in range(n):
        rng = _rng(base_seed + i)
        L = int(rng.choice([512, 768, 1024, 1536, 2048]))
        s = int(rng.choice([2, 3]))
        out.append(dict(L=L, s=s, sigma=0.8, P=7, noise=("poisson", 1e4), jitter=0.05,
                        n_iter=60, seeds=(base_seed + i, base_seed + i, base_seed + i)))
    return out


def serving_requests(n: int, rate_hz: float, seed: int = 7,
                     sizes=(512, 768, 1024, 1536, 2048, 3072, 4096), n_iter: int = 80):
    """Poisson arrival stream: list of (arrival_s, spec) for the serving workload."""
    rng = _rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate_hz)
        L = int(rng.choice(list(sizes)))
        s = int(rng.choice([2, 3]))
        out.append((t, dict(L=L, s=s, sigma=0.8, P=7, noise=("poisson", 1e4),
                            jitter=0.05, n_iter=n_iter, seeds=(seed * 7919 + i,) * 3)))
    return out
