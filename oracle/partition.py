"""The MISR objective split into subdomains, in float64 (test infrastructure only).

The paper distributes the solve by partitioning the high-resolution image into
subdomains (Sec. 3.1, Eq. subfunction): the objective becomes a sum of local
objectives (Eq. reformulated), each node evaluates its own on its part of the
image plus an overlap, the gradients are assembled by exchanging the border
contributions, and the scalars of the solver are the sums of the nodes' local
products (the consensus of Alg. 1).  This module writes that decomposition
out with the oracle's literal operators, so that the invariants the paper
states can be checked in float64:

  * the local objectives sum to the global one, and their gradients, placed
    back on the image, sum to the global gradient;
  * the solve driven by the local costs, gradients and summed local inner
    products reaches the same image as the undivided solve.

Ownership (one owner for every term): subdomain h owns the HR rectangle
[u0, u1) x [v0, v1), whose edges are multiples of the scale s; it owns the LR
pixels whose s x s block lies in its rectangle and the prior's pairs
(i, i + d) whose first pixel i does.  Its window is the rectangle grown by
halo_lr LR pixels (s * halo_lr HR pixels) on every side, clipped to the image;
the local objective is evaluated on the window alone (zero outside it).  The
overlap must cover the reach of the operator and of the prior, or the owned
terms see the window's zero padding instead of the neighbours' pixels.
"""
from __future__ import annotations

import numpy as np

from . import ops
from .scg import scg_minimize


def tiles(H: int, W: int, s: int, tile_hr: int):
    """Owned rectangles (u0, u1, v0, v1) of a grid of tile_hr x tile_hr HR
    pixels (tile_hr a multiple of s; the last row and column are ragged)."""
    if tile_hr % s:
        raise ValueError("tile edges must be multiples of the scale")
    return [(u0, min(H, u0 + tile_hr), v0, min(W, v0 + tile_hr))
            for u0 in range(0, H, tile_hr) for v0 in range(0, W, tile_hr)]


def window(rect, H: int, W: int, s: int, halo_lr: int):
    """The subdomain's window: its rectangle grown by halo_lr LR pixels,
    clipped to the image."""
    u0, u1, v0, v1 = rect
    e = s * halo_lr
    return max(0, u0 - e), min(H, u1 + e), max(0, v0 - e), min(W, v1 + e)


def local_cost_grad(x, y, shifts, psf, s, rect, halo_lr, lambda_reg=0.01, alpha_btv=0.4,
                    eps=1e-3, w=3, data_p=2, eps_data=1e-3):
    """One subdomain's objective (Eq. subfunction) from its window alone:
    the data term over its owned LR pixels of every frame and the prior over
    its owned pairs.  Returns (E_data_h, E_reg_h, gradient on the window,
    window)."""
    H, W = x.shape
    a0, a1, b0, b1 = win = window(rect, H, W, s, halo_lr)
    xw = np.ascontiguousarray(x[a0:a1, b0:b1])
    yw = np.ascontiguousarray(y[:, a0 // s:a1 // s, b0 // s:b1 // s])
    u0, u1, v0, v1 = rect
    r = ops.forward(xw, shifts, psf, s) - yw
    own = np.zeros(r.shape[1:], dtype=bool)
    own[(u0 - a0) // s:(u1 - a0) // s, (v0 - b0) // s:(v1 - b0) // s] = True
    r = np.where(own[None], r, 0.0)
    if data_p == 2:
        Ed = float(np.sum(r * r))
        rr = 2.0 * r
    else:
        Ed = float(np.sum(np.where(own[None], r * r / (np.sqrt(r * r + eps_data ** 2)
                                                       + eps_data), 0.0)))
        rr = r / np.sqrt(r * r + eps_data ** 2)
    gw = ops.adjoint(rr, shifts, psf, s, a1 - a0, b1 - b0)
    Er, gr = ops.btv_owned(xw, (u0 - a0, u1 - a0, v0 - b0, v1 - b0), lambda_reg, alpha_btv,
                           eps, w)
    return Ed, Er, gw + gr, win


def cost_grad(x, y, shifts, psf, s, rects, halo_lr, **kw):
    """Sum of the local objectives and the assembled gradient (every window's
    gradient added back onto the image: the border exchange).  Returns
    (J, grad, per-subdomain (E_data_h, E_reg_h))."""
    g = np.zeros_like(x)
    parts = []
    for rect in rects:
        Ed, Er, gw, (a0, a1, b0, b1) = local_cost_grad(x, y, shifts, psf, s, rect, halo_lr, **kw)
        g[a0:a1, b0:b1] += gw
        parts.append((Ed, Er))
    return sum(a + b for a, b in parts), g, parts


def dot(rects):
    """The consensus inner product: each subdomain's product over its owned
    pixels, summed."""
    def f(a, b):
        return float(sum(np.sum(a[u0:u1, v0:v1] * b[u0:u1, v0:v1])
                         for (u0, u1, v0, v1) in rects))
    return f


def solve(y, shifts, psf, s, x0, n_iter, tile_hr, halo_lr, sigma=1e-4, lam1=1e-6, **kw):
    """Moller's SCG driven by the subdomains: local costs and gradients
    (assembled), consensus inner products; the literal finite-difference
    curvature."""
    H, W = x0.shape
    rects = tiles(H, W, s, tile_hr)

    def f(x, need_grad=True):
        J, g, _ = cost_grad(x, y, shifts, psf, s, rects, halo_lr, **kw)
        return J, g
    return scg_minimize(f, x0, n_iter, sigma, lam1, dot=dot(rects))
