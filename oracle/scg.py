"""Scaled conjugate gradient, step by step, in float64 (test infrastructure only).

The paper solves its objective (Eq. objective) with SCG, citing M. F. Moller,
"A scaled conjugate gradient algorithm for fast supervised learning",
Neural Networks 6(4):525-533, 1993; the algorithm itself is not printed in the
paper, so this follows Moller's published method, with the loop bound of
Algorithm 1 (a fixed number of passes, failed ones included).  Notation:
g = grad J, r = -g (steepest descent), p the conjugate direction,
lam the Levenberg-Marquardt scale and lam_bar its raised value.

Readings of points the paper leaves open:
  * sigma = 1e-4 and lam_1 = 1e-6 (Moller's stated bounds); restart period N is
    the number of unknowns (H * W);
  * after a failed step the curvature is not recomputed: the scaled delta is
    carried into the next pass and re-scaled there;
  * no extra safeguard on the new direction: if p . r < 0, the step
    alpha = mu / delta is negative and still moves downhill along -p, which is
    how Moller's method treats it;
  * the pass stops early only if ||r||^2 == 0.
"""
from __future__ import annotations

import math

import numpy as np

from . import ops


def _dot_plain(a: np.ndarray, b: np.ndarray) -> float:
    """FP64 inner product by pairwise summation (no BLAS threads, which would
    contend with the OpenMP threads of the C operators)."""
    return float(np.add.reduce(np.multiply(a.ravel(), b.ravel())))


def moller_scale_delta(delta: float, lam: float, lam_bar: float, pi: float):
    """Steps 3-4: shift delta by (lam - lam_bar)*|p|^2 and make it positive.

    Returns (delta, lam, lam_bar)."""
    delta = delta + (lam - lam_bar) * pi
    if delta <= 0.0:
        lam_bar = 2.0 * (lam - delta / pi)
        delta = -delta + lam * pi
        lam = lam_bar
    return delta, lam, lam_bar


def moller_update_lambda(Delta: float, lam: float, delta: float, pi: float) -> float:
    """Steps 7-8's scale rule: shrink on a very good step, grow on a poor one."""
    if Delta >= 0.75:
        lam = lam / 4.0
    if Delta < 0.25:
        lam = lam + delta * (1.0 - Delta) / pi
    return lam


def scg_minimize(J_and_grad, x0: np.ndarray, n_iter: int, sigma: float = 1e-4,
        lam1: float = 1e-6, curvature=None, trace: bool = True, dot=None):
    """Minimise J from x0 with Moller's SCG for exactly ``n_iter`` passes.

    ``J_and_grad(x, need_grad) -> (J, g or None)``.
    ``curvature(x, p, sk) -> delta`` replaces the literal finite difference
    p^T (grad J(x + sk p) - grad J(x)) / sk when given (check mode).
    ``dot(a, b)`` replaces the inner product (the partitioned solve sums the
    subdomains' local products, Alg. 1's consensus).
    Returns (x, trace list of dicts, info dict).
    """
    _dot = dot or _dot_plain
    x = np.array(x0, dtype=np.float64, copy=True)
    N = x.size
    E, g = J_and_grad(x, True)
    r = -g
    p = r.copy()
    lam, lam_bar = lam1, 0.0
    success = True
    k = 1
    delta = pi = 0.0
    recs = []
    for it in range(n_iter):
        rr = _dot(r, r)
        if rr == 0.0:
            break
        # step 2: second-order information along p, only after a success
        if success:
            pi = _dot(p, p)
            sk = sigma / math.sqrt(pi)
            if curvature is None:
                _, g_s = J_and_grad(x + sk * p, True)
                s_vec = (g_s - g) / sk
                delta = _dot(p, s_vec)
            else:
                delta = float(curvature(x, p, sk))
        # steps 3-4: scale and force positive definiteness
        delta, lam, lam_bar = moller_scale_delta(delta, lam, lam_bar, pi)
        # step 5: step size
        mu = _dot(p, r)
        alpha = mu / delta
        # step 6: comparison parameter
        x_t = x + alpha * p
        E_t, g_t = J_and_grad(x_t, True)
        Delta = 2.0 * delta * (E - E_t) / (mu * mu)
        ok = Delta >= 0.0
        if ok:
            # step 7: accept
            x = x_t
            E = E_t
            r_new = -g_t
            lam_bar = 0.0
            success = True
            if k % N == 0:
                p_new = r_new.copy()
            else:
                beta = (_dot(r_new, r_new) - _dot(r_new, r)) / mu
                p_new = r_new + beta * p
            p = p_new
            r = r_new
            g = g_t
        else:
            lam_bar = lam
            success = False
        lam = moller_update_lambda(Delta, lam, delta, pi)
        k += 1
        if trace:
            recs.append(dict(it=it, E=E, E_t=E_t, delta=delta, mu=mu, alpha=alpha,
                             Delta=Delta, success=bool(ok), lam=lam))
    return x, recs, dict(passes=len(recs))


def misr_objective(y, shifts, psf, s, lambda_reg=0.01, alpha_btv=0.4, eps=1e-3, w=3,
                   data_p=2, eps_data=1e-3, warps=None):
    """J(x) and grad J(x) of the MISR objective through the C operators."""
    def f(x, need_grad=True):
        J, g, _ = ops.cost_grad(x, y, shifts, psf, s, lambda_reg, alpha_btv, eps, w,
                                data_p, eps_data, grad=need_grad, warps=warps)
        return J, g
    return f


def misr_curvature_exact(shifts, psf, s, lambda_reg=0.01, alpha_btv=0.4, eps=1e-3, w=3):
    def c(x, p, sk):
        return ops.curvature_exact(x, p, shifts, psf, s, sk, lambda_reg, alpha_btv, eps, w)[0]
    return c


def solve(prob_y, shifts, psf, s, x0, n_iter, lambda_reg=0.01, alpha_btv=0.4, eps=1e-3,
          w=3, sigma=1e-4, lam1=1e-6, exact_curvature=False, data_p=2, eps_data=1e-3,
          warps=None, progress=None):
    """SCG solve of the MISR objective (Eq. misr: L2 data term, or the
    Charbonnier-smoothed L1 term for data_p = 1), Moller's finite-difference
    curvature unless exact_curvature (L2, translational warps only); warps:
    per-frame affine coefficients (see ops) instead of the shifts.
    progress(n): called after the n-th objective evaluation (log lines of
    long runs; takes no part in the arithmetic)."""
    if exact_curvature and (data_p != 2 or warps is not None):
        raise ValueError("the closed-form curvature here covers the L2 data term and shifts")
    f = misr_objective(prob_y, shifts, psf, s, lambda_reg, alpha_btv, eps, w, data_p, eps_data,
                       warps)
    curv = misr_curvature_exact(shifts, psf, s, lambda_reg, alpha_btv, eps, w) \
        if exact_curvature else None
    if progress is not None:
        f = _counted(f, progress)
    return scg_minimize(f, x0, n_iter, sigma, lam1, curvature=curv)


def _counted(f, progress):
    n = [0]

    def g(x, need_grad):
        out = f(x, need_grad)
        n[0] += 1
        progress(n[0])
        return out
    return g
