"""The window arithmetic of the matrix-free general kernels, replayed on the
CPU in FP64 against the oracle (no GPU, no library).

A general A_k = D B_k M_k (Eq. sisr with an affine warp and a P x P PSF) is
applied on the device from its factors: the forward builds the warped image on
each LR tile's HR window and takes every LR pixel's Q x Q window times the
blur-and-bin kernel C_k (Q = s + P - 1); the adjoint forms the
back-projection B^T D^T r on the preimage of each HR tile and gathers, per
pixel, the candidate positions whose warped coordinate lies within one pixel
of it, with the bilinear tent weights.  The kernels rely on three facts that
this test checks on tiles, sizes and warps that stress them (ragged tiles,
scales 1-4, rotations up to 135 degrees):

* C_k reproduces D B_k (the forward equals the oracle's);
* every candidate of every pixel of a tile lies inside the tile's window, so
  the gathers need no bounds checks, and the window fits the per-frame cap
  the host derives from the inverse warp;
* the gathered adjoint equals the oracle's (it is the forward's transpose).

The tile sizes and caps below restate the kernels' constants (LR tiles of
8 x 64, HR tiles of 16 x 64, the cap floor(15 |g0| + 63 |g1| + 2 e) + 3).
"""
import math

import numpy as np
import pytest

import oracle

TI, TJ, TU, TV = 8, 64, 16, 64


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def _rot(theta, H, W, ty=0.0, tx=0.0):
    c, s_ = math.cos(theta), math.sin(theta)
    cy, cx = (H - 1) / 2, (W - 1) / 2
    return np.array([c, -s_, cy - c * cy + s_ * cx + ty, s_, c, cx - s_ * cy - c * cx + tx])


def _plan(s, P, m, h2):
    """Per-frame quantities the host computes: inverse warp, half extents,
    candidate counts, window caps, and the blur-and-bin kernel."""
    Q, R = s + P - 1, (P - 1) // 2
    det = m[0] * m[4] - m[1] * m[3]
    g = [m[4] / det, -m[1] / det, 0.0, -m[3] / det, m[0] / det, 0.0]
    g[2] = -(g[0] * m[2] + g[1] * m[5])
    g[5] = -(g[3] * m[2] + g[4] * m[5])
    eu, ev = abs(g[0]) + abs(g[1]), abs(g[3]) + abs(g[4])
    ru = math.floor((TU - 1) * abs(g[0]) + (TV - 1) * abs(g[1]) + 2 * eu) + 3
    rv = math.floor((TU - 1) * abs(g[3]) + (TV - 1) * abs(g[4]) + 2 * ev) + 3
    C = np.zeros((Q, Q))
    for al in range(Q):
        for be in range(Q):
            for a in range(s):
                for b in range(s):
                    ia, ib = a + 2 * R - al, b + 2 * R - be
                    if 0 <= ia < P and 0 <= ib < P:
                        C[al, be] += h2[ia, ib]
    return dict(m=m, g=g, eu=eu, ev=ev, ncu=math.floor(2 * eu) + 1, ncv=math.floor(2 * ev) + 1,
                ru=ru, rv=rv, C=C / (s * s), Q=Q, R=R)


def _sample(x, m, u, v):
    H, W = x.shape
    if not (0 <= u < H and 0 <= v < W):
        return 0.0
    r, c = m[0] * u + m[1] * v + m[2], m[3] * u + m[4] * v + m[5]
    r0, c0 = math.floor(r), math.floor(c)
    fa, fb = r - r0, c - c0
    acc = 0.0
    for dr, dc, wq in ((0, 0, (1 - fa) * (1 - fb)), (0, 1, (1 - fa) * fb),
                       (1, 0, fa * (1 - fb)), (1, 1, fa * fb)):
        if 0 <= r0 + dr < H and 0 <= c0 + dc < W:
            acc += wq * x[r0 + dr, c0 + dc]
    return acc


def _forward(x, s, f):
    """The forward's tiles: warped window, then the Q x Q kernel."""
    H, W = x.shape
    h, w, Q, R = H // s, W // s, f["Q"], f["R"]
    y = np.zeros((h, w))
    for i0 in range(0, h, TI):
        for j0 in range(0, w, TJ):
            ZR, ZC = s * (TI - 1) + Q, s * (TJ - 1) + Q
            z = np.array([[_sample(x, f["m"], s * i0 - R + a, s * j0 - R + b)
                           for b in range(ZC)] for a in range(ZR)])
            for i in range(i0, min(i0 + TI, h)):
                for j in range(j0, min(j0 + TJ, w)):
                    a, b = s * (i - i0), s * (j - j0)
                    y[i, j] = np.sum(f["C"] * z[a:a + Q, b:b + Q])
    return y


def _adjoint(r, s, H, W, f):
    """The adjoint's tiles: window bounds, back-projection, candidate gathers;
    asserts that the candidates stay inside the window and the window inside
    the cap."""
    h, w, Q, R = H // s, W // s, f["Q"], f["R"]
    g, m, eu, ev = f["g"], f["m"], f["eu"], f["ev"]
    x = np.zeros((H, W))
    for U0 in range(0, H, TU):
        for V0 in range(0, W, TV):
            U1, V1 = min(U0 + TU, H) - 1, min(V0 + TV, W) - 1
            uc = [g[0] * p + g[1] * q + g[2] for p in (U0, U1) for q in (V0, V1)]
            vc = [g[3] * p + g[4] * q + g[5] for p in (U0, U1) for q in (V0, V1)]
            ua, va = math.floor(min(uc) - eu) + 1, math.floor(min(vc) - ev) + 1
            ub, vb = math.floor(max(uc) + eu) + 1, math.floor(max(vc) + ev) + 1
            assert ub - ua + 1 <= f["ru"] and vb - va + 1 <= f["rv"]
            wt = np.zeros((ub - ua + 1, vb - va + 1))
            for u in range(max(ua, 0), min(ub, H - 1) + 1):
                for v in range(max(va, 0), min(vb, W - 1) + 1):
                    acc = 0.0
                    for i in range(h):
                        al = u - s * i + R
                        if not 0 <= al < Q:
                            continue
                        for j in range(w):
                            be = v - s * j + R
                            if 0 <= be < Q:
                                acc += f["C"][al, be] * r[i, j]
                    wt[u - ua, v - va] = acc
            for pr in range(U0, U1 + 1):
                for pc in range(V0, V1 + 1):
                    us = math.floor(g[0] * pr + g[1] * pc + g[2] - eu) + 1
                    vs = math.floor(g[3] * pr + g[4] * pc + g[5] - ev) + 1
                    assert ua <= us and us + f["ncu"] - 1 <= ub
                    assert va <= vs and vs + f["ncv"] - 1 <= vb
                    acc = 0.0
                    for a in range(f["ncu"]):
                        for b in range(f["ncv"]):
                            u, v = us + a, vs + b
                            dr = m[0] * u + m[1] * v + m[2] - pr
                            dc = m[3] * u + m[4] * v + m[5] - pc
                            acc += max(0, 1 - abs(dr)) * max(0, 1 - abs(dc)) * wt[u - ua, v - va]
                    x[pr, pc] += acc
    return x


CASES = [(20, 36, 2, 5, 0.03), (18, 27, 3, 3, 0.5), (16, 20, 4, 3, 1.2), (22, 70, 1, 3, 2.36)]


@pytest.mark.parametrize("H,W,s,P,theta", CASES)
def test_matrix_free_windows_reproduce_the_oracle(H, W, s, P, theta):
    rng = np.random.default_rng(H * W + P)
    m = _rot(theta, H, W, 0.37, -0.21)
    h2 = rng.uniform(0.1, 1.0, (P, P))
    h2 /= h2.sum()
    f = _plan(s, P, m, h2)
    x = rng.uniform(0, 1, (H, W))
    shifts, psf, warps = np.zeros((1, 2)), h2[None], m[None]
    y_o = oracle.forward(x, shifts, psf, s, warps=warps)[0]
    assert np.max(np.abs(_forward(x, s, f) - y_o)) <= 1e-12 * max(1.0, np.max(np.abs(y_o)))
    r = rng.standard_normal((H // s, W // s))
    x_o = oracle.adjoint(r[None], shifts, psf, s, H, W, warps=warps)
    x_m = _adjoint(r, s, H, W, f)
    assert np.max(np.abs(x_m - x_o)) <= 1e-12 * max(1.0, np.max(np.abs(x_o)))
