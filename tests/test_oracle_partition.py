"""Pins of the oracle's subdomain decomposition (Sec. 3.1, Eq. subfunction,
Eq. reformulated): the local objectives of subdomains that own disjoint
rectangles sum to the global objective, their assembled gradients to the
global gradient, and the solve driven by them reaches the undivided solve's
image.  A halo below the operator's reach breaks the sums (so the check can
fail)."""
import numpy as np
import pytest

import oracle
from oracle import partition
from oracle import scg as oscg
from gpu_common import problem

# (LR h, LR w, scale, PSF sigma, tile HR px, halo LR px): ragged last tiles
CASES = [(22, 19, 2, 0.8, 16, 4), (14, 17, 3, 1.0, 18, 3), (20, 20, 2, 0.6, 12, 8)]


@pytest.mark.parametrize("L,Lw,s,sigma,T,halo", CASES)
@pytest.mark.parametrize("data_p", [2, 1])
def test_local_objectives_sum_to_global(L, Lw, s, sigma, T, halo, data_p):
    p = problem(L, s, sigma, None, noise=("poisson", 1e4), jitter=0.05, seeds=(7, 8, 9), Lw=Lw)
    rng = np.random.default_rng(3)
    x = p.x0 + 0.02 * rng.standard_normal(p.x0.shape)
    kw = dict(data_p=data_p, eps_data=1e-2)
    J, g, (Ed, Er) = oracle.cost_grad(x, p.y, p.shifts, p.psf, s, **kw)
    rects = partition.tiles(p.H, p.W, s, T)
    assert len(rects) > 3
    Jp, gp, parts = partition.cost_grad(x, p.y, p.shifts, p.psf, s, rects, halo, **kw)
    assert abs(sum(a for a, _ in parts) - Ed) <= 1e-13 * Ed
    assert abs(sum(b for _, b in parts) - Er) <= 1e-13 * Er
    assert abs(Jp - J) <= 1e-13 * J
    assert np.max(np.abs(gp - g)) <= 1e-13 * np.max(np.abs(g))


def test_ownership_covers_every_term_once():
    """Every HR pixel, every LR pixel and every prior pair has exactly one
    owner."""
    H, W, s, T = 46, 38, 2, 16
    rects = partition.tiles(H, W, s, T)
    cover = np.zeros((H, W), int)
    for u0, u1, v0, v1 in rects:
        cover[u0:u1, v0:v1] += 1
        assert u0 % s == 0 and v0 % s == 0 and u1 % s == 0 and v1 % s == 0
    assert np.all(cover == 1)


def test_halo_below_reach_breaks_the_sum():
    """With no overlap the owned LR pixels near a border are evaluated on the
    window's zero padding: the sum no longer equals the global objective."""
    p = problem(22, 2, 0.8, None, noise=("poisson", 1e4), jitter=0.05, seeds=(7, 8, 9), Lw=19)
    J, g, _ = oracle.cost_grad(p.x0, p.y, p.shifts, p.psf, 2)
    rects = partition.tiles(p.H, p.W, 2, 16)
    Jp, gp, _ = partition.cost_grad(p.x0, p.y, p.shifts, p.psf, 2, rects, 0)
    assert abs(Jp - J) > 1e-6 * J
    assert np.max(np.abs(gp - g)) > 1e-6 * np.max(np.abs(g))


@pytest.mark.parametrize("L,Lw,s,sigma,T,halo", CASES[:2])
def test_partitioned_solve_equals_global(L, Lw, s, sigma, T, halo):
    """25 passes of the subdomain-driven solve against the undivided solve:
    the same accepted steps and the same image to rounding (x_tiled =
    x_untiled).  The two differ only in summation order (~1e-16 relative per
    sum); the literal finite-difference curvature divides a gradient
    difference by sigma / |p| (~1e-6 here), which lifts that to ~1e-9 in delta
    and ~1e-11 in the cost and the image, hence the bounds."""
    p = problem(L, s, sigma, None, noise=("poisson", 1e4), jitter=0.05, seeds=(7, 8, 9), Lw=Lw)
    n = 25
    x_g, tr_g, _ = oscg.solve(p.y, p.shifts, p.psf, s, p.x0, n)
    x_p, tr_p, _ = partition.solve(p.y, p.shifts, p.psf, s, p.x0, n, T, halo)
    assert [t["success"] for t in tr_p] == [t["success"] for t in tr_g]
    for a, b in zip(tr_p, tr_g):
        assert abs(a["E"] - b["E"]) <= 1e-10 * abs(b["E"])
    err = np.linalg.norm(x_p - x_g) / np.linalg.norm(x_g)
    assert err <= 1e-9, err
