"""Parity at the full workload sizes, in the launch configuration bench.py
times: the fused cost + gradient over a whole 2048^2 (x2, 4 frames) and
6144^2 (x3, 9 frames) image against the FP64 oracle element by element, and
the first SCG passes of the 2048^2 solve against the oracle's."""
import numpy as np
import pytest

import oracle
from oracle import scg as oscg
from gpu_common import TOL_OP, TOL_SCG, problem, rel_l2, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def misr():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2108_04315_amd import misr as m
    return m


@pytest.fixture(scope="module")
def ctx(misr):
    c = misr.Context(0)
    yield c
    c.close()


def _f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


@pytest.fixture(scope="module")
def plain2048():
    # 4 LR frames 1024^2 -> 2048^2 HR, 7x7 PSF sigma 0.8, Poisson 1e4, jittered shifts
    return problem(1024, 2, 0.8, None, noise=("poisson", 1e4), jitter=0.05, n_iter=100,
                   seeds=(1, 2, 3))


def test_cost_grad_full_2048(misr, ctx, plain2048):
    import torch
    p = plain2048
    op = misr.Operator(ctx, p.H, p.W, p.s, p.shifts, p.psf)
    y = _f32(p.y)
    rng = np.random.default_rng(4)
    for x in (_f32(p.x0), _f32(p.x0 + 0.01 * rng.standard_normal(p.x0.shape))):
        J, g_ref, parts = oracle.cost_grad(x, y, p.shifts, p.psf, p.s)
        cost, g = op.cost_grad(to_dev(x), to_dev(y))
        torch.cuda.synchronize()
        c = cost.cpu().numpy()
        err = rel_l2(to_np(g), g_ref)
        print(f"2048^2 cost rel err {abs(c[0] - J) / J:.2e}, gradient rel-L2 {err:.2e}")
        assert abs(c[0] - J) <= TOL_OP * J
        assert err <= TOL_OP


def test_scg_first_passes_full_2048(misr, ctx, plain2048):
    """Ten SCG passes of the 2048^2 solve (one captured graph, as bench.py
    runs it) against the oracle's ten passes: image and per-pass record."""
    p = plain2048
    n = 10
    x_o, tr_o, _ = oscg.solve(_f32(p.y), p.shifts, p.psf, p.s, _f32(p.x0), n)
    op = misr.Operator(ctx, p.H, p.W, p.s, p.shifts, p.psf)
    x = to_dev(_f32(p.x0))
    its, info = op.scg_solve(to_dev(_f32(p.y)), x, misr.default_params(n_iter=n))
    err = rel_l2(to_np(x), x_o)
    print(f"2048^2 after {n} passes: rel-L2 {err:.2e}")
    assert err <= TOL_SCG
    assert [t["success"] for t in its] == [t["success"] for t in tr_o]
    for a, b in zip(its, tr_o):
        assert abs(a["E"] - b["E"]) <= 1e-5 * abs(b["E"])


@pytest.mark.parametrize("dtype_name", ["float32", "bfloat16"])
def test_cost_grad_full_6144(misr, ctx, dtype_name):
    """9 LR frames 2048^2 -> 6144^2 HR (x3), PSF sigma 1.0: the precision
    workload's image, FP32 and bf16 storage (the oracle gets the same stored
    values, so the bound is the FP32 one)."""
    import torch
    dt = getattr(torch, dtype_name)
    p = problem(2048, 3, 1.0, None, noise=("poisson", 1e4), jitter=0.05, n_iter=100,
                seeds=(5, 6, 7))
    op = misr.Operator(ctx, p.H, p.W, p.s, p.shifts, p.psf)
    # stored values, rounded on the host: the oracle reads exactly what the device holds
    xh = torch.from_numpy(_f32(p.x0)).to(dt)
    yh = torch.from_numpy(_f32(p.y)).to(dt)
    xd, yd = xh.cuda(), yh.cuda()
    J, g_ref, _ = oracle.cost_grad(xh.double().numpy(), yh.double().numpy(), p.shifts, p.psf,
                                   p.s)
    cost, g = op.cost_grad(xd, yd)
    torch.cuda.synchronize()
    c = cost.cpu().numpy()
    err = rel_l2(to_np(g), g_ref)
    print(f"6144^2 {dtype_name}: cost rel err {abs(c[0] - J) / J:.2e}, gradient rel-L2 {err:.2e}")
    assert abs(c[0] - J) <= TOL_OP * J
    assert err <= TOL_OP
