"""GPU SCG solves (device-resident Moller state machine, graph-replayed passes)
against the FP64 oracle's literal SCG, through the C ABI."""
import numpy as np
import pytest

import oracle
from oracle import scg as oscg
from gpu_common import TOL_LOWP, TOL_SCG, compare_traces, problem, psnr, rel_l2, to_dev, to_np

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
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _oracle_solve(prob, n_iter, **kw):
    return oscg.solve(_f32(prob.y), prob.shifts, prob.psf, prob.s, _f32(prob.x0), n_iter, **kw)


def _gpu_solve(misr, ctx, prob, n_iter, dtype=None, **kw):
    import torch
    dtype = dtype or torch.float32
    op = misr.Operator(ctx, prob.H, prob.W, prob.s, prob.shifts, prob.psf)
    x = to_dev(_f32(prob.x0), dtype)
    y = to_dev(_f32(prob.y), dtype)
    its, info = op.scg_solve(y, x, misr.default_params(n_iter=n_iter, **kw))
    return to_np(x), its, info


def test_plain128_solve_matches_oracle(misr, ctx):
    """The plain 128^2 workload: 4 frames 64^2, x2, 5x5 PSF sigma 0.6,
    Gaussian noise 0.01, lambda 0.01, 50 SCG passes from bicubic x0."""
    prob = problem(64, 2, 0.6, 5, noise=("gauss", 0.01), jitter=0.0, n_iter=50,
                   seeds=(0, 0, 1))
    x_o, tr_o, _ = _oracle_solve(prob, 50)
    x_g, its, info = _gpu_solve(misr, ctx, prob, 50)
    assert info["n_passes"] == 50 and info["stop"] == 0
    err = rel_l2(x_g, x_o)
    print(f"plain128 rel-L2 vs oracle {err:.3e}, PSNR vs gt {psnr(x_g, prob.x_gt):.2f} dB")
    assert err <= TOL_SCG
    compare_traces(its, tr_o)


@pytest.mark.parametrize("L,s,sig,jit,n_iter", [(48, 3, 1.0, 0.05, 30), (40, 2, 0.8, 0.05, 40),
                                                (52, 2, 0.8, 0.05, 25)])
def test_small_solves_match_oracle(misr, ctx, L, s, sig, jit, n_iter):
    prob = problem(L, s, sig, None, noise=("poisson", 1e4), jitter=jit, n_iter=n_iter,
                   seeds=(L, L + 1, L + 2))
    x_o, tr_o, _ = _oracle_solve(prob, n_iter)
    x_g, its, info = _gpu_solve(misr, ctx, prob, n_iter)
    err = rel_l2(x_g, x_o)
    print(f"L={L} s={s}: rel-L2 {err:.3e}")
    assert err <= TOL_SCG
    compare_traces(its, tr_o)


def test_zero_passes_returns_x0_and_cost(misr, ctx):
    prob = problem(32, 2, 0.6, 5, noise=("gauss", 0.01), jitter=0.0, seeds=(1, 1, 2))
    x_g, its, info = _gpu_solve(misr, ctx, prob, 0)
    assert info["n_passes"] == 0
    assert np.array_equal(x_g, _f32(prob.x0))
    J, _, _ = oracle.cost_grad(_f32(prob.x0), _f32(prob.y), prob.shifts, prob.psf, 2)
    assert abs(info["E0"] - J) <= 1e-5 * J


def test_one_pass_closed_form(misr, ctx):
    """s = 1, P = 1, no shift, lambda = 0: x1 = y + (x0 - y) lam1 / (2 + lam1)."""
    import torch
    rng = np.random.default_rng(4)
    H, W = 70, 90
    y = _f32(rng.uniform(0, 1, (1, H, W)))
    x0 = _f32(rng.uniform(0, 1, (H, W)))
    op = misr.Operator(ctx, H, W, 1, np.zeros((1, 2)), [1.0])
    x = to_dev(x0)
    op.scg_solve(to_dev(y), x, misr.default_params(n_iter=1, lambda_reg=0.0))
    lam1 = 1e-6
    ref = y[0] + (x0 - y[0]) * lam1 / (2 + lam1)
    assert np.max(np.abs(to_np(x) - ref)) <= 1e-6


@pytest.mark.parametrize("dtype_name", ["float16", "bfloat16"])
def test_lowp_storage_solve(misr, ctx, dtype_name):
    """Frames and image stored in 16 bits, FP32 iterate (x_work = 0): within
    1e-2 of the FP64 oracle solve on the FP32 inputs, so the bound covers the
    rounding of y and x0 to 16 bits as well as of the result."""
    import torch
    dt = getattr(torch, dtype_name)
    prob = problem(48, 3, 1.0, 7, noise=("poisson", 1e4), jitter=0.05, n_iter=60,
                   seeds=(3, 4, 5))
    x_o, _, _ = _oracle_solve(prob, 60)
    x_g, its, info = _gpu_solve(misr, ctx, prob, 60, dtype=dt)
    err = rel_l2(x_g, x_o)
    print(f"{dtype_name} storage, FP32 iterate: rel-L2 {err:.3e}, PSNR vs oracle "
          f"{psnr(x_g, x_o):.2f} dB")
    assert err <= TOL_LOWP


@pytest.mark.parametrize("dtype_name", ["float16", "bfloat16"])
def test_lowp_fp32_iterate_is_rounded_fp32_solve(misr, ctx, dtype_name):
    """With x_work = 0 a 16-bit solve is the FP32 solve of the widened inputs,
    rounded to nearest even once at the end: bit for bit."""
    import torch
    dt = getattr(torch, dtype_name)
    prob = problem(40, 2, 0.8, None, noise=("poisson", 1e4), jitter=0.05, n_iter=20,
                   seeds=(7, 8, 9))
    op = misr.Operator(ctx, prob.H, prob.W, prob.s, prob.shifts, prob.psf)
    y16, x16 = to_dev(_f32(prob.y), dt), to_dev(_f32(prob.x0), dt)
    y32, x32 = y16.float(), x16.float()
    op.scg_solve(y32, x32, misr.default_params(n_iter=20))
    op.scg_solve(y16, x16, misr.default_params(n_iter=20))
    assert torch.equal(x16, x32.to(dt))


@pytest.mark.parametrize("dtype_name,x_rounding", [("float16", 0), ("float16", 1),
                                                   ("bfloat16", 0), ("bfloat16", 1)])
def test_lowp_iterate_in_storage(misr, ctx, dtype_name, x_rounding):
    """x_work = 1 keeps the iterate itself in 16 bits (x updates rounded on
    store, the trial point rounded the same way).  Steps below half a unit in
    the last place are lost, so the solve stalls short of the FP64 result;
    the error is reported, and bounded only loosely."""
    import torch
    dt = getattr(torch, dtype_name)
    prob = problem(48, 3, 1.0, 7, noise=("poisson", 1e4), jitter=0.05, n_iter=60,
                   seeds=(3, 4, 5))
    x_o, _, _ = _oracle_solve(prob, 60)
    x_g, its, info = _gpu_solve(misr, ctx, prob, 60, dtype=dt, x_work=1, x_rounding=x_rounding)
    err = rel_l2(x_g, x_o)
    print(f"{dtype_name} iterate in storage ({'stochastic' if x_rounding else 'nearest'}): "
          f"rel-L2 {err:.3e}, PSNR vs oracle {psnr(x_g, x_o):.2f} dB, "
          f"{info['n_success']} accepted")
    assert np.isfinite(x_g).all() and info["stop"] == 0
    assert err <= 0.2


def test_batch_equals_solo_and_oracle(misr, ctx):
    """Projections of different size and scale advanced in shared launches:
    each equals its own solo solve bit for bit, and the oracle within 1e-4."""
    import torch
    specs = [(40, 2, 0.8, 20), (30, 3, 1.0, 15), (56, 2, 0.8, 25), (24, 3, 1.0, 20)]
    probs = [problem(L, s, sig, None, jitter=0.05, n_iter=n, seeds=(i, i + 7, i + 9))
             for i, (L, s, sig, n) in enumerate(specs)]
    ops = [misr.Operator(ctx, p.H, p.W, p.s, p.shifts, p.psf) for p in probs]
    ys = [to_dev(_f32(p.y)) for p in probs]
    xs = [to_dev(_f32(p.x0)) for p in probs]
    prms = [misr.default_params(n_iter=n) for (_, _, _, n) in specs]
    outs = misr.scg_solve_batch(ops, ys, xs, prms)
    for i, p in enumerate(probs):
        xsolo = to_dev(_f32(p.x0))
        its, info = ops[i].scg_solve(ys[i], xsolo, misr.default_params(n_iter=specs[i][3]))
        assert torch.equal(xsolo, xs[i]), f"projection {i} differs from its solo solve"
        assert outs[i][1]["n_passes"] == specs[i][3]
        x_o, tr_o, _ = _oracle_solve(p, specs[i][3])
        assert rel_l2(to_np(xs[i]), x_o) <= TOL_SCG


def test_batch_mixing_tile_variants(misr, ctx):
    """Operators on different tile variants (0, the narrow 1, and 2 with its
    wider trial tiles) in one batch: one launch per (scale, band, variant)
    class, and every projection equals its solo solve bit for bit."""
    import torch
    specs = [(56, 2, 0.8, 20, 2), (40, 2, 0.8, 15, 1), (48, 2, 0.8, 20, 0), (30, 3, 1.0, 15, 1)]
    probs = [problem(L, s, sig, None, jitter=0.05, n_iter=n, seeds=(i + 3, i + 5, i + 8))
             for i, (L, s, sig, n, _) in enumerate(specs)]
    ops = [misr.Operator(ctx, p.H, p.W, p.s, p.shifts, p.psf) for p in probs]
    for op, sp in zip(ops, specs):
        op.set_tile(sp[4])
    ys = [to_dev(_f32(p.y)) for p in probs]
    xs = [to_dev(_f32(p.x0)) for p in probs]
    prms = [misr.default_params(n_iter=sp[3]) for sp in specs]
    misr.scg_solve_batch(ops, ys, xs, prms, trace=False)
    for i, p in enumerate(probs):
        xsolo = to_dev(_f32(p.x0))
        ops[i].scg_solve(ys[i], xsolo, misr.default_params(n_iter=specs[i][3]), trace=False)
        torch.cuda.synchronize()
        assert torch.equal(xsolo, xs[i]), f"projection {i} (variant {specs[i][4]}) differs"
    for op in ops:
        op.close()


def test_repeat_solves_deterministic(misr, ctx):
    import torch
    prob = problem(64, 2, 0.8, None, jitter=0.05, n_iter=20, seeds=(9, 9, 9))
    op = misr.Operator(ctx, prob.H, prob.W, 2, prob.shifts, prob.psf)
    y = to_dev(_f32(prob.y))
    outs = []
    for _ in range(3):
        x = to_dev(_f32(prob.x0))
        op.scg_solve(y, x, misr.default_params(n_iter=20), trace=False)
        torch.cuda.synchronize()
        outs.append(x.clone())
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[1], outs[2])


def test_nonfinite_input_stops_with_numeric(misr, ctx):
    prob = problem(32, 2, 0.6, 5, noise=("gauss", 0.01), jitter=0.0, seeds=(2, 2, 3))
    y = _f32(prob.y)
    y[1, 3, 4] = np.nan
    op = misr.Operator(ctx, prob.H, prob.W, 2, prob.shifts, prob.psf)
    x = to_dev(_f32(prob.x0))
    its, info = op.scg_solve(to_dev(y), x, misr.default_params(n_iter=10))
    assert info["stop"] == 2 and info["status"] == "E_NUMERIC"
    assert np.all(np.isfinite(to_np(x)))


def test_nonfinite_stop_reported_without_trace(misr, ctx):
    """A solve run without a trace returns at once (asynchronous); its
    non-finite stop is reported by misr_scg_status (E_NUMERIC, stop 2), and a
    later finite solve on the same operator reports OK."""
    import torch
    prob = problem(32, 2, 0.6, 5, noise=("gauss", 0.01), jitter=0.0, seeds=(2, 2, 3))
    y_bad = _f32(prob.y)
    y_bad[2, 5, 1] = np.nan
    op = misr.Operator(ctx, prob.H, prob.W, 2, prob.shifts, prob.psf)
    with pytest.raises(misr.MisrError):
        op.scg_status()   # no solve yet
    x = to_dev(_f32(prob.x0))
    assert op.scg_solve(to_dev(y_bad), x, misr.default_params(n_iter=10), trace=False) is None
    # a cost/gradient call in between does not change the report
    op.cost_grad(x, to_dev(_f32(prob.y)))
    st = op.scg_status()
    assert st["status"] == "E_NUMERIC" and st["stop"] == 2
    assert np.all(np.isfinite(to_np(x)))
    x = to_dev(_f32(prob.x0))
    op.scg_solve(to_dev(_f32(prob.y)), x, misr.default_params(n_iter=10), trace=False)
    st = op.scg_status(torch.cuda.current_stream())
    assert st["status"] == "OK" and st["stop"] == 0 and st["n_passes"] == 10


@pytest.mark.parametrize("eps_data", [1e-2, 1e-3])
def test_l1_data_solve_matches_oracle(misr, ctx, eps_data):
    """Eq. misr with p = 1 (Charbonnier-smoothed L1 data term): the device
    solve, whose update pass takes the closed-form L1 curvature, against the
    oracle's literal SCG (finite-difference curvature): image, success
    sequence and cost per pass."""
    n = 20
    prob = problem(40, 2, 0.8, None, noise=("poisson", 1e4), jitter=0.05, n_iter=n,
                   seeds=(11, 12, 13))
    x_o, tr_o, _ = _oracle_solve(prob, n, data_p=1, eps_data=eps_data)
    x_g, its, info = _gpu_solve(misr, ctx, prob, n, data_p=1, eps_data=eps_data)
    err = rel_l2(x_g, x_o)
    print(f"L1 data term, eps_data {eps_data}: rel-L2 {err:.3e}, {info['n_success']} accepted")
    assert err <= TOL_SCG
    compare_traces(its, tr_o)


def test_zero_gradient_start_stops_at_once(misr, ctx):
    """Degenerate case of Moller's method: a constant image that fits the
    frames exactly (x0 = 0, y = 0) has r = -grad J(x0) = 0 (zero residual, and
    the prior's psi(0) = 0), so the solve stops at the first pass (stop = 1)
    and returns x0 unchanged.  E0 is the prior's phi(0) = 0 evaluated in FP32
    per pair, exact up to rounding of eps (below n lambda eps 1e-6)."""
    import torch
    from paper_2108_04315_amd import synth
    H = W = 48
    op = misr.Operator(ctx, H, W, 2, synth.frame_shifts(2, 4, 0.05, 3), synth.psf_taps(0.8, 7))
    y = torch.zeros((4, H // 2, W // 2), device="cuda")
    x = torch.zeros((H, W), device="cuda")
    its, info = op.scg_solve(y, x, misr.default_params(n_iter=10))
    torch.cuda.synchronize()
    assert info["stop"] == 1 and info["n_success"] == 0
    assert 0.0 <= info["E0"] <= H * W * 0.01 * 1e-3 * 1e-6
    assert info["status"] == "OK" and not torch.any(x != 0)


def test_no_prior_and_single_frame_identity(misr, ctx):
    """lambda = 0 (pure least squares, Eq. l2misr) at scale 2, and the
    degenerate geometry s = 1, K = 1, P = 1 with no shift (A = I): both
    against the oracle's literal SCG.  The identity case converges to FP32
    resolution within about eight passes (later accept decisions then hinge
    on cost differences below FP32 rounding), so it runs six."""
    prob = problem(48, 2, 0.8, None, jitter=0.05, n_iter=20, seeds=(4, 5, 6))
    xg, its, _ = _gpu_solve(misr, ctx, prob, 20, lambda_reg=0.0)
    xo, tr, _ = _oracle_solve(prob, 20, lambda_reg=0.0)
    assert rel_l2(xg, xo) <= TOL_SCG
    compare_traces(its, tr)
    rng = np.random.default_rng(12)
    y = _f32(rng.uniform(0, 1, (1, 40, 36)))
    x0 = _f32(np.full((40, 36), 0.5))
    op = misr.Operator(ctx, 40, 36, 1, np.zeros((1, 2)), np.array([1.0]))
    x = to_dev(x0)
    its, _ = op.scg_solve(to_dev(y), x, misr.default_params(n_iter=6))
    xo, tr, _ = oscg.solve(y, np.zeros((1, 2)), np.array([1.0]), 1, x0, 6)
    assert rel_l2(to_np(x), xo) <= TOL_SCG
    compare_traces(its, tr)
