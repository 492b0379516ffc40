"""Writes the FP64 oracle's SCG results at the full workload sizes, for the
full-size parity tests (tests/test_gpu_fullsize.py) and the benchmark's
oracle leg.

    python tests/golden/make_fullsize_refs.py [--out DIR] [name ...]   (default: all)

Every input is drawn by the seeded generator (paper_2108_04315_amd.synth)
with clean frames from the oracle's own forward operator, rounded to float32
(what the FP32 GPU path receives), and solved by the oracle's literal SCG
(Moller's method with the finite-difference curvature) for the workload's
pass count, on at most OMP_NUM_THREADS host threads.  Nothing here calls the
HIP library.  Outputs go to tests/golden/fullsize/<name>.npz, or to DIR
(not tracked: 2-17 MB each):

  x        the oracle image (float32), whole for plain2048, else at `idx`
  idx      sorted flat pixel indices of the sample (int32; absent when whole)
  trace    per pass: E, E_t, delta, mu, alpha, Delta, lam, success (float64)
  y_sha    sha256 of the float32 frames, so a reader can check it regenerated
           the same inputs
  norm_x   ||x_oracle||_2 over the whole image; err_gt ||x_oracle - x_gt||_2
  meta     the recipe (JSON)

Workloads: plain2048 (4 LR frames 1024^2, x2, PSF sigma 0.8, 100 passes),
precision6144 (9 LR frames 2048^2, x3, sigma 1.0, 100 passes) and one
projection per (LR size, scale) class of the batched workload (LR
{512, 768, 1024, 1536, 2048}^2, x2 with 4 frames or x3 with 9, sigma 0.8,
60 passes); Poisson noise at 1e4 mean counts and +-0.05 LR-px jitter
throughout.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "fullsize")
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

TRACE_KEYS = ("E", "E_t", "delta", "mu", "alpha", "Delta", "lam", "success")


def specs():
    """name -> recipe (LR side L, scale s, PSF sigma, passes, seeds, sample size;
    sample 0 keeps the whole image)."""
    out = {
        "plain2048": dict(L=1024, s=2, sigma=0.8, n_iter=100, seeds=(1, 2, 3), sample=0),
        "precision6144": dict(L=2048, s=3, sigma=1.0, n_iter=100, seeds=(5, 6, 7),
                              sample=1 << 20),
    }
    for L in (512, 768, 1024, 1536, 2048):
        for s in (2, 3):
            out[f"batched_{L}x{s}"] = dict(L=L, s=s, sigma=0.8, n_iter=60,
                                           seeds=(3000 + L + s, 3001 + L + s, 3002 + L + s),
                                           sample=1 << 18)
    return out


def inputs(spec):
    """The workload's inputs as the FP32 path receives them (float64 arrays
    holding float32 values) and the sha256 of the float32 frames."""
    import oracle
    from paper_2108_04315_amd import synth
    p = synth.make_problem(oracle.forward, L=spec["L"], s=spec["s"], sigma=spec["sigma"],
                           P=None, noise=("poisson", 1e4), jitter=0.05,
                           n_iter=spec["n_iter"], seeds=tuple(spec["seeds"]))
    y32 = np.ascontiguousarray(p.y, dtype=np.float32)
    x032 = np.ascontiguousarray(p.x0, dtype=np.float32)
    sha = hashlib.sha256(y32.tobytes()).hexdigest()
    return p, y32.astype(np.float64), x032.astype(np.float64), sha


def sample_idx(n: int, m: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.unique(rng.integers(0, n, m, dtype=np.int64)).astype(np.int32)


def path(name: str) -> str:
    return os.path.join(OUT, name + ".npz")


def load(name: str):
    """The stored reference as a dict, or None if it has not been written."""
    f = path(name)
    if not os.path.exists(f):
        return None
    with np.load(f, allow_pickle=False) as z:
        d = {k: z[k] for k in z.files}
    d["meta"] = json.loads(str(d["meta"]))
    return d


def make(name: str, spec: dict, threads: int) -> None:
    import oracle
    from oracle import scg as oscg
    oracle.set_threads(threads)
    t0 = time.perf_counter()
    p, y, x0, sha = inputs(spec)
    t1 = time.perf_counter()
    print(f"{name}: inputs {p.H}x{p.W}, K={p.K} in {t1 - t0:.1f} s; solving "
          f"{spec['n_iter']} passes", flush=True)
    def progress(n):
        if n % 10 == 0:
            print(f"{name}: {n} evaluations, {time.perf_counter() - t1:.0f} s", flush=True)
    x, recs, _ = oscg.solve(y, p.shifts, p.psf, p.s, x0, spec["n_iter"], progress=progress)
    t2 = time.perf_counter()
    trace = np.array([[r[k] for k in TRACE_KEYS] for r in recs], dtype=np.float64)
    out = dict(trace=trace, y_sha=np.array(sha), norm_x=np.array(np.linalg.norm(x)),
               err_gt=np.array(np.linalg.norm(x - p.x_gt)))
    if spec["sample"]:
        idx = sample_idx(x.size, spec["sample"], seed=int(spec["seeds"][0]) + 77)
        out["idx"] = idx
        out["x"] = x.ravel()[idx].astype(np.float32)
    else:
        out["x"] = x.astype(np.float32)
    meta = dict(spec, name=name, H=p.H, W=p.W, K=p.K, passes=len(recs),
                n_success=int(sum(r["success"] for r in recs)), oracle_threads=threads,
                oracle_solve_s=t2 - t1, inputs="synth.make_problem with oracle.forward, "
                "Poisson 1e4, jitter 0.05, P = 2 ceil(3 sigma) + 1; float32-rounded y, x0")
    out["meta"] = np.array(json.dumps(meta))
    os.makedirs(OUT, exist_ok=True)
    tmp = path(name) + ".tmp.npz"
    np.savez_compressed(tmp, **out)
    os.replace(tmp, path(name))
    print(f"{name}: done in {t2 - t1:.1f} s ({len(recs)} passes, "
          f"{meta['n_success']} accepted)", flush=True)


def main(argv):
    global OUT
    if argv[:1] == ["--out"]:
        OUT, argv = os.path.abspath(argv[1]), argv[2:]
    todo = argv or list(specs())
    threads = len(os.sched_getaffinity(0))
    threads = min(threads, int(os.environ.get("OMP_NUM_THREADS", threads)))
    sp = specs()
    for name in todo:
        make(name, sp[name], threads)


if __name__ == "__main__":
    main(sys.argv[1:])
