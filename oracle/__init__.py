"""FP64 CPU checker for the MISR SCG hot path.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product library never imports,
links or runs anything in this package, and this package never imports the
product.

``ops``  -- ctypes shim over ``misr_oracle.c``: the literal 2-D operators
           (bilinear warp, translational or affine; P x P blur; s x s
           binning), J(x) and grad J(x).
``scg``  -- Moller's scaled conjugate gradient, step by step, in numpy.
``partition`` -- the objective split into subdomains that each own a
           rectangle of pixels (the paper's distributed decomposition), and
           the SCG driven by the subdomains' local costs, gradients and
           inner products.
"""
from .ops import (build, forward, adjoint, cost_grad, btv, btv_owned, curvature_exact, curvature_data_l1,
                  interpolate, upsample,
                  psi_quotient, num_threads, set_threads, warp, warp_T, warp_affine,
                  warp_affine_T, blur, blur_T, bin_, bin_T)
from .scg import scg_minimize, solve, moller_scale_delta, moller_update_lambda

__all__ = ["build", "forward", "adjoint", "cost_grad", "btv", "btv_owned", "curvature_exact",
           "curvature_data_l1", "interpolate", "upsample",
           "psi_quotient", "num_threads", "set_threads", "warp", "warp_T", "warp_affine",
           "warp_affine_T", "blur",
           "blur_T", "bin_", "bin_T", "scg_minimize", "solve", "moller_scale_delta", "moller_update_lambda"]
