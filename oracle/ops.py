"""ctypes shim over the FP64 oracle library (test infrastructure only).

Each function takes and returns float64 numpy arrays and forwards to the plain
C definitions in ``misr_oracle.c``.  Shapes: HR images (H, W); LR frames
(K, H//s, W//s); shifts (K, 2) as (dx, dy) in LR pixels; psf the 1-D taps whose
outer product is the 2-D PSF, or per-frame PSFs (see psf_frames); warps None
(translations from shifts) or (K, 6) affine coefficients per frame: frame k
samples x at row m0 u + m1 v + m2, column m3 u + m4 v + m5 (HR pixels).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "misr_oracle.c")
# MISR_ORACLE_SANITIZE=1 loads a build instrumented with AddressSanitizer and
# UndefinedBehaviorSanitizer (run under LD_PRELOAD of libasan; see build())
_SAN = os.environ.get("MISR_ORACLE_SANITIZE") == "1"
_LIB = os.path.join(_HERE, "libmisr_oracle_san.so" if _SAN else "libmisr_oracle.so")
_lib = None

_D = ctypes.c_double
_I = ctypes.c_int
_P = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True, sanitize: bool = _SAN) -> str:
    """Compile the oracle with gcc (OpenMP, -O2, no fast-math).  sanitize:
    the AddressSanitizer + UndefinedBehaviorSanitizer build
    (libmisr_oracle_san.so), which a process loads with
    MISR_ORACLE_SANITIZE=1 and LD_PRELOAD=$(gcc -print-file-name=libasan.so)."""
    lib = os.path.join(_HERE, "libmisr_oracle_san.so" if sanitize else "libmisr_oracle.so")
    if force or not os.path.exists(lib):
        tmp = lib + ".tmp"
        flags = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                 "-fno-omit-frame-pointer"] if sanitize else ["-O2"]
        subprocess.check_call(["gcc"] + flags + ["-fopenmp", "-fPIC", "-shared",
                                                 "-fno-fast-math", "-ffp-contract=off",
                                                 "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, lib)
    return lib


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    sig = {
        "orc_warp": [_I, _I, _D, _D, _P, _P],
        "orc_warp_T": [_I, _I, _D, _D, _P, _P],
        "orc_blur": [_I, _I, _I, _P, _P, _P],
        "orc_blur_T": [_I, _I, _I, _P, _P, _P],
        "orc_bin": [_I, _I, _I, _P, _P],
        "orc_bin_T": [_I, _I, _I, _P, _P],
        "orc_forward": [_I, _I, _I, _I, _P, _I, _P, _P, _P],
        "orc_forward_w": [_I, _I, _I, _I, _P, _P, _I, _P, _P, _P],
        "orc_adjoint_w": [_I, _I, _I, _I, _P, _P, _I, _P, _P, _P],
        "orc_warp_affine": [_I, _I, _P, _P, _P],
        "orc_warp_affine_T": [_I, _I, _P, _P, _P],
        "orc_cost_grad_w": [_I, _I, _I, _I, _P, _P, _I, _P, _D, _D, _D, _I, _I, _D, _P, _P,
                            _P, _P],
        "orc_adjoint": [_I, _I, _I, _I, _P, _I, _P, _P, _P],
        "orc_btv": [_I, _I, _D, _D, _D, _I, _P, _P],
        "orc_btv_owned": [_I, _I, _D, _D, _D, _I, _P, _I, _I, _I, _I, _P],
        "orc_cost_grad": [_I, _I, _I, _I, _P, _I, _P, _D, _D, _D, _I, _I, _D, _P, _P,
                          _P, _P],
        "orc_psi_quotient": [_D, _D, _D],
        "orc_curv_exact": [_I, _I, _I, _I, _P, _I, _P, _D, _D, _D, _I, _D, _P, _P, _P],
        "orc_curv_data_l1": [_I, _I, _I, _I, _P, _I, _P, _D, _D, _P, _P, _P],
        "orc_interpolate": [_I, _I, _I, _I, _P, _P, _P],
        "orc_upsample": [_I, _I, _I, _P, _P],
        "orc_num_threads": [],
        "orc_set_threads": [_I],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = None
    lib.orc_btv.restype = _D
    lib.orc_btv_owned.restype = _D
    lib.orc_cost_grad.restype = _D
    lib.orc_cost_grad_w.restype = _D
    lib.orc_psi_quotient.restype = _D
    lib.orc_curv_exact.restype = _D
    lib.orc_curv_data_l1.restype = _D
    lib.orc_num_threads.restype = _I
    _lib = lib
    return lib


def psf_frames(psf, K):
    """Each frame's P x P PSF as a (K, P, P) array (the blur B_k of frame k,
    Eq. sisr with A_k = D B_k M_k).  psf: (P,) taps shared by both axes and
    all frames (2-D PSF = outer product); (P, P) one 2-D PSF for all frames;
    (K, 2, P) per frame, row taps then column taps; (K, P, P) per frame."""
    psf = np.asarray(psf, dtype=np.float64)
    if psf.ndim == 1:
        return np.ascontiguousarray(np.broadcast_to(np.outer(psf, psf), (K,) + (psf.size,) * 2))
    if psf.ndim == 2:
        return np.ascontiguousarray(np.broadcast_to(psf, (K,) + psf.shape))
    if psf.shape[1] == 2 and psf.shape[2] != 2:
        return np.ascontiguousarray(np.einsum("ka,kb->kab", psf[:, 0], psf[:, 1]))
    return np.ascontiguousarray(psf)


def _p(a):
    return None if a is None else a.ctypes.data_as(_P)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return _load().orc_num_threads()


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def warp(x, tx, ty):
    x = _f64(x)
    out = np.empty_like(x)
    _load().orc_warp(x.shape[0], x.shape[1], tx, ty, _p(x), _p(out))
    return out


def warp_T(z, tx, ty):
    z = _f64(z)
    out = np.empty_like(z)
    _load().orc_warp_T(z.shape[0], z.shape[1], tx, ty, _p(z), _p(out))
    return out


def warp_affine(x, m):
    """Affine bilinear warp of one image: six coefficients m (general M_k)."""
    x, m = _f64(x), _f64(m)
    out = np.empty_like(x)
    _load().orc_warp_affine(x.shape[0], x.shape[1], _p(m), _p(x), _p(out))
    return out


def warp_affine_T(z, m):
    z, m = _f64(z), _f64(m)
    out = np.empty_like(z)
    _load().orc_warp_affine_T(z.shape[0], z.shape[1], _p(m), _p(z), _p(out))
    return out


def _warps(warps, K):
    if warps is None:
        return None
    w = _f64(warps).reshape(K, 6)
    return np.ascontiguousarray(w)


def blur(z, psf):
    z, psf = _f64(z), psf_frames(psf, 1)[0]
    out = np.empty_like(z)
    _load().orc_blur(z.shape[0], z.shape[1], psf.shape[0], _p(psf), _p(z), _p(out))
    return out


def blur_T(w, psf):
    w, psf = _f64(w), psf_frames(psf, 1)[0]
    out = np.empty_like(w)
    _load().orc_blur_T(w.shape[0], w.shape[1], psf.shape[0], _p(psf), _p(w), _p(out))
    return out


def bin_(z, s):
    z = _f64(z)
    out = np.empty((z.shape[0] // s, z.shape[1] // s))
    _load().orc_bin(z.shape[0], z.shape[1], s, _p(z), _p(out))
    return out


def bin_T(r, s, H, W):
    r = _f64(r)
    out = np.empty((H, W))
    _load().orc_bin_T(H, W, s, _p(r), _p(out))
    return out


def forward(x, shifts, psf, s, warps=None):
    """y_k = D B M_k x for every frame; returns (K, H//s, W//s)."""
    x, shifts = _f64(x), _f64(shifts)
    H, W = x.shape
    K = shifts.shape[0]
    psf = psf_frames(psf, K)
    wp = _warps(warps, K)
    y = np.empty((K, H // s, W // s))
    _load().orc_forward_w(H, W, s, K, _p(shifts), _p(wp), psf.shape[1], _p(psf), _p(x), _p(y))
    return y


def adjoint(r, shifts, psf, s, H, W, warps=None):
    """sum_k A_k^T r_k; returns (H, W)."""
    r, shifts = _f64(r), _f64(shifts)
    K = shifts.shape[0]
    psf = psf_frames(psf, K)
    wp = _warps(warps, K)
    x = np.empty((H, W))
    _load().orc_adjoint_w(H, W, s, K, _p(shifts), _p(wp), psf.shape[1], _p(psf), _p(r), _p(x))
    return x


def btv(x, lambda_reg=0.01, alpha_btv=0.4, eps=1e-3, w=3, grad=True):
    x = _f64(x)
    g = np.zeros_like(x) if grad else None
    E = _load().orc_btv(x.shape[0], x.shape[1], lambda_reg, alpha_btv, eps, w, _p(x), _p(g))
    return (E, g) if grad else E


def btv_owned(x, rect, lambda_reg=0.01, alpha_btv=0.4, eps=1e-3, w=3):
    """The BTV pairs one subdomain owns: first pixel in rect = (u0, u1, v0, v1),
    both pixels in the grid.  Returns (E, gradient of that part)."""
    x = _f64(x)
    g = np.zeros_like(x)
    u0, u1, v0, v1 = (int(v) for v in rect)
    E = _load().orc_btv_owned(x.shape[0], x.shape[1], lambda_reg, alpha_btv, eps, w, _p(x),
                              u0, u1, v0, v1, _p(g))
    return E, g


def cost_grad(x, y, shifts, psf, s, lambda_reg=0.01, alpha_btv=0.4, eps=1e-3, w=3,
              data_p=2, eps_data=1e-3, grad=True, warps=None):
    """Returns (J, grad J or None, (E_data, E_reg))."""
    x, y, shifts = _f64(x), _f64(y), _f64(shifts)
    H, W = x.shape
    K = shifts.shape[0]
    psf = psf_frames(psf, K)
    wp = _warps(warps, K)
    g = np.empty_like(x) if grad else None
    parts = np.zeros(2)
    J = _load().orc_cost_grad_w(H, W, s, K, _p(shifts), _p(wp), psf.shape[1], _p(psf),
                                lambda_reg, alpha_btv, eps, w, data_p, eps_data, _p(x), _p(y),
                                _p(g), _p(parts))
    return J, g, (float(parts[0]), float(parts[1]))


def psi_quotient(b, h, eps):
    return _load().orc_psi_quotient(float(b), float(h), float(eps))


def interpolate(y, shifts, s):
    """Multi-image interpolation of the K frames y (K, h, w) onto the HR grid."""
    y, shifts = _f64(y), _f64(shifts)
    K, h, w = y.shape
    x = np.empty((h * s, w * s))
    _load().orc_interpolate(h * s, w * s, s, K, _p(shifts), _p(y), _p(x))
    return x


def upsample(lr, s):
    """Keys bicubic upsampling (a = -1/2) of one LR frame by s."""
    lr = _f64(lr)
    h, w = lr.shape
    x = np.empty((h * s, w * s))
    _load().orc_upsample(h * s, w * s, s, _p(lr), _p(x))
    return x


def curvature_data_l1(x, p, y, shifts, psf, s, sk, eps_data=1e-3):
    """Data part of p^T (grad J(x + sk p) - grad J(x)) / sk for the
    Charbonnier L1 data term, closed form."""
    x, p, y, shifts = _f64(x), _f64(p), _f64(y), _f64(shifts)
    H, W = x.shape
    psf = psf_frames(psf, shifts.shape[0])
    return _load().orc_curv_data_l1(H, W, s, shifts.shape[0], _p(shifts), psf.shape[1], _p(psf),
                                    eps_data, sk, _p(x), _p(p), _p(y))


def curvature_exact(x, p, shifts, psf, s, sk, lambda_reg=0.01, alpha_btv=0.4, eps=1e-3,
                    w=3):
    """p^T (grad J(x + sk p) - grad J(x)) / sk for the L2 data term, closed form.

    Returns (delta, (data part, BTV part))."""
    x, p, shifts = _f64(x), _f64(p), _f64(shifts)
    H, W = x.shape
    psf = psf_frames(psf, shifts.shape[0])
    parts = np.zeros(2)
    d = _load().orc_curv_exact(H, W, s, shifts.shape[0], _p(shifts), psf.shape[1], _p(psf),
                               lambda_reg, alpha_btv, eps, w, sk, _p(x), _p(p), _p(parts))
    return d, (float(parts[0]), float(parts[1]))
