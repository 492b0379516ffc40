"""ctypes binding over libmisr.so (the C ABI declared in include/misr.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  Device buffers are torch tensors on a ROCm device (only their
``data_ptr()`` is passed); streams are torch streams (``cuda_stream`` handle).
If the shared library is missing this module raises on import: there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
# torch first: libmisr.so must bind to the HIP runtime torch has loaded (its
# streams and device pointers are the ones passed in); loading the library
# first would bring a second HIP runtime into the process.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
# MISR_SANITIZE=1 loads the build whose host code carries AddressSanitizer
# and UndefinedBehaviorSanitizer (python -m paper_2108_04315_amd.build
# --sanitize; run under LD_PRELOAD of libasan)
LIB_PATH = os.path.join(_HERE, "libmisr_san.so" if os.environ.get("MISR_SANITIZE") == "1"
                        else "libmisr.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} not built: run `python -m paper_2108_04315_amd.build`")
lib = C.CDLL(LIB_PATH)

# ----------------------------------------------------------------- constants
OK, E_INVAL, E_NOMEM, E_HIP, E_NUMERIC, E_BUSY, E_NOTFOUND, E_CANCELLED, E_TIMEOUT = range(9)
STATUS_NAMES = ["OK", "E_INVAL", "E_NOMEM", "E_HIP", "E_NUMERIC", "E_BUSY", "E_NOTFOUND",
                "E_CANCELLED", "E_TIMEOUT"]
F32, F16, BF16 = 0, 1, 2
REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED, REQ_CANCELLED = range(5)


class MisrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < 9 else status}: {msg}")
        self.status = status


# ------------------------------------------------------------------- structs
class misr_geometry(C.Structure):
    _fields_ = [("hr_h", C.c_int32), ("hr_w", C.c_int32), ("scale", C.c_int32),
                ("n_frames", C.c_int32), ("shifts_lr", C.POINTER(C.c_double)),
                ("psf_size", C.c_int32), ("psf_1d", C.POINTER(C.c_double)),
                ("psf_frames", C.POINTER(C.c_double)), ("warps", C.POINTER(C.c_double)),
                ("psf_2d", C.POINTER(C.c_double)), ("general_ell", C.c_int32)]


class misr_params(C.Structure):
    _fields_ = [("lambda_reg", C.c_double), ("alpha_btv", C.c_double), ("eps", C.c_double),
                ("btv_w", C.c_int32), ("data_p", C.c_int32), ("eps_data", C.c_double),
                ("scg_sigma", C.c_double), ("scg_lambda1", C.c_double), ("n_iter", C.c_int32),
                ("img_dtype", C.c_int32), ("tile_lr", C.c_int32), ("halo_lr", C.c_int32),
                ("x_rounding", C.c_int32), ("x_work", C.c_int32), ("x_init", C.c_int32),
                ("y_u16", C.c_int32), ("y_scale", C.c_double)]


class misr_scg_iter(C.Structure):
    _fields_ = [("E", C.c_double), ("E_t", C.c_double), ("delta", C.c_double),
                ("mu", C.c_double), ("alpha", C.c_double), ("Delta", C.c_double),
                ("lam", C.c_double), ("pi", C.c_double), ("rr", C.c_double),
                ("success", C.c_int32), ("pad_", C.c_int32)]


class misr_scg_trace(C.Structure):
    _fields_ = [("iters", C.POINTER(misr_scg_iter)), ("capacity", C.c_int32),
                ("n_passes", C.c_int32), ("n_success", C.c_int32), ("stop", C.c_int32),
                ("E0", C.c_double), ("E_final", C.c_double)]


DONE_CB = C.CFUNCTYPE(None, C.c_uint64, C.c_int, C.c_void_p)


class misr_request(C.Structure):
    _fields_ = [("geom", misr_geometry), ("params", misr_params), ("y", C.c_void_p),
                ("x0", C.c_void_p), ("x_out", C.c_void_p), ("on_device", C.c_int32),
                ("done_cb", DONE_CB), ("user", C.c_void_p)]


class misr_server_config(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_size_t), ("max_slots", C.c_int32),
                ("max_queue", C.c_int32), ("fail_alloc_n", C.c_int32), ("fill_mpx", C.c_int32),
                ("fail_list_n", C.c_int32), ("max_idle_ops", C.c_int32), ("order", C.c_int32)]


class misr_server_info(C.Structure):
    _fields_ = [("queued", C.c_int32), ("running", C.c_int32), ("n_ops", C.c_int32),
                ("n_idle_ops", C.c_int32), ("used_bytes", C.c_size_t)]


class misr_req_stats(C.Structure):
    _fields_ = [("t_submit_us", C.c_double), ("t_admit_us", C.c_double),
                ("t_done_us", C.c_double), ("n_passes", C.c_int32), ("n_success", C.c_int32),
                ("status", C.c_int), ("pad_", C.c_int32), ("E_final", C.c_double),
                ("bytes", C.c_size_t), ("op_bytes", C.c_size_t)]


_vp = C.c_void_p
_SIGS = {
    "misr_params_default": (None, [C.POINTER(misr_params)]),
    "misr_geometry_check": (C.c_int, [C.POINTER(misr_geometry)]),
    "misr_params_check": (C.c_int, [C.POINTER(misr_params)]),
    "misr_last_error": (C.c_char_p, []),
    "misr_ctx_create": (C.c_int, [C.c_int, C.POINTER(_vp)]),
    "misr_ctx_destroy": (C.c_int, [_vp]),
    "misr_op_create": (C.c_int, [_vp, C.POINTER(misr_geometry), C.POINTER(_vp)]),
    "misr_op_destroy": (C.c_int, [_vp]),
    "misr_op_band": (C.c_int, [_vp]),
    "misr_op_sparse_width": (C.c_int, [_vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "misr_op_tune": (C.c_int, [_vp, C.POINTER(misr_params), _vp, _vp, C.c_int,
                               C.POINTER(C.c_int32), C.POINTER(C.c_int32), _vp]),
    "misr_op_tile": (C.c_int, [_vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "misr_op_tile_variant": (C.c_int, [_vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "misr_op_set_tile": (C.c_int, [_vp, C.c_int]),
    "misr_forward": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp]),
    "misr_interpolate": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp]),
    "misr_upsample": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp]),
    "misr_adjoint": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp]),
    "misr_cost_grad": (C.c_int, [_vp, C.POINTER(misr_params), _vp, _vp, _vp, _vp, _vp]),
    "misr_cost_grad_noalloc": (C.c_int, [_vp, C.POINTER(misr_params), _vp, _vp, _vp, _vp,
                                         _vp]),
    "misr_cost_grad_noalloc_max_bytes": (C.c_size_t, []),
    "misr_scg_solve": (C.c_int, [_vp, C.POINTER(misr_params), _vp, _vp,
                                 C.POINTER(misr_scg_trace), _vp]),
    "misr_scg_status": (C.c_int, [_vp, C.POINTER(misr_scg_trace), _vp]),
    "misr_scg_solve_batch": (C.c_int, [C.c_int, C.POINTER(_vp), C.POINTER(misr_params),
                                       C.POINTER(_vp), C.POINTER(_vp),
                                       C.POINTER(misr_scg_trace), _vp]),
    "misr_time_pass": (C.c_int, [_vp, C.POINTER(misr_params), _vp, _vp, C.c_int, C.c_int,
                                 C.POINTER(C.c_double), _vp]),
    "misr_server_create": (C.c_int, [_vp, C.POINTER(misr_server_config), C.POINTER(_vp)]),
    "misr_server_submit": (C.c_int, [_vp, C.POINTER(misr_request), C.POINTER(C.c_uint64)]),
    "misr_server_poll": (C.c_int, [_vp, C.c_uint64, C.POINTER(C.c_int),
                                   C.POINTER(misr_req_stats)]),
    "misr_server_wait": (C.c_int, [_vp, C.c_uint64, C.c_int64]),
    "misr_server_cancel": (C.c_int, [_vp, C.c_uint64]),
    "misr_server_query": (C.c_int, [_vp, C.POINTER(misr_server_info)]),
    "misr_server_destroy": (C.c_int, [_vp]),
}
EXPORTS = []
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name, None)
    if _f is None:
        continue
    _f.restype = _res
    _f.argtypes = _args
    globals()[_name] = _f
    EXPORTS.append(_name)


def last_error() -> str:
    return lib.misr_last_error().decode(errors="replace")


def check(status: int) -> None:
    if status != OK:
        raise MisrError(status, last_error())


# ------------------------------------------------------------ torch helpers
def _torch():
    import torch
    return torch


_DT = {"float32": F32, "float16": F16, "bfloat16": BF16}


def dtype_code(t) -> int:
    return _DT[str(t.dtype).replace("torch.", "")]


def stream_handle(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t) -> C.c_void_p:
    return C.c_void_p(t.data_ptr())


def default_params(**kw) -> misr_params:
    p = misr_params()
    lib.misr_params_default(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def make_geometry(H: int, W: int, s: int, shifts, psf, warps=None, general_ell: bool = False):
    """Returns (misr_geometry, keepalive arrays).  psf: (P,) taps shared by
    all frames and both axes, (K, 2, P) per frame (vertical taps, then
    horizontal taps), or (K, P, P) non-separable per frame; warps: None or
    (K, 6) affine coefficients per frame (the general operator);
    general_ell: store a general operator as sparse matrices even where the
    matrix-free kernels apply."""
    g, keep = _make_geometry(H, W, s, shifts, psf, warps)
    g.general_ell = 1 if general_ell else 0
    return g, keep


def _make_geometry(H: int, W: int, s: int, shifts, psf, warps):
    sh = np.ascontiguousarray(np.asarray(shifts, dtype=np.float64).reshape(-1, 2))
    pa = np.asarray(psf, dtype=np.float64)
    dp = C.POINTER(C.c_double)
    wp = None if warps is None else np.ascontiguousarray(
        np.asarray(warps, dtype=np.float64).reshape(sh.shape[0], 6))
    wptr = None if wp is None else wp.ctypes.data_as(dp)
    if pa.ndim == 3 and pa.shape[1] == pa.shape[2] and pa.shape[1] != 2:
        p2 = np.ascontiguousarray(pa)
        g = misr_geometry(H, W, s, sh.shape[0], sh.ctypes.data_as(dp), p2.shape[1], None, None,
                          wptr, p2.ctypes.data_as(dp))
        return g, (sh, p2, wp)
    if pa.ndim == 3:
        pf = np.ascontiguousarray(pa)
        ps = np.ascontiguousarray(pf[0, 0])
        g = misr_geometry(H, W, s, sh.shape[0], sh.ctypes.data_as(dp), pf.shape[2],
                          ps.ctypes.data_as(dp), pf.ctypes.data_as(dp), wptr, None)
        return g, (sh, ps, pf, wp)
    ps = np.ascontiguousarray(pa.ravel())
    g = misr_geometry(H, W, s, sh.shape[0], sh.ctypes.data_as(dp), ps.size,
                      ps.ctypes.data_as(dp), None, wptr, None)
    return g, (sh, ps, wp)


class Context:
    """A libmisr context bound to one HIP device."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        check(lib.misr_ctx_create(device, C.byref(h)))
        self.h = h
        self.device = device

    def close(self):
        # the C context refuses to go while ops or servers still use it; then
        # it stays alive (the objects using it keep this wrapper referenced)
        if self.h and lib.misr_ctx_destroy(self.h) == OK:
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Operator:
    """Observation model A_k = D B_k M_k of one geometry (built once, reused);
    psf: (P,) taps for every frame and axis, (K, 2, P) per frame, or
    (K, P, P) non-separable per frame; warps: None (the shifts) or (K, 6)
    affine coefficients per frame.  A non-separable PSF or warps give the
    general operator (matrix-free where its kernels apply; general_ell stores
    it as sparse matrices instead)."""

    def __init__(self, ctx: Context, H: int, W: int, s: int, shifts, psf, warps=None,
                 general_ell: bool = False):
        self.ctx = ctx
        self.H, self.W, self.s = H, W, s
        self.shifts = np.asarray(shifts, dtype=np.float64).reshape(-1, 2)
        self.K = self.shifts.shape[0]
        g, keep = make_geometry(H, W, s, self.shifts, psf, warps, general_ell)
        h = C.c_void_p()
        check(lib.misr_op_create(ctx.h, C.byref(g), C.byref(h)))
        self.h = h

    @property
    def band(self) -> int:
        return lib.misr_op_band(self.h)

    @property
    def tile(self):
        """(rows, columns) of the image kernels' HR tile; (0, 0) if general."""
        a, t = C.c_int32(), C.c_int32()
        check(lib.misr_op_tile(self.h, C.byref(a), C.byref(t)))
        return a.value, t.value

    @property
    def tile_variant(self):
        """(variant, trial-pass tile width); variant -1 if general."""
        v, t = C.c_int32(), C.c_int32()
        check(lib.misr_op_tile_variant(self.h, C.byref(v), C.byref(t)))
        return v.value, t.value

    def set_tile(self, variant: int) -> None:
        """Selects a compiled tile variant: 0 widest (default), 1 about half as
        wide, 2 (where compiled) variant 0 with a wider trial-pass tile."""
        check(lib.misr_op_set_tile(self.h, variant))

    def tune(self, y, x, params: misr_params | None = None, reps: int = 10, stream=None):
        """Tile autotuner: times every compiled tile shape on (y, x) and keeps
        the fastest for this operator; returns the chosen (rows, columns)."""
        p = params or default_params()
        p.img_dtype = dtype_code(x)
        a, t = C.c_int32(), C.c_int32()
        check(lib.misr_op_tune(self.h, C.byref(p), _ptr(y), _ptr(x), reps, C.byref(a),
                               C.byref(t), stream_handle(stream)))
        return a.value, t.value

    @property
    def sparse_width(self):
        """(entries per row of A, of A^T) of a general operator; (0, 0) if banded."""
        a, t = C.c_int32(), C.c_int32()
        check(lib.misr_op_sparse_width(self.h, C.byref(a), C.byref(t)))
        return a.value, t.value

    def close(self):
        if self.h:
            h, self.h = self.h, None
            check(lib.misr_op_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- entry points, same names as the C ABI -----------------------------
    def forward(self, x, y=None, stream=None):
        torch = _torch()
        if y is None:
            y = torch.empty((self.K, self.H // self.s, self.W // self.s), dtype=x.dtype,
                            device=x.device)
        check(lib.misr_forward(self.h, dtype_code(x), _ptr(x), _ptr(y), stream_handle(stream)))
        return y

    def interpolate(self, y, x=None, stream=None):
        """Multi-image interpolation of the frames y onto the HR grid."""
        torch = _torch()
        if x is None:
            x = torch.empty((self.H, self.W), dtype=y.dtype, device=y.device)
        check(lib.misr_interpolate(self.h, dtype_code(y), _ptr(y), _ptr(x),
                                   stream_handle(stream)))
        return x

    def upsample(self, y, x=None, stream=None):
        """Bicubic upsampling of frame 0 (the solver's start point)."""
        torch = _torch()
        if x is None:
            x = torch.empty((self.H, self.W), dtype=y.dtype, device=y.device)
        check(lib.misr_upsample(self.h, dtype_code(y), _ptr(y), _ptr(x), stream_handle(stream)))
        return x

    def adjoint(self, r, x=None, stream=None):
        torch = _torch()
        if x is None:
            x = torch.empty((self.H, self.W), dtype=torch.float32, device=r.device)
        check(lib.misr_adjoint(self.h, dtype_code(r), _ptr(r), _ptr(x), stream_handle(stream)))
        return x

    def cost_grad(self, x, y, params: misr_params | None = None, g=None, cost=None,
                  stream=None):
        torch = _torch()
        p = params or default_params()
        p.img_dtype = dtype_code(x)
        if g is None:
            g = torch.empty((self.H, self.W), dtype=torch.float32, device=x.device)
        if cost is None:
            cost = torch.empty(3, dtype=torch.float64, device=x.device)
        check(lib.misr_cost_grad(self.h, C.byref(p), _ptr(x), _ptr(y), _ptr(g), _ptr(cost),
                                 stream_handle(stream)))
        return cost, g

    def cost_grad_noalloc(self, x, y, g, cost, params: misr_params | None = None,
                          stream=None) -> int:
        """misr_cost_grad_noalloc: the caller passes the outputs g (H x W
        float32) and cost (3 float64), both on the device; returns the status
        code (no exception, so that callers can test the rejections)."""
        p = params or default_params()
        p.img_dtype = dtype_code(x)
        return lib.misr_cost_grad_noalloc(self.h, C.byref(p), _ptr(x), _ptr(y), _ptr(g),
                                          _ptr(cost), stream_handle(stream))

    def scg_solve(self, y, x_inout, params: misr_params | None = None, trace: bool = True,
                  stream=None):
        """Runs the solve in place on x_inout; returns the per-pass trace (list of
        dicts) and a summary dict when ``trace`` (synchronises), else None."""
        p = params or default_params()
        p.img_dtype = dtype_code(x_inout)
        tr, recs = _new_trace(p.n_iter) if trace else (None, None)
        st = lib.misr_scg_solve(self.h, C.byref(p), _ptr(y), _ptr(x_inout),
                                C.byref(tr) if tr is not None else None, stream_handle(stream))
        if st not in (OK, E_NUMERIC):
            check(st)
        if tr is None:
            return None
        return _trace_out(tr, recs, st)

    def scg_status(self, stream=None) -> dict:
        """Outcome of the last scg_solve on this operator (waits for it): the
        summary dict of scg_solve(trace=True) without the per-pass records."""
        tr = misr_scg_trace()
        st = lib.misr_scg_status(self.h, C.byref(tr), stream_handle(stream))
        if st not in (OK, E_NUMERIC):
            check(st)
        return _trace_out(tr, [], st)[1]

    def time_pass(self, y, x, which: int, reps: int = 20, params: misr_params | None = None,
                  stream=None) -> float:
        """Mean duration (us) of one image pass (0: trial, 1: update; 2: one
        trial + update pair, as in a solve) at the solve's first trial point,
        timed with HIP events."""
        p = params or default_params()
        p.img_dtype = dtype_code(x)
        out = C.c_double()
        check(lib.misr_time_pass(self.h, C.byref(p), _ptr(y), _ptr(x), which, reps,
                                 C.byref(out), stream_handle(stream)))
        return out.value


def _new_trace(n: int):
    recs = (misr_scg_iter * max(1, n))()
    tr = misr_scg_trace()
    tr.iters = C.cast(recs, C.POINTER(misr_scg_iter))
    tr.capacity = max(1, n)
    return tr, recs


def _trace_out(tr, recs, status):
    its = [dict(E=r.E, E_t=r.E_t, delta=r.delta, mu=r.mu, alpha=r.alpha, Delta=r.Delta,
                lam=r.lam, pi=r.pi, rr=r.rr, success=bool(r.success))
           for r in list(recs)[:tr.n_passes]]
    return its, dict(n_passes=tr.n_passes, n_success=tr.n_success, stop=tr.stop, E0=tr.E0,
                     E_final=tr.E_final, status=STATUS_NAMES[status])


def scg_solve_batch(ops, ys, xs, params_list, trace: bool = True, stream=None):
    """Advances several solves together (one work list, shared launches)."""
    n = len(ops)
    op_arr = (C.c_void_p * n)(*[o.h.value for o in ops])
    y_arr = (C.c_void_p * n)(*[y.data_ptr() for y in ys])
    x_arr = (C.c_void_p * n)(*[x.data_ptr() for x in xs])
    prm = (misr_params * n)()
    for i, p in enumerate(params_list):
        prm[i] = p
        prm[i].img_dtype = dtype_code(xs[i])
    trs = recs = None
    if trace:
        pairs = [_new_trace(p.n_iter) for p in params_list]
        trs = (misr_scg_trace * n)(*[t for t, _ in pairs])
        recs = [r for _, r in pairs]
    st = lib.misr_scg_solve_batch(n, op_arr, prm, y_arr, x_arr, trs, stream_handle(stream))
    if st not in (OK, E_NUMERIC):
        check(st)
    if not trace:
        return None
    return [_trace_out(trs[i], recs[i], st) for i in range(n)]


class Server:
    """Continuous-batching server of SR solves (misr_server_*)."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int, max_slots: int = 64,
                 max_queue: int = 0, fail_alloc_n: int = 0, fill_mpx: int = 0,
                 fail_list_n: int = 0, max_idle_ops: int = 0, order: int = 0):
        cfg = misr_server_config(hbm_budget_bytes, max_slots, max_queue, fail_alloc_n, fill_mpx,
                                 fail_list_n, max_idle_ops, order)
        h = C.c_void_p()
        check(lib.misr_server_create(ctx.h, C.byref(cfg), C.byref(h)))
        self.h = h
        self._keep = {}

    def submit(self, H, W, s, shifts, psf, y, x0, x_out, params: misr_params | None = None,
               on_device: bool = True, warps=None, general_ell: bool = False) -> int:
        """Queues one solve; y, x0, x_out are device tensors (or host numpy
        arrays with on_device=False) that must stay alive until it finishes;
        x0 may be None with params.x_init > 0 (start point computed on the
        device); psf, warps and general_ell as for Operator."""
        g, keep = make_geometry(H, W, s, shifts, psf, warps, general_ell)
        p = params or default_params()
        if on_device:
            p.img_dtype = dtype_code(x_out)
            ptrs = (y.data_ptr(), x0.data_ptr() if x0 is not None else None, x_out.data_ptr())
        else:
            ptrs = (y.ctypes.data, x0.ctypes.data if x0 is not None else None, x_out.ctypes.data)
        req = misr_request(g, p, ptrs[0], ptrs[1], ptrs[2], 1 if on_device else 0,
                           DONE_CB(0), None)
        rid = C.c_uint64()
        check(lib.misr_server_submit(self.h, C.byref(req), C.byref(rid)))
        self._keep[rid.value] = (keep, y, x0, x_out)
        return rid.value

    def poll(self, rid: int):
        st = C.c_int()
        stats = misr_req_stats()
        check(lib.misr_server_poll(self.h, rid, C.byref(st), C.byref(stats)))
        return st.value, stats

    def info(self) -> dict:
        """Occupancy: queued and running requests, cached and idle operators,
        device bytes charged against the budget."""
        inf = misr_server_info()
        check(lib.misr_server_query(self.h, C.byref(inf)))
        return {k: getattr(inf, k) for k, _ in misr_server_info._fields_}

    def wait(self, rid: int, timeout_us: int = -1) -> int:
        return lib.misr_server_wait(self.h, rid, timeout_us)

    def cancel(self, rid: int) -> int:
        return lib.misr_server_cancel(self.h, rid)

    def close(self):
        if self.h:
            h, self.h = self.h, None
            check(lib.misr_server_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
