"""Host-side checks of libmisr.so that need no GPU: the library loads, exports
every function include/misr.h declares, and validates arguments on the host."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "misr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(misr_[a-z_0-9]+)\s*\(", src)) - {"misr_done_cb"})


@pytest.fixture(scope="module")
def misr():
    from paper_2108_04315_amd import misr as m
    return m


def test_every_declared_symbol_is_exported(misr):
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(misr.lib, n)]
    assert not missing, missing


def test_struct_layouts_match_header(misr, tmp_path):
    """The ctypes mirrors have the sizes and field offsets a C compiler gives
    the structs of include/misr.h."""
    structs = {"misr_geometry": misr.misr_geometry, "misr_params": misr.misr_params,
               "misr_scg_iter": misr.misr_scg_iter, "misr_scg_trace": misr.misr_scg_trace,
               "misr_request": misr.misr_request, "misr_server_config": misr.misr_server_config,
               "misr_req_stats": misr.misr_req_stats, "misr_server_info": misr.misr_server_info}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "misr.h"', "int main(void){"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{name}.{fname} %zu\\n", offsetof({name}, {fname}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(ln.split() for ln in subprocess.check_output([str(exe)], text=True).splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == C.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert int(got[f"{name}.{fname}"]) == getattr(cls, fname).offset, (name, fname)


def test_params_defaults_and_checks(misr):
    p = misr.default_params()
    assert (p.lambda_reg, p.alpha_btv, p.eps, p.btv_w, p.data_p) == (0.01, 0.4, 1e-3, 3, 2)
    assert (p.scg_sigma, p.scg_lambda1) == (1e-4, 1e-6)
    assert misr.lib.misr_params_check(C.byref(p)) == misr.OK
    for field, bad in [("alpha_btv", 1.0), ("alpha_btv", 0.0), ("lambda_reg", -1.0),
                       ("btv_w", 4), ("data_p", 3), ("scg_sigma", 0.0), ("scg_lambda1", -1.0),
                       ("n_iter", -1), ("eps", float("nan")), ("img_dtype", 7),
                       ("x_work", 2), ("x_rounding", 3)]:
        q = misr.default_params(**{field: bad})
        assert misr.lib.misr_params_check(C.byref(q)) == misr.E_INVAL, field
        assert misr.last_error()
    assert misr.lib.misr_params_check(None) == misr.E_INVAL


@pytest.mark.parametrize("kw,ok", [
    (dict(H=128, W=128, s=2, shifts=[[0, 0], [0.5, 0]], psf=[0.25, 0.5, 0.25]), True),
    (dict(H=127, W=128, s=2, shifts=[[0, 0]], psf=[1.0]), False),        # H % s
    (dict(H=128, W=128, s=5, shifts=[[0, 0]], psf=[1.0]), False),        # s > 4
    (dict(H=128, W=128, s=2, shifts=[[0, 0]], psf=[0.5, 0.5]), False),   # even P
    (dict(H=128, W=128, s=2, shifts=[[1.5, 0]], psf=[1.0]), False),      # |shift| > 1
    (dict(H=128, W=128, s=2, shifts=[[np.nan, 0]], psf=[1.0]), False),   # non-finite
    (dict(H=128, W=128, s=2, shifts=[[0, 0]] * 17, psf=[1.0]), False),   # K > 16
    (dict(H=12, W=12, s=3, shifts=[[0, 0], [1 / 3, 2 / 3]], psf=[1.0] * 1), True),
])
def test_geometry_checks(misr, kw, ok):
    g, keep = misr.make_geometry(kw["H"], kw["W"], kw["s"], kw["shifts"], kw["psf"])
    st = misr.lib.misr_geometry_check(C.byref(g))
    assert (st == misr.OK) == ok, misr.last_error()


def test_general_geometry_checks(misr):
    """General operators (affine warps, non-separable PSFs) are checked on the
    host: finite coefficients, the shift bound only where shifts are used."""
    K, H, W, s = 2, 16, 16, 2
    warps = np.array([[1.0, 0.0, 0.3, 0.0, 1.0, -0.4], [0.99, 0.05, 0.1, -0.05, 0.99, 0.2]])
    h2 = np.full((K, 3, 3), 1.0 / 9)
    cases = [
        (dict(shifts=np.zeros((K, 2)), psf=[1.0], warps=warps), True),
        (dict(shifts=np.zeros((K, 2)), psf=h2, warps=None), True),
        (dict(shifts=np.zeros((K, 2)), psf=h2, warps=warps), True),
        (dict(shifts=np.zeros((K, 2)), psf=[1.0], warps=np.where(warps == 0.3, np.nan, warps)),
         False),
        (dict(shifts=np.zeros((K, 2)), psf=np.where(h2 == h2[0, 0, 0], np.inf, h2), warps=None),
         False),
        (dict(shifts=[[1.5, 0.0], [0.0, 0.0]], psf=h2, warps=None), False),
    ]
    for kw, ok in cases:
        g, keep = misr.make_geometry(H, W, s, kw["shifts"], kw["psf"], kw["warps"])
        st = misr.lib.misr_geometry_check(C.byref(g))
        assert (st == misr.OK) == ok, (kw, misr.last_error())
    # warps make the shifts optional
    g, keep = misr.make_geometry(H, W, s, np.zeros((K, 2)), [1.0], warps)
    g.shifts_lr = None
    assert misr.lib.misr_geometry_check(C.byref(g)) == misr.OK
    g2, keep2 = misr.make_geometry(H, W, s, np.zeros((K, 2)), [1.0])
    g2.shifts_lr = None
    assert misr.lib.misr_geometry_check(C.byref(g2)) == misr.E_INVAL


def test_null_arguments_rejected_before_any_device_call(misr):
    assert misr.lib.misr_geometry_check(None) == misr.E_INVAL
    assert misr.lib.misr_op_create(None, None, None) == misr.E_INVAL
    assert misr.lib.misr_forward(None, 0, None, None, None) == misr.E_INVAL
    assert misr.lib.misr_scg_solve(None, None, None, None, None, None) == misr.E_INVAL
    assert misr.lib.misr_ctx_destroy(None) == misr.E_INVAL
    assert misr.lib.misr_op_sparse_width(None, None, None) == misr.E_INVAL
    assert misr.lib.misr_scg_status(None, None, None) == misr.E_INVAL
    assert misr.lib.misr_server_query(None, None) == misr.E_INVAL


def test_binding_has_no_cpu_fallback():
    """The product path imports the HIP library and nothing from the checker."""
    src = open(os.path.join(ROOT, "paper_2108_04315_amd", "misr.py")).read()
    assert "oracle" not in src
    for f in os.listdir(os.path.join(ROOT, "paper_2108_04315_amd", "csrc")):
        body = open(os.path.join(ROOT, "paper_2108_04315_amd", "csrc", f)).read()
        assert "oracle" not in body.lower(), f
