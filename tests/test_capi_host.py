"""CPU tests of the C ABI boundary: the library loads, exports every function include/*.h declares, and rejects bad
arguments before touching a device (no compute calls here)."""
import ctypes
import glob
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1508_02363_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(dbar_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


def test_header_declares_the_binding_list():
    assert declared_functions() == set(_lib.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if ln.strip()}
    missing = declared_functions() - exported
    assert not missing, missing
    for name in declared_functions():
        assert hasattr(lib, name)
    assert lib.dbar_version() >= 100


def _solve_rc(N=16, M=11, L=2.0, nk=1, tol=1e-12, k=(0.5, 0.25), Q=None):
    lib = _lib.load()
    g = _lib.Grid(N, M, L)
    n = max(N, 1) ** 2
    Qa = np.zeros(2 * n) if Q is None else Q
    ka = np.array(k, dtype=np.float64)
    S = np.zeros(2 * n * max(nk, 1))
    D = ctypes.POINTER(ctypes.c_double)
    return lib.dbar_solve(ctypes.byref(g), Qa.ctypes.data_as(D), nk, ka.ctypes.data_as(D), tol, None,
                          S.ctypes.data_as(D), None, None)


@pytest.mark.parametrize("kw", [dict(N=100), dict(N=4), dict(N=8192), dict(L=-1.0), dict(L=float("nan")),
                                dict(M=16), dict(M=-1), dict(nk=0), dict(tol=0.0), dict(tol=float("inf")),
                                dict(k=(float("nan"), 0.0))])
def test_invalid_arguments_are_rejected(kw):
    assert _solve_rc(**kw) == _lib.DBAR_EINVAL
    assert _lib.load().dbar_last_error().decode()


@pytest.mark.parametrize("opt", [dict(space=2), dict(space=-1), dict(method=2), dict(orth_window=-1),
                                 dict(orth_window=65)])
def test_invalid_solver_options_are_rejected(opt):
    lib = _lib.load()
    g = _lib.Grid(16, 11, 2.0)
    o = _lib.Opts()
    lib.dbar_default_opts(ctypes.byref(o))
    assert o.space == _lib.DBAR_SPACE_X
    for k, v in opt.items():
        setattr(o, k, v)
    Qa, ka, S = np.zeros(2 * 256), np.array([0.5, 0.25]), np.zeros(2 * 256)
    D = ctypes.POINTER(ctypes.c_double)
    rc = lib.dbar_solve(ctypes.byref(g), Qa.ctypes.data_as(D), 1, ka.ctypes.data_as(D), 1e-12, ctypes.byref(o),
                        S.ctypes.data_as(D), None, None)
    assert rc == _lib.DBAR_EINVAL and lib.dbar_last_error().decode()


def test_nan_in_potential_is_rejected():
    Q = np.zeros(2 * 16 * 16)
    Q[7] = np.nan
    rc = _solve_rc(Q=Q)
    assert rc in (_lib.DBAR_EINVAL, _lib.DBAR_EDEVICE)  # device check may come first on a CPU-only host


def test_request_footprint_is_monotone_in_grid_and_restart():
    lib = _lib.load()
    f = lambda N, r, p=_lib.DBAR_MIXED: lib.dbar_request_footprint(ctypes.byref(_lib.Grid(N, 11, 5.0)), p, r)
    assert f(256, 20) < f(512, 20) < f(1024, 20) < f(2048, 20)
    assert f(1024, 10) < f(1024, 20)
    assert f(1024, 20, _lib.DBAR_MIXED) < f(1024, 20, _lib.DBAR_FP64)
    # mixed precision at N=1024, restart 20: 21 FP32 basis vectors + 5 FP64 + 2 FP32 arrays of 2^20 elements
    assert f(1024, 20) >= (21 * 8 + 5 * 16 + 2 * 8) * 2 ** 20
    assert lib.dbar_request_footprint(ctypes.byref(_lib.Grid(100, 11, 5.0)), _lib.DBAR_MIXED, 20) == 0


def test_default_opts():
    o = _lib.Opts()
    _lib.load().dbar_default_opts(ctypes.byref(o))
    assert o.max_iter == 1000 and o.reorth == 1 and o.precision == _lib.DBAR_FP64 and o.inner_tol == 0.0
    assert o.orth_window == 2


def test_reflection_and_reconstruction_reject_bad_arguments():
    lib = _lib.load()
    D = ctypes.POINTER(ctypes.c_double)
    g = _lib.Grid(16, 11, 2.0)
    q = np.zeros(2 * 256)
    r = np.zeros(2)
    off = np.array([0.1, 0.0])  # L Re k = 0.2: not on the xi grid
    assert lib.dbar_reflection(ctypes.byref(g), q.ctypes.data_as(D), 1, off.ctypes.data_as(D), 1e-12, None,
                               r.ctypes.data_as(D), None) == _lib.DBAR_EINVAL
    on = np.array([0.5, -1.0])
    assert lib.dbar_reflection(ctypes.byref(g), q.ctypes.data_as(D), 1, on.ctypes.data_as(D), 1e-12, None,
                               None, None) == _lib.DBAR_EINVAL
    rr = np.zeros(2 * 256)
    rr[3] = np.inf
    qo = np.zeros(2 * 256)
    assert lib.dbar_reconstruct(ctypes.byref(g), rr.ctypes.data_as(D), 0.0, 1e-12, None, qo.ctypes.data_as(D),
                                None) == _lib.DBAR_EINVAL
    assert lib.dbar_reconstruct(ctypes.byref(g), qo.ctypes.data_as(D), float("nan"), 1e-12, None,
                                qo.ctypes.data_as(D), None) == _lib.DBAR_EINVAL
    assert lib.dbar_reconstruct(ctypes.byref(_lib.Grid(12, 11, 2.0)), qo.ctypes.data_as(D), 0.0, 1e-12, None,
                                qo.ctypes.data_as(D), None) == _lib.DBAR_EINVAL


def test_tuning_entry_points_validate_arguments():
    lib = _lib.load()
    g = _lib.Grid(100, 11, 2.0)
    assert lib.dbar_autotune(ctypes.byref(g), _lib.DBAR_MIXED, 16, None) == _lib.DBAR_EINVAL
    g = _lib.Grid(256, 11, 2.0)
    assert lib.dbar_autotune(ctypes.byref(g), 7, 16, None) == _lib.DBAR_EINVAL
    assert lib.dbar_autotune(ctypes.byref(g), _lib.DBAR_MIXED, 0, None) == _lib.DBAR_EINVAL
    assert lib.dbar_set_tile(256, _lib.DBAR_FP64, 99) == _lib.DBAR_EINVAL
    assert lib.dbar_set_tile(256, _lib.DBAR_MIXED, 0) == _lib.DBAR_EINVAL
    v, c, nv = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    assert lib.dbar_get_tile(256, _lib.DBAR_FP32, ctypes.byref(v), ctypes.byref(c), ctypes.byref(nv)) == 0
    assert v.value == 0 and nv.value >= 2 and c.value == 8  # default: 8 columns (64 B rows of FP32 complex)


@pytest.mark.parametrize("N,prec", [(2048, 0), (4096, 2), (16, 1), (12, 0)])
def test_noalloc_apply_rejects_sizes_and_options_on_the_host(N, prec):
    """The allocation-free entry point checks the grid against its scratch maximum (N <= 1024) and the precision
    before it touches a device: no buffer is dereferenced for these calls."""
    lib = _lib.load()
    g = _lib.Grid(N, 11, 2.0)
    k = np.array([0.5, 0.25])
    rc = lib.dbar_apply_noalloc(ctypes.byref(g), ctypes.c_void_p(16), k.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                ctypes.c_void_p(16), ctypes.c_void_p(16), prec, None)
    assert rc == _lib.DBAR_EINVAL
    msg = lib.dbar_last_error().decode()
    assert msg and (N <= 1024 or "1024" in msg)
