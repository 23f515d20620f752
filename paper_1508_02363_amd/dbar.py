"""Python binding of the D-bar GPU library: argument marshalling only (every step runs in the HIP library).

Host functions take numpy complex128 arrays; the ``*_device`` variant takes torch tensors on the GPU (complex128)
and runs on the current torch stream.  Array layouts are those of include/dbar.h: x-space a[iy, ix], xi-space
A[p2, p1] in FFT order (wave number m = p for p <= N/2, p - N otherwise, xi = m / L).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import _lib
from ._lib import (DBAR_EAGAIN, DBAR_ENOCONV, DBAR_FP32, DBAR_FP64, DBAR_METHOD_ITERATED,  # noqa: F401
                   DBAR_METHOD_PLAIN, DBAR_MIXED, DBAR_MODE_BATCHED, DBAR_MODE_PLAIN, DBAR_OK, DBAR_SPACE_X,
                   DBAR_SPACE_XI, DbarError, check)

_D = ctypes.POINTER(ctypes.c_double)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _c128(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _grid(N: int, L: float, M: int) -> _lib.Grid:
    return _lib.Grid(int(N), int(M), float(L))


@dataclass
class SolveInfo:
    status: int
    iters: int
    outer: int
    rel_residual: float
    m1: complex
    cond_estimate: float = 0.0
    err_estimate: float = 0.0


def default_opts() -> _lib.Opts:
    o = _lib.Opts()
    _lib.load().dbar_default_opts(ctypes.byref(o))
    return o


def make_opts(precision=DBAR_FP64, mode=DBAR_MODE_BATCHED, restart=0, max_iter=1000, batch=0, use_graph=1,
              reorth=1, check_every=4, inner_tol=0.0, method=DBAR_METHOD_PLAIN, space=DBAR_SPACE_X,
              orth_window=None, lanes=0) -> _lib.Opts:
    """Solver options; orth_window None keeps the library's default Gram-Schmidt window; lanes 0 the library's
    default split of a batch into concurrent parts."""
    o = default_opts()
    if orth_window is not None:
        o.orth_window = orth_window
    o.lanes = lanes
    o.method = method
    o.space = space
    o.precision, o.mode, o.restart, o.max_iter, o.batch = precision, mode, restart, max_iter, batch
    o.use_graph, o.reorth, o.check_every, o.inner_tol = use_graph, reorth, check_every, inner_tol
    return o


def _infos(arr) -> list[SolveInfo]:
    return [SolveInfo(i.status, i.iters, i.outer, i.rel_residual, complex(i.m1_re, i.m1_im), i.cond_estimate,
                      i.err_estimate) for i in arr]


def solve(Q: np.ndarray, ks, L: float, tol: float = 1e-12, M: int = 11, want_m: bool = True, **opt_kw):
    """Solve A(S) = b for every k in ``ks`` (host arrays).  Returns (S [nk,N,N], m [nk,N,N] or None, infos)."""
    Q = _c128(Q)
    N = Q.shape[0]
    ks = np.ascontiguousarray(np.atleast_1d(np.asarray(ks, dtype=np.complex128)))
    nk = ks.size
    S = np.empty((nk, N, N), np.complex128)
    m = np.empty((nk, N, N), np.complex128) if want_m else None
    info = (_lib.Info * nk)()
    g = _grid(N, L, M)
    o = make_opts(**opt_kw)
    rc = _lib.load().dbar_solve(ctypes.byref(g), _dptr(Q), nk, _dptr(ks.view(np.float64)), float(tol),
                                ctypes.byref(o), _dptr(S), _dptr(m) if m is not None else None, info)
    check(rc, allow=(DBAR_OK, DBAR_ENOCONV))
    return S, m, _infos(info)


def solve_device(Q, ks, L: float, tol: float = 1e-12, M: int = 11, want_m: bool = True, **opt_kw):
    """As solve, with torch complex128 tensors on the GPU (Q [N,N]); returns device tensors S, m and infos."""
    import torch
    if not (isinstance(Q, torch.Tensor) and Q.is_cuda and Q.dtype == torch.complex128):
        raise TypeError("Q must be a complex128 torch tensor on the GPU")
    Q = Q.contiguous()
    N = Q.shape[0]
    ks = np.ascontiguousarray(np.atleast_1d(np.asarray(ks, dtype=np.complex128)))
    nk = ks.size
    S = torch.empty((nk, N, N), dtype=torch.complex128, device=Q.device)
    m = torch.empty((nk, N, N), dtype=torch.complex128, device=Q.device) if want_m else None
    info = (_lib.Info * nk)()
    g = _grid(N, L, M)
    o = make_opts(**opt_kw)
    stream = torch.cuda.current_stream(Q.device).cuda_stream
    rc = _lib.load().dbar_solve_device(ctypes.byref(g), ctypes.c_void_p(Q.data_ptr()), nk,
                                       _dptr(ks.view(np.float64)), float(tol), ctypes.byref(o),
                                       ctypes.c_void_p(S.data_ptr()),
                                       ctypes.c_void_p(m.data_ptr()) if m is not None else None, info,
                                       ctypes.c_void_p(stream))
    check(rc, allow=(DBAR_OK, DBAR_ENOCONV))
    return S, m, _infos(info)


def reflection(q: np.ndarray, ks, L: float, tol: float = 1e-12, M: int = 11, **opt_kw):
    """DS II reflection coefficient r(k) = i h(i conj k) (Section 6 convention, every k on the xi grid).
    Returns (r [nk], infos)."""
    q = _c128(q)
    N = q.shape[0]
    ks = np.ascontiguousarray(np.atleast_1d(np.asarray(ks, dtype=np.complex128)).ravel())
    r = np.empty(ks.size, np.complex128)
    info = (_lib.Info * ks.size)()
    g = _grid(N, L, M)
    o = make_opts(**opt_kw)
    rc = _lib.load().dbar_reflection(ctypes.byref(g), _dptr(q), ks.size, _dptr(ks.view(np.float64)), float(tol),
                                     ctypes.byref(o), _dptr(r.view(np.float64)), info)
    check(rc, allow=(DBAR_OK, DBAR_ENOCONV))
    return r, _infos(info)


def reconstruct(r: np.ndarray, L: float, t: float = 0.0, tol: float = 1e-12, M: int = 11, want_info: bool = False,
                **opt_kw):
    """DS II potential q(x, y, t) on the x grid from r(k, 0) on the xi grid (laid out like S).  Returns q [N, N]
    (and the N*N infos with want_info)."""
    r = _c128(r)
    N = r.shape[0]
    q = np.empty((N, N), np.complex128)
    info = (_lib.Info * (N * N))() if want_info else None
    g = _grid(N, L, M)
    o = make_opts(**opt_kw)
    rc = _lib.load().dbar_reconstruct(ctypes.byref(g), _dptr(r), float(t), float(tol), ctypes.byref(o), _dptr(q),
                                      info)
    check(rc, allow=(DBAR_OK, DBAR_ENOCONV))
    return (q, _infos(info)) if want_info else q


def autotune(N: int, L: float, precision: int = DBAR_MIXED, batch: int = 16, M: int = 11) -> dict:
    """Time the operator for every column-tile width at grid size N (and batch sizes up to `batch`), keep the
    fastest; returns the timings and choices."""
    r = _lib.TuneResult()
    check(_lib.load().dbar_autotune(ctypes.byref(_grid(N, L, M)), int(precision), int(batch), ctypes.byref(r)))
    out = {"batch": r.batch, "batch_candidates": list(r.batch_candidates), "per_entry_ms": list(r.per_entry_ms)}
    for f, name in ((0, "fp64"), (1, "fp32")):
        nv = r.n_variants[f]
        if nv:
            out[name] = {"columns": list(r.columns[f])[:nv], "ms": list(r.ms[f])[:nv],
                         "chosen_columns": r.columns[f][r.chosen[f]]}
    return out


def set_tile(N: int, precision: int, variant: int):
    """Force the column-tile variant of grid size N for the FP64 or FP32 operator."""
    check(_lib.load().dbar_set_tile(int(N), int(precision), int(variant)))


def get_tile(N: int, precision: int) -> tuple[int, int, int]:
    """(variant, columns per tile, number of variants) for grid size N."""
    v, c, nv = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    check(_lib.load().dbar_get_tile(int(N), int(precision), ctypes.byref(v), ctypes.byref(c), ctypes.byref(nv)))
    return v.value, c.value, nv.value


def apply(Q: np.ndarray, k: complex, S: np.ndarray, L: float, M: int = 11, precision: int = DBAR_FP64):
    """One application A(S) = S + i F(q_k conj(h(S)))."""
    Q = _c128(Q)
    N = Q.shape[0]
    S = _c128(S, (N, N))
    out = np.empty((N, N), np.complex128)
    kk = np.array([complex(k)], np.complex128)
    g = _grid(N, L, M)
    check(_lib.load().dbar_apply(ctypes.byref(g), _dptr(Q), _dptr(kk.view(np.float64)), _dptr(S), _dptr(out),
                                 int(precision)))
    return out


def apply_noalloc(Q, k: complex, S, out, L: float, M: int = 11, precision: int = DBAR_FP64):
    """One application A(S) on torch complex128 device tensors (Q, S read, out written) through the allocation-free
    entry point (N <= 1024), queued on the current torch stream."""
    import torch
    for t in (Q, S, out):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()):
            raise TypeError("Q, S and out must be contiguous complex128 torch tensors on the GPU")
    N = Q.shape[0]
    kk = np.array([complex(k)], np.complex128)
    g = _grid(N, L, M)
    stream = torch.cuda.current_stream(Q.device).cuda_stream
    check(_lib.load().dbar_apply_noalloc(ctypes.byref(g), ctypes.c_void_p(Q.data_ptr()), _dptr(kk.view(np.float64)),
                                         ctypes.c_void_p(S.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                         int(precision), ctypes.c_void_p(stream)))
    return out


def transform(f: np.ndarray, L: float, inverse: bool = False, precision: int = DBAR_FP64):
    """The grid transform consistent with the continuous F (inverse=False) or its inverse."""
    f = _c128(f)
    N = f.shape[0]
    out = np.empty((N, N), np.complex128)
    g = _grid(N, L, 11)
    check(_lib.load().dbar_transform(ctypes.byref(g), 1 if inverse else 0, _dptr(f), _dptr(out), int(precision)))
    return out


def dbar_inverse(S: np.ndarray, L: float, M: int = 11, precision: int = DBAR_FP64):
    """The regularised h(S) = F^{-1}(S / xi) of Section 4.2."""
    S = _c128(S)
    N = S.shape[0]
    out = np.empty((N, N), np.complex128)
    g = _grid(N, L, M)
    check(_lib.load().dbar_dbar_inverse(ctypes.byref(g), _dptr(S), _dptr(out), int(precision)))
    return out


def timer_enable(on: bool = True):
    """Start (clear) or stop the per-stage launch timer."""
    check(_lib.load().dbar_timer_enable(1 if on else 0))


def timer_stages() -> list[dict]:
    """Per-stage totals recorded by the launch timer: name, total_ms, launches, bytes (algorithmic)."""
    lib = _lib.load()
    out = []
    for st in range(lib.dbar_timer_num_stages()):
        name = ctypes.create_string_buffer(64)
        ms, nb = ctypes.c_double(), ctypes.c_double()
        cnt = ctypes.c_int64()
        check(lib.dbar_timer_stage(st, name, 64, ctypes.byref(ms), ctypes.byref(cnt), ctypes.byref(nb)))
        if cnt.value:
            out.append(dict(stage=st, name=name.value.decode(), total_ms=ms.value, launches=cnt.value,
                            bytes=nb.value))
    return out


class Session:
    """Serving session: continuous batching of single-k solves (see include/dbar.h)."""

    def __init__(self, hbm_budget_bytes: int = 0, max_slots: int = 64, precision: int = DBAR_MIXED,
                 restart: int = 20):
        o = _lib.SessionOpts(int(hbm_budget_bytes), int(max_slots), int(precision), int(restart), 0)
        h = ctypes.c_void_p()
        check(_lib.load().dbar_session_create(ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._shape = {}

    def submit(self, Q: np.ndarray, k: complex, L: float, tol: float = 1e-10, M: int = 11) -> int:
        Q = _c128(Q)
        N = Q.shape[0]
        kk = np.array([complex(k)], np.complex128)
        t = ctypes.c_uint64()
        g = _grid(N, L, M)
        check(_lib.load().dbar_submit(self._h, ctypes.byref(g), _dptr(Q), _dptr(kk.view(np.float64)), float(tol),
                                      ctypes.byref(t)))
        self._shape[t.value] = N
        return t.value

    def _fetch(self, fn, ticket: int):
        N = self._shape.get(ticket)
        info = _lib.Info()
        lat = ctypes.c_double()
        if N is None:  # unknown here: let the library report it
            rc = fn(self._h, ctypes.c_uint64(ticket), None, None, ctypes.byref(info), ctypes.byref(lat))
            check(rc)
            return None
        S = np.empty((N, N), np.complex128)
        m = np.empty((N, N), np.complex128)
        rc = fn(self._h, ctypes.c_uint64(ticket), _dptr(S), _dptr(m), ctypes.byref(info), ctypes.byref(lat))
        if rc == DBAR_EAGAIN:
            return None
        check(rc, allow=(DBAR_OK, DBAR_ENOCONV))
        del self._shape[ticket]
        return S, m, _infos([info])[0], lat.value

    def poll(self, ticket: int):
        """(S, m, info, latency_s) if finished, else None."""
        return self._fetch(_lib.load().dbar_poll, ticket)

    def wait(self, ticket: int):
        return self._fetch(_lib.load().dbar_wait, ticket)

    def stats(self) -> dict:
        st = _lib.SessionStats()
        check(_lib.load().dbar_session_get_stats(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in st._fields_}

    def close(self):
        if self._h:
            _lib.load().dbar_session_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def request_footprint(N: int, L: float = 1.0, precision: int = DBAR_MIXED, restart: int = 0, M: int = 11) -> int:
    """Device bytes a serving request on an N x N grid holds while in flight (its share of a class workspace)."""
    return int(_lib.load().dbar_request_footprint(ctypes.byref(_grid(N, L, M)), int(precision), int(restart)))


def release():
    _lib.load().dbar_release()


def version() -> int:
    return _lib.load().dbar_version()
