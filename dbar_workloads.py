"""Seeded synthetic inputs for the D-bar CGO solver.

This module produces *inputs only*: potentials Q sampled on the periodic x-grid, lists of spectral parameters k and
request streams.  It holds no step of the method itself (no transform, no regularisation, no solver), so the oracle
and the GPU library can both be fed from it without sharing any of the method's arithmetic.

The potentials are the paper's own test functions and smooth generalisations of them:

* the Gaussian e^{-x^2-y^2} used for the DS II example (Section 6, reconstruction table) and the D-bar inversion test
  (Section 4, equation dbartest);
* sums of shifted Gaussians and a sech^2 profile (Schwartz-class potentials, as the method assumes in Theorem 3.1).

All random draws use ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def x_grid(N: int, L: float) -> np.ndarray:
    """Periodic grid points x_j = L(-pi + 2 pi j / N), j = 0..N-1 (Section 4.1, equation 'domain')."""
    return L * (-math.pi + 2.0 * math.pi * np.arange(N) / N)


def _xy(N: int, L: float):
    x = x_grid(N, L)
    X, Y = np.meshgrid(x, x, indexing="xy")  # X[iy, ix] = x_ix, Y[iy, ix] = y_iy
    return X, Y


def potential_gaussian(N: int, L: float, A: complex = 1.0) -> np.ndarray:
    """Q = A exp(-(x^2 + y^2)) on the N x N grid, row-major Q[iy, ix], complex128."""
    X, Y = _xy(N, L)
    return (complex(A) * np.exp(-(X * X + Y * Y))).astype(np.complex128)


def potential_sech2(N: int, L: float, A: complex) -> np.ndarray:
    """Q = A sech^2(sqrt(x^2 + y^2)), complex128, row-major Q[iy, ix]."""
    X, Y = _xy(N, L)
    r = np.sqrt(X * X + Y * Y)
    return (complex(A) / np.cosh(r) ** 2).astype(np.complex128)


def gaussian_sum_params(seed: int, n_terms: int = 3, center_max: float = 3.0, amp_max: float = 1.5,
                        sigma_lo: float = 0.7, sigma_hi: float = 1.5):
    """Seeded centres z_j (|z_j| <= center_max), widths sigma_j in [sigma_lo, sigma_hi], amplitudes |A_j| <= amp_max."""
    rng = np.random.default_rng(seed)
    zc = center_max * np.sqrt(rng.random(n_terms)) * np.exp(2j * np.pi * rng.random(n_terms))
    sig = sigma_lo + (sigma_hi - sigma_lo) * rng.random(n_terms)
    amp = amp_max * np.sqrt(rng.random(n_terms)) * np.exp(2j * np.pi * rng.random(n_terms))
    return zc, sig, amp


def potential_gaussian_sum(N: int, L: float, seed: int, n_terms: int = 3, amp_max: float = 1.5) -> np.ndarray:
    """Q = sum_j A_j exp(-|z - z_j|^2 / sigma_j^2) with seeded parameters (see gaussian_sum_params)."""
    X, Y = _xy(N, L)
    zc, sig, amp = gaussian_sum_params(seed, n_terms, amp_max=amp_max)
    Q = np.zeros((N, N), np.complex128)
    for c, s, a in zip(zc, sig, amp):
        Q += a * np.exp(-((X - c.real) ** 2 + (Y - c.imag) ** 2) / (s * s))
    return Q


def k_square_grid(lo: float, hi: float, n: int, exclude_zero: bool = True) -> np.ndarray:
    """k = a + i b with a, b in linspace(lo, hi, n); row-major over (b, a)."""
    a = np.linspace(lo, hi, n)
    A, B = np.meshgrid(a, a, indexing="xy")
    ks = (A + 1j * B).ravel()
    if exclude_zero:
        ks = ks[np.abs(ks) > 0]
    return ks.astype(np.complex128)


def k_xi_grid(N: int, L: float) -> np.ndarray:
    """Every point of the xi grid as a spectral parameter, laid out like an xi-space array in FFT order:
    k[p2, p1] = (m(p1) + i m(p2)) / L with m(p) = p for p <= N/2, p - N otherwise (Section 4.1, equation
    'xidomain'; Section 6 puts k on this grid)."""
    m = np.arange(N)
    m = np.where(m <= N // 2, m, m - N).astype(np.float64)
    return (m[None, :] + 1j * m[:, None]) / L


def k_disk(n: int, radius: float, seed: int) -> np.ndarray:
    """n values of k uniform in the disk |k| <= radius (seeded)."""
    rng = np.random.default_rng(seed)
    return (radius * np.sqrt(rng.random(n)) * np.exp(2j * np.pi * rng.random(n))).astype(np.complex128)


@dataclass
class Workload:
    name: str
    N: int
    L: float
    Q: np.ndarray
    ks: np.ndarray
    tol: float
    M: int = 11
    note: str = ""
    extra: dict = field(default_factory=dict)


def workload(name: str, n_k: int | None = None) -> Workload:
    """The named synthetic workloads.

    * ``plain_n128``: N=128, L=5, Q = exp(-x^2-y^2), k = 1 + 0.5i, tol 1e-12.
    * ``plain_n1024``: N=1024, L=5, Q = (0.8+0.6i) exp(-(x^2+y^2)), 16 k on a 4x4 grid in [-2,2]^2, tol 1e-12.
    * ``batched_n512``: N=512, L=5, 3-Gaussian sum (seed 3), 1024 k on a 32x32 grid in [-6,6]^2, tol 1e-12.
    * ``mixed_n4096``: N=4096, L=8, Q = (1.2-0.4i) sech^2(r), 64 k uniform in |k| <= 8 (seed 4), tol 1e-12.

    ``n_k`` truncates the k list (first n_k values) for smaller runs.
    """
    if name == "plain_n128":
        N, L = 128, 5.0
        w = Workload(name, N, L, potential_gaussian(N, L, 1.0), np.array([1 + 0.5j]), 1e-12)
    elif name == "plain_n1024":
        N, L = 1024, 5.0
        w = Workload(name, N, L, potential_gaussian(N, L, 0.8 + 0.6j), k_square_grid(-2, 2, 4), 1e-12)
    elif name == "batched_n512":
        N, L = 512, 5.0
        w = Workload(name, N, L, potential_gaussian_sum(N, L, seed=3), k_square_grid(-6, 6, 32), 1e-12)
    elif name == "mixed_n4096":
        N, L = 4096, 8.0
        w = Workload(name, N, L, potential_sech2(N, L, 1.2 - 0.4j), k_disk(64, 8.0, seed=4), 1e-12)
    else:
        raise KeyError(name)
    if n_k is not None:
        w.ks = w.ks[:n_k]
    return w


@dataclass
class Request:
    t_arrival: float
    N: int
    L: float
    k: complex
    family: str
    Q: np.ndarray
    tol: float


def serving_stream(n_requests: int, rate: float, seed: int = 5, sizes=(256, 512, 1024, 2048), L: float = 5.0,
                   k_radius: float = 6.0, tol: float = 1e-10, make_q: bool = True):
    """Poisson request stream: exponential inter-arrival times at ``rate`` requests/s, N uniform on ``sizes``,
    k uniform in |k| <= k_radius, Q from the Gaussian-sum family (|A_j| <= 2) or sech^2 (|A| <= 2), each with
    probability 1/2."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate)
        N = int(rng.choice(sizes))
        k = complex(k_radius * math.sqrt(rng.random()) * np.exp(2j * math.pi * rng.random()))
        if rng.random() < 0.5:
            fam = "gaussian_sum"
            sub = int(rng.integers(0, 2**31 - 1))
            Q = potential_gaussian_sum(N, L, seed=sub, amp_max=2.0) if make_q else None
        else:
            fam = "sech2"
            A = complex(2.0 * math.sqrt(rng.random()) * np.exp(2j * math.pi * rng.random()))
            Q = potential_sech2(N, L, A) if make_q else None
        out.append(Request(t, N, L, k, fam, Q, tol))
    return out
