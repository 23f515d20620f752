"""Pins for the oracle's full solve: the discrete system A(S) = b and the continuous CGO solution it approximates.

* dense LU of the assembled real 2N^2 x 2N^2 matrix on tiny grids (the plain definition of the discrete solution);
* Q = 0 gives S = 0, m = 0;
* Born scaling: for Q = eps Q1 the remainder S - S0 - S1 is O(eps^3) (Section 5.1, Neumann series);
* a manufactured CGO solution: m* = eps (1 - e^{-|z|^2})/z has dbar m* = eps e^{-|z|^2} and S* = -i eps e^{-|xi|^2/4};
  Q* is chosen so that eq:039 holds exactly;
* spectral convergence under grid doubling (Section 1, Section 4.1);
* the PDE residual dbar m - (1/2) q_k (conj(m) + 1) (eq:039), with dbar of the periodic part taken spectrally and of
  the closed-form part analytically;
* m^(1) = i S(0) (equation m1def) and the large-|z| behaviour m ~ m^(1)/z.
"""
import math

import numpy as np
import pytest

import dbar_workloads as W
from oracle import dbar_oracle as O


@pytest.mark.parametrize("N,k", [(8, 0.4 + 0.2j), (16, 1 + 0.5j), (32, -0.8 + 0.3j)])
def test_gmres_matches_dense_lu(N, k):
    L = 1.2 * N / 16 + 0.8
    g = O.make_grid(N, L)
    Q = (0.9 - 0.3j) * np.exp(-np.abs(g.z) ** 2)
    S_lu, Amat = O.dense_solve(g, Q, k)
    r = O.solve(g, Q, k, tol=1e-14)
    assert r.rel_residual <= 1e-14
    assert np.max(np.abs(r.S - S_lu)) <= 1e-13 * np.max(np.abs(S_lu))
    cond = np.linalg.cond(Amat)
    assert cond < 50, cond  # well conditioned: parity tolerances of order 1e-10 leave ample room


def test_zero_potential_gives_zero():
    g = O.make_grid(32, 3.0)
    r = O.solve(g, np.zeros((32, 32), np.complex128), 1 + 1j)
    assert r.iters == 0 and np.all(r.S == 0) and np.all(r.m == 0)


def test_born_scaling_is_cubic():
    """||S - eps S0 - eps^2 S1|| / eps^3 stays bounded as eps -> 0 (Neumann series of Section 5.1)."""
    g = O.make_grid(64, 4.0)
    k = 0.5 + 0.25j
    Q1 = np.exp(-np.abs(g.z) ** 2)
    S0 = O.rhs(g, Q1, k)
    S1 = S0 - O.apply_A(g, Q1, k, S0)
    ratios = []
    for eps in (0.2, 0.1, 0.05):
        r = O.solve(g, eps * Q1, k, tol=1e-14)
        rem = np.max(np.abs(r.S - eps * S0 - eps ** 2 * S1))
        ratios.append(rem / eps ** 3)
    assert max(ratios) / min(ratios) < 1.3, ratios
    slope = math.log(ratios[0] * 0.2 ** 3 / (ratios[2] * 0.05 ** 3)) / math.log(4)
    assert abs(slope - 3) < 0.15, slope


def _manufactured(g, eps, k):
    z = g.z
    with np.errstate(invalid="ignore", divide="ignore"):
        mstar = eps * (1 - np.exp(-np.abs(z) ** 2)) / z
    mstar[z == 0] = 0.0
    ek = np.exp(np.conj(k * z) - k * z)
    Qstar = 2 * eps * np.exp(-np.abs(z) ** 2) / (ek * (np.conj(mstar) + 1))
    Sstar = -1j * eps * np.exp(-np.abs(g.xi) ** 2 / 4)
    return mstar, Qstar, Sstar


@pytest.mark.parametrize("eps,k", [(0.5, 0.7 - 0.4j), (1.0, 1 + 0.5j)])
def test_manufactured_solution(eps, k):
    g = O.make_grid(128, 5.0)
    mstar, Qstar, Sstar = _manufactured(g, eps, k)
    r = O.solve(g, Qstar, k, tol=1e-14)
    assert np.max(np.abs(r.S - Sstar)) < 1e-12
    assert np.max(np.abs(r.m - mstar)) < 1e-12


def test_manufactured_spectral_convergence():
    eps, k = 0.8, 0.5 + 0.5j
    errs = []
    for N in (16, 32, 64):
        g = O.make_grid(N, 3.0)
        mstar, Qstar, Sstar = _manufactured(g, eps, k)
        r = O.solve(g, Qstar, k, tol=1e-14)
        errs.append(np.max(np.abs(r.m - mstar)))
    assert errs[0] > 10 * errs[1] > 100 * errs[2] or errs[2] < 1e-12, errs
    assert errs[1] ** 1.5 > errs[2] or errs[2] < 1e-12  # faster than any fixed power: exponent grows


def test_grid_doubling_plain_workload():
    """Potential e^{-x^2-y^2}, L = 5, k = 1 + 0.5i at N = 32..256 on the same domain: the error of m on common grid
    points against N = 256 falls faster than any power of N (each doubling gains more digits than the last)."""
    w = W.workload("plain_n128")
    k = w.ks[0]
    ms = {}
    for N in (32, 64, 128, 256):
        g = O.make_grid(N, w.L)
        Q = W.potential_gaussian(N, w.L, 1.0)
        ms[N] = O.solve(g, Q, k, tol=1e-14).m
    e = {N: np.max(np.abs(ms[N] - ms[256][::256 // N, ::256 // N])) for N in (32, 64, 128)}
    assert e[32] > 1e2 * e[64] and e[64] > 1e3 * e[128], e
    assert math.log(e[64] / e[128]) > 1.5 * math.log(e[32] / e[64]), e
    assert e[128] < 1e-7, e


def test_pde_residual_and_m1():
    w = W.workload("plain_n128")
    g = O.make_grid(w.N, w.L)
    k = w.ks[0]
    M = 11
    om = O.omega_table(g, M)
    r = O.solve(g, w.Q, k, tol=1e-14, om=om)
    # split m = F^{-1} R + sum_n d_n omega_n and differentiate each part exactly
    s = O.Fd_inv(g, r.S)
    d, dt = O.moments(g, s, M)
    c = O.G_coefficients(d)
    Gx = sum(c[n] * np.conj(g.xi) ** n for n in range(M + 1)) * np.exp(-np.abs(g.xi) ** 2)
    R = np.where(g.xi != 0, (r.S - Gx) / np.where(g.xi != 0, g.xi, 1), -0.5j * dt)
    dbar_periodic = O.Fd_inv(g, 0.5j * g.xi * R)
    u = np.abs(g.z) ** 2 / 4
    dbar_tail = sum(d[n] * 0.25j * (np.conj(g.z) / 4) ** n * np.exp(-u) / math.factorial(n) for n in range(M + 1))
    qk = w.Q * np.exp(np.conj(k * g.z) - k * g.z)
    res = dbar_periodic + dbar_tail - 0.5 * qk * (np.conj(r.m) + 1)
    assert np.max(np.abs(res)) < 1e-12
    # m^(1) = i S(0) = (1/pi) int dbar m
    m1_int = (g.dx ** 2 / math.pi) * np.sum(0.5 * qk * (np.conj(r.m) + 1))
    assert abs(r.m1 - m1_int) < 1e-12
    # far field: z m -> m^(1)
    edge = np.abs(g.z) > 0.9 * math.pi * w.L
    zm = (g.z * r.m)[edge]
    assert np.max(np.abs(zm - r.m1)) < 0.2 * abs(r.m1) + 1e-12
