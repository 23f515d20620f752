"""Pins for omega_n = c_n W_n / d_n, the closed-form inverse transform of the Gaussian-weighted Taylor terms.

Section 4.2, Lemma: W_n = F^{-1}(conj(xi)^n e^{-|xi|^2}/xi) has the closed form fourreg5 and the series fourreg5a,
and follows from fourreg by the derivative recursion fourreg3.  With c_n = (-i/2)^n d_n/n! the factorials cancel
and c_n W_n = d_n omega_n, omega_n = i P(n+1, |z|^2/4) / z^{n+1} (P the regularised lower incomplete gamma).
The references here are independent of the oracle's code: mpmath at 40 digits, scipy's gammainc, the PDE that W_n
satisfies, and the recursion between consecutive n.
"""
import math

import mpmath
import numpy as np
import pytest
from scipy.special import gammainc

from oracle import dbar_oracle as O


def _sample_points():
    rng = np.random.default_rng(1)
    r = np.concatenate([[1e-6, 1e-3, 0.05, 0.5, 1.0, 2.0, 3.9, 4.0, 4.1, 6.0, 6.9, 7.0, 7.1, 10.0, 20.0, 35.0],
                        rng.uniform(0, 25, 40)])
    th = rng.uniform(0, 2 * math.pi, r.size)
    return r * np.exp(1j * th)


@pytest.mark.parametrize("n", [0, 1, 2, 5, 8, 11, 15])
def test_omega_vs_mpmath(n):
    """omega_n(z) = i P(n+1, |z|^2/4) / z^{n+1}, evaluated with mpmath's regularised incomplete gamma at 40 digits."""
    mpmath.mp.dps = 40
    zs = _sample_points()
    got = O.omega(n, zs)
    for z, w in zip(zs, got):
        zz = mpmath.mpc(z.real, z.imag)
        u = abs(zz) ** 2 / 4
        P = mpmath.gammainc(n + 1, 0, u, regularized=True)
        ref = complex(1j * P / zz ** (n + 1))
        assert abs(w - ref) <= 4e-15 * abs(ref) + 1e-300, (n, z, w, ref)


def test_omega_vs_scipy_gammainc():
    zs = _sample_points()
    for n in range(0, 12):
        u = np.abs(zs) ** 2 / 4
        ref = 1j * gammainc(n + 1, u) / zs ** (n + 1)
        got = O.omega(n, zs)
        assert np.all(np.abs(got - ref) <= 1e-13 * np.abs(ref) + 1e-300)


def test_omega_at_origin_is_zero():
    assert O.omega(0, np.array([0j]))[0] == 0
    assert O.omega(7, np.array([0j]))[0] == 0


def test_fourreg5_equals_corrected_fourreg5a_and_printed_form_differs():
    """On 0.3 < |z| < 3 both forms are accurate; they agree once the factor e^{-|z|^2/4} is restored in fourreg5a.
    The series as printed (without that factor) is off by e^{|z|^2/4}: for n = 0 and z = 0.7 - 0.4i it gives
    -0.1086 + 0.1900i instead of -0.0923 + 0.1615i."""
    z = 0.7 - 0.4j
    u = abs(z) ** 2 / 4
    closed = 1j * (1 - math.exp(-u)) / z                       # fourreg5, n = 0, divided by (2i)^0 0!
    series = sum(u ** k / math.factorial(k + 1) for k in range(60))
    printed = 1j * (np.conj(z) / 4) * series                  # fourreg5a as printed
    corrected = printed * math.exp(-u)
    assert abs(corrected - closed) < 1e-16
    assert abs(printed - (-0.1086 + 0.1900j)) < 1e-4
    assert abs(closed - (-0.0923 + 0.1615j)) < 1e-4
    for n in range(0, 12):
        for zz in (0.35 + 0.1j, -1.2 + 0.9j, 2.1 - 1.9j):
            uu = abs(zz) ** 2 / 4
            cf = 1j * (1 - math.exp(-uu) * sum(uu ** k / math.factorial(k) for k in range(n + 1))) / zz ** (n + 1)
            sr = 1j * (np.conj(zz) / 4) ** (n + 1) * math.exp(-uu) * sum(
                uu ** k / math.factorial(k + n + 1) for k in range(80))
            # the closed form cancels near the origin: its rounding error scales with |z|^-(n+1), not with |sr|
            assert abs(cf - sr) <= 1e-14 * abs(zz) ** -(n + 1)
            assert abs(O.omega(n, np.array([zz]))[0] - sr) <= 1e-14 * abs(sr)


def _dbar(fun, z, h=1e-3):
    """dbar = (d/dx + i d/dy)/2 by 4th-order central differences."""
    dx = (-fun(z + 2 * h) + 8 * fun(z + h) - 8 * fun(z - h) + fun(z - 2 * h)) / (12 * h)
    dy = (-fun(z + 2j * h) + 8 * fun(z + 1j * h) - 8 * fun(z - 1j * h) + fun(z - 2j * h)) / (12 * h)
    return 0.5 * (dx + 1j * dy)


def _dz(fun, z, h=1e-3):
    dx = (-fun(z + 2 * h) + 8 * fun(z + h) - 8 * fun(z - h) + fun(z - 2 * h)) / (12 * h)
    dy = (-fun(z + 2j * h) + 8 * fun(z + 1j * h) - 8 * fun(z - 1j * h) + fun(z - 2j * h)) / (12 * h)
    return 0.5 * (dx - 1j * dy)


@pytest.mark.parametrize("n", [0, 1, 3, 6, 11])
def test_omega_satisfies_dbar_equation(n):
    """F(dbar f) = (i/2) xi F(f) gives dbar W_n = (i/2) F^{-1}(conj(xi)^n e^{-|xi|^2}) = (i/4)(i conj(z)/2)^n e^{-|z|^2/4},
    hence dbar omega_n = (i/4) (conj(z)/4)^n e^{-|z|^2/4} / n!  (a dropped term or wrong power fails this)."""
    zs = np.array([0.3 + 0.2j, 1.1 - 0.7j, -2.5 + 1.5j, 3.0 + 3.0j, -5.0 - 1.0j, 8.0 + 0.5j])
    f = lambda zz: O.omega(n, np.atleast_1d(zz))
    got = np.array([_dbar(f, z)[0] for z in zs])
    want = 0.25j * (np.conj(zs) / 4) ** n * np.exp(-np.abs(zs) ** 2 / 4) / math.factorial(n)
    # 4th-order differences of a degree-(n+1) polynomial-like function near the origin: allow 1e-6 relative
    assert np.all(np.abs(got - want) <= 1e-6 * np.maximum(np.abs(want), 1e-3 * np.abs(f(zs))))


@pytest.mark.parametrize("n", [0, 1, 4, 10])
def test_derivative_recursion_fourreg3(n):
    """W_n = (-2i d/dz)^n W_0 (equation fourreg3) gives omega_{n+1} = -(d/dz omega_n) / (n+1)."""
    zs = np.array([0.4 + 0.3j, 1.5 - 0.2j, -2.2 + 2.0j, 4.0 - 3.0j, 9.0 + 1.0j])
    f = lambda zz: O.omega(n, np.atleast_1d(zz))
    got = np.array([-_dz(f, z)[0] / (n + 1) for z in zs])
    want = O.omega(n + 1, zs)
    assert np.all(np.abs(got - want) <= 1e-8 * np.abs(want) + 1e-14)
