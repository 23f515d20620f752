"""Pins for the oracle's grids and discrete Fourier transform.

The discrete transform must approximate the continuous F(f)(xi) = (1/2pi) int f e^{-i xi.x} dx dy of Section 1 on the
grid of Section 4.1 (equations 'domain' and 'xidomain'), because analytically known pieces (the W_n of the Lemma in
Section 4.2) are added to discretely transformed ones.  These tests compare against closed-form transforms of
Gaussians, which fix scaling, phase, axis orientation and the sign convention of k independently of the code.
"""
import math

import numpy as np
import pytest

from oracle import dbar_oracle as O


def test_xi_grid_nyquist_positive():
    """Wave numbers xi in [-N/2+1, N/2]/L (equation xidomain): the Nyquist wave number is +N/(2L)."""
    for N, L in ((8, 1.0), (16, 4.0), (128, 5.0)):
        g = O.make_grid(N, L)
        xi1 = g.xi[0, :].real
        assert np.isclose(xi1.max(), N / (2 * L)) and np.isclose(xi1.min(), (-N / 2 + 1) / L)
        assert np.isclose(xi1[N // 2], N / (2 * L))
        xi2 = g.xi[:, 0].imag
        assert np.isclose(xi2[N // 2], N / (2 * L))


def test_x_grid_periodic_domain():
    """x in L[-pi, pi) with N points (equation domain): the left end is included, the right end is its image."""
    g = O.make_grid(16, 3.0)
    assert np.isclose(g.x[0], -3.0 * math.pi)
    assert np.isclose(g.x[-1] + g.dx, 3.0 * math.pi)
    assert np.isclose(g.z[16 // 2, 16 // 2], 0.0)


@pytest.mark.parametrize("N,L", [(128, 4.0), (256, 5.0)])
def test_Fd_of_gaussian(N, L):
    """F(e^{-|z|^2}) = (1/2) e^{-|xi|^2/4} (standard Gaussian integral)."""
    g = O.make_grid(N, L)
    got = O.Fd(g, np.exp(-np.abs(g.z) ** 2))
    want = 0.5 * np.exp(-np.abs(g.xi) ** 2 / 4)
    assert np.max(np.abs(got - want)) < 1e-15


def test_Fd_anisotropic_shifted_gaussian():
    """F(exp(-(x-x0)^2 - 4 (y-y0)^2)) = (1/(4)) exp(-xi1^2/4 - xi2^2/16) exp(-i(xi1 x0 + xi2 y0)).
    An x/y transposition, a wrong phase sign or a shifted origin all fail this."""
    g = O.make_grid(256, 4.0)
    x0, y0 = 1.3, -0.7
    X, Y = g.z.real, g.z.imag
    f = np.exp(-(X - x0) ** 2 - 4 * (Y - y0) ** 2)
    xi1, xi2 = g.xi.real, g.xi.imag
    want = (1.0 / (2 * math.pi)) * (math.pi / 2.0) * np.exp(-xi1 ** 2 / 4 - xi2 ** 2 / 16) \
        * np.exp(-1j * (xi1 * x0 + xi2 * y0))
    got = O.Fd(g, f)
    assert np.max(np.abs(got - want)) < 1e-15


def test_Fd_inverse_roundtrip_and_continuous_inverse():
    """F^{-1} F = identity on the grid, and F^{-1}((1/2) e^{-|xi|^2/4}) = e^{-|z|^2}."""
    g = O.make_grid(128, 4.0)
    rng = np.random.default_rng(0)
    f = rng.standard_normal((128, 128)) + 1j * rng.standard_normal((128, 128))
    assert np.max(np.abs(O.Fd_inv(g, O.Fd(g, f)) - f)) < 1e-13
    back = O.Fd_inv(g, 0.5 * np.exp(-np.abs(g.xi) ** 2 / 4))
    assert np.max(np.abs(back - np.exp(-np.abs(g.z) ** 2))) < 1e-15


@pytest.mark.parametrize("k", [1 + 0.5j, -0.7 + 1.3j, 2.0 - 1.0j])
def test_rhs_is_shifted_transform(k):
    """b = -i F(Q e^{conj(kz)-kz}) = -i Qhat(xi + 2i conj(k)) (Section 5.1, equation S0): for Q = A e^{-|z|^2},
    b = -(iA/2) exp(-|xi + 2i conj(k)|^2/4).  This fixes the sign and orientation of the k-dependent phase."""
    g = O.make_grid(128, 4.0)
    A = 0.8 + 0.6j
    Q = A * np.exp(-np.abs(g.z) ** 2)
    want = -(1j * A / 2) * np.exp(-np.abs(g.xi + 2j * np.conj(k)) ** 2 / 4)
    assert np.max(np.abs(O.rhs(g, Q, k) - want)) < 1e-15


def test_e_k_is_unimodular_phase():
    """e^{conj(kz)-kz} = e^{-2i(k2 x + k1 y)} has modulus one (eq:039)."""
    g = O.make_grid(32, 2.0)
    k = 1.7 - 0.4j
    ek = O.e_k(g, k)
    assert np.max(np.abs(np.abs(ek) - 1)) < 1e-14
    want = np.exp(-2j * (k.imag * g.z.real + k.real * g.z.imag))
    assert np.max(np.abs(ek - want)) < 1e-12
