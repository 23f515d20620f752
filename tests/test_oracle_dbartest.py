"""The paper's worked example for the regularised D-bar inversion (Section 4.2, equation dbartest and Fig. 1).

For f = exp(-a (z-b)(conj(z)-c)) the decaying solution of dbar u = f is u = (1 - f)/(a (z-b)) (the printed
coefficient a/(z-b) leaves dbar u = a^2 f; the form used here satisfies the equation for every a, checked below by
finite differences).  Since F(dbar u) = (i/2) xi F(u), the regularised inverse of S/xi applied to S = F f is
h = F^{-1}(F(f)/xi) = (i/2) u.  The paper reports, for a = 1/2, b = 1, c = i, L = 4:
machine precision at N = 128 and M = 11, exponential decay in M saturating near M = 11, and machine precision
reached for N about 2^6.
"""
import json
import os

import numpy as np
import pytest

from oracle import dbar_oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
FIX = json.load(open(os.path.join(HERE, "golden", "dbartest_fig1.json")))
A, B, C, L = FIX["a"], complex(*FIX["b"]), complex(*FIX["c"]), FIX["L"]
TOL = FIX["machine_precision_bound"]


def _exact(z):
    f = np.exp(-A * (z - B) * (np.conj(z) - C))
    return f, 0.5j * (1 - f) / (A * (z - B))


def _err(N, M, zero_at_origin=False):
    g = O.make_grid(N, L)
    f, want = _exact(g.z)
    h, _, _ = O.regularised_h(g, O.Fd(g, f), M, zero_at_origin=zero_at_origin)
    return np.max(np.abs(h - want))


def test_corrected_dbartest_closed_form_by_finite_differences():
    z0 = np.array([0.3 + 0.4j, -1.0 + 0.2j, 2.0 - 1.5j])
    h = 1e-4
    u = lambda z: (1 - np.exp(-A * (z - B) * (np.conj(z) - C))) / (A * (z - B))
    dx = (u(z0 + h) - u(z0 - h)) / (2 * h)
    dy = (u(z0 + 1j * h) - u(z0 - 1j * h)) / (2 * h)
    dbar = 0.5 * (dx + 1j * dy)
    f = np.exp(-A * (z0 - B) * (np.conj(z0) - C))
    assert np.max(np.abs(dbar - f)) < 1e-7
    printed = lambda z: A / (z - B) * (1 - np.exp(-A * (z - B) * (np.conj(z) - C)))
    dxp = (printed(z0 + h) - printed(z0 - h)) / (2 * h)
    dyp = (printed(z0 + 1j * h) - printed(z0 - 1j * h)) / (2 * h)
    assert np.max(np.abs(0.5 * (dxp + 1j * dyp) - f)) > 1e-2  # printed coefficient is wrong for a = 1/2


def test_machine_precision_at_N128_M11():
    assert _err(128, 11) < TOL


def test_machine_precision_reached_near_N64():
    errs = {N: _err(N, 11) for N in FIX["fig1_right"]["N_values"]}
    assert errs[64] < TOL
    assert errs[16] > errs[32] > errs[64]
    assert errs[16] > 1e-3 and errs[32] > 1e-6


def test_exponential_decay_in_M_then_saturation():
    Ms = FIX["fig1_left"]["M_values"]
    errs = [_err(128, M) for M in Ms]
    # strict decrease up to M = 11 by at least a factor 10 per two terms, saturation afterwards
    for e0, e1, M in zip(errs, errs[1:], Ms[1:]):
        if M <= 11:
            assert e1 < 0.1 * e0, (M, e0, e1)
    assert errs[Ms.index(11)] < TOL and errs[-1] < TOL


def test_zero_at_singular_point_loses_spectral_accuracy():
    """Setting the regularised integrand to zero at xi = 0 (the rule of the first-order method reviewed in Section 2)
    instead of taking its limit leaves a constant error of order dS/dxi(0)/(2 pi L^2) in h."""
    assert _err(128, 11, zero_at_origin=True) > 1e-4


@pytest.mark.parametrize("b,c,a", [(0.0, 0.0, 1.0), (0.5 - 0.5j, -0.3j, 2.0), (-1.0 + 0.3j, 0.2 + 0.1j, 0.7)])
def test_other_dbartest_parameters(b, c, a):
    g = O.make_grid(128, 4.0)
    f = np.exp(-a * (g.z - b) * (np.conj(g.z) - c))
    at_b = g.z == b
    with np.errstate(invalid="ignore", divide="ignore"):
        want = 0.5j * (1 - f) / (a * (g.z - b))
    want[at_b] = 0.5j * (np.conj(b) - c)  # the removable singularity: (1 - f)/(a(z-b)) -> conj(b) - c
    h, _, _ = O.regularised_h(g, O.Fd(g, f), 11)
    assert np.max(np.abs(h - want)) < 5 * TOL
