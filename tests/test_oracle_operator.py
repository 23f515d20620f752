"""Pins for the oracle's operator A(S) = S + i F(q_k conj(h(S))) (Section 4 algorithm with Q -> q_k, Section 5.1).

The reference is the closed-form first Born term: for Q = A e^{-|z|^2},
    S0 = -i F(q_k) = -(iA/2) e^{-|xi + 2i conj(k)|^2/4}                                  (equation S0)
    S1 = K(S0)   = -i |A|^2 F[ e^{-2|z|^2} (z + conj(k)) phi1((conj(z) - k)(z + conj(k))) / 2 ],  phi1(w) = (e^w - 1)/w.
S1 is derived from S0, the D-bar inversion of a complex Gaussian (equation dbartest with the corrected coefficient)
and equation MainEQa; the printed S1 mixes in the halved-k convention of Section 6 (conj(z) - conj(k), |k|^2/4).
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import dbar_oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
BORN = json.load(open(os.path.join(HERE, "golden", "born_section5.json")))


def phi1(w):
    w = np.asarray(w, np.complex128)
    out = np.empty_like(w)
    sm = np.abs(w) < 1e-2
    out[~sm] = (np.exp(w[~sm]) - 1.0) / w[~sm]
    ws = w[sm]
    acc = np.zeros_like(ws)
    for j in range(12, -1, -1):  # Horner on sum_j w^j/(j+1)!
        acc = acc * ws + 1.0 / math.factorial(j + 1)
    out[sm] = acc
    return out


def born_S1(g, A, k):
    w = (np.conj(g.z) - k) * (g.z + np.conj(k))
    return -1j * abs(A) ** 2 * O.Fd(g, 0.5 * np.exp(-2 * np.abs(g.z) ** 2) * (g.z + np.conj(k)) * phi1(w))


@pytest.mark.parametrize("case", BORN["cases"])
def test_first_born_term(case):
    g = O.make_grid(case["N"], case["L"])
    A, k = complex(*case["A"]), complex(*case["k"])
    Q = A * np.exp(-np.abs(g.z) ** 2)
    S0 = O.rhs(g, Q, k)
    S0a = -(1j * A / 2) * np.exp(-np.abs(g.xi + 2j * np.conj(k)) ** 2 / 4)
    assert np.max(np.abs(S0 - S0a)) < BORN["bound"]
    K_S0 = S0 - O.apply_A(g, Q, k, S0)          # A = I - K
    assert np.max(np.abs(K_S0 - born_S1(g, A, k))) < BORN["bound"]


def test_born_intermediate_solves_dbar():
    """X = F^{-1}(S0/xi) = (A/2)(e^{-|k|^2} - e^{conj(k)conj(z) - kz - |z|^2})/(z - conj(k)) satisfies dbar X = q_k/2;
    the oracle's h(S0) must equal it on the grid."""
    g = O.make_grid(128, 4.0)
    A, k = 0.8 + 0.6j, 1 + 0.5j
    Q = A * np.exp(-np.abs(g.z) ** 2)
    h, _, _ = O.regularised_h(g, O.rhs(g, Q, k), 11)
    z = g.z
    num = np.exp(-abs(k) ** 2) - np.exp(np.conj(k) * np.conj(z) - k * z - np.abs(z) ** 2)
    X = 0.5 * A * num / (z - np.conj(k))
    assert np.max(np.abs(h - X)) < 1e-13


def test_operator_is_real_linear_not_complex_linear():
    g = O.make_grid(32, 3.0)
    rng = np.random.default_rng(2)
    Q = (0.5 + 0.2j) * np.exp(-np.abs(g.z) ** 2)
    k = 0.3 - 0.2j
    S1 = np.exp(-np.abs(g.xi) ** 2 / 3) * (rng.standard_normal((32, 32)) + 1j * rng.standard_normal((32, 32)))
    S2 = np.exp(-np.abs(g.xi) ** 2 / 3) * (rng.standard_normal((32, 32)) + 1j * rng.standard_normal((32, 32)))
    a, b = 0.7, -1.9
    lhs = O.apply_A(g, Q, k, a * S1 + b * S2)
    rhs = a * O.apply_A(g, Q, k, S1) + b * O.apply_A(g, Q, k, S2)
    assert np.max(np.abs(lhs - rhs)) < 1e-13 * np.max(np.abs(lhs))
    # i S is not mapped to i A(S): the conjugation makes K anti-linear
    assert np.max(np.abs(O.apply_A(g, Q, k, 1j * S1) - 1j * O.apply_A(g, Q, k, S1))) > 1e-3


def test_moments_are_taylor_coefficients():
    """d^n S/d conj(xi)^n (0) = (-i/2)^n F(z^n F^{-1} S)(0) (equation fourreeg4): check against the analytic
    derivatives of S(xi) = (1/2) e^{-|xi - xi0|^2/4} (the transform of e^{-|z|^2} e^{i Re(conj(xi0) z)})."""
    g = O.make_grid(128, 5.0)
    xi0 = 0.6 - 0.3j
    S = 0.5 * np.exp(-np.abs(g.xi - xi0) ** 2 / 4)
    s = O.Fd_inv(g, S)
    d, dt = O.moments(g, s, 11)
    c = O.G_coefficients(d)
    # S = (1/2) e^{-(xi - xi0)(conj(xi) - conj(xi0))/4}; d^n/d conj(xi)^n at 0: (1/2) e^{-|xi0|^2/4} (xi0/4)^n
    for n in range(12):
        want = 0.5 * math.exp(-abs(xi0) ** 2 / 4) * (xi0 / 4) ** n / math.factorial(n)
        # z^n amplifies rounding for larger n (noted after equation fourreeg4); low orders stay at 1e-15
        assert abs(c[n] - want) < 1e-15 * (1 + 3 * n * n), n
    # dS/dxi (0) = (1/2) e^{-|xi0|^2/4} conj(xi0)/4 = (-i/2) dt
    assert abs((-0.5j) * dt - 0.5 * math.exp(-abs(xi0) ** 2 / 4) * np.conj(xi0) / 4) < 1e-15
