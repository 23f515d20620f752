"""Pins for the DS II reflection coefficient r(k) = i h(i conj k) (Section 6, equation rviah).

* First Born approximation: for q = eps e^{-|z|^2}, h = -i F(q) + O(eps^3) (equation eqh is h - K0 K0 h = -iF(q) with
  K0 linear in q), hence r(k) = F(q)(i conj k) + O(eps^3) = (eps/2) e^{-|k|^2/4} + O(eps^3).
* The relation with the CGO solutions: r = (M1^(1) - M2^(1))/2 (equation eq:023), where M_j solve the plain D-bar
  problems with potentials +q and -q and the halved exponent; M^(1) = i S(0) (equation m1def).
"""
import numpy as np
import pytest

from oracle import dbar_oracle as O


def test_born_limit_is_cubic():
    g = O.make_grid(64, 3.2)
    q1 = np.exp(-np.abs(g.z) ** 2)
    k = (3 + 2j) / 3.2  # on the xi grid
    born = 0.5 * np.exp(-abs(k) ** 2 / 4)
    rem = []
    for eps in (0.2, 0.1, 0.05):
        r = O.reflection_coefficient(g, eps * q1, k, tol=1e-14)
        rem.append(abs(r - eps * born) / eps ** 3)
    assert max(rem) / min(rem) < 1.3, rem
    assert abs(O.reflection_coefficient(g, 1e-4 * q1, k) - 1e-4 * born) < 1e-12


@pytest.mark.parametrize("k", [(1 + 1j) / 3.2, (4 - 2j) / 3.2])
def test_reflection_equals_half_difference_of_m1(k):
    """r = (M1^(1) - M2^(1))/2 with M1, M2 the CGO solutions for +q and -q (plain method, parameter k/2)."""
    g = O.make_grid(128, 3.2)
    q = (0.7 - 0.2j) * np.exp(-np.abs(g.z) ** 2)
    r = O.reflection_coefficient(g, q, k, tol=1e-14)
    m1p = O.solve(g, q, k / 2, tol=1e-14).m1
    m1m = O.solve(g, -q, k / 2, tol=1e-14).m1
    assert abs(r - 0.5 * (m1p - m1m)) < 1e-12
