"""Pins for the oracle's iterated CGO solver (Section 5: equations dbarinvShift, Sform, eqh, eqh2, the Section 5.3
algorithm).

* The shifted regularised inverse F^{-1}(h/(xi - a)), a = 2i conj(k), against its closed form: for
  h = F(e^{-|z|^2}), (xi - a) u^ = h means dbar(e^{-i a.x} u) = (i/2) e^{-|z|^2} e^{-i a.x}, and
  e^{-|z|^2} e^{-i a.x} = e^{-|k|^2} e^{-(z - conj k)(conj z + k)} is a complex Gaussian, whose dbar-inverse is the
  corrected dbartest formula.  The plain regularisation of the rolled array (the Section 4 method) is visibly worse
  once a approaches the edge of the xi domain (the situation of Fig. 3).
* k = 0: the iterated system is the plain one iterated once; both give the same S and m.
* moderate k with 2k on the grid: both methods resolve the solution; they agree to the discretisation error.
* large k (Fig. 2: k = 8.5936, L = 3.2, N = 128): the iterated method matches a high-resolution plain solution to
  rounding while the plain method at N = 128 does not (the disparate-support failure of Section 5.1).
"""
import numpy as np
import pytest

import dbar_workloads as W
from oracle import dbar_oracle as O


def exact_shifted_inverse(g, k):
    """u = F^{-1}(F(e^{-|z|^2}) / (xi - 2i conj k)) in closed form."""
    z = g.z
    kc = np.conj(k)
    with np.errstate(invalid="ignore", divide="ignore"):
        v = np.exp(-abs(k) ** 2) * (1 - np.exp(-(z - kc) * (np.conj(z) + k))) / (z - kc)
    at = np.abs(z - kc) < 1e-14
    v[at] = np.exp(-abs(k) ** 2) * (np.conj(kc) + k)  # limit (conj(z) + k) at z = conj(k)
    ek = np.exp(np.conj(k * z) - k * z)  # e^{-i a.x}
    return np.conj(ek) * 0.5j * v


@pytest.mark.parametrize("k", [0.0, 0.25 + 0.5j, 1.0 - 0.75j, 2.0 + 1.25j])
def test_shifted_inverse_closed_form(k):
    g = O.make_grid(128, 4.0)
    h = O.Fd(g, np.exp(-np.abs(g.z) ** 2))
    got = O.shifted_inverse(g, h, k, 11)
    assert np.max(np.abs(got - exact_shifted_inverse(g, k))) < 1e-12  # |u| <= 0.5; moments weighted by |z|^n


def test_shifted_inverse_at_zero_shift_is_the_plain_inverse():
    g = O.make_grid(64, 3.0)
    rng = np.random.default_rng(4)
    S = O.Fd(g, np.exp(-np.abs(g.z) ** 2) * (rng.standard_normal((64, 64)) + 1j * rng.standard_normal((64, 64))))
    assert np.max(np.abs(O.shifted_inverse(g, S, 0.0, 11) - O.regularised_h(g, S, 11)[0])) < 1e-15


def test_shift_beats_plain_regularisation_near_the_edge():
    """With a near the edge of the xi domain the plain inverse of the rolled array (regularised at 0, as in
    Section 4) loses accuracy, the shifted regularisation does not (Section 5.1, Fig. 3)."""
    g = O.make_grid(64, 4.0)          # xi_max = 8
    k = 1.5 + 2.0j                    # a = (2 k2, 2 k1) = (4, 3): |a| = 5
    h = O.Fd(g, np.exp(-np.abs(g.z) ** 2))
    exact = exact_shifted_inverse(g, k)
    m1, m2 = O.shift_index(g, k)
    ha = np.roll(h, (-m2, -m1), axis=(0, 1))
    plain = np.exp(k * g.z - np.conj(k * g.z)) * O.regularised_h(g, ha, 11)[0]
    e_shift = np.max(np.abs(O.shifted_inverse(g, h, k, 11) - exact))
    e_plain = np.max(np.abs(plain - exact))
    assert e_shift < 1e-6 and e_plain > 100 * e_shift, (e_shift, e_plain)


def test_shift_index_requires_grid_point():
    g = O.make_grid(32, 3.0)
    with pytest.raises(ValueError):
        O.shift_index(g, 0.1 + 0.1j)
    assert O.shift_index(g, 0.5 + 1.0j) == (6, 3)  # (2 k2 L, 2 k1 L)


def test_iterated_equals_plain_at_k_zero():
    g = O.make_grid(128, 4.0)
    Q = W.potential_gaussian(128, 4.0, 0.8 + 0.6j)
    p = O.solve(g, Q, 0.0, tol=1e-14)
    it = O.solve_iterated(g, Q, 0.0, tol=1e-14)
    assert np.max(np.abs(p.S - it.S)) < 1e-14 and np.max(np.abs(p.m - it.m)) < 1e-14
    assert abs(p.m1 - it.m1) < 1e-15


def test_iterated_agrees_with_plain_at_moderate_k():
    g = O.make_grid(256, 5.0)
    Q = W.potential_gaussian(256, 5.0, 0.8 + 0.6j)
    k = 0.4 + 0.2j
    p = O.solve(g, Q, k, tol=1e-14)
    it = O.solve_iterated(g, Q, k, tol=1e-14)
    assert it.iters < p.iters  # the once-iterated operator contracts faster
    assert np.max(np.abs(p.m - it.m)) < 1e-12 and abs(p.m1 - it.m1) < 1e-13


def test_large_k_fig2_parameters():
    """k = 8.5936 (2kL = 55 on the grid for L = 3.2), N = 128: the iterated method reaches the N = 512 solution."""
    L, k = 3.2, 55 / 6.4
    g = O.make_grid(128, L)
    gr = O.make_grid(512, L)
    Q = W.potential_gaussian(128, L, 1.0)
    ref = O.solve(gr, W.potential_gaussian(512, L, 1.0), k, tol=1e-14)
    it = O.solve_iterated(g, Q, k, tol=1e-14)
    pl = O.solve(g, Q, k, tol=1e-14)
    assert abs(it.m1 - ref.m1) < 1e-13
    assert np.max(np.abs(it.m - ref.m[::4, ::4])) < 1e-12
    assert abs(pl.m1 - ref.m1) > 1e-6  # the plain method cannot represent S here
