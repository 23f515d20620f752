"""Pins for the oracle's DS II inverse scattering (Section 6: equations dbarrecA, dbarrecB, qRec, rt).

* The paper's reconstruction table (Section 6.2): for q(x, y, 0) = e^{-x^2-y^2}, M = 11, the L-infinity error of
  q -> r -> q at (N, L) = (8, 0.7515), (16, 1.075), (32, 1.5) is 7.09e-3, 3.1872e-4, 1.665e-6.  The oracle's
  discretisation error must be of that size (a wrong factor, sign or index in either transform gives an O(1) error).
* The small-amplitude limit of DS II: for q0 = eps e^{-|z|^2} the nonlinear terms of equation DSIIa are O(eps^3),
  so q(t) = eps u(x, t) v(y, t) + O(eps^3) with u = e^{-x^2/(1+2it)}/sqrt(1+2it), v = e^{-y^2/(1-2it)}/sqrt(1-2it)
  (the Gaussian solutions of i u_t + u_xx/2 = 0 and i v_t - v_yy/2 = 0).  This pins the time factor of equation rt
  in the Section 6 convention; the alternatives (the factor for the unhalved k, or the opposite sign) are off by
  several percent.
"""
import numpy as np
import pytest

from oracle import dbar_oracle as O


def gaussian(g, amp=1.0):
    return amp * np.exp(-np.abs(g.z) ** 2)


@pytest.mark.parametrize("N,L,paper", [(8, 0.7515, 7.09e-3), (16, 1.075, 3.1872e-4),
                                       pytest.param(32, 1.5, 1.665e-6, marks=pytest.mark.slow)])
def test_reconstruction_table(N, L, paper):
    g = O.make_grid(N, L)
    q0 = gaussian(g)
    q = O.reconstruct_potential(g, O.reflection_grid(g, q0))
    err = np.max(np.abs(q - q0))
    assert 0.5 * paper < err < 1.25 * paper, (err, paper)


def test_dual_grid_contains_the_x_grid():
    g = O.make_grid(16, 1.3)
    gp = O.dual_grid(g)
    assert np.allclose(gp.x[1] - gp.x[0], 1.0 / g.L)
    # every z of the x grid is a point of the dual xi grid: m = z L' integer
    m = g.z * gp.L
    assert np.max(np.abs(m - np.round(m))) < 1e-12


def test_small_amplitude_time_evolution():
    N, L, eps = 16, 1.3, 1e-3
    g = O.make_grid(N, L)
    r = O.reflection_grid(g, gaussian(g, eps))
    x, y = g.z.real, g.z.imag
    for t in (0.0, 0.3):
        lin = eps * np.exp(-x ** 2 / (1 + 2j * t)) / np.sqrt(1 + 2j * t) * np.exp(-y ** 2 / (1 - 2j * t)) / np.sqrt(
            1 - 2j * t)
        q = O.reconstruct_potential(g, O.evolve_reflection(g, r, t))
        assert np.max(np.abs(q - lin)) < 1e-4 * eps, t
    # the reflection coefficient keeps its modulus (Section 6.1)
    assert np.allclose(np.abs(O.evolve_reflection(g, r, 0.7)), np.abs(r), rtol=1e-15, atol=0)


def test_stored_n64_round_trip_matches_the_table():
    """tests/golden/reconstruction_n64.json holds the oracle's own N = 64 round trip (8192 solves, written by
    make_reconstruction_golden.py); its error is the table's 1.736e-9 to within the same margin as the rows above."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                       "reconstruction_n64.json")))
    assert 0.5 * gold["paper_error"] < gold["oracle_error"] < 1.25 * gold["paper_error"]
    g = O.make_grid(gold["N"], gold["L"])
    for s in gold["samples"][:3]:  # spot-check three stored reflection values against a fresh oracle solve
        k = g.xi[s["p2"], s["p1"]]
        assert abs(O.reflection_coefficient(g, np.exp(-np.abs(g.z) ** 2), k) - complex(*s["r"])) < 1e-13
