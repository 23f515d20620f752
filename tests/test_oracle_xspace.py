"""CPU pins of the iteration space the GPU solver uses: GMRES on s = F^{-1} S instead of S.

The discrete transforms of the paper's conventions (Section 1's F with the grid scalings of the x and xi domains)
satisfy F^{-1} F = identity and <F u, F v> = c <u, v> for the real inner product Re sum conj(u) v, with one constant
c for all u, v; hence GMRES on F^{-1} A F takes the images of the steps on A and reports the same residual ratio.
The x-space forms of the plain operator (Section 4) and of the iterated one (equation eqh2) follow by applying
F^{-1}; these tests check them against the oracle's operators written in xi-space."""
import numpy as np

import dbar_workloads as W
from oracle import dbar_oracle as O


def _rand(rng, N):
    return rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))


def _smooth(g, rng):
    return np.exp(-np.abs(g.z) ** 2 / 3) * _rand(rng, g.N)


def _ip(u, v):
    return float(np.sum((np.conj(u) * v).real))


def test_transform_pair_is_a_scaled_unitary_map():
    rng = np.random.default_rng(1)
    for N, L in ((16, 2.0), (32, 3.0)):
        g = O.make_grid(N, L)
        u, v = _rand(rng, N), _rand(rng, N)
        assert np.allclose(O.Fd_inv(g, O.Fd(g, u)), u, rtol=0, atol=1e-13 * np.abs(u).max())
        c = _ip(O.Fd(g, u), O.Fd(g, u)) / _ip(u, u)
        assert abs(_ip(O.Fd(g, u), O.Fd(g, v)) - c * _ip(u, v)) <= 1e-12 * c * np.sqrt(_ip(u, u) * _ip(v, v))
        dx = 2 * np.pi * L / N
        assert abs(c - (dx * dx / (2 * np.pi)) ** 2 * N * N) <= 1e-12 * c  # c = cf^2 N^2


def test_plain_operator_in_x_space():
    """F^{-1} A(F s) = s + i q_k conj(h(F s)) and F^{-1} b = -i q_k (b = -i F(q_k))."""
    rng = np.random.default_rng(2)
    N, L, k = 32, 3.0, 0.7 - 0.4j
    g = O.make_grid(N, L)
    Q = W.potential_gaussian_sum(N, L, seed=5)
    qk = Q * O.e_k(g, k)
    s = _smooth(g, rng)
    S = O.Fd(g, s)
    lhs = O.Fd_inv(g, O.apply_A(g, Q, k, S))
    h, _, _ = O.regularised_h(g, S, 11)
    rhs = s + 1j * qk * np.conj(h)
    assert np.max(np.abs(lhs - rhs)) <= 1e-12 * np.max(np.abs(rhs))
    assert np.allclose(O.Fd_inv(g, -1j * O.Fd(g, qk)), -1j * qk, rtol=0, atol=1e-13 * np.abs(qk).max())


def test_iterated_operator_in_x_space():
    """F^{-1} B(F eta) = eta + i Q conj(h0(F psi)) with psi = F^{-1} H(F eta) = -i Q conj(F^{-1}((F eta)/(xi - a)))
    (equation eqh2 on eta; h0 the regularised inverse about xi = 0)."""
    rng = np.random.default_rng(3)
    N, L = 32, 3.0
    k = (3 - 2j) / (2 * L)  # 2 k L integer: the shift lies on the grid
    g = O.make_grid(N, L)
    Q = W.potential_gaussian_sum(N, L, seed=6)
    eta = _smooth(g, rng)
    h = O.Fd(g, eta)
    lhs = O.Fd_inv(g, O.apply_B(g, Q, k, h))
    psi = -1j * Q * np.conj(O.shifted_inverse(g, h, k, 11))
    h0, _, _ = O.regularised_h(g, O.Fd(g, psi), 11)
    rhs = eta + 1j * Q * np.conj(h0)
    assert np.max(np.abs(lhs - rhs)) <= 1e-12 * np.max(np.abs(rhs))


def test_gmres_residual_ratio_is_the_same_in_both_spaces():
    """The residual ratio ||b - A S|| / ||b|| equals ||F^{-1}b - F^{-1}A(S)|| / ||F^{-1}b|| for any S."""
    rng = np.random.default_rng(4)
    N, L, k = 32, 3.0, 1.1 + 0.3j
    g = O.make_grid(N, L)
    Q = W.potential_gaussian_sum(N, L, seed=7)
    b = -1j * O.Fd(g, Q * O.e_k(g, k))
    S = O.Fd(g, _smooth(g, rng))
    r = b - O.apply_A(g, Q, k, S)
    ratio_xi = np.linalg.norm(r) / np.linalg.norm(b)
    ratio_x = np.linalg.norm(O.Fd_inv(g, r)) / np.linalg.norm(O.Fd_inv(g, b))
    assert abs(ratio_xi - ratio_x) <= 1e-13 * ratio_xi
