"""Oracle for the Fourier-spectral D-bar method (Klein & McLaughlin, "Spectral approach to D-bar problems").

TEST INFRASTRUCTURE ONLY.  This module is a plain, slow, obviously-correct CPU implementation in float64/complex128
of what the GPU library computes.  Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark may
import it; the GPU library never does, and this module imports nothing from it.

What is computed (paper Section 4, "Algorithm for computing a solution to the D-bar equation", with the potential Q
replaced by q_k = Q e^{conj(kz) - kz} as in Section 5.1, equation MainEQDS):

    A(S) = S + i F( q_k * conj(h(S)) ),     b = -i F(q_k),     solve A(S) = b,     m = h(S),

where h(S) is the regularised inverse transform of S/xi (Section 4.2, equations Sreg, Gchoice, fourreeg4 and the
closed forms fourreg / fourreg5 / fourreg5a), and A is real-linear (because of the conjugation), so GMRES runs on the
real vector [Re S, Im S] of length 2 N^2.

Readings taken where the paper is silent or garbled (each also recorded in the design notes):

* the value of (S - G)/xi at xi = 0 is the limit d S/d xi (0) = (-i/2) F(conj(z) F^{-1} S)(0), which follows from the
  Taylor expansion of S about xi = 0 displayed before equation Gchoice (the paper does not state it);
* the small-|z| series fourreg5a is missing a factor exp(-|z|^2/4); it is restored here (it is needed for
  fourreg5a to equal fourreg5, as the paper claims it does);
* the discrete transform is scaled and phased so that it approximates the continuous F of Section 1 on the grid of
  equations 'domain' and 'xidomain' (positive Nyquist wave number +N/(2L)).

Array layout: x-space arrays are indexed [iy, ix] with x_j = L(-pi + 2 pi j/N); xi-space arrays are indexed [p2, p1]
in FFT order, p <-> wave number m = p for p <= N/2 and m = p - N otherwise, xi = m / L.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Grid", "make_grid", "Fd", "Fd_inv", "omega", "omega_table", "moments", "G_coefficients", "regularised_h",
    "apply_A", "rhs", "gmres_real", "dense_matrix", "solve", "dense_solve", "SolveResult",
    "shift_index", "shifted_inverse", "apply_B", "solve_iterated",
    "reflection_coefficient", "reflection_grid", "evolve_reflection", "dual_grid", "reconstruct_potential",
]


# ----------------------------------------------------------------------------------------------------------------
# Grids (Section 4.1, equations 'domain' and 'xidomain')
# ----------------------------------------------------------------------------------------------------------------

@dataclass
class Grid:
    N: int
    L: float
    x: np.ndarray        # 1-D x_j
    z: np.ndarray        # [iy, ix] complex z = x + i y
    xi: np.ndarray       # [p2, p1] complex xi = xi1 + i xi2
    phase: np.ndarray    # [p2, p1] (-1)^(m1 + m2)
    dx: float


def make_grid(N: int, L: float) -> Grid:
    """x_j = L(-pi + 2 pi j / N) (periodic, N points), wave numbers m in [-N/2+1, N/2], xi = m / L."""
    j = np.arange(N)
    x = L * (-math.pi + 2.0 * math.pi * j / N)
    m = np.where(j <= N // 2, j, j - N)
    X, Y = np.meshgrid(x, x, indexing="xy")
    M1, M2 = np.meshgrid(m, m, indexing="xy")
    z = X + 1j * Y
    xi = M1 / L + 1j * (M2 / L)
    phase = np.where((M1 + M2) % 2 == 0, 1.0, -1.0)
    return Grid(N, L, x, z, xi, phase, 2.0 * math.pi * L / N)


# ----------------------------------------------------------------------------------------------------------------
# Discrete Fourier transform consistent with F(f)(xi) = (1/2pi) int f e^{-i xi.x} dx dy (Section 1)
# ----------------------------------------------------------------------------------------------------------------

def Fd(g: Grid, f: np.ndarray) -> np.ndarray:
    """Riemann sum of the continuous transform on the grid: (dx^2/2pi) sum_j f_j e^{-i xi_m . x_j}.
    Since e^{-i xi_m x_j} = (-1)^m e^{-2 pi i m j / N}, this is (dx^2/2pi) (-1)^(m1+m2) FFT2(f)."""
    return (g.dx * g.dx / (2.0 * math.pi)) * g.phase * np.fft.fft2(f)


def Fd_inv(g: Grid, S: np.ndarray) -> np.ndarray:
    """Riemann sum of the continuous inverse: (1/(2 pi L^2)) sum_m S_m e^{+i xi_m . x_j}."""
    N, L = g.N, g.L
    return (N * N / (2.0 * math.pi * L * L)) * np.fft.ifft2(g.phase * S)


# ----------------------------------------------------------------------------------------------------------------
# omega_n = c_n W_n / d_n: the closed-form inverse transform of the Gaussian-weighted anti-holomorphic Taylor terms
# (Lemma of Section 4.2: equations fourreg5, fourreg5a; the factorials cancel as noted after the algorithm)
# ----------------------------------------------------------------------------------------------------------------

def omega(n: int, z: np.ndarray) -> np.ndarray:
    """omega_n(z) such that c_n W_n = d_n omega_n, with c_n = (-i/2)^n d_n / n! and
    W_n = F^{-1}(conj(xi)^n e^{-|xi|^2} / xi).

    From fourreg5:  omega_n = i / z^{n+1} * (1 - e^{-u} sum_{k=0}^{n} u^k / k!),  u = |z|^2 / 4.
    From fourreg5a (with the factor e^{-u} restored): omega_n = i (conj(z)/4)^{n+1} e^{-u} sum_{k>=0} u^k/(k+n+1)!.
    The series form is used where u < n + 1 (no cancellation there); the closed form elsewhere.  omega_n(0) = 0.
    """
    z = np.asarray(z, dtype=np.complex128)
    u = (z.real ** 2 + z.imag ** 2) / 4.0
    out = np.zeros_like(z)
    small = u < (n + 1)
    # closed form (fourreg5)
    big = ~small
    if np.any(big):
        zb, ub = z[big], u[big]
        term = np.ones_like(ub)
        acc = np.ones_like(ub)
        for k in range(1, n + 1):
            term = term * ub / k
            acc = acc + term
        out[big] = 1j * (1.0 - np.exp(-ub) * acc) / zb ** (n + 1)
    # series (corrected fourreg5a)
    if np.any(small):
        zs, us = z[small], u[small]
        term = np.full_like(us, 1.0 / math.factorial(n + 1))
        acc = term.copy()
        for k in range(1, 400):
            term = term * us / (k + n + 1)
            acc = acc + term
            if np.all(term <= 1e-18 * acc):
                break
        out[small] = 1j * (np.conj(zs) / 4.0) ** (n + 1) * np.exp(-us) * acc
    return out


def omega_table(g: Grid, M: int) -> np.ndarray:
    """Stored omega_n(z_j) for n = 0..M on the grid (the paper stores the W_n 'beforehand')."""
    return np.stack([omega(n, g.z) for n in range(M + 1)])


# ----------------------------------------------------------------------------------------------------------------
# Taylor coefficients at xi = 0 by summation (equation fourreeg4 and the cost remark after the algorithm)
# ----------------------------------------------------------------------------------------------------------------

def moments(g: Grid, s: np.ndarray, M: int):
    """d_n = F(z^n s)(0) = (dx^2/2pi) sum_j z_j^n s_j for n = 0..M, and dt = F(conj(z) s)(0)."""
    w = g.dx * g.dx / (2.0 * math.pi)
    d = np.array([w * np.sum(g.z ** n * s) for n in range(M + 1)], dtype=np.complex128)
    dt = w * np.sum(np.conj(g.z) * s)
    return d, dt


def G_coefficients(d: np.ndarray) -> np.ndarray:
    """c_n = (1/n!) d^n S / d conj(xi)^n (0) = (-i/2)^n d_n / n!  (fourreeg4 and Gchoice)."""
    return np.array([(-0.5j) ** n * d[n] / math.factorial(n) for n in range(len(d))], dtype=np.complex128)


def regularised_h(g: Grid, S: np.ndarray, M: int, om: np.ndarray | None = None, zero_at_origin: bool = False):
    """h = F^{-1}(S/xi) with the regularisation of Section 4.2 (equations Sreg, Gchoice and S0Taylor):

        s   = F^{-1} S
        d_n = F(z^n s)(0),  dt = F(conj(z) s)(0)
        G   = e^{-|xi|^2} sum_n c_n conj(xi)^n
        R   = (S - G)/xi  for xi != 0,   R(0) = (-i/2) dt   (the limit dS/dxi(0))
        h   = F^{-1} R + sum_n c_n W_n = F^{-1} R + sum_n d_n omega_n

    ``zero_at_origin=True`` sets R(0) = 0 instead (used only by a test that shows this breaks spectral accuracy).
    Returns (h, d, dt).
    """
    if om is None:
        om = omega_table(g, M)
    s = Fd_inv(g, S)
    d, dt = moments(g, s, M)
    c = G_coefficients(d)
    xib = np.conj(g.xi)
    Gx = np.zeros_like(S)
    p = np.ones_like(S)
    for n in range(M + 1):
        Gx = Gx + c[n] * p
        p = p * xib
    Gx = np.exp(-np.abs(g.xi) ** 2) * Gx
    R = np.empty_like(S)
    nz = g.xi != 0
    R[nz] = (S[nz] - Gx[nz]) / g.xi[nz]
    R[~nz] = 0.0 if zero_at_origin else (-0.5j) * dt
    h = Fd_inv(g, R)
    for n in range(M + 1):
        h = h + d[n] * om[n]
    return h, d, dt


# ----------------------------------------------------------------------------------------------------------------
# The operator and right-hand side (Section 4 algorithm, Q -> q_k of Section 5.1)
# ----------------------------------------------------------------------------------------------------------------

def e_k(g: Grid, k: complex) -> np.ndarray:
    """e^{conj(kz) - kz} on the grid (equation eq:039)."""
    kz = complex(k) * g.z
    return np.exp(np.conj(kz) - kz)


def rhs(g: Grid, Q: np.ndarray, k: complex) -> np.ndarray:
    """b = -i F(Q e^{conj(kz)-kz})."""
    return -1j * Fd(g, Q * e_k(g, k))


def apply_A(g: Grid, Q: np.ndarray, k: complex, S: np.ndarray, M: int = 11, om=None, qk=None) -> np.ndarray:
    """A(S) = S + i F(q_k conj(h(S)))."""
    if qk is None:
        qk = Q * e_k(g, k)
    h, _, _ = regularised_h(g, S, M, om)
    return S + 1j * Fd(g, qk * np.conj(h))


# ----------------------------------------------------------------------------------------------------------------
# GMRES (Saad & Schultz) on the real form, modified Gram-Schmidt, Givens rotations, restarts
# ----------------------------------------------------------------------------------------------------------------

def _to_real(S: np.ndarray) -> np.ndarray:
    return np.concatenate([S.real.ravel(), S.imag.ravel()])


def _to_complex(v: np.ndarray, shape) -> np.ndarray:
    n = v.size // 2
    return (v[:n] + 1j * v[n:]).reshape(shape)


def gmres_real(matvec, b: np.ndarray, tol: float, restart: int = 40, max_iter: int = 2000):
    """Restarted GMRES on a real linear system (matvec: R^n -> R^n), x0 = 0, modified Gram-Schmidt.
    Stops when the recomputed true residual ||b - A x|| / ||b|| <= tol.  Returns (x, iterations, true_rel_res)."""
    n = b.size
    bnorm = np.linalg.norm(b)
    x = np.zeros(n)
    if bnorm == 0.0:
        return x, 0, 0.0
    its = 0
    r = b.copy()
    rel = 1.0
    while its < max_iter:
        beta = np.linalg.norm(r)
        V = np.zeros((restart + 1, n))
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        gvec = np.zeros(restart + 1)
        gvec[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(restart):
            w = matvec(V[j])
            its += 1
            for i in range(j + 1):
                H[i, j] = np.dot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = math.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            gvec[j + 1] = -sn[j] * gvec[j]
            gvec[j] = cs[j] * gvec[j]
            j_done = j + 1
            if abs(gvec[j + 1]) <= 0.1 * tol * bnorm or its >= max_iter:
                break
        y = np.linalg.solve(np.triu(H[:j_done, :j_done]), gvec[:j_done])
        x = x + V[:j_done].T @ y
        r = b - matvec(x)
        rel = np.linalg.norm(r) / bnorm
        if rel <= tol:
            break
    return x, its, rel


@dataclass
class SolveResult:
    S: np.ndarray
    m: np.ndarray
    m1: complex
    iters: int
    rel_residual: float


def solve(g: Grid, Q: np.ndarray, k: complex, tol: float = 1e-13, M: int = 11, restart: int = 40,
          max_iter: int = 2000, om=None) -> SolveResult:
    """Solve A(S) = b for one k; return S, m = h(S), m^(1) = i S(0) (equation m1def), iterations and true residual."""
    if om is None:
        om = omega_table(g, M)
    qk = Q * e_k(g, k)
    b = -1j * Fd(g, qk)
    shape = b.shape

    def mv(v):
        return _to_real(apply_A(g, Q, k, _to_complex(v, shape), M, om, qk))

    xr, its, rel = gmres_real(mv, _to_real(b), tol, restart, max_iter)
    S = _to_complex(xr, shape)
    h, _, _ = regularised_h(g, S, M, om)
    return SolveResult(S, h, 1j * S[0, 0], its, rel)


# ----------------------------------------------------------------------------------------------------------------
# Dense mode for tiny grids: the assembled real 2N^2 x 2N^2 matrix and a direct LU solve
# ----------------------------------------------------------------------------------------------------------------

def dense_matrix(g: Grid, Q: np.ndarray, k: complex, M: int = 11) -> np.ndarray:
    """Columns A(e_j) and A(i e_j) of the real-linear operator on [Re S, Im S]."""
    n = g.N * g.N
    om = omega_table(g, M)
    qk = Q * e_k(g, k)
    Amat = np.zeros((2 * n, 2 * n))
    for j in range(n):
        for part in (0, 1):
            E = np.zeros(n, np.complex128)
            E[j] = 1.0 if part == 0 else 1j
            col = apply_A(g, Q, k, E.reshape(g.N, g.N), M, om, qk)
            Amat[:, j + part * n] = _to_real(col)
    return Amat


def dense_solve(g: Grid, Q: np.ndarray, k: complex, M: int = 11):
    """S from numpy.linalg.solve (LAPACK gesv) on the assembled matrix; also returns the matrix."""
    Amat = dense_matrix(g, Q, k, M)
    b = _to_real(rhs(g, Q, k))
    x = np.linalg.solve(Amat, b)
    return _to_complex(x, (g.N, g.N)), Amat


# ----------------------------------------------------------------------------------------------------------------
# The iterated integral equation for large k (Section 5.2 equations Sform, eqh, eqh2; Section 5.3 algorithm) with
# the shifted regularisation of Section 5.1 (equation dbarinvShift).  2k lies on the xi grid (Section 5.3), so the
# shift by 2i conj(k) is an index roll.
# ----------------------------------------------------------------------------------------------------------------

def shift_index(g: Grid, k: complex):
    """Grid offsets (m1, m2) of a = 2i conj(k) = 2 k2 + 2i k1 on the xi grid: m1 = 2 k2 L, m2 = 2 k1 L."""
    k = complex(k)
    m1, m2 = 2.0 * k.imag * g.L, 2.0 * k.real * g.L
    r1, r2 = int(round(m1)), int(round(m2))
    if abs(m1 - r1) > 1e-9 or abs(m2 - r2) > 1e-9:
        raise ValueError("the iterated method needs 2k on the xi grid: 2 k1 L and 2 k2 L must be integers")
    return r1, r2


def shifted_inverse(g: Grid, h: np.ndarray, k: complex, M: int, om=None) -> np.ndarray:
    """F^{-1}(h / (xi - a)), a = 2i conj(k), for h concentrated near xi = 0, regularised about the singular point
    xi = a (equation dbarinvShift): with G_a = e^{-|xi - a|^2} sum_n c_n conj(xi - a)^n built from the Taylor
    coefficients of h at a,

        F^{-1}(h/(xi - a)) = F^{-1}((h - G_a)/(xi - a)) + F^{-1}(G_a/(xi - a)),

    where xi - a is formed from the grid's own xi (not reduced modulo the period), so the quotient is smooth inside
    the domain and only jumps at its edge, where h vanishes.  The Taylor coefficients are
    d^n h / d conj(xi)^n (a) = (-i/2)^n F(z^n e^{-i a.x} F^{-1} h)(0) (equation fourreeg4 at xi = a), and by the shift
    theorem F^{-1}(G_a/(xi - a)) = e^{i a.x} sum_n c_n W_n.  Note e^{-i a.x} = e^{conj(kz) - kz}.  The value of
    (h - G_a)/(xi - a) at xi = a is the limit dh/dxi(a)."""
    if om is None:
        om = omega_table(g, M)
    shift_index(g, k)  # a must be a grid point
    a = 2j * np.conj(complex(k))
    ek = e_k(g, k)
    s = Fd_inv(g, h)
    d, dt = moments(g, s * ek, M)
    c = G_coefficients(d)
    zeta = g.xi - a
    Ga = np.zeros_like(h)
    p = np.ones_like(h)
    for n in range(M + 1):
        Ga = Ga + c[n] * p
        p = p * np.conj(zeta)
    Ga = np.exp(-np.abs(zeta) ** 2) * Ga
    R = np.empty_like(h)
    nz = np.abs(zeta) > 1e-12
    R[nz] = (h[nz] - Ga[nz]) / zeta[nz]
    R[~nz] = (-0.5j) * dt
    r = Fd_inv(g, R)
    tail = np.zeros_like(r)
    for n in range(M + 1):
        tail = tail + d[n] * om[n]
    return r + np.conj(ek) * tail


def apply_B(g: Grid, Q: np.ndarray, k: complex, h: np.ndarray, M: int = 11, om=None) -> np.ndarray:
    """Left-hand side of equation eqh2: h - K0(H),  H = -i F(Q conj(F^{-1}(h/(xi - 2i conj k)))),
    K0(S) = -i F(Q conj(F^{-1}(S/xi))) (equation shift, with q = Q)."""
    H = -1j * Fd(g, Q * np.conj(shifted_inverse(g, h, k, M, om)))
    r, _, _ = regularised_h(g, H, M, om)
    return h + 1j * Fd(g, Q * np.conj(r))


def solve_iterated(g: Grid, Q: np.ndarray, k: complex, tol: float = 1e-13, M: int = 11, restart: int = 40,
                   max_iter: int = 2000, om=None) -> SolveResult:
    """Solve eqh2 for h with GMRES (right-hand side -i F(Q)).  Then f = H (the simplification after eqh2 shows
    K0(h o (xi + a)) o (xi + a) = H), S = f + h o (xi + a) (equation Sform; the second term is an index roll and
    is meaningful only while it stays inside the xi domain), m = F^{-1}(S/xi) = F^{-1}(f/xi) + e^{-i a.x} F^{-1}(h/(xi-a))
    (shift theorem), and m^(1) = i S(0) = i (f(0) + h(a)) (equation m1def)."""
    if om is None:
        om = omega_table(g, M)
    b = -1j * Fd(g, Q)
    shape = b.shape

    def mv(v):
        return _to_real(apply_B(g, Q, k, _to_complex(v, shape), M, om))

    xr, its, rel = gmres_real(mv, _to_real(b), tol, restart, max_iter)
    h = _to_complex(xr, shape)
    m1i, m2i = shift_index(g, k)
    ha = np.roll(h, (-m2i, -m1i), axis=(0, 1))
    si = shifted_inverse(g, h, k, M, om)
    f = -1j * Fd(g, Q * np.conj(si))
    S = f + ha
    rf, _, _ = regularised_h(g, f, M, om)
    m = rf + e_k(g, k) * si
    res = SolveResult(S, m, 1j * (f[0, 0] + ha[0, 0]), its, rel)
    res.h = h
    res.f = f
    return res


# ----------------------------------------------------------------------------------------------------------------
# DS II reflection coefficient (Section 6: equations MainEQDSpm, hpmdef, rviah, m1def, eq:023)
# ----------------------------------------------------------------------------------------------------------------

def reflection_coefficient(g: Grid, q: np.ndarray, k: complex, tol: float = 1e-13, M: int = 11, om=None) -> complex:
    """r(k) = i h(i conj k) (equation rviah) in the convention of Section 6 (k replaced by k/2, so that k lies on the
    xi grid): h solves the iterated equation for the potential q with spectral parameter k/2, whose shift is
    2i conj(k/2) = i conj(k).  The value at xi = i conj(k) is read at grid offsets (k2 L, k1 L)."""
    res = solve_iterated(g, q, complex(k) / 2.0, tol=tol, M=M, om=om)
    k = complex(k)
    p1, p2 = int(round(k.imag * g.L)) % g.N, int(round(k.real * g.L)) % g.N
    return 1j * res.h[p2, p1]


def reflection_grid(g: Grid, q: np.ndarray, tol: float = 1e-13, M: int = 11) -> np.ndarray:
    """r(k) for every k on the xi grid of g (Section 6 convention), laid out like S: r[p2, p1] is r at
    k = xi[p2, p1]."""
    om = omega_table(g, M)
    r = np.zeros((g.N, g.N), dtype=complex)
    for p2 in range(g.N):
        for p1 in range(g.N):
            r[p2, p1] = reflection_coefficient(g, q, g.xi[p2, p1], tol=tol, M=M, om=om)
    return r


def evolve_reflection(g: Grid, r: np.ndarray, t: float) -> np.ndarray:
    """r(k, t) = r(k, 0) exp(-i t (k^2 + conj(k)^2)/4) (equation rt), applied with k on the xi grid (the Section 6
    convention, in which the Remark of Section 6 writes the same factor as exp(-i t Re(k^2)/2))."""
    return r * np.exp(-0.5j * t * (g.xi ** 2).real)


def dual_grid(g: Grid) -> Grid:
    """The xi grid of g read as an x-space grid: spacing 1/L, points m/L for m = -N/2 .. N/2-1, i.e. half-length
    L' = N/(2 pi L).  Its own xi grid has spacing 2 pi L / N and contains every point of g's x grid."""
    return make_grid(g.N, g.N / (2.0 * math.pi * g.L))


def reconstruct_potential(g: Grid, r: np.ndarray, tol: float = 1e-13, M: int = 11) -> np.ndarray:
    """q on the x grid of g from r on its xi grid (equations dbarrecA, dbarrecB, qRec): the same D-bar problem with
    z and k interchanged and q replaced by conj(r), so q(z) = i h(i conj z) where h solves the iterated equation on
    the dual grid with potential conj(r) and spectral parameter z/2.  The FFT-ordered r is moved to the dual x
    grid by an fftshift; its Nyquist row and column (k = +N/(2L)) land at -N/(2L), the periodic image."""
    gp = dual_grid(g)
    P = np.fft.fftshift(np.conj(r))
    om = omega_table(gp, M)
    q = np.zeros((g.N, g.N), dtype=complex)
    for j2 in range(g.N):
        for j1 in range(g.N):
            q[j2, j1] = reflection_coefficient(gp, P, g.z[j2, j1], tol=tol, M=M, om=om)
    return q
