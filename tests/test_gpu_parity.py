"""GPU parity: the HIP library (through its C ABI) against the oracle, element by element on seeded inputs.

Tolerances (relative to the largest magnitude of the reference):
* FP64 transforms: 1e-13 (a length-N FFT accumulates O(eps log N) relative error, eps = 1.1e-16);
* FP64 operator / regularised inverse: 1e-12 (adds z^n-weighted moment sums, whose rounding grows with |z|^n, and
  the closed-form tail evaluated by a different but equally accurate recurrence);
* FP32 transforms and operator: 2e-5 (eps_32 = 6e-8 times the same growth factors);
* FP64 solves: 1e-10 relative L-infinity error of S and m (GMRES stops at a relative residual of 1e-12; the dense
  LU pins show condition numbers below 50, so the error bound kappa * tol is far below 1e-10).
"""
import numpy as np
import pytest

import dbar_workloads as W
from oracle import dbar_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1508_02363_amd import dbar as D  # noqa: E402


def relerr(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def rand_c(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def smooth_xi(g, rng, width=3.0):
    """A random smooth, rapidly decaying xi-space function (as the Krylov vectors are)."""
    base = rand_c(rng, (g.N, g.N))
    return O.Fd(g, np.exp(-np.abs(g.z) ** 2 / width) * O.Fd_inv(g, base * np.exp(-np.abs(g.xi) ** 2 / 8)))


SIZES = [8, 16, 32, 64, 128, 256, 512]


@pytest.mark.parametrize("N", SIZES + [1024, 2048, 4096])
def test_transform_fp64(N):
    rng = np.random.default_rng(N)
    L = 0.25 * N / 8 + 1.0
    g = O.make_grid(N, L)
    f = rand_c(rng, (N, N))
    assert relerr(D.transform(f, L), O.Fd(g, f)) < 1e-13
    assert relerr(D.transform(f, L, inverse=True), O.Fd_inv(g, f)) < 1e-13


@pytest.mark.parametrize("N", [16, 128, 1024, 4096])
def test_transform_fp32(N):
    rng = np.random.default_rng(N + 1)
    L = 3.0
    g = O.make_grid(N, L)
    f = rand_c(rng, (N, N))
    assert relerr(D.transform(f, L, precision=D.DBAR_FP32), O.Fd(g, f)) < 2e-5
    assert relerr(D.transform(f, L, inverse=True, precision=D.DBAR_FP32), O.Fd_inv(g, f)) < 2e-5


@pytest.mark.parametrize("N", SIZES + [1024, 2048])
def test_regularised_inverse_random(N):
    rng = np.random.default_rng(100 + N)
    L = max(1.0, N / 32.0)
    g = O.make_grid(N, L)
    S = smooth_xi(g, rng)
    want, _, _ = O.regularised_h(g, S, 11)
    assert relerr(D.dbar_inverse(S, L), want) < 1e-12


def test_regularised_inverse_dbartest_fig1():
    """The paper's inversion test (a = 1/2, b = 1, c = i, L = 4, N = 128, M = 11): GPU equals the exact inverse to
    machine precision, as the oracle does."""
    g = O.make_grid(128, 4.0)
    f = np.exp(-0.5 * (g.z - 1.0) * (np.conj(g.z) - 1j))
    exact = 0.5j * (1 - f) / (0.5 * (g.z - 1.0))
    h = D.dbar_inverse(O.Fd(g, f), 4.0)
    assert np.max(np.abs(h - exact)) < 1e-13


@pytest.mark.parametrize("N,k", [(8, 0.3 + 0.1j), (16, 1 + 0.5j), (32, -0.7 + 0.2j), (64, 1.5 - 1.0j),
                                 (128, 1 + 0.5j), (256, -2.0 + 2.0j), (512, 3.0 - 1.0j), (1024, -1.5 - 2.5j),
                                 (2048, 4.0 + 0.5j)])
def test_apply_fp64(N, k):
    rng = np.random.default_rng(200 + N)
    L = max(1.0, N / 32.0)
    g = O.make_grid(N, L)
    Q = (0.8 + 0.6j) * np.exp(-np.abs(g.z) ** 2)
    S = smooth_xi(g, rng)
    assert relerr(D.apply(Q, k, S, L), O.apply_A(g, Q, k, S)) < 1e-12


@pytest.mark.parametrize("N,L", [(16, 1.0), (128, 4.0), (512, 16.0), (2048, 6.0), (2048, 16.0)])
def test_apply_fp32(N, L):
    """The FP32 operator on S (the xi-space form) against the oracle's FP64 one, for L up to 16.  Beyond, this form
    loses accuracy (measured against the FP64 operator at N = 1024 and 2048: about 1e-6 at L = 16, 1e-4 at 24, 1e-3
    at 32, O(1) from 48 on): the FP32 rounding of S (relative to S's size) becomes through the inverse transform an
    error floor over the whole x grid, which its moments weight by |z|^n up to (pi L sqrt 2)^M.  The x-space form
    (the default) rounds s itself, relative to each value, and has no such limit (test_mixed_solve_at_large_L)."""
    rng = np.random.default_rng(300 + N)
    g = O.make_grid(N, L)
    Q = W.potential_gaussian_sum(N, L, seed=N)
    S = smooth_xi(g, rng)
    k = 0.5 - 0.25j
    err = relerr(D.apply(Q, k, S, L, precision=D.DBAR_FP32), O.apply_A(g, Q, k, S))
    print(f"FP32 operator N={N} L={L}: err {err:.2e}", flush=True)
    assert err < 2e-5


def test_mixed_solve_at_large_L():
    """The default mixed solver (GMRES on s in x-space) at N = 2048, L = 64 (the xi grid reaches |xi| = 16, where
    e^{-|xi|^2} has vanished, as the regularisation needs): it converges as at small L, equals the FP64 solver's
    result, and the oracle's FP64 operator confirms the residual of one k."""
    N, L = 2048, 64.0
    Q = W.potential_gaussian_sum(N, L, seed=7, amp_max=1.0)
    ks = [0.5 + 0.5j, 1.5 - 1j]
    print(f"mixed and FP64 solves N={N} L={L}", flush=True)
    S, m, info = D.solve(Q, ks, L, tol=1e-12, precision=D.DBAR_MIXED)
    S64, m64, info64 = D.solve(Q, ks, L, tol=1e-12, precision=D.DBAR_FP64)
    for j in range(len(ks)):
        assert info[j].status == 0 and info[j].rel_residual <= 1e-12, j
        assert relerr(S[j], S64[j]) < 1e-10 and relerr(m[j], m64[j]) < 1e-10, j
    del m, S64, m64
    print(f"oracle operator N={N} L={L}", flush=True)
    g = O.make_grid(N, L)
    b = O.rhs(g, Q, ks[0])
    r = b - O.apply_A(g, Q, ks[0], S[0])
    assert np.linalg.norm(r) / np.linalg.norm(b) < 1e-11


def test_residual_that_is_not_finite_is_not_converged():
    """An entry whose FP64 residual is not finite never counts as converged: it ends with DBAR_ENOCONV (and a residual
    that is not finite).  The mixed solver on S at N = 512, L = 64 takes its FP32 operator out of its range (see
    test_apply_fp32) and its iterates overflow; whatever the entries' outcome, a status of 0 must come with a finite
    S within tol."""
    N, L = 512, 64.0
    Q = W.potential_gaussian_sum(N, L, seed=7, amp_max=1.0)
    print(f"mixed xi-space solve N={N} L={L}", flush=True)
    S, m, info = D.solve(Q, [0.5 + 0.5j, 1.5 - 1j], L, tol=1e-12, precision=D.DBAR_MIXED, space=D.DBAR_SPACE_XI,
                         max_iter=300)
    for j, i in enumerate(info):
        print(f"entry {j}: status {i.status}, residual {i.rel_residual:.2e}, cycles {i.outer}", flush=True)
        if i.status == 0:
            assert np.all(np.isfinite(S[j])) and np.all(np.isfinite(m[j])) and i.rel_residual <= 1e-12, j
        else:
            assert i.status == D.DBAR_ENOCONV, j


def test_apply_born_closed_form():
    """K(S0) on the GPU equals the corrected closed-form first Born term (Section 5.1)."""
    from test_oracle_operator import born_S1
    g = O.make_grid(128, 4.0)
    A, k = 0.8 + 0.6j, 1 + 0.5j
    Q = A * np.exp(-np.abs(g.z) ** 2)
    S0 = O.rhs(g, Q, k)
    K_S0 = S0 - D.apply(Q, k, S0, 4.0)
    assert np.max(np.abs(K_S0 - born_S1(g, A, k))) < 1e-13


@pytest.mark.parametrize("mode", [D.DBAR_MODE_PLAIN, D.DBAR_MODE_BATCHED])
def test_solve_plain_n128(mode):
    w = W.workload("plain_n128")
    g = O.make_grid(w.N, w.L)
    ref = O.solve(g, w.Q, w.ks[0], tol=1e-13)
    S, m, info = D.solve(w.Q, w.ks, w.L, tol=w.tol, mode=mode)
    assert info[0].status == 0 and info[0].rel_residual <= w.tol
    assert relerr(S[0], ref.S) < 1e-10
    assert relerr(m[0], ref.m) < 1e-10
    assert abs(info[0].m1 - ref.m1) < 1e-10 * abs(ref.m1)


def test_solve_batched_small_grid_many_k():
    """Eight k values in one batch on N = 64 against the oracle, with different iteration counts per k."""
    N, L = 64, 3.0
    g = O.make_grid(N, L)
    Q = W.potential_gaussian_sum(N, L, seed=7)
    ks = W.k_disk(8, 2.0, seed=8)
    S, m, info = D.solve(Q, ks, L, tol=1e-12, batch=8)
    for j, k in enumerate(ks):
        ref = O.solve(g, Q, k, tol=1e-13)
        assert info[j].status == 0
        assert relerr(S[j], ref.S) < 1e-10, j
        assert relerr(m[j], ref.m) < 1e-10, j


def test_solve_zero_potential():
    N, L = 32, 3.0
    S, m, info = D.solve(np.zeros((N, N)), [1 + 1j, 0.5], L, tol=1e-12)
    assert np.all(S == 0) and np.all(m == 0)
    assert info[0].iters == 0 and info[0].status == 0


def test_mixed_solve_meeting_tol_in_its_first_cycle():
    """The first cycle's residual evaluation of a mixed solve leaves S and m unwritten (it cannot be the last when tol
    is far below the inner tolerance), and an entry that meets tol there all the same runs one more cycle, whose
    evaluation writes them.  A potential of 2^-66 times small integers at k = 0 makes the first cycle exact to FP64
    rounding (the right-hand side is FP32-exact and the operator the identity to 1e-20): the outputs must still be
    the solution, equal to the FP64 solver's and the oracle's."""
    N, L = 32, 3.0
    rng = np.random.default_rng(5)
    Q = (rng.integers(-4, 5, (N, N)) + 1j * rng.integers(-4, 5, (N, N))) * 2.0 ** -66
    S, m, info = D.solve(Q, [0.0], L, tol=1e-12, precision=D.DBAR_MIXED)
    S64, m64, info64 = D.solve(Q, [0.0], L, tol=1e-12, precision=D.DBAR_FP64)
    print(f"first-cycle solve: cycles {info[0].outer}, iterations {info[0].iters}, "
          f"residual {info[0].rel_residual:.2e}", flush=True)
    assert info[0].status == 0 and info[0].rel_residual <= 1e-12
    assert np.all(np.isfinite(S)) and np.any(S != 0)
    assert relerr(S[0], S64[0]) < 1e-10 and relerr(m[0], m64[0]) < 1e-10
    ref = O.solve(O.make_grid(N, L), Q, 0.0, tol=1e-13)
    assert relerr(S[0], ref.S) < 1e-10 and relerr(m[0], ref.m) < 1e-10


def test_solve_mixed_precision_n128():
    w = W.workload("plain_n128")
    g = O.make_grid(w.N, w.L)
    ref = O.solve(g, w.Q, w.ks[0], tol=1e-13)
    S, m, info = D.solve(w.Q, w.ks, w.L, tol=1e-12, precision=D.DBAR_MIXED)
    assert info[0].status == 0 and info[0].rel_residual <= 1e-12
    assert relerr(S[0], ref.S) < 1e-10
    assert relerr(m[0], ref.m) < 1e-10


def test_graph_replay_equals_direct_launches():
    """Krylov iterations replayed from captured HIP graphs give bit-identical results to direct launches, over two
    consecutive calls (the second replays the graphs captured by the first)."""
    N, L = 64, 3.0
    Q = W.potential_gaussian_sum(N, L, seed=21)
    ks = W.k_disk(6, 2.5, seed=22)
    S0, m0, i0 = D.solve(Q, ks, L, tol=1e-12, batch=6, use_graph=0)
    for _ in range(2):
        S1, m1, i1 = D.solve(Q, ks, L, tol=1e-12, batch=6, use_graph=1)
        assert np.array_equal(S0, S1) and np.array_equal(m0, m1)
        assert [a.iters for a in i0] == [a.iters for a in i1]


def test_solve_two_gram_schmidt_passes():
    w = W.workload("plain_n128")
    g = O.make_grid(w.N, w.L)
    ref = O.solve(g, w.Q, w.ks[0], tol=1e-13)
    S, m, info = D.solve(w.Q, w.ks, w.L, tol=1e-12, reorth=2)
    assert info[0].status == 0 and relerr(S[0], ref.S) < 1e-10 and relerr(m[0], ref.m) < 1e-10


def test_max_iter_reports_no_convergence():
    """Forced from the host: two iterations cannot reach 1e-12; the call reports DBAR_ENOCONV per k and still
    writes the best iterate (its residual is below the initial one)."""
    w = W.workload("plain_n128")
    S, m, info = D.solve(w.Q, w.ks, w.L, tol=1e-12, max_iter=2, restart=2)
    assert info[0].status == D.DBAR_ENOCONV
    assert 1e-12 < info[0].rel_residual < 1.0
    assert np.all(np.isfinite(S)) and np.all(np.isfinite(m))


@pytest.mark.parametrize("space", [D.DBAR_SPACE_X, D.DBAR_SPACE_XI])
@pytest.mark.parametrize("prec", [D.DBAR_FP64, D.DBAR_MIXED])
def test_iterated_method_fig2_case(prec, space):
    """Section 5.3 solver on the GPU against the oracle's, at the Fig. 2 parameters (k = 8.5936 = 55/6.4, L = 3.2,
    N = 128), where the plain method cannot represent the solution; GMRES on F^{-1} h (default) and on h."""
    L, k, N = 3.2, 55 / 6.4, 128
    g = O.make_grid(N, L)
    Q = W.potential_gaussian(N, L, 1.0)
    ref = O.solve_iterated(g, Q, k, tol=1e-14)
    S, m, info = D.solve(Q, [k], L, tol=1e-12, method=D.DBAR_METHOD_ITERATED, precision=prec, space=space)
    assert info[0].status == 0 and info[0].rel_residual <= 1e-12
    assert relerr(S[0], ref.S) < 1e-10
    assert relerr(m[0], ref.m) < 1e-10
    assert abs(info[0].m1 - ref.m1) < 1e-10 * abs(ref.m1)


def test_iterated_method_batch():
    N, L = 64, 3.2
    g = O.make_grid(N, L)
    Q = W.potential_gaussian_sum(N, L, seed=31, amp_max=1.0)
    ks = [0.0, 2.5 + 2.5j, -5.0 + 1.25j, 3.75 - 6.25j]  # 2 k L on the grid (1/6.4 steps)
    S, m, info = D.solve(Q, ks, L, tol=1e-12, batch=4, method=D.DBAR_METHOD_ITERATED)
    for j, k in enumerate(ks):
        ref = O.solve_iterated(g, Q, k, tol=1e-14)
        assert info[j].status == 0, j
        assert relerr(S[j], ref.S) < 1e-10 and relerr(m[j], ref.m) < 1e-10, j


def test_iterated_method_rejects_k_off_the_grid():
    with pytest.raises(D.DbarError) as e:
        D.solve(np.zeros((32, 32)) + 0.1, [0.3 + 0.1j], 3.0, method=D.DBAR_METHOD_ITERATED)
    assert e.value.code == D._lib.DBAR_EINVAL


def test_release_frees_the_iterated_workspace():
    """dbar_release gives back every device array of the library's workspaces (both lanes'), including the two FP64
    arrays only the iterated x-space method allocates (32 MiB per lane here): free device memory after a release is
    the same after a plain solve and after an iterated one.  (A first solve and release come before the reference
    reading: the runtime keeps what it sets up at the first launches, such as the loaded code and the queues' scratch,
    for the process.)"""
    N, L = 512, 3.2
    Q = W.potential_gaussian(N, L, 1.0)
    free = []
    for method in (D.DBAR_METHOD_PLAIN, D.DBAR_METHOD_PLAIN, D.DBAR_METHOD_ITERATED):
        print(f"N={N} 8 k, batch 4 in two lanes, method {method}, then release", flush=True)
        S, m, info = D.solve(Q, [0.0] * 8, L, tol=1e-10, batch=4, lanes=2, method=method)
        assert all(i.status == 0 for i in info)
        D.release()
        torch.cuda.synchronize()
        free.append(torch.cuda.mem_get_info()[0])
    assert abs(free[2] - free[1]) <= 4 << 20, free


def test_ragged_batches_equal_single_solves():
    """nk = 7 in batches of 3 (3 + 3 + 1) gives the same S as one k per launch."""
    N, L = 64, 3.0
    Q = W.potential_gaussian_sum(N, L, seed=41)
    ks = W.k_disk(7, 2.0, seed=42)
    S3, m3, i3 = D.solve(Q, ks, L, tol=1e-12, batch=3)
    S1, m1, i1 = D.solve(Q, ks, L, tol=1e-12, mode=D.DBAR_MODE_PLAIN)
    assert all(a.status == 0 for a in i3 + i1)
    for j in range(7):
        assert relerr(S3[j], S1[j]) < 1e-10 and relerr(m3[j], m1[j]) < 1e-10, j


@pytest.mark.parametrize("M", [0, 5, 15])
def test_taylor_order_extremes(M):
    """M = 0 (G = c_0 e^{-|xi|^2}) and M = 15 (the largest order the kernels carry) against the oracle; any M other
    than 11 runs the generic unrolled paths of the moment and tail kernels."""
    N, L = 128, 4.0
    rng = np.random.default_rng(M)
    g = O.make_grid(N, L)
    Q = (0.8 + 0.6j) * np.exp(-np.abs(g.z) ** 2)
    S = smooth_xi(g, rng)
    k = 0.75 - 0.5j
    assert relerr(D.dbar_inverse(S, L, M=M), O.regularised_h(g, S, M)[0]) < 1e-12
    assert relerr(D.apply(Q, k, S, L, M=M), O.apply_A(g, Q, k, S, M)) < 1e-12
    assert relerr(D.apply(Q, k, S, L, M=M, precision=D.DBAR_FP32), O.apply_A(g, Q, k, S, M)) < 2e-5
    ref = O.solve(g, Q, k, tol=1e-13, M=M)
    Sg, mg, info = D.solve(Q, [k], L, tol=1e-12, M=M, precision=D.DBAR_MIXED)
    assert info[0].status == 0 and relerr(Sg[0], ref.S) < 1e-10 and relerr(mg[0], ref.m) < 1e-10
    # the iterated method (fused steps, shifted moments and tail at this order)
    ki = (3 - 2j) / (2 * L)
    refi = O.solve_iterated(g, Q, ki, tol=1e-13, M=M)
    Si, mi, infoi = D.solve(Q, [ki], L, tol=1e-12, M=M, precision=D.DBAR_MIXED, method=D.DBAR_METHOD_ITERATED)
    assert infoi[0].status == 0 and relerr(Si[0], refi.S) < 1e-10 and relerr(mi[0], refi.m) < 1e-10


def test_default_batch_with_many_k():
    """batch = 0 lets the library choose entries per launch (tuned, else 64 or about 2^24 / N^2 on small grids, capped
    by nk and by memory)."""
    N, L = 32, 2.0
    g = O.make_grid(N, L)
    Q = W.potential_gaussian(N, L, 0.5 + 0.2j)
    ks = W.k_square_grid(-1.5, 1.5, 9)  # 80 k
    S, m, info = D.solve(Q, ks, L, tol=1e-12)
    assert len(info) == len(ks) and all(i.status == 0 for i in info)
    for j in (0, 41, 79):
        ref = O.solve(g, Q, ks[j], tol=1e-13)
        assert relerr(S[j], ref.S) < 1e-10, j


@pytest.mark.parametrize("prec", [D.DBAR_FP64, D.DBAR_MIXED])
def test_plain_method_at_k_zero(prec):
    """k = 0 (e_k = 1: the operator K0 of Section 5.1) in a batch with nonzero k."""
    N, L = 64, 3.0
    g = O.make_grid(N, L)
    Q = W.potential_gaussian_sum(N, L, seed=51)
    ks = [0.0, 0.5 - 1.0j, 0.0 + 0.0j]
    S, m, info = D.solve(Q, ks, L, tol=1e-12, batch=3, precision=prec)
    for j, k in enumerate(ks):
        ref = O.solve(g, Q, k, tol=1e-13)
        assert info[j].status == 0 and relerr(S[j], ref.S) < 1e-10 and relerr(m[j], ref.m) < 1e-10, j
    assert np.array_equal(S[0], S[2])


@pytest.mark.parametrize("space", [D.DBAR_SPACE_X, D.DBAR_SPACE_XI])
@pytest.mark.parametrize("prec", [D.DBAR_FP64, D.DBAR_MIXED])
def test_solve_in_both_spaces(prec, space):
    """GMRES on s = F^{-1} S (default) and on S itself: both against the oracle, N = 64 (several column tiles),
    a ragged batch of 5 with k = 0 in it."""
    N, L = 64, 3.0
    g = O.make_grid(N, L)
    Q = W.potential_gaussian_sum(N, L, seed=61)
    ks = [0.0] + list(W.k_disk(6, 2.5, seed=62))
    S, m, info = D.solve(Q, ks, L, tol=1e-12, batch=5, precision=prec, space=space)
    for j, k in enumerate(ks):
        ref = O.solve(g, Q, k, tol=1e-13)
        assert info[j].status == 0 and info[j].rel_residual <= 1e-12, j
        assert relerr(S[j], ref.S) < 1e-10 and relerr(m[j], ref.m) < 1e-10, j
        assert abs(info[j].m1 - ref.m1) <= 1e-10 * max(abs(ref.m1), 1e-300), j


def test_spaces_take_the_same_krylov_steps():
    """F is unitary up to a constant, so FP64 GMRES on s and on S runs the same iterations (up to rounding) and
    reports the same residual ratio."""
    N, L = 128, 5.0
    Q = W.potential_gaussian_sum(N, L, seed=63)
    ks = W.k_disk(8, 3.0, seed=64)
    Sx, mx, ix = D.solve(Q, ks, L, tol=1e-12, batch=8, space=D.DBAR_SPACE_X, orth_window=0)
    Sq, mq, iq = D.solve(Q, ks, L, tol=1e-12, batch=8, space=D.DBAR_SPACE_XI)
    for j in range(len(ks)):
        assert abs(ix[j].iters - iq[j].iters) <= 1, j
        assert relerr(Sx[j], Sq[j]) < 1e-10 and relerr(mx[j], mq[j]) < 1e-10, j


@pytest.mark.parametrize("prec", [D.DBAR_FP64, D.DBAR_MIXED])
def test_gram_schmidt_window_reaches_the_full_solution(prec):
    """Orthogonalising each new basis vector against the last few only changes the Krylov steps, not the answer: every
    window gives S and m of the fully orthogonalised solve to the tolerance, with the FP64 residual met, and the
    oracle's S at k = 0."""
    N, L = 128, 5.0
    g = O.make_grid(N, L)
    Q = W.potential_gaussian_sum(N, L, seed=65)
    ks = np.concatenate([[0.0], W.k_disk(6, 3.0, seed=66)])
    S0, m0, i0 = D.solve(Q, ks, L, tol=1e-12, batch=7, precision=prec, orth_window=0)
    ref = O.solve(g, Q, ks[0], tol=1e-13)
    for win in (1, 2, 3):
        S, m, info = D.solve(Q, ks, L, tol=1e-12, batch=7, precision=prec, orth_window=win)
        for j in range(len(ks)):
            assert info[j].status == 0 and info[j].rel_residual <= 1e-12, (win, j)
            assert relerr(S[j], S0[j]) < 1e-10 and relerr(m[j], m0[j]) < 1e-10, (win, j)
            assert info[j].iters <= 2 * i0[j].iters + 4, (win, j)
        assert relerr(S[0], ref.S) < 1e-10, win


@pytest.mark.parametrize("prec", [D.DBAR_FP64, D.DBAR_MIXED])
def test_gram_schmidt_window_with_short_restarts(prec):
    """Restart lengths shorter than a cycle's convergence (several restarts per refinement cycle), with windows up to the
    restart length: the same converged S and m as the full method with a long restart."""
    N, L = 64, 4.0
    Q = W.potential_gaussian_sum(N, L, seed=67)
    ks = W.k_disk(5, 2.5, seed=68)
    S0, m0, _ = D.solve(Q, ks, L, tol=1e-12, batch=5, precision=prec, orth_window=0, restart=40)
    for restart, win in ((4, 2), (4, 4), (6, 1)):
        S, m, info = D.solve(Q, ks, L, tol=1e-12, batch=5, precision=prec, orth_window=win, restart=restart)
        for j in range(len(ks)):
            assert info[j].status == 0 and info[j].rel_residual <= 1e-12, (restart, win, j)
            assert relerr(S[j], S0[j]) < 1e-10 and relerr(m[j], m0[j]) < 1e-10, (restart, win, j)


@pytest.mark.parametrize("prec", [D.DBAR_FP64, D.DBAR_MIXED])
def test_strong_potential_converges_with_the_default_window(prec):
    """A potential six times the benchmark's, where orthogonalising against the last two vectors alone stalls: the
    default solve notices the stalled cycle, orthogonalises fully from then on, and converges to the full method's
    solution (and the oracle's at one k)."""
    N, L = 64, 4.0
    g = O.make_grid(N, L)
    Q = 6.0 * (0.8 + 0.6j) * np.exp(-np.abs(g.z) ** 2)
    ks = np.array([0.5 + 0.5j, -1 + 0.3j, 2 - 1j])
    S0, m0, i0 = D.solve(Q, ks, L, tol=1e-12, batch=3, precision=prec, orth_window=0)
    S, m, info = D.solve(Q, ks, L, tol=1e-12, batch=3, precision=prec)
    for j in range(len(ks)):
        assert info[j].status == 0 and info[j].rel_residual <= 1e-12, j
        assert relerr(S[j], S0[j]) < 1e-10 and relerr(m[j], m0[j]) < 1e-10, j
        assert info[j].iters <= 3 * i0[j].iters + 40, j
    ref = O.solve(g, Q, ks[0], tol=1e-13)
    assert relerr(S[0], ref.S) < 1e-10


@pytest.mark.parametrize("prec", [D.DBAR_FP64, D.DBAR_MIXED])
def test_iterated_fused_step_matches_separate_update(prec):
    """The iterated method on F^{-1} h with its Gram-Schmidt update fused into B's first launch (one pass) and with
    separate update launches (two passes): the same S, m and m1 to the tolerance, iteration counts within one."""
    N, L = 64, 3.0
    Q = W.potential_gaussian_sum(N, L, seed=73)
    ks = [0.0, (3 - 1j) / (2 * L), (-5 + 6j) / (2 * L), (9 + 2j) / (2 * L)]
    S1, m1, i1 = D.solve(Q, ks, L, tol=1e-12, batch=4, precision=prec, method=D.DBAR_METHOD_ITERATED, reorth=1)
    S2, m2, i2 = D.solve(Q, ks, L, tol=1e-12, batch=4, precision=prec, method=D.DBAR_METHOD_ITERATED, reorth=2)
    for j in range(len(ks)):
        assert i1[j].status == 0 and i1[j].rel_residual <= 1e-12, j
        assert relerr(S1[j], S2[j]) < 1e-10 and relerr(m1[j], m2[j]) < 1e-10, j
        assert abs(i1[j].m1 - i2[j].m1) <= 1e-10 * max(abs(i2[j].m1), 1e-300), j
        if prec == D.DBAR_FP64:
            assert abs(i1[j].iters - i2[j].iters) <= 1, j


@pytest.mark.parametrize("prec", [D.DBAR_FP64, D.DBAR_MIXED])
def test_iterated_method_spaces_agree_on_a_batch(prec):
    """The iterated solver on F^{-1} h and on h: a ragged batch of 6 grid k (2kL integer, one k = 0), S, m and m1 to
    the oracle's tolerance, iteration counts within one."""
    N, L = 64, 3.0
    g = O.make_grid(N, L)
    Q = W.potential_gaussian_sum(N, L, seed=71)
    ks = [0.0, (1 + 2j) / (2 * L), (-3 + 1j) / (2 * L), (5 - 4j) / (2 * L), (-7 - 2j) / (2 * L), (2 + 9j) / (2 * L)]
    out = {}
    for sp in (D.DBAR_SPACE_X, D.DBAR_SPACE_XI):
        out[sp] = D.solve(Q, ks, L, tol=1e-12, batch=4, precision=prec, method=D.DBAR_METHOD_ITERATED, space=sp)
    for j, k in enumerate(ks[:3]):
        ref = O.solve_iterated(g, Q, k, tol=1e-13)
        S, m, info = out[D.DBAR_SPACE_X]
        assert info[j].status == 0 and relerr(S[j], ref.S) < 1e-10 and relerr(m[j], ref.m) < 1e-10, j
    Sx, mx, ix = out[D.DBAR_SPACE_X]
    Sq, mq, iq = out[D.DBAR_SPACE_XI]
    for j in range(len(ks)):
        assert relerr(Sx[j], Sq[j]) < 1e-10 and relerr(mx[j], mq[j]) < 1e-10, j
        assert abs(ix[j].m1 - iq[j].m1) <= 1e-10 * max(abs(iq[j].m1), 1e-300), j
        if prec == D.DBAR_FP64:
            assert abs(ix[j].iters - iq[j].iters) <= 1, j


@pytest.mark.parametrize("method", [D.DBAR_METHOD_PLAIN, D.DBAR_METHOD_ITERATED])
def test_device_outputs_equal_host_outputs(method):
    """solve_device writes S and m straight into the caller's tensors (several batches of a ragged k list): the
    values, m1 and the iteration counts equal those of the host-buffer call (which stages them), bit for bit."""
    N, L = 64, 3.0
    Q = W.potential_gaussian_sum(N, L, seed=81)
    ks = [0.0, (2 - 1j) / (2 * L), (-4 + 3j) / (2 * L), (1 + 5j) / (2 * L), (-6 - 2j) / (2 * L)]
    kw = dict(tol=1e-12, batch=2, precision=D.DBAR_MIXED, method=method)
    Sh, mh, ih = D.solve(Q, ks, L, **kw)
    Sd, md, idv = D.solve_device(torch.from_numpy(Q).to("cuda:0"), ks, L, **kw)
    assert np.array_equal(Sd.cpu().numpy(), Sh) and np.array_equal(md.cpu().numpy(), mh)
    assert [i.iters for i in idv] == [i.iters for i in ih] and [i.m1 for i in idv] == [i.m1 for i in ih]


def test_device_outputs_zero_potential():
    """b = 0: no residual is evaluated, yet the caller's (uninitialised) tensors come back as S = m = 0."""
    N, L = 32, 3.0
    Qd = torch.zeros((N, N), dtype=torch.complex128, device="cuda:0")
    for method, ks in ((D.DBAR_METHOD_PLAIN, [1 + 1j, 0.5]), (D.DBAR_METHOD_ITERATED, [0.0, 1.0 / (2 * L)])):
        S, m, info = D.solve_device(Qd, ks, L, tol=1e-12, method=method)
        assert torch.all(S == 0) and torch.all(m == 0) and all(i.status == 0 and i.iters == 0 for i in info)


@pytest.mark.parametrize("prec", [D.DBAR_FP64, D.DBAR_MIXED])
def test_graphs_follow_the_grid_parameters(prec):
    """Captured Krylov graphs keep their kernels' arguments (the transform scales from L, the M-specialised kernels) by
    value: a later solve with the same N, batch and restart but another L or M must not replay them.  Each solve with
    graphs equals the same solve with direct launches, bit for bit and in iteration counts."""
    N = 64
    ks = W.k_disk(4, 2.0, seed=32)
    for (L1, M1), (L2, M2) in (((3.0, 11), (4.0, 11)), ((4.0, 11), (4.0, 5))):
        Q1 = W.potential_gaussian_sum(N, L1, seed=31)
        Q2 = W.potential_gaussian_sum(N, L2, seed=31)
        D.solve(Q1, ks, L1, M=M1, tol=1e-12, batch=4, precision=prec, use_graph=1)  # captures
        Sg, mg, ig = D.solve(Q2, ks, L2, M=M2, tol=1e-12, batch=4, precision=prec, use_graph=1)
        Sd, md, idd = D.solve(Q2, ks, L2, M=M2, tol=1e-12, batch=4, precision=prec, use_graph=0)
        assert [(a.iters, a.outer) for a in ig] == [(a.iters, a.outer) for a in idd], (L2, M2)
        assert np.array_equal(Sg, Sd) and np.array_equal(mg, md), (L2, M2)


@pytest.mark.parametrize("prec", [D.DBAR_FP64, D.DBAR_MIXED])
def test_batch_entries_do_not_depend_on_each_other(prec):
    """A strong potential (six times the benchmark's), where some entries stall under the Gram-Schmidt window and
    switch to full orthogonalisation: every entry of the batch takes the same steps and reaches the same bits as the
    same k solved alone, whatever the other entries did."""
    N, L = 64, 4.0
    g = O.make_grid(N, L)
    Q = 6.0 * (0.8 + 0.6j) * np.exp(-np.abs(g.z) ** 2)
    ks = np.array([0.5 + 0.5j, -1 + 0.3j, 2 - 1j, 0.1 - 0.2j])
    S, m, info = D.solve(Q, ks, L, tol=1e-12, batch=len(ks), precision=prec)
    for j, k in enumerate(ks):
        S1, m1, i1 = D.solve(Q, [k], L, tol=1e-12, batch=1, precision=prec)
        assert (info[j].iters, info[j].outer) == (i1[0].iters, i1[0].outer), j
        assert np.array_equal(S[j], S1[0]) and np.array_equal(m[j], m1[0]), j


@pytest.mark.parametrize("prec,method", [(D.DBAR_FP64, D.DBAR_METHOD_PLAIN), (D.DBAR_MIXED, D.DBAR_METHOD_PLAIN),
                                         (D.DBAR_MIXED, D.DBAR_METHOD_ITERATED)])
def test_lanes_give_the_same_results(prec, method):
    """A batched solve split into two concurrent lanes (the default for batches of 16 or more: two parts, each on a
    stream and workspace of its own) returns exactly what one lane returns: 20 k at batch 16 make parts of 8, 8 and
    4 (the last one the first lane's second part), with device outputs written by both lanes."""
    N, L = 64, 4.0
    g = O.make_grid(N, L)
    Q = (0.8 + 0.6j) * np.exp(-np.abs(g.z) ** 2)
    rng = np.random.default_rng(21)
    if method == D.DBAR_METHOD_ITERATED:  # 2k on the xi grid
        ks = (rng.integers(-8, 9, 20) + 1j * rng.integers(-8, 9, 20)) / (2 * L)
    else:
        ks = 2.0 * np.sqrt(rng.random(20)) * np.exp(2j * np.pi * rng.random(20))
    kw = dict(tol=1e-12, batch=16, precision=prec, method=method)
    print(f"lanes: precision {prec} method {method}", flush=True)
    S1, m1, i1 = D.solve(Q, ks, L, lanes=1, **kw)
    S2, m2, i2 = D.solve(Q, ks, L, lanes=2, **kw)
    Qd = torch.from_numpy(Q).to("cuda:0")
    Sd, md, idv = D.solve_device(Qd, ks, L, lanes=2, **kw)
    torch.cuda.synchronize()
    for j in range(len(ks)):
        assert i1[j].status == 0 and (i1[j].iters, i1[j].outer) == (i2[j].iters, i2[j].outer), j
        assert i1[j].m1 == i2[j].m1 and i1[j].rel_residual == i2[j].rel_residual, j
        assert np.array_equal(S1[j], S2[j]) and np.array_equal(m1[j], m2[j]), j
        assert (idv[j].iters, idv[j].outer) == (i1[j].iters, i1[j].outer), j
    assert np.array_equal(Sd.cpu().numpy(), S1) and np.array_equal(md.cpu().numpy(), m1)
    ref = O.solve(g, Q, ks[0], tol=1e-13) if method == D.DBAR_METHOD_PLAIN else None
    if ref is not None:
        assert relerr(S2[0], ref.S) < 1e-10 and relerr(m2[0], ref.m) < 1e-10


@pytest.mark.parametrize("prec", [D.DBAR_FP64, D.DBAR_MIXED])
def test_error_estimate_reported_per_result(prec):
    """Every result carries a condition estimate from its Krylov Hessenberg matrix and err_estimate = estimate x the
    FP64 residual; on the small-grid workload the estimate stays within the dense-LU condition numbers measured on
    the CPU (below 50), and the error against the oracle is at the level the estimate states."""
    w = W.workload("plain_n128")
    g = O.make_grid(w.N, w.L)
    ref = O.solve(g, w.Q, w.ks[0], tol=1e-13)
    S, m, info = D.solve(w.Q, w.ks, w.L, tol=1e-12, precision=prec)
    i = info[0]
    print(f"cond_estimate {i.cond_estimate:.3f} err_estimate {i.err_estimate:.2e} "
          f"err vs oracle {relerr(S[0], ref.S):.2e}")
    assert 1.0 <= i.cond_estimate < 50.0
    assert i.err_estimate == pytest.approx(i.cond_estimate * i.rel_residual, rel=1e-12)
    assert i.err_estimate < 50 * 1e-12
    _, _, i0 = D.solve(np.zeros((32, 32)), [1.0], 3.0, tol=1e-12, precision=prec)
    assert i0[0].cond_estimate == 0.0 and i0[0].err_estimate == 0.0
