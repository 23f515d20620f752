"""GPU parity at the workloads' full sizes, in the launch configurations the benchmark and the batched path use.

* N = 1024, 16 k, batch 16, mixed precision (the benchmark's step): S and m against oracle solves for sampled k
  (the oracle's solve at N = 1024 takes seconds), and all 16 against the FP64 batched path.
* N = 512, the 1024 k of the 32 x 32 grid in [-6, 6]^2, FP64 batched after autotuning: every entry converges, and
  sampled k agree with the oracle.
* N = 4096, 64 k in |k| <= 8, mixed precision: every entry converges to the FP64 residual; S and m of sampled k
  against oracle solutions stored by tests/golden/make_fullsize_golden.py (an oracle solve at this size takes minutes,
  so it runs outside the test), element by element at ~2000 stored points each, to 1e-10 relative to the array's
  maximum; and for one k the oracle's own FP64 operator confirms ||b - A(S)|| / ||b||.
* N = 2048: the same against stored oracle solutions, for the plain and the iterated method.
"""
import json
import os

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


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    path = os.path.join(GOLDEN, f"fullsize_{name}.json")
    return json.load(open(path)) if os.path.exists(path) else None


def golden_err(arr, gold, key):
    """max |arr - oracle| over the stored points of `key` ("S" or "m"), relative to the oracle array's maximum."""
    idx = np.asarray(gold[f"{key}_idx"], dtype=np.int64)
    ref = np.asarray(gold[key], dtype=np.float64)
    got = np.asarray(arr).reshape(-1)[idx]
    return float(np.max(np.abs(got - (ref[:, 0] + 1j * ref[:, 1]))) / gold[f"max_abs_{key}"])


def test_bench_config_n1024_mixed():
    w = W.workload("plain_n1024")
    Qd = torch.from_numpy(w.Q).to("cuda:0")
    S, m, info = D.solve_device(Qd, w.ks, w.L, tol=w.tol, batch=len(w.ks), precision=D.DBAR_MIXED)
    S64, m64, info64 = D.solve_device(Qd, w.ks, w.L, tol=w.tol, batch=len(w.ks), precision=D.DBAR_FP64)
    S, m, S64, m64 = (t.cpu().numpy() for t in (S, m, S64, m64))
    assert all(i.status == 0 and i.rel_residual <= w.tol for i in info)
    for j in range(len(w.ks)):
        assert relerr(S[j], S64[j]) < 1e-10 and relerr(m[j], m64[j]) < 1e-10, j
    g = O.make_grid(w.N, w.L)
    om = O.omega_table(g, w.M)
    for j in (0, 9):
        print(f"oracle solve N=1024 k={w.ks[j]}", flush=True)
        ref = O.solve(g, w.Q, w.ks[j], tol=1e-13, om=om)
        assert relerr(S[j], ref.S) < 1e-10, j
        assert relerr(m[j], ref.m) < 1e-10, j


def test_batched_n512_all_k_autotuned():
    w = W.workload("batched_n512")
    try:
        tune = D.autotune(w.N, w.L, precision=D.DBAR_FP64, batch=64)
        print("tuning", tune, flush=True)
        Qd = torch.from_numpy(w.Q).to("cuda:0")
        S, m, info = D.solve_device(Qd, w.ks, w.L, tol=w.tol, precision=D.DBAR_FP64, want_m=False)
        assert len(info) == 1024 and all(i.status == 0 and i.rel_residual <= w.tol for i in info)
        g = O.make_grid(w.N, w.L)
        om = O.omega_table(g, w.M)
        for j in (0, 517, 1023):  # corner k = -6-6i, an interior one, corner 6+6i
            print(f"oracle solve N=512 k={w.ks[j]}", flush=True)
            ref = O.solve(g, w.Q, w.ks[j], tol=1e-13, om=om)
            assert relerr(S[j].cpu().numpy(), ref.S) < 1e-10, j
    finally:
        D.set_tile(w.N, D.DBAR_FP64, 0)


C4_GOLDEN = (0, 3, 14, 51)  # k indices with stored oracle solutions (|k| = 7.77, 2.28, 7.94, 1.64)


def test_mixed_n4096_against_oracle_solutions():
    """The 64-k N = 4096 workload in the benchmark's launch configuration (mixed precision, default batch): S and m of
    the k with stored oracle solutions, element by element; and the FP64 path at the same k."""
    w = W.workload("mixed_n4096")
    Qd = torch.from_numpy(w.Q).to("cuda:0")
    print("N=4096 mixed, 64 k", flush=True)
    S, m, info = D.solve_device(Qd, w.ks, w.L, tol=w.tol, precision=D.DBAR_MIXED)
    assert len(info) == 64 and all(i.status == 0 and i.rel_residual <= w.tol for i in info)
    golds = {j: golden(f"c4_k{j}") for j in C4_GOLDEN}
    golds = {j: gd for j, gd in golds.items() if gd is not None}
    assert 0 in golds and 3 in golds
    for j, gd in golds.items():
        assert np.allclose(gd["k"], [w.ks[j].real, w.ks[j].imag], rtol=0, atol=1e-15)
        eS, em = golden_err(S[j].cpu().numpy(), gd, "S"), golden_err(m[j].cpu().numpy(), gd, "m")
        print(f"N=4096 k[{j}]={w.ks[j]:.3f}: mixed err S {eS:.2e} m {em:.2e}, err_estimate {info[j].err_estimate:.1e}",
              flush=True)
        assert eS < 1e-10 and em < 1e-10, j
        assert abs(info[j].m1 - complex(*gd["m1"])) < 1e-10 * gd["max_abs_S"], j
    del S, m
    sel = sorted(golds)
    S64, m64, info64 = D.solve_device(Qd, w.ks[sel], w.L, tol=w.tol, precision=D.DBAR_FP64)
    for i, j in enumerate(sel):
        assert info64[i].status == 0
        eS, em = golden_err(S64[i].cpu().numpy(), golds[j], "S"), golden_err(m64[i].cpu().numpy(), golds[j], "m")
        print(f"N=4096 k[{j}]: FP64 err S {eS:.2e} m {em:.2e}", flush=True)
        assert eS < 1e-10 and em < 1e-10, j


def test_mixed_n4096_residual_by_oracle_operator():
    w = W.workload("mixed_n4096")
    Qd = torch.from_numpy(w.Q).to("cuda:0")
    S, _, info = D.solve_device(Qd, w.ks, w.L, tol=w.tol, precision=D.DBAR_MIXED, want_m=False)
    assert len(info) == 64 and all(i.status == 0 and i.rel_residual <= w.tol for i in info)
    j = 5
    print(f"oracle operator N=4096 k={w.ks[j]}", flush=True)
    g = O.make_grid(w.N, w.L)
    om = O.omega_table(g, w.M)
    Sj = S[j].cpu().numpy()
    del S
    b = O.rhs(g, w.Q, w.ks[j])
    r = b - O.apply_A(g, w.Q, w.ks[j], Sj, w.M, om)
    assert np.linalg.norm(r) / np.linalg.norm(b) < 1e-11


@pytest.mark.parametrize("method", [D.DBAR_METHOD_PLAIN, D.DBAR_METHOD_ITERATED])
def test_n2048_residual_and_m_by_oracle(method):
    """N = 2048 (two waves per row line, one row per tile: the largest grid whose oracle operator runs in seconds
    besides N = 4096): a batch of 8 mixed solves, S and m of one k against the stored oracle solution (and the FP64
    path's at that k), the oracle's FP64 operator applied to the GPU's S, and m against the oracle's h(S) (iterated
    method: its equation for h and its m)."""
    N, L = 2048, 6.0
    Q = W.potential_gaussian_sum(N, L, seed=91, amp_max=1.5)
    ks = [(m1 + 1j * m2) / (2 * L) for m1, m2 in ((0, 0), (5, -3), (-8, 2), (12, 7), (-3, -11), (9, 9), (1, 4),
                                                   (-6, 6))]
    Qd = torch.from_numpy(Q).to("cuda:0")
    S, m, info = D.solve_device(Qd, ks, L, tol=1e-12, precision=D.DBAR_MIXED, method=method)
    assert all(i.status == 0 and i.rel_residual <= 1e-12 for i in info)
    j = 3
    gd = golden("n2048_k3" if method == D.DBAR_METHOD_PLAIN else "n2048_it_k3")
    assert gd is not None and np.allclose(gd["k"], [ks[j].real, ks[j].imag], rtol=0, atol=1e-15)
    eS, em = golden_err(S[j].cpu().numpy(), gd, "S"), golden_err(m[j].cpu().numpy(), gd, "m")
    print(f"N=2048 method={method}: err S {eS:.2e} m {em:.2e} vs stored oracle solution", flush=True)
    assert eS < 1e-10 and em < 1e-10
    S64, m64, info64 = D.solve_device(Qd, [ks[j]], L, tol=1e-12, precision=D.DBAR_FP64, method=method)
    assert info64[0].status == 0 and info64[0].rel_residual <= 1e-12
    eS, em = golden_err(S64[0].cpu().numpy(), gd, "S"), golden_err(m64[0].cpu().numpy(), gd, "m")
    print(f"N=2048 method={method}: FP64 err S {eS:.2e} m {em:.2e} vs stored oracle solution", flush=True)
    assert eS < 1e-10 and em < 1e-10
    del S64, m64
    print(f"oracle operator N=2048 k={ks[j]} method={method}", flush=True)
    g = O.make_grid(N, L)
    om = O.omega_table(g, 11)
    Sj, mj = S[j].cpu().numpy(), m[j].cpu().numpy()
    del S, m
    if method == D.DBAR_METHOD_PLAIN:
        b = O.rhs(g, Q, ks[j])
        r = b - O.apply_A(g, Q, ks[j], Sj, 11, om)
        assert np.linalg.norm(r) / np.linalg.norm(b) < 1e-11
        h, _, _ = O.regularised_h(g, Sj, 11, om)
        assert relerr(mj, h) < 1e-12
    else:
        # S solves the plain equation too (Sform): its residual under the plain operator is small
        b = O.rhs(g, Q, ks[j])
        r = b - O.apply_A(g, Q, ks[j], Sj, 11, om)
        assert np.linalg.norm(r) / np.linalg.norm(b) < 1e-10
