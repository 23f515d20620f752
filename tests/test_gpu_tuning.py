"""The column-tile tuner: every tile width computes the same operator and the same solves (only the order of the
moment partial sums changes), and the tuner's choice is one of the valid widths."""
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


@pytest.mark.parametrize("N", [64, 256, 1024, 4096])
def test_tile_variants_agree(N):
    """Every column-tile width (the default, the wider ones, the half-width one) gives the oracle's operator in FP64
    and FP32, and the same mixed solves."""
    L = max(1.0, N / 32.0) if N < 1024 else (5.0 if N == 1024 else 8.0)
    print(f"tile variants N={N}", flush=True)
    g = O.make_grid(N, L)
    rng = np.random.default_rng(N)
    Q = W.potential_gaussian_sum(N, L, seed=N)
    S = O.Fd(g, np.exp(-np.abs(g.z) ** 2 / 3) * (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))))
    k = 0.5 - 0.25j
    ref = O.apply_A(g, Q, k, S)
    try:
        for prec, tol in ((D.DBAR_FP64, 1e-12), (D.DBAR_FP32, 2e-5)):
            nv = D.get_tile(N, prec)[2]
            assert nv >= 1
            for v in range(nv):
                D.set_tile(N, prec, v)
                assert D.get_tile(N, prec)[0] == v
                assert relerr(D.apply(Q, k, S, L, precision=prec), ref) < tol, (prec, v)
        ks = W.k_disk(4 if N < 4096 else 2, 1.5, seed=N)
        base = None
        for v in range(D.get_tile(N, D.DBAR_FP32)[2]):
            D.set_tile(N, D.DBAR_FP32, v)
            D.set_tile(N, D.DBAR_FP64, min(v, D.get_tile(N, D.DBAR_FP64)[2] - 1))
            Sv, mv, info = D.solve(Q, ks, L, tol=1e-12, batch=len(ks), precision=D.DBAR_MIXED, want_m=N < 4096)
            assert all(i.status == 0 for i in info)
            if base is None:
                base = Sv
            else:
                for j in range(len(ks)):
                    assert relerr(Sv[j], base[j]) < 1e-11, (v, j)
    finally:
        D.set_tile(N, D.DBAR_FP64, 0)
        D.set_tile(N, D.DBAR_FP32, 0)


def test_autotune_reports_and_keeps_a_valid_choice():
    N, L = 512, 5.0
    try:
        r = D.autotune(N, L, precision=D.DBAR_MIXED, batch=16)
        for name, prec in (("fp64", D.DBAR_FP64), ("fp32", D.DBAR_FP32)):
            t = r[name]
            assert len(t["ms"]) == D.get_tile(N, prec)[2] and all(ms > 0 for ms in t["ms"])
            best = int(np.argmin(t["ms"]))
            assert D.get_tile(N, prec)[1] == t["columns"][best] == t["chosen_columns"]
        assert r["batch"] in r["batch_candidates"]
    finally:
        D.set_tile(N, D.DBAR_FP64, 0)
        D.set_tile(N, D.DBAR_FP32, 0)


def test_set_tile_rejects_invalid_variants():
    with pytest.raises(D.DbarError):
        D.set_tile(1024, D.DBAR_FP32, 7)
    with pytest.raises(D.DbarError):
        D.set_tile(100, D.DBAR_FP64, 0)


def test_library_batch_in_two_lanes_gives_the_same_results():
    """With the library's own batch size (batch = 0: here the tuner's choice, at most 2 entries per launch) and more k
    than one batch, each of two lanes takes that many entries per launch (the default rule); every result equals the
    one-lane solve's bit for bit."""
    N, L = 32, 3.0
    try:
        t = D.autotune(N, L, precision=D.DBAR_MIXED, batch=2)
        assert t["batch"] in (1, 2)
        g = O.make_grid(N, L)
        Q = (0.5 - 0.4j) * np.exp(-np.abs(g.z) ** 2)
        ks = np.linspace(-1.5, 1.5, 7) + 0.3j
        print(f"library batch {t['batch']}, 7 k, one lane then the default", flush=True)
        S1, m1, i1 = D.solve(Q, ks, L, tol=1e-12, precision=D.DBAR_MIXED, lanes=1)
        S2, m2, i2 = D.solve(Q, ks, L, tol=1e-12, precision=D.DBAR_MIXED)
        for j in range(len(ks)):
            assert i1[j].status == 0 and (i1[j].iters, i1[j].outer) == (i2[j].iters, i2[j].outer), j
            assert i1[j].rel_residual == i2[j].rel_residual and i1[j].m1 == i2[j].m1, j
        assert np.array_equal(S1, S2) and np.array_equal(m1, m2)
        ref = O.solve(g, Q, ks[3], tol=1e-13)
        assert relerr(S2[3], ref.S) < 1e-10 and relerr(m2[3], ref.m) < 1e-10
    finally:
        D.set_tile(N, D.DBAR_FP64, 0)
        D.set_tile(N, D.DBAR_FP32, 0)
