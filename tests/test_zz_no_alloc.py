"""GPU test of the allocation-free operator entry point (dbar_apply_noalloc): its result equals dbar_apply's (the
entry point it is a variant of) within the operator's parity bar -- FP64 1e-12 and FP32 2e-5 relative to the largest
magnitude -- on two calls in a row, the second on a smaller grid, and the FP64 result equals the oracle's operator;
captured into a HIP graph, every replay equals the eager call."""
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


def smooth_xi(g, rng):
    base = rng.standard_normal((g.N, g.N)) + 1j * rng.standard_normal((g.N, g.N))
    return O.Fd(g, np.exp(-np.abs(g.z) ** 2 / 3.0) * O.Fd_inv(g, base * np.exp(-np.abs(g.xi) ** 2 / 8)))


@pytest.mark.parametrize("prec,tol", [(D.DBAR_FP64, 1e-12), (D.DBAR_FP32, 2e-5)])
def test_noalloc_apply_equals_apply_on_two_calls(prec, tol):
    dev = torch.device("cuda:0")
    for N, L, k in ((1024, 5.0, -0.6 + 1.4j), (256, 4.0, 1.0 + 0.5j)):  # the maximum size, then a smaller grid
        print(f"noalloc apply N={N} precision={prec}", flush=True)
        rng = np.random.default_rng(N + prec)
        g = O.make_grid(N, L)
        Q = W.potential_gaussian_sum(N, L, seed=N)
        S = smooth_xi(g, rng)
        ref = D.apply(Q, k, S, L, precision=prec)
        Qd, Sd = torch.from_numpy(Q).to(dev), torch.from_numpy(S).to(dev)
        out = torch.full_like(Sd, float("nan"))
        D.apply_noalloc(Qd, k, Sd, out, L, precision=prec)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.all(np.isfinite(got))
        assert relerr(got, ref) < tol, N
        if prec == D.DBAR_FP64 and N <= 256:
            assert relerr(got, O.apply_A(g, Q, k, S)) < 1e-12


@pytest.mark.parametrize("prec", [D.DBAR_FP64, D.DBAR_FP32])
def test_noalloc_apply_replays_in_a_captured_graph(prec):
    """Captured into a HIP graph (code under graph capture is among the callers it is for) and replayed three times,
    with eager calls on another grid between the replays (they leave other contents in the shared scratch array):
    every replay writes the eager call's result, bit for bit."""
    dev = torch.device("cuda:0")
    N, L, k = 128, 4.0, 0.8 - 0.3j
    rng = np.random.default_rng(7 + prec)
    g = O.make_grid(N, L)
    Qd = torch.from_numpy(W.potential_gaussian_sum(N, L, seed=3)).to(dev)
    Sd = torch.from_numpy(smooth_xi(g, rng)).to(dev)
    ref = torch.full_like(Sd, float("nan"))
    out = torch.full_like(Sd, float("nan"))
    print(f"noalloc apply eager N={N} precision={prec}", flush=True)
    D.apply_noalloc(Qd, k, Sd, ref, L, precision=prec)
    torch.cuda.synchronize()
    ref_h = ref.cpu().numpy()
    assert np.all(np.isfinite(ref_h))
    N2, L2 = 64, 3.0
    g2 = O.make_grid(N2, L2)
    Q2 = torch.from_numpy(W.potential_gaussian_sum(N2, L2, seed=4)).to(dev)
    S2 = torch.from_numpy(smooth_xi(g2, rng)).to(dev)
    o2 = torch.empty_like(S2)
    print("capture", flush=True)
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(graph, stream=side):
        D.apply_noalloc(Qd, k, Sd, out, L, precision=prec)
    torch.cuda.synchronize()
    for r in range(3):
        D.apply_noalloc(Q2, 1.1j, S2, o2, L2, precision=prec)  # eager work on the shared scratch between replays
        out.fill_(float("nan"))
        torch.cuda.synchronize()
        print(f"replay {r}", flush=True)
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref_h), r
