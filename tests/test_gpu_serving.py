"""GPU tests of the serving session (continuous batching): every result equals the same request solved alone, within
the mixed-precision tolerance, and matches the oracle; the session's bookkeeping is consistent.

Tolerance: requests ask for ||b - A S|| <= 1e-10 ||b|| (FP64 residual after FP32 inner solves).  The discrete system
has condition numbers below 50 (dense LU pins), so two such solves agree to about 1e-9; the test uses 1e-8 against
the oracle and 1e-9 between alone and mixed runs."""
import time

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


def _requests(n, seed=11):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        N = int(rng.choice([32, 64]))
        L = 3.0
        k = complex(2.0 * np.sqrt(rng.random()) * np.exp(2j * np.pi * rng.random()))
        if i % 2:
            Q = W.potential_gaussian_sum(N, L, seed=int(rng.integers(1 << 30)), amp_max=1.0)
        else:
            Q = W.potential_sech2(N, L, complex(np.exp(2j * np.pi * rng.random())))
        out.append((Q, k, L, N))
    return out


def test_alone_equals_mixed_and_oracle():
    reqs = _requests(24)
    # all at once: the two grid sizes run concurrently and requests join as slots free up (max_slots=8)
    with D.Session(max_slots=8) as s:
        tickets = [s.submit(Q, k, L, tol=1e-10) for (Q, k, L, N) in reqs]
        mixed = [s.wait(t) for t in tickets]
        st = s.stats()
    assert st["submitted"] == 24 and st["completed"] == 24 and st["in_flight"] == 0 and st["queued"] == 0
    # one at a time
    alone = []
    with D.Session(max_slots=8) as s:
        for (Q, k, L, N) in reqs:
            alone.append(s.wait(s.submit(Q, k, L, tol=1e-10)))
    bitwise = 0
    for j, ((Q, k, L, N), a, m) in enumerate(zip(reqs, alone, mixed)):
        assert a[2].status == 0 and m[2].status == 0
        assert a[2].rel_residual <= 1e-10 and m[2].rel_residual <= 1e-10
        assert relerr(m[0], a[0]) <= 1e-9, j
        assert relerr(m[1], a[1]) <= 1e-9, j
        bitwise += int(np.array_equal(m[0], a[0]))
        if j < 4:
            g = O.make_grid(N, L)
            ref = O.solve(g, Q, k, tol=1e-13)
            assert relerr(m[0], ref.S) <= 1e-8 and relerr(m[1], ref.m) <= 1e-8, j
    print(f"bitwise identical alone/mixed: {bitwise}/{len(reqs)}")


def test_poll_and_latency():
    Q, k, L, N = _requests(1, seed=3)[0]
    with D.Session() as s:
        t = s.submit(Q, k, L, tol=1e-10)
        res = None
        t0 = time.time()
        while res is None and time.time() - t0 < 60:
            res = s.poll(t)
            time.sleep(0.001)
        assert res is not None
        S, m, info, lat = res
        assert info.status == 0 and 0 < lat < 60
        with pytest.raises(D.DbarError):
            s.poll(t)  # fetched once: now unknown


def test_zero_potential_request():
    with D.Session() as s:
        S, m, info, lat = s.wait(s.submit(np.zeros((32, 32)), 1 + 1j, 3.0))
        assert np.all(S == 0) and np.all(m == 0) and info.status == 0
