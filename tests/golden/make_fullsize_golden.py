"""Write fullsize_<case>.json: oracle solutions at grid sizes where an oracle solve takes minutes, for element-by-element
GPU parity at those sizes (Section 4 algorithm with Q -> q_k of Section 5.1, GMRES tolerance of Section 4.1; the
iterated case follows Section 5.3).

Calls only the oracle (and the seeded input generators).  Each case is one oracle solve to a true relative residual
of 1e-13; the file keeps the oracle's S and m at sampled grid points (half uniform over the grid, half where the
array is at least 1e-6 of its maximum, plus the origin of S), their maxima, m^(1), the iteration count and the
oracle's residual.  Run from the repository root, one case per process (they are independent):

    python tests/golden/make_fullsize_golden.py c4_k0        # N = 4096, |k| = 7.77   (about an hour on one core)
    python tests/golden/make_fullsize_golden.py c4_k3        # N = 4096, |k| = 2.28
    python tests/golden/make_fullsize_golden.py n2048_k3     # N = 2048, plain method
    python tests/golden/make_fullsize_golden.py n2048_it_k3  # N = 2048, iterated method
    python tests/golden/make_fullsize_golden.py c5_r14       # N = 2048 request of the seeded request stream
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import dbar_workloads as W  # noqa: E402
from oracle import dbar_oracle as O  # noqa: E402

TOL = 1e-13
N_UNIFORM = 512     # sampled points per array, uniform over the grid
N_SIGNIF = 512      # sampled points per array where |value| >= 1e-6 max|value|


def n2048_case():
    """The N = 2048 workload of the full-size GPU tests: L = 6, seeded Gaussian sum (seed 91, |A_j| <= 1.5), k with
    2kL integer so that the iterated method applies too."""
    N, L = 2048, 6.0
    Q = W.potential_gaussian_sum(N, L, seed=91, amp_max=1.5)
    k = (12 + 7j) / (2 * L)
    return N, L, Q, k, "N=2048, L=6, Gaussian sum seed 91 (|A_j| <= 1.5), k = (12+7i)/12"


def case(name: str):
    if name.startswith("c4_k"):
        j = int(name[4:])
        w = W.workload("mixed_n4096")
        return dict(N=w.N, L=w.L, Q=w.Q, k=complex(w.ks[j]), method="plain", k_index=j,
                    workload=f"mixed_n4096: N=4096, L=8, Q=(1.2-0.4i)sech^2(r), k index {j} of 64 uniform in |k|<=8 "
                             f"(seed 4)")
    if name in ("n2048_k3", "n2048_it_k3"):
        N, L, Q, k, desc = n2048_case()
        return dict(N=N, L=L, Q=Q, k=k, method="iterated" if "_it_" in name else "plain", k_index=3, workload=desc)
    if name.startswith("c5_r"):
        j = int(name[4:])
        r = W.serving_stream(j + 1, rate=1.0, seed=5)[j]
        return dict(N=r.N, L=r.L, Q=r.Q, k=complex(r.k), method="plain", k_index=j,
                    workload=f"request {j} of the seeded request stream (seed 5): N={r.N}, L={r.L}, {r.family} "
                             f"potential, k={r.k:.6f}")
    raise KeyError(name)


def sample(rng, a: np.ndarray) -> np.ndarray:
    flat = np.abs(a).ravel()
    uni = rng.choice(flat.size, N_UNIFORM, replace=False)
    big = np.flatnonzero(flat >= 1e-6 * flat.max())
    sig = rng.choice(big, min(N_SIGNIF, big.size), replace=False)
    return np.unique(np.concatenate([[0], uni, sig]))


def main(name: str):
    c = case(name)
    N, L, Q, k = c["N"], c["L"], c["Q"], c["k"]
    g = O.make_grid(N, L)
    t0 = time.time()
    om = O.omega_table(g, 11)
    print(f"{name}: omega tables {time.time() - t0:.0f} s", flush=True)
    calls = [0]
    inner = O.apply_A if c["method"] == "plain" else O.apply_B
    attr = "apply_A" if c["method"] == "plain" else "apply_B"

    def counted(*a, **kw):  # progress only: the oracle's own operator, unchanged
        calls[0] += 1
        t = time.time()
        out = inner(*a, **kw)
        print(f"{name}: operator application {calls[0]} ({time.time() - t:.1f} s)", flush=True)
        return out

    setattr(O, attr, counted)
    t0 = time.time()
    solver = O.solve if c["method"] == "plain" else O.solve_iterated
    res = solver(g, Q, k, tol=TOL, M=11, restart=20, om=om)
    dt = time.time() - t0
    setattr(O, attr, inner)
    print(f"{name}: {res.iters} iterations, residual {res.rel_residual:.2e}, {dt:.0f} s", flush=True)
    rng = np.random.default_rng(20000 + N + 97 * c["k_index"])
    iS, im = sample(rng, res.S), sample(rng, res.m)
    Sf, mf = res.S.ravel(), res.m.ravel()
    out = {
        "source": "oracle solve (Section 4 algorithm, Q -> q_k of Section 5.1" +
                  ("; iterated equation of Section 5.3" if c["method"] == "iterated" else "") +
                  f"), GMRES to a true relative residual of {TOL:g}",
        "workload": c["workload"], "N": N, "L": L, "M": 11, "k": [k.real, k.imag], "method": c["method"],
        "oracle_iters": int(res.iters), "oracle_rel_residual": float(res.rel_residual), "oracle_seconds": dt,
        "max_abs_S": float(np.max(np.abs(res.S))), "max_abs_m": float(np.max(np.abs(res.m))),
        "m1": [res.m1.real, res.m1.imag],
        "S_idx": iS.tolist(), "S": [[float(v.real), float(v.imag)] for v in Sf[iS]],
        "m_idx": im.tolist(), "m": [[float(v.real), float(v.imag)] for v in mf[im]],
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"fullsize_{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print(f"{name}: wrote {path}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1])
