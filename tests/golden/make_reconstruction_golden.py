"""Write reconstruction_n64.json: the oracle's DS II round trip q0 -> r -> q for the N = 64 row of the Section 6.2
reconstruction table (q0 = e^{-x^2-y^2}, L = 2.1213, M = 11; the paper reports an L-infinity error of 1.736e-9).

Calls only the oracle.  Stores the oracle's error, r at sampled k and q at sampled z, for GPU parity at a size the
oracle cannot redo inside a test (8192 iterated solves).  Run from the repository root:
    python tests/golden/make_reconstruction_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import dbar_oracle as O  # noqa: E402

N, L, M, TOL = 64, 2.1213, 11, 1e-13


def main():
    g = O.make_grid(N, L)
    q0 = np.exp(-np.abs(g.z) ** 2)
    r = O.reflection_grid(g, q0, tol=TOL, M=M)
    q = O.reconstruct_potential(g, r, tol=TOL, M=M)
    rng = np.random.default_rng(64)
    idx = [(0, 0), (N // 2, N // 2), (N - 1, N - 1), (N // 2, 0), (0, N // 2)]
    idx += [tuple(int(v) for v in rng.integers(0, N, 2)) for _ in range(19)]
    out = {
        "source": "Section 6.2, reconstruction table, row N = 2^6 (L = 2.1213, M = 11, q0 = exp(-x^2-y^2))",
        "paper_error": 1.736e-9,
        "N": N, "L": L, "M": M, "tol": TOL,
        "oracle_error": float(np.max(np.abs(q - q0))),
        "samples": [{"p2": a, "p1": b, "r": [r[a, b].real, r[a, b].imag], "q": [q[a, b].real, q[a, b].imag]}
                    for a, b in idx],
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "reconstruction_n64.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("oracle error", out["oracle_error"])


if __name__ == "__main__":
    main()
