"""Write tests/golden/cube32_oracle.npz: the CPU oracle on the 32^3 cube-grid
workload (N = 32768, leaf 64, eta 1, eps 1e-4, contrast seed 0).

Calls only the oracle and the seeded input generators.  Stored:
  ranks_k   (level, cluster, k, margin_lo, margin_hi) construction ranks and the
            ratios sigma_k / thr, sigma_{k+1} / thr of each decision;
  ranks_kt  (level, cluster, k~, margin_lo, margin_hi) Step 0 ranks and their
            ratios sigma_p / tau, sigma_{p+1} / tau;
  x         M^-1 b for b = exp(-j k z) (one forward and backward sweep, Algs. 5-6);
  lam       M^-H g for g seeded from numpy's PCG64 (seed 9), the adjoint of eq. 35;
  x_refined b refined to 1e-12 against the H^2 matrix.

Run from the repository root:  python tests/golden/make_cube32_fixture.py
(about 10-20 minutes and 20 GB of host memory on 8 cores).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import h2_oracle as O  # noqa: E402
from paper_1703_06155_amd import inputs as I  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "cube32_oracle.npz")


def adjoint_rhs(n: int) -> np.ndarray:
    rng = np.random.default_rng(9)
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def main() -> None:
    pr = I.config(1)
    t0 = time.perf_counter()
    H = O.construct(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps)
    print(f"construct {time.perf_counter() - t0:.1f} s", flush=True)
    t0 = time.perf_counter()
    Fz = O.factor(H)
    print(f"factor {time.perf_counter() - t0:.1f} s", flush=True)
    b = pr.rhs[:, 0]
    x = O.solve(Fz, b)
    lam = O.solve_adjoint(Fz, adjoint_rhs(pr.n))
    xr, hist = O.refine(Fz, b, tol=1e-12, max_iter=20)
    print(f"solves done, refinement history {hist}", flush=True)
    rk = []
    for (l, t), k in sorted(O.forced_construction(H).items(), key=lambda e: (-e[0][0], e[0][1])):
        m = H.sig_margin[l][t]
        rk.append((l, t, k, m[0], m[1]))
    rkt = [(l, i, kt, m[0], m[1]) for (l, i, n, k, kt, m) in Fz.stats]
    np.savez_compressed(OUT, ranks_k=np.array(rk, dtype=np.float64), ranks_kt=np.array(rkt, dtype=np.float64),
                        x=x, lam=lam, x_refined=xr, refine_history=np.array(hist),
                        n=pr.n, final_n=Fz.final_n)
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
