"""The 32^3 workload (N = 32768, leaf 64, eta 1, eps 1e-4), in the configuration
the benchmark times, against the CPU oracle element by element.

tests/golden/cube32_oracle.npz was written by tests/golden/make_cube32_fixture.py,
which calls only the oracle and the seeded input generators: the oracle's rank
decisions with their margins, x = M^-1 b for b = exp(-j k z) (Algs. 5-6), the
adjoint lam = M^-H g (seeded g) and the solution refined to 1e-12 against the
H^2 matrix.  With the ranks pinned to the oracle's, the GPU's factors are the
same approximation: x and lam must agree to 1e-10 relative (norm-wise) and
to 5e-10 of their largest entry entry-wise; without pinning, ranks must agree
except where a singular value lies within 1e-3 relative of its threshold."""
import os

import numpy as np
import pytest

import paper_1703_06155_amd as h2
from paper_1703_06155_amd import inputs as I

pytestmark = pytest.mark.gpu

FIXTURE = os.path.join(os.path.dirname(__file__), "golden", "cube32_oracle.npz")


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _fixture():
    d = np.load(FIXTURE, allow_pickle=False)
    rk = {(int(r[0]), int(r[1])): (int(r[2]), r[3], r[4]) for r in d["ranks_k"]}
    rkt = {(int(r[0]), int(r[1])): (int(r[2]), r[3], r[4]) for r in d["ranks_kt"]}
    return d, rk, rkt


def _maxrel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _in_band(lo, hi):
    return abs(lo - 1) < 1e-3 or abs(hi - 1) < 1e-3


def test_cube32_pinned_ranks_elementwise_against_oracle():
    torch = _torch()
    d, rk, rkt = _fixture()
    pr = I.config(1)
    keys = sorted(rk, key=lambda lt: (-lt[0], lt[1]))
    forced = np.array([(l, t, rk[(l, t)][0], rkt[(l, t)][0] if (l, t) in rkt else -1) for l, t in keys],
                      dtype=np.int32)
    G = h2.H2(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps, forced_ranks=forced).factor()
    try:
        got = {(int(l), int(t)): (int(k), int(kt)) for l, t, k, kt in G.forced_ranks()}
        assert all(got[key] == (rk[key][0], rkt[key][0]) for key in rkt)
        b = torch.from_numpy(pr.rhs[:, 0].copy()).cuda()
        x = G.solve(b).cpu().numpy()
        ex = _maxrel(x, d["x"])
        g = np.random.default_rng(9)
        g = g.standard_normal(pr.n) + 1j * g.standard_normal(pr.n)
        lam = G.solve_adjoint(torch.from_numpy(g).cuda()).cpu().numpy()
        el = _maxrel(lam, d["lam"])
        xr = G.solve(b, tol=1e-12, max_iter=20).cpu().numpy()
        er = _maxrel(xr, d["x_refined"])
        nx = float(np.linalg.norm(x - d["x"]) / np.linalg.norm(d["x"]))
        nl = float(np.linalg.norm(lam - d["lam"]) / np.linalg.norm(d["lam"]))
        print(f"32^3 vs oracle, ranks pinned: x {ex:.2e} (norm-wise {nx:.2e}), lam {el:.2e} (norm-wise {nl:.2e}), "
              f"refined x {er:.2e}")
        # the 1e-10 relative bar, norm-wise; entry-wise the largest deviation over the largest
        # entry sits at 1e-10 .. 3e-10: the GPU's bases (Gram eigenvectors, rotated twice) and
        # the oracle's (SVD) differ at rounding level in the directions next to the
        # truncation threshold (5 % gaps at eps = 1e-4), and those differences reach the
        # solution unevenly
        assert nx < 1e-10 and nl < 1e-10
        assert ex < 5e-10 and el < 5e-10
        assert er < 1e-8
    finally:
        G.close()


def test_cube32_free_ranks_against_oracle():
    _torch()
    d, rk, rkt = _fixture()
    pr = I.config(1)
    G = h2.H2(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps).factor()
    try:
        got = {(int(l), int(t)): (int(k), int(kt)) for l, t, k, kt in G.forced_ranks()}
    finally:
        G.close()
    bad = []
    same_k = 0
    for key, (k, lo, hi) in rk.items():
        if got[key][0] != k:
            if not _in_band(lo, hi):
                bad.append(("k", key, got[key][0], k, lo, hi))
            continue
        same_k += 1
        if key in rkt:
            kt, flo, fhi = rkt[key]
            if got[key][1] != kt and not _in_band(flo, fhi):
                bad.append(("kt", key, got[key][1], kt, flo, fhi))
    assert not bad, bad[:5]
    assert same_k >= len(rk) - 8


def test_cube32_mixed_form_against_oracle():
    """The mixed form on the 32^3 workload, ranks pinned to the oracle's: part of the
    Schur flops go through the FP32 branch (the ledger's routed fraction is above 0),
    the unrefined solve differs from the FP64 oracle's M^-1 b by that branch's
    rounding only, and refinement against the FP64 H^2 matrix reaches the oracle's
    refined solution."""
    torch = _torch()
    d, rk, rkt = _fixture()
    pr = I.config(1)
    keys = sorted(rk, key=lambda lt: (-lt[0], lt[1]))
    forced = np.array([(l, t, rk[(l, t)][0], rkt[(l, t)][0] if (l, t) in rkt else -1) for l, t in keys],
                      dtype=np.int32)
    G = h2.H2(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps, forced_ranks=forced,
              precision="mixed").factor()
    try:
        frac = G.kernel_ledger()["schur_fp32_flop_frac"]
        b = torch.from_numpy(pr.rhs[:, 0].copy()).cuda()
        x = G.solve(b).cpu().numpy()
        nx = float(np.linalg.norm(x - d["x"]) / np.linalg.norm(d["x"]))
        xr, info = G.solve(b, tol=1e-12, max_iter=30, info=True)
        er = _maxrel(xr.cpu().numpy(), d["x_refined"])
        print(f"32^3 mixed vs oracle: FP32 fraction of Schur flops {frac:.3f}, unrefined x {nx:.2e} norm-wise, "
              f"refined x {er:.2e} after {info['iterations']} iterations")
        assert frac > 0.1
        assert nx < 1e-4
        assert info["rel_residual"] <= 1e-12 and er < 1e-8
    finally:
        G.close()
