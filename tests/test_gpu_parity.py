"""HIP path vs the CPU oracle through the C ABI (needs an MI355X)."""
import numpy as np
import pytest

import paper_1703_06155_amd as h2
from oracle import h2_oracle as O
from paper_1703_06155_amd import inputs as I

pytestmark = pytest.mark.gpu

# small problems the oracle finishes in seconds; several tiles, ragged leaves, multiple levels; the last
# two have clusters of about 108 and 144 unknowns (the wide-cluster paths of Step 0 and of the partial LU)
CASES = [((8, 8, 8), 16, 1e-4), ((10, 7, 9), 12, 1e-5), ((6, 6, 6), 8, 1e-6), ((9, 5, 3), 7, 1e-3),
         ((12, 12, 12), 27, 1e-4), ((12, 12, 24), 27, 1e-4), ((12, 12, 12), 110, 1e-4), ((16, 12, 12), 150, 1e-4)]
IDS = ["8^3_leaf16", "10x7x9_leaf12", "6^3_leaf8", "9x5x3_leaf7", "12^3_leaf27", "12x12x24_leaf27", "12^3_leaf110",
       "16x12x12_leaf150"]


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


_cache = {}


def _oracle(grid, leaf, eps, eta=1.0):
    key = (grid, leaf, eps, eta)
    if key not in _cache:
        pr = I.make_problem("t", grid, leaf, eps, eta=eta)
        H = O.construct(pr.points, pr.k, pr.h, pr.chi, leaf, eta, eps)
        Fz = O.factor(H)
        _cache[key] = (pr, H, Fz)
    return _cache[key]


def _forced(H, Fz):
    return h2.forced_ranks_from_oracle(O.forced_construction(H), O.forced_from(Fz))


def _gpu(pr, H, Fz, forced=True, **kw):
    fr = _forced(H, Fz) if forced else None
    return h2.H2(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps, forced_ranks=fr, **kw)


def _rel(a, b):
    """Largest entry-wise difference relative to the largest entry of the reference."""
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("grid,leaf,eps", CASES, ids=IDS)
def test_matvec_matches_oracle(grid, leaf, eps):
    torch = _torch()
    pr, H, Fz = _oracle(grid, leaf, eps)
    G = _gpu(pr, H, Fz)
    rng = np.random.default_rng(7)
    x = rng.standard_normal((pr.n, 2)) + 1j * rng.standard_normal((pr.n, 2))
    y = G.matvec(torch.from_numpy(x)).cpu().numpy()
    yo = O.h2_matvec(H, x)
    assert _rel(y, yo) < 1e-11
    ya = G.matvec(torch.from_numpy(x), adjoint=True).cpu().numpy()
    assert _rel(ya, O.h2_matvec(H, x, adjoint=True)) < 1e-11


@pytest.mark.parametrize("grid,leaf,eps", CASES, ids=IDS)
def test_solution_matches_oracle_fp64(grid, leaf, eps):
    """FP64 form with the oracle's rank decisions: solution within 1e-10 relative."""
    torch = _torch()
    pr, H, Fz = _oracle(grid, leaf, eps)
    G = _gpu(pr, H, Fz).factor()
    b = pr.rhs[:, 0]
    x = G.solve(torch.from_numpy(b)).cpu().numpy()
    xo = O.solve(Fz, b)
    assert _rel(x, xo) < 1e-10
    fr = G.forced_ranks()
    assert np.array_equal(fr, _forced(H, Fz))


@pytest.mark.parametrize("grid,leaf,eps", CASES[:3], ids=IDS[:3])
def test_adjoint_matches_oracle(grid, leaf, eps):
    torch = _torch()
    pr, H, Fz = _oracle(grid, leaf, eps)
    G = _gpu(pr, H, Fz).factor()
    rng = np.random.default_rng(11)
    g = rng.standard_normal(pr.n) + 1j * rng.standard_normal(pr.n)
    lam = G.solve_adjoint(torch.from_numpy(g)).cpu().numpy()
    assert _rel(lam, O.solve_adjoint(Fz, g)) < 1e-10
    b = pr.rhs[:, 0]
    x = G.solve(torch.from_numpy(b)).cpu().numpy()
    # <M^-1 b, g> = <b, M^-H g> for the computed operator itself
    assert abs(np.vdot(g, x) - np.vdot(lam, b)) <= 1e-12 * abs(np.vdot(g, x))


def test_multi_rhs_equals_columns():
    torch = _torch()
    pr, H, Fz = _oracle(*CASES[1])
    G = _gpu(pr, H, Fz).factor()
    B = I.plane_waves(pr.points, I.directions(5, 3))
    X = G.solve(torch.from_numpy(B)).cpu().numpy()
    for j in range(5):
        xj = G.solve(torch.from_numpy(B[:, j].copy())).cpu().numpy()
        assert _rel(X[:, j], xj) < 1e-14
    assert _rel(X, O.solve(Fz, B)) < 1e-10


def test_eta_zero_is_dense_lu():
    torch = _torch()
    pr = I.make_problem("t", (8, 8, 8), 16, 1e-4, eta=0.0)
    G = h2.H2(pr.points, pr.k, pr.h, pr.chi, 16, 0.0, 1e-4).factor()
    b = pr.rhs[:, 0]
    x = G.solve(torch.from_numpy(b)).cpu().numpy()
    A = O.dense_A(pr.points, pr.k, pr.h, pr.chi)
    assert _rel(x, np.linalg.solve(A, b)) < 1e-12


def test_refinement_reaches_1e_8_against_h2_matrix():
    torch = _torch()
    pr, H, Fz = _oracle(*CASES[0])
    G = h2.H2(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps, eps_fill=1e-2).factor()
    b = pr.rhs[:, 0]
    x, info = G.solve(torch.from_numpy(b), tol=1e-10, max_iter=30, info=True)
    x = x.cpu().numpy()
    assert info["rel_residual"] <= 1e-10 and info["rel_residual_first"] > 1e-8
    ro = np.linalg.norm(O.h2_matvec(H, x) - b) / np.linalg.norm(b)
    assert ro < 1e-9


@pytest.mark.parametrize("grid,leaf,eps", CASES, ids=IDS)
def test_free_ranks_match_oracle_outside_band(grid, leaf, eps):
    """Without pinning, construction and factor ranks equal the oracle's unless a singular
    value lies within 1e-3 relative of its threshold."""
    _torch()
    pr, H, Fz = _oracle(grid, leaf, eps)
    G = h2.H2(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps).factor()
    got = {(int(l), int(t)): (int(k), int(kt)) for l, t, k, kt in G.forced_ranks()}
    fk = O.forced_from(Fz)
    margin_f = {(l, i): m for (l, i, n, k, kt, m) in Fz.stats}
    bad = []
    for (l, t), k in O.forced_construction(H).items():
        mk = H.sig_margin[l][t]
        in_band_k = abs(mk[0] - 1) < 1e-3 or abs(mk[1] - 1) < 1e-3
        if got[(l, t)][0] != k and not in_band_k:
            bad.append(("k", l, t, got[(l, t)][0], k, mk))
        if (l, t) in fk and got[(l, t)][0] == k:
            mf = margin_f.get((l, t), (np.inf, 0.0))
            in_band_f = abs(mf[0] - 1) < 1e-3 or abs(mf[1] - 1) < 1e-3
            if got[(l, t)][1] != fk[(l, t)] and not in_band_f:
                bad.append(("kt", l, t, got[(l, t)][1], fk[(l, t)], mf))
    assert not bad, bad[:5]


def test_adjoint_multi_rhs_equals_columns():
    """The tile (many right-hand sides) and vector (few) sweep kernels agree."""
    torch = _torch()
    pr, H, Fz = _oracle(*CASES[1])
    G = _gpu(pr, H, Fz).factor()
    rng = np.random.default_rng(5)
    Gm = rng.standard_normal((pr.n, 6)) + 1j * rng.standard_normal((pr.n, 6))
    L = G.solve_adjoint(torch.from_numpy(Gm)).cpu().numpy()
    for j in (0, 3, 5):
        lj = G.solve_adjoint(torch.from_numpy(Gm[:, j].copy())).cpu().numpy()
        assert _rel(L[:, j], lj) < 1e-13
    assert _rel(L, O.solve_adjoint(Fz, Gm)) < 1e-10
