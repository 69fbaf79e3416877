"""Sweeps replayed from captured HIP graphs give exactly the results of the
direct launches, on every replay, with other GPU work and synchronisations in
between, for both directions and several right-hand-side counts, and again
after a refactorization (which drops and recaptures the graphs)."""
import numpy as np
import pytest

import paper_1703_06155_amd as h2
from paper_1703_06155_amd import inputs as I

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.mark.parametrize("grid,leaf,eps", [((10, 7, 9), 12, 1e-5), ((16, 16, 16), 64, 1e-4)],
                         ids=["10x7x9_leaf12", "16^3_leaf64"])
def test_graph_replays_equal_direct_launches(grid, leaf, eps):
    torch = _torch()
    pr = I.make_problem("t", grid, leaf, eps)
    G = h2.H2(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps).factor()
    rng = np.random.default_rng(5)
    B3 = torch.from_numpy(rng.standard_normal((pr.n, 3)) + 1j * rng.standard_normal((pr.n, 3)))
    B8 = torch.from_numpy(rng.standard_normal((pr.n, 8)) + 1j * rng.standard_normal((pr.n, 8)))
    b1 = torch.from_numpy(pr.rhs[:, 0].copy())

    def run():
        return (G.solve(b1).cpu().numpy(), G.solve(B3).cpu().numpy(), G.solve(B8).cpu().numpy(),
                G.solve_adjoint(B3).cpu().numpy(), G.solve(b1, tol=1e-8).cpu().numpy())

    ref = run()
    G.set_sweep_graph(True)
    for rep in range(4):
        out = run()
        for a, r in zip(out, ref):
            assert np.array_equal(a, r), f"replay {rep} differs"
        # unrelated eager work and a synchronisation between replays
        G.matvec(B3)
        torch.cuda.synchronize()
    # a new factorization drops the graphs; the recaptured ones match the direct launches again
    chi2 = I.contrast(pr.n, seed=42)
    G.set_contrast(chi2).factor()
    G.set_sweep_graph(False)
    ref2 = run()
    G.set_sweep_graph(True)
    for rep in range(3):
        out = run()
        for a, r in zip(out, ref2):
            assert np.array_equal(a, r), f"replay {rep} after refactorization differs"
