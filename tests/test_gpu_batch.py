"""Batched factor and solve of independent problems (rectangular box grids of
the batching workload's recipe, scaled down) against the same calls made one
handle at a time: results must be bit-identical."""
import numpy as np
import pytest

import paper_1703_06155_amd as h2
from paper_1703_06155_amd import inputs as I

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def test_batch_equals_one_by_one():
    torch = _torch()
    probs = I.batch_problems(count=6, nrhs=4, sides=(6, 14), leaf=16)
    solo, batch = [], []
    for pr in probs:
        solo.append(h2.H2(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps).factor())
        batch.append(h2.H2(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps))
    h2.factor_batch(batch)
    rhs = [torch.from_numpy(pr.rhs.copy()) for pr in probs]
    xs, infos = h2.solve_batch(batch, rhs, tol=1e-8, info=True)
    for k, pr in enumerate(probs):
        x1, i1 = solo[k].solve(rhs[k], tol=1e-8, info=True)
        assert np.array_equal(xs[k].cpu().numpy(), x1.cpu().numpy()), k
        assert infos[k]["iterations"] == i1["iterations"]
        assert infos[k]["rel_residual"] <= 1e-8
    # plain batched solve with graph-replayed sweeps equals the direct launches
    for G in batch:
        G.set_sweep_graph(True)
    xg = h2.solve_batch(batch, rhs)
    for k in range(len(probs)):
        assert np.array_equal(xg[k].cpu().numpy(), solo[k].solve(rhs[k]).cpu().numpy()), k


def test_batch_rejects_duplicates_and_empty():
    _torch()
    pr = I.batch_problems(count=1, nrhs=1, sides=(6, 8), leaf=16)[0]
    G = h2.H2(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps)
    with pytest.raises(h2.H2Error):
        h2.factor_batch([G, G])
    with pytest.raises(h2.H2Error):
        h2.factor_batch([])


def test_batch_mixed_equals_one_by_one_and_refines():
    """The mixed form (complex FP32 Schur terms and projections) batched: bit-identical
    to one handle at a time, refined to the FP64 form's residual of 1e-8."""
    torch = _torch()
    probs = I.batch_problems(count=4, nrhs=4, sides=(8, 16), leaf=16)
    solo, batch = [], []
    for pr in probs:
        solo.append(h2.H2(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps, precision="mixed").factor())
        batch.append(h2.H2(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps, precision="mixed"))
    h2.factor_batch(batch)
    rhs = [torch.from_numpy(pr.rhs.copy()) for pr in probs]
    xs, infos = h2.solve_batch(batch, rhs, tol=1e-8, info=True)
    for k, pr in enumerate(probs):
        x1, i1 = solo[k].solve(rhs[k], tol=1e-8, info=True)
        assert np.array_equal(xs[k].cpu().numpy(), x1.cpu().numpy()), k
        assert infos[k]["rel_residual"] <= 1e-8, infos[k]
        ref = h2.H2(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps).factor()
        xr = ref.solve(rhs[k], tol=1e-8).cpu().numpy()
        rel = np.linalg.norm(xs[k].cpu().numpy() - xr) / np.linalg.norm(xr)
        print(f"problem {k}: N={pr.n} mixed iterations {infos[k]['iterations']}, vs refined FP64 {rel:.1e}")
        assert rel <= 1e-6
