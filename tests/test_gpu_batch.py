"""Batched factor and solve of independent problems (rectangular box grids of
the batching workload's recipe, scaled down) against the same calls made one
handle at a time, in both batch schedules (fused launches across problems and
one stream per handle): results must be bit-identical.  A fused batch that
mixes precisions, stop levels, tree depths and a problem without admissible
blocks; small problems with ranks pinned to the oracle's against its solves."""
import numpy as np
import pytest

import paper_1703_06155_amd as h2
from oracle import h2_oracle as O
from paper_1703_06155_amd import inputs as I

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.mark.parametrize("mode", ["fused", "streams"])
def test_batch_equals_one_by_one(mode):
    torch = _torch()
    probs = I.batch_problems(count=6, nrhs=4, sides=(6, 14), leaf=16)
    solo, batch = [], []
    for pr in probs:
        solo.append(h2.H2(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps).factor())
        batch.append(h2.H2(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps))
    h2.factor_batch(batch, mode=mode)
    for k in range(len(probs)):
        assert np.array_equal(batch[k].stats(), solo[k].stats()), k
    rhs = [torch.from_numpy(pr.rhs.copy()) for pr in probs]
    xs, infos = h2.solve_batch(batch, rhs, tol=1e-8, info=True, mode=mode)
    for k, pr in enumerate(probs):
        x1, i1 = solo[k].solve(rhs[k], tol=1e-8, info=True)
        assert np.array_equal(xs[k].cpu().numpy(), x1.cpu().numpy()), k
        assert infos[k]["iterations"] == i1["iterations"]
        assert infos[k]["rel_residual"] <= 1e-8
    # plain batched solve with graph-replayed sweeps equals the direct launches
    for G in batch:
        G.set_sweep_graph(True)
    xg = h2.solve_batch(batch, rhs, mode=mode)
    for k in range(len(probs)):
        assert np.array_equal(xg[k].cpu().numpy(), solo[k].solve(rhs[k]).cpu().numpy()), k
    # one right-hand side: the matrix-vector sweep kernels
    r1 = [r[:, :1].contiguous() for r in rhs]
    x1 = h2.solve_batch(batch, r1, tol=1e-8, mode=mode)
    for k in range(len(probs)):
        assert np.array_equal(x1[k].cpu().numpy(), solo[k].solve(r1[k], tol=1e-8).cpu().numpy()), k


def test_batch_rejects_duplicates_and_empty():
    _torch()
    pr = I.batch_problems(count=1, nrhs=1, sides=(6, 8), leaf=16)[0]
    G = h2.H2(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps)
    for mode in ("fused", "streams"):
        with pytest.raises(h2.H2Error):
            h2.factor_batch([G, G], mode=mode)
        with pytest.raises(h2.H2Error):
            h2.factor_batch([], mode=mode)
    with pytest.raises(ValueError):
        h2.factor_batch([G], mode="other")


def _settings(k, pr, G):
    """Per-problem settings of the heterogeneous batch: every third problem in the mixed
    form, every other one stopped one level early when its tree allows."""
    if k % 3 == 1:
        G.set_precision("mixed")
    if k % 2 == 0:
        l0, L = G.stop_level_range()
        if L > l0:
            G.set_stop_level(l0 + 1)
    return G


def test_fused_batch_of_mixed_settings_equals_one_by_one():
    torch = _torch()
    probs = I.batch_problems(count=7, nrhs=3, sides=(5, 18), leaf=12)
    # a box too small for any admissible block: the whole matrix is one dense LU
    probs.append(I.make_problem("tiny", (3, 3, 2), 16, 1e-4, nrhs=3))
    solo, batch = [], []
    for k, pr in enumerate(probs):
        solo.append(_settings(k, pr, h2.H2(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps)).factor())
        batch.append(_settings(k, pr, h2.H2(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps)))
    depths = {G.stop_level_range()[1] for G in solo}
    assert solo[-1].stop_level_range()[0] < 0
    assert len(depths) > 1, "the batch should hold trees of different depths"
    h2.factor_batch(batch)
    for k, pr in enumerate(probs):
        assert np.array_equal(batch[k].stats(), solo[k].stats()), k
        b = torch.from_numpy(pr.rhs.copy()).cuda()
        assert np.array_equal(batch[k].solve(b).cpu().numpy(), solo[k].solve(b).cpu().numpy()), k
        assert np.array_equal(batch[k].solve_adjoint(b).cpu().numpy(), solo[k].solve_adjoint(b).cpu().numpy()), k
    # fused batched solves (three columns, then one), refined and plain, against single solves
    rhs = [torch.from_numpy(pr.rhs.copy()).cuda() for pr in probs]
    for cols in (3, 1):
        rr = [r[:, :cols].contiguous() for r in rhs]
        xs, infos = h2.solve_batch(batch, rr, tol=1e-9, info=True)
        x0 = h2.solve_batch(batch, rr)
        for k in range(len(probs)):
            xk, ik = solo[k].solve(rr[k], tol=1e-9, info=True)
            assert np.array_equal(xs[k].cpu().numpy(), xk.cpu().numpy()), (cols, k)
            assert infos[k]["iterations"] == ik["iterations"], (cols, k)
            assert np.array_equal(x0[k].cpu().numpy(), solo[k].solve(rr[k]).cpu().numpy()), (cols, k)
    # a tolerance out of reach in one step: reported for the batch, every problem still solved
    with pytest.raises(h2.H2Error) as ei:
        h2.solve_batch(batch, rhs, tol=1e-300, max_iter=1)
    assert ei.value.status == h2.H2_ERR_NOCONV and "batch item" in str(ei.value)
    # the same handles again: the work item table of the shared launches is reused
    h2.factor_batch(batch)
    for k, pr in enumerate(probs):
        b = torch.from_numpy(pr.rhs.copy()).cuda()
        assert np.array_equal(batch[k].solve(b).cpu().numpy(), solo[k].solve(b).cpu().numpy()), k
    for G in solo + batch:
        G.close()


def test_fused_batch_against_oracle():
    """Three small problems, ranks pinned to the oracle's, factored in one fused batch:
    M^-1 b and M^-H g agree with the oracle's sweeps (Algs. 5-6) to 1e-10 of their
    largest entry."""
    torch = _torch()
    probs = I.batch_problems(count=3, nrhs=2, sides=(7, 12), leaf=14)
    hs, refs = [], []
    for pr in probs:
        H = O.construct(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps)
        Fz = O.factor(H)
        fr = h2.forced_ranks_from_oracle(O.forced_construction(H), O.forced_from(Fz))
        hs.append(h2.H2(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps, forced_ranks=fr))
        refs.append(Fz)
    h2.factor_batch(hs)
    for pr, G, Fz in zip(probs, hs, refs):
        x = G.solve(torch.from_numpy(pr.rhs.copy()).cuda()).cpu().numpy()
        xo = O.solve(Fz, pr.rhs)
        g = np.random.default_rng(5).standard_normal(pr.rhs.shape) + 0.25j
        lam = G.solve_adjoint(torch.from_numpy(g).cuda()).cpu().numpy()
        lo = O.solve_adjoint(Fz, g)
        ex = float(np.abs(x - xo).max() / np.abs(xo).max())
        el = float(np.abs(lam - lo).max() / np.abs(lo).max())
        print(f"{pr.name} N={pr.n}: fused batch vs oracle x {ex:.1e}, lam {el:.1e}")
        assert ex < 1e-10 and el < 1e-10
        G.close()


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
