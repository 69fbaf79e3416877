"""Refinement error paths: a non-finite residual and a residual that stays
above the tolerance both end in H2_ERR_NOCONV (never in a reported success)."""
import numpy as np
import pytest

import paper_1703_06155_amd as h2
from paper_1703_06155_amd import inputs as I

pytestmark = pytest.mark.gpu


def _solver():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    pr = I.make_problem("t", (8, 8, 8), 16, 1e-4)
    return torch, pr, h2.H2(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps).factor()


def test_nonfinite_residual_is_an_error():
    torch, pr, G = _solver()
    b = pr.rhs[:, 0].copy()
    b[5] = complex(np.nan, 0.0)
    with pytest.raises(h2.H2Error) as e:
        G.solve(torch.from_numpy(b), tol=1e-8, max_iter=5)
    assert e.value.status == h2.H2_ERR_NOCONV
    assert "not finite" in str(e.value)
    with pytest.raises(h2.H2Error) as e:
        G.solve_adjoint(torch.from_numpy(b), tol=1e-8, max_iter=5)
    assert e.value.status == h2.H2_ERR_NOCONV


def test_unreached_tolerance_reports_the_residual():
    torch, pr, G = _solver()
    b = torch.from_numpy(pr.rhs[:, 0].copy())
    with pytest.raises(h2.H2Error) as e:
        G.solve(b, tol=1e-30, max_iter=1)
    assert e.value.status == h2.H2_ERR_NOCONV
    assert "after 1 iterations" in str(e.value)
    # the handle stays usable
    x, info = G.solve(b, tol=1e-8, info=True)
    assert info["rel_residual"] <= 1e-8
