"""Per-kernel timing and roofline ledger (h2_set_kernel_timing, h2_kernel_ledger):
the events leave the results unchanged, every family reports a time, and the
ledger's Schur figures equal those of h2_factor_timing."""
import numpy as np
import pytest

import paper_1703_06155_amd as h2
from paper_1703_06155_amd import inputs as I

pytestmark = pytest.mark.gpu


def test_kernel_ledger_and_timing():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    pr = I.make_problem("t", (12, 12, 12), 27, 1e-4)
    G = h2.H2(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps)
    with pytest.raises(h2.H2Error):
        G.kernel_ledger()
    b = torch.from_numpy(pr.rhs[:, 0].copy()).cuda()
    G.factor()
    x0 = G.solve(b).cpu().numpy()
    led0 = G.kernel_ledger()
    for f in ("gram_fill", "step0_basis", "projection", "partial_lu", "panels"):
        assert led0[f][0] == -1.0, f  # not measured without kernel timing
    G.set_kernel_timing(True).factor()
    x1 = G.solve(b).cpu().numpy()
    assert np.array_equal(x0, x1)
    led = G.kernel_ledger()
    tm = G.timing()
    for f in h2.KERNEL_FAMILIES:
        ms, flops, nbytes = led[f]
        assert ms >= 0.0 and flops >= 0.0 and nbytes > 0.0, (f, led[f])
    for f in ("gram_fill", "projection", "partial_lu", "panels", "schur", "final_lu"):
        assert led[f][1] > 0.0, f
    assert led["schur"][1] == tm[6] and led["schur"][2] == tm[9]
    assert abs(led["schur"][0] - tm[3]) <= 1e-9 * max(1.0, tm[3])
    assert led["sweep_bytes_per_rhs"] > 0 and led["matvec_bytes"] > 0
    # the families cover the factorization's colour phases
    phases = tm[1] + tm[2]
    fam = sum(led[f][0] for f in ("gram_fill", "step0_basis", "projection", "partial_lu", "panels"))
    assert fam <= phases * 1.5 + 1.0, (fam, phases)
    G.set_kernel_timing(False)
