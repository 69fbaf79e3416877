"""The library's deferred Schur updates (host-only query, no device) against a
plain simulation of the deferral on the oracle's structure.

Eliminating cluster i updates every block (a, b), a <= b, with a and b in i's
inadmissible list (Sec. III-A, eq. 12).  The simulation keeps a pending list per
block; before a colour is eliminated it flushes the blocks that colour processes
(those with a cluster of that colour), then adds the colour's updates; whatever
is left is flushed at the level's end.  Compared per flush: the blocks, and each
block's eliminated clusters in the order they are summed.
"""
import numpy as np
import pytest

import paper_1703_06155_amd as h2
from paper_1703_06155_amd import inputs as I
from oracle import h2_oracle as O


def simulate(S, l):
    col = S.colour[l]
    nb = {}
    for (t, s) in S.near[l]:
        nb.setdefault(t, []).append(s)
    groups = O.colour_groups(S, l)
    pending = {}
    events = []
    for c, cl in enumerate(groups):
        flush = {}
        for key in sorted(pending):
            a, b = key
            if col[a] == c or col[b] == c:
                flush[key] = pending.pop(key)
        events.append(flush)
        for i in cl:
            for a in nb[i]:
                for b in nb[i]:
                    if a <= b:
                        pending.setdefault((a, b), []).append(int(i))
    events.append(pending)
    return len(groups), events


def library_events(rec, ncol):
    events = [dict() for _ in range(ncol + 1)]
    seen = []
    for ev, a, b, i in rec.tolist():
        blocks = events[ev]
        if (a, b) not in blocks:
            blocks[(a, b)] = []
            seen.append((ev, a, b))
        blocks[(a, b)].append(i)
    return events, seen


@pytest.mark.parametrize("grid,leaf,eta", [((10, 9, 8), 16, 1.0), ((12, 12, 12), 27, 1.0), ((13, 7, 11), 20, 0.7)])
def test_schur_schedule_matches_simulated_deferral(grid, leaf, eta):
    pr = I.make_problem("sched", grid, leaf, 1e-4)
    S = O.build_structure(pr.points, pr.h, leaf, eta)
    assert S.l0 is not None
    for l in sorted({S.L, S.L - 1, S.l0}):
        if l < S.l0:
            continue
        ncol, rec = h2.schur_schedule(pr.points, pr.h, leaf, eta, l)
        ncol_o, expected = simulate(S, l)
        assert ncol == ncol_o
        got, order = library_events(rec, ncol)
        for ev in range(ncol + 1):
            assert got[ev] == expected[ev], f"level {l} flush {ev}"
        # within a flush the blocks come once each, in a fixed order (contiguous runs)
        assert len(order) == sum(len(e) for e in got)
        # every update is summed exactly once
        nb = {}
        for (t, s) in S.near[l]:
            nb[t] = nb.get(t, 0) + 1
        assert rec.shape[0] == sum(d * (d + 1) // 2 for d in nb.values())


def test_schur_schedule_rejects_levels_outside_the_factored_range():
    pr = I.make_problem("sched", (10, 9, 8), 16, 1e-4)
    S = O.build_structure(pr.points, pr.h, 16, 1.0)
    with pytest.raises(h2.H2Error):
        h2.schur_schedule(pr.points, pr.h, 16, 1.0, S.L + 1)
    with pytest.raises(h2.H2Error):
        h2.schur_schedule(pr.points, pr.h, 16, 1.0, S.l0 - 1)
