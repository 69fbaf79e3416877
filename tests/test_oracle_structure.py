"""Pins for the oracle's cluster tree, block partition and colouring (Sec. II, eq. 1)."""
import json
import os

import numpy as np
import pytest

from oracle import h2_oracle as O
from paper_1703_06155_amd import inputs as I

GOLD = os.path.join(os.path.dirname(__file__), "golden", "structure_counts.json")


def _cases():
    with open(GOLD) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: "x".join(map(str, c["grid"])) + f"_leaf{c['leaf']}")
def test_structure_counts(case):
    """Tree depth, leaf sizes, l0, pair counts, degrees and colours of the stated rules."""
    pts = I.cube_grid(*case["grid"])
    S = O.build_structure(pts, I.CELL, case["leaf"], 1.0)
    L = S.L
    sz = np.array([c.size for c in S.clusters[L]])
    assert L == case["L"]
    assert sz.size == case["leaves"] and sz.min() == case["leaf_min"] and sz.max() == case["leaf_max"]
    assert S.l0 == case["l0"]
    assert len(S.adm[L]) == case["adm_leaf"] and len(S.near[L]) == case["near_leaf"]
    deg = np.bincount([t for (t, s) in S.near[L] if t != s], minlength=sz.size)
    assert deg.max() == case["deg_max"]
    nb = [set() for _ in range(sz.size)]
    for (t, s) in S.near[L]:
        nb[t].add(s)
    two = np.array([len(set().union(*[nb[a] for a in nb[t]]) - nb[t]) for t in range(sz.size)])
    assert round(float(two.mean()), 1) == case["twohop_mean"] and two.max() == case["twohop_max"]
    assert int(S.colour[L].max()) + 1 == case["colours"]
    for l, (na, nn) in case.get("per_level", {}).items():
        assert (len(S.adm[int(l)]), len(S.near[int(l)])) == (na, nn)


def _partition_owner(S, n):
    """Brute force: for every (row, col) index pair, count the blocks that cover it."""
    cover = np.zeros((n, n), dtype=np.int64)
    for l in range(S.L + 1):
        for (t, s) in S.adm[l]:
            cover[np.ix_(S.clusters[l][t], S.clusters[l][s])] += 1
    for (t, s) in S.near[S.L]:
        cover[np.ix_(S.clusters[S.L][t], S.clusters[S.L][s])] += 1
    return cover


@pytest.mark.parametrize("grid,leaf,eta", [((8, 8, 8), 16, 1.0), ((10, 7, 9), 12, 1.0),
                                           ((6, 6, 6), 8, 1.0), ((9, 5, 3), 7, 0.7),
                                           ((8, 8, 8), 16, 0.0)])
def test_partition_and_admissibility(grid, leaf, eta):
    """Blocks tile the N x N index set exactly once; eq. 1 holds on admissible blocks only."""
    pts = I.cube_grid(*grid)
    h = I.CELL
    S = O.build_structure(pts, h, leaf, eta)
    n = pts.shape[0]
    assert np.all(_partition_owner(S, n) == 1)
    # the tree: children partition the parent, every leaf within leafsize, uniform depth
    assert all(c.size <= leaf for c in S.clusters[S.L])
    for l in range(S.L):
        for t, c in enumerate(S.clusters[l]):
            kids = np.concatenate([S.clusters[l + 1][2 * t], S.clusters[l + 1][2 * t + 1]])
            assert np.array_equal(kids, c)
    assert sorted(S.perm.tolist()) == list(range(n))

    def box(idx):
        p = pts[idx]
        return p.min(0) - h / 2, p.max(0) + h / 2

    def cond(t, s, l):
        a, b = box(S.clusters[l][t]), box(S.clusters[l][s])
        diam = max(np.linalg.norm(a[1] - a[0]), np.linalg.norm(b[1] - b[0]))
        # distance between the two boxes, by brute force over the cell corners' projections
        gap = [max(0.0, b[0][d] - a[1][d], a[0][d] - b[1][d]) for d in range(3)]
        return diam <= eta * float(np.sqrt(sum(g * g for g in gap))) * (1 + 1e-10)

    for l in range(1, S.L + 1):
        for (t, s) in S.adm[l]:
            assert cond(t, s, l)
            assert (t // 2, s // 2) in set(S.near[l - 1])
        for (t, s) in S.near[l]:
            assert not cond(t, s, l)
    if eta == 0.0:
        assert S.l0 is None


@pytest.mark.parametrize("grid,leaf", [((16, 16, 16), 32), ((13, 27, 19), 48)])
def test_colouring_is_proper_and_greedy(grid, leaf):
    """No two inadmissible neighbours share a colour; each colour is the smallest free one."""
    pts = I.cube_grid(*grid)
    S = O.build_structure(pts, I.CELL, leaf, 1.0)
    for l in range(S.l0, S.L + 1):
        col = S.colour[l]
        nb = {}
        for (t, s) in S.near[l]:
            if t != s:
                assert col[t] != col[s]
                nb.setdefault(t, []).append(s)
        for t in range(col.size):
            earlier = {col[s] for s in nb.get(t, []) if s < t}
            assert col[t] == min(set(range(col[t] + 1)) - earlier)


def test_far_field_is_complement_of_near_field():
    """F*(t) (admissible blocks of t and its ancestors) = all columns outside t's near field."""
    pts = I.cube_grid(10, 7, 9)
    S = O.build_structure(pts, I.CELL, 12, 1.0)
    n = pts.shape[0]
    for l in range(S.l0, S.L + 1):
        for t in range(len(S.clusters[l])):
            near_cols = np.concatenate([S.clusters[l][s] for (a, s) in S.near[l] if a == t])
            comp = np.setdiff1d(np.arange(n), near_cols)
            assert np.array_equal(O.far_field(S, l, t), comp)
