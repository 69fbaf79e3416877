"""Plain FP64 CPU oracle for the accuracy-controlled H^2 direct solver.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never does.

It restates, in slow and readable NumPy/SciPy (complex128), what Ma & Jiao,
"Accuracy Directly Controlled Fast Direct Solutions of General H^2-Matrices"
(arXiv:1703.06155) compute:

* cluster tree, admissibility and block partition        (Sec. II, eq. 1)
* nested cluster bases and coupling matrices             (Sec. II, eqs. 2-3)
* level-by-level factorization, Steps 0-3                (Sec. III-A/B, eqs. 4-33, Algs. 1-4)
* product-form factors and their inverse                 (Sec. III-C, eqs. 34-35)
* early stop: a dense LU once a level brings few zeros    (Sec. III-C, closing remark)
* forward / backward substitution                        (Sec. IV, eqs. 36-42, Algs. 5-6)
* the relative residual used as the accuracy measure      (Sec. VI-B)

plus the adjoint solve, the H^2 matrix-vector product, iterative refinement
and the contrast gradient that the solver's interface adds around them.

Readings of points the paper leaves open (each one is listed with its reason
in the design notes):
  R1  the factorized matrix is the complex-symmetric Z = A D^-1 with
      D = diag(k^2 h^3 chi); one basis per cluster serves rows and columns,
      as eqs. 2, 5, 7-8 and 16 require;
  R2  within a tree level clusters are processed colour by colour (greedy
      colouring of the level's inadmissible graph, clusters of one colour are
      never inadmissible with each other); the clusters of one colour take
      each step of Alg. 1 together, on the state left by the previous colour;
  R3  uniform-depth bisection at the bounding-box midpoint of the longest side;
  R4  admissibility on cell-support boxes (centres +- h/2), with a relative
      tie tolerance of 1e-10;
  R5  construction keeps sigma_j > eps*sigma_1 of each cluster's far-field
      block row; Step 0 keeps sigma_j(W) > eps_fill*max(nu_i, sigma_1(W));
  R6  partial pivoting inside the eliminated diagonal block F_i'i';
  R7  fill-ins are stored as the increment that the Schur complement adds;
  R8  the eliminated coordinates come first in Q = [V_perp  V] (eq. 4).

Parity pins (tests/test_oracle_*.py): tree and partition invariants and
counts, kernel entries against closed forms, nested-basis identities, the
Step 0 rank rule on fill-ins of designed spectrum and the eq. 17 bound on
the dropped fill-ins, zero introduction (eqs. 7-8), the
no-truncation limit against a dense solve of the represented matrix, the
eta = 0 limit against dense LU, the early stop at every level from l0 to L
against a dense solve of the represented matrix (no truncation), the adjoint
dot-product identity, accuracy versus eps, linear storage on rods, and the
gradient against finite differences of a dense solve.  No function here is
"parity unpinned".
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

# --------------------------------------------------------------------------
# Matrix entries (the synthetic VIE kernel); R1
# --------------------------------------------------------------------------


def self_term(k: float, h: float) -> complex:
    """(1 + jka) e^{-jka} - 1 with a the radius of the sphere of volume h^3."""
    a = (3.0 / (4.0 * math.pi)) ** (1.0 / 3.0) * h
    return (1.0 + 1j * k * a) * np.exp(-1j * k * a) - 1.0


def dense_A(points, k, h, chi):
    """User matrix A_ij = k^2 chi_j h^3 e^{-jkr}/(4 pi r), A_ii = 1 + chi_i c."""
    d = points[:, None, :] - points[None, :, :]
    r = np.sqrt((d * d).sum(-1))
    np.fill_diagonal(r, 1.0)
    A = np.exp(-1j * k * r) / (4.0 * np.pi * r) * (k * k * h ** 3 * chi)[None, :]
    np.fill_diagonal(A, 1.0 + chi * self_term(k, h))
    return A


def z_block(points, rows, cols, k, h, chi):
    """Entries Z[rows, cols] of Z = A D^-1 (R1); rows/cols index the points."""
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    d = points[rows][:, None, :] - points[cols][None, :, :]
    r = np.sqrt((d * d).sum(-1))
    same = rows[:, None] == cols[None, :]
    r = np.where(same, 1.0, r)
    Z = np.exp(-1j * k * r) / (4.0 * np.pi * r)
    if same.any():
        diag = (1.0 + chi * self_term(k, h)) / (k * k * h ** 3 * chi)
        Z = np.where(same, diag[rows][:, None], Z)
    return Z


def dense_Z(points, k, h, chi):
    idx = np.arange(points.shape[0])
    return z_block(points, idx, idx, k, h, chi)


# --------------------------------------------------------------------------
# Cluster tree and block partition (Sec. II, eq. 1); R3, R4
# --------------------------------------------------------------------------


def split_cluster(points, idx):
    """Bisect at the midpoint of the longest bounding-box side (first axis on ties)."""
    if idx.size == 0:
        return idx, idx
    p = points[idx]
    lo, hi = p.min(0), p.max(0)
    axis = int(np.argmax(hi - lo))
    mid = 0.5 * (lo[axis] + hi[axis])
    left = p[:, axis] < mid
    return idx[left], idx[~left]


@dataclass
class Structure:
    L: int
    clusters: list            # clusters[l][t] -> point indices (original numbering)
    perm: np.ndarray          # tree order -> original index
    start: list               # start[l][t] offset of cluster t in tree order
    near: list                # near[l] sorted list of inadmissible (t, s), incl. (t, t)
    adm: list                 # adm[l] sorted list of admissible (t, s)
    l0: int | None            # coarsest level with an admissible block
    colour: list              # colour[l][t] (-1 for empty clusters)
    boxes: list               # (lo, hi) cell-support box per cluster per level

    def size(self, l, t):
        return self.clusters[l][t].size


def build_structure(points, h, leaf, eta):
    """Tree (uniform depth), lockstep block tree and per-level greedy colouring."""
    n = points.shape[0]
    levels = [[np.arange(n)]]
    while any(c.size > leaf for c in levels[-1]):
        nxt = []
        for c in levels[-1]:
            nxt.extend(split_cluster(points, c))
        levels.append(nxt)
    L = len(levels) - 1
    perm = np.concatenate(levels[L]).astype(np.int64)
    start = []
    for l in range(L + 1):
        sizes = np.array([c.size for c in levels[l]], dtype=np.int64)
        start.append(np.concatenate([[0], np.cumsum(sizes)[:-1]]))
        # every cluster lists its points in tree order (children concatenated)
        levels[l] = [perm[start[l][t]:start[l][t] + sizes[t]] for t in range(sizes.size)]
    boxes = []
    for l in range(L + 1):
        bl = []
        for c in levels[l]:
            if c.size == 0:
                bl.append(None)
            else:
                p = points[c]
                bl.append((p.min(0) - 0.5 * h, p.max(0) + 0.5 * h))
        boxes.append(bl)

    def diam(b):
        return float(np.linalg.norm(b[1] - b[0]))

    def dist(b1, b2):
        gap = np.maximum(0.0, np.maximum(b2[0] - b1[1], b1[0] - b2[1]))
        return float(np.linalg.norm(gap))

    near = [[(0, 0)]]
    adm = [[]]
    for l in range(1, L + 1):
        nl, al = [], []
        for (t, s) in near[l - 1]:
            for tc in (2 * t, 2 * t + 1):
                if boxes[l][tc] is None:
                    continue
                for sc in (2 * s, 2 * s + 1):
                    if boxes[l][sc] is None:
                        continue
                    bt, bs = boxes[l][tc], boxes[l][sc]
                    if max(diam(bt), diam(bs)) <= eta * dist(bt, bs) * (1.0 + 1e-10):
                        al.append((tc, sc))
                    else:
                        nl.append((tc, sc))
        near.append(sorted(nl))
        adm.append(sorted(al))
    l0 = next((l for l in range(L + 1) if adm[l]), None)

    colour = []
    for l in range(L + 1):
        nb = {}
        for (t, s) in near[l]:
            if t != s:
                nb.setdefault(t, []).append(s)
        col = -np.ones(len(levels[l]), dtype=np.int64)
        for t in range(len(levels[l])):
            if levels[l][t].size == 0:
                continue
            used = {col[s] for s in nb.get(t, []) if col[s] >= 0}
            c = 0
            while c in used:
                c += 1
            col[t] = c
        colour.append(col)
    return Structure(L, levels, perm, start, near, adm, l0, colour, boxes)


def colour_groups(S, l):
    """Clusters of level l grouped by colour, colours ascending, indices ascending."""
    col = S.colour[l]
    return [list(np.nonzero(col == c)[0]) for c in range(int(col.max()) + 1)]


def far_field(S, l, t):
    """F*(t): columns of all admissible blocks of t and of its ancestors."""
    parts = []
    tt = t
    for ll in range(l, -1, -1):
        for (a, b) in S.adm[ll]:
            if a == tt:
                parts.append(S.clusters[ll][b])
        tt //= 2
    if not parts:
        return np.zeros(0, dtype=np.int64)
    return np.sort(np.concatenate(parts))


# --------------------------------------------------------------------------
# H^2 construction: truncated SVD of far-field block rows (eqs. 2-3); R5
# --------------------------------------------------------------------------


@dataclass
class H2Matrix:
    S: Structure
    points: np.ndarray
    k: float
    h: float
    chi: np.ndarray
    eps: float
    rank: list                # rank[l][t] construction rank k_t
    nu: list                  # nu[l][t] largest singular value of the far-field row
    basis: list               # basis[L][t] = V_t (leaf) ; basis[l][t] = T_t (l < L)
    expanded: list            # expanded[l][t] = script-V_t (#t x k_t)
    coupling: list            # coupling[l][(t, s)] = S_ts for (t, s) in adm[l]
    near_blocks: dict         # (t, s) in near[L] -> Z[t, s]
    sig_margin: list          # per cluster: (sigma_k/thr, sigma_{k+1}/thr)


def _truncate(sig, thr, cap):
    k = int(np.count_nonzero(sig > thr))
    return min(k, cap)


def construct(points, k, h, chi, leaf, eta, eps, forced_ranks=None, structure=None):
    """Nested bases from truncated SVDs of the far-field block rows, couplings S_ts."""
    S = structure if structure is not None else build_structure(points, h, leaf, eta)
    L = S.L
    rank = [np.zeros(len(S.clusters[l]), dtype=np.int64) for l in range(L + 1)]
    nu = [np.zeros(len(S.clusters[l])) for l in range(L + 1)]
    margin = [[(np.inf, 0.0)] * len(S.clusters[l]) for l in range(L + 1)]
    basis = [[None] * len(S.clusters[l]) for l in range(L + 1)]
    expanded = [[None] * len(S.clusters[l]) for l in range(L + 1)]
    # Y[t] = script-V_t^H Z[t, :] for the level below (nested reuse)
    Y_prev = None
    lmin = S.l0 if S.l0 is not None else L + 1
    for l in range(L, lmin - 1, -1):
        Y_cur = [None] * len(S.clusters[l])
        for t, idx in enumerate(S.clusters[l]):
            if idx.size == 0:
                basis[l][t] = np.zeros((0, 0), complex)
                expanded[l][t] = np.zeros((0, 0), complex)
                Y_cur[t] = np.zeros((0, points.shape[0]), complex)
                continue
            far = far_field(S, l, t)
            if l == L:
                row = z_block(points, idx, np.arange(points.shape[0]), k, h, chi)
                Bhat = row[:, far]
                cap = idx.size
            else:
                c1, c2 = 2 * t, 2 * t + 1
                rowstack = np.vstack([Y_prev[c1], Y_prev[c2]])
                Bhat = rowstack[:, far]
                cap = rowstack.shape[0]
            if far.size == 0 or Bhat.shape[0] == 0:
                U = np.zeros((Bhat.shape[0], 0), complex)
                sig = np.zeros(0)
            else:
                U, sig, _ = np.linalg.svd(Bhat, full_matrices=False)
            s1 = sig[0] if sig.size else 0.0
            thr = eps * s1
            kt = _truncate(sig, thr, cap) if s1 > 0 else 0
            if forced_ranks is not None and (l, t) in forced_ranks:
                kt = min(int(forced_ranks[(l, t)]), cap, sig.size)
            if s1 > 0:
                above = sig[kt - 1] / thr if kt > 0 else np.inf
                below = sig[kt] / thr if kt < sig.size else 0.0
                margin[l][t] = (above, below)
            rank[l][t] = kt
            nu[l][t] = s1
            Bt = U[:, :kt].copy()
            basis[l][t] = Bt
            if l == L:
                expanded[l][t] = Bt
                Y_cur[t] = Bt.conj().T @ row
            else:
                E1, E2 = expanded[l + 1][2 * t], expanded[l + 1][2 * t + 1]
                k1 = E1.shape[1]
                expanded[l][t] = np.vstack([E1 @ Bt[:k1], E2 @ Bt[k1:]])
                Y_cur[t] = Bt.conj().T @ rowstack
        Y_prev = Y_cur
    coupling = [dict() for _ in range(L + 1)]
    for l in range(lmin, L + 1):
        for (t, s) in S.adm[l]:
            if t <= s:
                Zts = z_block(points, S.clusters[l][t], S.clusters[l][s], k, h, chi)
                Sts = expanded[l][t].conj().T @ Zts @ expanded[l][s].conj()
                coupling[l][(t, s)] = Sts
                coupling[l][(s, t)] = Sts.T.copy()
    near_blocks = {}
    for (t, s) in S.near[L]:
        near_blocks[(t, s)] = z_block(points, S.clusters[L][t], S.clusters[L][s], k, h, chi)
    return H2Matrix(S, points, k, h, chi, eps, rank, nu, basis, expanded, coupling,
                    near_blocks, margin)


def h2_dense(H):
    """Dense reconstruction of Z_H2 in the original point numbering."""
    n = H.points.shape[0]
    Z = np.zeros((n, n), complex)
    S = H.S
    for (t, s), B in H.near_blocks.items():
        Z[np.ix_(S.clusters[S.L][t], S.clusters[S.L][s])] = B
    for l in range(S.L + 1):
        for (t, s), C in H.coupling[l].items():
            Z[np.ix_(S.clusters[l][t], S.clusters[l][s])] = (
                H.expanded[l][t] @ C @ H.expanded[l][s].T)
    return Z


def h2_matvec_z(H, v):
    """Z_H2 v block by block: inadmissible leaf blocks plus V_t S_ts V_s^T (eq. 2)."""
    v = np.asarray(v, complex)
    out = np.zeros_like(v)
    S = H.S
    for (t, s), B in H.near_blocks.items():
        out[S.clusters[S.L][t]] += B @ v[S.clusters[S.L][s]]
    for l in range(S.L + 1):
        for (t, s), C in H.coupling[l].items():
            xs = H.expanded[l][s].T @ v[S.clusters[l][s]]
            out[S.clusters[l][t]] += H.expanded[l][t] @ (C @ xs)
    return out


def d_scale(H):
    return H.k * H.k * H.h ** 3 * H.chi


def h2_matvec(H, x, adjoint=False):
    """A_H2 x = Z_H2 (D x); with adjoint=True, A_H2^H x = D conj(Z_H2) x (Z_H2 symmetric)."""
    x = np.asarray(x, complex)
    D = d_scale(H)
    if x.ndim == 2:
        D = D[:, None]
    if not adjoint:
        return h2_matvec_z(H, D * x)
    return D * np.conj(h2_matvec_z(H, np.conj(x)))


# --------------------------------------------------------------------------
# Factorization (Sec. III, Algs. 1-4)
# --------------------------------------------------------------------------


def _pivot_apply(piv, X):
    """Apply LAPACK row interchanges (row j <-> row piv[j], j ascending)."""
    X = X.copy()
    for j, p in enumerate(piv):
        if p != j:
            X[[j, p]] = X[[p, j]]
    return X


def _pivot_apply_T(piv, X):
    """Inverse of _pivot_apply (interchanges in reverse order)."""
    X = X.copy()
    for j in range(len(piv) - 1, -1, -1):
        p = piv[j]
        if p != j:
            X[[j, p]] = X[[p, j]]
    return X


class SingularPivot(RuntimeError):
    pass


def _lu(F):
    if F.shape[0] == 0:
        return np.zeros((0, 0), complex), np.zeros(0, dtype=np.int32)
    lu, piv = sla.lu_factor(F, check_finite=True)
    if F.shape[0] and np.min(np.abs(np.diag(lu))) == 0.0:
        raise SingularPivot("zero pivot in partial LU")
    return lu, piv


def _tri(lu, b, lower, unit=False, trans="N"):
    """Triangular solve with the packed LU factor; empty systems pass through."""
    if lu.shape[0] == 0:
        return b.copy()
    return sla.solve_triangular(lu, b, lower=lower, unit_diagonal=unit, trans=trans)


def _Linv(lu, piv, X):
    """L^-1 P X for the pivoted LU (unit lower)."""
    if lu.shape[0] == 0 or X.size == 0:
        return np.zeros((lu.shape[0], X.shape[1]), complex)
    return sla.solve_triangular(lu, _pivot_apply(piv, X), lower=True, unit_diagonal=True)


def _right_Uinv(lu, X):
    """X U^-1."""
    if lu.shape[0] == 0 or X.size == 0:
        return np.zeros((X.shape[0], lu.shape[0]), complex)
    return sla.solve_triangular(lu, X.T, trans="T", lower=False).T


@dataclass
class ClusterFactor:
    n: int
    k: int
    kt: int
    r: int
    Q: np.ndarray             # Q~_i = [B~perp, B~] (n x n, unitary)
    lu: np.ndarray
    piv: np.ndarray
    partners: list            # N+(i) ascending (includes i)
    C: dict                   # a -> C_a = Z_ai' U^-1   (current rows of a x r)
    R: dict                   # a -> R_a = L^-1 P Z_i'a (r x current cols of a)
    sig_margin: tuple = (np.inf, 0.0)


@dataclass
class Factorization:
    H: H2Matrix
    levels: list              # levels[j] for l = L - j: dict with clusters, order, merge info
    final_lu: tuple
    final_n: int
    order_mode: str
    ledger: dict = field(default_factory=dict)
    stats: list = field(default_factory=list)


def fill_spectrum(Bi, W, nu_i, efill, cap):
    """Step 0 of one cluster (eqs. 16-17 / 25-26): the directions of the fill-ins
    W outside the current basis Bi, and how many of them to add.

    G = P W W^H P^H with P = I - Bi Bi^H (eq. 16); its eigenvectors U and the
    square roots sig of its eigenvalues, largest first, are the left singular
    vectors and singular values of P W.  The threshold is
    tau = efill * max(nu_i, sig_1) (R5: relative to the larger of the cluster's
    construction sigma_1 and the fill-ins' own); p = #{sig_j > tau}, at most
    cap.  Returns (U, sig, tau, p, margin), margin = (sig_p / tau,
    sig_{p+1} / tau) for the rank-parity band.
    """
    n_i = Bi.shape[0]
    P = np.eye(n_i) - Bi @ Bi.conj().T
    G = P @ (W @ W.conj().T) @ P.conj().T
    G = 0.5 * (G + G.conj().T)
    lam, U = np.linalg.eigh(G)
    lam, U = lam[::-1], U[:, ::-1]
    sig = np.sqrt(np.maximum(lam, 0.0))
    tau = efill * max(nu_i, sig[0])
    p = _truncate(sig, tau, cap) if tau > 0 else 0
    margin = (np.inf, 0.0)
    if tau > 0:
        margin = (sig[p - 1] / tau if p > 0 else np.inf,
                  sig[p] / tau if p < sig.size else 0.0)
    return U, sig, tau, p, margin


def factor(H, eps_fill=None, order="colour", forced_kt=None, trace=None, step0_trace=None, stop_level=None):
    """Level-by-level factorization Z_H2 = L U in product form (eq. 34).

    order="colour": clusters of one colour take each step together (R2);
    order="sequential": one cluster at a time in the same colour-major order.
    forced_kt maps (level, cluster) -> k~ to pin the Step 0 rank decisions.
    trace / step0_trace (lists, test use) receive the state at the start of
    every level / the fill-ins W and threshold of every Step 0.
    stop_level (default l0): the last level factored; the matrix merged to the
    level above it is then factored densely (Sec. III-C: when a level brings
    few zeros, the rest is better done by a dense LU).
    """
    S = H.S
    L = S.L
    efill = H.eps if eps_fill is None else eps_fill
    ledger = {"gemm": 0.0, "lu": 0.0, "trsm": 0.0}
    if S.l0 is None:
        # no admissible block anywhere: a dense LU of the whole matrix (Alg. 1, line 14)
        Zt = np.zeros((S.perm.size, S.perm.size), complex)
        for (t, s), B in H.near_blocks.items():
            a0, b0 = S.start[L][t], S.start[L][s]
            Zt[a0:a0 + B.shape[0], b0:b0 + B.shape[1]] = B
        return Factorization(H, [], _lu(Zt), Zt.shape[0], order, ledger)

    ls = S.l0 if stop_level is None else int(stop_level)
    if not S.l0 <= ls <= L:
        raise ValueError(f"stop_level must lie in [l0, L] = [{S.l0}, {L}]")
    # level-L state
    nsz = np.array([c.size for c in S.clusters[L]], dtype=np.int64)
    B = [H.basis[L][t] for t in range(len(nsz))]
    kk = H.rank[L].copy()
    nu = H.nu[L].copy()
    Z = {key: val.copy() for key, val in H.near_blocks.items()}
    fills = {}
    levels = []
    stats = []
    for l in range(L, ls - 1, -1):
        if trace is not None:
            trace.append(dict(level=l, n=nsz.copy(), B=list(B), Z={a: v.copy() for a, v in Z.items()},
                              fills={a: v.copy() for a, v in fills.items()}))
        ncl = len(S.clusters[l])
        nearset = set(S.near[l])
        partners = [[] for _ in range(ncl)]
        for (t, s) in S.near[l]:
            partners[t].append(s)
        done = np.zeros(ncl, bool)
        r = np.zeros(ncl, dtype=np.int64)
        kt = kk.copy()
        facs = [None] * ncl

        def cur(a):
            return nsz[a] - r[a] if done[a] else nsz[a]

        groups = colour_groups(S, l)
        if order == "sequential":
            groups = [[i] for g in groups for i in g]
        for grp in groups:
            grp = [i for i in grp if S.clusters[l][i].size > 0]
            if not grp:
                continue
            gset = set(grp)
            Qs = {}
            # Steps 0 and 1 (Alg. 2; eqs. 16-19 / 25-28)
            for i in grp:
                n_i, k_i = nsz[i], kk[i]
                Bi = B[i]
                cols = [fills[(i, b)] for b in sorted(b for (a, b) in fills if a == i)]
                margin = (np.inf, 0.0)
                if cols and n_i > 0:
                    W = np.hstack(cols)
                    U, sig, tau, p, margin = fill_spectrum(Bi, W, nu[i], efill, n_i - k_i)
                    ledger["gemm"] += 8.0 * n_i * n_i * W.shape[1]
                    if step0_trace is not None:
                        step0_trace.append(dict(level=l, cluster=i, W=W, tau=tau, p=p))
                else:
                    U = np.zeros((n_i, 0), complex)
                    p = 0
                if forced_kt is not None and (l, i) in forced_kt:
                    p = int(forced_kt[(l, i)]) - k_i
                    if p < 0 or p > n_i - k_i:
                        raise ValueError("forced rank out of range")
                Uadd = U[:, :p]
                if p > 0:
                    Uadd = Uadd - Bi @ (Bi.conj().T @ Uadd)
                    Uadd, _ = np.linalg.qr(Uadd)
                Bt = np.hstack([Bi, Uadd])
                ktil = k_i + p
                if ktil == 0:
                    Qfull = np.eye(n_i, dtype=complex)
                else:
                    Qfull, _ = np.linalg.qr(Bt, mode="complete")
                Qs[i] = np.hstack([Qfull[:, ktil:], Bt])
                kt[i] = ktil
                stats.append((l, i, n_i, k_i, ktil, margin))
                facs[i] = ClusterFactor(n_i, k_i, ktil, n_i - ktil, Qs[i], None, None,
                                        sorted(partners[i]), {}, {}, margin)
            # Step 2 (Alg. 3; eqs. 5, 30): Q^H Z Qbar on blocks of row/column i
            for key in list(Z.keys()):
                x, y = key
                if x in gset or y in gset:
                    M = Z[key]
                    if x in gset:
                        M = Qs[x].conj().T @ M
                        ledger["gemm"] += 8.0 * M.shape[0] ** 2 * M.shape[1]
                    if y in gset:
                        M = M @ Qs[y].conj()
                        ledger["gemm"] += 8.0 * M.shape[0] * M.shape[1] ** 2
                    Z[key] = M
            for key in list(fills.keys()):
                x, y = key
                if x in gset or y in gset:
                    M = fills[key]
                    if x in gset:
                        M = (Qs[x].conj().T @ M)[nsz[x] - kt[x]:]
                    if y in gset:
                        M = (M @ Qs[y].conj())[:, nsz[y] - kt[y]:]
                    fills[key] = M
            # Step 3 (Alg. 4; eqs. 9-15)
            for i in grp:
                f = facs[i]
                ri = f.r
                F = Z[(i, i)][:ri, :ri]
                lu, piv = _lu(F)
                f.lu, f.piv = lu, piv
                ledger["lu"] += 8.0 / 3.0 * ri ** 3
                parts = f.partners
                Zia = [Z[(i, a)][:ri, ri:] if a == i else Z[(i, a)][:ri, :] for a in parts]
                Zai = [Z[(a, i)][ri:, :ri] if a == i else Z[(a, i)][:, :ri] for a in parts]
                wc = np.cumsum([0] + [m.shape[1] for m in Zia])
                wr = np.cumsum([0] + [m.shape[0] for m in Zai])
                Rcat = _Linv(lu, piv, np.hstack(Zia))
                Ccat = _right_Uinv(lu, np.vstack(Zai))
                for j, a in enumerate(parts):
                    f.R[a] = Rcat[:, wc[j]:wc[j + 1]]
                    f.C[a] = Ccat[wr[j]:wr[j + 1], :]
                ledger["trsm"] += 4.0 * ri * ri * (wc[-1] + wr[-1])
                # all fill-in blocks of eq. 12 at once, then scattered to their blocks
                X = -(Ccat @ Rcat)
                ledger["gemm"] += 8.0 * wr[-1] * wc[-1] * ri
                for ja, a in enumerate(parts):
                    for jb, b in enumerate(parts):
                        Xab = X[wr[ja]:wr[ja + 1], wc[jb]:wc[jb + 1]]
                        if a == i and b == i:
                            Z[(i, i)][ri:, ri:] += Xab
                        elif a == i:
                            Z[(i, b)][ri:, :] += Xab
                        elif b == i:
                            Z[(a, i)][:, ri:] += Xab
                        elif (a, b) in nearset:
                            Z[(a, b)] += Xab
                        elif (a, b) in fills:
                            fills[(a, b)] += Xab
                        else:
                            fills[(a, b)] = Xab.copy()
            for i in grp:
                ri = facs[i].r
                for a in facs[i].partners:
                    if a == i:
                        Z[(i, i)] = Z[(i, i)][ri:, ri:]
                    else:
                        Z[(i, a)] = Z[(i, a)][ri:, :]
                        Z[(a, i)] = Z[(a, i)][:, ri:]
                r[i] = ri
                done[i] = True
        # coupling update at level l (eqs. 20-22, 33); merge to level l - 1 (Fig. 2 g-i)
        admset = set(S.adm[l])
        St = {}
        for (a, b) in S.adm[l]:
            M = np.zeros((kt[a], kt[b]), complex)
            C0 = H.coupling[l][(a, b)]
            M[:C0.shape[0], :C0.shape[1]] = C0
            if (a, b) in fills:
                M += fills[(a, b)]
            St[(a, b)] = M
        pl = l - 1
        npar = len(S.clusters[pl])
        n_par = np.zeros(npar, dtype=np.int64)
        off1 = np.zeros(npar, dtype=np.int64)
        for p in range(npar):
            off1[p] = kt[2 * p] if S.clusters[l][2 * p].size else 0
            n_par[p] = off1[p] + (kt[2 * p + 1] if S.clusters[l][2 * p + 1].size else 0)

        def place(dst, a, b, M):
            ra = 0 if a % 2 == 0 else off1[a // 2]
            cb = 0 if b % 2 == 0 else off1[b // 2]
            dst[ra:ra + M.shape[0], cb:cb + M.shape[1]] += M

        if pl >= ls:
            parent_pairs = S.near[pl]
        else:
            nz = [p for p in range(npar) if S.clusters[pl][p].size]
            parent_pairs = [(p, q) for p in nz for q in nz]
        Znew = {}
        for (p, q) in parent_pairs:
            Znew[(p, q)] = np.zeros((n_par[p], n_par[q]), complex)
        for (a, b), M in Z.items():
            place(Znew[(a // 2, b // 2)], a, b, M)
        for (a, b), M in St.items():
            place(Znew[(a // 2, b // 2)], a, b, M)
        fnew = {}
        for (a, b), M in fills.items():
            if (a, b) in admset:
                continue
            key = (a // 2, b // 2)
            if pl < ls:
                # the dense final block holds every pair: the carried fill lands there
                place(Znew[key], a, b, M)
                continue
            if key in Znew:
                raise AssertionError("ancestor-admissible fill under an inadmissible parent")
            if key not in fnew:
                fnew[key] = np.zeros((n_par[key[0]], n_par[key[1]]), complex)
            place(fnew[key], a, b, M)
        levels.append(dict(level=l, facs=facs, kt=kt.copy(), n=nsz.copy(), off1=off1,
                           n_par=n_par, groups=[g for g in groups]))
        if pl < ls and pl >= S.l0:
            _add_far_blocks(H, pl, l, n_par, off1, Znew)
        # parent bases: transfer matrices padded with zero rows (eq. 23)
        if pl >= ls:
            Bn = []
            for p in range(npar):
                if S.clusters[pl][p].size == 0:
                    Bn.append(np.zeros((0, 0), complex))
                    continue
                T = H.basis[pl][p]
                c1, c2 = 2 * p, 2 * p + 1
                k1 = H.rank[l][c1] if S.clusters[l][c1].size else 0
                k2 = H.rank[l][c2] if S.clusters[l][c2].size else 0
                M = np.zeros((n_par[p], T.shape[1]), complex)
                M[:k1] = T[:k1]
                M[off1[p]:off1[p] + k2] = T[k1:k1 + k2]
                Bn.append(M)
            B = Bn
            kk = H.rank[pl].copy()
            nu = H.nu[pl].copy()
        nsz = n_par
        Z = Znew
        fills = fnew
    # final dense block at level ls - 1 (Alg. 1, line 14)
    pl = ls - 1
    nz = [p for p in range(len(S.clusters[pl])) if S.clusters[pl][p].size]
    offs = {}
    o = 0
    for p in nz:
        offs[p] = o
        o += nsz[p]
    Zf = np.zeros((o, o), complex)
    for (p, q), M in Z.items():
        Zf[offs[p]:offs[p] + M.shape[0], offs[q]:offs[q] + M.shape[1]] = M
    if fills:
        raise AssertionError("fill-ins left outside the final block")
    ledger["lu"] += 8.0 / 3.0 * o ** 3
    return Factorization(H, levels, _lu(Zf), o, order, ledger, stats)


def _add_far_blocks(H, pl, l, n_par, off1, Znew):
    """Early stop: the blocks of level-pl pairs that are admissible at pl or at an
    ancestor level l' (eqs. 2-3) in the merged coordinates of level pl:
    B_p E_p S_{p'q'} E_q^T B_q^T, with B_p the padded transfer matrix (eq. 23) and
    E_p the product of the transfer-matrix rows along the path from p up to p'."""
    S = H.S
    near = set(S.near[pl])
    adm = [set(S.adm[m]) for m in range(S.L + 1)]
    nz = [p for p in range(len(S.clusters[pl])) if S.clusters[pl][p].size]
    Bp = {}
    for p in nz:
        T = H.basis[pl][p]
        k1 = H.rank[l][2 * p] if S.clusters[l][2 * p].size else 0
        k2 = H.rank[l][2 * p + 1] if S.clusters[l][2 * p + 1].size else 0
        M = np.zeros((n_par[p], T.shape[1]), complex)
        M[:k1] = T[:k1]
        M[off1[p]:off1[p] + k2] = T[k1:k1 + k2]
        Bp[p] = M

    def expanded(p, lev):
        """B_p E_p: the columns of the level-lev ancestor's basis, restricted to p."""
        X = Bp[p]
        c = p
        for m in range(pl, lev, -1):
            par = c // 2
            k_first = H.rank[m][2 * par] if S.clusters[m][2 * par].size else 0
            rows = slice(0, H.rank[m][c]) if c % 2 == 0 else slice(k_first, k_first + H.rank[m][c])
            X = X @ H.basis[m - 1][par][rows]
            c = par
        return X

    for p in nz:
        for q in nz:
            if (p, q) in near:
                continue
            for lev in range(pl, S.l0 - 1, -1):
                pa, qa = p >> (pl - lev), q >> (pl - lev)
                if (pa, qa) in adm[lev]:
                    Znew[(p, q)] += expanded(p, lev) @ H.coupling[lev][(pa, qa)] @ expanded(q, lev).T
                    break
            else:
                raise AssertionError("pair covered by no admissible block")


# --------------------------------------------------------------------------
# Solve (Sec. IV, Algs. 5-6) and its adjoint
# --------------------------------------------------------------------------


def _leaf_segments(Fz, v):
    S = Fz.H.S
    vt = v[S.perm]
    return [vt[S.start[S.L][t]:S.start[S.L][t] + S.clusters[S.L][t].size].copy()
            for t in range(len(S.clusters[S.L]))]


def _from_leaf_segments(Fz, segs, like):
    S = Fz.H.S
    out = np.zeros_like(like)
    out[S.perm] = np.concatenate(segs) if segs else np.zeros(0, complex)
    return out


def _cur_slice(lev, a, processed):
    """Current coordinates of cluster a's vector segment (kept part once processed)."""
    f = lev["facs"][a]
    return slice(f.r, None) if processed else slice(0, None)


def _colour_of(Fz, l):
    return Fz.H.S.colour[l]


def _before(Fz, l, a, i):
    """True if cluster a was eliminated before cluster i at level l."""
    col = _colour_of(Fz, l)
    if Fz.order_mode == "sequential":
        return (col[a], a) < (col[i], i)
    return col[a] < col[i]


def _merge_up(lev, segs):
    """P_l: parent vector = [kept(c1); kept(c2)]."""
    npar = len(lev["n_par"])
    out = []
    for p in range(npar):
        parts = []
        for c in (2 * p, 2 * p + 1):
            f = lev["facs"][c]
            if f is not None:
                parts.append(segs[c][f.r:])
        out.append(np.concatenate(parts) if parts else np.zeros(0, complex))
    return out


def _scatter_down(lev, psegs, segs):
    """P_l^T: children kept parts from the parent vector."""
    for p in range(len(lev["n_par"])):
        o = 0
        for c in (2 * p, 2 * p + 1):
            f = lev["facs"][c]
            if f is not None:
                segs[c][f.r:] = psegs[p][o:o + f.kt]
                o += f.kt


def _final_concat(Fz, segs):
    return np.concatenate([s for s in segs if s.size]) if segs else np.zeros(0, complex)


def _final_split(Fz, v, segs):
    o = 0
    for p in range(len(segs)):
        m = segs[p].size
        segs[p] = v[o:o + m].copy()
        o += m


def _solve_z(Fz, b):
    """y = Z^-1 b in the product form: Alg. 5 then Alg. 6 (eqs. 37, 41)."""
    S = Fz.H.S
    if not Fz.levels:
        lu, piv = Fz.final_lu
        bt = b[S.perm]
        y = sla.lu_solve((lu, piv), bt)
        out = np.zeros_like(b)
        out[S.perm] = y
        return out
    segs = _leaf_segments(Fz, b)
    saved = []
    for lev in Fz.levels:
        l = lev["level"]
        facs = lev["facs"]
        for grp in lev["groups"]:
            grp = [i for i in grp if facs[i] is not None]
            for i in grp:
                segs[i] = facs[i].Q.conj().T @ segs[i]
            for i in grp:
                f = facs[i]
                segs[i][:f.r] = _tri(f.lu, _pivot_apply(f.piv, segs[i][:f.r]), True, True)
            for i in grp:
                f = facs[i]
                yi = segs[i][:f.r]
                for a in f.partners:
                    if a == i:
                        segs[i][f.r:] -= f.C[a] @ yi
                    else:
                        sl = _cur_slice(lev, a, _before(Fz, l, a, i))
                        segs[a][sl] -= f.C[a] @ yi
        saved.append([s.copy() for s in segs])
        segs = _merge_up(lev, segs)
    lu, piv = Fz.final_lu
    yf = sla.lu_solve((lu, piv), _final_concat(Fz, segs))
    _final_split(Fz, yf, segs)
    for j in range(len(Fz.levels) - 1, -1, -1):
        lev = Fz.levels[j]
        l = lev["level"]
        facs = lev["facs"]
        child = saved[j]
        _scatter_down(lev, segs, child)
        segs = child
        for grp in reversed(lev["groups"]):
            grp = [i for i in grp if facs[i] is not None]
            for i in grp:
                f = facs[i]
                acc = segs[i][:f.r].copy()
                for a in f.partners:
                    if a == i:
                        acc -= f.R[a] @ segs[i][f.r:]
                    else:
                        sl = _cur_slice(lev, a, _before(Fz, l, a, i))
                        acc -= f.R[a] @ segs[a][sl]
                segs[i][:f.r] = _tri(f.lu, acc, False)
            for i in grp:
                segs[i] = facs[i].Q.conj() @ segs[i]
    return _from_leaf_segments(Fz, segs, b)


def _solve_z_adjoint(Fz, g):
    """lambda = Z^-H g: the conjugate transpose of the sweeps, applied in reverse."""
    S = Fz.H.S
    if not Fz.levels:
        lu, piv = Fz.final_lu
        y = sla.lu_solve((lu, piv), g[S.perm], trans=2)
        out = np.zeros_like(g)
        out[S.perm] = y
        return out
    segs = _leaf_segments(Fz, g)
    saved = []
    # U^-H: leaf to root, colours ascending; per colour Q^T then U_c^-H
    for lev in Fz.levels:
        l = lev["level"]
        facs = lev["facs"]
        for grp in lev["groups"]:
            grp = [i for i in grp if facs[i] is not None]
            for i in grp:
                segs[i] = facs[i].Q.T @ segs[i]
            for i in grp:
                f = facs[i]
                gi = _tri(f.lu, segs[i][:f.r], False, trans="C")
                segs[i][:f.r] = gi
                for a in f.partners:
                    if a == i:
                        segs[i][f.r:] -= f.R[a].conj().T @ gi
                    else:
                        sl = _cur_slice(lev, a, _before(Fz, l, a, i))
                        segs[a][sl] -= f.R[a].conj().T @ gi
        saved.append([s.copy() for s in segs])
        segs = _merge_up(lev, segs)
    lu, piv = Fz.final_lu
    yf = sla.lu_solve((lu, piv), _final_concat(Fz, segs), trans=2)
    _final_split(Fz, yf, segs)
    # L^-H: root to leaf, colours descending; per colour L_c^-H then Q
    for j in range(len(Fz.levels) - 1, -1, -1):
        lev = Fz.levels[j]
        l = lev["level"]
        facs = lev["facs"]
        child = saved[j]
        _scatter_down(lev, segs, child)
        segs = child
        for grp in reversed(lev["groups"]):
            grp = [i for i in grp if facs[i] is not None]
            for i in grp:
                f = facs[i]
                acc = segs[i][:f.r].copy()
                for a in f.partners:
                    if a == i:
                        acc -= f.C[a].conj().T @ segs[i][f.r:]
                    else:
                        sl = _cur_slice(lev, a, _before(Fz, l, a, i))
                        acc -= f.C[a].conj().T @ segs[a][sl]
                w = _tri(f.lu, acc, True, True, trans="C")
                segs[i][:f.r] = _pivot_apply_T(f.piv, w)
            for i in grp:
                segs[i] = facs[i].Q @ segs[i]
    return _from_leaf_segments(Fz, segs, g)


def _columns(fn, Fz, b):
    b = np.asarray(b, complex)
    if b.ndim == 1:
        return fn(Fz, b)
    return np.stack([fn(Fz, b[:, j]) for j in range(b.shape[1])], axis=1)


def solve(Fz, b):
    """x = M^-1 b for the user matrix A = Z D: y = Z^-1 b, x = D^-1 y (R1)."""
    D = d_scale(Fz.H)
    y = _columns(_solve_z, Fz, b)
    return y / (D if y.ndim == 1 else D[:, None])


def solve_adjoint(Fz, g):
    """lambda = M^-H g = Z^-H D^-1 g (D is real)."""
    D = d_scale(Fz.H)
    g = np.asarray(g, complex)
    return _columns(_solve_z_adjoint, Fz, g / (D if g.ndim == 1 else D[:, None]))


def refine(Fz, b, tol=1e-8, max_iter=20):
    """Iterative refinement x += M^-1 (b - A_H2 x) until ||b - A_H2 x|| <= tol ||b||."""
    b = np.asarray(b, complex)
    x = solve(Fz, b)
    nb = np.linalg.norm(b)
    hist = []
    for it in range(max_iter + 1):
        res = b - h2_matvec(Fz.H, x)
        rel = np.linalg.norm(res) / nb
        hist.append(rel)
        if rel <= tol or it == max_iter:
            break
        x = x + solve(Fz, res)
    return x, hist


def contrast_gradient(Fz, x, gx):
    """Gradients of a real loss through x = A^-1 b: (dL/db, dL/dchi).

    With lambda = A^-H gx (gx the loss gradient w.r.t. x in the conjugate
    convention), dL/db = lambda and, because column j of A depends on chi_j
    as chi_j (k^2 h^3 G_:j + c e_j) + e_j,
    dL/dchi_j = Re(conj(lambda_j) x_j - conj(gx_j) x_j) / chi_j.
    """
    lam = solve_adjoint(Fz, gx)
    chi = Fz.H.chi
    if x.ndim == 1:
        gchi = np.real(np.conj(lam) * x - np.conj(gx) * x) / chi
    else:
        gchi = (np.real(np.conj(lam) * x - np.conj(gx) * x) / chi[:, None]).sum(1)
    return lam, gchi


# --------------------------------------------------------------------------
# Bookkeeping: ranks per level and factor storage
# --------------------------------------------------------------------------


def rank_table(Fz):
    """Per level: list of (cluster, n, k, k~, r) for nonempty clusters."""
    out = {}
    for lev in Fz.levels:
        rows = []
        for i, f in enumerate(lev["facs"]):
            if f is not None:
                rows.append((i, f.n, f.k, f.kt, f.r))
        out[lev["level"]] = rows
    return out


def forced_from(Fz):
    """(level, cluster) -> k~ taken from a factorization (for rank-pinned runs)."""
    return {(lev["level"], i): f.kt for lev in Fz.levels for i, f in enumerate(lev["facs"])
            if f is not None}


def forced_construction(H):
    """(level, cluster) -> k taken from a construction."""
    S = H.S
    lmin = S.l0 if S.l0 is not None else S.L + 1
    return {(l, t): int(H.rank[l][t]) for l in range(lmin, S.L + 1)
            for t in range(len(S.clusters[l])) if S.clusters[l][t].size}


def factor_storage(Fz):
    """Complex entries held by the factors (Q~, LU of F, L and U panels, final LU)."""
    tot = 0
    for lev in Fz.levels:
        for f in lev["facs"]:
            if f is None:
                continue
            tot += f.Q.size + f.r * f.r
            tot += sum(v.size for v in f.C.values()) + sum(v.size for v in f.R.values())
    return tot + Fz.final_n ** 2


def h2_storage(H):
    """Complex entries of the H^2 representation (near blocks, bases, transfers, couplings)."""
    tot = sum(v.size for v in H.near_blocks.values())
    for l in range(len(H.basis)):
        for B in H.basis[l]:
            if B is not None:
                tot += B.size
        tot += sum(v.size for v in H.coupling[l].values())
    return tot
