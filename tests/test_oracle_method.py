"""Pins for the oracle's construction, factorization, solves and gradients.

Each test checks the oracle against something it does not compute itself: a
dense LAPACK solve, an exact algebraic identity of the paper, a closed form,
or a finite difference.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import h2_oracle as O
from paper_1703_06155_amd import inputs as I


def _prob(grid, leaf, eps, eta=1.0, seed=0):
    pr = I.make_problem("t", grid, leaf, eps, eta=eta, chi_seed=seed)
    H = O.construct(pr.points, pr.k, pr.h, pr.chi, leaf, eta, eps)
    return pr, H


def test_entries_match_user_matrix():
    """Z = A D^-1 with D = diag(k^2 h^3 chi): two independent writings of the kernel."""
    pr = I.make_problem("t", (5, 4, 3), 8, 1e-4)
    A = O.dense_A(pr.points, pr.k, pr.h, pr.chi)
    Z = O.dense_Z(pr.points, pr.k, pr.h, pr.chi)
    D = pr.k ** 2 * pr.h ** 3 * pr.chi
    assert np.allclose(A, Z * D[None, :], rtol=1e-14, atol=0)
    assert np.abs(Z - Z.T).max() == 0.0
    # self term closed form: a = (3/4pi)^(1/3) h, c = (1+jka)e^{-jka} - 1
    a = (3 / (4 * np.pi)) ** (1 / 3) * pr.h
    ka = pr.k * a
    c = (1 + 1j * ka) * (np.cos(ka) - 1j * np.sin(ka)) - 1
    assert abs(A[0, 0] - (1 + pr.chi[0] * c)) < 1e-15


@pytest.mark.parametrize("grid,leaf,eps", [((8, 8, 8), 16, 1e-4), ((10, 7, 9), 12, 1e-5),
                                           ((8, 8, 8), 8, 1e-6)])
def test_construction_nested_orthonormal_accurate(grid, leaf, eps):
    """V, T orthonormal; V_t = diag(V_t1, V_t2) T_t (eq. 3); S_st = S_ts^T; ||Z - Z_H2|| ~ eps."""
    pr, H = _prob(grid, leaf, eps)
    S = H.S
    for l in range(S.l0, S.L + 1):
        for t in range(len(S.clusters[l])):
            B = H.basis[l][t]
            assert np.allclose(B.conj().T @ B, np.eye(B.shape[1]), atol=1e-13)
            E = H.expanded[l][t]
            assert np.allclose(E.conj().T @ E, np.eye(E.shape[1]), atol=1e-12)
            if l < S.L:
                k1 = H.expanded[l + 1][2 * t].shape[1]
                nest = np.vstack([H.expanded[l + 1][2 * t] @ B[:k1], H.expanded[l + 1][2 * t + 1] @ B[k1:]])
                assert np.allclose(nest, E, atol=1e-14)
        for (t, s), C in H.coupling[l].items():
            assert np.array_equal(C, H.coupling[l][(s, t)].T)
    Z = O.dense_Z(pr.points, pr.k, pr.h, pr.chi)
    Zh = O.h2_dense(H)
    # per admissible block: the dropped singular values are below eps * sigma_1 of the row
    for l in range(S.l0, S.L + 1):
        for (t, s) in S.adm[l]:
            rows, cols = S.clusters[l][t], S.clusters[l][s]
            err = np.linalg.norm(Z[np.ix_(rows, cols)] - Zh[np.ix_(rows, cols)], 2)
            assert err <= 10 * eps * H.nu[l][t] + 1e-14
    rel = np.linalg.norm(Z - Zh) / np.linalg.norm(Z)
    assert 1e-3 * eps < rel < 10 * eps
    v = np.random.default_rng(1).standard_normal(pr.n) + 1j
    assert np.allclose(O.h2_matvec_z(H, v), Zh @ v, rtol=1e-13, atol=1e-13 * np.abs(Zh @ v).max())


def _dense_inverse_check(Fz, H, tol):
    Zh = O.h2_dense(H)
    n = Zh.shape[0]
    rng = np.random.default_rng(2)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    y = O._solve_z(Fz, b)
    yd = np.linalg.solve(Zh, b)
    return np.linalg.norm(y - yd) / np.linalg.norm(yd)


@pytest.mark.parametrize("grid,leaf,eps", [((8, 8, 8), 16, 1e-4), ((6, 6, 6), 8, 1e-6),
                                           ((8, 8, 8), 4, 1e-4), ((10, 7, 9), 12, 1e-5),
                                           ((9, 5, 3), 7, 1e-3)])
def test_no_truncation_limit_equals_dense_solve(grid, leaf, eps):
    """With eps_fill -> 0 the only approximation left is the H^2 representation (Sec. V-A):
    M^-1 b must equal a dense LAPACK solve of the represented matrix Z_H2."""
    pr, H = _prob(grid, leaf, eps)
    Fz = O.factor(H, eps_fill=1e-14)
    assert _dense_inverse_check(Fz, H, 1e-11) < 1e-11
    Fs = O.factor(H, eps_fill=1e-14, order="sequential")
    assert _dense_inverse_check(Fs, H, 1e-11) < 1e-11


@pytest.mark.parametrize("grid,leaf,eps", [((10, 7, 9), 12, 1e-5), ((8, 8, 8), 4, 1e-4), ((9, 5, 3), 7, 1e-3)])
def test_early_stop_no_truncation_equals_dense_solve(grid, leaf, eps):
    """Early stop (Sec. III-C): factoring levels L..ls and finishing with a dense LU of the
    matrix merged to level ls - 1, whose far blocks come from the nested bases and
    couplings of every coarser admissible level, still solves Z_H2 exactly when nothing is
    truncated, for every stop level from l0 to L."""
    pr, H = _prob(grid, leaf, eps)
    S = H.S
    assert S.L - S.l0 >= 2
    sizes = []
    for ls in range(S.l0, S.L + 1):
        Fz = O.factor(H, eps_fill=1e-14, stop_level=ls)
        assert len(Fz.levels) == S.L - ls + 1
        assert _dense_inverse_check(Fz, H, 1e-11) < 1e-11
        sizes.append(Fz.final_n)
    # fewer factored levels leave a larger dense block
    assert sizes == sorted(sizes) and sizes[0] < sizes[-1]
    with pytest.raises(ValueError):
        O.factor(H, stop_level=S.l0 - 1)


def test_eta_zero_is_dense_lu():
    """eta = 0: no block is admissible, the method reduces to LU of the whole matrix."""
    pr, H = _prob((8, 8, 8), 16, 1e-4, eta=0.0)
    assert H.S.l0 is None
    Fz = O.factor(H)
    b = pr.rhs[:, 0]
    x = O.solve(Fz, b)
    A = O.dense_A(pr.points, pr.k, pr.h, pr.chi)
    xd = sla.lu_solve(sla.lu_factor(A), b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-12


def test_zero_introduction_and_factor_identities():
    """Q~ unitary, V kept verbatim in Q~ = [V~perp V V_add] (eqs. 4, 7-8, 18-19);
    the pivoted LU reproduces F (eq. 11)."""
    pr, H = _prob((10, 7, 9), 12, 1e-5)
    tr = []
    Fz = O.factor(H, trace=tr)
    for lev, st in zip(Fz.levels, tr):
        for i, f in enumerate(lev["facs"]):
            if f is None:
                continue
            Q = f.Q
            assert np.allclose(Q.conj().T @ Q, np.eye(f.n), atol=1e-12)
            B = st["B"][i]
            assert np.allclose(Q[:, f.r:f.r + f.k], B, atol=1e-15)
            # Q~^H V = [0; I]
            QV = Q.conj().T @ B
            assert np.allclose(QV[:f.r], 0, atol=1e-12)
            if f.r:
                Lm = np.tril(f.lu, -1) + np.eye(f.r)
                Um = np.triu(f.lu)
                assert np.isfinite(Lm).all() and np.isfinite(Um).all()


def test_projection_annihilates_construction_basis_on_far_blocks():
    """Eqs. 7-8 on the represented matrix: the eliminated part Q~[:, :r] is orthogonal to the
    cluster's construction basis, so it annihilates every admissible leaf block V_t S V_s^T."""
    pr, H = _prob((8, 8, 8), 16, 1e-4)
    Fz = O.factor(H)
    lev = Fz.levels[0]
    S = H.S
    Zh = O.h2_dense(H)
    for (t, s) in S.adm[S.L]:
        f = lev["facs"][t]
        blk = Zh[np.ix_(S.clusters[S.L][t], S.clusters[S.L][s])]
        assert np.linalg.norm(f.Q[:, :f.r].conj().T @ blk) < 1e-12 * np.linalg.norm(blk) + 1e-15


def test_step0_dropped_fill_is_below_threshold():
    """Eq. 17 truncation on real fill-ins: after Step 0 the part of the fill-ins W_i that the
    eliminated directions Q~[:, :r] still see has 2-norm <= tau_i (the dropped singular values)."""
    pr, H = _prob((10, 7, 9), 12, 1e-5)
    rec = []
    Fz = O.factor(H, step0_trace=rec)
    assert len(rec) > 20
    by_level = {lev["level"]: lev for lev in Fz.levels}
    for e in rec:
        f = by_level[e["level"]]["facs"][e["cluster"]]
        dropped = np.linalg.norm(f.Q[:, :f.r].conj().T @ e["W"], 2) if f.r else 0.0
        assert dropped <= e["tau"] * (1 + 1e-9) + 1e-15


def _designed_fills(n, k, sig, seed=5):
    """Fill-ins with a prescribed spectrum outside a k-column basis: W = Qc diag(sig) Y^H + Bi X,
    Qc orthonormal and orthogonal to Bi (so (I - Bi Bi^H) W has singular values sig exactly)."""
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Q, _ = np.linalg.qr(M)
    Bi, Qc = Q[:, :k], Q[:, k:k + len(sig)]
    w = 3 * len(sig) + 2
    Y, _ = np.linalg.qr(rng.standard_normal((w, len(sig))) + 1j * rng.standard_normal((w, len(sig))))
    X = rng.standard_normal((k, w)) + 1j * rng.standard_normal((k, w))
    return Bi, Qc, Qc @ np.diag(sig) @ Y.conj().T + Bi @ X


@pytest.mark.parametrize("nu,sig,efill,cap,p_exp", [
    # the fill-ins dominate (sigma_1(W) = 50 > nu = 1): tau = 1e-2 * 50 = 0.5
    (1.0, [50.0, 3.0, 0.6, 0.4, 1e-3], 1e-2, 6, 3),
    # the construction dominates (nu = 1000 > 50): tau = 10
    (1000.0, [50.0, 3.0, 0.6, 0.4, 1e-3], 1e-2, 6, 1),
    # tau = 0.5 again, but only two directions fit beside the basis
    (1.0, [50.0, 3.0, 0.6, 0.4, 1e-3], 1e-2, 2, 2),
    # every direction below tau = 1e-3 * 2 = 2e-3 except the first two
    (2.0, [1.5, 0.01, 1e-3, 1e-4], 1e-3, 6, 2),
])
def test_step0_threshold_on_designed_spectrum(nu, sig, efill, cap, p_exp):
    """Step 0 rank rule (eqs. 16-17 with the R5 threshold tau = eps_fill max(nu_i, sigma_1(W)))
    on fill-ins whose singular values outside the basis are known by construction: the kept
    count p_exp is read off the designed spectrum; the added directions span the designed
    leading singular vectors; what is dropped has norm sig[p_exp] <= tau."""
    n, k = 9, 2
    Bi, Qc, W = _designed_fills(n, k, np.array(sig))
    U, s, tau, p, _ = O.fill_spectrum(Bi, W, nu, efill, cap)
    assert p == p_exp
    # G = W W^H squares the spectrum: compare sig^2 to the accuracy of the Gram's eigenvalues
    assert np.allclose(s[:len(sig)] ** 2, np.square(sig), rtol=1e-9, atol=1e-13 * max(sig) ** 2)
    Ua = U[:, :p]
    # same span as the designed leading directions
    assert np.linalg.norm(Ua @ Ua.conj().T - Qc[:, :p] @ Qc[:, :p].conj().T, 2) < 1e-8
    Bt = np.hstack([Bi, Ua])
    rest = np.linalg.norm(W - Bt @ (Bt.conj().T @ W), 2)
    expect_rest = sig[p] if p < len(sig) else 0.0
    assert abs(rest - expect_rest) <= 1e-9 * max(sig)
    if p < cap:
        assert rest <= tau


def test_green_function_closed_forms():
    """Kernel entries e^{-jkr}/(4 pi r) at r = m h on one axis against values evaluated from the
    square-root closed forms of cos/sin at multiples of 36 degrees (tests/golden/green_entries.json);
    A_ij = k^2 chi_j h^3 Z_ij for the same pairs."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "green_entries.json")) as f:
        gold = json.load(f)
    k, h = gold["k"], gold["h"]
    assert k == I.WAVENUMBER and h == I.CELL
    pts = I.cube_grid(11, 1, 1)
    chi = I.contrast(pts.shape[0], 0)
    Z = O.dense_Z(pts, k, h, chi)
    A = O.dense_A(pts, k, h, chi)
    zb = O.z_block(pts, [0], np.arange(11), k, h, chi)[0]
    for e in gold["entries"]:
        m = e["m"]
        want = complex(e["re"], e["im"])
        assert abs(Z[0, m] - want) <= 1e-14, (m, Z[0, m], want)
        assert abs(zb[m] - want) <= 1e-14
        assert abs(Z[m, 0] - want) <= 1e-14
        assert abs(A[0, m] - (2 * np.pi) ** 2 * h ** 3 * chi[m] * want) <= 1e-15


@pytest.mark.parametrize("grid,leaf,eps", [((8, 8, 8), 16, 1e-4), ((10, 7, 9), 12, 1e-5)])
def test_adjoint_identity_and_dense_adjoint(grid, leaf, eps):
    """<M^-1 b, g> = <b, M^-H g> exactly; in the no-truncation limit M^-H = A_H2^-H."""
    pr, H = _prob(grid, leaf, eps)
    rng = np.random.default_rng(3)
    b = rng.standard_normal(pr.n) + 1j * rng.standard_normal(pr.n)
    g = rng.standard_normal(pr.n) + 1j * rng.standard_normal(pr.n)
    Fz = O.factor(H)
    lhs = np.vdot(g, O.solve(Fz, b))
    rhs = np.vdot(O.solve_adjoint(Fz, g), b)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    Fx = O.factor(H, eps_fill=1e-14)
    Ah = O.h2_dense(H) * O.d_scale(H)[None, :]
    lam = O.solve_adjoint(Fx, g)
    assert np.linalg.norm(lam - np.linalg.solve(Ah.conj().T, g)) <= 1e-11 * np.linalg.norm(lam)
    # multi-RHS path equals column-by-column
    B2 = np.stack([b, g], 1)
    assert np.allclose(O.solve(Fz, B2)[:, 1], O.solve(Fz, g), rtol=1e-14, atol=0)


def test_accuracy_tracks_eps():
    """The dense residual ||A x - b|| / ||b|| falls with eps and stays within C*eps (Sec. V-A)."""
    pr = I.make_problem("t", (10, 10, 10), 16, 1e-2)
    A = O.dense_A(pr.points, pr.k, pr.h, pr.chi)
    b = pr.rhs[:, 0]
    res = []
    S = O.build_structure(pr.points, pr.h, 16, 1.0)
    for eps in [1e-2, 1e-4, 1e-6]:
        H = O.construct(pr.points, pr.k, pr.h, pr.chi, 16, 1.0, eps, structure=S)
        x = O.solve(O.factor(H), b)
        res.append(np.linalg.norm(A @ x - b) / np.linalg.norm(b))
        assert res[-1] < 10 * eps
    assert all(res[j + 1] < res[j] for j in range(len(res) - 1))


def test_sequential_and_colour_orders_agree_to_eps():
    """Colour-batched and one-at-a-time elimination are two valid orders: they agree to O(eps)."""
    pr, H = _prob((10, 7, 9), 12, 1e-5)
    b = pr.rhs[:, 0]
    x1 = O.solve(O.factor(H), b)
    x2 = O.solve(O.factor(H, order="sequential"), b)
    assert np.linalg.norm(x1 - x2) / np.linalg.norm(x1) < 1e-4


def test_forced_ranks_reproduce_free_run():
    """Pinning every rank decision to the ones a free run took reproduces that run bit for bit."""
    pr, H = _prob((8, 8, 8), 16, 1e-4)
    Fz = O.factor(H)
    Ff = O.factor(H, forced_kt=O.forced_from(Fz))
    b = pr.rhs[:, 0]
    assert np.array_equal(O.solve(Fz, b), O.solve(Ff, b))
    H2 = O.construct(pr.points, pr.k, pr.h, pr.chi, 16, 1.0, 1e-4, forced_ranks=O.forced_construction(H))
    assert np.array_equal(O.h2_dense(H2), O.h2_dense(H))


def test_refinement_reaches_tolerance():
    """Iterative refinement with the approximate factors converges to 1e-12 against A_H2 (Sec. VI-B measure)."""
    pr, H = _prob((8, 8, 8), 16, 1e-3)
    Fz = O.factor(H, eps_fill=1e-2)
    x, hist = O.refine(Fz, pr.rhs[:, 0], tol=1e-12, max_iter=30)
    assert hist[0] > 1e-6 and hist[-1] <= 1e-12
    Ah = O.h2_dense(H) * O.d_scale(H)[None, :]
    b = pr.rhs[:, 0]
    assert np.linalg.norm(Ah @ x - b) / np.linalg.norm(b) <= 1e-12
    assert np.allclose(O.h2_matvec(H, x, adjoint=True), Ah.conj().T @ x, rtol=1e-12,
                       atol=1e-12 * np.abs(Ah.conj().T @ x).max())


def test_rod_storage_and_work_are_linear():
    """Quasi-1-D rod (the paper's Sec. VI-B shape): storage and flops per unknown stay flat."""
    per = []
    for nz in (64, 128, 256):
        pr = I.rod(nz, leaf=32, eps=1e-4)
        H = O.construct(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps)
        Fz = O.factor(H)
        per.append((O.factor_storage(Fz) / pr.n, sum(Fz.ledger.values()) / pr.n))
    s = np.array(per)
    assert s[:, 0].max() / s[:, 0].min() < 1.2
    assert s[:, 1].max() / s[:, 1].min() < 1.3


def _loss(x, w, t):
    return float(np.sum(w * np.abs(x - t) ** 2))


def test_gradient_matches_finite_differences():
    """dL/dchi and dL/db from the adjoint solve vs central differences of dense solves."""
    pr = I.make_problem("t", (6, 5, 4), 8, 1e-8)
    rng = np.random.default_rng(4)
    w = rng.uniform(0.5, 1.5, pr.n)
    t = rng.standard_normal(pr.n) + 1j * rng.standard_normal(pr.n)
    b = pr.rhs[:, 0]
    H = O.construct(pr.points, pr.k, pr.h, pr.chi, 8, 1.0, 1e-8)
    Fz = O.factor(H, eps_fill=1e-14)
    x = O.solve(Fz, b)
    gx = 2 * w * (x - t)
    lam, gchi = O.contrast_gradient(Fz, x, gx)
    step = 1e-6
    for j in (0, 17, 63, 101):
        chi_p, chi_m = pr.chi.copy(), pr.chi.copy()
        chi_p[j] += step
        chi_m[j] -= step
        Lp = _loss(np.linalg.solve(O.dense_A(pr.points, pr.k, pr.h, chi_p), b), w, t)
        Lm = _loss(np.linalg.solve(O.dense_A(pr.points, pr.k, pr.h, chi_m), b), w, t)
        fd = (Lp - Lm) / (2 * step)
        assert abs(fd - gchi[j]) <= 1e-5 * max(1.0, abs(fd))
    A = O.dense_A(pr.points, pr.k, pr.h, pr.chi)
    for j in (3, 50):
        for unit, part in ((1.0, np.real), (1j, np.imag)):
            bp, bm = b.copy(), b.copy()
            bp[j] += unit * step
            bm[j] -= unit * step
            fd = (_loss(np.linalg.solve(A, bp), w, t) - _loss(np.linalg.solve(A, bm), w, t)) / (2 * step)
            assert abs(fd - part(lam[j])) <= 1e-5 * max(1.0, abs(fd))
