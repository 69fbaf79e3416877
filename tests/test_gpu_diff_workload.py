"""The differentiation workload: a 48^3 cube grid (N = 110592, h = lambda/10,
contrast U[0.5, 1.5] seed 0), leaf 32, eta 1, eps 1e-6.

Loss L = sum_o |E_s(r_o) - E_t(r_o)|^2 over 256 observation points on a sphere
of radius twice the box edge around the box centre (Fibonacci lattice), with
E_s(r_o) = sum_j k^2 chi_j h^3 G(r_o, c_j) x_j from the solution x = A^-1 b and
E_t the same field for a second contrast (seed 1).  dL/dchi and dL/db come
from torch.autograd through the H^2 solve (the adjoint sweeps, both solves
refined).  They are checked against central finite differences of the refined
H^2 solve on 32 seeded cells (seed 2; the contrast is changed through
h2_set_contrast, ranks pinned to the base factorization so that both sides of
a difference use the same rank profile), and, on the 16^3 grid (N = 4096,
leaf 32, eps 1e-6), against the gradient of a dense FP64 adjoint solve."""
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


def _observation_kernel(pr, nobs=256):
    """G(r_o, c_j) from every cell to nobs points on the sphere of radius twice the box edge."""
    lo, hi = pr.points.min(0) - pr.h / 2, pr.points.max(0) + pr.h / 2
    obs = I.fibonacci_sphere(nobs, (lo + hi) / 2, 2.0 * float(np.max(hi - lo)))
    r = np.linalg.norm(obs[:, None, :] - pr.points[None, :, :], axis=2)
    return np.exp(-1j * pr.k * r) / (4 * np.pi * r)


def _field(torch, Gobs_t, chi_t, x, k2h3):
    return Gobs_t @ (k2h3 * chi_t.to(torch.complex128) * x)


def test_differentiation_workload_against_central_differences(capsys):
    import time
    torch = _torch()

    def _log(msg):
        # progress straight to the terminal: the whole test runs for minutes
        with capsys.disabled():
            print(f"[48^3 gradient] {msg}", flush=True)

    from paper_1703_06155_amd.autograd import h2_solve
    t0 = time.perf_counter()
    pr = I.config(4)
    k2h3 = pr.k ** 2 * pr.h ** 3
    tol = 1e-13
    Gobs_t = torch.from_numpy(_observation_kernel(pr)).cuda()
    b = torch.from_numpy(pr.rhs[:, 0].copy()).cuda()
    chi_t_target = I.contrast(pr.n, seed=1)
    _log(f"observation kernel ready ({time.perf_counter() - t0:.1f} s)")
    G = h2.H2(pr.points, pr.k, pr.h, chi_t_target, pr.leaf, pr.eta, pr.eps)
    _log(f"built ({time.perf_counter() - t0:.1f} s)")
    G.factor()
    _log(f"factored, stats {G.stats()[:, [0, 3, 7]].tolist()} ({time.perf_counter() - t0:.1f} s)")
    Et = _field(torch, Gobs_t, torch.from_numpy(chi_t_target).cuda(), G.solve(b, tol=tol, max_iter=30), k2h3)
    _log(f"target field ({time.perf_counter() - t0:.1f} s)")
    G.set_contrast(pr.chi).factor()
    ranks = G.forced_ranks()
    G.close()
    G = h2.H2(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps, forced_ranks=ranks).factor()
    _log(f"pinned handle factored ({time.perf_counter() - t0:.1f} s)")
    b_t = b.clone().requires_grad_(True)
    chi_t = torch.from_numpy(pr.chi.copy()).cuda().requires_grad_(True)
    x = h2_solve(b_t, chi_t, G, tol, 30)
    L = (_field(torch, Gobs_t, chi_t, x, k2h3) - Et).abs().pow(2).sum()
    L.backward()
    grad = chi_t.grad.cpu().numpy()
    assert np.all(np.isfinite(grad)) and np.all(np.isfinite(b_t.grad.cpu().numpy()))

    def loss_at(chi):
        G.set_contrast(chi).factor()
        xx = G.solve(b, tol=tol, max_iter=30)
        return (_field(torch, Gobs_t, torch.from_numpy(chi).cuda(), xx, k2h3) - Et).abs().pow(2).sum().item()

    cells = np.random.default_rng(2).choice(pr.n, 32, replace=False)
    errs = []
    for j in cells:
        d = 1e-6 * pr.chi[j]
        cp, cm = pr.chi.copy(), pr.chi.copy()
        cp[j] += d
        cm[j] -= d
        fd = (loss_at(cp) - loss_at(cm)) / (2 * d)
        errs.append((int(j), fd, float(grad[j])))
        _log(f"cell {j}: FD {fd:.6e}, adjoint {grad[j]:.6e} ({time.perf_counter() - t0:.1f} s)")
    scale = max(abs(g) for _, _, g in errs)
    worst = max(abs(fd - g) for _, fd, g in errs) / scale
    print(f"48^3 eps 1e-6: L = {L.item():.6e}, FD vs adjoint on 32 cells: max |diff| / max |grad| = {worst:.2e}")
    assert worst <= 1e-4, errs

    # dL/db: directional derivative along a seeded direction by central differences
    G.set_contrast(pr.chi).factor()
    rng = np.random.default_rng(3)
    v = torch.from_numpy(rng.standard_normal(pr.n) + 1j * rng.standard_normal(pr.n)).cuda()
    chi_c = torch.from_numpy(pr.chi).cuda()

    def loss_b(bb):
        xx = G.solve(bb, tol=tol, max_iter=30)
        return (_field(torch, Gobs_t, chi_c, xx, k2h3) - Et).abs().pow(2).sum().item()

    t = 1e-6 * torch.linalg.vector_norm(b).item() / torch.linalg.vector_norm(v).item()
    fd_b = (loss_b(b + t * v) - loss_b(b - t * v)) / (2 * t)
    # L is real and b complex: PyTorch's gradient is 2 dL/d conj(b), so dL along v is Re <grad, v>
    ad_b = torch.real(torch.vdot(b_t.grad, v)).item()
    G.close()
    assert abs(fd_b - ad_b) <= 1e-5 * abs(ad_b), (fd_b, ad_b)


def test_small_workload_gradient_against_dense_fp64_adjoint():
    """16^3 (N = 4096), leaf 32, eps 1e-6: the adjoint gradient through the refined
    H^2 solve against x = A^-1 b and lambda = A^-H g from dense FP64 LAPACK solves."""
    torch = _torch()
    from paper_1703_06155_amd.autograd import h2_solve
    pr = I.config(0)
    k2h3 = pr.k ** 2 * pr.h ** 3
    Gobs = _observation_kernel(pr)
    Et = np.random.default_rng(1).standard_normal(256) + 1j * np.random.default_rng(2).standard_normal(256)
    b = pr.rhs[:, 0]
    # dense FP64 reference
    A = O.dense_A(pr.points, pr.k, pr.h, pr.chi)
    x_ref = np.linalg.solve(A, b)
    res = Gobs @ (k2h3 * pr.chi * x_ref) - Et
    L_ref = float(np.sum(np.abs(res) ** 2))
    w = 2.0 * k2h3 * (Gobs.conj().T @ res)
    gx = pr.chi * w
    lam = np.linalg.solve(A.conj().T, gx)
    gchi_ref = np.real(np.conj(lam - gx) * x_ref) / pr.chi + np.real(np.conj(w) * x_ref)
    # GPU
    G = h2.H2(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps).factor()
    b_t = torch.from_numpy(b.copy()).cuda().requires_grad_(True)
    chi_t = torch.from_numpy(pr.chi.copy()).cuda().requires_grad_(True)
    x = h2_solve(b_t, chi_t, G, 1e-12, 20)
    L = (_field(torch, torch.from_numpy(Gobs).cuda(), chi_t, x, k2h3) - torch.from_numpy(Et).cuda()).abs().pow(2).sum()
    L.backward()
    e_L = abs(L.item() - L_ref) / L_ref
    e_b = np.linalg.norm(b_t.grad.cpu().numpy() - lam) / np.linalg.norm(lam)
    e_chi = np.linalg.norm(chi_t.grad.cpu().numpy() - gchi_ref) / np.linalg.norm(gchi_ref)
    print(f"16^3 eps 1e-6 vs dense FP64 adjoint: loss {e_L:.1e}, dL/db {e_b:.1e}, dL/dchi {e_chi:.1e}")
    G.close()
    assert e_L < 1e-5 and e_b < 1e-4 and e_chi < 1e-4
