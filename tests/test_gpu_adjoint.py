"""Differentiable solve (adjoint) on the GPU against the oracle gradient and central
finite differences."""
import dataclasses

import numpy as np
import pytest
import torch

import gen
import oracle

pytestmark = pytest.mark.gpu


def _mods():
    from paper_1205_6113_amd import adjoint
    return adjoint


def _problem(scale):
    return gen.scaled_config(5, scale) if scale < 1.0 else gen.config5()


def _loss_fn(p, dev):
    obs = torch.as_tensor(p.meta["obs"], device=dev)
    d = torch.as_tensor(p.meta["d"], device=dev)

    def loss(x):
        r = x[obs] - d
        return 0.5 * (r * r).sum()
    return loss


def test_tpfa_values_match_generator():
    adj = _mods()
    p = gen.scaled_config(5, 0.2)
    nx, ny, nz = p.dims
    grid = adj.TpfaGrid(nx, ny, nz, p.kz_ratio, p.dirichlet_x)
    assert np.array_equal(grid.row_ptr, p.row_ptr) and np.array_equal(grid.col, p.col)
    val = grid.values(torch.as_tensor(p.logk.ravel(), device="cuda")).cpu().numpy()
    assert np.max(np.abs(val - p.val) / np.abs(p.val).max()) <= 1e-14


@pytest.mark.parametrize("scale", [0.25])
def test_gradient_matches_oracle_and_fd(scale):
    adj = _mods()
    p = _problem(scale)
    dev = torch.device("cuda")
    nx, ny, nz = p.dims
    grid = adj.TpfaGrid(nx, ny, nz, p.kz_ratio, p.dirichlet_x)
    logk = torch.as_tensor(p.logk.ravel(), device=dev).requires_grad_(True)
    b = torch.as_tensor(p.b, device=dev).requires_grad_(True)
    loss_fn = _loss_fn(p, dev)
    x = adj.tpfa_solve(logk, b, grid, tol=1e-12)
    L = loss_fn(x)
    L.backward()
    g_logk = logk.grad.cpu().numpy()
    g_b = b.grad.cpu().numpy()
    # oracle gradient (its own TPFA chain rule) at the same tolerance
    h = oracle.Hierarchy(p.n, p.row_ptr, p.col, p.val)
    ref = oracle.misfit_gradient(p, h, tol=1e-12)
    assert abs(L.item() - ref["loss"]) <= 1e-9 * abs(ref["loss"])
    eb = np.linalg.norm(g_b - ref["grad_b"]) / np.linalg.norm(ref["grad_b"])
    ek = np.linalg.norm(g_logk - ref["grad_logk"]) / np.linalg.norm(ref["grad_logk"])
    assert eb <= 1e-8 and ek <= 1e-8, (eb, ek)
    # central finite differences with the preconditioner frozen at log k
    fz = adj.FrozenPreconditionerSolve(logk.detach(), grid)
    hstep = 1e-6
    gmax = np.abs(g_logk).max()
    for c in p.meta["fd_cells"][:5]:
        vals = []
        for sgn in (1.0, -1.0):
            lk = logk.detach().clone()
            lk[int(c)] += sgn * hstep
            xs, it, rel, st = fz.solve(lk, b.detach(), tol=1e-13)
            assert st == 0
            vals.append(loss_fn(xs).item())
        g_fd = (vals[0] - vals[1]) / (2 * hstep)
        assert abs(g_fd - g_logk[c]) <= 1e-5 * max(abs(g_logk[c]), 1e-3 * gmax), (int(c), g_fd, g_logk[c])
    # dL/db: L is quadratic in b, so the central difference is exact up to solve error
    for c in range(3):
        vals = []
        for sgn in (1.0, -1.0):
            bb = b.detach().clone()
            bb[c] += sgn * 1e-3
            xs, _, _, _ = fz.solve(logk.detach(), bb, tol=1e-13)
            vals.append(loss_fn(xs).item())
        g_fd = (vals[0] - vals[1]) / 2e-3
        assert abs(g_fd - g_b[c]) <= 1e-6 * max(abs(g_b[c]), 1e-3 * np.abs(g_b).max())
    fz.close()


def test_gradient_with_reused_setup():
    """A sequence of differentiable solves at log k0 + small steps, all with the
    preconditioner set up once at log k0: each loss and gradient equals that of a fresh
    setup at its own log k (the oracle's at the last step) to the solve tolerance."""
    adj = _mods()
    p = _problem(0.25)
    dev = torch.device("cuda")
    nx, ny, nz = p.dims
    grid = adj.TpfaGrid(nx, ny, nz, p.kz_ratio, p.dirichlet_x)
    lk0 = torch.as_tensor(p.logk.ravel(), device=dev)
    b = torch.as_tensor(p.b, device=dev)
    loss_fn = _loss_fn(p, dev)
    fz = adj.FrozenPreconditionerSolve(lk0, grid)
    rng = np.random.default_rng(11)
    try:
        for step in range(3):
            dlk = torch.as_tensor(0.02 * (step + 1) * rng.standard_normal(p.n), device=dev)
            lk_r = (lk0 + dlk).requires_grad_(True)
            L_r = loss_fn(adj.tpfa_solve(lk_r, b, grid, tol=1e-12, setup=fz))
            L_r.backward()
            lk_f = (lk0 + dlk).requires_grad_(True)
            L_f = loss_fn(adj.tpfa_solve(lk_f, b, grid, tol=1e-12))
            L_f.backward()
            assert abs(L_r.item() - L_f.item()) <= 1e-9 * abs(L_f.item())
            gr, gf = lk_r.grad.cpu().numpy(), lk_f.grad.cpu().numpy()
            assert np.linalg.norm(gr - gf) <= 1e-8 * np.linalg.norm(gf), step
        # the last step against the oracle's gradient at that log k (matrix from the generator)
        lk = (lk0 + dlk).cpu().numpy().reshape(p.logk.shape)
        rp, ci, val, keep = gen.tpfa_system(lk, p.kz_ratio, p.dirichlet_x)
        assert np.array_equal(rp, p.row_ptr) and np.array_equal(ci, p.col)
        q = dataclasses.replace(p, logk=lk, val=val)
        ref = oracle.misfit_gradient(q, oracle.Hierarchy(q.n, q.row_ptr, q.col, q.val), tol=1e-12)
        assert abs(L_r.item() - ref["loss"]) <= 1e-9 * abs(ref["loss"])
        assert np.linalg.norm(gr - ref["grad_logk"]) <= 1e-8 * np.linalg.norm(ref["grad_logk"])
    finally:
        fz.close()


def test_reused_setup_rejects_another_grid():
    adj = _mods()
    dev = torch.device("cuda")
    g1 = adj.TpfaGrid(4, 4, 2)
    g2 = adj.TpfaGrid(4, 4, 2)
    lk = torch.zeros(g1.n, device=dev, dtype=torch.float64)
    fz = adj.FrozenPreconditionerSolve(lk, g1)
    try:
        with pytest.raises(ValueError):
            adj.tpfa_solve(lk, torch.ones(g1.n, device=dev, dtype=torch.float64), g2, setup=fz)
    finally:
        fz.close()


def test_two_cell_closed_form():
    """1-D two cells between Dirichlet faces: x = A^{-1} b with the harmonic face
    transmissibility; dL/dlog k from the adjoint equals the analytic derivative."""
    adj = _mods()
    dev = torch.device("cuda")
    grid = adj.TpfaGrid(2, 1, 1, 1.0, True)
    lk0 = np.array([0.3, -0.7])

    def solve_np(lk):
        k = np.exp(lk)
        T = 2 * k[0] * k[1] / (k[0] + k[1])
        A = np.array([[T + 2 * k[0], -T], [-T, T + 2 * k[1]]])
        return np.linalg.solve(A, np.array([1.0, 2.0]))

    def L_np(lk):
        x = solve_np(lk)
        return 0.5 * (x[1] - 0.25) ** 2

    logk = torch.tensor(lk0, device=dev, dtype=torch.float64, requires_grad=True)
    b = torch.tensor([1.0, 2.0], device=dev, dtype=torch.float64)
    x = adj.tpfa_solve(logk, b, grid, tol=1e-14)
    L = 0.5 * (x[1] - 0.25) ** 2
    L.backward()
    eps = 1e-6
    g_ref = np.array([(L_np(lk0 + eps * e) - L_np(lk0 - eps * e)) / (2 * eps) for e in np.eye(2)])
    assert np.allclose(logk.grad.cpu().numpy(), g_ref, rtol=1e-7, atol=1e-12)
    assert np.allclose(x.detach().cpu().numpy(), solve_np(lk0), rtol=1e-13)


def test_c5_full_size_gradient():
    """The differentiable workload at full size (96 x 96 x 48, 442,368 unknowns, 200
    observation cells): the adjoint gradient against the oracle's gradient (relative
    l2 <= 1e-8, both with solves to 1e-12) and against central differences at
    h = 1e-6 on the workload's 20 check cells (solves to 1e-13 with the preconditioner
    frozen at log k), each within 1e-5 max(|g|, 1e-3 ||g||_inf)."""
    adj = _mods()
    p = gen.config5()
    print(f"[case] c5 full size n={p.n}", flush=True)
    dev = torch.device("cuda")
    nx, ny, nz = p.dims
    grid = adj.TpfaGrid(nx, ny, nz, p.kz_ratio, p.dirichlet_x)
    logk = torch.as_tensor(p.logk.ravel(), device=dev).requires_grad_(True)
    b = torch.as_tensor(p.b, device=dev).requires_grad_(True)
    loss_fn = _loss_fn(p, dev)
    x = adj.tpfa_solve(logk, b, grid, tol=1e-12)
    L = loss_fn(x)
    L.backward()
    g_logk = logk.grad.cpu().numpy()
    g_b = b.grad.cpu().numpy()
    h = oracle.Hierarchy(p.n, p.row_ptr, p.col, p.val)
    ref = oracle.misfit_gradient(p, h, tol=1e-12)
    assert abs(L.item() - ref["loss"]) <= 1e-9 * abs(ref["loss"])
    eb = np.linalg.norm(g_b - ref["grad_b"]) / np.linalg.norm(ref["grad_b"])
    ek = np.linalg.norm(g_logk - ref["grad_logk"]) / np.linalg.norm(ref["grad_logk"])
    print(f"[case] c5 gradient vs oracle: b {eb:.2e} logk {ek:.2e}", flush=True)
    assert eb <= 1e-8 and ek <= 1e-8, (eb, ek)
    fz = adj.FrozenPreconditionerSolve(logk.detach(), grid)
    try:
        hstep = 1e-6
        gmax = np.abs(g_logk).max()
        cells = p.meta["fd_cells"]
        assert len(cells) == 20
        worst = 0.0
        for c in cells:
            vals = []
            for sgn in (1.0, -1.0):
                lk = logk.detach().clone()
                lk[int(c)] += sgn * hstep
                xs, it, rel, st = fz.solve(lk, b.detach(), tol=1e-13)
                assert st == 0
                vals.append(loss_fn(xs).item())
            g_fd = (vals[0] - vals[1]) / (2 * hstep)
            bar = max(abs(g_logk[c]), 1e-3 * gmax)
            worst = max(worst, abs(g_fd - g_logk[c]) / bar)
            assert abs(g_fd - g_logk[c]) <= 1e-5 * bar, (int(c), g_fd, g_logk[c])
        print(f"[case] c5 central differences: worst {worst:.2e} of the per-cell bar", flush=True)
    finally:
        fz.close()
