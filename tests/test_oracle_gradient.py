"""Pins of the oracle's misfit gradient (the differentiable form) on the CPU.

The oracle computes dL/db and dL/dlog k of L = 1/2 ||x[obs] - d||^2 with
A(log k) x = b by an adjoint solve and a face-by-face chain rule
(`oracle.misfit_gradient`, `oracle.tpfa_logk_gradient`). These tests check it
against what does not share that code path:

* a two-cell problem whose derivative is written out by hand (forward
  sensitivity dx = -A^{-1} (dA/dlog k) x with the closed-form derivative of the
  harmonic transmissibility, dense 2 x 2 algebra);
* central finite differences of L with dense direct solves of the generator's
  matrix (no oracle solve, no oracle chain rule), on small grids with kz/kx != 1,
  Dirichlet x-faces and eliminated well columns;
* dL/db = lambda against central differences in b (L is quadratic in b, so the
  difference is exact up to rounding).
"""
import numpy as np
import pytest

import gen
import oracle


def _problem(logk, kz_ratio, dirichlet_x, wells, obs, d, b_seed=21):
    """A Problem for the misfit gradient, assembled by the generator only."""
    logk = np.asarray(logk, dtype=np.float64)
    if logk.ndim == 2:
        logk = logk[None]
    rp, ci, v, keep = gen.tpfa_system(logk, kz_ratio, dirichlet_x, wells)
    n = rp.size - 1
    nz, ny, nx = logk.shape
    b = np.random.default_rng(b_seed).standard_normal(n)
    p = gen.Problem(name="pin", n=n, row_ptr=rp, col=ci, val=v, b=b, tol=1e-12, dims=(nx, ny, nz),
                    logk=logk, kz_ratio=kz_ratio, dirichlet_x=dirichlet_x,
                    keep=None if keep.size == nx * ny * nz else keep)
    p.meta["obs"] = np.asarray(obs, dtype=np.int64)
    p.meta["d"] = np.asarray(d, dtype=np.float64)
    return p


def _dense_loss(logk, kz_ratio, dirichlet_x, wells, obs_cells, d, b):
    """L(log k, b) with a dense LAPACK solve of the generator's matrix."""
    rp, ci, v, keep = gen.tpfa_system(logk, kz_ratio, dirichlet_x, wells)
    n = rp.size - 1
    x = np.linalg.solve(gen.csr_to_dense(n, rp, ci, v), b)
    unk = np.full(np.asarray(logk).size, -1, dtype=np.int64)
    unk[keep] = np.arange(n)
    r = x[unk[obs_cells]] - d
    return 0.5 * float(r @ r)


def test_two_cell_gradient_closed_form():
    """Two cells in a row between Dirichlet faces (x = 0 and x = 2): a_00 = T + 2 k_0,
    a_11 = T + 2 k_1, a_01 = -T with T = 2 k_0 k_1 / (k_0 + k_1). By hand,
    dT/dlog k_0 = 2 k_0 k_1^2 / (k_0 + k_1)^2 and d(2 k_0)/dlog k_0 = 2 k_0 (mirror for
    cell 1); the forward sensitivity dx/dlog k_c = -A^{-1} (dA/dlog k_c) x gives
    dL/dlog k_c = (x_1 - d) (dx/dlog k_c)_1 for L = 1/2 (x_1 - d)^2."""
    lk = np.array([0.3, -0.7])
    k0, k1 = np.exp(lk)
    T = 2 * k0 * k1 / (k0 + k1)
    A = np.array([[T + 2 * k0, -T], [-T, T + 2 * k1]])
    b = np.array([1.0, 2.0])
    d = 0.25
    x = np.linalg.solve(A, b)
    dT0 = 2 * k0 * k1 * k1 / (k0 + k1) ** 2
    dT1 = 2 * k1 * k0 * k0 / (k0 + k1) ** 2
    dA0 = np.array([[dT0 + 2 * k0, -dT0], [-dT0, dT0]])
    dA1 = np.array([[dT1, -dT1], [-dT1, dT1 + 2 * k1]])
    g_ref = np.array([(x[1] - d) * (-np.linalg.solve(A, dA @ x))[1] for dA in (dA0, dA1)])
    # dL/db by hand: (x_1 - d) * (A^{-1})_{1,:} (A symmetric)
    gb_ref = (x[1] - d) * np.linalg.inv(A)[1]

    p = _problem(lk.reshape(1, 1, 2), 1.0, True, (), obs=[1], d=[d])
    p.b = b
    h = oracle.Hierarchy(p.n, p.row_ptr, p.col, p.val)
    out = oracle.misfit_gradient(p, h, tol=1e-15)
    assert np.allclose(out["x"], x, rtol=1e-14, atol=0)
    assert np.allclose(out["grad_logk"], g_ref, rtol=1e-12, atol=1e-15), (out["grad_logk"], g_ref)
    assert np.allclose(out["grad_b"], gb_ref, rtol=1e-12, atol=1e-15)


CASES = [
    # (nx, ny, nz, kz_ratio, dirichlet_x, wells)
    (7, 6, 4, 0.3, True, ()),               # anisotropic z faces, Dirichlet x-faces
    (6, 6, 3, 2.5, False, ((1, 1), (4, 3))),  # no-flow box with two eliminated well columns
    (9, 7, 1, 1.0, True, ()),               # one layer (no z faces)
]


@pytest.mark.parametrize("case", CASES, ids=["aniso-dirichlet", "wells", "one-layer"])
def test_logk_gradient_vs_central_differences(case):
    nx, ny, nz, kz, dirx, wells = case
    rng = np.random.default_rng(31 + nx)
    logk = 1.5 * gen.correlated_field((nz, ny, nx), 2.0, rng) if nz > 1 else \
        1.5 * gen.correlated_field((ny, nx), 2.0, rng)[None]
    N = nx * ny * nz
    idx = np.arange(N)
    removed = np.zeros(N, dtype=bool)
    for (wi, wj) in wells:
        removed |= (idx % nx == wi) & ((idx // nx) % ny == wj)
    kept = np.nonzero(~removed)[0]
    obs = np.sort(np.random.default_rng(41).choice(kept, size=min(12, kept.size), replace=False))
    d = np.random.default_rng(42).standard_normal(obs.size)
    p = _problem(logk, kz, dirx, wells, obs, d)
    h = oracle.Hierarchy(p.n, p.row_ptr, p.col, p.val)
    out = oracle.misfit_gradient(p, h, tol=1e-14)
    g = out["grad_logk"]
    # loss agrees with a dense solve
    L0 = _dense_loss(logk, kz, dirx, wells, obs, d, p.b)
    assert abs(out["loss"] - L0) <= 1e-11 * abs(L0)
    hstep = 1e-5
    gmax = np.abs(g).max()
    cells = np.random.default_rng(43).choice(kept, size=min(10, kept.size), replace=False)
    # eliminated (p = 0) cells have no unknown, but their permeability still sets the
    # transmissibility added to the neighbours' diagonals
    cells = np.concatenate([cells, np.nonzero(removed)[0][:4]])
    for c in cells:
        vals = []
        for sgn in (1.0, -1.0):
            lk = logk.copy().reshape(-1)
            lk[c] += sgn * hstep
            vals.append(_dense_loss(lk.reshape(logk.shape), kz, dirx, wells, obs, d, p.b))
        g_fd = (vals[0] - vals[1]) / (2 * hstep)
        assert abs(g_fd - g[c]) <= 1e-7 * max(abs(g[c]), 1e-2 * gmax), (int(c), g_fd, g[c])


def test_b_gradient_is_adjoint_vs_central_differences():
    nx, ny, nz = 6, 5, 3
    logk = 1.0 * gen.correlated_field((nz, ny, nx), 2.0, np.random.default_rng(51))
    obs = np.sort(np.random.default_rng(52).choice(nx * ny * nz, size=10, replace=False))
    d = np.random.default_rng(53).standard_normal(obs.size)
    p = _problem(logk, 0.5, True, (), obs, d)
    h = oracle.Hierarchy(p.n, p.row_ptr, p.col, p.val)
    out = oracle.misfit_gradient(p, h, tol=1e-14)
    gb = out["grad_b"]
    step = 1e-3
    for c in range(0, p.n, 7):
        vals = []
        for sgn in (1.0, -1.0):
            bb = p.b.copy()
            bb[c] += sgn * step
            vals.append(_dense_loss(logk, 0.5, True, (), obs, d, bb))
        g_fd = (vals[0] - vals[1]) / (2 * step)
        assert abs(g_fd - gb[c]) <= 1e-9 * max(abs(gb[c]), 1e-3 * np.abs(gb).max()), (c, g_fd, gb[c])


def test_zero_misfit_has_zero_gradient():
    """A perfect fit (d = x[obs]) is a minimum of L: loss and gradient vanish."""
    nx, ny, nz = 5, 4, 2
    logk = np.zeros((nz, ny, nx))
    p = _problem(logk, 1.0, True, (), obs=[7, 12], d=[0.0, 0.0])
    h = oracle.Hierarchy(p.n, p.row_ptr, p.col, p.val)
    x = h.pcg(oracle.PREC_COMBINED, p.b, 1e-14, 1000)["x"]
    p.meta["d"] = x[[7, 12]].copy()
    out = oracle.misfit_gradient(p, h, tol=1e-14)
    assert out["loss"] <= 1e-25
    assert np.abs(out["grad_logk"]).max() <= 1e-12 and np.abs(out["grad_b"]).max() <= 1e-12
