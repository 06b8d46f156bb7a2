"""Pins of the oracle against what the paper and the mathematics fix (CPU only).

Each test names the passage it follows. None of them re-types the oracle's own
formulas: they compare against textbook/library routines, closed forms,
invariants and theorems.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

import gen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tiny_problem(nx, ny, nz, seed, sigma=1.0, dirichlet=True, kz=1.0):
    rng = np.random.default_rng(seed)
    logk = sigma * rng.standard_normal((nz, ny, nx))
    rp, ci, v, _ = gen.tpfa_system(logk, kz, dirichlet)
    n = rp.size - 1
    return n, rp, ci, v, gen.csr_to_dense(n, rp, ci, v)


def random_spd_mmatrix(n, density, seed):
    """Random symmetric M-matrix: negative off-diagonals, strictly dominant diagonal."""
    rng = np.random.default_rng(seed)
    a = np.zeros((n, n))
    for i in range(n):
        for j in range(i + 1, n):
            if j == i + 1 or rng.random() < density:
                w = rng.uniform(0.1, 2.0)
                a[i, j] = a[j, i] = -w
    np.fill_diagonal(a, -a.sum(axis=1) + rng.uniform(0.01, 0.5, n))
    return a


def dense_to_csr(a):
    n = a.shape[0]
    rp = [0]
    ci = []
    v = []
    for i in range(n):
        nz = np.nonzero(a[i])[0]
        ci.extend(nz.tolist())
        v.extend(a[i, nz].tolist())
        rp.append(len(ci))
    return n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(v, np.float64)


# ---------------------------------------------------------------- PCG --------

@pytest.mark.parametrize("dims,seed", [((4, 4, 1), 11), ((8, 8, 1), 12), ((4, 4, 4), 13), ((6, 5, 3), 14)])
@pytest.mark.parametrize("which", [oracle.PREC_COMBINED, oracle.PREC_AMG, oracle.PREC_ILU,
                                   oracle.PREC_ADDITIVE, oracle.PREC_NONE])
def test_pcg_matches_cholesky_solve(dims, seed, which):
    """PCG with any SPD preconditioner converges to A^{-1} b (Section 2, Remark 2.2)."""
    n, rp, ci, v, A = tiny_problem(*dims, seed, sigma=1.0)
    h = oracle.Hierarchy(n, rp, ci, v, max_coarse=8)
    b = np.random.default_rng(seed + 100).standard_normal(n)
    c = sla.cho_factor(A, lower=True)
    x_ref = sla.cho_solve(c, b)
    r = h.pcg(which, b, 1e-14, 2000)
    assert r["status"] == oracle.OR_OK
    assert np.linalg.norm(r["x"] - x_ref) / np.linalg.norm(x_ref) <= 1e-10


def test_pcg_zero_rhs_and_tolerance_before_first_iteration():
    n, rp, ci, v, A = tiny_problem(5, 5, 1, 3)
    h = oracle.Hierarchy(n, rp, ci, v, max_coarse=4)
    r = h.pcg(oracle.PREC_COMBINED, np.zeros(n), 1e-8, 100)
    assert r["iters"] == 0 and r["status"] == oracle.OR_OK and not r["x"].any()
    b = np.ones(n)
    r = h.pcg(oracle.PREC_COMBINED, b, 1e-8, 100, x0=np.linalg.solve(A, b))
    assert r["iters"] == 0 and r["hist"][0] <= 1e-8


def test_pcg_maxit_reports_last_iterate():
    n, rp, ci, v, A = tiny_problem(8, 8, 1, 4, sigma=2.0)
    h = oracle.Hierarchy(n, rp, ci, v, max_coarse=4)
    b = np.random.default_rng(0).standard_normal(n)
    r = h.pcg(oracle.PREC_NONE, b, 1e-14, 3)
    assert r["status"] == oracle.OR_E_MAXIT and r["iters"] == 3
    assert r["hist"].size == 4 and np.all(np.isfinite(r["hist"]))
    # CG minimises the A-norm of the error over the Krylov space: it decreases
    x_ref = np.linalg.solve(A, b)
    errs = []
    for k in (1, 2, 3):
        xk = h.pcg(oracle.PREC_NONE, b, 1e-14, k)["x"]
        e = xk - x_ref
        errs.append(e @ A @ e)
    assert errs[0] > errs[1] > errs[2]
    assert np.array_equal(xk, r["x"])


# ---------------------------------------------------------------- ILU(0) -----

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_ilu0_tridiagonal_equals_exact_lu(seed):
    """ILU(0) of a tridiagonal matrix has no dropped fill, so it is the exact LU
    (Algorithm 3.1 with k = 0); compared with LAPACK's LU (no row exchanges occur
    for these diagonally dominant matrices)."""
    rng = np.random.default_rng(seed)
    n = 40
    off = -rng.uniform(0.5, 2.0, n - 1)
    d = np.zeros(n)
    d[:-1] -= off
    d[1:] -= off
    d += rng.uniform(0.0, 1.0, n)
    A = np.diag(d) + np.diag(off, 1) + np.diag(off, -1)
    n_, rp, ci, v = dense_to_csr(A)
    lu, st = oracle.ilu0(n, rp, ci, v)
    assert st == oracle.OR_OK
    P, L, U = sla.lu(A)
    assert np.array_equal(P, np.eye(n))
    LU = gen.csr_to_dense(n, rp, ci, lu)
    L_or = np.tril(LU, -1) + np.eye(n)
    U_or = np.triu(LU)
    assert np.max(np.abs(L_or - L)) <= 1e-15 * np.max(np.abs(L))
    assert np.max(np.abs(U_or - U)) <= 1e-15 * np.max(np.abs(U))


def test_ilu0_one_dimensional_tpfa_is_exact():
    n, rp, ci, v, A = tiny_problem(30, 1, 1, 5, sigma=1.5)
    lu, st = oracle.ilu0(n, rp, ci, v)
    LU = gen.csr_to_dense(n, rp, ci, lu)
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    assert np.max(np.abs(L @ U - A)) <= 1e-13 * np.max(np.abs(A))


@pytest.mark.parametrize("dims,seed", [((7, 6, 1), 1), ((5, 4, 3), 2), ((9, 9, 2), 3)])
def test_ilu0_defining_property(dims, seed):
    """(LU)_ij = a_ij on the pattern of A; positive pivots on an M-matrix;
    U = diag(U) L^T for symmetric A (the IC(0) form of Section 3.3)."""
    n, rp, ci, v, A = tiny_problem(*dims, seed, sigma=2.0)
    lu, st = oracle.ilu0(n, rp, ci, v)
    assert st == oracle.OR_OK
    LU = gen.csr_to_dense(n, rp, ci, lu)
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    prod = L @ U
    mask = A != 0
    assert np.max(np.abs(prod[mask] - A[mask])) <= 1e-13 * np.max(np.abs(A))
    assert (~mask & (np.abs(prod) > 1e-12)).any() or dims[1] == 1  # some fill was dropped
    assert np.all(np.diag(U) > 0)
    assert np.max(np.abs(U - np.diag(np.diag(U)) @ L.T)) <= 1e-12 * np.max(np.abs(U))


def _ilu1_fill_closed_form(nx, ny, nz):
    """Level-1 fill of ILU on the natural-order 5/7-point grid pattern, from grid
    coordinates: the pivot m = i - e_a (an earlier neighbour of i) carries its later
    neighbour j = m + e_b (b != a) into row i, so (i, i - e_a + e_b) has level 1
    (and (j, i) by symmetry of the argument)."""
    dims = [nx, ny, nz]
    strides = [1, nx, nx * ny]
    fill = set()
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                c = [x, y, z]
                i = x + nx * (y + ny * z)
                for a in range(3):
                    if c[a] < 1:
                        continue
                    for b in range(3):
                        if b == a or c[b] + 1 >= dims[b]:
                            continue
                        j = i - strides[a] + strides[b]
                        fill.add((i, j))
                        fill.add((j, i))
    return fill


@pytest.mark.parametrize("dims", [(7, 6, 1), (5, 4, 3)])
def test_iluk_level1_pattern_closed_form(dims):
    """ILU(1) (Algorithm 3.1, k = 1) keeps the pattern of A plus exactly the level-1
    fill of the grid stencil, derived above from coordinates; every entry's level is
    0 on the pattern of A and 1 on the fill."""
    n, rp, ci, v, A = tiny_problem(*dims, 31, sigma=1.0)
    h = oracle.Hierarchy(n, rp, ci, v, ilu_k=1)
    frp, fci, fv, lev = h.ilu_factor()
    got = {(i, int(j)): int(l) for i in range(n) for j, l in zip(fci[frp[i]:frp[i + 1]], lev[frp[i]:frp[i + 1]])}
    base = {(i, int(j)) for i in range(n) for j in ci[rp[i]:rp[i + 1]]}
    fill = _ilu1_fill_closed_form(*dims)
    assert set(got) == base | fill
    assert all(got[e] == 0 for e in base) and all(got[e] == 1 for e in fill - base)


def test_iluk_k0_is_ilu0_bitwise():
    """k = 0 keeps the pattern of A and reproduces ILU(0) bit for bit."""
    n, rp, ci, v, A = tiny_problem(6, 5, 3, 33, sigma=1.5)
    h = oracle.Hierarchy(n, rp, ci, v, ilu_k=0)
    frp, fci, fv, lev = h.ilu_factor()
    lu, st = oracle.ilu0(n, rp, ci, v)
    assert np.array_equal(frp, rp) and np.array_equal(fci, ci) and np.array_equal(fv, lu)
    assert not lev.any()


@pytest.mark.parametrize("k", [1, 2, 3])
def test_iluk_defining_property(k):
    """R = A - LU vanishes on the kept pattern (the ILU(k) condition of Section 3.1)."""
    n, rp, ci, v, A = tiny_problem(6, 5, 3, 34 + k, sigma=1.5)
    h = oracle.Hierarchy(n, rp, ci, v, ilu_k=k)
    frp, fci, fv, lev = h.ilu_factor()
    F = gen.csr_to_dense(n, frp, fci, fv)
    LU = (np.tril(F, -1) + np.eye(n)) @ np.triu(F)
    rows = np.repeat(np.arange(n), np.diff(frp))
    assert np.max(np.abs((LU - A)[rows, fci])) <= 1e-14 * np.max(np.abs(A))
    assert lev.max() <= k


def test_iluk_with_all_fill_is_exact_lu():
    """With k at least the largest level that occurs nothing is dropped: the factor
    is the exact LU (LAPACK, no row exchanges for this SPD M-matrix)."""
    n, rp, ci, v, A = tiny_problem(7, 6, 1, 36, sigma=1.0)
    h = oracle.Hierarchy(n, rp, ci, v, ilu_k=n)
    frp, fci, fv, lev = h.ilu_factor()
    F = gen.csr_to_dense(n, frp, fci, fv)
    P, L, U = sla.lu(A)
    assert np.array_equal(P, np.eye(n))
    assert np.max(np.abs(np.tril(F, -1) + np.eye(n) - L)) <= 1e-14
    assert np.max(np.abs(np.triu(F) - U)) <= 1e-14 * np.max(np.abs(U))


def test_iluk_combined_is_spd():
    """Theorem 2.1 with B = ILU(1): B_co stays symmetric positive definite."""
    n, rp, ci, v, A = tiny_problem(6, 6, 2, 37, sigma=2.0)
    h = oracle.Hierarchy(n, rp, ci, v, max_coarse=8, ilu_k=1)
    Bco = h.dense_operator(oracle.PREC_COMBINED)
    assert np.max(np.abs(Bco - Bco.T)) <= 1e-12 * np.max(np.abs(Bco))
    assert np.linalg.eigvalsh(0.5 * (Bco + Bco.T)).min() > 0


def test_ilu0_reports_nonpositive_pivot():
    A = np.array([[1.0, 2.0, 0.0], [2.0, 1.0, 0.5], [0.0, 0.5, 1.0]])  # indefinite
    n, rp, ci, v = dense_to_csr(A)
    _, st = oracle.ilu0(n, rp, ci, v)
    assert st == oracle.OR_E_NOT_SPD


# ---------------------------------------------------------------- RS AMG -----

def poisson_1d(n):
    A = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    return dense_to_csr(A)


def test_rs_1d_closed_form():
    """Classical coarsening + RS interpolation + Galerkin on tridiag(-1,2,-1)
    (Section 3.2), against the hand-derived fixture."""
    g = json.load(open(os.path.join(GOLDEN, "rs_1d_poisson.json")))
    n, rp, ci, v = poisson_1d(g["n"])
    h = oracle.Hierarchy(n, rp, ci, v, max_coarse=4)
    assert h.nlev >= 2
    assert h.cf(0).tolist() == g["cf"]
    prp, pci, pv = h.prolongation(0)
    rows = [[[int(pci[q]), float(pv[q])] for q in range(prp[i], prp[i + 1])] for i in range(n)]
    assert rows == g["p_rows"]
    crp, cci, cv = h.level(1)
    m = g["m"]
    Ac = gen.csr_to_dense(m, crp, cci, cv)
    expect = g["coarse_diag"] * np.eye(m) + g["coarse_offdiag"] * (np.eye(m, k=1) + np.eye(m, k=-1))
    assert np.array_equal(Ac, expect)


def _strength(A, theta=0.25):
    n = A.shape[0]
    S = []
    for i in range(n):
        off = [(-A[i, j]) for j in range(n) if j != i and A[i, j] != 0]
        mx = max(off) if off else 0.0
        S.append({j for j in range(n) if j != i and A[i, j] < 0 and -A[i, j] >= theta * mx})
    return S


@pytest.mark.parametrize("seed", range(6))
def test_rs_splitting_invariants(seed):
    """Properties any classical C/F splitting of this reading must have:
    (i) every F point with strong couplings has a strong C neighbour;
    (ii) every strong F-F pair (i, j) shares a C point of C_i among S_j (the
    second-pass guarantee); (iii) points without strong couplings are F."""
    rng = np.random.default_rng(seed)
    if seed % 2:
        A = random_spd_mmatrix(60, 0.08, seed)
    else:
        _, _, _, _, A = tiny_problem(7, 6, 2, seed, sigma=2.0, kz=0.1)
    n, rp, ci, v = dense_to_csr(A)
    cf, nc = oracle.rs_split(n, rp, ci, v)
    assert nc == int(cf.sum()) and 0 < nc < n
    S = _strength(A)
    for i in range(n):
        if not S[i]:
            assert cf[i] == 0
            continue
        if cf[i] == 1:
            continue
        Ci = {j for j in S[i] if cf[j] == 1}
        assert Ci, i
        for j in S[i]:
            if cf[j] == 0:
                assert S[j] & Ci, (i, j)
    del rng


def _grid(nx, ny, diag, couplings):
    """Dense matrix on an nx x ny grid: a_ii = diag, a_ij = -w for each (dx, dy, w)."""
    n = nx * ny
    a = np.zeros((n, n))
    for y in range(ny):
        for x in range(nx):
            i = x + nx * y
            a[i, i] = diag
            for dx, dy, w in couplings:
                for sx, sy in ((dx, dy), (-dx, -dy)):
                    if 0 <= x + sx < nx and 0 <= y + sy < ny:
                        a[i, x + sx + nx * (y + sy)] = -w
    return a


def _rs_2d_matrix(name):
    five = [(1, 0, 1.0), (0, 1, 1.0)]
    nine = five + [(1, 1, 1.0), (1, -1, 1.0)]
    if name == "five_point_3x3":
        return _grid(3, 3, 4.0, five)
    if name == "five_point_4x4":
        return _grid(4, 4, 4.0, five)
    if name == "nine_point_3x3":
        return _grid(3, 3, 8.0, nine)
    if name == "nine_point_5x5":
        return _grid(5, 5, 8.0, nine)
    if name == "anisotropic_5x3":
        return _grid(5, 3, 2.2, [(1, 0, 1.0), (0, 1, 0.1)])
    cpl = _RS_2D[name]["couplings"]
    n = 1 + max(max(i, j) for i, j, _ in cpl)
    a = np.zeros((n, n))
    for i, j, w in cpl:
        a[i, j] = a[j, i] = -w
    np.fill_diagonal(a, 1.0 - a.sum(axis=1))
    return a


_RS_2D = json.load(open(os.path.join(GOLDEN, "rs_2d_handworked.json")))["cases"]


@pytest.mark.parametrize("name", sorted(_RS_2D))
def test_rs_handworked_grids(name):
    """Classical splitting and interpolation (Section 3.2) on 2-D grids and on small
    graphs chosen so that a wrong tie-break, lambda counted over S_i instead of S_i^T,
    or a missing lambda update changes the splitting; against splittings and weights
    worked by hand (fixture tests/golden/rs_2d_handworked.json, derivations in it)."""
    g = _RS_2D[name]
    A = _rs_2d_matrix(name)
    n, rp, ci, v = dense_to_csr(A)
    cf, nc = oracle.rs_split(n, rp, ci, v)
    assert cf.tolist() == g["cf"], name
    h = oracle.Hierarchy(n, rp, ci, v, max_coarse=1, max_levels=2)
    assert h.nlev == 2 and h.cf(0).tolist() == g["cf"]
    prp, pci, pv = h.prolongation(0)
    if "p_rows" in g:
        for i in range(n):
            got = list(zip(pci[prp[i]:prp[i + 1]].tolist(), pv[prp[i]:prp[i + 1]].tolist()))
            want = [(c, w) for c, w in g["p_rows"][i]]
            assert [c for c, _ in got] == [c for c, _ in want], (name, i)
            assert np.allclose([w for _, w in got], [w for _, w in want], rtol=1e-14, atol=0), (name, i)
    if "p_weight_edge_rows" in g:
        nx = g["nx"]
        for i in range(n):
            if g["cf"][i]:
                continue
            y = i // nx
            want = g["p_weight_middle_row"] if y == 1 else g["p_weight_edge_rows"]
            for q in range(prp[i], prp[i + 1]):
                assert abs(pv[q] - want) <= 1e-14 * want, (name, i)
    if "coarse" in g:
        crp, cci, cv = h.level(1)
        m = crp.size - 1
        assert np.array_equal(gen.csr_to_dense(m, crp, cci, cv), np.array(g["coarse"]))


def test_rs_interpolation_preserves_constants_on_zero_row_sum():
    """Classical interpolation reproduces constants where the row sum of A is zero
    and every coupling is strong and negative (a_ii = -sum a_ij)."""
    n, rp, ci, v, A = tiny_problem(8, 8, 1, 7, sigma=0.3, dirichlet=False)
    A = A.copy()
    A[0, 0] += 1.0  # make it nonsingular at one corner only
    n, rp, ci, v = dense_to_csr(A)
    h = oracle.Hierarchy(n, rp, ci, v, max_coarse=4, theta=0.0)
    prp, pci, pv = h.prolongation(0)
    P = np.zeros((n, int(h.cf(0).sum())))
    for i in range(n):
        P[i, pci[prp[i]:prp[i + 1]]] = pv[prp[i]:prp[i + 1]]
    rs = A.sum(axis=1)
    ones = P @ np.ones(P.shape[1])
    for i in range(n):
        if abs(rs[i]) < 1e-12:
            assert abs(ones[i] - 1.0) <= 1e-12, i


def test_galerkin_is_ptap():
    """A_l = P_l^T A_{l+1} P_l (Section 3.2) checked against dense products."""
    n, rp, ci, v, A = tiny_problem(9, 8, 3, 21, sigma=1.5)
    h = oracle.Hierarchy(n, rp, ci, v, max_coarse=10)
    for d in range(h.nlev - 1):
        fn, _ = h.level_sizes()[d]
        cn, _ = h.level_sizes()[d + 1]
        Af = gen.csr_to_dense(fn, *h.level(d))
        prp, pci, pv = h.prolongation(d)
        P = gen.csr_to_dense(fn, prp, pci, pv)[:, :cn] if cn <= fn else None
        P = np.zeros((fn, cn))
        for i in range(fn):
            P[i, pci[prp[i]:prp[i + 1]]] = pv[prp[i]:prp[i + 1]]
        Ac = gen.csr_to_dense(cn, *h.level(d + 1))
        assert np.max(np.abs(Ac - P.T @ Af @ P)) <= 1e-13 * np.max(np.abs(Af))
        assert np.array_equal(Ac, Ac.T) or np.max(np.abs(Ac - Ac.T)) <= 1e-14 * np.max(np.abs(Ac))


# ---------------------------------------------------------------- V-cycle ----

def test_one_level_hierarchy_is_exact():
    """With n <= max_coarse the hierarchy is one level: B_0 = A_0^{-1} (Algorithm 3.2),
    so V = A^{-1}, B_co = A^{-1} and PCG needs one iteration."""
    n, rp, ci, v, A = tiny_problem(6, 6, 2, 31, sigma=2.0)
    h = oracle.Hierarchy(n, rp, ci, v, max_coarse=256)
    assert h.nlev == 1
    Ainv = np.linalg.inv(A)
    V = h.dense_operator(oracle.OP_VCYCLE)
    assert np.max(np.abs(V - Ainv)) <= 1e-12 * np.max(np.abs(Ainv))
    Bco = h.dense_operator(oracle.PREC_COMBINED)
    assert np.max(np.abs(Bco - Ainv)) <= 1e-11 * np.max(np.abs(Ainv))
    b = np.random.default_rng(1).standard_normal(n)
    r = h.pcg(oracle.PREC_COMBINED, b, 1e-10, 10)
    assert r["iters"] == 1
    chol = h.coarse_cholesky()
    assert np.max(np.abs(chol - np.linalg.cholesky(A))) <= 1e-13 * np.max(np.abs(chol))


@pytest.mark.parametrize("dims,seed", [((10, 10, 1), 41), ((6, 6, 5), 42)])
def test_vcycle_symmetric_and_contractive(dims, seed):
    """The V-cycle with forward GS before and backward GS after the coarse
    correction is symmetric, and ||I - V A||_A < 1 (Section 3.3)."""
    n, rp, ci, v, A = tiny_problem(*dims, seed, sigma=2.0)
    h = oracle.Hierarchy(n, rp, ci, v, max_coarse=12)
    assert h.nlev >= 3
    V = h.dense_operator(oracle.OP_VCYCLE)
    assert np.max(np.abs(V - V.T)) <= 1e-12 * np.max(np.abs(V))
    Lc = np.linalg.cholesky(A)
    E = np.eye(n) - V @ A
    # A-norm of E = 2-norm of Lc^T E Lc^{-T}
    M = Lc.T @ E @ np.linalg.inv(Lc.T)
    assert np.linalg.norm(M, 2) < 1.0
    # power iteration agrees
    x = np.random.default_rng(0).standard_normal(n)
    for _ in range(200):
        y = x - h.apply(oracle.OP_VCYCLE, A @ x)
        rho = math.sqrt((y @ A @ y) / (x @ A @ x))
        x = y / math.sqrt(y @ A @ y)
    assert rho < 1.0


def test_backward_gs_is_adjoint_of_forward_gs():
    n, rp, ci, v, A = tiny_problem(5, 4, 3, 51, sigma=1.0)
    h = oracle.Hierarchy(n, rp, ci, v, max_coarse=4)
    F = h.dense_operator(oracle.OP_FGS)
    B = h.dense_operator(oracle.OP_BGS)
    assert np.max(np.abs(F - np.linalg.inv(np.tril(A)))) <= 1e-13 * np.max(np.abs(F))
    assert np.max(np.abs(B - F.T)) <= 1e-13 * np.max(np.abs(F))


# ---------------------------------------------------------------- B_co -------

def _dense_parts(h, A, S_op, ST_op):
    S = h.dense_operator(S_op)
    ST = h.dense_operator(ST_op)
    B = h.dense_operator(oracle.PREC_ILU)
    return S, ST, B


@pytest.mark.parametrize("combo", ["vcycle", "gs"])
def test_error_propagator_eq22_and_explicit_eq23(combo):
    """eq. (2.2): I - B_co A = (I - S^T A)(I - B A)(I - S A);
    eq. (2.3): B_co = S~ + (I - S^T A) B (I - A S) with S~ = S + S^T - S^T A S.
    S^T is the transpose of the dense S (not the oracle's S^T operator)."""
    n, rp, ci, v, A = tiny_problem(6, 5, 2, 61, sigma=1.5)
    h = oracle.Hierarchy(n, rp, ci, v, max_coarse=8)
    if combo == "vcycle":
        S = h.dense_operator(oracle.OP_VCYCLE)
        Bco = h.dense_operator(oracle.PREC_COMBINED)
    else:
        S = h.dense_operator(oracle.OP_FGS)
        Bco = h.dense_operator(oracle.OP_COMBINED_GS)
    B = h.dense_operator(oracle.PREC_ILU)
    I = np.eye(n)
    lhs = I - Bco @ A
    rhs = (I - S.T @ A) @ (I - B @ A) @ (I - S @ A)
    assert np.max(np.abs(lhs - rhs)) <= 1e-12 * max(1.0, np.max(np.abs(lhs)))
    St = S + S.T - S.T @ A @ S
    rhs2 = St + (I - S.T @ A) @ B @ (I - A @ S)
    assert np.max(np.abs(Bco - rhs2)) <= 1e-12 * np.max(np.abs(Bco))
    # S~ with S = V-cycle is the two-cycle AMG(GS) comparator
    if combo == "vcycle":
        Samg = h.dense_operator(oracle.PREC_AMG)
        assert np.max(np.abs(Samg - St)) <= 1e-12 * np.max(np.abs(St))


@pytest.mark.parametrize("dims,seed", [((6, 6, 1), 71), ((4, 4, 4), 72), ((7, 5, 3), 73)])
def test_theorem_2_1_combined_is_spd(dims, seed):
    """Theorem 2.1 / Corollary 3.1: B_co is symmetric positive definite."""
    n, rp, ci, v, A = tiny_problem(*dims, seed, sigma=2.0)
    h = oracle.Hierarchy(n, rp, ci, v, max_coarse=6)
    Bco = h.dense_operator(oracle.PREC_COMBINED)
    assert np.max(np.abs(Bco - Bco.T)) <= 1e-12 * np.max(np.abs(Bco))
    assert np.linalg.eigvalsh(0.5 * (Bco + Bco.T)).min() > 0


def test_theorem_2_1_random_vectors_on_config1():
    """<B u, v> = <u, B v> and u^T B u > 0 for random vectors at a full config size."""
    p = gen.config1()
    h = oracle.Hierarchy(p.n, p.row_ptr, p.col, p.val)
    rng = np.random.default_rng(5)
    for _ in range(20):
        u = rng.standard_normal(p.n)
        w = rng.standard_normal(p.n)
        Bu = h.apply(oracle.PREC_COMBINED, u)
        Bw = h.apply(oracle.PREC_COMBINED, w)
        assert abs(Bu @ w - u @ Bw) <= 1e-12 * abs(Bu @ w) + 1e-12 * np.linalg.norm(Bu) * np.linalg.norm(w)
        assert u @ Bu > 0


def test_theorem_2_2_condition_bound():
    """Theorem 2.2 with B scaled so that m_1 > 1 >= m_0: kappa(B_co A) is below
    [(1-m_1)(1-rho)+m_1]/[(1-m_0)(1-rho)+m_0] and below kappa(B A)."""
    n, rp, ci, v, A = tiny_problem(6, 6, 2, 81, sigma=2.0)
    h1 = oracle.Hierarchy(n, rp, ci, v, max_coarse=8)
    B = h1.dense_operator(oracle.PREC_ILU)
    ev = np.sort(np.linalg.eigvals(B @ A).real)
    omega = 1.0 / ev[0]
    m0, m1 = omega * ev[0], omega * ev[-1]
    assert m1 > 1.0 >= m0 - 1e-12
    h = oracle.Hierarchy(n, rp, ci, v, max_coarse=8, b_scale=omega)
    Bco = h.dense_operator(oracle.PREC_COMBINED)
    St = h.dense_operator(oracle.PREC_AMG)
    rho = np.max(np.linalg.eigvals(np.eye(n) - St @ A).real)
    assert 0 <= rho < 1
    evc = np.sort(np.linalg.eigvals(Bco @ A).real)
    kappa = evc[-1] / evc[0]
    bound = ((1 - m1) * (1 - rho) + m1) / ((1 - m0) * (1 - rho) + m0)
    assert kappa <= bound * (1 + 1e-10)
    assert kappa < m1 / m0


def test_degenerate_components():
    """S = 0 makes Algorithm 2.1 the plain B step; B = 0 leaves the symmetrised
    smoother S~ = two V-cycles: identical PCG histories."""
    n, rp, ci, v, A = tiny_problem(8, 7, 2, 91, sigma=1.5)
    b = np.random.default_rng(3).standard_normal(n)
    h_s0 = oracle.Hierarchy(n, rp, ci, v, max_coarse=8, s_scale=0.0)
    h = oracle.Hierarchy(n, rp, ci, v, max_coarse=8)
    r0 = h_s0.pcg(oracle.PREC_COMBINED, b, 1e-10, 500)
    r1 = h.pcg(oracle.PREC_ILU, b, 1e-10, 500)
    assert r0["iters"] == r1["iters"]
    assert np.array_equal(r0["hist"], r1["hist"])
    h_b0 = oracle.Hierarchy(n, rp, ci, v, max_coarse=8, b_scale=0.0)
    r2 = h_b0.pcg(oracle.PREC_COMBINED, b, 1e-10, 500)
    r3 = h.pcg(oracle.PREC_AMG, b, 1e-10, 500)
    assert r2["iters"] == r3["iters"]
    assert np.allclose(r2["hist"], r3["hist"], rtol=1e-9, atol=0)


def test_additive_form_eq27():
    """B^ = S~ + B (eq. 2.7 with W_1 = V, A_1^{-1} = B) is SPD."""
    n, rp, ci, v, A = tiny_problem(5, 5, 3, 95, sigma=1.0)
    h = oracle.Hierarchy(n, rp, ci, v, max_coarse=8)
    Badd = h.dense_operator(oracle.PREC_ADDITIVE)
    St = h.dense_operator(oracle.PREC_AMG)
    B = h.dense_operator(oracle.PREC_ILU)
    assert np.max(np.abs(Badd - (St + B))) <= 1e-13 * np.max(np.abs(Badd))
    assert np.linalg.eigvalsh(0.5 * (Badd + Badd.T)).min() > 0


def test_swapped_roles_variant_is_spd_here():
    n, rp, ci, v, A = tiny_problem(5, 5, 2, 97, sigma=1.0)
    h = oracle.Hierarchy(n, rp, ci, v, max_coarse=8)
    Bs = h.dense_operator(oracle.OP_COMBINED_SWAP)
    assert np.max(np.abs(Bs - Bs.T)) <= 1e-11 * np.max(np.abs(Bs))


def test_amg_ilu_is_exact_where_ilu0_is():
    """AMG(ILU(0)) of Table 5.2 (ILU(0) as the finest-level smoother, two cycles):
    on a tridiagonal matrix ILU(0) is the exact LU, so the pre-smoothing already
    solves the system, the coarse correction and the post-smoothing add nothing and
    the operator is A^{-1} (compared with LAPACK's solve), on a hierarchy with
    several levels."""
    rng = np.random.default_rng(21)
    n = 300
    off = -rng.uniform(0.5, 2.0, n - 1)
    d = np.zeros(n)
    d[:-1] -= off
    d[1:] -= off
    d += rng.uniform(0.0, 0.2, n)
    A = np.diag(d) + np.diag(off, 1) + np.diag(off, -1)
    n_, rp, ci, v = dense_to_csr(A)
    h = oracle.Hierarchy(n, rp, ci, v, max_coarse=16)
    assert h.nlev >= 3
    f = rng.standard_normal(n)
    z = h.apply(oracle.PREC_AMG_ILU, f)
    x = sla.solve(A, f, assume_a="pos")
    assert np.linalg.norm(z - x) <= 1e-11 * np.linalg.norm(x)
    # the AMG(GS) comparator is not exact here: the pin separates the two smoothers
    zg = h.apply(oracle.PREC_AMG, f)
    assert np.linalg.norm(zg - x) > 1e-8 * np.linalg.norm(x)


@pytest.mark.parametrize("dims,seed", [((6, 6, 1), 71), ((4, 4, 4), 72)])
def test_amg_ilu_symmetric_positive_here(dims, seed):
    """With A symmetric, ILU(0) = L D L^T up to rounding, so AMG(ILU(0)) is
    symmetric; on these M-matrices ILU(0) converges and the operator is SPD."""
    n, rp, ci, v, A = tiny_problem(*dims, seed, sigma=2.0)
    h = oracle.Hierarchy(n, rp, ci, v, max_coarse=6)
    assert h.nlev >= 2
    V = h.dense_operator(oracle.PREC_AMG_ILU)
    assert np.max(np.abs(V - V.T)) <= 1e-12 * np.max(np.abs(V))
    assert np.linalg.eigvalsh(0.5 * (V + V.T)).min() > 0


@pytest.mark.parametrize("omega", [1.0, 8.0])
def test_bbar_error_propagator(omega):
    """Remark after Theorem 2.1: I - B-bar A = (I - BA)(I - S~A)(I - BA), here with
    B = omega * ILU(0) and S~ the two-cycle AMG(GS) operator, both as dense matrices
    taken from their own operators."""
    n, rp, ci, v, A = tiny_problem(6, 5, 2, 61, sigma=1.5)
    h1 = oracle.Hierarchy(n, rp, ci, v, max_coarse=8)
    B = omega * h1.dense_operator(oracle.PREC_ILU)
    St = h1.dense_operator(oracle.PREC_AMG)
    h = oracle.Hierarchy(n, rp, ci, v, max_coarse=8, b_scale=omega)
    Bb = h.dense_operator(oracle.PREC_BBAR)
    I = np.eye(n)
    lhs = I - Bb @ A
    rhs = (I - B @ A) @ (I - St @ A) @ (I - B @ A)
    assert np.max(np.abs(lhs - rhs)) <= 1e-11 * max(1.0, np.max(np.abs(lhs)))


def test_bbar_without_b_is_the_two_cycle_smoother():
    """B = 0 leaves I - B-bar A = I - S~A: B-bar is the AMG(GS) comparator, bitwise."""
    n, rp, ci, v, A = tiny_problem(8, 7, 2, 91, sigma=1.5)
    h0 = oracle.Hierarchy(n, rp, ci, v, max_coarse=8, b_scale=0.0)
    h = oracle.Hierarchy(n, rp, ci, v, max_coarse=8)
    rng = np.random.default_rng(4)
    for _ in range(3):
        r = rng.standard_normal(n)
        assert np.array_equal(h0.apply(oracle.PREC_BBAR, r), h.apply(oracle.PREC_AMG, r))


@pytest.mark.parametrize("dims,seed", [((6, 6, 1), 71), ((8, 7, 2), 91), ((12, 12, 2), 5)])
def test_bbar_loses_definiteness_where_bco_keeps_it(dims, seed):
    """The remark's warning: with B scaled so that I - BA is far from a contraction
    (omega = 8, largest eigenvalue of BA well above 2) the wrong-order B-bar is
    indefinite and PCG with it breaks down, while B_co built from the same S and B
    stays SPD (Theorem 2.1 needs only B SPD) and PCG with it converges."""
    n, rp, ci, v, A = tiny_problem(*dims, seed, sigma=2.0)
    h = oracle.Hierarchy(n, rp, ci, v, max_coarse=6, b_scale=8.0)
    Bb = h.dense_operator(oracle.PREC_BBAR)
    Bc = h.dense_operator(oracle.PREC_COMBINED)
    B = h.dense_operator(oracle.PREC_ILU)
    assert np.max(np.linalg.eigvals(8.0 * B @ A).real) > 2.0
    assert np.linalg.eigvalsh(0.5 * (Bb + Bb.T)).min() < 0
    assert np.max(np.abs(Bc - Bc.T)) <= 1e-12 * np.max(np.abs(Bc))
    assert np.linalg.eigvalsh(0.5 * (Bc + Bc.T)).min() > 0
    b = np.random.default_rng(3).standard_normal(n)
    assert h.pcg(oracle.PREC_BBAR, b, 1e-10, 300)["status"] == oracle.OR_E_BREAKDOWN
    assert h.pcg(oracle.PREC_COMBINED, b, 1e-10, 300)["status"] == oracle.OR_OK


def test_table_5_2_ordering_qualitative():
    """Qualitative ordering of Table 5.2 on a scaled synthetic case:
    B_co needs the fewest iterations; ILU(0) the most. (parity unpinned: the
    paper's matrices are not available, only the ordering is checked.)"""
    p = gen.scaled_config(2, 0.25)
    h = oracle.Hierarchy(p.n, p.row_ptr, p.col, p.val)
    it = {w: h.pcg(w, p.b, 1e-8, 5000)["iters"] for w in (oracle.PREC_COMBINED, oracle.PREC_AMG, oracle.PREC_ILU)}
    assert it[oracle.PREC_COMBINED] <= it[oracle.PREC_AMG] < it[oracle.PREC_ILU]


# ---------------------------------------------------------------- input ------

def test_validation_errors():
    n, rp, ci, v = poisson_1d(5)
    assert oracle.validate(n, rp, ci, v) == oracle.OR_OK
    bad = ci.copy()
    bad[1], bad[0] = bad[0], bad[1]
    assert oracle.validate(n, rp, bad, v) == oracle.OR_E_ARG
    vv = v.copy()
    vv[0] = -1.0
    assert oracle.validate(n, rp, ci, vv) == oracle.OR_E_NOT_SPD
    vv = v.copy()
    vv[1] = -0.5
    assert oracle.validate(n, rp, ci, vv) == oracle.OR_E_ARG  # not symmetric
    assert oracle.validate(0, np.zeros(1, np.int32), ci, v) == oracle.OR_E_ARG
