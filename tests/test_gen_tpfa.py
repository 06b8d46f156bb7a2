"""The TPFA input generators against hand-derived closed forms (CPU only)."""
import numpy as np
import pytest

import gen


def test_constant_k_3x3_closed_form():
    """Constant k = 1 on a 3x3 grid with Dirichlet x-faces: the 5-point Laplacian
    with +2 on the diagonal for each Dirichlet face (T_b = 2k)."""
    rp, ci, v, _ = gen.tpfa_system(np.zeros((1, 3, 3)), 1.0, True)
    A = gen.csr_to_dense(9, rp, ci, v)
    E = np.zeros((9, 9))
    for j in range(3):
        for i in range(3):
            c = i + 3 * j
            deg = 0
            for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                ii, jj = i + di, j + dj
                if 0 <= ii < 3 and 0 <= jj < 3:
                    E[c, ii + 3 * jj] = -1.0
                    deg += 1
            E[c, c] = deg + (2.0 if i in (0, 2) else 0.0)
    assert np.array_equal(A, E)


def test_two_cell_harmonic_transmissibility():
    k1, k2 = 3.0, 0.5
    rp, ci, v, _ = gen.tpfa_system(np.log(np.array([[[k1, k2]]])), 1.0, False)
    A = gen.csr_to_dense(2, rp, ci, v)
    T = 2 * k1 * k2 / (k1 + k2)
    assert np.allclose(A, [[T, -T], [-T, T]], rtol=1e-15)


def test_kz_ratio_scales_vertical_faces():
    logk = np.zeros((2, 1, 1))
    rp, ci, v, _ = gen.tpfa_system(logk, 0.1, False)
    A = gen.csr_to_dense(2, rp, ci, v)
    assert np.allclose(A, [[0.1, -0.1], [-0.1, 0.1]])


@pytest.mark.parametrize("maker", [lambda: gen.config1(16, 12), lambda: gen.scaled_config(2, 0.125),
                                   lambda: gen.scaled_config(3, 0.15), lambda: gen.scaled_config(5, 0.15)])
def test_symmetric_m_matrix_and_row_sums(maker):
    p = maker()
    A = gen.csr_to_dense(p.n, p.row_ptr, p.col, p.val)
    assert np.array_equal(A, A.T)
    off = A - np.diag(np.diag(A))
    assert np.all(off <= 0)
    rs = A.sum(axis=1)
    assert np.all(rs >= -1e-12 * np.abs(np.diag(A)))
    # rows sum to zero unless they touch a Dirichlet face or an eliminated well
    nx, ny, nz = p.dims
    cells = p.keep if p.keep is not None else np.arange(p.n)
    touches_x = (cells % nx == 0) | (cells % nx == nx - 1)
    interior = ~touches_x if p.dirichlet_x else np.ones(p.n, bool)
    if p.keep is not None:
        full = np.zeros(nx * ny * nz, bool)
        full[p.keep] = True
        for off_ in (1, -1, nx, -nx, nx * ny, -nx * ny):
            nb = cells + off_
            ok = (nb >= 0) & (nb < full.size)
            interior &= ~(ok & ~full[np.clip(nb, 0, full.size - 1)])
    assert np.all(np.abs(rs[interior]) <= 1e-12 * np.abs(np.diag(A)[interior]))
    # sorted columns
    for i in range(min(p.n, 500)):
        c = p.col[p.row_ptr[i]:p.row_ptr[i + 1]]
        assert np.all(np.diff(c) > 0)


def test_generators_are_deterministic():
    a, b = gen.config1(), gen.config1()
    assert np.array_equal(a.val, b.val) and np.array_equal(a.b, b.b)
    c, d = gen.scaled_config(3, 0.2), gen.scaled_config(3, 0.2)
    assert np.array_equal(c.val, d.val) and np.array_equal(c.b, d.b)


def test_correlated_field_statistics():
    f = gen.correlated_field((32, 32, 32), 4.0, np.random.default_rng(0))
    assert abs(f.mean()) < 1e-12 and abs(f.std() - 1.0) < 1e-12
    # neighbouring cells are strongly correlated, distant ones are not
    c1 = np.corrcoef(f[:, :, :-1].ravel(), f[:, :, 1:].ravel())[0, 1]
    c16 = np.corrcoef(f[:, :, :16].ravel(), f[:, :, 16:].ravel())[0, 1]
    assert c1 > 0.9 and abs(c16) < 0.2


def test_full_config_sizes():
    """Sizes of the benchmark workloads."""
    p1 = gen.config1()
    assert (p1.n, p1.nnz) == (4096, 20224)
    assert gen.config4_sizes()[:3] == gen.config4_sizes()[:3]
    assert all(32 <= m <= 96 for m in gen.config4_sizes())
