"""The one-wave sweep kernel's schedule, pack and hand-off order, checked on the CPU.

A sequential emulation of the kernel (blocks in ticket order, the kernel's step ring
including the padding steps it runs past a block's end, every load addressed as the
kernel addresses it) must stay inside every array, read a block's own values only after
they are written and other blocks' values only from blocks earlier in the ticket
order, write every row exactly once into a slot of its own, and produce
(D+L)^{-1} f, (D+U)^{-1} f and the unit-lower solve to rounding against a direct
triangular solve. Blocks are contiguous (M = 1) or unions of M segments spaced by the
matrix's dominant coupling distance.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import gen
import oracle
from tests import host_lib


def _tri(n, rp, ci, v, forward, unit):
    a = gen.csr_to_dense(n, rp, ci, v)
    t = np.tril(a) if forward else np.triu(a)
    if unit:
        np.fill_diagonal(t, 1.0)
    return t


def _check(n, rp, ci, v, W, M=1, ring=8, dense=True):
    f = np.random.default_rng(n + W + M).standard_normal(n)
    shapes = set()
    for forward in (True, False):
        for unit in ((False, True) if forward else (False,)):
            st, x, shape = host_lib.wave_emulate(n, rp, ci, v, forward, W, f, M=M, unit=unit, ring=ring)
            assert st == 0, (n, W, M, forward, unit, st)
            if dense:
                t = _tri(n, rp, ci, v, forward, unit)
                xr = sla.solve_triangular(t, f, lower=forward, unit_diagonal=unit)
            else:
                import scipy.sparse as sp
                import scipy.sparse.linalg as spl
                a = sp.csr_matrix((v, ci, rp), shape=(n, n))
                t = sp.tril(a) if forward else sp.triu(a)
                if unit:
                    t = t - sp.diags(t.diagonal()) + sp.eye(n)
                xr = spl.spsolve_triangular(t.tocsr(), f, lower=forward)
            err = np.linalg.norm(x - xr) / np.linalg.norm(xr)
            assert err <= 1e-12, (n, W, M, forward, unit, err)
            shapes.add(shape)
    return shapes


@pytest.mark.parametrize("W", [7, 37, 256, 4096])
def test_contiguous_blocks_fine_levels(W):
    for p in (gen.config1(), gen.config1(37, 23), gen.scaled_config(2, 0.15), gen.scaled_config(3, 0.12)):
        shapes = _check(p.n, p.row_ptr, p.col, p.val, W)
        # seven-point and five-point rows: at most three dependency entries
        assert all(tb * k <= 4 for tb, k, *_ in shapes), shapes


@pytest.mark.parametrize("W,M", [(64, 2), (96, 4), (128, 4), (500, 4), (13, 3)])
def test_segmented_blocks_three_dimensional(W, M):
    """Blocks of M segments spaced one plane apart (the dominant coupling) on 3-D grids,
    with and without eliminated well columns (irregular plane lengths)."""
    for p in (gen.scaled_config(2, 0.15), gen.scaled_config(3, 0.12), gen.scaled_config(5, 0.15)):
        shapes = _check(p.n, p.row_ptr, p.col, p.val, W, M=M, dense=p.n <= 2500)
        for tb, k, nblk, nsteps, R, m, stride in shapes:
            assert stride > 0 and R <= W * M
            if stride >= W:
                assert m == M


def test_full_size_fine_level_segmented():
    """The 128 x 128 x 64 level in the blocks the setup uses (4 segments of 1024 or 4096
    rows): every bound and hand-off checked, solution against a sparse triangular solve."""
    p = gen.config2()
    for W, M in ((1024, 4), (4096, 4)):
        f = np.ones(p.n)
        st, x, shape = host_lib.wave_emulate(p.n, p.row_ptr, p.col, p.val, True, W, f, M=M)
        assert st == 0, (W, M, st)
        assert shape[5] == M and 16000 < shape[6] <= 16384, shape


def test_coarse_levels_wider_rows():
    """Galerkin coarse levels (rows of tens of entries) take wider shapes; rows longer
    than 64 dependency entries have no pack (status -5)."""
    p = gen.scaled_config(2, 0.2)
    h = oracle.Hierarchy(p.n, p.row_ptr, p.col, p.val)
    seen = set()
    for d in range(1, h.nlev - 1):
        rp, ci, v = h.level(d)
        n = rp.size - 1
        low = max(int(np.sum(ci[rp[i]:rp[i + 1]] < i)) for i in range(n))
        if low > 64:
            st, _, _ = host_lib.wave_emulate(n, rp, ci, v, True, 512, np.ones(n))
            assert st == -5
            continue
        if n > 3000:
            continue
        for W, M in ((64, 1), (512, 1), (64, 4)):
            st, _, _ = host_lib.wave_emulate(n, rp, ci, v, True, W, np.ones(n), M=M)
            if st == -6:  # blocks in a cycle: the setup falls back to contiguous blocks
                continue
            seen |= _check(n, rp, ci, v, W, M=M)
    assert any(tb >= 4 for tb, *_ in seen), seen


def test_ring_depths_and_single_block():
    p = gen.config1(16, 16)
    for ring in (1, 2, 8, 16):
        _check(p.n, p.row_ptr, p.col, p.val, 5, ring=ring)
    _check(p.n, p.row_ptr, p.col, p.val, p.n)


def _block_diag(problems):
    rps, cis, vs, parts, off, nnz = [np.zeros(1, np.int64)], [], [], [0], 0, 0
    for p in problems:
        rps.append(np.asarray(p.row_ptr[1:], np.int64) + nnz)
        cis.append(np.asarray(p.col, np.int64) + off)
        vs.append(np.asarray(p.val))
        off += p.n
        nnz += int(p.row_ptr[-1])
        parts.append(off)
    return off, np.concatenate(rps), np.concatenate(cis), np.concatenate(vs), parts


@pytest.mark.parametrize("W,M", [(96, 4), (256, 1), (64, 2)])
def test_batch_parts_own_schedules(W, M):
    """A batch's block-diagonal level: each system scheduled with its own coupling
    distance (3-D systems of different plane sizes, a 2-D one, a tiny one), the systems'
    blocks interleaved in one ticket order; bounds, hand-offs and the solution checked."""
    probs = [gen.scaled_config(2, 0.15), gen.config1(9, 7), gen.scaled_config(3, 0.12), gen.config1(3, 2),
             gen.scaled_config(5, 0.15)]
    n, rp, ci, v, parts = _block_diag(probs)
    f = np.random.default_rng(W + M).standard_normal(n)
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    a = sp.csr_matrix((v, ci, rp), shape=(n, n))
    for forward in (True, False):
        for unit in ((False, True) if forward else (False,)):
            st, x, shape = host_lib.wave_emulate(n, rp, ci, v, forward, W, f, M=M, unit=unit, parts=parts)
            assert st == 0, (W, M, forward, unit, st)
            t = sp.tril(a) if forward else sp.triu(a)
            if unit:
                t = t - sp.diags(t.diagonal()) + sp.eye(n)
            xr = spl.spsolve_triangular(t.tocsr(), f, lower=forward)
            assert np.linalg.norm(x - xr) / np.linalg.norm(xr) <= 1e-12
            tb, k, nblk, nsteps, R, m, stride = shape
            assert R <= W * M
            assert nblk >= len(probs)  # blocks never span two systems


def test_long_rows_have_no_one_wave_pack():
    """Rows with more than 64 dependency entries get no one-wave pack (status -5): the
    setup gives such levels to the four-wave kernel."""
    p = gen.wide_band(3000, 160)
    st, _, _ = host_lib.wave_emulate(p.n, p.row_ptr, p.col, p.val, True, 256, np.ones(p.n))
    assert st == -5
    p = gen.wide_band(3000, 40)
    rows = np.repeat(np.arange(p.n), np.diff(p.row_ptr))
    v = np.where(p.col == rows, 1.0, p.val / 160.0)  # bounded unit-lower solve
    assert _check(p.n, p.row_ptr, p.col, v, 256, dense=False)


def test_four_wave_blocks_never_span_systems():
    """With a batch's system boundaries given, every boundary is a block start and no
    block is longer than R (the per-system masks rely on it); without them, the starts
    are those of the plain rule."""
    probs = [gen.scaled_config(2, 0.15), gen.config1(9, 7), gen.scaled_config(3, 0.12), gen.config1(3, 2)]
    n, rp, ci, v, parts = _block_diag(probs)
    for R in (7, 256, 2048):
        st = host_lib.block_starts(n, rp, ci, v, R, parts)
        assert st[0] == 0 and st[-1] == n and np.all(np.diff(st) > 0) and np.all(np.diff(st) <= R)
        assert set(parts) <= set(st.tolist())
        plain = host_lib.block_starts(n, rp, ci, v, R)
        assert plain[0] == 0 and plain[-1] == n and np.all(np.diff(plain) <= R)
