"""Row products with very uneven row lengths (hub rows of hundreds of entries beside rows
of three), on the GPU: the SpMV of small launches takes several entries per lane at once,
and a hub row runs through many such batches with a ragged last one. Checked against a
dense product, then a B_co solve against the oracle's iteration count and solution.
"""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu


def hub_laplacian(n=3000, hubs=((17, 450), (1234, 333), (2999, 97)), seed=3):
    """Graph Laplacian of a path plus hub nodes joined to many random nodes, with unit
    conductances, shifted by 0.05 I: symmetric positive definite, rows of 3 to ~450."""
    rng = np.random.default_rng(seed)
    edges = {(i, i + 1) for i in range(n - 1)}
    for h, deg in hubs:
        for j in rng.choice(np.delete(np.arange(n), h), deg, replace=False):
            edges.add((min(h, j), max(h, j)))
    a = np.zeros((n, n))
    for i, j in edges:
        a[i, j] = a[j, i] = -1.0
    a[np.diag_indices(n)] = -a.sum(axis=1) + 0.05
    rp = [0]
    ci, v = [], []
    for i in range(n):
        nz = np.nonzero(a[i])[0]
        ci.extend(nz.tolist())
        v.extend(a[i, nz].tolist())
        rp.append(len(ci))
    return a, np.array(rp, np.int32), np.array(ci, np.int32), np.array(v)


def test_uneven_rows_spmv_and_solve():
    import paper_1205_6113_amd as cpc
    a, rp, ci, v = hub_laplacian()
    n = a.shape[0]
    lens = np.diff(rp)
    assert lens.max() > 300 and lens.min() <= 3
    rng = np.random.default_rng(7)
    with cpc.Solver(n, rp, ci, v) as s:
        for rep in range(2):
            x = rng.standard_normal(n)
            y = s.spmv(torch.as_tensor(x, device="cuda"), level=0).cpu().numpy()
            yr = a @ x
            assert np.linalg.norm(y - yr) <= 1e-14 * np.linalg.norm(yr), rep
        b = rng.standard_normal(n)
        xg, it, rel, st = s.solve(torch.as_tensor(b, device="cuda"), tol=1e-10)
        assert st == 0
        xg = xg.cpu().numpy()
    h = oracle.Hierarchy(n, rp, ci, v)
    ref = h.pcg(oracle.PREC_COMBINED, b, 1e-10, 10000)
    # the oracle's residual history passes 1e-10 by orders of magnitude: same count
    assert ref["status"] == 0 and it == ref["iters"], (it, ref["iters"])
    xo = ref["x"]
    assert np.linalg.norm(xg - xo) <= 1e-10 * np.linalg.norm(xo)
    assert np.linalg.norm(a @ xg - b) <= 1.5e-10 * np.linalg.norm(b)
