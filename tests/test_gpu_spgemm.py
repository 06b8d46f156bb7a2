"""The sparse product behind the Galerkin matrices (Section 3.2) on the device, through
cpc_spgemm, against a sequential evaluation in the canonical order written here (entry
(i, j) accumulated from 0.0 over the column order of row i of X, products rounded
before each addition): bit for bit, including rows with more distinct columns than the
kernels' LDS table (4096), which take the wide-row path."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

CAP = 4096


def canonical(x, y):
    xrp, xci, xv = x
    yrp, yci, yv = y
    rp, ci, v = [0], [], []
    for i in range(xrp.size - 1):
        acc = {}
        for p in range(xrp[i], xrp[i + 1]):
            k, xk = int(xci[p]), float(xv[p])
            for q in range(yrp[k], yrp[k + 1]):
                j = int(yci[q])
                acc[j] = acc.get(j, 0.0) + xk * float(yv[q])
        for j in sorted(acc):
            ci.append(j)
            v.append(acc[j])
        rp.append(len(ci))
    return np.array(rp, np.int32), np.array(ci, np.int32), np.array(v, np.float64)


def csr(rows, ncols, rng):
    """rows: list of column lists (distinct); values uniform on [-1, 1)."""
    rp = np.zeros(len(rows) + 1, np.int32)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.concatenate([np.asarray(r, np.int32) for r in rows]) if rp[-1] else np.zeros(0, np.int32)
    assert ci.size == 0 or (ci.min() >= 0 and ci.max() < ncols)
    return rp, ci, rng.uniform(-1.0, 1.0, ci.size)


def check(x, y, ncols):
    import paper_1205_6113_amd as cpc
    want = canonical(x, y)
    got = cpc.spgemm(x, y, ncols)
    assert np.array_equal(got[0], want[0])
    assert np.array_equal(got[1], want[1])
    assert np.array_equal(got[2], want[2])  # bit for bit: same order of the same roundings
    return np.diff(want[0])


def test_narrow_rows_random():
    rng = np.random.default_rng(1)
    ninner, ncols = 400, 900
    xr = [sorted(rng.choice(ninner, rng.integers(0, 30), replace=False).tolist()) for _ in range(300)]
    yr = [rng.choice(ncols, rng.integers(1, 12), replace=False).tolist() for _ in range(ninner)]  # unsorted
    lens = check(csr(xr, ninner, rng), csr(yr, ncols, rng), ncols)
    assert lens.max() < CAP


def test_wide_rows_beside_narrow_ones():
    """Rows just under, at and over the table's capacity, beside narrow rows, and more
    wide rows than the wide path's workgroups (so each workgroup takes several)."""
    rng = np.random.default_rng(2)
    ncols = 6000
    ninner = ncols
    # row k of Y: columns k and (7k + 3) mod ncols: a row of X over a set K of inner
    # indices reaches the union of those columns
    yr = [sorted({k, (7 * k + 3) % ncols}) for k in range(ninner)]
    y = csr(yr, ncols, rng)
    xr = []
    targets = [CAP - 1, CAP, CAP + 1, 5999] + [4200 + 10 * t for t in range(70)]
    for t, want in enumerate(targets):
        # choose inner indices until the union of reached columns has `want` entries
        order = rng.permutation(ninner)
        cols, ks = set(), []
        for k in order:
            new = set(yr[k]) - cols
            if len(cols) + len(new) > want:
                continue
            cols |= new
            ks.append(int(k))
            if len(cols) == want:
                break
        assert len(cols) == want
        xr.append(ks)  # unsorted: the canonical order is the stored order
        if t % 3 == 0:
            xr.append(sorted(rng.choice(ninner, 8, replace=False).tolist()))
    lens = check(csr(xr, ninner, rng), y, ncols)
    assert (lens >= CAP).sum() >= 72 and (lens == CAP - 1).sum() >= 1


def test_hierarchy_with_wide_galerkin_rows():
    """A chain whose every unknown couples to one hub (a well column seen by a whole
    layer): the hub's rows of A P and of the coarse matrix hold more columns than the
    LDS table, so the setup's Galerkin products take the wide-row path. The hierarchy
    (C/F splitting, P, every A_l) is bit-identical to the oracle's and PCG matches it."""
    import gen
    import oracle
    import torch
    import paper_1205_6113_amd as cpc
    p = gen.hub_chain()
    h = oracle.Hierarchy(p.n, p.row_ptr, p.col, p.val)
    rp1, _, _ = h.level(1)
    assert np.diff(rp1).max() > CAP
    ro = h.pcg(oracle.PREC_COMBINED, p.b, p.tol, 1000)
    with cpc.Solver(p.n, p.row_ptr, p.col, p.val) as s:
        assert s.hierarchy()["nlev"] == h.nlev
        for d in range(h.nlev):
            rp, ci, v = s.level(d)
            orp, oci, ov = h.level(d)
            assert np.array_equal(rp, orp) and np.array_equal(ci, oci) and np.array_equal(v, ov), d
            if d + 1 < h.nlev:
                prp, pci, pv, cf = s.prolongation(d)
                q = h.prolongation(d)
                assert np.array_equal(cf, h.cf(d)) and np.array_equal(prp, q[0]) and np.array_equal(pci, q[1])
                assert np.array_equal(pv, q[2]), d
        x, it, rel, st = s.solve(torch.as_tensor(p.b, device="cuda"), tol=p.tol)
        assert st == 0 and it == ro["iters"], (it, ro["iters"])
        assert np.linalg.norm(x.cpu().numpy() - ro["x"]) <= 1e-10 * np.linalg.norm(ro["x"])
