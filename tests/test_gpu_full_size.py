"""Parity at the full workload sizes, in the configuration bench.py times (tuned setup,
HIP-graph iterations): the 1,048,448-unknown C2 system in FP64 and the 1,122,000-unknown
C3 system with the FP32 preconditioner, against the oracle on the same inputs.
"""
import numpy as np
import pytest
import torch

import gen
import oracle

pytestmark = pytest.mark.gpu


def relerr(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def true_relres(p, x):
    rows = np.repeat(np.arange(p.n), np.diff(p.row_ptr))
    ax = np.zeros(p.n)
    np.add.at(ax, rows, p.val * x[p.col])
    return float(np.linalg.norm(p.b - ax) / np.linalg.norm(p.b))


def test_c2_fp64_full_size():
    import paper_1205_6113_amd as cpc
    p = gen.config2()
    print(f"[case] c2 n={p.n} nnz={p.nnz}", flush=True)
    h = oracle.Hierarchy(p.n, p.row_ptr, p.col, p.val)
    s = cpc.Solver(p.n, p.row_ptr, p.col, p.val)
    try:
        info = s.hierarchy()
        assert info["nlev"] == h.nlev
        assert info["n"] == [n for n, _ in h.level_sizes()]
        assert info["nnz"] == [z for _, z in h.level_sizes()]
        b = torch.as_tensor(p.b, device="cuda")
        ro = h.pcg(oracle.PREC_COMBINED, p.b, p.tol, 10000)
        x, it, rel, st = s.solve(b, tol=p.tol)
        assert st == 0 and ro["status"] == 0
        assert it == ro["iters"], (it, ro["iters"])
        assert true_relres(p, x.cpu().numpy()) <= p.tol
        x2, it2, _, _ = s.solve(b, tol=0.0, maxit=ro["iters"])
        assert relerr(x2.cpu().numpy(), ro["x"]) <= 1e-10
        r = np.random.default_rng(17).standard_normal(p.n)
        z = s.apply("combined", torch.as_tensor(r, device="cuda")).cpu().numpy()
        assert relerr(z, h.apply(oracle.PREC_COMBINED, r)) <= 1e-11
    finally:
        s.close()


def test_c3_fp32_preconditioner_full_size():
    import paper_1205_6113_amd as cpc
    p = gen.config3()
    print(f"[case] c3 n={p.n} nnz={p.nnz}", flush=True)
    h = oracle.Hierarchy(p.n, p.row_ptr, p.col, p.val)
    s = cpc.Solver(p.n, p.row_ptr, p.col, p.val, precision="fp32")
    try:
        ro = h.pcg(oracle.PREC_COMBINED, p.b, p.tol, 10000)
        x, it, rel, st = s.solve(torch.as_tensor(p.b, device="cuda"), tol=p.tol)
        assert st == 0 and ro["status"] == 0
        assert abs(it - ro["iters"]) <= 1
        x = x.cpu().numpy()
        assert true_relres(p, x) <= p.tol
        assert relerr(x, ro["x"]) <= 1e-8
    finally:
        s.close()
