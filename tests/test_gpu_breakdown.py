"""PCG breakdown detected on the device (Algorithm 2.1 driven by PCG: a non-positive
or non-finite <r, z> or <p, Ap> stops the iteration), single and batched. A non-finite
right-hand side drives the scalars non-finite; the oracle reports a breakdown on the
same input. In a batch the breakdown stays with its system: the others converge to
the oracle's solutions of them alone."""
import numpy as np
import pytest
import torch

import gen
import oracle

pytestmark = pytest.mark.gpu


def test_single_solve_reports_breakdown():
    import paper_1205_6113_amd as cpc
    p = gen.config1(16, 16)
    b = p.b.copy()
    b[5] = np.inf
    h = oracle.Hierarchy(p.n, p.row_ptr, p.col, p.val)
    assert h.pcg(oracle.PREC_COMBINED, b, p.tol, 100)["status"] == oracle.OR_E_BREAKDOWN
    with cpc.Solver(p.n, p.row_ptr, p.col, p.val) as s:
        _, it, _, st = s.solve(torch.as_tensor(b, device="cuda"), tol=p.tol, maxit=100)
        assert st == cpc.CPC_E_BREAKDOWN, st
        # the handle stays usable: a finite right-hand side solves as before
        x, it2, _, st2 = s.solve(torch.as_tensor(p.b, device="cuda"), tol=p.tol, maxit=100)
        ro = h.pcg(oracle.PREC_COMBINED, p.b, p.tol, 100)
        assert st2 == 0 and it2 == ro["iters"]
        assert np.linalg.norm(x.cpu().numpy() - ro["x"]) <= 1e-10 * np.linalg.norm(ro["x"])


def test_batch_breakdown_stays_with_its_system():
    import paper_1205_6113_amd as cpc
    probs = gen.config4(sizes=[9, 12, 10])
    bad = 1
    bs_all = [p.b.copy() for p in probs]
    bs_all[bad][3] = np.nan
    assert oracle.Hierarchy(probs[bad].n, probs[bad].row_ptr, probs[bad].col, probs[bad].val).pcg(
        oracle.PREC_COMBINED, bs_all[bad], 1e-8, 100)["status"] == oracle.OR_E_BREAKDOWN
    b = torch.as_tensor(np.concatenate(bs_all), device="cuda")
    with cpc.BatchSolver([(p.n, p.row_ptr, p.col, p.val) for p in probs]) as bsv:
        x, it, rel, st = bsv.solve(b, tol=1e-8, maxit=100)
        assert st == cpc.CPC_E_BREAKDOWN, st
        xs = x.cpu().numpy()
        for s, p in enumerate(probs):
            if s == bad:
                continue
            r = oracle.Hierarchy(p.n, p.row_ptr, p.col, p.val).pcg(oracle.PREC_COMBINED, p.b, 1e-8, 100)
            assert it[s] == r["iters"], (s, it[s], r["iters"])
            xo = xs[bsv.offsets[s]:bsv.offsets[s] + p.n]
            assert np.linalg.norm(xo - r["x"]) <= 1e-10 * np.linalg.norm(r["x"]), s
