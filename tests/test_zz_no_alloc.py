"""cpc_solve_noalloc (the solve with its scratch in a static device array, nothing
allocated) against cpc_solve on the same handles: two calls in a row, the second on a
smaller system, each compared with the graph-replayed solve of cpc_solve."""
import numpy as np
import pytest
import torch

import gen

pytestmark = pytest.mark.gpu


def _check(p, prec_args):
    import paper_1205_6113_amd as cpc
    b = torch.as_tensor(p.b, device="cuda")
    with cpc.Solver(p.n, p.row_ptr, p.col, p.val, **prec_args) as s:
        x_ref, it_ref, rel_ref, st_ref = s.solve(b, tol=p.tol)
        x = torch.full_like(b, float("nan"))
        x, it, rel, st = s.solve_noalloc(b, x, tol=p.tol)
        assert st == st_ref == 0
        assert it == it_ref, (it, it_ref)
        err = float(torch.linalg.norm(x - x_ref) / torch.linalg.norm(x_ref))
        assert err <= 1e-10, err
        assert abs(rel - rel_ref) <= 1e-12 * rel_ref
        # a fixed iteration count (tol = 0) and an initial guess give the same as cpc_solve
        k = max(1, it_ref - 1)
        xa, ita, _, sta = s.solve(b, tol=0.0, maxit=k)
        xb = torch.zeros_like(b)
        xb, itb, _, stb = s.solve_noalloc(b, xb, tol=0.0, maxit=k)
        assert ita == itb == k and sta == stb
        assert float(torch.linalg.norm(xa - xb) / torch.linalg.norm(xa)) <= 1e-10
        return err


def test_noalloc_matches_solve_then_smaller_system():
    big = gen.scaled_config(2, 0.25)    # 32 x 32 x 16 with two wells: several sweep blocks
    small = gen.scaled_config(1, 0.5)   # 32 x 32 two-dimensional
    assert small.n < big.n
    print(f"[case] noalloc n={big.n} then n={small.n}", flush=True)
    e1 = _check(big, {})
    e2 = _check(small, {})
    print(f"[case] noalloc errors {e1:.2e} {e2:.2e}", flush=True)


def test_noalloc_fp32_preconditioner_and_batch_rejected():
    import paper_1205_6113_amd as cpc
    from paper_1205_6113_amd import _lib
    p = gen.scaled_config(1, 0.75)
    _check(p, {"precision": "fp32"})
    probs = gen.config4(sizes=[9, 10])
    with cpc.BatchSolver([(q.n, q.row_ptr, q.col, q.val) for q in probs]) as bs:
        it = __import__("ctypes").c_int32(0)
        rel = __import__("ctypes").c_double(0.0)
        b = torch.zeros(bs.n, dtype=torch.float64, device="cuda")
        st = bs._lib.cpc_solve_noalloc(bs._h, b.data_ptr(), b.data_ptr(), 0, 1e-8, 10,
                                       __import__("ctypes").byref(it), __import__("ctypes").byref(rel))
        assert st == _lib.CPC_E_ARG
