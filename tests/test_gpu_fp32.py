"""FP32 preconditioner inside FP64 PCG against the FP64 oracle.

The preconditioner's matrices and vectors are stored in FP32 with FP64 row sums;
PCG vectors, the outer residuals of Algorithm 2.1, reductions and the coarsest
solve stay FP64.

Bars. Operators (S, B and B_co of Algorithm 2.1 applied to one vector): relative
error <= 1e-6 against the FP64 oracle, i.e. about 17 units of FP32 rounding
(u = 6.0e-8): every stored entry and every vector handed between kernels is rounded
once to FP32 and the row sums are FP64, so the error is a small multiple of u (the
measured errors are 2.7e-9 .. 1.1e-7). Solve: the true relative residual meets the
requested tolerance, PCG takes at most one more iteration than in FP64, and the
solution differs from the FP64 oracle's by <= 1e-10 (the preconditioner's FP32
perturbation changes the search directions by O(u) and the iterate by O(u) times the
remaining error; measured <= 1.3e-14)."""
import numpy as np
import pytest
import torch

import gen
import oracle

pytestmark = pytest.mark.gpu


def _true_relres(p, x):
    rows = np.repeat(np.arange(p.n), np.diff(p.row_ptr))
    ax = np.zeros(p.n)
    np.add.at(ax, rows, p.val * x[p.col])
    return float(np.linalg.norm(p.b - ax) / np.linalg.norm(p.b))


@pytest.mark.parametrize("case", ["c3s", "c2m", "c1"])
def test_fp32_preconditioner_reaches_fp64_accuracy(case):
    import paper_1205_6113_amd as cpc
    p = {"c3s": gen.scaled_config(3, 0.2), "c2m": gen.scaled_config(2, 0.3), "c1": gen.config1()}[case]
    h = oracle.Hierarchy(p.n, p.row_ptr, p.col, p.val)
    ro = h.pcg(oracle.PREC_COMBINED, p.b, p.tol, 10000)
    b = torch.as_tensor(p.b, device="cuda")
    with cpc.Solver(p.n, p.row_ptr, p.col, p.val, precision="fp32") as s32, \
            cpc.Solver(p.n, p.row_ptr, p.col, p.val, precision="fp64") as s64:
        # operators: FP32 storage rounding only
        r = np.random.default_rng(1).standard_normal(p.n)
        for op, which in (("vcycle", oracle.OP_VCYCLE), ("ilu", oracle.PREC_ILU), ("combined", oracle.PREC_COMBINED)):
            z = s32.apply(op, torch.as_tensor(r, device="cuda")).cpu().numpy()
            zr = h.apply(which, r)
            err = np.linalg.norm(z - zr) / np.linalg.norm(zr)
            print(f"[fp32] {case} {op}: operator error {err:.3e}", flush=True)
            assert err <= 1e-6, (case, op, err)
        x32, it32, rel32, st32 = s32.solve(b, tol=p.tol)
        x64, it64, rel64, st64 = s64.solve(b, tol=p.tol)
    assert st32 == 0 and st64 == 0
    x32 = x32.cpu().numpy()
    tr = _true_relres(p, x32)
    err = np.linalg.norm(x32 - ro["x"]) / np.linalg.norm(ro["x"])
    print(f"[fp32] {case}: iters fp32={it32} fp64={it64} oracle={ro['iters']} true relres={tr:.3e} "
          f"x err vs fp64 oracle={err:.3e}")
    assert tr <= p.tol * 1.05
    assert it32 <= it64 + 1
    assert err <= 1e-10


@pytest.mark.parametrize("form", ["never", "always", "block"])
def test_fp32_every_smoother_form(form):
    """The FP32 preconditioner with each Gauss-Seidel form forced (level-scheduled
    sweeps only, whole-level explicit inverses where they fit, block substitution
    with 2048-row blocks): the combined operator within 1e-6 of the FP64 oracle and
    the solve to the FP64 oracle's solution within 1e-10, as above."""
    import paper_1205_6113_amd as cpc
    p = gen.scaled_config(2, 0.3)
    h = oracle.Hierarchy(p.n, p.row_ptr, p.col, p.val)
    ro = h.pcg(oracle.PREC_COMBINED, p.b, p.tol, 10000)
    b = torch.as_tensor(p.b, device="cuda")
    with cpc.Solver(p.n, p.row_ptr, p.col, p.val, precision="fp32", dense_smoother=form) as s:
        kinds = s.hierarchy()["smoother"]
        want = {"never": "sweep", "always": "dense", "block": "block"}[form]
        assert want in kinds, kinds
        r = np.random.default_rng(3).standard_normal(p.n)
        z = s.apply("combined", torch.as_tensor(r, device="cuda")).cpu().numpy()
        zr = h.apply(oracle.PREC_COMBINED, r)
        err_op = np.linalg.norm(z - zr) / np.linalg.norm(zr)
        x, it, rel, st = s.solve(b, tol=p.tol)
    assert st == 0
    x = x.cpu().numpy()
    err = np.linalg.norm(x - ro["x"]) / np.linalg.norm(ro["x"])
    print(f"[fp32] form {form} ({kinds}): operator error {err_op:.3e}, iters {it} (oracle {ro['iters']}), "
          f"x err {err:.3e}", flush=True)
    assert err_op <= 1e-6
    assert _true_relres(p, x) <= p.tol * 1.05
    assert it <= ro["iters"] + 1
    assert err <= 1e-10
