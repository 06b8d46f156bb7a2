"""Batched solve of independent systems of different sizes against per-system oracle
solves (each system's hierarchy in the batch is the one a solve of it alone builds)."""
import numpy as np
import pytest
import torch

import gen
import oracle

pytestmark = pytest.mark.gpu


def small_batch():
    sizes = [9, 14, 11, 16, 10, 12, 8]
    return gen.config4(sizes=sizes)


def test_batch_matches_per_system_oracle():
    import paper_1205_6113_amd as cpc
    probs = small_batch()
    refs = []
    for p in probs:
        h = oracle.Hierarchy(p.n, p.row_ptr, p.col, p.val)
        refs.append(h.pcg(oracle.PREC_COMBINED, p.b, p.tol, 1000))
    b = torch.as_tensor(np.concatenate([p.b for p in probs]), device="cuda")
    with cpc.BatchSolver([(p.n, p.row_ptr, p.col, p.val) for p in probs]) as bs:
        assert list(bs.sizes) == [p.n for p in probs]
        x, it, rel, st = bs.solve(b, tol=1e-8)
        assert st == 0
        xs = x.cpu().numpy()
        for s, (p, r) in enumerate(zip(probs, refs)):
            assert it[s] == r["iters"], (s, it[s], r["iters"])
            xo = xs[bs.offsets[s]:bs.offsets[s] + p.n]
            err = np.linalg.norm(xo - r["x"]) / np.linalg.norm(r["x"])
            assert err <= 1e-10, (s, err)
        # a second solve on the same handle (graph replay) gives identical results
        x2, it2, _, _ = bs.solve(b, tol=1e-8)
        assert np.array_equal(x2.cpu().numpy(), xs) and list(it2) == list(it)


def test_batch_hierarchy_levels_match_single_solves():
    import paper_1205_6113_amd as cpc
    probs = small_batch()[:3]
    with cpc.BatchSolver([(p.n, p.row_ptr, p.col, p.val) for p in probs]) as bs:
        info = bs.hierarchy()
        nl = [oracle.Hierarchy(p.n, p.row_ptr, p.col, p.val).nlev for p in probs]
        assert info["nlev"] == max(nl)
        assert info["n"][0] == sum(p.n for p in probs)


def test_batch_with_one_level_systems():
    """Systems of at most max_coarse rows (their own coarsest level) beside multi-level
    ones, in any position: per-system iteration counts and x as the oracle's solves of
    each system alone (a one-level system converges in one iteration, B_co = A^{-1})."""
    import paper_1205_6113_amd as cpc
    probs = gen.config4(sizes=[4, 10, 3, 12, 6])  # 64, 1000, 27, 1728, 216 unknowns
    refs = []
    for p in probs:
        h = oracle.Hierarchy(p.n, p.row_ptr, p.col, p.val)
        refs.append((h.nlev, h.pcg(oracle.PREC_COMBINED, p.b, p.tol, 1000)))
    assert sorted(nl for nl, _ in refs)[0] == 1 and max(nl for nl, _ in refs) > 1
    b = torch.as_tensor(np.concatenate([p.b for p in probs]), device="cuda")
    for prec in ("combined", "amg"):
        with cpc.BatchSolver([(p.n, p.row_ptr, p.col, p.val) for p in probs], prec=prec) as bs:
            x, it, rel, st = bs.solve(b, tol=1e-8)
            assert st == 0
            xs = x.cpu().numpy()
            for s, (p, (nl, r)) in enumerate(zip(probs, refs)):
                xo = xs[bs.offsets[s]:bs.offsets[s] + p.n]
                if prec == "combined":
                    assert it[s] == r["iters"], (s, it[s], r["iters"])
                    err = np.linalg.norm(xo - r["x"]) / np.linalg.norm(r["x"])
                    assert err <= 1e-10, (s, err)
                if nl == 1:
                    assert it[s] == 1, (prec, s, it[s])
                    xd = np.linalg.solve(gen.csr_to_dense(p.n, p.row_ptr, p.col, p.val), p.b)
                    assert np.linalg.norm(xo - xd) <= 1e-12 * np.linalg.norm(xd)


_MID_REFS = {}


def _mid_batch():
    """Four systems of 27,000-85,184 unknowns: every level 0 is split into several sweep
    blocks, and the coarse levels reach the block-substitution and explicit-inverse
    forms, as the systems of the 64-system workload do."""
    probs = gen.config4(sizes=[36, 44, 30, 40])
    if not _MID_REFS:
        for s, p in enumerate(probs):
            h = oracle.Hierarchy(p.n, p.row_ptr, p.col, p.val)
            _MID_REFS[s] = h.pcg(oracle.PREC_COMBINED, p.b, p.tol, 1000)
    return probs, _MID_REFS


@pytest.mark.parametrize("forms", ["never", "block", "auto"])
def test_batch_mid_size_systems_every_smoother_form(forms):
    """Per-system iteration counts equal to the oracle's and x within 1e-10 (equal
    counts under the same stopping rule put both at the oracle's iteration count), with
    the Gauss-Seidel smoother forced to level-scheduled sweeps, to block substitution,
    or left to the setup tuner; the forms each level got are checked."""
    import paper_1205_6113_amd as cpc
    probs, refs = _mid_batch()
    print(f"[case] batch forms={forms} sizes={[p.n for p in probs]}", flush=True)
    b = torch.as_tensor(np.concatenate([p.b for p in probs]), device="cuda")
    with cpc.BatchSolver([(p.n, p.row_ptr, p.col, p.val) for p in probs], dense_smoother=forms) as bs:
        info = bs.hierarchy()
        smoothed = [k for k in info["smoother"] if k != "none"]
        if forms == "never":
            assert set(smoothed) == {"sweep"}, info["smoother"]
            assert info["n"][0] > 2 * info["block_rows"][0]  # several sweep blocks on level 0
        elif forms == "block":
            assert "block" in smoothed, info["smoother"]
        x, it, rel, st = bs.solve(b, tol=1e-8)
        assert st == 0
        xs = x.cpu().numpy()
        for s, p in enumerate(probs):
            r = refs[s]
            assert it[s] == r["iters"], (forms, s, it[s], r["iters"])
            xo = xs[bs.offsets[s]:bs.offsets[s] + p.n]
            err = np.linalg.norm(xo - r["x"]) / np.linalg.norm(r["x"])
            assert err <= 1e-10, (forms, s, err)


def test_batch_fp32_preconditioner():
    """The batch with the FP32 preconditioner (FP64 PCG): every system reaches the
    tolerance on its true residual, takes at most one iteration more than the FP64
    oracle, and its solution lies within 1e-10 of the oracle's (the bars of the
    single-system FP32 test)."""
    import paper_1205_6113_amd as cpc
    probs, refs = _mid_batch()
    b = torch.as_tensor(np.concatenate([p.b for p in probs]), device="cuda")
    with cpc.BatchSolver([(p.n, p.row_ptr, p.col, p.val) for p in probs], precision="fp32") as bs:
        x, it, rel, st = bs.solve(b, tol=1e-8)
        assert st == 0
        xs = x.cpu().numpy()
        for s, p in enumerate(probs):
            r = refs[s]
            xo = xs[bs.offsets[s]:bs.offsets[s] + p.n]
            rows = np.repeat(np.arange(p.n), np.diff(p.row_ptr))
            ax = np.zeros(p.n)
            np.add.at(ax, rows, p.val * xo[p.col])
            tr = np.linalg.norm(p.b - ax) / np.linalg.norm(p.b)
            err = np.linalg.norm(xo - r["x"]) / np.linalg.norm(r["x"])
            print(f"[fp32 batch] system {s}: iters {it[s]} (oracle {r['iters']}), true relres {tr:.2e}, "
                  f"x err {err:.2e}", flush=True)
            assert tr <= 1e-8 * 1.05 and it[s] <= r["iters"] + 1 and err <= 1e-10, (s, tr, it[s], err)


def test_batch_zero_rhs_system_stops_at_once():
    """A system with b = 0 stops before the first iteration (x = 0, no iterations) and is
    masked out of every preconditioner launch; the others converge as when solved
    alone."""
    import paper_1205_6113_amd as cpc
    probs = gen.config4(sizes=[10, 12, 9])
    zero = 1
    bs_all = [p.b.copy() for p in probs]
    bs_all[zero][:] = 0.0
    b = torch.as_tensor(np.concatenate(bs_all), device="cuda")
    with cpc.BatchSolver([(p.n, p.row_ptr, p.col, p.val) for p in probs]) as bsv:
        x0 = torch.full_like(b, 7.0)  # overwritten: the solve starts from x = 0
        x, it, rel, st = bsv.solve(b, x=x0, tol=1e-8)
        assert st == 0
        xs = x.cpu().numpy()
        for s, p in enumerate(probs):
            xo = xs[bsv.offsets[s]:bsv.offsets[s] + p.n]
            if s == zero:
                assert it[s] == 0 and np.all(xo == 0.0), (it[s], np.abs(xo).max())
                continue
            r = oracle.Hierarchy(p.n, p.row_ptr, p.col, p.val).pcg(oracle.PREC_COMBINED, p.b, 1e-8, 1000)
            assert it[s] == r["iters"], (s, it[s], r["iters"])
            assert np.linalg.norm(xo - r["x"]) <= 1e-10 * np.linalg.norm(r["x"]), s
