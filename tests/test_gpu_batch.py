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


def test_batch_rejects_one_level_system():
    import paper_1205_6113_amd as cpc
    from paper_1205_6113_amd import _lib
    probs = gen.config4(sizes=[4, 10])  # 64 unknowns <= max_coarse
    with pytest.raises(cpc.CpcError) as e:
        cpc.BatchSolver([(p.n, p.row_ptr, p.col, p.val) for p in probs])
    assert e.value.status == _lib.CPC_E_ARG
