"""The library's host SETUP code against the oracle (CPU only).

The library and the oracle are independent implementations of the same readings
(ILU(0) of Algorithm 3.1 with k = 0; classical coarsening and interpolation of
Section 3.2). Their outputs must agree bit for bit, since the coarsening decisions
compare values against thresholds.
"""
import re
from pathlib import Path

import numpy as np
import pytest

import gen
import oracle
from tests import host_lib

ROOT = Path(__file__).resolve().parent.parent


def problems():
    return {
        "c1": gen.config1(),
        "c2s": gen.scaled_config(2, 0.2),
        "c3s": gen.scaled_config(3, 0.2),
        "c5s": gen.scaled_config(5, 0.2),
    }


@pytest.fixture(scope="module")
def hiers():
    out = {}
    for k, p in problems().items():
        out[k] = (p, oracle.Hierarchy(p.n, p.row_ptr, p.col, p.val))
    return out


def test_ilu0_bitwise(hiers):
    for k, (p, h) in hiers.items():
        lu, st = host_lib.ilu0(p.n, p.row_ptr, p.col, p.val)
        assert st == 0
        assert np.array_equal(lu, h.ilu()), k


@pytest.mark.parametrize("k", [0, 1, 2])
def test_iluk_bitwise(k):
    """ILU(k) of the library (heap-ordered pivots) and of the oracle (linked row list):
    same pattern, levels and values bit for bit."""
    for name in ("c1", "c2s"):
        p = problems()[name]
        h = oracle.Hierarchy(p.n, p.row_ptr, p.col, p.val, ilu_k=k)
        got, st = host_lib.iluk(p.n, p.row_ptr, p.col, p.val, k)
        assert st == 0
        ref = h.ilu_factor()
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), (name, k)


def test_coarsening_and_interpolation_bitwise(hiers):
    """C/F splitting and P identical to the oracle on every level of the oracle's
    hierarchy (the library's splitting of the oracle's A_l)."""
    for k, (p, h) in hiers.items():
        for d in range(h.nlev - 1):
            rp, ci, v = h.level(d)
            n = rp.size - 1
            cf, nc = host_lib.rs_coarsen(n, rp, ci, v)
            assert np.array_equal(cf, h.cf(d)), (k, d)
            prp, pci, pv = host_lib.rs_interp(n, rp, ci, v, cf)
            orp, oci, ov = h.prolongation(d)
            assert np.array_equal(prp, orp) and np.array_equal(pci, oci), (k, d)
            assert np.array_equal(pv, ov), (k, d)


@pytest.mark.parametrize("seed", range(4))
def test_coarsening_random_m_matrices(seed):
    from tests.test_oracle_pins import random_spd_mmatrix, dense_to_csr
    A = random_spd_mmatrix(80, 0.06, 100 + seed)
    n, rp, ci, v = dense_to_csr(A)
    cf_o, nc_o = oracle.rs_split(n, rp, ci, v)
    cf_l, nc_l = host_lib.rs_coarsen(n, rp, ci, v)
    assert nc_o == nc_l and np.array_equal(cf_o, cf_l)


@pytest.mark.parametrize("key", ["c1", "c2s", "c5s"])
@pytest.mark.parametrize("forward", [True, False])
@pytest.mark.parametrize("R", [1, 7, 64, 300, 100000])
@pytest.mark.parametrize("cap", [0, 40])
def test_sweep_schedule_protocol(hiers, key, forward, R, cap):
    """The persistent sweep's schedule: every dependency is met and every wait can
    be met, on the finest level and on a dense coarse level; with an entry cap, every
    level of two or more rows holds at most cap dependency entries."""
    p, h = hiers[key]
    for d in sorted({0, min(2, h.nlev - 1)}):
        rp, ci, v = h.level(d)
        n = rp.size - 1
        s = host_lib.sweep(n, rp, ci, v, forward, R, cap)
        host_lib.check_sweep_schedule(n, rp, ci, s, forward, cap)


def test_sweep_depth_matches_grid_formula():
    """Lexicographic order on an nx x ny x nz 7-point grid: depth nx + ny + nz - 2."""
    p = gen.scaled_config(5, 0.2)  # no eliminated cells
    nx, ny, nz = p.dims
    s = host_lib.sweep(p.n, p.row_ptr, p.col, p.val, True, p.n)
    assert s["global_depth"] == nx + ny + nz - 2
    assert s["max_local"] == nx + ny + nz - 2


def test_dense_inverse(hiers):
    p, h = hiers["c1"]
    d = h.nlev - 1
    rp, ci, v = h.level(d)
    n = rp.size - 1
    inv, st = host_lib.dense_inverse(n, rp, ci, v)
    A = gen.csr_to_dense(n, rp, ci, v)
    assert st == 0
    assert np.max(np.abs(inv @ A - np.eye(n))) <= 1e-10


def test_c_abi_exports_every_declared_symbol():
    """libcpc.so loads and exports each function declared in include/cpc.h."""
    import ctypes
    from paper_1205_6113_amd import _lib
    header = (ROOT / "include" / "cpc.h").read_text()
    declared = set(re.findall(r"^(?:cpc_status|void|const char\*)\s+(cpc_[a-z_0-9]+)\(", header, re.M))
    assert declared == set(_lib.EXPORTS)
    lib = ctypes.CDLL(str(_lib.LIB_PATH))
    for name in declared:
        assert hasattr(lib, name), name


def test_setup_rejects_bad_input_on_host():
    """Input-contract and ILU(0) pivot errors are returned before any GPU call."""
    import paper_1205_6113_amd as cpc
    from paper_1205_6113_amd import _lib
    p = gen.config1(6, 5)
    bad = p.col.copy()
    bad[[0, 1]] = bad[[1, 0]]
    assert cpc.setup_status(p.n, p.row_ptr, bad, p.val)[0] == _lib.CPC_E_ARG
    v = p.val.copy()
    v[1] *= 2.0
    assert cpc.setup_status(p.n, p.row_ptr, p.col, v)[0] == _lib.CPC_E_ARG  # not symmetric
    v = p.val.copy()
    v[p.row_ptr[3] + 1] = -5.0  # a negative value on a diagonal position? use explicit diag
    diag_pos = [k for k in range(p.row_ptr[3], p.row_ptr[4]) if p.col[k] == 3][0]
    v = p.val.copy()
    v[diag_pos] = 0.0
    assert cpc.setup_status(p.n, p.row_ptr, p.col, v)[0] == _lib.CPC_E_NOT_SPD
    assert cpc.setup_status(0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))[0] == _lib.CPC_E_ARG
    st, msg = cpc.setup_status(3, np.array([0, 2, 5, 7]), np.array([0, 1, 0, 1, 2, 1, 2]),
                               np.array([1, 2, 2, 1, .5, .5, 1.]))
    assert st == _lib.CPC_E_NOT_SPD and "ILU" in msg


def test_option_and_ilu_fill_errors_on_host():
    """Options out of range are rejected before any GPU call; ILU(k) pivot failures are
    reported as for ILU(0); a batch asks for ILU(0) only."""
    import ctypes
    import paper_1205_6113_amd as cpc
    from paper_1205_6113_amd import _lib
    p = gen.config1(6, 5)
    assert cpc.setup_status(p.n, p.row_ptr, p.col, p.val, ilu_fill=17)[0] == _lib.CPC_E_ARG
    assert cpc.setup_status(p.n, p.row_ptr, p.col, p.val, ilu_fill=-1)[0] == _lib.CPC_E_ARG
    assert cpc.setup_status(p.n, p.row_ptr, p.col, p.val, prec=7)[0] == _lib.CPC_E_ARG
    st, msg = cpc.setup_status(3, np.array([0, 2, 5, 7]), np.array([0, 1, 0, 1, 2, 1, 2]),
                               np.array([1, 2, 2, 1, .5, .5, 1.]), ilu_fill=1)
    assert st == _lib.CPC_E_NOT_SPD and "ILU" in msg
    lib = _lib.load()
    o = cpc.options(ilu_fill=1)
    n = (ctypes.c_int32 * 1)(p.n)
    rp = np.ascontiguousarray(p.row_ptr, np.int32)
    ci = np.ascontiguousarray(p.col, np.int32)
    v = np.ascontiguousarray(p.val, np.float64)
    P = ctypes.c_void_p
    rps = (P * 1)(rp.ctypes.data)
    cis = (P * 1)(ci.ctypes.data)
    vs = (P * 1)(v.ctypes.data)
    h = ctypes.c_void_p()
    st = lib.cpc_setup_batch(1, n, rps, cis, vs, ctypes.byref(o), None, ctypes.byref(h))
    assert st == _lib.CPC_E_ARG and "single systems" in _lib.last_error()
