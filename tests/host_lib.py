"""ctypes access to libcpc_host.so (the library's host SETUP code) for CPU tests."""
import ctypes
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parent.parent
HOST_LIB = ROOT / "paper_1205_6113_amd" / "libcpc_host.so"
_lib = None


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def lib():
    global _lib
    if _lib is None:
        if not HOST_LIB.exists():
            from paper_1205_6113_amd import build
            build.build()
        L = ctypes.CDLL(str(HOST_LIB))
        P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        L.cpch_ilu0.argtypes = [I, P, P, P, P]
        L.cpch_iluk.argtypes = [I, P, P, P, I, P, P, P, P]
        L.cpch_iluk.restype = ctypes.c_long
        L.cpch_rs_coarsen.argtypes = [I, P, P, P, D, P]
        L.cpch_rs_interp.argtypes = [I, P, P, P, D, P, P, P, P]
        L.cpch_rs_interp.restype = ctypes.c_long
        L.cpch_sweep.argtypes = [I, P, P, P, I, I, I, P, P, P, P, P, P, P, P, P, P]
        L.cpch_dense_inverse.argtypes = [I, P, P, P, P]
        L.cpch_wave_emulate.argtypes = [I, P, P, P, I, I, I, I, I, P, P, P, P, I]
        L.cpch_block_starts.argtypes = [I, P, P, P, I, P, I, P, I]
        _lib = L
    return _lib


def _csr(rp, ci, v):
    return (np.ascontiguousarray(rp, np.int32), np.ascontiguousarray(ci, np.int32),
            np.ascontiguousarray(v, np.float64))


def ilu0(n, rp, ci, v):
    rp, ci, v = _csr(rp, ci, v)
    lu = np.empty_like(v)
    st = lib().cpch_ilu0(n, _p(rp), _p(ci), _p(v), _p(lu))
    return lu, st


def iluk(n, rp, ci, v, k):
    rp, ci, v = _csr(rp, ci, v)
    nnz = lib().cpch_iluk(n, _p(rp), _p(ci), _p(v), int(k), None, None, None, None)
    if nnz < 0:
        return None, int(-nnz)
    frp = np.empty(n + 1, np.int32)
    fci = np.empty(nnz, np.int32)
    fv = np.empty(nnz, np.float64)
    lev = np.empty(nnz, np.int32)
    lib().cpch_iluk(n, _p(rp), _p(ci), _p(v), int(k), _p(frp), _p(fci), _p(fv), _p(lev))
    return (frp, fci, fv, lev), 0


def rs_coarsen(n, rp, ci, v, theta=0.25):
    rp, ci, v = _csr(rp, ci, v)
    cf = np.empty(n, np.int32)
    nc = lib().cpch_rs_coarsen(n, _p(rp), _p(ci), _p(v), float(theta), _p(cf))
    return cf, nc


def rs_interp(n, rp, ci, v, cf, theta=0.25):
    rp, ci, v = _csr(rp, ci, v)
    cf = np.ascontiguousarray(cf, np.int32)
    prp = np.empty(n + 1, np.int32)
    nnz = lib().cpch_rs_interp(n, _p(rp), _p(ci), _p(v), float(theta), _p(cf), None, None, None)
    pci = np.empty(max(nnz, 1), np.int32)
    pv = np.empty(max(nnz, 1), np.float64)
    lib().cpch_rs_interp(n, _p(rp), _p(ci), _p(v), float(theta), _p(cf), _p(prp), _p(pci), _p(pv))
    return prp, pci[:nnz], pv[:nnz]


def sweep(n, rp, ci, v, forward, R, max_entries=0):
    rp, ci, v = _csr(rp, ci, v)
    sizes = np.zeros(7, np.int32)
    L = lib()
    L.cpch_sweep(n, _p(rp), _p(ci), _p(v), int(forward), int(R), int(max_entries), _p(sizes), None, None, None,
                 None, None, None, None, None, None)
    nblk, nl, nw = int(sizes[0]), int(sizes[1]), int(sizes[2])
    out = {
        "perm": np.empty(n, np.int32), "blk_beg": np.empty(nblk, np.int32), "blk_end": np.empty(nblk, np.int32),
        "lvl_ptr": np.empty(nl + 1, np.int32), "wait_ptr": np.empty(nl + 1, np.int32),
        "wait_blk": np.empty(max(nw, 1), np.int32), "wait_need": np.empty(max(nw, 1), np.int32),
        "publish": np.empty(max(nl, 1), np.int32), "blk_row": np.empty(nblk + 1, np.int32),
    }
    L.cpch_sweep(n, _p(rp), _p(ci), _p(v), int(forward), int(R), int(max_entries), _p(sizes), _p(out["perm"]),
                 _p(out["blk_beg"]),
                 _p(out["blk_end"]), _p(out["lvl_ptr"]), _p(out["wait_ptr"]), _p(out["wait_blk"]),
                 _p(out["wait_need"]), _p(out["publish"]), _p(out["blk_row"]))
    out.update(nblk=nblk, nlev=nl, nwait=nw, global_depth=int(sizes[3]), max_local=int(sizes[4]),
               R=int(sizes[5]), max_level_entries=int(sizes[6]))
    out["wait_blk"] = out["wait_blk"][:nw]
    out["wait_need"] = out["wait_need"][:nw]
    return out


def dense_inverse(n, rp, ci, v):
    rp, ci, v = _csr(rp, ci, v)
    inv = np.empty((n, n))
    st = lib().cpch_dense_inverse(n, _p(rp), _p(ci), _p(v), _p(inv))
    return inv, st


def check_sweep_schedule(n, rp, ci, s, forward, cap=0):
    """Simulate the persistent sweep's protocol and check that (a) every row is
    processed exactly once in its own block, (b) every dependency is either an
    earlier local level of the same block or a row of a block taken earlier whose
    completion the block has waited for, and (c) every wait can be met (the awaited
    block publishes a progress value at least as large). Returns the number of waits."""
    nblk = s["nblk"]
    perm, lp = s["perm"], s["lvl_ptr"]
    blk_of = np.repeat(np.arange(nblk), np.diff(s["blk_row"]))
    row_blk = np.full(n, -1, np.int64)
    row_lev = np.full(n, -1, np.int64)
    final_pub = np.zeros(nblk, np.int64)
    for b in range(nblk):
        for lv in range(s["blk_beg"][b], s["blk_end"][b]):
            m = lv - s["blk_beg"][b]
            rows = perm[lp[lv]:lp[lv + 1]]
            assert rows.size > 0
            assert np.all(blk_of[rows] == b), "row outside its block"
            assert np.all(row_blk[rows] == -1), "row processed twice"
            row_blk[rows] = b
            row_lev[rows] = m
            if s["publish"][lv]:
                final_pub[b] = m + 1
    assert np.all(row_blk >= 0), "row never processed"
    rp_ = np.asarray(rp)
    ci_ = np.asarray(ci)
    ndep = np.array([np.count_nonzero(ci_[rp_[i]:rp_[i + 1]] < i) if forward else
                     np.count_nonzero(ci_[rp_[i]:rp_[i + 1]] > i) for i in range(n)])
    worst = 0
    for lv in range(len(lp) - 1):
        rows = perm[lp[lv]:lp[lv + 1]]
        ent = int(ndep[rows].sum())
        if rows.size > 1:
            worst = max(worst, ent)
            if cap > 0:
                assert ent <= cap, "level over the entry cap"
    assert worst == s["max_level_entries"]
    order = {b: (b if forward else nblk - 1 - b) for b in range(nblk)}  # ticket of each block
    rp = np.asarray(rp)
    ci = np.asarray(ci)
    for b in range(nblk):
        waited = {}
        for lv in range(s["blk_beg"][b], s["blk_end"][b]):
            m = lv - s["blk_beg"][b]
            for w in range(s["wait_ptr"][lv], s["wait_ptr"][lv + 1]):
                ob, need = int(s["wait_blk"][w]), int(s["wait_need"][w])
                assert order[ob] < order[b], "wait on a block taken later (deadlock)"
                assert final_pub[ob] >= need, "wait can never be met"
                waited[ob] = max(waited.get(ob, 0), need)
            for i in perm[lp[lv]:lp[lv + 1]]:
                cols = ci[rp[i]:rp[i + 1]]
                deps = cols[cols < i] if forward else cols[cols > i]
                for j in deps:
                    if row_blk[j] == b:
                        assert row_lev[j] < m, "same-block dependency not at an earlier level"
                    else:
                        assert order[row_blk[j]] < order[b]
                        assert waited.get(int(row_blk[j]), 0) >= row_lev[j] + 1, "dependency not waited for"
    return s["nwait"]


def wave_emulate(n, rp, ci, v, forward, W, f, M=1, unit=False, ring=8, parts=None):
    """Sequential emulation of the one-wave sweep kernel on its pack (see
    cpch_wave_emulate): returns (status, x, (tb, k, nblk, nsteps, R, M, stride)).
    parts: row boundaries of the diagonal blocks scheduled on their own (a batch)."""
    rp, ci, v = _csr(rp, ci, v)
    f = np.ascontiguousarray(f, np.float64)
    x = np.zeros(n)
    shape = np.zeros(7, np.int32)
    pa = None if parts is None else np.ascontiguousarray(parts, np.int32)
    st = lib().cpch_wave_emulate(n, _p(rp), _p(ci), _p(v), int(forward), int(W), int(M), int(unit), int(ring),
                                 _p(f), _p(x), _p(shape), None if pa is None else _p(pa),
                                 0 if pa is None else len(pa) - 1)
    return st, x, tuple(int(t) for t in shape)


def block_starts(n, rp, ci, v, R, parts=None):
    """Block starts of the four-wave sweep schedule (cpch_block_starts)."""
    rp, ci, v = _csr(rp, ci, v)
    out = np.zeros(n + 2, np.int32)
    pa = None if parts is None else np.ascontiguousarray(parts, np.int32)
    k = lib().cpch_block_starts(n, _p(rp), _p(ci), _p(v), int(R), None if pa is None else _p(pa),
                                0 if pa is None else len(pa) - 1, _p(out), out.size)
    return out[:k]
