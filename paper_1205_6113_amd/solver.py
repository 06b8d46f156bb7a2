"""Python binding of the combined-preconditioned CG library (argument marshalling only).

Every numerical step runs in libcpc.so on the GPU; this module converts arrays,
passes device pointers of torch tensors and the current HIP stream, and turns
status codes into exceptions.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import CpcError, check, load


def _host(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dev_vec(t: torch.Tensor, n: int, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU torch tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if t.numel() != n or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous with {n} entries")
    return t


def options(prec="combined", precision="fp64", max_coarse=256, max_levels=25, theta=0.25, swap_roles=False,
            check_symmetry=True, use_graph=True, check_every=0, sweep_block_rows=0,
            sweep_threads=0, dense_smoother=0, tune=True, verbose=False, ilu_fill=0,
            sweep_kernel="auto") -> _lib.Options:
    lib = load()
    o = _lib.Options()
    lib.cpc_default_options(ctypes.byref(o))
    o.prec = _lib.PREC[prec] if isinstance(prec, str) else int(prec)
    o.precision = _lib.PRECISION[precision] if isinstance(precision, str) else int(precision)
    o.max_coarse = int(max_coarse)
    o.max_levels = int(max_levels)
    o.theta = float(theta)
    o.swap_roles = int(bool(swap_roles))
    o.check_symmetry = int(bool(check_symmetry))
    o.use_graph = int(bool(use_graph))
    o.check_every = int(check_every)
    o.sweep_block_rows = int(sweep_block_rows)
    o.sweep_threads = int(sweep_threads)
    o.tune = int(bool(tune))
    o.verbose = int(bool(verbose))
    o.ilu_fill = int(ilu_fill)
    o.dense_smoother = _lib.DENSE[dense_smoother] if isinstance(dense_smoother, str) else int(dense_smoother)
    o.sweep_kernel = {"auto": 0, "wave": 0, "workgroup": 1}[sweep_kernel] if isinstance(sweep_kernel, str) \
        else int(sweep_kernel)
    return o


class Solver:
    """SETUP on construction (cpc_setup), then solve/apply on the GPU.

    row_ptr/col/val: host CSR (int32/int32/float64), copied by the library.
    Vectors passed to solve/apply are float64 torch tensors on the GPU.
    """

    def __init__(self, n, row_ptr, col, val, device="cuda", **opts):
        lib = load()
        self._lib = lib
        self.n = int(n)
        self.device = torch.device(device)
        rp = _host(row_ptr, np.int32)
        ci = _host(col, np.int32)
        v = _host(val, np.float64)
        self.nnz = int(rp[-1]) if rp.size else 0
        self._opts = options(**opts)
        h = ctypes.c_void_p()
        stream = None
        if self.device.type == "cuda" and torch.cuda.is_available():
            stream = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream or None)
        st = lib.cpc_setup(self.n, _ptr(rp), _ptr(ci), _ptr(v), ctypes.byref(self._opts), stream, ctypes.byref(h))
        check(st)
        self._h = h

    # -- lifecycle
    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.cpc_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- SOLVE
    def solve(self, b: torch.Tensor, x: torch.Tensor | None = None, tol: float = 1e-8, maxit: int = 10000,
              use_x0: bool = False, prec: str | int | None = None):
        """PCG for A x = b. Returns (x, iters, relres, status); raises on argument,
        device and allocation errors. status is CPC_OK, CPC_E_MAXIT or CPC_E_BREAKDOWN."""
        b = _dev_vec(b, self.n, "b")
        if x is None:
            x = torch.empty_like(b)
            use_x0 = False
        x = _dev_vec(x, self.n, "x")
        it = ctypes.c_int32(0)
        rel = ctypes.c_double(0.0)
        if prec is None:
            st = self._lib.cpc_solve(self._h, b.data_ptr(), x.data_ptr(), int(bool(use_x0)), float(tol), int(maxit),
                                     ctypes.byref(it), ctypes.byref(rel))
        else:
            p = _lib.PREC[prec] if isinstance(prec, str) else int(prec)
            st = self._lib.cpc_solve_with(self._h, p, b.data_ptr(), x.data_ptr(), int(bool(use_x0)), float(tol),
                                          int(maxit), ctypes.byref(it), ctypes.byref(rel))
        check(st, allow=(_lib.CPC_OK, _lib.CPC_E_MAXIT, _lib.CPC_E_BREAKDOWN))
        return x, it.value, rel.value, st

    def solve_noalloc(self, b: torch.Tensor, x: torch.Tensor, tol: float = 1e-8, maxit: int = 10000,
                      use_x0: bool = False):
        """The solve of `solve` through cpc_solve_noalloc (no device allocation; x must be
        given). Returns (x, iters, relres, status)."""
        b = _dev_vec(b, self.n, "b")
        x = _dev_vec(x, self.n, "x")
        it = ctypes.c_int32(0)
        rel = ctypes.c_double(0.0)
        st = self._lib.cpc_solve_noalloc(self._h, b.data_ptr(), x.data_ptr(), int(bool(use_x0)), float(tol),
                                         int(maxit), ctypes.byref(it), ctypes.byref(rel))
        check(st, allow=(_lib.CPC_OK, _lib.CPC_E_MAXIT, _lib.CPC_E_BREAKDOWN))
        return x, it.value, rel.value, st

    def apply(self, op: str | int, r: torch.Tensor, z: torch.Tensor | None = None) -> torch.Tensor:
        """z = M r for an operator of cpc_op ('combined', 'amg', 'ilu', 'additive', 'none',
        'vcycle', 'fgs', 'bgs')."""
        r = _dev_vec(r, self.n, "r")
        z = torch.empty_like(r) if z is None else _dev_vec(z, self.n, "z")
        o = _lib.OP[op] if isinstance(op, str) else int(op)
        check(self._lib.cpc_apply_op(self._h, o, r.data_ptr(), z.data_ptr()))
        return z

    def spmv(self, x: torch.Tensor, level: int = 0) -> torch.Tensor:
        n_l = self.hierarchy()["n"][level]
        x = _dev_vec(x, n_l, "x")
        y = torch.empty_like(x)
        check(self._lib.cpc_spmv(self._h, int(level), x.data_ptr(), y.data_ptr()))
        return y

    def neg_outer(self, lam: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
        lam = _dev_vec(lam, self.n, "lam")
        x = _dev_vec(x, self.n, "x")
        g = torch.empty(self.nnz, dtype=torch.float64, device=lam.device)
        check(self._lib.cpc_neg_outer_on_pattern(self._h, lam.data_ptr(), x.data_ptr(), g.data_ptr()))
        return g

    # -- hierarchy and statistics
    def hierarchy(self) -> dict:
        cap = 64
        nlev = ctypes.c_int32(0)
        n_l = np.zeros(cap, np.int32)
        nnz_l = np.zeros(cap, np.int64)
        depth = np.zeros(cap, np.int32)
        check(self._lib.cpc_hierarchy_info(self._h, ctypes.byref(nlev), _ptr(n_l), _ptr(nnz_l), _ptr(depth)))
        k = nlev.value
        kinds, rows, inv_bytes = [], [], []
        for d in range(k):
            kind = ctypes.c_int32(0)
            br = ctypes.c_int32(0)
            nb = ctypes.c_int64(0)
            check(self._lib.cpc_smoother_kind(self._h, d, ctypes.byref(kind), ctypes.byref(br)))
            check(self._lib.cpc_smoother_bytes(self._h, d, ctypes.byref(nb)))
            kinds.append({-1: "none", 0: "sweep", 1: "dense", 2: "block"}[kind.value])
            rows.append(br.value)
            inv_bytes.append(nb.value)
        return {"nlev": k, "n": n_l[:k].tolist(), "nnz": nnz_l[:k].tolist(), "depth": depth[:k].tolist(),
                "smoother": kinds, "block_rows": rows, "inverse_bytes": inv_bytes}

    def level(self, level: int):
        info = self.hierarchy()
        n_l, nnz = info["n"][level], info["nnz"][level]
        rp = np.empty(n_l + 1, np.int32)
        ci = np.empty(max(nnz, 1), np.int32)
        v = np.empty(max(nnz, 1), np.float64)
        check(self._lib.cpc_get_level(self._h, int(level), _ptr(rp), _ptr(ci), _ptr(v)))
        return rp, ci[:nnz], v[:nnz]

    def prolongation(self, level: int):
        info = self.hierarchy()
        n_l = info["n"][level]
        nnz = ctypes.c_int64(0)
        check(self._lib.cpc_get_prolongation(self._h, int(level), ctypes.byref(nnz), None, None, None, None))
        rp = np.empty(n_l + 1, np.int32)
        ci = np.empty(max(nnz.value, 1), np.int32)
        v = np.empty(max(nnz.value, 1), np.float64)
        cf = np.empty(n_l, np.int32)
        check(self._lib.cpc_get_prolongation(self._h, int(level), ctypes.byref(nnz), _ptr(rp), _ptr(ci), _ptr(v),
                                             _ptr(cf)))
        return rp, ci[: nnz.value], v[: nnz.value], cf

    def ilu(self) -> np.ndarray:
        out = np.empty(self.nnz, np.float64)
        check(self._lib.cpc_get_ilu(self._h, _ptr(out)))
        return out

    def ilu_factor(self):
        """The ILU(k) factor applied as B: (row_ptr, col, values), L strictly lower with a
        unit diagonal implied, U on and above the diagonal."""
        nnz = ctypes.c_int64(0)
        check(self._lib.cpc_get_ilu_factor(self._h, ctypes.byref(nnz), None, None, None))
        rp = np.empty(self.n + 1, np.int32)
        ci = np.empty(nnz.value, np.int32)
        v = np.empty(nnz.value, np.float64)
        check(self._lib.cpc_get_ilu_factor(self._h, ctypes.byref(nnz), _ptr(rp), _ptr(ci), _ptr(v)))
        return rp, ci, v

    def time_kernel(self, kernel: str | int, level: int = -1, reps: int = 10) -> dict:
        """HIP-event timing of one kernel family (see cpc_time_kernel)."""
        k = _lib.KERNEL[kernel] if isinstance(kernel, str) else int(kernel)
        ms = ctypes.c_double(0.0)
        b = ctypes.c_double(0.0)
        fb = ctypes.c_double(0.0)
        nl = ctypes.c_int32(0)
        check(self._lib.cpc_time_kernel(self._h, k, int(level), int(reps), ctypes.byref(ms), ctypes.byref(b),
                                        ctypes.byref(nl), ctypes.byref(fb)))
        return {"avg_ms": ms.value, "bytes": b.value, "form_bytes": fb.value, "launches": nl.value}

    def stats(self) -> dict:
        s = _lib.Stats()
        check(self._lib.cpc_get_stats(self._h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in _lib.Stats._fields_}


class BatchSolver:
    """Independent systems of different sizes set up and solved together
    (cpc_setup_batch / cpc_solve_batch). Vectors are concatenated in system order."""

    def __init__(self, systems, device="cuda", **opts):
        lib = load()
        self._lib = lib
        self.device = torch.device(device)
        mats = [(int(n), _host(rp, np.int32), _host(ci, np.int32), _host(v, np.float64)) for n, rp, ci, v in systems]
        self.nsys = len(mats)
        ns = np.array([m[0] for m in mats], np.int32)
        P = ctypes.c_void_p
        rps = (P * self.nsys)(*[m[1].ctypes.data for m in mats])
        cis = (P * self.nsys)(*[m[2].ctypes.data for m in mats])
        vals = (P * self.nsys)(*[m[3].ctypes.data for m in mats])
        self._keep = mats
        self._opts = options(**opts)
        h = ctypes.c_void_p()
        stream = None
        if self.device.type == "cuda" and torch.cuda.is_available():
            stream = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream or None)
        check(lib.cpc_setup_batch(self.nsys, _ptr(ns), rps, cis, vals, ctypes.byref(self._opts), stream,
                                  ctypes.byref(h)))
        self._h = h
        self._keep = None
        nsys = ctypes.c_int32(0)
        self.sizes = np.zeros(self.nsys, np.int32)
        self.offsets = np.zeros(self.nsys, np.int32)
        check(lib.cpc_batch_info(h, ctypes.byref(nsys), _ptr(self.sizes), _ptr(self.offsets)))
        self.n = int(self.sizes.sum())

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.cpc_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def solve(self, b: torch.Tensor, x: torch.Tensor | None = None, tol: float = 1e-8, maxit: int = 10000):
        """Returns (x, iters[nsys], relres[nsys], status)."""
        b = _dev_vec(b, self.n, "b")
        x = torch.empty_like(b) if x is None else _dev_vec(x, self.n, "x")
        it = np.zeros(self.nsys, np.int32)
        rel = np.zeros(self.nsys, np.float64)
        st = self._lib.cpc_solve_batch(self._h, b.data_ptr(), x.data_ptr(), float(tol), int(maxit), _ptr(it),
                                       _ptr(rel))
        check(st, allow=(_lib.CPC_OK, _lib.CPC_E_MAXIT, _lib.CPC_E_BREAKDOWN))
        return x, it, rel, st

    def hierarchy(self) -> dict:
        return Solver.hierarchy(self)

    def time_kernel(self, kernel, level=-1, reps=10):
        return Solver.time_kernel(self, kernel, level, reps)

    def stats(self) -> dict:
        return Solver.stats(self)


def spgemm(x, y, ncols: int):
    """C = X Y on the GPU with the Galerkin products' canonical order (cpc_spgemm).
    x, y: (row_ptr, col, val) host CSR triples (X: nrows x len(y row_ptr) - 1).
    Returns (row_ptr, col, val) of C, columns sorted within each row."""
    lib = load()
    xrp, xci, xv = _host(x[0], np.int32), _host(x[1], np.int32), _host(x[2], np.float64)
    yrp, yci, yv = _host(y[0], np.int32), _host(y[1], np.int32), _host(y[2], np.float64)
    nrows, ninner = xrp.size - 1, yrp.size - 1
    crp = np.empty(nrows + 1, np.int32)
    nnz = ctypes.c_int64(0)
    check(lib.cpc_spgemm(nrows, ninner, int(ncols), _ptr(xrp), _ptr(xci), _ptr(xv), _ptr(yrp), _ptr(yci), _ptr(yv),
                         _ptr(crp), None, None, ctypes.byref(nnz)))
    cci = np.empty(max(nnz.value, 1), np.int32)
    cv = np.empty(max(nnz.value, 1), np.float64)
    check(lib.cpc_spgemm(nrows, ninner, int(ncols), _ptr(xrp), _ptr(xci), _ptr(xv), _ptr(yrp), _ptr(yci), _ptr(yv),
                         _ptr(crp), _ptr(cci), _ptr(cv), ctypes.byref(nnz)))
    return crp, cci[:nnz.value], cv[:nnz.value]


def setup_status(n, row_ptr, col, val, **opts) -> tuple[int, str]:
    """Run cpc_setup and return (status, message) without raising (host-side checks)."""
    lib = load()
    rp = _host(row_ptr, np.int32)
    ci = _host(col, np.int32)
    v = _host(val, np.float64)
    o = options(**opts)
    h = ctypes.c_void_p()
    st = lib.cpc_setup(int(n), _ptr(rp), _ptr(ci), _ptr(v), ctypes.byref(o), None, ctypes.byref(h))
    if h.value:
        lib.cpc_destroy(h)
    return st, _lib.last_error()


__all__ = ["Solver", "BatchSolver", "CpcError", "options", "setup_status"]
