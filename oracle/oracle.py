"""ctypes wrapper around the plain-C oracle, plus the NumPy parts of the oracle.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline of the benchmark; never by the product library.

The C part (cpc_oracle.c) holds the method: ILU(0) (Algorithm 3.1, k = 0), the
classical AMG setup and V-cycle (Section 3.2, Algorithm 3.2), the combined
preconditioner (Algorithm 2.1) and PCG. This module adds the gradient of a
least-squares misfit through the TPFA matrix (the differentiable form), written
from the chain rule in NumPy.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

OR_OK, OR_E_ARG, OR_E_NOT_SPD, OR_E_BREAKDOWN, OR_E_MAXIT, OR_E_NOMEM = 0, 1, 2, 3, 4, 6
PREC_COMBINED, PREC_AMG, PREC_ILU, PREC_ADDITIVE, PREC_NONE = 0, 1, 2, 3, 4
OP_VCYCLE, OP_FGS, OP_BGS, OP_COMBINED_GS, OP_COMBINED_SWAP = 5, 6, 7, 8, 9
PREC_AMG_ILU, PREC_BBAR = 10, 11

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "cpc_oracle.c"
_LIB = _HERE / "liboracle.so"
_lib = None


class _Opts(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_double), ("max_coarse", ctypes.c_int),
                ("max_levels", ctypes.c_int), ("check_symmetry", ctypes.c_int),
                ("s_scale", ctypes.c_double), ("b_scale", ctypes.c_double), ("ilu_k", ctypes.c_int)]


def build_oracle(force: bool = False) -> Path:
    """Compile the C oracle with gcc (no FMA contraction)."""
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB.with_suffix(".so.tmp")
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o", str(tmp),
                               str(_SRC), "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build_oracle()
    lib = ctypes.CDLL(str(_LIB))
    P = ctypes.c_void_p
    I = ctypes.c_int
    D = ctypes.c_double
    lib.or_setup.restype = P
    lib.or_setup.argtypes = [I, P, P, P, ctypes.POINTER(_Opts), ctypes.POINTER(I)]
    lib.or_free.argtypes = [P]
    lib.or_validate.argtypes = [I, P, P, P, I]
    lib.or_ilu0.argtypes = [I, P, P, P, P]
    lib.or_rs_split.argtypes = [I, P, P, P, D, P]
    lib.or_apply.argtypes = [P, I, P, P]
    lib.or_pcg.argtypes = [P, I, P, P, I, D, I, ctypes.POINTER(I), P, ctypes.POINTER(D)]
    lib.or_nlev.argtypes = [P]
    lib.or_level_n.argtypes = [P, I]
    lib.or_level_nnz.argtypes = [P, I]
    lib.or_level_nnz.restype = ctypes.c_long
    lib.or_p_nnz.argtypes = [P, I]
    lib.or_p_nnz.restype = ctypes.c_long
    lib.or_get_level.argtypes = [P, I, P, P, P]
    lib.or_get_p.argtypes = [P, I, P, P, P]
    lib.or_get_cf.argtypes = [P, I, P]
    lib.or_get_ilu.argtypes = [P, P]
    lib.or_ilu_nnz.argtypes = [P]
    lib.or_ilu_nnz.restype = ctypes.c_long
    lib.or_get_ilu_factor.argtypes = [P, P, P, P, P]
    lib.or_get_chol.argtypes = [P, P]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _csr_args(row_ptr, col, val):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col, dtype=np.int32)
    v = np.ascontiguousarray(val, dtype=np.float64)
    return rp, ci, v


def validate(n, row_ptr, col, val, check_symmetry=True) -> int:
    lib = _load()
    rp, ci, v = _csr_args(row_ptr, col, val)
    return lib.or_validate(int(n), _ptr(rp), _ptr(ci), _ptr(v), int(bool(check_symmetry)))


def ilu0(n, row_ptr, col, val):
    """ILU(0) values on the pattern of A (strict lower = L, rest = U) and status."""
    lib = _load()
    rp, ci, v = _csr_args(row_ptr, col, val)
    lu = np.empty_like(v)
    st = lib.or_ilu0(int(n), _ptr(rp), _ptr(ci), _ptr(v), _ptr(lu))
    return lu, st


def rs_split(n, row_ptr, col, val, theta=0.25):
    """Classical C/F splitting (1 = C, 0 = F) of one level and the number of C points."""
    lib = _load()
    rp, ci, v = _csr_args(row_ptr, col, val)
    cf = np.empty(n, dtype=np.int32)
    nc = lib.or_rs_split(int(n), _ptr(rp), _ptr(ci), _ptr(v), float(theta), _ptr(cf))
    return cf, nc


class Hierarchy:
    """SETUP of the oracle: ILU(0) factors + classical AMG hierarchy."""

    def __init__(self, n, row_ptr, col, val, theta=0.25, max_coarse=256, max_levels=25,
                 check_symmetry=True, s_scale=1.0, b_scale=1.0, ilu_k=0):
        lib = _load()
        self._lib = lib
        self.n = int(n)
        rp, ci, v = _csr_args(row_ptr, col, val)
        o = _Opts(float(theta), int(max_coarse), int(max_levels), int(bool(check_symmetry)),
                  float(s_scale), float(b_scale), int(ilu_k))
        st = ctypes.c_int(0)
        self._h = lib.or_setup(self.n, _ptr(rp), _ptr(ci), _ptr(v), ctypes.byref(o), ctypes.byref(st))
        self.status = st.value
        if not self._h:
            raise OracleError(self.status)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.or_free(h)
            self._h = None

    @property
    def nlev(self) -> int:
        return self._lib.or_nlev(self._h)

    def level(self, d: int):
        n = self._lib.or_level_n(self._h, d)
        nnz = self._lib.or_level_nnz(self._h, d)
        rp = np.empty(n + 1, np.int32)
        ci = np.empty(nnz, np.int32)
        v = np.empty(nnz, np.float64)
        self._lib.or_get_level(self._h, d, _ptr(rp), _ptr(ci), _ptr(v))
        return rp, ci, v

    def prolongation(self, d: int):
        n = self._lib.or_level_n(self._h, d)
        nnz = self._lib.or_p_nnz(self._h, d)
        rp = np.empty(n + 1, np.int32)
        ci = np.empty(max(nnz, 1), np.int32)
        v = np.empty(max(nnz, 1), np.float64)
        self._lib.or_get_p(self._h, d, _ptr(rp), _ptr(ci), _ptr(v))
        return rp, ci[:nnz], v[:nnz]

    def cf(self, d: int):
        n = self._lib.or_level_n(self._h, d)
        out = np.empty(n, np.int32)
        self._lib.or_get_cf(self._h, d, _ptr(out))
        return out

    def ilu(self):
        nnz = self._lib.or_level_nnz(self._h, 0)
        out = np.empty(nnz, np.float64)
        self._lib.or_get_ilu(self._h, _ptr(out))
        return out

    def ilu_factor(self):
        """The ILU(k) factor B applies: (row_ptr, col, values, level of fill); L strictly
        lower with unit diagonal implied, U on and above the diagonal."""
        nnz = self._lib.or_ilu_nnz(self._h)
        rp = np.empty(self.n + 1, np.int32)
        ci = np.empty(nnz, np.int32)
        v = np.empty(nnz, np.float64)
        lev = np.empty(nnz, np.int32)
        self._lib.or_get_ilu_factor(self._h, _ptr(rp), _ptr(ci), _ptr(v), _ptr(lev))
        return rp, ci, v, lev

    def coarse_cholesky(self):
        n0 = self._lib.or_level_n(self._h, self.nlev - 1)
        out = np.empty((n0, n0), np.float64)
        self._lib.or_get_chol(self._h, _ptr(out))
        return out

    def level_sizes(self):
        return [(self._lib.or_level_n(self._h, d), self._lib.or_level_nnz(self._h, d)) for d in range(self.nlev)]

    def apply(self, which: int, r: np.ndarray) -> np.ndarray:
        r = np.ascontiguousarray(r, dtype=np.float64)
        z = np.empty_like(r)
        st = self._lib.or_apply(self._h, int(which), _ptr(r), _ptr(z))
        if st:
            raise OracleError(st)
        return z

    def dense_operator(self, which: int) -> np.ndarray:
        """Columns B e_j of a linear operator (tiny problems only)."""
        n = self.n
        out = np.empty((n, n))
        e = np.zeros(n)
        for j in range(n):
            e[:] = 0.0
            e[j] = 1.0
            out[:, j] = self.apply(which, e)
        return out

    def pcg(self, which: int, b: np.ndarray, tol: float, maxit: int, x0: np.ndarray | None = None):
        """Returns dict(x, iters, hist, true_relres, status)."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros_like(b) if x0 is None else np.ascontiguousarray(x0, dtype=np.float64).copy()
        hist = np.zeros(maxit + 1)
        it = ctypes.c_int(0)
        tr = ctypes.c_double(0.0)
        st = self._lib.or_pcg(self._h, int(which), _ptr(b), _ptr(x), int(x0 is not None), float(tol), int(maxit),
                              ctypes.byref(it), _ptr(hist), ctypes.byref(tr))
        return {"x": x, "iters": it.value, "hist": hist[: it.value + 1].copy(), "true_relres": tr.value,
                "status": st}


class OracleError(RuntimeError):
    def __init__(self, status):
        super().__init__(f"oracle status {status}")
        self.status = status


# ---------------------------------------------------------------------------
# Gradient of L = 1/2 || x[obs] - d ||^2 with A(log k) x = b (the differentiable
# form). Adjoint: A^T lam = P^T (P x - d), A = A^T. Then dL/db = lam and
# dL/dA_ij = -lam_i x_j. With a_ii = sum_f T_f (+ T_b), a_ij = -T_f, one interior
# face f = (i, j) contributes dL/dT_f = -(lam_i - lam_j)(x_i - x_j); a Dirichlet
# face of cell c contributes dL/dT_b = -lam_c x_c. The chain rule to log k uses
# T = 2 s k_a k_b / (k_a + k_b) (s = kz_ratio on z faces, 1 otherwise):
# dT/dlog k_a = 2 s k_a k_b^2 / (k_a + k_b)^2, and T_b = 2 k_c: dT_b/dlog k_c = T_b.
# ---------------------------------------------------------------------------

def tpfa_logk_gradient(logk, kz_ratio, dirichlet_x, lam_cells, x_cells, removed=None):
    """dL/dlog k for every cell, given adjoint and state on the full cell grid
    (entries of eliminated cells must be 0, which is their Dirichlet value).
    Faces touching an eliminated (p = 0) cell act like a Dirichlet face:
    dT/dlog k of the kept cell times -(lam_c x_c)."""
    lk = np.asarray(logk, dtype=np.float64)
    if lk.ndim == 2:
        lk = lk[None]
    nz, ny, nx = lk.shape
    k = np.exp(lk)
    lam = np.asarray(lam_cells, dtype=np.float64).reshape(nz, ny, nx)
    x = np.asarray(x_cells, dtype=np.float64).reshape(nz, ny, nx)
    g = np.zeros_like(k)
    for axis, s in ((2, 1.0), (1, 1.0), (0, kz_ratio)):
        if lk.shape[axis] < 2:
            continue
        sl_a = [slice(None)] * 3
        sl_b = [slice(None)] * 3
        sl_a[axis] = slice(0, -1)
        sl_b[axis] = slice(1, None)
        sl_a, sl_b = tuple(sl_a), tuple(sl_b)
        ka, kb = s * k[sl_a], s * k[sl_b]
        dT_da = 2.0 * ka * kb * kb / (ka + kb) ** 2
        dT_db = 2.0 * kb * ka * ka / (ka + kb) ** 2
        dL_dT = -(lam[sl_a] - lam[sl_b]) * (x[sl_a] - x[sl_b])
        g[sl_a] += dT_da * dL_dT
        g[sl_b] += dT_db * dL_dT
    if dirichlet_x:
        tb = 2.0 * k
        g[:, :, 0] += -tb[:, :, 0] * lam[:, :, 0] * x[:, :, 0]
        g[:, :, nx - 1] += -tb[:, :, nx - 1] * lam[:, :, nx - 1] * x[:, :, nx - 1]
    if removed is not None:
        g.reshape(-1)[np.asarray(removed)] = 0.0
    return g.reshape(-1)


def misfit_gradient(problem, hier: Hierarchy, tol=1e-12, maxit=10000, which=PREC_COMBINED):
    """Forward solve, adjoint solve and the gradient of the misfit with respect to
    b and log k, all in the oracle. Returns dict(loss, x, lam, grad_b, grad_logk)."""
    b = problem.b
    fwd = hier.pcg(which, b, tol, maxit)
    x = fwd["x"]
    obs = problem.meta["obs"]
    d = problem.meta["d"]
    cell_of = problem.keep if problem.keep is not None else np.arange(problem.n)
    # observation cells are grid cells; map them to unknowns
    unk = np.full(int(np.prod(problem.logk.shape)), -1, dtype=np.int64)
    unk[cell_of] = np.arange(problem.n)
    ou = unk[obs]
    assert np.all(ou >= 0)
    resid = x[ou] - d
    loss = 0.5 * float(resid @ resid)
    rhs = np.zeros(problem.n)
    np.add.at(rhs, ou, resid)
    adj = hier.pcg(which, rhs, tol, maxit)
    lam = adj["x"]
    N = unk.size
    lam_c = np.zeros(N)
    x_c = np.zeros(N)
    lam_c[cell_of] = lam
    x_c[cell_of] = x
    g = tpfa_logk_gradient(problem.logk, problem.kz_ratio, problem.dirichlet_x, lam_c, x_c)
    return {"loss": loss, "x": x, "lam": lam, "grad_b": lam.copy(), "grad_logk": g,
            "fwd_iters": fwd["iters"], "adj_iters": adj["iters"],
            "fwd_relres": fwd["true_relres"], "adj_relres": adj["true_relres"]}
