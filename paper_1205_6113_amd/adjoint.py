"""Differentiable TPFA solve: x = A(log k)^{-1} b as a torch.autograd.Function.

forward: the TPFA matrix values are assembled on the GPU (cpc_tpfa_values), the
solver is set up on them and PCG with the combined preconditioner solves A x = b.
backward: A is symmetric, so the adjoint lam = A^{-1} (dL/dx) reuses the same
hierarchy and PCG; dL/db = lam, and dL/dlog k comes from cpc_tpfa_logk_grad (the
chain rule through the face transmissibilities, equivalent to contracting the
pattern-restricted -lam x^T of cpc_neg_outer_on_pattern with dA/dlog k).
This module only marshals arguments; every step runs in libcpc.so.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import check, load
from .solver import Solver


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream or None)


@dataclass
class TpfaGrid:
    """Grid of unit cells with the TPFA conventions of cpc.h."""
    nx: int
    ny: int
    nz: int
    kz_ratio: float = 1.0
    dirichlet_x: bool = True

    def __post_init__(self):
        lib = load()
        n = self.nx * self.ny * self.nz
        rp = np.empty(n + 1, np.int32)
        check(lib.cpc_tpfa_pattern(self.nx, self.ny, self.nz, rp.ctypes.data_as(ctypes.c_void_p), None))
        ci = np.empty(int(rp[-1]), np.int32)
        check(lib.cpc_tpfa_pattern(self.nx, self.ny, self.nz, rp.ctypes.data_as(ctypes.c_void_p),
                                   ci.ctypes.data_as(ctypes.c_void_p)))
        self.n = n
        self.row_ptr = rp
        self.col = ci
        self._rp_dev = {}

    def row_ptr_dev(self, device) -> torch.Tensor:
        key = str(device)
        if key not in self._rp_dev:
            self._rp_dev[key] = torch.as_tensor(self.row_ptr, device=device)
        return self._rp_dev[key]

    def values(self, logk: torch.Tensor) -> torch.Tensor:
        """Matrix values (device FP64, CSR order of row_ptr/col) for log k."""
        logk = logk.detach().contiguous()
        assert logk.dtype == torch.float64 and logk.is_cuda and logk.numel() == self.n
        val = torch.empty(int(self.row_ptr[-1]), dtype=torch.float64, device=logk.device)
        check(load().cpc_tpfa_values(self.nx, self.ny, self.nz, float(self.kz_ratio), int(self.dirichlet_x),
                                     logk.data_ptr(), self.row_ptr_dev(logk.device).data_ptr(), val.data_ptr(),
                                     _stream(logk.device)))
        return val

    def logk_grad(self, logk: torch.Tensor, lam: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
        logk = logk.detach().contiguous()
        g = torch.empty_like(logk)
        check(load().cpc_tpfa_logk_grad(self.nx, self.ny, self.nz, float(self.kz_ratio), int(self.dirichlet_x),
                                        logk.data_ptr(), lam.contiguous().data_ptr(), x.contiguous().data_ptr(),
                                        g.data_ptr(), _stream(logk.device)))
        return g


class _TpfaSolveFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, logk, b, grid: TpfaGrid, tol: float, maxit: int, opts: dict, setup):
        if setup is not None:
            # the caller's preconditioner, built for a nearby log k; PCG runs on A(log k)
            x, it, rel, st = setup.solve(logk.detach(), b.detach().contiguous(), tol=tol, maxit=maxit)
            solver = None
        else:
            val = grid.values(logk)
            torch.cuda.current_stream(logk.device).synchronize()
            solver = Solver(grid.n, grid.row_ptr, grid.col, val.cpu().numpy(), device=logk.device, **opts)
            x, it, rel, st = solver.solve(b.detach().contiguous(), tol=tol, maxit=maxit)
        if st != _lib.CPC_OK:
            if solver is not None:
                solver.close()
            raise _lib.CpcError(st, f"forward solve did not converge (iters {it}, relres {rel:.3e})")
        ctx.solver = solver
        ctx.setup = setup
        ctx.grid = grid
        ctx.tol = tol
        ctx.maxit = maxit
        ctx.stats = {"forward_iters": it, "forward_relres": rel}
        ctx.save_for_backward(logk.detach(), x)
        return x

    @staticmethod
    def backward(ctx, gx):
        logk, x = ctx.saved_tensors
        if ctx.setup is not None:
            lam, it, rel, st = ctx.setup.solve(logk, gx.detach().contiguous(), tol=ctx.tol, maxit=ctx.maxit)
        else:
            lam, it, rel, st = ctx.solver.solve(gx.detach().contiguous(), tol=ctx.tol, maxit=ctx.maxit)
            ctx.solver.close()
        if st != _lib.CPC_OK:
            raise _lib.CpcError(st, f"adjoint solve did not converge (iters {it}, relres {rel:.3e})")
        grad_logk = ctx.grid.logk_grad(logk, lam, x) if ctx.needs_input_grad[0] else None
        grad_b = lam if ctx.needs_input_grad[1] else None
        return grad_logk, grad_b, None, None, None, None, None


def tpfa_solve(logk: torch.Tensor, b: torch.Tensor, grid: TpfaGrid, tol: float = 1e-10, maxit: int = 10000,
               setup: "FrozenPreconditionerSolve | None" = None, **opts) -> torch.Tensor:
    """x = A(log k)^{-1} b, differentiable with respect to log k and b.

    Without `setup` every call builds the preconditioner for A(log k) (cpc_setup) and
    frees it after the backward pass. With `setup`, a FrozenPreconditionerSolve built
    for a nearby log k0 on the same grid, the forward and the adjoint PCG run on
    A(log k) with the preconditioner of A(log k0): no setup per call. The solution and
    the gradient are those of A(log k) to the tolerance; only the iteration count
    depends on how far log k is from log k0.
    """
    if setup is not None and setup.grid is not grid:
        raise ValueError("setup was built on another grid")
    return _TpfaSolveFn.apply(logk, b, grid, tol, maxit, opts, setup)


class FrozenPreconditionerSolve:
    """Solves with matrices A(log k') near A(log k) while keeping the preconditioner
    built for A(log k) (cpc_set_operator_values): for finite-difference checks, and as
    the `setup` of tpfa_solve, so that a sequence of differentiable solves at nearby
    log k (an optimisation loop) sets up once."""

    def __init__(self, logk: torch.Tensor, grid: TpfaGrid, **opts):
        self.grid = grid
        val = grid.values(logk)
        torch.cuda.current_stream(logk.device).synchronize()
        self.solver = Solver(grid.n, grid.row_ptr, grid.col, val.cpu().numpy(), device=logk.device, **opts)
        self._vals = None

    def solve(self, logk: torch.Tensor, b: torch.Tensor, tol: float = 1e-13, maxit: int = 10000):
        self._vals = self.grid.values(logk)
        check(self.solver._lib.cpc_set_operator_values(self.solver._h, self._vals.data_ptr()))
        x, it, rel, st = self.solver.solve(b, tol=tol, maxit=maxit)
        check(self.solver._lib.cpc_set_operator_values(self.solver._h, None))
        return x, it, rel, st

    def close(self):
        self.solver.close()
