"""Symmetric M-matrices with long rows: every unknown of a 1-D chain coupled to a
random subset of its `band` nearest neighbours on each side.

Galerkin coarse levels of large 3-D pressure systems carry rows of well over a
hundred entries; this generator gives the finest level such rows at a size the tests
can afford. With numpy.random.default_rng(seed): first the upper weights, an (n, band)
array uniform on [0.1, 1) (entry [i, k] for the coupling (i, i + k + 1)), then an
(n, band) array uniform on [0, 1) keeping the couplings below `density` (k = 0 always
kept, so the chain stays connected); w_ij = w_ji, a_ij = -w_ij,
a_ii = (1 + shift) * sum_j w_ij. Holes in the band keep ILU(0) from being the exact
factorisation. Nothing here solves anything.
"""
from __future__ import annotations

import numpy as np

from .tpfa import Problem


def wide_band(n: int = 12000, band: int = 160, density: float = 0.6, shift: float = 1e-3,
              seed: int = 9) -> Problem:
    rng = np.random.default_rng(seed)
    up = rng.uniform(0.1, 1.0, (n, band))  # up[i, k]: weight of the coupling (i, i + k + 1)
    on = rng.uniform(0.0, 1.0, (n, band)) < density
    on[:, 0] = True
    rows = np.repeat(np.arange(n), 2 * band + 1)
    offs = np.tile(np.arange(-band, band + 1), n)
    cols = rows + offs
    keep = (cols >= 0) & (cols < n)
    rows, offs, cols = rows[keep], offs[keep], cols[keep]
    lo = np.minimum(rows, cols)
    k = np.abs(offs) - 1
    keep = (offs == 0) | on[lo, np.maximum(k, 0)]
    rows, offs, cols, lo, k = rows[keep], offs[keep], cols[keep], lo[keep], k[keep]
    w = np.where(offs == 0, 0.0, up[lo, np.maximum(k, 0)])
    rs = np.bincount(rows, weights=w, minlength=n)
    val = np.where(offs == 0, (1.0 + shift) * rs[rows], -w)
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rp[1:])
    b = np.random.default_rng(seed + 100).standard_normal(n)
    return Problem(name=f"chain-{n}-band{band}-{density}", n=n, row_ptr=rp.astype(np.int32), col=cols.astype(np.int32),
                   val=np.ascontiguousarray(val), b=b, tol=1e-8, dims=(n, 1, 1), logk=np.zeros((1, 1, n)),
                   kz_ratio=1.0, dirichlet_x=False)


def hub_chain(nc: int = 8400, seed: int = 3) -> Problem:
    """A chain of nc unknowns, every one weakly coupled to a hub (unknown 0) that is
    itself strongly coupled to an anchor (unknown 1); chain unknown i is 2 + i.

    With numpy.random.default_rng(seed): chain couplings uniform on [0.5, 1.5), hub
    couplings uniform on [0.05, 0.1), then diagonal shifts uniform on [0.01, 0.1) added
    to the negated row sums; anchor coupling 100. The hub row holds every chain unknown,
    so the Galerkin products of the hub's row (and, one level down, of the coarse hub)
    have more than nc / 2 distinct columns: a well column seen by a whole reservoir
    layer. Nothing here solves anything."""
    rng = np.random.default_rng(seed)
    n = nc + 2
    cw = rng.uniform(0.5, 1.5, nc - 1)
    hw = rng.uniform(0.05, 0.1, nc)
    rows, cols, w = [], [], []
    for i in range(nc - 1):
        rows.append(2 + i)
        cols.append(3 + i)
        w.append(cw[i])
    for i in range(nc):
        rows.append(0)
        cols.append(2 + i)
        w.append(hw[i])
    rows.append(0)
    cols.append(1)
    w.append(100.0)
    rows, cols, w = np.array(rows), np.array(cols), np.array(w)
    r = np.concatenate([rows, cols])
    c = np.concatenate([cols, rows])
    v = -np.concatenate([w, w])
    rs = np.bincount(r, weights=-v, minlength=n)
    diag = rs + rng.uniform(0.01, 0.1, n)
    r = np.concatenate([r, np.arange(n)])
    c = np.concatenate([c, np.arange(n)])
    v = np.concatenate([v, diag])
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(r, minlength=n), out=rp[1:])
    b = np.random.default_rng(seed + 100).standard_normal(n)
    return Problem(name=f"hub-chain-{nc}", n=n, row_ptr=rp.astype(np.int32), col=c.astype(np.int32),
                   val=np.ascontiguousarray(v), b=b, tol=1e-8, dims=(n, 1, 1), logk=np.zeros((1, 1, n)),
                   kz_ratio=1.0, dirichlet_x=False)
