"""Cell-centred two-point-flux (TPFA) pressure matrices with seeded heterogeneous
permeability.

The paper's experiments use mixed-hybrid FEM systems from real reservoirs
(Section 5, Table 5.1) that are not available. These generators stand in for
them: scalar pressure equations -div(k grad p) = f (the model problem of
Section 4 with c = 0) on unit cubic cells, with permeability fields whose
heterogeneity is of the same kind (lognormal, strongly varying, channelised).

Conventions (fixed for every generator here):
  * cell (i, j, k) has index i + nx*(j + ny*k); x is fastest, k = 0 is the top layer;
    fields are stored as arrays of shape (nz, ny, nx);
  * interior face transmissibility T = 2 k_a k_b / (k_a + k_b) (harmonic mean over
    two half cells of unit size); x/y faces use k, z faces use kz = kz_ratio * k;
  * a Dirichlet face (p = 0) adds T_b = 2 k to the diagonal and nothing to the RHS;
  * matrix rows: a_ii = sum of the cell's face transmissibilities, a_ij = -T_ij;
    columns are sorted within each row;
  * random numbers come from numpy.random.default_rng(seed) in the order written
    in each function.
Nothing in this module solves, factors or coarsens anything.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Problem:
    name: str
    n: int
    row_ptr: np.ndarray  # int32 [n+1]
    col: np.ndarray  # int32 [nnz]
    val: np.ndarray  # float64 [nnz]
    b: np.ndarray  # float64 [n]
    tol: float
    dims: tuple  # (nx, ny, nz)
    logk: np.ndarray  # float64 (nz, ny, nx)
    kz_ratio: float
    dirichlet_x: bool
    keep: np.ndarray | None = None  # cell index of each unknown when cells were eliminated
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])


def correlated_field(shape, corr_len: float, rng: np.random.Generator) -> np.ndarray:
    """Gaussian random field with correlation exp(-r^2 / (2 l^2)).

    White N(0,1) noise is convolved periodically (FFT) with exp(-r^2 / l^2) and
    the result is standardised to empirical mean 0 and standard deviation 1.
    One standard_normal draw of the full shape is taken from rng.
    """
    shape = tuple(int(s) for s in shape)
    w = rng.standard_normal(shape)
    r2 = np.zeros(shape)
    for ax, s in enumerate(shape):
        d = np.arange(s)
        d = np.minimum(d, s - d).astype(np.float64)
        bshape = [1] * len(shape)
        bshape[ax] = s
        r2 = r2 + (d * d).reshape(bshape)
    kern = np.exp(-r2 / (corr_len * corr_len))
    axes = list(range(len(shape)))
    f = np.fft.irfftn(np.fft.rfftn(w, axes=axes) * np.fft.rfftn(kern, axes=axes), s=shape, axes=axes)
    f = f - f.mean()
    return f / f.std()


def channel_facies(nx: int, ny: int, rng: np.random.Generator, nchan: int = 3) -> np.ndarray:
    """Boolean (ny, nx) mask of sinuous channels running along y.

    For each channel, in this order: x0 ~ U[0, nx), a ~ U[2, 8], lam ~ U[40, 120],
    phi ~ U[0, 2 pi), width ~ U{3..7}. Cell (i, j) is in the channel when
    |i - (x0 + a sin(2 pi j / lam + phi))| < width / 2.
    """
    mask = np.zeros((ny, nx), dtype=bool)
    ii = np.arange(nx)[None, :].astype(np.float64)
    jj = np.arange(ny)[:, None].astype(np.float64)
    for _ in range(nchan):
        x0 = rng.uniform(0.0, float(nx))
        a = rng.uniform(2.0, 8.0)
        lam = rng.uniform(40.0, 120.0)
        phi = rng.uniform(0.0, 2.0 * math.pi)
        width = int(rng.integers(3, 8))
        centre = x0 + a * np.sin(2.0 * math.pi * jj / lam + phi)
        mask |= np.abs(ii - centre) < 0.5 * width
    return mask


def tpfa_system(logk: np.ndarray, kz_ratio: float = 1.0, dirichlet_x: bool = True,
                wells=()):
    """Assemble the TPFA matrix for log-permeability `logk` of shape (nz, ny, nx).

    dirichlet_x: p = 0 on the x = 0 and x = nx faces of the box (other faces no-flow).
    wells: (i, j) columns whose cells have p = 0 for every k; those unknowns are
        eliminated (their face transmissibilities stay on the neighbours' diagonals).
    Returns (row_ptr int32, col int32, val float64, keep int64) where keep[r] is the
    cell index of unknown r.
    """
    logk = np.asarray(logk, dtype=np.float64)
    if logk.ndim == 2:
        logk = logk[None, :, :]
    nz, ny, nx = logk.shape
    N = nx * ny * nz
    k = np.exp(logk).ravel()
    idx = np.arange(N, dtype=np.int64)
    ci = idx % nx
    cj = (idx // nx) % ny
    ck = idx // (nx * ny)

    def face_t(ka, kb):
        return 2.0 * ka * kb / (ka + kb)

    # neighbour offsets in increasing column order: zm, ym, xm, xp, yp, zp
    dirs = [
        (ck > 0, -nx * ny, kz_ratio),
        (cj > 0, -nx, 1.0),
        (ci > 0, -1, 1.0),
        (ci < nx - 1, 1, 1.0),
        (cj < ny - 1, nx, 1.0),
        (ck < nz - 1, nx * ny, kz_ratio),
    ]
    nb_idx = []
    nb_t = []
    diag = np.zeros(N)
    for valid, off, ratio in dirs:
        nb = np.where(valid, idx + off, 0)
        t = np.where(valid, face_t(ratio * k, ratio * k[nb]), 0.0)
        diag += t
        nb_idx.append(np.where(valid, nb, -1))
        nb_t.append(t)
    if dirichlet_x:
        diag += np.where(ci == 0, 2.0 * k, 0.0)
        diag += np.where(ci == nx - 1, 2.0 * k, 0.0)

    removed = np.zeros(N, dtype=bool)
    for (wi, wj) in wells:
        removed[(ci == wi) & (cj == wj)] = True
    keep = np.nonzero(~removed)[0]
    newidx = np.full(N, -1, dtype=np.int64)
    newidx[keep] = np.arange(keep.size)

    cols = np.full((N, 7), -1, dtype=np.int64)
    vals = np.zeros((N, 7))
    slot = [0, 1, 2, 4, 5, 6]
    for s, nb, t in zip(slot, nb_idx, nb_t):
        ok = nb >= 0
        ok[ok] &= ~removed[nb[ok]]
        cols[ok, s] = newidx[nb[ok]]
        vals[ok, s] = -t[ok]
    cols[:, 3] = newidx
    vals[:, 3] = diag
    cols = cols[keep]
    vals = vals[keep]
    mask = cols >= 0
    counts = mask.sum(axis=1)
    row_ptr = np.zeros(keep.size + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = cols[mask].astype(np.int32)
    val = vals[mask]
    return row_ptr.astype(np.int32), col, val, keep


def _problem(name, logk, kz_ratio, dirichlet_x, wells, b_fn, tol, meta=None):
    rp, col, val, keep = tpfa_system(logk, kz_ratio, dirichlet_x, wells)
    n = rp.size - 1
    b = b_fn(n)
    lk = logk if logk.ndim == 3 else logk[None]
    nz, ny, nx = lk.shape
    return Problem(name=name, n=n, row_ptr=rp, col=col, val=val, b=np.ascontiguousarray(b, dtype=np.float64),
                   tol=tol, dims=(nx, ny, nz), logk=lk, kz_ratio=kz_ratio, dirichlet_x=dirichlet_x,
                   keep=None if keep.size == nx * ny * nz else keep, meta=dict(meta or {}))


def _normal_rhs(seed):
    return lambda n: np.random.default_rng(seed).standard_normal(n)


def config1(nx: int = 64, ny: int = 64) -> Problem:
    """2-D nx x ny, log k ~ N(0,1) i.i.d. (seed 1), Dirichlet x-faces, b = e at cell (nx/2, ny/2)."""
    rng = np.random.default_rng(1)
    logk = rng.standard_normal((1, ny, nx))

    def rhs(n):
        b = np.zeros(n)
        b[nx // 2 + nx * (ny // 2)] = 1.0
        return b

    return _problem(f"2d-{nx}x{ny}-lognormal-iid", logk, 1.0, True, (), rhs, 1e-8)


def config2(nx: int = 128, ny: int = 128, nz: int = 64, wells=((32, 32), (95, 95))) -> Problem:
    """3-D nx x ny x nz, correlated log k (sigma 2, l = 8, seed 2), kz/kx = 0.1, no-flow outer
    faces, p = 0 on two vertical well columns (eliminated), b ~ N(0,1) (seed 12)."""
    rng = np.random.default_rng(2)
    logk = 2.0 * correlated_field((nz, ny, nx), 8.0, rng)
    return _problem(f"3d-{nx}x{ny}x{nz}-corr-sigma2-wells", logk, 0.1, False, wells, _normal_rhs(12), 1e-8)


def config3(nx: int = 60, ny: int = 220, nz: int = 85, ntop: int = 35) -> Problem:
    """3-D nx x ny x nz: top `ntop` layers independent 2-D correlated fields (l = 8, sigma 3),
    remaining layers binary facies (background k = 1, three channels of k = 1000 per layer),
    kz/kx = 0.01, Dirichlet x-faces, b ~ N(0,1) (seed 13). Seed 3 drives the field: all top
    layers are drawn first, then the channel layers in order."""
    rng = np.random.default_rng(3)
    logk = np.zeros((nz, ny, nx))
    for kk in range(min(ntop, nz)):
        logk[kk] = 3.0 * correlated_field((ny, nx), 8.0, rng)
    for kk in range(min(ntop, nz), nz):
        m = channel_facies(nx, ny, rng)
        logk[kk] = np.where(m, math.log(1000.0), 0.0)
    return _problem(f"3d-{nx}x{ny}x{nz}-layered-channels", logk, 0.01, True, (), _normal_rhs(13), 1e-8)


def config4_sizes(nsys: int = 64, lo: int = 32, hi: int = 96, seed: int = 4):
    """Edge lengths m_s ~ UniformInt[lo, hi] (inclusive) of the batch systems."""
    return [int(m) for m in np.random.default_rng(seed).integers(lo, hi + 1, size=nsys)]


def config4(nsys: int = 64, lo: int = 32, hi: int = 96, sizes=None):
    """Batch of independent m^3 systems: log k ~ N(0, 2^2) i.i.d. (seed 4000+s), Dirichlet
    x-faces, kz/kx = 1, b ~ N(0,1) (seed 5000+s)."""
    if sizes is None:
        sizes = config4_sizes(nsys, lo, hi)
    out = []
    for s, m in enumerate(sizes):
        logk = 2.0 * np.random.default_rng(4000 + s).standard_normal((m, m, m))
        out.append(_problem(f"batch{s}-{m}^3", logk, 1.0, True, (), _normal_rhs(5000 + s), 1e-8, {"m": m}))
    return out


def config5(nx: int = 96, ny: int = 96, nz: int = 48, nobs: int = 200, nfd: int = 20) -> Problem:
    """Differentiable-solve workload: correlated log k (sigma 2, l = 6, seed 5), kz/kx = 1,
    Dirichlet x-faces, b ~ N(0,1) (seed 15); `nobs` observation cells drawn without
    replacement (seed 7); observed data d ~ N(0,1) (seed 6); `nfd` finite-difference
    check cells drawn without replacement (seed 8)."""
    rng = np.random.default_rng(5)
    logk = 2.0 * correlated_field((nz, ny, nx), 6.0, rng)
    p = _problem(f"3d-{nx}x{ny}x{nz}-corr-sigma2-adjoint", logk, 1.0, True, (), _normal_rhs(15), 1e-8)
    N = nx * ny * nz
    p.meta["obs"] = np.sort(np.random.default_rng(7).choice(N, size=min(nobs, N), replace=False)).astype(np.int64)
    p.meta["d"] = np.random.default_rng(6).standard_normal(p.meta["obs"].size)
    p.meta["fd_cells"] = np.random.default_rng(8).choice(N, size=min(nfd, N), replace=False).astype(np.int64)
    return p


def scaled_config(which: int, scale: float) -> Problem:
    """Same recipe as config `which` (1, 2, 3 or 5) on a grid shrunk by `scale` per axis,
    for parity cases the oracle finishes in seconds."""
    def sz(v):
        return max(2, int(round(v * scale)))
    if which == 1:
        return config1(sz(64), sz(64))
    if which == 2:
        nx, ny = sz(128), sz(128)
        return config2(nx, ny, sz(64), wells=((nx // 4, ny // 4), (3 * nx // 4 - 1, 3 * ny // 4 - 1)))
    if which == 3:
        return config3(sz(60), sz(220), sz(85), ntop=max(1, int(round(35 * scale))))
    if which == 5:
        return config5(sz(96), sz(96), sz(48), nobs=min(200, sz(96) * sz(96) * sz(48) // 4), nfd=5)
    raise ValueError(which)


def csr_to_dense(n, row_ptr, col, val) -> np.ndarray:
    a = np.zeros((n, n))
    rows = np.repeat(np.arange(n), np.diff(np.asarray(row_ptr, dtype=np.int64)))
    a[rows, np.asarray(col)] = np.asarray(val)
    return a
