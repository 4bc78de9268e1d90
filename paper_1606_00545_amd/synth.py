"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module builds matrices and vectors only. It contains none of the solver's
arithmetic (no products, factorisations or solves): every right-hand side
b = A x_true is formed by whichever side consumes the inputs.

Workloads (the paper's SuiteSparse matrices are not available, so these stand in
for its test problems; the 3D Poisson matrix of Sec. 3.1/3.2 is reproduced
exactly by :func:`poisson3d`):

* :func:`poisson2d` / :func:`poisson3d` -- constant-coefficient 5/7-point
  Dirichlet Poisson operators (diagonal 4 or 6, off-diagonals -1).
* :func:`lognormal_tpfa` -- cell-centred two-point-flux diffusion with
  lognormal cell permeability, harmonic-mean face transmissibilities and a
  half-cell Dirichlet boundary term on the diagonal (a reservoir-like SPD
  M-matrix), optionally with the z transmissibilities scaled.
* :func:`powerlaw_random` -- nonsymmetric random sparse matrix with power-law
  row lengths and a dominant diagonal.

Natural ordering throughout: cell c = x + nx*(y + ny*z). Columns within each CSR
row are strictly ascending and no explicit zeros are stored.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class CSR:
    """Host CSR triple (Ap row starts, Aj column indices, Ax values), int32/float64."""
    n: int
    Ap: np.ndarray
    Aj: np.ndarray
    Ax: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.Ap[-1])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.Ax, self.Aj, self.Ap), shape=(self.n, self.n))


def _assemble(n: int, offsets, valid, values) -> CSR:
    """Assemble a banded matrix from per-offset validity masks and values.

    ``offsets`` must be given in ascending order so that each row's columns come
    out ascending.
    """
    lens = np.zeros(n, dtype=np.int64)
    for m in valid:
        lens += m
    Ap = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=Ap[1:])
    nnz = int(Ap[-1])
    Aj = np.empty(nnz, dtype=np.int32)
    Ax = np.empty(nnz, dtype=np.float64)
    fill = Ap[:-1].copy()
    rows = np.arange(n, dtype=np.int64)
    for d, m, v in zip(offsets, valid, values):
        idx = rows[m]
        pos = fill[idx]
        Aj[pos] = (idx + d).astype(np.int32)
        Ax[pos] = v[m] if isinstance(v, np.ndarray) else v
        fill[idx] += 1
    return CSR(n, Ap.astype(np.int32), Aj, Ax)


def _grid(nx, ny, nz):
    c = np.arange(nx * ny * nz, dtype=np.int64)
    return c % nx, (c // nx) % ny, c // (nx * ny)


def poisson1d(m: int) -> CSR:
    """3-point Dirichlet Poisson on m interior points: 2 on the diagonal, -1 off it."""
    x, _, _ = _grid(m, 1, 1)
    valid = [x > 0, np.ones(m, bool), x < m - 1]
    return _assemble(m, [-1, 0, 1], valid, [-1.0, 2.0, -1.0])


def poisson2d(m: int) -> CSR:
    """5-point Dirichlet Poisson on an m x m interior grid: 4 on the diagonal, -1 off it."""
    n = m * m
    x, y, _ = _grid(m, m, 1)
    offs = [-m, -1, 0, 1, m]
    valid = [y > 0, x > 0, np.ones(n, bool), x < m - 1, y < m - 1]
    vals = [-1.0, -1.0, 4.0, -1.0, -1.0]
    return _assemble(n, offs, valid, vals)


def poisson3d(m: int) -> CSR:
    """7-point Dirichlet Poisson on an m^3 interior grid: 6 on the diagonal, -1 off it."""
    n = m ** 3
    x, y, z = _grid(m, m, m)
    s = m * m
    offs = [-s, -m, -1, 0, 1, m, s]
    valid = [z > 0, y > 0, x > 0, np.ones(n, bool), x < m - 1, y < m - 1, z < m - 1]
    vals = [-1.0, -1.0, -1.0, 6.0, -1.0, -1.0, -1.0]
    return _assemble(n, offs, valid, vals)


def lognormal_tpfa(shape, sigma: float, rng: np.random.Generator,
                   zscale: float = 1.0) -> CSR:
    """Cell-centred TPFA diffusion with lognormal permeability.

    kappa_c = exp(sigma * N(0,1)) per cell; interior face transmissibility is the
    harmonic mean 2 k_c k_d / (k_c + k_d) (unit spacing); a Dirichlet boundary face
    contributes 2 k_c (half-cell distance) to the diagonal only. Faces normal to z
    are multiplied by ``zscale`` (layered anisotropy). ``shape`` is (nx, ny) or
    (nx, ny, nz). The result is a symmetric, weakly diagonally dominant M-matrix.
    """
    if len(shape) == 2:
        nx, ny = shape
        nz = 1
    else:
        nx, ny, nz = shape
    n = nx * ny * nz
    kap = np.exp(sigma * rng.standard_normal(n))
    x, y, z = _grid(nx, ny, nz)
    sxy = nx * ny

    def harm(a, b):
        return 2.0 * a * b / (a + b)

    # transmissibility of the face between c and c+stride (valid where the neighbour exists)
    tx = np.zeros(n)
    ty = np.zeros(n)
    tz = np.zeros(n)
    mx = x < nx - 1
    my = y < ny - 1
    mz = z < nz - 1
    tx[mx] = harm(kap[mx], kap[np.nonzero(mx)[0] + 1])
    ty[my] = harm(kap[my], kap[np.nonzero(my)[0] + nx])
    if nz > 1:
        tz[mz] = zscale * harm(kap[mz], kap[np.nonzero(mz)[0] + sxy])

    # diagonal: sum of the faces, in a fixed order (-z,-y,-x,+x,+y,+z), boundary faces 2*k_c
    diag = np.zeros(n)
    bx = 2.0 * kap
    bz = zscale * 2.0 * kap

    def add(mask_int, t_int, t_bnd):
        return np.where(mask_int, t_int, t_bnd)

    if nz > 1:
        tzm = np.zeros(n)
        tzm[z > 0] = tz[np.nonzero(z > 0)[0] - sxy]
        diag += add(z > 0, tzm, bz)
    tym = np.zeros(n)
    tym[y > 0] = ty[np.nonzero(y > 0)[0] - nx]
    diag += add(y > 0, tym, bx)
    txm = np.zeros(n)
    txm[x > 0] = tx[np.nonzero(x > 0)[0] - 1]
    diag += add(x > 0, txm, bx)
    diag += add(mx, tx, bx)
    diag += add(my, ty, bx)
    if nz > 1:
        diag += add(mz, tz, bz)

    if nz > 1:
        offs = [-sxy, -nx, -1, 0, 1, nx, sxy]
        valid = [z > 0, y > 0, x > 0, np.ones(n, bool), mx, my, mz]
        vals = [-tzm, -tym, -txm, diag, -tx, -ty, -tz]
    else:
        offs = [-nx, -1, 0, 1, nx]
        valid = [y > 0, x > 0, np.ones(n, bool), mx, my]
        vals = [-tym, -txm, diag, -tx, -ty]
    return _assemble(n, offs, valid, vals)


POWERLAW_ALPHA = 2.291427762117685  # P(L) ~ L^-alpha on L = 4..512 has mean 12


def powerlaw_random(n: int, rng: np.random.Generator, lmin: int = 4, lmax: int = 512,
                    alpha: float = POWERLAW_ALPHA) -> CSR:
    """Random nonsymmetric matrix with power-law row lengths and a dominant diagonal.

    Row length L in [lmin, lmax] with P(L) proportional to L^-alpha (mean 12 for the
    defaults). Each row holds its diagonal plus L-1 distinct off-diagonal columns
    drawn uniformly; off-diagonal values ~ N(0,1); diagonal = 1 + sum |off|.
    """
    Ls = np.arange(lmin, lmax + 1, dtype=np.int64)
    w = Ls.astype(np.float64) ** (-alpha)
    cdf = np.cumsum(w / w.sum())
    cdf[-1] = 1.0
    lens = Ls[np.searchsorted(cdf, rng.random(n), side="right").clip(0, len(Ls) - 1)]
    lens = np.minimum(lens, n)
    noff = lens - 1
    rows = np.repeat(np.arange(n, dtype=np.int64), noff)
    m = rows.size
    cols = rng.integers(0, max(n - 1, 1), size=m, dtype=np.int64)
    cols = cols + (cols >= rows)  # skip the diagonal
    # redraw duplicates until every row's off-diagonal columns are distinct
    while True:
        key = rows * n + cols
        order = np.argsort(key, kind="stable")
        ks = key[order]
        dup = np.zeros(m, dtype=bool)
        dup[order[1:][ks[1:] == ks[:-1]]] = True
        nd = int(dup.sum())
        if nd == 0:
            break
        c = rng.integers(0, max(n - 1, 1), size=nd, dtype=np.int64)
        cols[dup] = c + (c >= rows[dup])
    order = np.argsort(rows * n + cols, kind="stable")
    rows = rows[order]
    cols = cols[order]
    offv = rng.standard_normal(m)
    # insert the diagonal in column order
    Ap = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=Ap[1:])
    nnz = int(Ap[-1])
    Aj = np.empty(nnz, dtype=np.int32)
    Ax = np.empty(nnz, dtype=np.float64)
    offstart = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(noff, out=offstart[1:])
    below = np.zeros(n, dtype=np.int64)  # number of off-diagonals left of the diagonal
    lt = cols < rows
    np.add.at(below, rows[lt], 1)
    k = np.arange(m, dtype=np.int64) - offstart[rows]  # rank within the row's off-diagonals
    pos = Ap[rows] + k + (k >= below[rows])
    Aj[pos] = cols.astype(np.int32)
    Ax[pos] = offv
    dpos = Ap[:-1] + below
    Aj[dpos] = np.arange(n, dtype=np.int32)
    absum = np.zeros(n)
    np.add.at(absum, rows, np.abs(offv))
    Ax[dpos] = 1.0 + absum
    return CSR(n, Ap.astype(np.int32), Aj, Ax)


def uniform_vector(n: int, rng: np.random.Generator) -> np.ndarray:
    """x_true ~ U[-1, 1]."""
    return rng.uniform(-1.0, 1.0, n)


# ----------------------------------------------------------------------------
# named workloads


def workload_c1():
    """2D 5-point Poisson, 64x64 interior, seed 1: (A, x_true)."""
    rng = np.random.default_rng(1)
    A = poisson2d(64)
    return A, uniform_vector(A.n, rng)


def workload_diffusion3d(m: int, sigma: float = 2.0, seed: int = 2, zscale: float = 1.0):
    """3D 7-point lognormal TPFA diffusion on an m^3 grid: (A, x_true).

    m=128, sigma=2, seed=2 is the 2.1M-unknown heterogeneous diffusion workload;
    m=192 with zscale=0.01, seed=4 is the anisotropic mixed-precision workload.
    """
    rng = np.random.default_rng(seed)
    A = lognormal_tpfa((m, m, m), sigma, rng, zscale=zscale)
    return A, uniform_vector(A.n, rng)


def circuit_like(n: int, rng: np.random.Generator, nlong: int = 200, long_min: int = 2000,
                 long_max: int = 20000) -> CSR:
    """Banded rows with a few very long ones, the shape of circuit matrices (a stand-in
    for the paper's circuit and power-network test matrices, which are not available).

    Row i holds its diagonal and 2-6 further distinct columns within +-64 of it;
    `nlong` rows (spread evenly) instead hold long_min..long_max distinct random
    columns and the diagonal. Values ~ N(0,1) off the diagonal, diagonal = 1 + sum |off|.
    """
    k = rng.integers(2, 7, size=n)  # further columns drawn per banded row (duplicates merge)
    offs = rng.integers(1, 65, size=(n, 6)) * np.where(rng.random((n, 6)) < 0.5, -1, 1)
    cand = np.clip(np.arange(n)[:, None] + offs, 0, n - 1)
    cand = np.where(np.arange(6)[None, :] < k[:, None], cand, n)  # n marks an unused draw
    cand = np.sort(np.concatenate([cand, np.arange(n)[:, None]], axis=1), axis=1)
    keep = cand < n
    keep[:, 1:] &= cand[:, 1:] != cand[:, :-1]
    long_rows = np.unique(np.linspace(0, n - 1, nlong).astype(np.int64)) if nlong else np.zeros(0, np.int64)
    keep[long_rows] = False
    lens = keep.sum(axis=1).astype(np.int64)
    long_cols = []
    for i in long_rows:
        L = int(rng.integers(long_min, long_max + 1))
        c = np.unique(np.concatenate([rng.choice(n, size=min(L, n), replace=False), [i]]))
        long_cols.append(c)
        lens[i] = c.size
    Ap = np.zeros(n + 1, np.int64)
    np.cumsum(lens, out=Ap[1:])
    Aj = np.empty(int(Ap[-1]), np.int32)
    rank = np.cumsum(keep, axis=1) - 1
    r, j = np.nonzero(keep)
    Aj[Ap[r] + rank[r, j]] = cand[r, j]
    for i, c in zip(long_rows, long_cols):
        Aj[Ap[i]:Ap[i + 1]] = c
    Ax = rng.standard_normal(Aj.size)
    rows = np.repeat(np.arange(n), lens)
    diag = Aj == rows
    Ax[diag] = 0.0
    rowabs = np.zeros(n)
    np.add.at(rowabs, rows, np.abs(Ax))
    Ax[diag] = 1.0 + rowabs[rows[diag]]
    return CSR(n, Ap.astype(np.int32), Aj, Ax)


def workload_powerlaw(n: int = 4_000_000, seed: int = 3):
    """Power-law random nonsymmetric matrix (mean row length 12, max 512): (A, x)."""
    rng = np.random.default_rng(seed)
    A = powerlaw_random(n, rng)
    return A, uniform_vector(A.n, rng)


@dataclass
class Request:
    rid: int
    dim: int
    m: int
    sigma: float
    seed: int


def serving_requests(count: int, seed: int = 5, nmin: float = 1e3, nmax: float = 1e6):
    """Serving trace: per-request (2D or 3D, grid size, sigma, seed).

    n is log-uniform in [nmin, nmax]; m = round(sqrt(n)) or round(cbrt(n));
    sigma ~ U[0.5, 3]; the request's own matrix seed is 5000 + id.
    """
    rng = np.random.default_rng(seed)
    out = []
    for rid in range(count):
        dim = 2 if rng.random() < 0.5 else 3
        n = math.exp(rng.uniform(math.log(nmin), math.log(nmax)))
        m = max(2, int(round(n ** (1.0 / dim))))
        sigma = float(rng.uniform(0.5, 3.0))
        out.append(Request(rid, dim, m, sigma, 5000 + rid))
    return out


def request_system(req: Request):
    """(A, x_true) of one serving request."""
    rng = np.random.default_rng(req.seed)
    shape = (req.m,) * req.dim
    A = lognormal_tpfa(shape, req.sigma, rng)
    return A, uniform_vector(A.n, rng)


def poisson_arrivals(count: int, rate: float, seed: int = 6) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, count))
