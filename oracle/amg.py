"""AMG oracle (test infrastructure only): the setup and the V-cycle of Sec. 2.8,
Alg. 5, written out plainly in FP64 with numpy/scipy. Only the tests and the
benchmark's CPU leg use it; it shares no code with the GPU library.

* strength(A, theta): classical Ruge-Stueben strength. j strongly influences i
  (j in S_i) when -a_ij >= theta * max_{k != i} (-a_ik) and that maximum is
  positive.
* rs_split(n, S): Ruge-Stueben coarsening, first pass. Points with no strong
  connection either way are F. Every other point starts undecided with measure
  lambda_i = |S_i^T| (how many points it strongly influences). Repeatedly the
  undecided point of largest measure (smallest index on ties) becomes C; the
  undecided points it strongly influences become F, and each undecided point
  that strongly influences a new F point gains 1; each undecided point that
  strongly influences the new C point loses 1.
* direct_interpolation(A, S, cf, theta): "RSD" (Stueben's direct interpolation).
  A C point injects its coarse value. An F point i interpolates from its strong
  C neighbours, separately for negative and positive couplings:
  w_ij = -alpha_i a_ij / a_ii for j in C_i^- = C & S_i (the strong negative
  couplings above), w_ij = -beta_i a_ij / a_ii for j in C_i^+, the C points j
  with a_ij > 0 and a_ij >= theta * max_{k != i} a_ik (strong positive couplings,
  used for interpolation only, not for the coarsening);
  alpha_i = sum_{k != i, a_ik < 0} a_ik / sum_{j in C_i^-} a_ij and beta_i likewise
  over the positive entries; when C_i^+ is empty, the positive entries are added
  to the diagonal instead.
* galerkin(A, P): A_c = P^T A P (R = P^T), in a stated order: (AP)_iJ sums
  a_ik p_kJ over row i of A in column order; (A_c)_IJ sums p_iI (AP)_iJ over the
  fine rows i in ascending order. Every entry touched is kept, zero or not.
* hierarchy(A, ...): levels A_0 = A, A_{l+1} = galerkin(A_l, P_l) until a level
  has at most coarse_size rows, max_levels levels exist, or coarsening stops (no C
  point, or no reduction); the coarsest level is solved exactly.
* vcycle / solve: Alg. 5 with damped Jacobi pre- and post-smoothing,
  x <- x + omega D^{-1} (b - A x), nu1 and nu2 sweeps; or with the Chebyshev
  polynomial smoother that Sec. 2.8 and the AMG tables list beside the Jacobi
  ones ("Chev"). The paper gives no detail of it; the reading taken here is the
  textbook Chebyshev semi-iteration (Saad, Iterative Methods for Sparse Linear
  Systems, Sec. 12.1) on D^{-1} A over the interval [a, b] = [cheb_lower * lmax,
  lmax], lmax = max_i sum_j |a_ij| / |a_ii| (Gershgorin's bound on the spectrum of
  D^{-1} A): nu sweeps give x = x0 + q(D^{-1} A) D^{-1} r0 whose error is
  p_nu(D^{-1} A) e0 with p_nu(t) = T_nu((theta - t) / delta) / T_nu(theta / delta),
  theta = (b + a) / 2, delta = (b - a) / 2 -- the polynomial of degree nu that is
  smallest on [a, b] among those with p(0) = 1 -- by the three-term recurrence:
  z = D^{-1} (b - A x), d = z / theta, then nu times: x += d, z -= D^{-1} A d,
  rho' = 1 / (2 theta / delta - rho) (rho starting at delta / theta),
  d = rho' rho d + (2 rho' / delta) z, rho = rho'. Each sweep costs one product
  with A, as a Jacobi sweep does.
"""
from __future__ import annotations

import heapq
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp


def _csr(A) -> sp.csr_matrix:
    M = sp.csr_matrix((np.asarray(A.Ax, np.float64), np.asarray(A.Aj), np.asarray(A.Ap)), shape=(A.n, A.n))
    M.sort_indices()
    return M


def strength(M: sp.csr_matrix, theta: float):
    """S as a CSR pattern (row i: the points that strongly influence i), columns ascending."""
    n = M.shape[0]
    Sp, Sj = [0], []
    for i in range(n):
        cols = M.indices[M.indptr[i]:M.indptr[i + 1]]
        vals = M.data[M.indptr[i]:M.indptr[i + 1]]
        off = cols != i
        m = (-vals[off]).max(initial=0.0)
        if m > 0.0:
            Sj.extend(int(c) for c, v in zip(cols[off], vals[off]) if -v >= theta * m)
        Sp.append(len(Sj))
    return np.array(Sp, np.int64), np.array(Sj, np.int64)


def _transpose_pattern(n, Sp, Sj):
    cnt = np.bincount(Sj, minlength=n) if Sj.size else np.zeros(n, np.int64)
    Tp = np.concatenate([[0], np.cumsum(cnt)])
    Tj = np.empty(Sj.size, np.int64)
    fill = Tp[:-1].copy()
    for i in range(n):
        for j in Sj[Sp[i]:Sp[i + 1]]:
            Tj[fill[j]] = i
            fill[j] += 1
    return Tp, Tj


def rs_split(n, Sp, Sj):
    """cf[i] = 1 for C, 0 for F (first pass of Ruge-Stueben coarsening)."""
    Tp, Tj = _transpose_pattern(n, Sp, Sj)
    U, C, F = 0, 1, 2
    state = np.full(n, U, np.int8)
    lam = (Tp[1:] - Tp[:-1]).astype(np.int64)
    for i in range(n):
        if Sp[i + 1] == Sp[i] and Tp[i + 1] == Tp[i]:
            state[i] = F  # no strong connection either way
    heap = [(-int(lam[i]), i) for i in range(n) if state[i] == U]
    heapq.heapify(heap)
    while heap:
        negl, i = heapq.heappop(heap)
        if state[i] != U or -negl != lam[i]:
            continue  # stale entry
        state[i] = C
        for j in Tj[Tp[i]:Tp[i + 1]]:  # points i strongly influences
            if state[j] == U:
                state[j] = F
                for k in Sj[Sp[j]:Sp[j + 1]]:  # points that strongly influence the new F point
                    if state[k] == U:
                        lam[k] += 1
                        heapq.heappush(heap, (-int(lam[k]), int(k)))
        for k in Sj[Sp[i]:Sp[i + 1]]:  # points that strongly influence the new C point
            if state[k] == U:
                lam[k] -= 1
                heapq.heappush(heap, (-int(lam[k]), int(k)))
    return (state == C).astype(np.int8)


def direct_interpolation(M: sp.csr_matrix, Sp, Sj, cf, theta=0.25):
    """P (n x nc) as a scipy CSR matrix with columns ascending."""
    n = M.shape[0]
    cidx = np.cumsum(cf) - 1  # coarse index of each C point
    nc = int(cf.sum())
    Pp, Pj, Px = [0], [], []
    for i in range(n):
        if cf[i]:
            Pj.append(int(cidx[i]))
            Px.append(1.0)
            Pp.append(len(Pj))
            continue
        cols = M.indices[M.indptr[i]:M.indptr[i + 1]]
        vals = M.data[M.indptr[i]:M.indptr[i + 1]]
        strong = set(int(j) for j in Sj[Sp[i]:Sp[i + 1]])  # strong negative couplings
        mpos = max((v for j, v in zip(cols, vals) if j != i and v > 0), default=0.0)
        strong |= set(int(j) for j, v in zip(cols, vals) if j != i and v > 0 and v >= theta * mpos)
        aii = 0.0
        sneg = spos = cneg = cpos = 0.0
        for j, v in zip(cols, vals):
            if j == i:
                aii = v
            elif v < 0:
                sneg += v
            else:
                spos += v
        Ci = [(int(j), v) for j, v in zip(cols, vals) if j != i and j in strong and cf[j]]
        for j, v in Ci:
            if v < 0:
                cneg += v
            else:
                cpos += v
        if cpos == 0.0:
            aii += spos  # no positive coupling to interpolate from: lump onto the diagonal
        alpha = sneg / cneg if cneg != 0.0 else 0.0
        beta = spos / cpos if cpos != 0.0 else 0.0
        for j, v in Ci:
            w = -(alpha if v < 0 else beta) * v / aii
            Pj.append(int(cidx[j]))
            Px.append(w)
        Pp.append(len(Pj))
    P = sp.csr_matrix((np.array(Px), np.array(Pj, np.int64), np.array(Pp, np.int64)), shape=(n, nc))
    P.sort_indices()
    return P


def galerkin(M: sp.csr_matrix, P: sp.csr_matrix) -> sp.csr_matrix:
    n, nc = P.shape
    AP = []
    for i in range(n):
        acc = {}
        for e in range(M.indptr[i], M.indptr[i + 1]):
            k, a = int(M.indices[e]), float(M.data[e])
            for f in range(P.indptr[k], P.indptr[k + 1]):
                J = int(P.indices[f])
                acc[J] = acc.get(J, 0.0) + a * float(P.data[f])
        AP.append(acc)
    rows = [dict() for _ in range(nc)]
    for i in range(n):
        for f in range(P.indptr[i], P.indptr[i + 1]):
            I, p = int(P.indices[f]), float(P.data[f])
            acc = rows[I]
            for J, v in AP[i].items():
                acc[J] = acc.get(J, 0.0) + p * v
    Cp, Cj, Cx = [0], [], []
    for I in range(nc):
        for J in sorted(rows[I]):
            Cj.append(J)
            Cx.append(rows[I][J])
        Cp.append(len(Cj))
    return sp.csr_matrix((np.array(Cx), np.array(Cj, np.int64), np.array(Cp, np.int64)), shape=(nc, nc))


def gershgorin_dinv_a(M: sp.csr_matrix) -> float:
    """max_i sum_j |a_ij| / |a_ii|: every eigenvalue of D^{-1} A lies in a disc around 1
    of radius sum_{j != i} |a_ij| / |a_ii| for some row i (Gershgorin), so this bounds
    its spectral radius. Row sums in column order."""
    lmax = 0.0
    for i in range(M.shape[0]):
        s, d = 0.0, 0.0
        for e in range(M.indptr[i], M.indptr[i + 1]):
            v = float(M.data[e])
            s += abs(v)
            if M.indices[e] == i:
                d = v
        lmax = max(lmax, s / abs(d))
    return lmax


@dataclass
class Level:
    A: sp.csr_matrix
    cf: np.ndarray = None
    P: sp.csr_matrix = None
    dinv: np.ndarray = field(default=None)
    lmax: float = 0.0  # Gershgorin bound of D^{-1} A (Chebyshev smoothing only)


@dataclass
class Hierarchy:
    levels: list
    omega: float
    nu1: int
    nu2: int
    smoother: str = "jacobi"
    cheb_lower: float = 0.3


def hierarchy(A, theta=0.25, max_levels=8, coarse_size=64, omega=2.0 / 3.0, nu1=3, nu2=3, smoother="jacobi",
              cheb_lower=0.3) -> Hierarchy:
    assert smoother in ("jacobi", "chebyshev")
    M = _csr(A)
    levels = []
    while True:
        lev = Level(M, dinv=1.0 / M.diagonal())
        if smoother == "chebyshev":
            lev.lmax = gershgorin_dinv_a(M)
        levels.append(lev)
        n = M.shape[0]
        if n <= coarse_size or len(levels) == max_levels:
            break
        Sp, Sj = strength(M, theta)
        cf = rs_split(n, Sp, Sj)
        nc = int(cf.sum())
        if nc == 0 or nc == n:
            break
        P = direct_interpolation(M, Sp, Sj, cf, theta)
        lev.cf, lev.P = cf, P
        M = galerkin(M, P)
    return Hierarchy(levels, omega, nu1, nu2, smoother, cheb_lower)


def _jacobi(lev: Level, x, b, omega, sweeps):
    for _ in range(sweeps):
        x = x + omega * lev.dinv * (b - lev.A @ x)
    return x


def chebyshev(A, dinv, lmax, x, b, degree, cheb_lower=0.3):
    """`degree` sweeps of the Chebyshev smoother on [cheb_lower * lmax, lmax] (the
    recurrence in the module docstring), from x."""
    if degree == 0:
        return x
    hi = lmax
    lo = cheb_lower * lmax
    theta = (hi + lo) / 2.0
    delta = (hi - lo) / 2.0
    sigma = theta / delta
    rho = 1.0 / sigma
    z = dinv * (b - A @ x)
    d = z / theta
    for k in range(degree):
        x = x + d
        if k == degree - 1:
            break
        z = z - dinv * (A @ d)
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = (rho_new * rho) * d + (2.0 * rho_new / delta) * z
        rho = rho_new
    return x


def _smooth(H: Hierarchy, lev: Level, x, b, sweeps):
    if H.smoother == "chebyshev":
        return chebyshev(lev.A, lev.dinv, lev.lmax, x, b, sweeps, H.cheb_lower)
    return _jacobi(lev, x, b, H.omega, sweeps)


def vcycle(H: Hierarchy, b, x=None, l=0):
    """Alg. 5 from level l: pre-smooth, restrict the residual, recurse, prolongate, post-smooth;
    the coarsest level is solved exactly."""
    lev = H.levels[l]
    if l == len(H.levels) - 1:
        return np.linalg.solve(lev.A.toarray(), b)
    x = np.zeros_like(b) if x is None else x
    x = _smooth(H, lev, x, b, H.nu1)
    r = b - lev.A @ x
    xc = vcycle(H, lev.P.T @ r, None, l + 1)
    x = x + lev.P @ xc
    return _smooth(H, lev, x, b, H.nu2)


@dataclass
class AmgResult:
    x: np.ndarray
    iterations: int
    rel_res: float
    converged: bool


def solve(H: Hierarchy, b, rtol=1e-8, maxit=100) -> AmgResult:
    """V-cycles from x = 0 until ||b - A x|| <= rtol ||b|| (FP64 residual) or maxit."""
    A = H.levels[0].A
    nb = np.linalg.norm(b)
    x = np.zeros_like(b)
    if nb == 0.0:
        return AmgResult(x, 0, 0.0, True)
    res = 1.0
    for it in range(1, maxit + 1):
        x = vcycle(H, b, x)
        res = np.linalg.norm(b - A @ x) / nb
        if res <= rtol:
            return AmgResult(x, it, res, True)
    return AmgResult(x, maxit, res, False)
