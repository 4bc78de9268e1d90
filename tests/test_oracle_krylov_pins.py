"""More pins of the oracle's Krylov solvers (Sec. 2.7, Alg. 4).

* BiCGSTAB's breakdown tests ("rho = 0 ... fails" in Alg. 4, and (r0, v) = 0) and
  its restart from the current iterate, on 3 x 3 integer systems with the identity
  preconditioner whose first pass was worked out by hand. Every quantity of that
  pass is a small dyadic rational, so FP64 arithmetic is exact in any order and the
  oracle must reach the exact-zero breakdown test. A wrong breakdown test, a
  shadow residual that is not reset on restart, or a wrong restart cap changes the
  pass count, the restart count or the status below.
* A skew-symmetric A, where (r, A r) = 0 for every r: every cycle breaks down in its
  first pass, so the solver gives up with BREAKDOWN after 3 restarts and x = x0.
* The Arnoldi relation of GMRES: with Z = M^{-1} V, A Z_m = V_{m+1} Hbar_m and
  V^T V = I to rounding, on the oracle's own basis and Hessenberg matrix."""
import numpy as np
import pytest

import oracle as O
from paper_1606_00545_amd import synth
from tests._mats import from_dense, identity_factor, random_sparse


def _bicg(A, b, **kw):
    return O.bicgstab(from_dense(np.array(A, float)), identity_factor(len(b)), np.array(b, float), **kw)


# Breakdown by rho: A = [[-1,2,1],[-1,-2,1],[2,2,1]], b = (-2,0,0), x0 = 0, M = I.
# Pass 1 (by hand): r0 = r = b, rho_1 = (r0, r) = 4, p = b, v = A p = (2, 2, -4),
# (r0, v) = -4, alpha = -1, s = r - alpha v = (0, 2, -4), t = A s = (0, -8, 0),
# omega = (t, s)/(t, t) = -16/64 = -1/4, x_1 = alpha p + omega s = (2, -1/2, 1),
# r_1 = s - omega t = (0, 0, -4). Pass 2: rho_2 = (r0, r_1) = 0 -> breakdown.
# Restart from x_1 (new shadow residual r_1): exact arithmetic gives s = 0 at the
# half step of the third pass of that cycle, so 1 + 3 = 4 passes and one restart.
RHO0 = ([[-1, 2, 1], [-1, -2, 1], [2, 2, 1]], [-2, 0, 0], [2.0, -0.5, 1.0])
# Breakdown by (r0, v): A = [[-2,2,1],[-2,1,2],[2,0,1]], b = (0,0,1).
# Pass 1: rho_1 = 1, v = (1, 2, 1), (r0, v) = 1, alpha = 1, s = (-1, -2, 0),
# t = (-2, 0, -2), omega = 2/8 = 1/4, x_1 = (-1/4, -1/2, 1), r_1 = (-1/2, -2, 1/2).
# Pass 2: rho_2 = 1/2, beta = (rho_2/rho_1)(alpha/omega) = 2,
# p = r_1 + beta (p - omega v) = (-1, -3, 2), v = A p = (-2, 3, 0), (r0, v) = 0 ->
# breakdown inside pass 2 (which does not count). Restart: 3 more passes.
R0V0 = ([[-2, 2, 1], [-2, 1, 2], [2, 0, 1]], [0, 0, 1], [-0.25, -0.5, 1.0])


@pytest.mark.parametrize("case", [RHO0, R0V0], ids=["rho", "r0v"])
def test_bicgstab_first_pass_is_exact(case):
    A, b, x1 = case
    r = _bicg(A, b, maxit=1, rtol=1e-10)
    assert r.status == O.NOT_CONVERGED and r.iterations == 1
    assert r.x.tolist() == x1  # exact: every quantity of the pass is a small dyadic rational


@pytest.mark.parametrize("case", [RHO0, R0V0], ids=["rho", "r0v"])
def test_bicgstab_breakdown_then_restart_converges(case):
    A, b, _ = case
    xs = np.linalg.solve(np.array(A, float), np.array(b, float))
    r = _bicg(A, b, rtol=1e-10)
    assert r.status == O.OK
    assert r.restarts == 1 and r.iterations == 4
    assert np.abs(r.x - xs).max() < 1e-13


def test_bicgstab_breakdown_in_every_cycle_gives_up():
    n = 4
    A = np.eye(n, k=1) - np.eye(n, k=-1)  # skew-symmetric: (r, A r) = 0 for every r; det = 1
    b = np.arange(1.0, n + 1)
    r = O.bicgstab(from_dense(A), identity_factor(n), b, rtol=1e-10)
    assert r.status == O.BREAKDOWN
    assert r.iterations == 0 and r.restarts == 3
    assert (r.x == 0).all()
    # the same with a nonzero start: the iterate is left where it was
    x0 = np.array([1.0, -2.0, 0.5, 3.0])
    r = O.bicgstab(from_dense(A), identity_factor(n), b, x0=x0, rtol=1e-10)
    assert r.status == O.BREAKDOWN and r.restarts == 3 and (r.x == x0).all()


def test_bicgstab_restart_count_is_zero_without_restart():
    rng = np.random.default_rng(3)
    A = synth.lognormal_tpfa((8, 8, 6), 1.0, rng)
    F = O.iluk(A.n, A.Ap, A.Aj, A.Ax, 0)
    r = O.bicgstab(A, F, rng.standard_normal(A.n), rtol=1e-8)
    assert r.status == O.OK and r.restarts == 0


@pytest.mark.parametrize("prec,m", [("identity", 20), ("ilu0", 5)])
def test_gmres_arnoldi_relation_and_orthogonality(prec, m):
    """Right-preconditioned Arnoldi: A M^{-1} V_m = V_{m+1} Hbar_m and V^T V = I. Modified
    Gram-Schmidt loses orthogonality in proportion to how far the residual has fallen, so
    the step counts keep the residual above 1e-4 (unpreconditioned: above 0.1)."""
    rng = np.random.default_rng(11)
    A = synth.lognormal_tpfa((9, 8, 7), 2.0, rng)
    F = identity_factor(A.n) if prec == "identity" else O.iluk(A.n, A.Ap, A.Aj, A.Ax, 0)
    b = rng.standard_normal(A.n)
    r = O.gmres(A, F, b, restart=m, maxit=m, rtol=1e-300, arnoldi=True)
    assert r.steps == m and r.rel_res > 1e-4
    V = r.V  # (m+1) x n
    Z = np.array([O.trsv_upper(F, O.trsv_lower(F, v)) for v in V[:m]])
    AZ = np.array([O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, z) for z in Z])  # m x n, row j = A z_j
    VH = r.Hbar.T @ V                                                   # row j = sum_i h_ij v_i
    assert np.linalg.norm(AZ - VH) <= 1e-13 * np.linalg.norm(AZ)
    assert np.abs(V @ V.T - np.eye(m + 1)).max() <= 1e-12
    # Hessenberg: nothing below the first subdiagonal, a positive subdiagonal
    assert (np.tril(r.Hbar, -2) == 0).all()
    assert (np.diag(r.Hbar, -1) > 0).all()


def test_gmres_arnoldi_basis_spans_the_krylov_space():
    """v_1 = r_0 / ||r_0||, and each v_{j+1} lies in span{v_1, A M^{-1} v_1, ...}: the
    triangular change of basis to the power basis is exact to rounding."""
    rng = np.random.default_rng(5)
    A = random_sparse(60, 0.08, rng)
    b = rng.standard_normal(A.n)
    m = 6
    r = O.gmres(A, identity_factor(A.n), b, restart=m, maxit=m, rtol=1e-300, arnoldi=True)
    V = r.V
    assert np.allclose(V[0], b / np.linalg.norm(b), rtol=0, atol=1e-15)
    K = [b / np.linalg.norm(b)]
    for _ in range(m):
        K.append(O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, K[-1]))
    K = np.array(K)
    Q, _ = np.linalg.qr(K.T)  # orthonormal basis of the Krylov space, same span by construction
    assert np.linalg.norm(V.T - Q @ (Q.T @ V.T)) <= 1e-10 * np.linalg.norm(V)
