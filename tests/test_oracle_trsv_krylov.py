"""Pins for the oracle's triangular solves (Sec. 2.6) and Krylov solvers (Sec. 2.7, Alg. 4)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
from paper_1606_00545_amd import synth
from tests._mats import from_dense, identity_factor, random_sparse, to_dense, tridiag


def _factor_dense(F):
    D = to_dense(F.n, F.LUp, F.LUj, F.LUx)
    return np.tril(D, -1) + np.eye(F.n), np.triu(D)


@pytest.mark.parametrize("k", [0, 2])
def test_trsv_matches_dense_solves(k):
    rng = np.random.default_rng(4)
    A = random_sparse(60, 0.06, rng)
    F = O.iluk(A.n, A.Ap, A.Aj, A.Ax, k)
    L, U = _factor_dense(F)
    b = rng.standard_normal(A.n)
    y = O.trsv_lower(F, b)
    x = O.trsv_upper(F, y)
    assert np.abs(y - np.linalg.solve(L, b)).max() < 1e-12 * np.abs(y).max()
    assert np.abs(x - np.linalg.solve(U, y)).max() < 1e-12 * np.abs(x).max()
    import scipy.sparse as sp
    y2 = spla.spsolve_triangular(sp.csr_matrix(L), b, lower=True)
    assert np.abs(y - y2).max() < 1e-12 * np.abs(y).max()


def test_trsv_componentwise_backward_error():
    """Substitution is componentwise backward stable: |b - L y| <= gamma_w |L| |y|."""
    rng = np.random.default_rng(8)
    A = synth.lognormal_tpfa((6, 7, 5), 2.0, rng)
    F = O.iluk(A.n, A.Ap, A.Aj, A.Ax, 1)
    L, U = _factor_dense(F)
    b = rng.standard_normal(A.n)
    y = O.trsv_lower(F, b)
    x = O.trsv_upper(F, y)
    u = 2.0 ** -53
    w = int(np.diff(F.LUp).max()) + 1
    gam = w * u / (1 - w * u)
    assert (np.abs(b - L @ y) <= gam * (np.abs(L) @ np.abs(y)) + 1e-300).all()
    assert (np.abs(y - U @ x) <= gam * (np.abs(U) @ np.abs(x)) + 1e-300).all()


def _rel_res(A, x, b):
    return np.linalg.norm(b - A.to_scipy() @ x) / np.linalg.norm(b)


def test_gmres_exact_preconditioner_converges_in_one_step():
    rng = np.random.default_rng(1)
    A = tridiag(200, rng)
    F = O.iluk(A.n, A.Ap, A.Aj, A.Ax, 0)  # exact LU for a tridiagonal matrix
    b = rng.standard_normal(A.n)
    r = O.gmres(A, F, b, rtol=1e-12)
    assert r.status == O.OK and r.iterations == 1 and _rel_res(A, r.x, b) < 1e-12


def test_bicgstab_exact_preconditioner_converges_in_one_step():
    rng = np.random.default_rng(2)
    A = tridiag(200, rng)
    F = O.iluk(A.n, A.Ap, A.Aj, A.Ax, 0)
    b = rng.standard_normal(A.n)
    r = O.bicgstab(A, F, b, rtol=1e-12)
    assert r.status == O.OK and r.iterations == 1 and _rel_res(A, r.x, b) < 1e-12


def test_gmres_distinct_eigenvalues_bound():
    """A diagonal matrix with d distinct eigenvalues: unpreconditioned GMRES terminates in <= d steps."""
    n, d = 80, 5
    vals = np.repeat(np.arange(1.0, d + 1), n // d)
    A = from_dense(np.diag(vals))
    b = np.random.default_rng(0).standard_normal(n)
    r = O.gmres(A, identity_factor(n), b, restart=50, rtol=1e-13)
    assert r.status == O.OK and r.iterations <= d
    assert np.abs(r.x - b / vals).max() < 1e-12


def test_gmres_full_krylov_reaches_machine_precision():
    rng = np.random.default_rng(12)
    A = random_sparse(30, 0.2, rng)
    b = rng.standard_normal(30)
    r = O.gmres(A, identity_factor(30), b, restart=30, rtol=1e-14, maxit=30)
    D = to_dense(A.n, A.Ap, A.Aj, A.Ax)
    assert r.iterations <= 30
    assert np.linalg.norm(r.x - np.linalg.solve(D, b)) / np.linalg.norm(r.x) < 1e-12


@pytest.mark.parametrize("solver", ["gmres", "bicgstab"])
def test_solvers_reach_tolerance_and_match_dense_solution(solver):
    rng = np.random.default_rng(3)
    A = synth.lognormal_tpfa((12, 12, 10), 2.0, rng)
    xt = rng.uniform(-1, 1, A.n)
    b = O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, xt)
    F = O.iluk(A.n, A.Ap, A.Aj, A.Ax, 0)
    r = (O.gmres(A, F, b, restart=30) if solver == "gmres" else O.bicgstab(A, F, b))
    assert r.status == O.OK
    assert _rel_res(A, r.x, b) <= 1e-8
    assert abs(r.rel_res - _rel_res(A, r.x, b)) < 1e-10
    xd = np.linalg.solve(to_dense(A.n, A.Ap, A.Aj, A.Ax), b)
    assert np.linalg.norm(r.x - xd) / np.linalg.norm(xd) < 1e-5


def _scipy_prec(F):
    L, U = _factor_dense(F)
    import scipy.linalg as sl
    return spla.LinearOperator(L.shape, matvec=lambda v: sl.solve_triangular(
        U, sl.solve_triangular(L, v, lower=True, unit_diagonal=True)))


def test_gmres_tracks_scipy_gmres():
    """Same Krylov space, same minimisation: iterate counts agree with scipy's GMRES(m)
    (left-preconditioned there, right here) to within a few steps, and both solve the system."""
    rng = np.random.default_rng(7)
    A = synth.lognormal_tpfa((10, 10, 8), 1.5, rng)
    b = rng.standard_normal(A.n)
    F = O.iluk(A.n, A.Ap, A.Aj, A.Ax, 0)
    r = O.gmres(A, F, b, restart=10, rtol=1e-10)
    it = [0]
    xs, info = spla.gmres(A.to_scipy(), b, M=_scipy_prec(F), restart=10, rtol=1e-10, atol=0,
                          maxiter=200, callback=lambda _: it.__setitem__(0, it[0] + 1),
                          callback_type="pr_norm")
    assert info == 0 and r.status == O.OK
    assert abs(r.iterations - it[0]) <= max(3, it[0] // 5)
    assert np.linalg.norm(r.x - xs) / np.linalg.norm(xs) < 1e-7


def test_bicgstab_tracks_scipy_bicgstab():
    rng = np.random.default_rng(8)
    A = random_sparse(300, 0.02, rng)
    b = rng.standard_normal(A.n)
    F = O.iluk(A.n, A.Ap, A.Aj, A.Ax, 0)
    r = O.bicgstab(A, F, b, rtol=1e-10)
    it = [0]
    xs, info = spla.bicgstab(A.to_scipy(), b, M=_scipy_prec(F), rtol=1e-10, atol=0,
                             callback=lambda _: it.__setitem__(0, it[0] + 1))
    assert info == 0 and r.status == O.OK
    assert abs(r.iterations - it[0]) <= 2
    assert np.linalg.norm(r.x - xs) / np.linalg.norm(xs) < 1e-8


def test_zero_rhs_gives_zero_solution():
    rng = np.random.default_rng(1)
    A = tridiag(10, rng)
    F = O.iluk(A.n, A.Ap, A.Aj, A.Ax, 0)
    for f in (O.gmres, O.bicgstab):
        r = f(A, F, np.zeros(10), x0=np.ones(10))
        assert r.status == O.OK and r.iterations == 0 and (r.x == 0).all()


def test_not_converged_when_maxit_too_small():
    rng = np.random.default_rng(3)
    A = synth.lognormal_tpfa((10, 10, 10), 2.0, rng)
    b = rng.standard_normal(A.n)
    F = O.iluk(A.n, A.Ap, A.Aj, A.Ax, 0)
    r = O.gmres(A, F, b, maxit=3)
    assert r.status == O.NOT_CONVERGED and r.iterations == 3 and r.rel_res > 1e-8
    r = O.bicgstab(A, F, b, maxit=2)
    assert r.status == O.NOT_CONVERGED and r.iterations == 2
