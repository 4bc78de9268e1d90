"""Pins of the oracle's preconditioned conjugate gradient (Sec. 2.7).

CG is fixed by properties of the method that hold independently of its code: one
step with the exact preconditioner, at most k steps for k distinct eigenvalues,
monotone decrease of the A-norm error, agreement with scipy's CG on the same
preconditioner, and the breakdown of an indefinite problem."""
import numpy as np
import scipy.linalg as sl
import scipy.sparse.linalg as spla

import oracle as O
from paper_1606_00545_amd import synth
from tests._mats import from_dense, identity_factor, to_dense


def _rel_res(A, x, b):
    return np.linalg.norm(b - A.to_scipy() @ x) / np.linalg.norm(b)


def test_exact_preconditioner_converges_in_one_step():
    A = synth.poisson1d(200)  # tridiagonal: ILU(0) is the exact LU
    b = np.random.default_rng(1).uniform(-1, 1, A.n)
    r = O.cg(A, O.iluk(A.n, A.Ap, A.Aj, A.Ax, 0), b, rtol=1e-12)
    assert r.status == O.OK and r.iterations == 1 and _rel_res(A, r.x, b) <= 1e-12


def test_distinct_eigenvalues_bound():
    rng = np.random.default_rng(2)
    vals = np.repeat([1.0, 2.5, 4.0, 7.5, 9.0], 8)  # 5 distinct eigenvalues
    A = from_dense(np.diag(rng.permutation(vals)))
    b = rng.standard_normal(A.n)
    r = O.cg(A, identity_factor(A.n), b, rtol=1e-12)
    assert r.status == O.OK and r.iterations <= 5


def test_a_norm_error_decreases_monotonically():
    A = synth.lognormal_tpfa((9, 8, 7), 1.5, np.random.default_rng(3))
    D = to_dense(A.n, A.Ap, A.Aj, A.Ax)
    xs = np.random.default_rng(4).uniform(-1, 1, A.n)
    b = D @ xs
    F = O.iluk(A.n, A.Ap, A.Aj, A.Ax, 0)
    errs = []
    for k in range(1, 21):  # converges (rtol 1e-14) at step 22
        r = O.cg(A, F, b, maxit=k, rtol=1e-14)
        assert r.iterations == k
        e = r.x - xs
        errs.append(float(e @ D @ e))
    assert all(b2 < a2 for a2, b2 in zip(errs, errs[1:]))


def test_tracks_scipy_cg():
    rng = np.random.default_rng(5)
    A = synth.lognormal_tpfa((12, 11, 10), 2.0, rng)
    b = rng.standard_normal(A.n)
    F = O.iluk(A.n, A.Ap, A.Aj, A.Ax, 1)
    D = to_dense(F.n, F.LUp, F.LUj, F.LUx)
    L = np.tril(D, -1) + np.eye(F.n)
    U = np.triu(D)
    M = spla.LinearOperator(D.shape, matvec=lambda v: sl.solve_triangular(
        U, sl.solve_triangular(L, v, lower=True, unit_diagonal=True)))
    it = [0]
    xsc, info = spla.cg(A.to_scipy(), b, M=M, rtol=1e-10, atol=0, maxiter=500,
                        callback=lambda _: it.__setitem__(0, it[0] + 1))
    r = O.cg(A, F, b, rtol=1e-10)
    assert info == 0 and r.status == O.OK
    assert abs(r.iterations - it[0]) <= 1
    assert np.linalg.norm(r.x - xsc) / np.linalg.norm(xsc) < 1e-8


def test_indefinite_problem_breaks_down():
    A = from_dense(np.diag([1.0, -1.0]))
    r = O.cg(A, identity_factor(2), np.array([1.0, 1.0]))  # (p, Ap) = 0 at the first step
    assert r.status == O.BREAKDOWN


def test_zero_rhs_and_not_converged():
    A = synth.poisson2d(16)
    F = O.iluk(A.n, A.Ap, A.Aj, A.Ax, 0)
    r = O.cg(A, F, np.zeros(A.n))
    assert r.status == O.OK and r.iterations == 0 and not r.x.any()
    r = O.cg(A, F, np.ones(A.n), maxit=2, rtol=1e-12)
    assert r.status == O.NOT_CONVERGED and r.iterations == 2
