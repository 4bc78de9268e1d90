"""GPU solvers: restarted GMRES and BiCGSTAB (FP64 and mixed precision) against the oracle.

Krylov iterates are not unique across implementations (CGS2 on the device, MGS in the
oracle; fused multiply-adds), so parity is judged by the FP64 true residual computed by
the oracle's SpMV, the distance to the oracle's solution, and the iteration counts."""
import numpy as np
import pytest

import oracle as O
from paper_1606_00545_amd import hec, synth
from tests._gpu import dev, empty, host
from tests._mats import tridiag

pytestmark = pytest.mark.gpu


def _system(kind):
    if kind == "poisson2d_64":
        A, xt = synth.workload_c1()
    elif kind == "tpfa3d_24":
        A, xt = synth.workload_diffusion3d(24, sigma=2.0, seed=21)
    elif kind == "tpfa2d_aniso":
        rng = np.random.default_rng(22)
        A = synth.lognormal_tpfa((70, 45), 2.5, rng)
        xt = rng.uniform(-1, 1, A.n)
    b = O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, xt)
    return A, xt, b


def _rel_res(A, x, b):
    return np.linalg.norm(b - O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, x)) / np.linalg.norm(b)


def _setup(A, k=0, f32=False):
    Mh = hec.hec_from_csr(A, keep_f32=f32)
    F = hec.ilu_factor(A, k=k, keep_f32=f32)
    lv = hec.level_schedule(F)
    return Mh, F, lv


@pytest.mark.parametrize("kind", ["poisson2d_64", "tpfa3d_24", "tpfa2d_aniso"])
@pytest.mark.parametrize("k", [0, 1])
def test_gmres_fp64_matches_oracle(kind, k):
    A, xt, b = _system(kind)
    Fo = O.iluk(A.n, A.Ap, A.Aj, A.Ax, k)
    ro = O.gmres(A, Fo, b, restart=30, rtol=1e-8)
    Mh, F, lv = _setup(A, k)
    x = empty(A.n)
    info = hec.gmres_solve(Mh, F, lv, dev(b), x, restart=30, rtol=1e-8)
    x = host(x)
    rr = _rel_res(A, x, b)
    assert info["status"] == hec.OK and rr <= 1e-8
    assert abs(info["rel_res_true"] - rr) <= 1e-10
    assert abs(info["iterations"] - ro.iterations) <= max(2, ro.iterations // 10)
    # both are 1e-8-residual solutions of the same system
    assert np.linalg.norm(x - ro.x) / np.linalg.norm(ro.x) < 1e-4
    print(f"{kind} k={k}: gpu it={info['iterations']} oracle it={ro.iterations} res={rr:.2e} "
          f"|x-x_o|/|x_o|={np.linalg.norm(x - ro.x) / np.linalg.norm(ro.x):.2e}")


@pytest.mark.parametrize("kind", ["poisson2d_64", "tpfa3d_24", "tpfa2d_aniso"])
def test_bicgstab_fp64_matches_oracle(kind):
    A, xt, b = _system(kind)
    Fo = O.iluk(A.n, A.Ap, A.Aj, A.Ax, 0)
    ro = O.bicgstab(A, Fo, b, rtol=1e-8)
    Mh, F, lv = _setup(A, 0)
    x = empty(A.n)
    info = hec.bicgstab_solve(Mh, F, lv, dev(b), x, rtol=1e-8)
    x = host(x)
    rr = _rel_res(A, x, b)
    assert info["status"] == hec.OK and rr <= 1e-8
    assert abs(info["iterations"] - ro.iterations) <= max(3, ro.iterations // 5)
    assert np.linalg.norm(x - ro.x) / np.linalg.norm(ro.x) < 1e-4
    print(f"{kind}: gpu it={info['iterations']} oracle it={ro.iterations} res={rr:.2e}")


@pytest.mark.parametrize("kind,k", [("tpfa3d_24", 0), ("tpfa3d_24", 1), ("tpfa2d_aniso", 0)])
@pytest.mark.parametrize("target", [1e-8, 1e-10])
def test_gmres_mixed_precision_reaches_fp64_tolerance(kind, k, target):
    A, xt, b = _system(kind)
    Mh, F, lv = _setup(A, k, f32=True)
    x = empty(A.n)
    info = hec.gmres_solve(Mh, F, lv, dev(b), x, restart=30, rtol=target, precision=1)
    x = host(x)
    rr = _rel_res(A, x, b)
    assert info["status"] == hec.OK and rr <= target and info["ir_steps"] >= 1
    Fo = O.iluk(A.n, A.Ap, A.Aj, A.Ax, k)
    ro = O.gmres(A, Fo, b, restart=30, rtol=target)
    err = np.linalg.norm(x - ro.x) / np.linalg.norm(ro.x)
    print(f"mixed {kind} k={k} target={target}: it={info['iterations']} ir={info['ir_steps']} "
          f"res={rr:.2e} |x-x_o|/|x_o|={err:.2e}")
    assert err < 1e-3


def test_exact_preconditioner_one_iteration():
    A = tridiag(5000, np.random.default_rng(1))
    b = np.random.default_rng(2).uniform(-1, 1, A.n)
    Mh, F, lv = _setup(A)
    for solver in ("gmres", "bicgstab"):
        x = empty(A.n)
        f = hec.gmres_solve if solver == "gmres" else hec.bicgstab_solve
        info = f(Mh, F, lv, dev(b), x, rtol=1e-12)
        assert info["iterations"] == 1 and _rel_res(A, host(x), b) <= 1e-12


def test_zero_rhs_and_initial_guess():
    A, xt, b = _system("poisson2d_64")
    Mh, F, lv = _setup(A)
    x = dev(np.ones(A.n))
    info = hec.gmres_solve(Mh, F, lv, dev(np.zeros(A.n)), x, x0_zero=False)
    assert info["iterations"] == 0 and (host(x) == 0).all()
    # a converged initial guess needs no iteration
    x = dev(xt)
    info = hec.gmres_solve(Mh, F, lv, dev(b), x, x0_zero=False, rtol=1e-6)
    assert info["iterations"] == 0 and info["status"] == hec.OK
    # restart from a partial solve (resume from a saved iterate)
    x = empty(A.n)
    i1 = hec.gmres_solve(Mh, F, lv, dev(b), x, maxit=10, check=False)
    assert i1["status"] == hec.NOT_CONVERGED and i1["iterations"] == 10
    i2 = hec.gmres_solve(Mh, F, lv, dev(b), x, x0_zero=False)
    assert i2["status"] == hec.OK and _rel_res(A, host(x), b) <= 1e-8


def test_not_converged_status_and_best_iterate():
    A, xt, b = _system("tpfa3d_24")
    Mh, F, lv = _setup(A)
    x = empty(A.n)
    info = hec.bicgstab_solve(Mh, F, lv, dev(b), x, maxit=3, check=False)
    assert info["status"] == hec.NOT_CONVERGED and info["iterations"] == 3
    assert abs(_rel_res(A, host(x), b) - info["rel_res_true"]) < 1e-12


def test_solves_are_deterministic():
    A, xt, b = _system("tpfa3d_24")
    Mh, F, lv = _setup(A)
    outs = []
    for _ in range(2):
        x = empty(A.n)
        hec.gmres_solve(Mh, F, lv, dev(b), x)
        outs.append(host(x))
    assert np.array_equal(outs[0].view(np.uint64), outs[1].view(np.uint64))


@pytest.mark.parametrize("kind,k", [("poisson3d_24", 0), ("poisson3d_24", 2), ("tpfa3d_24", 1), ("poisson2d_64", 0)])
def test_cg_matches_oracle(kind, k):
    if kind == "poisson3d_24":
        A = synth.poisson3d(24)
        xt = np.random.default_rng(31).uniform(-1, 1, A.n)
        b = O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, xt)
    else:
        A, xt, b = _system(kind)
    Fo = O.iluk(A.n, A.Ap, A.Aj, A.Ax, k)
    ro = O.cg(A, Fo, b, rtol=1e-8)
    Mh, F, lv = _setup(A, k)
    x = empty(A.n)
    info = hec.cg_solve(Mh, F, lv, dev(b), x, rtol=1e-8)
    x = host(x)
    rr = _rel_res(A, x, b)
    print(f"cg {kind} k={k}: gpu it={info['iterations']} oracle it={ro.iterations} res={rr:.2e}")
    assert ro.status == O.OK and info["status"] == hec.OK and rr <= 1e-8
    assert abs(info["iterations"] - ro.iterations) <= max(2, ro.iterations // 20)
    assert np.linalg.norm(x - ro.x) / np.linalg.norm(ro.x) < 1e-5


def test_cg_breakdown_on_indefinite_system():
    from tests._mats import from_dense
    D = np.diag(np.r_[np.full(50, 2.0), np.full(50, -2.0)])  # symmetric indefinite, exact LU = D
    A = from_dense(D)
    Mh, F, lv = _setup(A, 0)
    b = np.ones(100)
    with pytest.raises(hec.HecError):
        hec.cg_solve(Mh, F, lv, dev(b), empty(100), rtol=1e-10)


@pytest.mark.parametrize("restart", [1, 4, 5, 8, 9, 16, 17, 32])
@pytest.mark.parametrize("precision", [0, 1])
def test_gmres_restart_lengths_match_oracle(restart, precision):
    """Restart lengths at the edges of the Gram-Schmidt pass's vector bounds (4, 8,
    16, 32 basis vectors) and the largest restart, FP64 and mixed: the FP64 residual
    is reached, and FP64 iteration counts stay within the usual margin of the
    oracle's (MGS) for the same restart."""
    A, xt, b = _system("tpfa3d_24")
    Fo = O.iluk(A.n, A.Ap, A.Aj, A.Ax, 0)
    ro = O.gmres(A, Fo, b, restart=restart, rtol=1e-8, maxit=4000)
    Mh, F, lv = _setup(A, 0, f32=precision == 1)
    x = empty(A.n)
    info = hec.gmres_solve(Mh, F, lv, dev(b), x, restart=restart, rtol=1e-8, maxit=4000, precision=precision)
    rr = _rel_res(A, host(x), b)
    assert info["status"] == hec.OK and rr <= 1e-8
    if precision == 0:
        assert abs(info["iterations"] - ro.iterations) <= max(2, ro.iterations // 10)
    print(f"restart {restart} precision {precision}: gpu it={info['iterations']} oracle it={ro.iterations} res={rr:.2e}")


# Alg. 4's breakdowns on 3 x 3 integer systems with the identity preconditioner (the ILU(0)
# of the identity matrix): every quantity of the first pass is a small dyadic rational, so
# the device reaches the same exact-zero tests as the oracle, whatever its summation order.
_BREAK_CASES = {
    "rho": ([[-1, 2, 1], [-1, -2, 1], [2, 2, 1]], [-2, 0, 0]),  # (r0, r) = 0 after pass 1
    "r0v": ([[-2, 2, 1], [-2, 1, 2], [2, 0, 1]], [0, 0, 1]),    # (r0, v) = 0 inside pass 2
}


def _identity_preconditioned(D):
    from tests._mats import from_dense
    A = from_dense(np.array(D, float))
    n = A.n
    Mh = hec.hec_from_csr(A)
    I = from_dense(np.eye(n))
    F = hec.ilu_factor(I, k=0)
    lv = hec.level_schedule(F)
    return A, Mh, F, lv


@pytest.mark.parametrize("case", sorted(_BREAK_CASES))
def test_bicgstab_breakdown_restart_matches_oracle(case):
    """A breakdown in pass 2, a restart from the current x, then convergence at the
    half step (s small: x += alpha p*) of the third pass of the second cycle."""
    from tests._mats import identity_factor
    D, bl = _BREAK_CASES[case]
    A, Mh, F, lv = _identity_preconditioned(D)
    b = np.array(bl, float)
    ro = O.bicgstab(A, identity_factor(3), b, rtol=1e-10)
    assert ro.status == O.OK and ro.restarts == 1 and ro.iterations == 4
    x = empty(3)
    info = hec.bicgstab_solve(Mh, F, lv, dev(b), x, rtol=1e-10)
    xh = host(x)
    assert info["status"] == hec.OK
    assert (info["iterations"], info["restarts"]) == (ro.iterations, ro.restarts)
    assert np.abs(xh - ro.x).max() <= 1e-13 * np.abs(ro.x).max()
    # one pass only: the iterate after pass 1 is exact on both sides
    x1 = empty(3)
    i1 = hec.bicgstab_solve(Mh, F, lv, dev(b), x1, maxit=1, rtol=1e-10, check=False)
    r1 = O.bicgstab(A, identity_factor(3), b, maxit=1, rtol=1e-10)
    assert i1["status"] == hec.NOT_CONVERGED and i1["iterations"] == 1
    assert host(x1).tolist() == r1.x.tolist()


def test_bicgstab_breakdown_status_after_three_restarts():
    """Skew-symmetric A: (r, A r) = 0 for every r, so every cycle breaks down in its first
    pass; the solver returns BREAKDOWN with x left at x0, as the oracle does."""
    from tests._mats import identity_factor
    n = 4
    D = np.eye(n, k=1) - np.eye(n, k=-1)
    A, Mh, F, lv = _identity_preconditioned(D)
    b = np.arange(1.0, n + 1)
    ro = O.bicgstab(A, identity_factor(n), b, rtol=1e-10)
    assert ro.status == O.BREAKDOWN and ro.restarts == 3 and ro.iterations == 0
    x = dev(np.array([1.0, -2.0, 0.5, 3.0]))
    info = hec.bicgstab_solve(Mh, F, lv, dev(b), x, rtol=1e-10, x0_zero=False, check=False)
    assert info["status"] == hec.BREAKDOWN
    assert (info["iterations"], info["restarts"]) == (0, 3)
    assert host(x).tolist() == [1.0, -2.0, 0.5, 3.0]
    with pytest.raises(hec.HecError) as e:
        hec.bicgstab_solve(Mh, F, lv, dev(b), empty(n), rtol=1e-10)
    assert e.value.code == hec.BREAKDOWN


def test_mixed_refinement_that_stalls_finishes_in_fp64():
    """A 2D lognormal system (428 x 428, sigma 2.56: request 1132 of the serving trace) on
    which the FP32 inner solves stop resolving the correction just above 1e-8: the
    refinement finishes with FP64 cycles and reaches the tolerance, like the FP64 solve."""
    spec = synth.serving_requests(2000)[1132]
    A, xt = synth.request_system(spec)
    assert A.n == 183184
    b = O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, xt)
    M = hec.hec_from_csr(A, keep_f32=True)
    F = hec.ilu_factor(A, k=0, keep_f32=True)
    lv = hec.level_schedule(F)
    for prec in (1, 0):
        x = empty(A.n)
        info = hec.gmres_solve(M, F, lv, dev(b), x, rtol=1e-8, precision=prec)
        assert info["status"] == hec.OK and info["rel_res_true"] <= 1e-8, (prec, info)
        r = b - O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, host(x))
        assert np.linalg.norm(r) <= 1e-8 * np.linalg.norm(b)
