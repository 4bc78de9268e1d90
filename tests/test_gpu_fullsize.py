"""GPU parity at the benchmark's full size (3D lognormal diffusion, 128^3, 2.1M unknowns),
in the launch configuration the benchmark times: HEC SpMV and the level-scheduled
preconditioner solve against the oracle element by element, and the GMRES/BiCGSTAB
solutions by their FP64 true residual computed with the oracle's SpMV."""
import numpy as np
import pytest

import oracle as O
from paper_1606_00545_amd import hec, synth
from tests._gpu import abs_product, dev, empty, host

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53


@pytest.fixture(scope="module")
def system():
    A, xt = synth.workload_diffusion3d(128, sigma=2.0, seed=2)
    b = O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, xt)
    Mh = hec.hec_from_csr(A)
    F = hec.ilu_factor(A, k=0)
    lv = hec.level_schedule(F)
    return A, xt, b, Mh, F, lv


def test_fullsize_spmv(system):
    A, xt, b, Mh, F, lv = system
    y = empty(A.n)
    hec.hec_spmv(Mh, dev(xt), y)
    y = host(y)
    err = np.abs(y - b)
    assert (err <= 2 * 9 * U64 * abs_product(A, xt)).all()
    assert np.linalg.norm(y - b) <= 1e-12 * np.linalg.norm(b)


def test_fullsize_trsv(system):
    A, xt, b, Mh, F, lv = system
    Fo = O.iluk(A.n, A.Ap, A.Aj, A.Ax, 0)
    LUp, LUj, LUx = hec.ilu_export(F)
    assert np.array_equal(LUj, Fo.LUj)
    assert np.max(np.abs(LUx - Fo.LUx) / np.abs(Fo.LUx).max()) <= 1e-13
    r = np.random.default_rng(5).uniform(-1, 1, A.n)
    x_o = O.trsv_upper(Fo, O.trsv_lower(Fo, r))
    x = empty(A.n)
    hec.trsv_levels(F, lv, dev(r), x, hec.LU)
    x = host(x)
    assert np.linalg.norm(x - x_o) <= 1e-12 * np.linalg.norm(x_o)
    g = hec.levels_export(lv)
    assert (g["nlev_lower"], g["nlev_upper"]) == (382, 382)


@pytest.mark.parametrize("solver", ["gmres", "bicgstab"])
def test_fullsize_solve_true_residual(system, solver):
    A, xt, b, Mh, F, lv = system
    x = empty(A.n)
    if solver == "gmres":
        info = hec.gmres_solve(Mh, F, lv, dev(b), x, restart=30, rtol=1e-8)
    else:
        info = hec.bicgstab_solve(Mh, F, lv, dev(b), x, rtol=1e-8)
    xh = host(x)
    rr = np.linalg.norm(b - O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, xh)) / np.linalg.norm(b)
    print(f"{solver}: iterations {info['iterations']} rel_res {rr:.3e} "
          f"|x - x_true|/|x_true| {np.linalg.norm(xh - xt) / np.linalg.norm(xt):.3e}")
    assert info["status"] == hec.OK and rr <= 1e-8
    # the oracle's iteration counts on this system (tests/golden/make_fullsize_iterations.py)
    want = _oracle_iterations()["gmres30" if solver == "gmres" else "bicgstab"]
    assert abs(info["iterations"] - want) <= max(3, want // 10)


def _oracle_iterations():
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fullsize_iterations.txt")
    out = {}
    with open(path) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                name, it = line.split()[:2]
                out[name] = int(it)
    return out
