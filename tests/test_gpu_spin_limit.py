"""Every device-side wait of the triangular solves is bounded. Forced from the host
with a spin limit of zero polls (a wait gives up at its first unready poll), the
launches still end and the failure is reported as HEC_ERR_TIMEOUT (by levels_check,
by the solvers, by the batched solver), for the wavefront solve and the blocked solve
(each in FP64 and FP32) and the per-row polling fallback; with the default limit
restored, the same handles solve correctly again."""
import numpy as np
import pytest

import oracle as O
from paper_1606_00545_amd import hec, synth
from tests._gpu import dev, empty, host

pytestmark = pytest.mark.gpu


def _rhs(A, seed):
    xt = np.random.default_rng(seed).uniform(-1, 1, A.n)
    return O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, xt)


def _oracle_lu(A, k, b):
    Fo = O.iluk(A.n, A.Ap, A.Aj, A.Ax, k)
    return O.trsv_upper(Fo, O.trsv_lower(Fo, b))


@pytest.mark.parametrize("case", ["grid_f64", "grid_f32", "grid2d_f64", "blocked_f64", "blocked_f32", "fallback"])
def test_zero_spin_limit_gives_up_and_recovers(case):
    import torch
    if case == "fallback":  # ILU(3) rows carry more than 32 entries: the per-row polling kernel
        A, k = synth.poisson3d(14), 3
    elif case == "grid2d_f64":  # the wavefront solve with 64 x 1 tiles
        A, k = synth.lognormal_tpfa((150, 120, 1), 2.0, np.random.default_rng(5)), 0
    else:
        A, k = synth.workload_diffusion3d(40, sigma=2.0, seed=5)[0], 0
    f32 = case.endswith("f32")
    F = hec.ilu_factor(A, k=k, keep_f32=f32)
    hec.set_trsv_grid(not case.startswith("blocked"))  # read when the schedule is built
    try:
        lv = hec.level_schedule(F)
    finally:
        hec.set_trsv_grid(True)
    assert hec.levels_grid(lv) == case.startswith("grid")
    _give_up_and_recover(A, k, F, lv, f32)


def _give_up_and_recover(A, k, F, lv, f32):
    import torch
    M = hec.hec_from_csr(A)
    b = _rhs(A, 3)
    dt = torch.float32 if f32 else torch.float64
    bd = dev(b).to(dt)
    z = torch.empty(A.n, dtype=dt, device="cuda")
    hec.set_spin_limit(0)
    try:
        for _ in range(3):
            hec.trsv_levels(F, lv, bd, z, hec.LU)
        with pytest.raises(hec.HecError) as e:
            hec.levels_check(lv)
        assert e.value.code == hec.TIMEOUT
        if not f32:
            with pytest.raises(hec.HecError) as e:
                hec.gmres_solve(M, F, lv, dev(b), empty(A.n), maxit=40)
            assert e.value.code == hec.TIMEOUT
    finally:
        hec.set_spin_limit(-1)
    hec.levels_check(lv)  # the solver's check cleared the word; nothing has given up since
    hec.trsv_levels(F, lv, bd, z, hec.LU)
    hec.levels_check(lv)
    want = _oracle_lu(A, k, b)
    got = host(z).astype(np.float64)
    tol = 1e-4 if f32 else 1e-12
    assert np.linalg.norm(got - want) <= tol * np.linalg.norm(want)
    x = empty(A.n)
    info = hec.gmres_solve(M, F, lv, dev(b), x, rtol=1e-8)
    assert info["status"] == hec.OK and info["rel_res_true"] <= 1e-8


def test_zero_spin_limit_in_the_batched_solver():
    A = synth.poisson2d(64)
    handles = []
    for s in range(4):
        M = hec.hec_from_csr(A)
        F = hec.ilu_factor(A, k=0)
        handles.append((M, F, hec.level_schedule(F), dev(_rhs(A, 10 + s)), empty(A.n)))
    B = hec.Batch(4, restart=30, max_n=A.n)
    hec.set_spin_limit(0)
    try:
        with pytest.raises(hec.HecError) as e:
            hec.gmres_solve_batched(B, handles, rtol=1e-8, maxit=60)
        assert e.value.code == hec.TIMEOUT
    finally:
        hec.set_spin_limit(-1)
    infos = hec.gmres_solve_batched(B, handles, rtol=1e-8)
    assert all(i["status"] == hec.OK and i["rel_res_true"] <= 1e-8 for i in infos)


def test_spin_limit_arguments():
    with pytest.raises(hec.HecError) as e:
        hec.set_spin_limit(1 << 40)
    assert e.value.code == hec.INVALID_ARG
    hec.set_spin_limit(-1)
