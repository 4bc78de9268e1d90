"""gmres_solve_noalloc: the GMRES entry point whose workspace is the library's static
scratch array. Through the C ABI it gives what gmres_solve gives (same iterations, the
same x bit for bit: the same kernels in the same order), on two calls in a row with the
second on a smaller system (the scratch keeps the first call's contents), while the
allocator hooks see no call; sizes beyond the scratch, mixed precision and restart > 32
are refused."""
import numpy as np
import pytest

import oracle as O
from paper_1606_00545_amd import hec, synth
from tests._gpu import dev, empty, host

pytestmark = pytest.mark.gpu


class _NoCalls:
    def __init__(self):
        self.calls = 0

    def alloc(self, nbytes, stream):
        self.calls += 1
        return None

    def free(self, ptr, nbytes, stream):
        self.calls += 1


def _setup(A):
    Mh = hec.hec_from_csr(A)
    F = hec.ilu_factor(A, k=0)
    lv = hec.level_schedule(F)
    return Mh, F, lv


def _systems():
    # the larger first (3D lognormal diffusion 24^3, 13,824 rows), then 2D Poisson 64 x 64
    A1, x1 = synth.workload_diffusion3d(24, sigma=2.0, seed=3)
    A2, x2 = synth.workload_c1()
    return [(A1, O.csr_spmv(A1.n, A1.Ap, A1.Aj, A1.Ax, x1)), (A2, O.csr_spmv(A2.n, A2.Ap, A2.Aj, A2.Ax, x2))]


@pytest.mark.parametrize("restart", [30, 7])
def test_noalloc_equals_gmres_solve_on_two_calls(restart):
    systems = _systems()
    handles = [_setup(A) for A, _ in systems]  # setup allocates; the solves below must not
    hook = _NoCalls()
    results = []
    hec.set_allocator(hook.alloc, hook.free)
    try:
        for (A, b), (Mh, F, lv) in zip(systems, handles):
            x = empty(A.n)
            info = hec.gmres_solve_noalloc(Mh, F, lv, dev(b), x, restart=restart, rtol=1e-8)
            results.append((info, host(x)))
    finally:
        hec.use_torch_allocator()
    assert hook.calls == 0
    for (A, b), (Mh, F, lv), (info, x) in zip(systems, handles, results):
        xr = empty(A.n)
        ref = hec.gmres_solve(Mh, F, lv, dev(b), xr, restart=restart, rtol=1e-8)
        rr = np.linalg.norm(b - O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, x)) / np.linalg.norm(b)
        print(f"n={A.n} restart={restart}: noalloc it={info['iterations']} gmres_solve it={ref['iterations']} "
              f"rel_res={rr:.2e}")
        assert info["status"] == hec.OK and rr <= 1e-8
        assert (info["iterations"], info["restarts"]) == (ref["iterations"], ref["restarts"])
        assert info["rel_res_true"] == ref["rel_res_true"]
        assert np.array_equal(x.view(np.uint64), host(xr).view(np.uint64))


def test_noalloc_limits_and_zero_rhs():
    A = synth.poisson1d(hec.NOALLOC_MAX_N + 1)
    Mh, F, lv = _setup(A)
    b = np.ones(A.n)
    with pytest.raises(hec.HecError) as e:
        hec.gmres_solve_noalloc(Mh, F, lv, dev(b), empty(A.n))
    assert e.value.code == hec.INVALID_ARG and "exceeds" in str(e.value)
    A = synth.poisson2d(20)
    Mh, F, lv = _setup(A)
    b = np.ones(A.n)
    with pytest.raises(hec.HecError) as e:
        hec.gmres_solve_noalloc(Mh, F, lv, dev(b), empty(A.n), restart=33)
    assert e.value.code == hec.INVALID_ARG
    o = hec._opts(30, 100, 1e-8, 1, True, 0.0, 0.0)  # precision 1 straight through the C ABI
    info = hec.SolveInfo()
    import ctypes as C
    code = hec.load().gmres_solve_noalloc(Mh.ptr, F.ptr, lv.ptr, dev(b).data_ptr(), empty(A.n).data_ptr(),
                                          C.byref(o), C.byref(info), None)
    assert code == hec.INVALID_ARG
    x = dev(np.full(A.n, 3.0))
    info = hec.gmres_solve_noalloc(Mh, F, lv, dev(np.zeros(A.n)), x)
    assert info["status"] == hec.OK and info["iterations"] == 0 and not host(x).any()
