"""GPU parity at the full sizes of the other workloads.

* power-law random matrix, n = 4,000,000 (mean row length 12, max 512): HEC
  conversion bit-exact against the oracle at ELL widths 8/12/16/24 and plain CSR,
  SpMV in FP64 (1e-12) and FP32 (error bound) against the oracle's CSR product;
* anisotropic 3D diffusion 192^3 (n = 7,077,888) with ILU(1): factor pattern
  bit-exact, preconditioner solve within 1e-12 of the oracle (1e-4 from the FP32
  factor copy; these plans take two solver wavefronts per part), and the FP64 and
  mixed-precision GMRES solutions checked by their FP64 true residual (1e-10)
  computed with the oracle's SpMV.
"""
import numpy as np
import pytest

import oracle as O
from paper_1606_00545_amd import hec, synth
from tests._gpu import abs_product, dev, empty, host

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53
U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def powerlaw():
    A, x = synth.workload_powerlaw()
    y = O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, x)
    return A, x, y


@pytest.mark.parametrize("width", [0, 8, 12, 16, 24])
def test_powerlaw_hec_and_spmv(powerlaw, width):
    import torch
    A, x, y_ref = powerlaw
    M = hec.hec_from_csr(A, ell_width=width, keep_f32=True)
    g = hec.hec_export(M)
    o = O.hec_from_csr(A.n, A.Ap, A.Aj, A.Ax, width)
    assert (g["K"], g["ld"], g["nnz_rem"]) == (o.K, o.ld, o.rem_col.size)
    assert np.array_equal(g["ell_col"], o.ell_col)
    assert np.array_equal(g["ell_val"].view(np.uint64), o.ell_val.view(np.uint64))
    assert np.array_equal(g["rem_ptr"], o.rem_ptr) and np.array_equal(g["rem_col"], o.rem_col)
    assert np.array_equal(g["rem_val"].view(np.uint64), o.rem_val.view(np.uint64))
    del g, o
    xd = dev(x)
    y = empty(A.n)
    hec.hec_spmv(M, xd, y)
    y = host(y)
    ax = abs_product(A, x)
    K = 512
    assert (np.abs(y - y_ref) <= 2 * K * U64 * ax).all()
    assert np.linalg.norm(y - y_ref) <= 1e-12 * np.linalg.norm(y_ref)
    y32 = empty(A.n, "f32")
    hec.hec_spmv(M, dev(x, torch.float32), y32, vals=hec.F32)
    y32 = host(y32).astype(np.float64)
    assert (np.abs(y32 - y_ref) <= (K + 4) * U32 * ax * 1.01).all()


@pytest.fixture(scope="module")
def aniso():
    A, xt = synth.workload_diffusion3d(192, sigma=2.0, seed=4, zscale=0.01)
    b = O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, xt)
    Mh = hec.hec_from_csr(A, keep_f32=True)
    F = hec.ilu_factor(A, k=1, keep_f32=True)
    lv = hec.level_schedule(F)
    return A, xt, b, Mh, F, lv


def test_aniso_ilu1_factor_and_trsv(aniso):
    A, xt, b, Mh, F, lv = aniso
    Fo = O.iluk(A.n, A.Ap, A.Aj, A.Ax, 1)
    LUp, LUj, LUx = hec.ilu_export(F)
    assert np.array_equal(LUp, Fo.LUp) and np.array_equal(LUj, Fo.LUj)
    assert LUp[-1] == 91_350_144
    scale = np.maximum(np.abs(Fo.LUx), 1e-3 * np.abs(Fo.LUx).max())
    assert np.max(np.abs(LUx - Fo.LUx) / scale) <= 1e-12
    del LUp, LUj, LUx
    g = hec.levels_export(lv)
    assert (g["nlev_lower"], g["nlev_upper"]) == (1147, 1147)
    r = np.random.default_rng(9).uniform(-1, 1, A.n)
    x_o = O.trsv_upper(Fo, O.trsv_lower(Fo, r))
    x = empty(A.n)
    hec.trsv_levels(F, lv, dev(r), x, hec.LU)
    x = host(x)
    assert np.linalg.norm(x - x_o) <= 1e-12 * np.linalg.norm(x_o)
    # the same pair from the FP32 factor copy (its plans run two solver wavefronts per part)
    import torch
    x32 = empty(A.n, "f32")
    hec.trsv_levels(F, lv, dev(r, torch.float32), x32, hec.LU)
    rel = np.linalg.norm(host(x32).astype(np.float64) - x_o) / np.linalg.norm(x_o)
    assert rel < 1e-4, rel


@pytest.mark.parametrize("precision", [0, 1])
def test_aniso_gmres_reaches_1e10(aniso, precision):
    A, xt, b, Mh, F, lv = aniso
    x = empty(A.n)
    info = hec.gmres_solve(Mh, F, lv, dev(b), x, restart=30, rtol=1e-10, ir_rtol=1e-10,
                           precision=precision, maxit=20000)
    xh = host(x)
    rr = np.linalg.norm(b - O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, xh)) / np.linalg.norm(b)
    print(f"precision {precision}: iterations {info['iterations']} refinement steps {info['ir_steps']} "
          f"rel_res {rr:.3e} |x-x_true|/|x_true| {np.linalg.norm(xh - xt) / np.linalg.norm(xt):.3e} "
          f"{info['seconds']:.2f}s")
    assert info["status"] == hec.OK and rr <= 1e-10
