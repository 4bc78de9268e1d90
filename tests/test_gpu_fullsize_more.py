"""GPU parity at the full sizes of the other workloads.

* power-law random matrix, n = 4,000,000 (mean row length 12, max 512): HEC
  conversion bit-exact against the oracle at ELL widths 8/12/16/24 and plain CSR,
  SpMV in FP64 (1e-12) and FP32 (error bound) against the oracle's CSR product;
* anisotropic 3D diffusion 192^3 (n = 7,077,888) with ILU(1): factor pattern
  bit-exact, preconditioner solve within 1e-12 of the oracle (1e-4 from the FP32
  factor copy; these plans take two solver wavefronts per part), and the FP64 and
  mixed-precision GMRES solutions checked by their FP64 true residual (1e-10)
  computed with the oracle's SpMV;
* 2D lognormal diffusion 1000 x 1000 (n = 1,000,000), ILU(0): the wavefront
  preconditioner solve with 64 x 1 tiles within 1e-12 of the oracle's substitution,
  componentwise on sampled rows, and within 1e-4 from the FP32 factor copy.
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


@pytest.fixture(scope="module")
def plane():
    A = synth.lognormal_tpfa((1000, 1000, 1), 2.0, np.random.default_rng(12))
    M = hec.ilu_factor(A, k=0, keep_f32=True)
    lv = hec.level_schedule(M)
    return A, O.iluk(A.n, A.Ap, A.Aj, A.Ax, 0), M, lv


def test_plane_1000_wavefront_trsv(plane):
    """The largest 2D requests of the serving trace (1000 x 1000, ILU(0)): the wavefront
    solve with 64 x 1 tiles (16 along x, the last one ragged) against the oracle's
    substitution, lone triangles and the L-then-U chain, FP64 within 1e-12 (and
    componentwise on sampled rows: the residual of row i against the exact products of
    its own entries) and from the FP32 copy within 1e-4."""
    import torch
    A, Fo, M, lv = plane
    assert hec.levels_grid(lv)
    g = hec.levels_export(lv)
    assert (g["nlev_lower"], g["nlev_upper"]) == (1999, 1999)
    r = np.random.default_rng(13).uniform(-1, 1, A.n)
    y_o = O.trsv_lower(Fo, r)
    x_o = O.trsv_upper(Fo, y_o)
    y, x, x1 = empty(A.n), empty(A.n), empty(A.n)
    hec.trsv_levels(M, lv, dev(r), y, hec.LOWER)
    hec.trsv_levels(M, lv, dev(r), x, hec.LU)
    hec.trsv_levels(M, lv, dev(y_o), x1, hec.UPPER)
    hec.levels_check(lv)
    y, x, x1 = host(y), host(x), host(x1)
    for got, ref in ((y, y_o), (x, x_o), (x1, x_o)):
        assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
    rows = np.random.default_rng(14).choice(A.n, 2000, replace=False)
    for i in rows:  # row i of L y = r (unit diagonal): |r_i - y_i - sum l_ij y_j| within the rounding of its terms
        lo, hi = Fo.LUp[i], Fo.LUp[i + 1]
        cols, vals = Fo.LUj[lo:hi], Fo.LUx[lo:hi]
        low = cols < i
        res = r[i] - y[i] - np.dot(vals[low], y[cols[low]])
        assert abs(res) <= 2 * 4 * U64 * (abs(r[i]) + abs(y[i]) + np.dot(np.abs(vals[low]), np.abs(y[cols[low]])))
    x32 = empty(A.n, "f32")
    hec.trsv_levels(M, lv, dev(r, torch.float32), x32, hec.LU)
    hec.levels_check(lv)
    assert np.linalg.norm(host(x32).astype(np.float64) - x_o) <= 1e-4 * np.linalg.norm(x_o)
