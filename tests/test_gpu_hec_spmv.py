"""GPU parity: HEC conversion (bit-exact) and SpMV (1e-12) against the oracle."""
import numpy as np
import pytest

import oracle as O
from paper_1606_00545_amd import hec, synth
from tests._gpu import abs_product, dev, empty, host
from tests._mats import random_sparse

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def _mats():
    rng = np.random.default_rng(42)
    yield "poisson2d_64", synth.poisson2d(64)
    yield "tpfa3d_13x11x9", synth.lognormal_tpfa((13, 11, 9), 2.0, np.random.default_rng(1))
    yield "powerlaw_3000", synth.powerlaw_random(3000, rng)
    yield "random_777", random_sparse(777, 0.01, rng, dominant=False)


MATS = dict(_mats())


@pytest.mark.parametrize("name", list(MATS))
@pytest.mark.parametrize("width", [-1, 0, 3, 8])
def test_hec_conversion_is_bit_exact(name, width):
    A = MATS[name]
    M = hec.hec_from_csr(A, ell_width=width, keep_f32=True)
    g = hec.hec_export(M, f32=True)
    o = O.hec_from_csr(A.n, A.Ap, A.Aj, A.Ax, width)
    assert (g["K"], g["ld"], g["nnz"], g["nnz_rem"]) == (o.K, o.ld, A.nnz, o.rem_col.size)
    assert np.array_equal(g["ell_col"], o.ell_col)
    assert np.array_equal(g["ell_val"].view(np.uint64), o.ell_val.view(np.uint64))
    assert np.array_equal(g["rem_ptr"], o.rem_ptr)
    assert np.array_equal(g["rem_col"], o.rem_col)
    assert np.array_equal(g["rem_val"].view(np.uint64), o.rem_val.view(np.uint64))
    # FP32 copies are the round-to-nearest-even images of the FP64 values
    assert np.array_equal(g["ell_val32"], o.ell_val.astype(np.float32))
    assert np.array_equal(g["rem_val32"], o.rem_val.astype(np.float32))


def test_hec_conversion_degenerate_sizes():
    for n in (0, 1):
        Ap = np.zeros(n + 1, np.int32)
        Aj = np.zeros(0, np.int32)
        Ax = np.zeros(0)
        if n == 1:
            Ap[1] = 1
            Aj = np.zeros(1, np.int32)
            Ax = np.array([2.5])
        A = synth.CSR(n, Ap, Aj, Ax)
        M = hec.hec_from_csr(A)
        g = hec.hec_export(M)
        o = O.hec_from_csr(n, Ap, Aj, Ax)
        assert (g["K"], g["ld"]) == (o.K, o.ld)
        assert np.array_equal(g["ell_col"], o.ell_col) and np.array_equal(g["ell_val"], o.ell_val)


def _check_spmv(A, y_gpu, x, alpha, beta, y0, eps_rel, u):
    ref = O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, x, alpha, beta, y0)
    lens = np.diff(A.Ap)
    K = int(lens.max()) if A.n else 0
    bound = (abs(alpha) * abs_product(A, x) + abs(beta) * np.abs(y0)) * (2 * (K + 2) * u) + 1e-300
    err = np.abs(y_gpu - ref)
    assert (err <= bound).all(), float((err / bound).max())
    if np.linalg.norm(ref) > 0:
        assert np.linalg.norm(y_gpu - ref) <= eps_rel * np.linalg.norm(ref)


@pytest.mark.parametrize("name", list(MATS))
@pytest.mark.parametrize("width", [-1, 0, 3])
@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (-1.0, 1.0), (0.5, -2.0)])
def test_spmv_fp64_matches_oracle(name, width, alpha, beta):
    import torch
    A = MATS[name]
    rng = np.random.default_rng(7)
    x = rng.uniform(-1, 1, A.n)
    y0 = rng.uniform(-1, 1, A.n)
    M = hec.hec_from_csr(A, ell_width=width)
    xd, yd = dev(x), dev(y0)
    hec.hec_spmv(M, xd, yd, alpha, beta)
    _check_spmv(A, host(yd), x, alpha, beta, y0, 1e-12, U64)


def test_spmv_beta_zero_does_not_read_y():
    A = MATS["powerlaw_3000"]
    x = np.random.default_rng(3).uniform(-1, 1, A.n)
    for width in (-1, 0):
        M = hec.hec_from_csr(A, ell_width=width)
        yd = dev(np.full(A.n, np.nan))
        hec.hec_spmv(M, dev(x), yd, 1.0, 0.0)
        y = host(yd)
        assert np.isfinite(y).all()
        _check_spmv(A, y, x, 1.0, 0.0, np.zeros(A.n), 1e-12, U64)


@pytest.mark.parametrize("name", ["tpfa3d_13x11x9", "powerlaw_3000"])
@pytest.mark.parametrize("xt,yt", [("f32", "f32"), ("f64", "f64"), ("f32", "f64")])
def test_spmv_fp32_values_error_bound(name, xt, yt):
    """FP32 values (and FP32 accumulation): |y32 - y64| <= (u32 + gamma_len)|A||x| up to
    the rounding of x and y themselves."""
    import torch
    A = MATS[name]
    x = np.random.default_rng(9).uniform(-1, 1, A.n)
    M = hec.hec_from_csr(A, keep_f32=True)
    xd = dev(x, torch.float32 if xt == "f32" else torch.float64)
    yd = empty(A.n, yt)
    hec.hec_spmv(M, xd, yd, 1.0, 0.0, vals=hec.F32)
    y = host(yd).astype(np.float64)
    ref = O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, x)
    K = int(np.diff(A.Ap).max())
    bound = abs_product(A, x) * ((K + 4) * U32) * 1.01
    assert (np.abs(y - ref) <= bound).all()


def test_spmv_rejects_missing_fp32_copy():
    A = MATS["poisson2d_64"]
    M = hec.hec_from_csr(A)
    with pytest.raises(hec.HecError) as e:
        hec.hec_spmv(M, empty(A.n, "f32"), empty(A.n, "f32"), vals=hec.F32)
    assert e.value.code == hec.INVALID_ARG


def test_spmv_deterministic():
    A = MATS["powerlaw_3000"]
    x = dev(np.random.default_rng(1).uniform(-1, 1, A.n))
    M = hec.hec_from_csr(A, ell_width=4)
    ys = []
    for _ in range(3):
        y = empty(A.n)
        hec.hec_spmv(M, x, y)
        ys.append(host(y))
    assert all(np.array_equal(ys[0].view(np.uint64), y.view(np.uint64)) for y in ys)


@pytest.mark.parametrize("width", list(range(1, 10)))
def test_spmv_every_slab_width(width):
    """Every ELL width the product fixes at compile time (1-8) and the run-time width
    (9), each with a CSR remainder behind it, in FP64 and with FP32 values and vectors."""
    import torch
    A = MATS["powerlaw_3000"]
    rng = np.random.default_rng(40 + width)
    x = rng.uniform(-1, 1, A.n)
    y0 = rng.uniform(-1, 1, A.n)
    M = hec.hec_from_csr(A, ell_width=width, keep_f32=True)
    assert hec.hec_info(M)["K"] == width
    yd = dev(y0)
    hec.hec_spmv(M, dev(x), yd, 0.5, -2.0)
    _check_spmv(A, host(yd), x, 0.5, -2.0, y0, 1e-12, U64)
    y32 = empty(A.n, "f32")
    hec.hec_spmv(M, dev(x, torch.float32), y32, vals=hec.F32)
    ref = O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, x)
    K = int(np.diff(A.Ap).max())
    assert (np.abs(host(y32).astype(np.float64) - ref) <= abs_product(A, x) * ((K + 4) * U32) * 1.01).all()
