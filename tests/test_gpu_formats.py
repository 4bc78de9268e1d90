"""GPU parity of the ELL and HYB formats (Sec. 2.1) beside HEC and CSR: the
layouts bit-exact against the oracle's, and SpMV within the componentwise bound of
the product against the oracle's CSR product; the HYB remainder's entry-parallel
kernel is exercised on rows that span many of its 512-entry tiles, tiles that are
one row throughout, empty rows, a remainder shorter than a tile and the
all-COO case (fewer than 4096 rows)."""
import numpy as np
import pytest

import oracle as O
from paper_1606_00545_amd import hec, synth
from tests._gpu import abs_product, dev, empty, host
from tests._mats import random_sparse

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def _long_rows(n, seed):
    """Sparse rows plus a few very long ones (one of 5000 entries: about ten tiles) and empty rows."""
    rng = np.random.default_rng(seed)
    rows = []
    for i in range(n):
        if i in (7, n // 2):
            L = 5000 if i == 7 else 1300
        elif i % 97 == 5:
            L = 0
        else:
            L = int(rng.integers(1, 12))
        rows.append(np.sort(rng.choice(n, size=min(L, n), replace=False)))
    Ap = np.concatenate([[0], np.cumsum([r.size for r in rows])]).astype(np.int32)
    Aj = np.concatenate(rows).astype(np.int32)
    return synth.CSR(n, Ap, Aj, rng.uniform(-1, 1, Ap[-1]))


def _mats():
    yield "tpfa3d_41x37x23", synth.lognormal_tpfa((41, 37, 23), 2.0, np.random.default_rng(1))
    yield "powerlaw_20000", synth.powerlaw_random(20000, np.random.default_rng(2), lmax=512)
    yield "long_rows_9000", _long_rows(9000, 3)
    yield "random_777", random_sparse(777, 0.01, np.random.default_rng(4), dominant=False)
    yield "poisson3d_16", synth.poisson3d(16)


MATS = dict(_mats())


def _layouts(A):
    maxrow = int(np.diff(A.Ap).max())
    return {"ell": (maxrow, False), "hyb": (hec.WIDTH_HYB, True), "hyb_k2": (2, True), "coo": (0, True)}


def _check(A, y, x, alpha, beta, y0, u):
    ref = O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, x, alpha, beta, y0)
    K = int(np.diff(A.Ap).max())
    bound = (abs(alpha) * abs_product(A, x) + abs(beta) * np.abs(y0)) * (2 * (K + 2) * u) + 1e-300
    err = np.abs(y - ref)
    assert (err <= bound).all(), float((err / bound).max())


@pytest.mark.parametrize("name", list(MATS))
@pytest.mark.parametrize("layout", ["ell", "hyb", "hyb_k2", "coo"])
def test_layout_is_bit_exact(name, layout):
    A = MATS[name]
    width, coo = _layouts(A)[layout]
    M = hec.hec_from_csr(A, ell_width=width, coo=coo, keep_f32=True)
    g = hec.hec_export(M, f32=True)
    if width == hec.WIDTH_HYB:
        o = O.hyb_from_csr(A.n, A.Ap, A.Aj, A.Ax)
    else:
        o = O.hyb_from_csr(A.n, A.Ap, A.Aj, A.Ax, ell_width=min(width, int(np.diff(A.Ap).max())))
    assert g["K"] == o.ell.K and g["nnz_rem"] == o.coo_col.size
    assert np.array_equal(g["ell_col"], o.ell.ell_col)
    assert np.array_equal(g["ell_val"].view(np.uint64), o.ell.ell_val.view(np.uint64))
    assert np.array_equal(g["rem_ptr"], o.ell.rem_ptr)
    assert np.array_equal(g["rem_col"], o.coo_col)
    assert np.array_equal(g["rem_val"].view(np.uint64), o.coo_val.view(np.uint64))
    if layout == "ell":
        assert g["nnz_rem"] == 0


@pytest.mark.parametrize("name", list(MATS))
@pytest.mark.parametrize("layout", ["ell", "hyb", "hyb_k2", "coo"])
@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (-1.0, 1.0), (0.5, -2.0)])
def test_spmv_fp64_matches_oracle(name, layout, alpha, beta):
    A = MATS[name]
    width, coo = _layouts(A)[layout]
    rng = np.random.default_rng(11)
    x = rng.uniform(-1, 1, A.n)
    y0 = rng.uniform(-1, 1, A.n)
    M = hec.hec_from_csr(A, ell_width=width, coo=coo)
    yd = dev(y0)
    hec.hec_spmv(M, dev(x), yd, alpha, beta)
    _check(A, host(yd), x, alpha, beta, y0, U64)


@pytest.mark.parametrize("name", ["powerlaw_20000", "long_rows_9000", "random_777"])
def test_hyb_fp32_values_and_determinism(name):
    import torch
    A = MATS[name]
    x = np.random.default_rng(12).uniform(-1, 1, A.n)
    M = hec.hec_from_csr(A, ell_width=hec.WIDTH_HYB, coo=True, keep_f32=True)
    outs = []
    for _ in range(3):
        yd = empty(A.n)
        hec.hec_spmv(M, dev(x), yd)
        outs.append(host(yd))
    assert all(np.array_equal(outs[0].view(np.uint64), o.view(np.uint64)) for o in outs)
    y32 = empty(A.n, "f32")
    hec.hec_spmv(M, dev(x, torch.float32), y32, vals=hec.F32)
    ref = O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, x)
    K = int(np.diff(A.Ap).max())
    assert (np.abs(host(y32).astype(np.float64) - ref) <= abs_product(A, x) * ((K + 4) * U32) * 1.01).all()


def test_hyb_beta_zero_does_not_read_y_and_rejects_bad_flags():
    A = MATS["long_rows_9000"]
    x = np.random.default_rng(13).uniform(-1, 1, A.n)
    for width in (hec.WIDTH_HYB, 0):
        M = hec.hec_from_csr(A, ell_width=width, coo=True)
        yd = dev(np.full(A.n, np.nan))
        hec.hec_spmv(M, dev(x), yd, 1.0, 0.0)
        y = host(yd)
        assert np.isfinite(y).all()
        _check(A, y, x, 1.0, 0.0, np.zeros(A.n), U64)
    n, Ap, Aj, Ax = A.n, A.Ap, A.Aj, A.Ax
    import ctypes as C
    out = C.c_void_p()
    rc = hec.load().hec_from_csr(n, Ap.ctypes.data, Aj.ctypes.data, Ax.ctypes.data, -1, 8, None, C.byref(out))
    assert rc == hec.INVALID_ARG


@pytest.mark.parametrize("name", ["long_rows_9000", "powerlaw_20000"])
@pytest.mark.parametrize("width", [-1, 0, 2])
@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (0.5, -2.0)])
def test_hec_csr_remainder_long_rows(name, width, alpha, beta):
    """HEC's CSR remainder with rows of 1024 remainder entries or more (5000 and
    1300 in long_rows_9000), which take one workgroup each, beside short rows,
    empty rows and the pure-CSR case (width 0); FP64 within the bound, repeated
    calls bit-identical, FP32 values within their bound."""
    import torch
    A = MATS[name]
    rng = np.random.default_rng(17)
    x = rng.uniform(-1, 1, A.n)
    y0 = rng.uniform(-1, 1, A.n)
    M = hec.hec_from_csr(A, ell_width=width, keep_f32=True)
    outs = []
    for _ in range(2):
        yd = dev(y0)
        hec.hec_spmv(M, dev(x), yd, alpha, beta)
        outs.append(host(yd))
    assert np.array_equal(outs[0].view(np.uint64), outs[1].view(np.uint64))
    _check(A, outs[0], x, alpha, beta, y0, U64)
    y32 = empty(A.n, "f32")
    hec.hec_spmv(M, dev(x, torch.float32), y32, vals=hec.F32)
    ref = O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, x)
    K = int(np.diff(A.Ap).max())
    assert (np.abs(host(y32).astype(np.float64) - ref) <= abs_product(A, x) * ((K + 4) * U32) * 1.01).all()
