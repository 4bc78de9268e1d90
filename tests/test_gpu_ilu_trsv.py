"""GPU parity: ILU(k) pattern (bit-exact) and values, level schedules (bit-exact),
and level-scheduled triangular solves (1e-12) against the oracle."""
import numpy as np
import pytest

import oracle as O
from paper_1606_00545_amd import hec, synth
from tests._gpu import dev, empty, host
from tests._mats import random_sparse, to_dense

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def _cases():
    yield "poisson2d_64_k0", synth.poisson2d(64), 0
    yield "poisson2d_64_k0_blocked", synth.poisson2d(64), 0
    yield "tpfa3d_k0", synth.lognormal_tpfa((17, 13, 11), 2.0, np.random.default_rng(2)), 0
    yield "tpfa3d_k1", synth.lognormal_tpfa((17, 13, 11), 2.0, np.random.default_rng(2)), 1
    yield "tpfa3d_k2", synth.lognormal_tpfa((9, 8, 7), 1.0, np.random.default_rng(3)), 2
    yield "tpfa2d_k3", synth.lognormal_tpfa((31, 23), 2.0, np.random.default_rng(4)), 3
    yield "random_k1", random_sparse(500, 0.008, np.random.default_rng(5)), 1
    # several parts in the blocked solve, ragged last part
    yield "tpfa3d_41x37x23_k0", synth.lognormal_tpfa((41, 37, 23), 2.0, np.random.default_rng(6)), 0
    # the same factor with level-blocked plans (the wavefront plans switched off when it is scheduled)
    yield "tpfa3d_41x37x23_k0_blocked", synth.lognormal_tpfa((41, 37, 23), 2.0, np.random.default_rng(6)), 0
    yield "tpfa3d_k0_blocked", synth.lognormal_tpfa((17, 13, 11), 2.0, np.random.default_rng(2)), 0
    yield "tpfa3d_41x37x23_k1", synth.lognormal_tpfa((41, 37, 23), 2.0, np.random.default_rng(6)), 1
    yield "tpfa2d_301x97_k2", synth.lognormal_tpfa((301, 97), 1.5, np.random.default_rng(7)), 2
    yield "random_20000_k1", random_sparse(20000, 0.0004, np.random.default_rng(8)), 1


CASES = {name: (A, k) for name, A, k in _cases()}


@pytest.fixture(scope="module")
def built():
    out = {}
    for name, (A, k) in CASES.items():
        F = O.iluk(A.n, A.Ap, A.Aj, A.Ax, k)
        M = hec.ilu_factor(A, k=k, keep_f32=True)
        hec.set_trsv_grid(not name.endswith("_blocked"))
        try:
            lv = hec.level_schedule(M)
        finally:
            hec.set_trsv_grid(True)
        assert hec.levels_grid(lv) == (name in ("poisson2d_64_k0", "tpfa3d_k0", "tpfa3d_41x37x23_k0"))
        out[name] = (A, k, F, M, lv)
    return out


@pytest.mark.parametrize("name", list(CASES))
def test_ilu_pattern_exact_values_close(built, name):
    A, k, F, M, lv = built[name]
    LUp, LUj, LUx = hec.ilu_export(M)
    assert np.array_equal(LUp, F.LUp) and np.array_equal(LUj, F.LUj)
    # entrywise relative error, floored at 1e-3 of the largest entry for tiny fill values
    scale = np.maximum(np.abs(F.LUx), 1e-3 * np.abs(F.LUx).max())
    assert np.max(np.abs(LUx - F.LUx) / scale) <= 1e-12


@pytest.mark.parametrize("name", list(CASES))
def test_level_schedules_bit_exact(built, name):
    A, k, F, M, lv = built[name]
    g = hec.levels_export(lv)
    lo = O.level_schedule(F.n, F.LUp, F.LUj, "lower")
    up = O.level_schedule(F.n, F.LUp, F.LUj, "upper")
    assert g["nlev_lower"] == lo.nlev and g["nlev_upper"] == up.nlev
    assert np.array_equal(g["lower_ptr"], lo.level_ptr) and np.array_equal(g["lower_perm"], lo.perm)
    assert np.array_equal(g["upper_ptr"], up.level_ptr) and np.array_equal(g["upper_perm"], up.perm)


def _lu_dense(F):
    D = to_dense(F.n, F.LUp, F.LUj, F.LUx)
    return np.tril(D, -1) + np.eye(F.n), np.triu(D)


@pytest.mark.parametrize("name", list(CASES))
def test_trsv_fp64_matches_oracle(built, name):
    A, k, F, M, lv = built[name]
    rng = np.random.default_rng(11)
    b = rng.uniform(-1, 1, A.n)
    y_o = O.trsv_lower(F, b)
    x_o = O.trsv_upper(F, y_o)
    bd = dev(b)
    y, z, x = empty(A.n), empty(A.n), empty(A.n)
    hec.trsv_levels(M, lv, bd, y, hec.LOWER)
    hec.trsv_levels(M, lv, dev(y_o), z, hec.UPPER)
    hec.trsv_levels(M, lv, bd, x, hec.LU)
    y, z, x = host(y), host(z), host(x)
    for got, ref in ((y, y_o), (z, x_o), (x, x_o)):
        assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
    # componentwise backward error of the device result (substitution is backward stable)
    if A.n <= 3000:
        L, U = _lu_dense(F)
        w = int(np.diff(F.LUp).max()) + 2
        gam = 2 * w * U64
        assert (np.abs(b - L @ y) <= gam * (np.abs(L) @ np.abs(y)) + 1e-300).all()
        assert (np.abs(y_o - U @ z) <= gam * (np.abs(U) @ np.abs(z)) + 1e-300).all()


@pytest.mark.parametrize("name", ["tpfa3d_k0", "tpfa3d_k0_blocked", "tpfa3d_k1", "random_k1"])
def test_trsv_fp32_copy(built, name):
    """FP32 factor + FP32 vectors: same schedule; error against FP64 stated by a
    forward-error bound cond-free check on the residual of the FP32 result."""
    import torch
    A, k, F, M, lv = built[name]
    b = np.random.default_rng(12).uniform(-1, 1, A.n)
    x = empty(A.n, "f32")
    hec.trsv_levels(M, lv, dev(b, torch.float32), x, hec.LU)
    x = host(x).astype(np.float64)
    x_o = O.trsv_upper(F, O.trsv_lower(F, b))
    rel = np.linalg.norm(x - x_o) / np.linalg.norm(x_o)
    assert rel < 1e-4, rel


def test_trsv_repeated_calls_reuse_counters(built):
    """The persistent solve resets its own chunk counters: many calls in a row agree bit for bit."""
    A, k, F, M, lv = built["tpfa3d_k1"]
    b = dev(np.random.default_rng(13).uniform(-1, 1, A.n))
    outs = []
    for _ in range(5):
        x = empty(A.n)
        hec.trsv_levels(M, lv, b, x, hec.LU)
        outs.append(host(x))
    assert all(np.array_equal(outs[0].view(np.uint64), o.view(np.uint64)) for o in outs)


def test_zero_pivot_reported_by_device_factorisation():
    D = np.array([[1.0, 1.0, 0.0], [1.0, 1.0, 1.0], [0.0, 1.0, 3.0]])  # u_11 = 0
    from tests._mats import from_pattern
    A = from_pattern(D != 0, D)
    with pytest.raises(hec.HecError) as e:
        hec.ilu_factor(A)
    assert e.value.code == hec.ZERO_PIVOT
    with pytest.raises(O.OracleError) as e2:
        O.iluk(A.n, A.Ap, A.Aj, A.Ax, 0)
    assert e2.value.code == O.ZERO_PIVOT


def test_single_row_and_diagonal_systems():
    A = synth.CSR(1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([4.0]))
    M = hec.ilu_factor(A)
    lv = hec.level_schedule(M)
    x = empty(1)
    hec.trsv_levels(M, lv, dev(np.array([2.0])), x, hec.LU)
    assert host(x)[0] == 0.5
    n = 1000
    A = synth.CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.arange(1.0, n + 1))
    M = hec.ilu_factor(A)
    lv = hec.level_schedule(M)
    assert hec.levels_info(lv)["nlev_lower"] == 1
    x = empty(n)
    hec.trsv_levels(M, lv, dev(np.ones(n)), x, hec.LU)
    assert np.array_equal(host(x), 1.0 / np.arange(1.0, n + 1))
