"""GPU restricted additive Schwarz ILU (Sec. 2.5) against the oracle's block-by-block
definition: extended blocks bit-exact, each block's factor on the pattern exactly
and within 1e-12 in value, the preconditioner solve within 1e-12, and GMRES with it
converging to the FP64 true residual (FP64 and mixed precision)."""
import numpy as np
import pytest

import oracle as O
from paper_1606_00545_amd import hec, synth
from tests._gpu import dev, empty, host

pytestmark = pytest.mark.gpu


def _cases():
    t3 = lambda: synth.lognormal_tpfa((17, 13, 11), 2.0, np.random.default_rng(41))
    yield "tpfa3d_1x0", t3, 1, 0, 0
    yield "tpfa3d_4x0", t3, 4, 0, 0
    yield "tpfa3d_8x1", t3, 8, 1, 0
    yield "tpfa3d_32x2", t3, 32, 2, 0
    yield "tpfa2d_61x45_8x1_k1", lambda: synth.lognormal_tpfa((61, 45), 2.5, np.random.default_rng(42)), 8, 1, 1
    yield "powerlaw_4000_16x1", lambda: synth.powerlaw_random(4000, np.random.default_rng(43), lmax=48), 16, 1, 0
    yield "tpfa3d_40_256x1", lambda: synth.lognormal_tpfa((40, 40, 40), 2.0, np.random.default_rng(44)), 256, 1, 0


CASES = {c[0]: c[1:] for c in _cases()}


@pytest.fixture(scope="module")
def built():
    cache = {}

    def get(name):
        if name not in cache:
            mk, nb, ov, k = CASES[name]
            A = mk()
            blocks = O.ras_factor(A, nb, ov, k)
            F = hec.ilu_factor_ras(A, nb, ov, k=k, keep_f32=True)
            lv = hec.level_schedule(F)
            cache[name] = (A, nb, ov, k, blocks, F, lv)
        return cache[name]
    return get


@pytest.mark.parametrize("name", list(CASES))
def test_ras_blocks_and_factor(built, name):
    A, nb, ov, k, blocks, F, lv = built(name)
    g = hec.ilu_ras_export(F)
    assert g["n_sys"] == A.n and g["nblocks"] == len(blocks)
    assert np.array_equal(g["block_start"], np.cumsum([0] + [B.ext.size for B in blocks]))
    assert np.array_equal(g["ext_row"], np.concatenate([B.ext for B in blocks]))
    for b, B in enumerate(blocks):  # own[i] = stacked row of i in its own block
        s0 = g["block_start"][b]
        assert np.array_equal(g["own"][B.rows], s0 + np.searchsorted(B.ext, B.rows))
    LUp, LUj, LUx = hec.ilu_export(F)
    for b, B in enumerate(blocks):
        s0, s1 = g["block_start"][b], g["block_start"][b + 1]
        Fo = B.factor
        bp = LUp[s0:s1 + 1] - LUp[s0]
        assert np.array_equal(bp, Fo.LUp)
        assert np.array_equal(LUj[LUp[s0]:LUp[s1]] - s0, Fo.LUj)
        got = LUx[LUp[s0]:LUp[s1]]
        scale = np.maximum(np.abs(Fo.LUx), 1e-3 * np.abs(Fo.LUx).max())
        assert np.max(np.abs(got - Fo.LUx) / scale) <= 1e-12


@pytest.mark.parametrize("name", list(CASES))
def test_ras_preconditioner_solve(built, name):
    import torch
    A, nb, ov, k, blocks, F, lv = built(name)
    r = np.random.default_rng(45).uniform(-1, 1, A.n)
    z_o = O.ras_apply(blocks, r)
    z = empty(A.n)
    for _ in range(3):  # repeated calls reuse the internal sentinel-filled vectors
        hec.trsv_levels(F, lv, dev(r), z, hec.LU)
    z = host(z)
    assert np.linalg.norm(z - z_o) <= 1e-12 * np.linalg.norm(z_o)
    z32 = empty(A.n, "f32")
    hec.trsv_levels(F, lv, dev(r, torch.float32), z32, hec.LU)
    assert np.linalg.norm(host(z32) - z_o) <= 1e-4 * np.linalg.norm(z_o)
    with pytest.raises(hec.HecError):
        hec.trsv_levels(F, lv, dev(r), empty(A.n), hec.LOWER)


@pytest.mark.parametrize("name", ["tpfa3d_8x1", "tpfa2d_61x45_8x1_k1", "tpfa3d_40_256x1"])
@pytest.mark.parametrize("precision", [0, 1])
def test_gmres_with_ras(built, name, precision):
    A, nb, ov, k, blocks, F, lv = built(name)
    xt = np.random.default_rng(46).uniform(-1, 1, A.n)
    b = O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, xt)
    Mh = hec.hec_from_csr(A, keep_f32=True)
    x = empty(A.n)
    info = hec.gmres_solve(Mh, F, lv, dev(b), x, restart=30, rtol=1e-8, precision=precision)
    xh = host(x)
    rr = np.linalg.norm(b - O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, xh)) / np.linalg.norm(b)
    print(f"{name} precision {precision}: it {info['iterations']} res {rr:.2e}")
    assert info["status"] == hec.OK and rr <= 1e-8


def test_ras_rejects_bad_arguments():
    A = synth.poisson2d(8)
    with pytest.raises(hec.HecError):
        hec.ilu_factor_ras(A, 0, 0)
    with pytest.raises(hec.HecError):
        hec.ilu_factor_ras(A, 2, -1)
