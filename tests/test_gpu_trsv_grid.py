"""GPU parity of the wavefront triangular solve (ILU(0) factors of 7-point stencils on 3D
grids and 5-point stencils on 2D grids, Sec. 2.6, Eq. (11)) against the oracle's
substitution: lone lower and upper solves and the L-then-U chain, FP64 within 1e-12 and
with a componentwise backward-error bound, FP32 within the FP32 bound, ragged tiles along
both tile axes, columns along x, y or z, and the level-blocked kernel on the same
schedule for comparison. Calls in any order
reuse the face buffers and counters correctly (bit-identical repeats)."""
import numpy as np
import pytest

import oracle as O
from paper_1606_00545_amd import hec, synth
from tests._gpu import dev, empty, host
from tests._mats import to_dense

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53

# (shape, seed): columns along z (cubic, ragged 19 x 13), along x (41 longest), along y,
# one tile with a ragged second one, the smallest grid with a plan, long columns (many
# steps at which every lane of a whole tile has a row, next to ragged tiles); 2D grids
# (64 x 1 tiles): one tile, three along x with a ragged last (columns along y), two
# along y (columns along x), and single tiles with 20 and with 16 (the fewest) of their
# 64 lanes in the grid
SHAPES = [((24, 24, 24), 1), ((19, 13, 30), 2), ((41, 37, 23), 3), ((13, 45, 16), 4), ((9, 8, 10), 5),
          ((8, 8, 8), 6), ((19, 13, 70), 7), ((64, 64, 1), 8), ((130, 200, 1), 9), ((150, 70, 1), 10),
          ((20, 33, 1), 11), ((16, 300, 1), 12)]


@pytest.fixture(scope="module")
def built():
    out = {}
    for shape, seed in SHAPES:
        A = synth.lognormal_tpfa(shape, 2.0, np.random.default_rng(seed))
        F = O.iluk(A.n, A.Ap, A.Aj, A.Ax, 0)
        M = hec.ilu_factor(A, k=0, keep_f32=True)
        lv = hec.level_schedule(M)
        out[shape] = (A, F, M, lv)
    return out


@pytest.fixture(autouse=True)
def _grid_on():
    hec.set_trsv_grid(True)
    yield
    hec.set_trsv_grid(True)


@pytest.mark.parametrize("shape", [s for s, _ in SHAPES])
def test_wavefront_fp64_matches_oracle(built, shape):
    A, F, M, lv = built[shape]
    assert hec.levels_grid(lv)
    b = np.random.default_rng(31).uniform(-1, 1, A.n)
    y_o = O.trsv_lower(F, b)
    x_o = O.trsv_upper(F, y_o)
    bd = dev(b)
    y, z, x = empty(A.n), empty(A.n), empty(A.n)
    hec.trsv_levels(M, lv, bd, y, hec.LOWER)
    hec.trsv_levels(M, lv, dev(y_o), z, hec.UPPER)
    hec.trsv_levels(M, lv, bd, x, hec.LU)
    hec.levels_check(lv)
    y, z, x = host(y), host(z), host(x)
    for got, ref in ((y, y_o), (z, x_o), (x, x_o)):
        assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
    if A.n <= 3000:  # componentwise backward error (substitution is backward stable)
        D = to_dense(F.n, F.LUp, F.LUj, F.LUx)
        L, U = np.tril(D, -1) + np.eye(F.n), np.triu(D)
        gam = 2 * 9 * U64
        assert (np.abs(b - L @ y) <= gam * (np.abs(L) @ np.abs(y)) + 1e-300).all()
        assert (np.abs(y_o - U @ z) <= gam * (np.abs(U) @ np.abs(z)) + 1e-300).all()


@pytest.mark.parametrize("shape", [(24, 24, 24), (41, 37, 23), (130, 200, 1)])
def test_wavefront_agrees_with_blocked_kernel(built, shape):
    """The switch is read when a schedule is built: a second schedule of the same factor
    built with it off has level-blocked plans and gives the same results within rounding."""
    A, F, M, lv = built[shape]
    hec.set_trsv_grid(False)
    try:
        lvb = hec.level_schedule(M)
    finally:
        hec.set_trsv_grid(True)
    assert hec.levels_grid(lv) and not hec.levels_grid(lvb)
    gb, bb = hec.levels_export(lv), hec.levels_export(lvb)  # the same level schedules either way
    for k in ("lower_ptr", "lower_perm", "upper_ptr", "upper_perm"):
        assert np.array_equal(gb[k], bb[k])
    bd = dev(np.random.default_rng(32).uniform(-1, 1, A.n))
    xg, xb = empty(A.n), empty(A.n)
    hec.trsv_levels(M, lv, bd, xg, hec.LU)
    hec.trsv_levels(M, lvb, bd, xb, hec.LU)
    hec.levels_check(lv)
    hec.levels_check(lvb)
    xg, xb = host(xg), host(xb)
    assert np.linalg.norm(xg - xb) <= 1e-13 * np.linalg.norm(xb)


@pytest.mark.parametrize("shape", [(24, 24, 24), (19, 13, 30), (150, 70, 1)])
def test_wavefront_fp32(built, shape):
    import torch
    A, F, M, lv = built[shape]
    b = np.random.default_rng(33).uniform(-1, 1, A.n)
    x = empty(A.n, "f32")
    hec.trsv_levels(M, lv, dev(b, torch.float32), x, hec.LU)
    hec.levels_check(lv)
    x_o = O.trsv_upper(F, O.trsv_lower(F, b))
    rel = np.linalg.norm(host(x).astype(np.float64) - x_o) / np.linalg.norm(x_o)
    assert rel < 1e-4, rel


def test_calls_in_any_order_repeat_bit_for_bit(built):
    """Lone solves and chains interleaved (each launch fills the face buffer a later one
    uses): every repeat of a call gives the same bits."""
    A, F, M, lv = built[(19, 13, 30)]
    b = dev(np.random.default_rng(34).uniform(-1, 1, A.n))
    seq = [hec.LU, hec.LOWER, hec.LU, hec.UPPER, hec.UPPER, hec.LU, hec.LOWER, hec.LOWER, hec.LU]
    first = {}
    for which in seq:
        x = empty(A.n)
        hec.trsv_levels(M, lv, b, x, which)
        got = host(x)
        if which in first:
            assert np.array_equal(first[which].view(np.uint64), got.view(np.uint64)), which
        else:
            first[which] = got
    hec.levels_check(lv)


def test_no_plan_where_it_does_not_apply():
    for A, k in ((synth.poisson3d(16), 1), (synth.poisson2d(64), 1),
                 (synth.lognormal_tpfa((7, 30, 30), 1.0, np.random.default_rng(3)), 0),
                 (synth.lognormal_tpfa((12, 90, 1), 1.0, np.random.default_rng(3)), 0)):
        lv = hec.level_schedule(hec.ilu_factor(A, k=k))
        assert not hec.levels_grid(lv)
