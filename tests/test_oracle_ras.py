"""Pins of the oracle's restricted additive Schwarz preconditioner (Sec. 2.5).

Each check reduces RAS to something fixed independently: closed-form extended
blocks on chains and grids, the global ILU when nothing is dropped, Jacobi when
every block is one row, and the exact inverse of the block-diagonal part when the
block factorisation is exact."""
import numpy as np
import pytest

import oracle as O
from paper_1606_00545_amd import synth
from tests._mats import random_sparse, to_dense


def _global_apply(A, r, k=0):
    F = O.iluk(A.n, A.Ap, A.Aj, A.Ax, k)
    return O.trsv_upper(F, O.trsv_lower(F, r))


@pytest.mark.parametrize("n,nb,ov", [(37, 4, 0), (37, 4, 2), (40, 5, 1), (9, 9, 3), (10, 1, 5)])
def test_chain_extension_closed_form(n, nb, ov):
    A = synth.poisson1d(n)
    R = -(-n // nb)
    for b, (own, ext) in enumerate(O.ras_blocks(A.n, A.Ap, A.Aj, nb, ov)):
        s0, e0 = b * R, min(n, (b + 1) * R)
        assert np.array_equal(own, np.arange(s0, e0))
        assert np.array_equal(ext, np.arange(max(0, s0 - ov), min(n, e0 + ov)))


def test_grid_line_blocks_one_layer_closed_form():
    m = 8
    A = synth.poisson2d(m)  # blocks of 2 whole grid lines: one layer adds the neighbouring lines
    for b, (own, ext) in enumerate(O.ras_blocks(A.n, A.Ap, A.Aj, 4, 1)):
        a, c = 2 * b, 2 * b + 2
        assert np.array_equal(ext, np.arange(max(0, (a - 1) * m), min(m * m, (c + 1) * m)))


@pytest.mark.parametrize("k", [0, 1])
def test_one_block_is_the_global_ilu(k):
    A = synth.lognormal_tpfa((7, 6, 5), 2.0, np.random.default_rng(1))
    r = np.random.default_rng(2).uniform(-1, 1, A.n)
    z = O.ras_apply(O.ras_factor(A, 1, 0, k), r)
    assert np.array_equal(z.view(np.uint64), _global_apply(A, r, k).view(np.uint64))


def test_overlap_covering_everything_is_the_global_ilu():
    A = synth.poisson2d(6)  # graph diameter 10: 10 layers reach every row from any block
    r = np.random.default_rng(3).uniform(-1, 1, A.n)
    blocks = O.ras_factor(A, 3, 10)
    assert all(B.ext.size == A.n for B in blocks)
    z = O.ras_apply(blocks, r)
    assert np.array_equal(z.view(np.uint64), _global_apply(A, r).view(np.uint64))


def test_one_row_blocks_are_jacobi():
    A = synth.lognormal_tpfa((9, 7), 1.5, np.random.default_rng(4))
    r = np.random.default_rng(5).uniform(-1, 1, A.n)
    z = O.ras_apply(O.ras_factor(A, A.n, 0), r)
    d = to_dense(A.n, A.Ap, A.Aj, A.Ax).diagonal()
    assert np.array_equal(z, r / d)


def test_uncoupled_blocks_lose_nothing():
    rng = np.random.default_rng(6)
    D = np.zeros((40, 40))
    for s in (0, 20):  # two independent 20 x 20 blocks
        B = to_dense(*_dense_parts(random_sparse(20, 0.15, rng)))
        D[s:s + 20, s:s + 20] = B
    from tests._mats import from_dense
    A = from_dense(D)
    r = rng.uniform(-1, 1, 40)
    z = O.ras_apply(O.ras_factor(A, 2, 0), r)
    assert np.array_equal(z.view(np.uint64), _global_apply(A, r).view(np.uint64))


def _dense_parts(A):
    return A.n, A.Ap, A.Aj, A.Ax


def test_exact_block_factors_invert_the_block_diagonal_part():
    rng = np.random.default_rng(7)
    A = random_sparse(30, 0.2, rng)
    D = to_dense(A.n, A.Ap, A.Aj, A.Ax)
    nb = 3
    blocks = O.ras_factor(A, nb, 0, k=30)  # level 30 >= block size: complete LU of each block
    r = rng.uniform(-1, 1, 30)
    z = O.ras_apply(blocks, r)
    BD = np.zeros_like(D)
    for s in range(0, 30, 10):
        BD[s:s + 10, s:s + 10] = D[s:s + 10, s:s + 10]
    assert np.allclose(BD @ z, r, rtol=0, atol=1e-12 * np.abs(r).max())


def test_restriction_keeps_each_blocks_own_rows():
    # tridiagonal blocks: ILU(0) is the exact LU, so each block's solve is A_ext^{-1} r_ext
    n, nb, ov = 30, 4, 2
    A = synth.poisson1d(n)
    D = to_dense(A.n, A.Ap, A.Aj, A.Ax)
    r = np.random.default_rng(8).uniform(-1, 1, n)
    z = O.ras_apply(O.ras_factor(A, nb, ov), r)
    R = -(-n // nb)
    for b in range(nb):
        s0, e0 = b * R, min(n, (b + 1) * R)
        lo, hi = max(0, s0 - ov), min(n, e0 + ov)
        zb = np.linalg.solve(D[lo:hi, lo:hi], r[lo:hi])
        assert np.allclose(z[s0:e0], zb[s0 - lo:e0 - lo], rtol=1e-13, atol=1e-14)
