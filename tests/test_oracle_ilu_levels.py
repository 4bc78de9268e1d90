"""Pins for the oracle's ILU(k) (Sec. 2.4, Alg. 2, Eq. (9)-(10)) and level schedule (Sec. 2.6, Eq. (11))."""
from collections import deque

import numpy as np
import pytest
import scipy.linalg

import oracle as O
from paper_1606_00545_amd import synth
from tests._mats import random_sparse, to_dense, tridiag


def _lu_dense(F):
    D = to_dense(F.n, F.LUp, F.LUj, F.LUx)
    L = np.tril(D, -1) + np.eye(F.n)
    U = np.triu(D)
    return L, U


def _fill_path_levels(A):
    """Level of fill by the incomplete fill-path characterisation (Hysom & Pothen):
    lev(i,j) = (length of the shortest path i -> j in the graph of A whose interior
    vertices are all numbered below min(i,j)) - 1. Brute force BFS per pair."""
    n = A.n
    adj = [list(A.Aj[A.Ap[i]:A.Ap[i + 1]]) for i in range(n)]
    lev = {}
    for i in range(n):
        for j in range(n):
            if i == j:
                lev[(i, j)] = 0
                continue
            lim = min(i, j)
            dist = {i: 0}
            q = deque([i])
            found = None
            while q and found is None:
                u = q.popleft()
                for v in adj[u]:
                    if v == j:
                        found = dist[u] + 1
                        break
                    if v < lim and v not in dist:
                        dist[v] = dist[u] + 1
                        q.append(v)
            if found is not None:
                lev[(i, j)] = found - 1
    return lev


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_iluk_pattern_equals_fill_path_levels(seed, k):
    rng = np.random.default_rng(100 + seed)
    A = random_sparse(14, 0.15, rng)
    F = O.iluk(A.n, A.Ap, A.Aj, A.Ax, k)
    got = {}
    for i in range(F.n):
        for e in range(F.LUp[i], F.LUp[i + 1]):
            got[(i, int(F.LUj[e]))] = int(F.LUlev[e])
    want = {ij: l for ij, l in _fill_path_levels(A).items() if l <= k}
    assert got == want


def test_ilu0_pattern_is_pattern_of_A():
    rng = np.random.default_rng(5)
    A = random_sparse(40, 0.08, rng)
    F = O.iluk(A.n, A.Ap, A.Aj, A.Ax, 0)
    assert np.array_equal(F.LUp, A.Ap) and np.array_equal(F.LUj, A.Aj)
    assert (F.LUlev == 0).all()


@pytest.mark.parametrize("k", [0, 1, 2])
def test_lu_product_reproduces_A_on_the_kept_pattern(k):
    """ILU(k) property: (LU)_ij = A_ij for every kept (i,j)."""
    rng = np.random.default_rng(11)
    A = synth.lognormal_tpfa((4, 5, 6), 2.0, rng)
    F = O.iluk(A.n, A.Ap, A.Aj, A.Ax, k)
    L, U = _lu_dense(F)
    LU = L @ U
    DA = to_dense(A.n, A.Ap, A.Aj, A.Ax)
    kept = to_dense(F.n, F.LUp, F.LUj, np.ones(F.LUj.size)) != 0
    err = np.abs(LU - DA)[kept].max() / np.abs(DA).max()
    assert err < 1e-14
    # off the kept pattern the product generally differs (the dropped fill)
    if k == 0:
        assert np.abs(LU - DA)[~kept].max() > 1e-3


def test_ilu0_of_tridiagonal_is_exact_lu():
    rng = np.random.default_rng(3)
    A = tridiag(30, rng)
    F = O.iluk(A.n, A.Ap, A.Aj, A.Ax, 0)
    L, U = _lu_dense(F)
    DA = to_dense(A.n, A.Ap, A.Aj, A.Ax)
    assert np.abs(L @ U - DA).max() < 1e-14 * np.abs(DA).max()


def test_ilu_with_large_k_is_dense_lu():
    """k >= n keeps every fill entry: the no-pivot LU. Diagonal dominance by columns
    makes partial pivoting choose no row exchanges, so scipy's LU is the same factorisation."""
    rng = np.random.default_rng(9)
    n = 25
    A = random_sparse(n, 0.2, rng, dominant=False)
    D = to_dense(A.n, A.Ap, A.Aj, A.Ax)
    colsum = np.abs(D).sum(0) - np.abs(np.diag(D))
    D[np.arange(n), np.arange(n)] = 1.0 + colsum
    from tests._mats import from_dense
    A = from_dense(D)
    F = O.iluk(A.n, A.Ap, A.Aj, A.Ax, n)
    L, U = _lu_dense(F)
    P, Ls, Us = scipy.linalg.lu(D)
    assert np.array_equal(P, np.eye(n))
    assert np.abs(L - Ls).max() < 1e-13 and np.abs(U - Us).max() < 1e-13 * np.abs(U).max()


def test_ilu0_2d_poisson_recurrence():
    """5-point Poisson ILU(0): u_ii = 4 - 1/u_{i-1,i-1} - 1/u_{i-m,i-m} (absent neighbours
    dropped), U off-diagonals stay -1, L_{i,i-1} = -1/u_{i-1,i-1}, L_{i,i-m} = -1/u_{i-m,i-m}."""
    m = 9
    A = synth.poisson2d(m)
    F = O.iluk(A.n, A.Ap, A.Aj, A.Ax, 0)
    D = to_dense(F.n, F.LUp, F.LUj, F.LUx)
    u = np.zeros(A.n)
    for i in range(A.n):
        x, y = i % m, i // m
        t = 4.0
        if x > 0:
            t -= 1.0 / u[i - 1]
        if y > 0:
            t -= 1.0 / u[i - m]
        u[i] = t
    assert np.abs(np.diag(D) - u).max() < 1e-14
    for i in range(A.n):
        x, y = i % m, i // m
        if x < m - 1:
            assert D[i, i + 1] == -1.0
        if y < m - 1:
            assert D[i, i + m] == -1.0
        if x > 0:
            assert abs(D[i, i - 1] + 1.0 / u[i - 1]) < 1e-15
        if y > 0:
            assert abs(D[i, i - m] + 1.0 / u[i - m]) < 1e-15


def test_iluk_fill_counts_3d():
    """3D 7-point ILU(1) adds fill at offsets +-(nx-1), +-(nx*ny-1), +-(nx*ny-nx)."""
    nx, ny, nz = 4, 5, 6
    A = synth.poisson3d(4)  # cubic helper for the 7-point closed form
    F = O.iluk(A.n, A.Ap, A.Aj, A.Ax, 1)
    m = 4
    assert F.LUp[-1] - A.nnz == 2 * 3 * (m - 1) ** 2 * m
    rng = np.random.default_rng(1)
    B = synth.lognormal_tpfa((nx, ny, nz), 1.0, rng)
    G = O.iluk(B.n, B.Ap, B.Aj, B.Ax, 1)
    fill = set()
    for i in range(B.n):
        cols = set(G.LUj[G.LUp[i]:G.LUp[i + 1]]) - set(B.Aj[B.Ap[i]:B.Ap[i + 1]])
        fill |= {int(c) - i for c in cols}
    s = nx * ny
    assert fill == {nx - 1, -(nx - 1), s - 1, -(s - 1), s - nx, -(s - nx)}


def test_ilu_zero_pivot_and_missing_diagonal():
    from tests._mats import from_dense, from_pattern
    D = np.array([[0.0, 1.0], [1.0, 1.0]])
    P = np.ones((2, 2), bool)
    A = from_pattern(P, D)  # stored zero on the diagonal
    with pytest.raises(O.OracleError) as e:
        O.iluk(A.n, A.Ap, A.Aj, A.Ax, 0)
    assert e.value.code == O.ZERO_PIVOT
    A = from_dense(np.array([[1.0, 1.0], [1.0, 0.0]]))
    with pytest.raises(O.OracleError) as e:
        O.iluk(A.n, A.Ap, A.Aj, A.Ax, 0)
    assert e.value.code == O.INVALID


# ---------------------------------------------------------------- level schedule

def _check_schedule(n, Lp, Lj, lv, which):
    lev = lv.lev
    for i in range(n):
        deps = [int(j) for j in Lj[Lp[i]:Lp[i + 1]] if (j < i if which == "lower" else j > i)]
        for j in deps:  # every dependency sits in a strictly earlier level
            assert lev[j] < lev[i]
        if lev[i] > 0:  # tight: some dependency is exactly one level earlier
            assert max(lev[j] for j in deps) == lev[i] - 1
        else:
            assert not deps
    assert lv.level_ptr[0] == 0 and lv.level_ptr[-1] == n
    assert sorted(lv.perm.tolist()) == list(range(n))
    for q in range(lv.nlev):
        rows = lv.perm[lv.level_ptr[q]:lv.level_ptr[q + 1]]
        assert (lev[rows] == q).all() and (np.diff(rows) > 0).all()


@pytest.mark.parametrize("which", ["lower", "upper"])
def test_level_schedule_invariants_random(which):
    rng = np.random.default_rng(21)
    A = random_sparse(200, 0.02, rng)
    lv = O.level_schedule(A.n, A.Ap, A.Aj, which)
    _check_schedule(A.n, A.Ap, A.Aj, lv, which)


@pytest.mark.parametrize("k,dim", [(0, 2), (1, 2), (0, 3), (1, 3)])
def test_level_schedule_closed_forms(k, dim):
    """Natural ordering: 2D ILU(0) level x+y, ILU(1) x+2y; 3D ILU(0) x+y+z, ILU(1) x+2y+3z.
    The upper schedule mirrors it with (nx-1-x, ...)."""
    rng = np.random.default_rng(2)
    shape = (5, 7) if dim == 2 else (4, 5, 6)
    A = synth.lognormal_tpfa(shape, 1.0, rng)
    F = O.iluk(A.n, A.Ap, A.Aj, A.Ax, k)
    coef = {(0, 2): (1, 1), (1, 2): (1, 2), (0, 3): (1, 1, 1), (1, 3): (1, 2, 3)}[(k, dim)]
    c = np.arange(A.n)
    nx, ny = shape[0], shape[1]
    xyz = [c % nx, (c // nx) % ny] + ([c // (nx * ny)] if dim == 3 else [])
    for which in ("lower", "upper"):
        lv = O.level_schedule(F.n, F.LUp, F.LUj, which)
        _check_schedule(F.n, F.LUp, F.LUj, lv, which)
        if which == "lower":
            want = sum(a * v for a, v in zip(coef, xyz))
        else:
            want = sum(a * (s - 1 - v) for a, s, v in zip(coef, shape, xyz))
        assert np.array_equal(lv.lev, want)
        assert lv.nlev == sum(a * (s - 1) for a, s in zip(coef, shape)) + 1


def test_level_counts_at_workload_sizes():
    """2D 64x64 ILU(0): 127 levels (2m-1)."""
    A = synth.poisson2d(64)
    lv = O.level_schedule(A.n, A.Ap, A.Aj, "lower")
    assert lv.nlev == 127


def test_zero_pivot_in_last_row_is_reported():
    """u_nn = 0 is never used to eliminate, but it is the divisor of the backward solve."""
    from tests._mats import from_pattern
    D = np.array([[1.0, 1.0], [1.0, 1.0]])  # u_11 = 1 - 1*1 = 0
    A = from_pattern(np.ones((2, 2), bool), D)
    with pytest.raises(O.OracleError) as e:
        O.iluk(A.n, A.Ap, A.Aj, A.Ax, 0)
    assert e.value.code == O.ZERO_PIVOT
