"""Pins of the AMG oracle (Sec. 2.8, Alg. 5).

Closed forms of Ruge-Stueben coarsening and direct interpolation on the 1D
Laplacian; preservation of constants by direct interpolation on zero-row-sum
rows; the first pass of the coarsening against a brute-force rescan on small
random strength graphs; the Galerkin coarse-grid correction being exact on the
coarse space; the symmetry of the V-cycle operator with matching pre- and
post-smoothing; exact Jacobi on a diagonal matrix; and the single-level case."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import amg
from paper_1606_00545_amd import synth
from tests._mats import from_dense


def test_1d_laplacian_closed_forms():
    n = 17
    H = amg.hierarchy(synth.poisson1d(n), coarse_size=2)
    lev = H.levels[0]
    assert np.array_equal(lev.cf, (np.arange(n) % 2 == 1).astype(np.int8))  # every other point is C
    P = lev.P.toarray()
    for i in range(n):
        if i % 2:
            assert P[i].tolist() == [1.0 if c == i // 2 else 0.0 for c in range(P.shape[1])]
        else:  # linear interpolation from the two C neighbours (one at the ends)
            want = np.zeros(P.shape[1])
            for j in (i - 1, i + 1):
                if 0 <= j < n:
                    want[j // 2] = 0.5
            assert np.array_equal(P[i], want)
    Ac = H.levels[1].A.toarray()
    nc = Ac.shape[0]
    assert np.array_equal(Ac, np.diag(np.ones(nc)) - 0.5 * (np.eye(nc, k=1) + np.eye(nc, k=-1)))


def test_direct_interpolation_preserves_constants_on_zero_row_sums():
    A = synth.poisson3d(10)
    H = amg.hierarchy(A, coarse_size=10)
    M, P = H.levels[0].A, H.levels[0].P
    rowsum = np.asarray(M.sum(axis=1)).ravel()
    psum = np.asarray(P.sum(axis=1)).ravel()
    z = rowsum == 0
    assert z.any()
    assert np.allclose(psum[z], 1.0, rtol=0, atol=1e-14)
    assert (psum[~z] <= 1.0 + 1e-14).all()


def _brute_split(n, Sp, Sj):
    """Ruge-Stueben first pass by rescanning every undecided point at each step."""
    T = [[] for _ in range(n)]
    for i in range(n):
        for j in Sj[Sp[i]:Sp[i + 1]]:
            T[j].append(i)
    state = ["U"] * n
    lam = [len(T[i]) for i in range(n)]
    for i in range(n):
        if Sp[i + 1] == Sp[i] and not T[i]:
            state[i] = "F"
    while "U" in state:
        best = max((lam[i], -i) for i in range(n) if state[i] == "U")
        i = -best[1]
        state[i] = "C"
        for j in T[i]:
            if state[j] == "U":
                state[j] = "F"
                for k in Sj[Sp[j]:Sp[j + 1]]:
                    if state[k] == "U":
                        lam[k] += 1
        for k in Sj[Sp[i]:Sp[i + 1]]:
            if state[k] == "U":
                lam[k] -= 1
    return np.array([s == "C" for s in state], np.int8)


@pytest.mark.parametrize("seed", range(6))
def test_first_pass_matches_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = 60
    D = np.zeros((n, n))
    for i in range(n):
        for j in rng.choice(n, size=int(rng.integers(0, 6)), replace=False):
            if j != i:
                D[i, j] = -rng.uniform(0.05, 1.0)
        D[i, i] = 1.0 - D[i].sum()
    M = sp.csr_matrix(D)
    M.sort_indices()
    Sp, Sj = amg.strength(M, 0.25)
    assert np.array_equal(amg.rs_split(n, Sp, Sj), _brute_split(n, Sp, Sj))


def test_coarse_grid_correction_is_exact_on_the_coarse_space():
    # with no smoothing and an exact coarse solve, one cycle returns P y for b = A P y
    A = synth.lognormal_tpfa((9, 8, 7), 1.5, np.random.default_rng(3))
    H = amg.hierarchy(A, max_levels=2, coarse_size=1, nu1=0, nu2=0)
    assert len(H.levels) == 2
    P = H.levels[0].P
    y = np.random.default_rng(4).uniform(-1, 1, P.shape[1])
    b = H.levels[0].A @ (P @ y)
    x = amg.vcycle(H, b)
    assert np.linalg.norm(x - P @ y) <= 1e-12 * np.linalg.norm(P @ y)


def test_vcycle_operator_is_symmetric():
    A = synth.lognormal_tpfa((12, 10, 8), 2.0, np.random.default_rng(5))
    H = amg.hierarchy(A, coarse_size=20)
    assert len(H.levels) >= 3
    rng = np.random.default_rng(6)
    u, v = rng.uniform(-1, 1, A.n), rng.uniform(-1, 1, A.n)
    a, b = u @ amg.vcycle(H, v), v @ amg.vcycle(H, u)
    assert abs(a - b) <= 1e-12 * (abs(a) + abs(b))


def test_diagonal_matrix_is_one_level_and_exact():
    d = np.arange(1.0, 101.0)
    A = from_dense(np.diag(d))
    H = amg.hierarchy(A, coarse_size=10)
    assert len(H.levels) == 1  # no strong connections: nothing to coarsen
    b = np.ones(100)
    r = amg.solve(H, b)
    assert r.iterations == 1 and np.allclose(r.x, 1.0 / d, rtol=1e-15, atol=0)


def test_jacobi_with_unit_weight_is_exact_on_a_diagonal_level():
    d = np.arange(2.0, 202.0)
    A = from_dense(np.diag(d))
    H = amg.hierarchy(A, coarse_size=1000, omega=1.0)
    lev = H.levels[0]
    x = amg._jacobi(lev, np.zeros(200), np.ones(200), 1.0, 1)
    assert np.array_equal(x, 1.0 / d)


def test_3d_poisson_converges_in_few_cycles():
    A = synth.poisson3d(20)
    H = amg.hierarchy(A)
    b = np.random.default_rng(7).uniform(-1, 1, A.n)
    r = amg.solve(H, b, rtol=1e-8)
    assert r.converged and r.iterations <= 12
    assert np.linalg.norm(b - H.levels[0].A @ r.x) <= 1e-8 * np.linalg.norm(b)


def _non_m_matrix():
    """5 x 5, diagonal 4, the 1D chain -1 couplings, and positive couplings
    a_03 = a_30 = 0.5, a_24 = a_42 = 0.3, a_04 = a_40 = 0.05."""
    D = 4.0 * np.eye(5) - np.eye(5, k=1) - np.eye(5, k=-1)
    for (i, j), v in {(0, 3): 0.5, (2, 4): 0.3, (0, 4): 0.05}.items():
        D[i, j] = D[j, i] = v
    return from_dense(D)


def test_direct_interpolation_positive_couplings_worked_example():
    """Sec. 2.8's RSD on a matrix with positive off-diagonal entries, by hand (theta = 0.25).
    Strength (negative couplings) is that of the 1D chain, so the first pass gives
    C = {1, 3} (point 1 first: largest measure, smallest index; 0 and 2 become F, 3 gains
    one; then 3; 4 becomes F). Strong positive couplings (a_ij >= theta * the row's largest
    positive entry): row 0 -> {3} (0.05 < 0.125 is weak), row 2 -> {4}, row 4 -> {2}.
    Row 0: alpha = -1/-1 = 1, beta = (0.5 + 0.05)/0.5 = 1.1 (its strong positive neighbour 3
      is C), w_01 = -1 * (-1)/4 = 0.25, w_03 = -1.1 * 0.5/4 = -0.1375.
    Row 2: its strong positive neighbour 4 is F, so 0.3 is lumped: a_22 -> 4.3, alpha = 1,
      w_21 = w_23 = 1/4.3.
    Row 4: positive neighbours 0 and 2 are F: a_44 -> 4 + 0.35, w_43 = 1/4.35."""
    H = amg.hierarchy(_non_m_matrix(), coarse_size=1)
    lev = H.levels[0]
    assert lev.cf.tolist() == [0, 1, 0, 1, 0]
    want = np.array([[0.25, -0.1375], [1, 0], [1 / 4.3, 1 / 4.3], [0, 1], [0, 1 / 4.35]])
    assert np.allclose(lev.P.toarray(), want, rtol=1e-15, atol=0)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_direct_interpolation_weight_sums_on_non_m_matrices(seed):
    """For an F row, alpha_i and beta_i make the weights sum to -(sum_{j != i} a_ij)/a_ii when
    the row interpolates from both signs, and to -(negative sum)/(a_ii + positive sum) when
    its positive entries are lumped; both branches occur on these matrices."""
    rng = np.random.default_rng(seed)
    A = synth.poisson2d(14)
    M = A.to_scipy().tolil()
    n = A.n
    for _ in range(60):  # symmetric positive couplings between random pairs of points
        i, j = rng.integers(0, n, 2)
        if i != j:
            v = rng.uniform(0.05, 0.8)
            M[i, j] = M[j, i] = v
    M = M.tocsr()
    M.sort_indices()
    H = amg.hierarchy(from_dense(M.toarray()), coarse_size=8)
    lev = H.levels[0]
    P, cf = lev.P.tocsr(), lev.cf
    Sp, Sj = amg.strength(lev.A, 0.25)
    seen = set()
    for i in range(n):
        if cf[i]:
            continue
        row = M.getrow(i)
        cols, vals = row.indices, row.data
        aii = vals[cols == i][0]
        off = cols != i
        neg, pos = vals[off & (vals < 0)].sum(), vals[off & (vals > 0)].sum()
        mpos = vals[off & (vals > 0)].max(initial=0.0)
        spos = [j for j, v in zip(cols, vals) if j != i and v > 0 and v >= 0.25 * mpos and cf[j]]
        sneg = [j for j in Sj[Sp[i]:Sp[i + 1]] if cf[j]]
        if not sneg:
            continue
        wsum = P.getrow(i).sum()
        if spos:
            seen.add("beta")
            assert abs(wsum + (neg + pos) / aii) <= 1e-14
        else:
            seen.add("lumped" if pos > 0 else "plain")
            assert abs(wsum + neg / (aii + pos)) <= 1e-14
    assert {"beta", "lumped"} <= seen


# ---------------------------------------------------------------- Chebyshev smoother

def _cheb_T(nu, y):
    """The Chebyshev polynomial of the first kind from its trigonometric / hyperbolic form."""
    if abs(y) <= 1.0:
        return np.cos(nu * np.arccos(y))
    if y > 1.0:
        return np.cosh(nu * np.arccosh(y))
    return (-1) ** nu * np.cosh(nu * np.arccosh(-y))


def test_gershgorin_bound_closed_forms():
    # 1D and 2D Dirichlet Poisson: interior rows give (2 + 1 + 1) / 2 and (4 + 4) / 4
    assert amg.gershgorin_dinv_a(amg._csr(synth.poisson1d(50))) == 2.0
    assert amg.gershgorin_dinv_a(amg._csr(synth.poisson2d(9))) == 2.0
    # a hand example: rows (4 + 1 + 2) / 4, (1 + 5) / 5, (3 + 2) / 2
    D = np.array([[4.0, -1.0, 2.0], [1.0, 5.0, 0.0], [0.0, -3.0, 2.0]])
    assert amg.gershgorin_dinv_a(amg._csr(from_dense(D))) == 2.5
    # it bounds the spectral radius of D^{-1} A
    A = synth.lognormal_tpfa((9, 8, 7), 2.0, np.random.default_rng(4))
    M = amg._csr(A).toarray()
    rad = np.abs(np.linalg.eigvals(M / np.diag(M)[:, None])).max()
    assert rad <= amg.gershgorin_dinv_a(amg._csr(A)) * (1 + 1e-14)


@pytest.mark.parametrize("nu", [1, 2, 3, 4, 6])
@pytest.mark.parametrize("lower", [0.3, 0.1])
def test_chebyshev_on_1d_poisson_eigenvectors(nu, lower):
    """On v_j(i) = sin(i j pi / (m + 1)), an eigenvector of D^{-1} A for the 1D Dirichlet
    Poisson matrix with eigenvalue mu_j = 1 - cos(j pi / (m + 1)), nu sweeps from x = v_j
    with b = 0 leave p_nu(mu_j) v_j, p_nu(t) = T_nu((theta - t) / delta) / T_nu(theta / delta)
    on the interval [lower * 2, 2] (2 = the Gershgorin bound): a wrong coefficient of the
    recurrence changes the polynomial."""
    m = 63
    M = amg._csr(synth.poisson1d(m))
    lmax = amg.gershgorin_dinv_a(M)
    lo = lower * lmax
    theta, delta = (lmax + lo) / 2, (lmax - lo) / 2
    i = np.arange(1, m + 1)
    for j in (1, 7, 20, 32, 45, 63):
        v = np.sin(i * j * np.pi / (m + 1))
        mu = 1.0 - np.cos(j * np.pi / (m + 1))
        x = amg.chebyshev(M, 1.0 / M.diagonal(), lmax, v.copy(), np.zeros(m), nu, lower)
        p = _cheb_T(nu, (theta - mu) / delta) / _cheb_T(nu, theta / delta)
        assert np.linalg.norm(x - p * v) <= 1e-13 * np.linalg.norm(v), (j, p)
        if lo <= mu <= lmax:  # equioscillation: |p| <= 1 / T_nu(theta / delta) on the interval
            assert abs(p) <= 1.0 / _cheb_T(nu, theta / delta) * (1 + 1e-12)


def test_chebyshev_on_2d_poisson_eigenvectors():
    """The same on the 2D 5-point operator: v = sin (x) sin, mu = 1 - (cos(j pi h) + cos(k pi h)) / 2."""
    m, nu = 20, 4
    M = amg._csr(synth.poisson2d(m))
    lmax = amg.gershgorin_dinv_a(M)
    lo = 0.3 * lmax
    theta, delta = (lmax + lo) / 2, (lmax - lo) / 2
    h = np.pi / (m + 1)
    g = np.arange(1, m + 1)
    for j, k in ((1, 1), (3, 17), (10, 10), (20, 5), (20, 20)):
        v = np.outer(np.sin(g * k * h), np.sin(g * j * h)).ravel()  # row index y, column x
        mu = 1.0 - (np.cos(j * h) + np.cos(k * h)) / 2
        x = amg.chebyshev(M, 1.0 / M.diagonal(), lmax, v.copy(), np.zeros(m * m), nu)
        p = _cheb_T(nu, (theta - mu) / delta) / _cheb_T(nu, theta / delta)
        assert np.linalg.norm(x - p * v) <= 1e-13 * np.linalg.norm(v)


def test_chebyshev_degree_one_is_jacobi_with_weight_one_over_theta():
    A = synth.lognormal_tpfa((11, 9), 1.5, np.random.default_rng(3))
    M = amg._csr(A)
    rng = np.random.default_rng(4)
    x0, b = rng.uniform(-1, 1, A.n), rng.uniform(-1, 1, A.n)
    dinv = 1.0 / M.diagonal()
    lmax = amg.gershgorin_dinv_a(M)
    theta = (lmax + 0.3 * lmax) / 2
    x1 = amg.chebyshev(M, dinv, lmax, x0.copy(), b, 1)
    lev = amg.Level(M, dinv=dinv)
    xj = amg._jacobi(lev, x0.copy(), b, 1.0 / theta, 1)
    assert np.abs(x1 - xj).max() <= 1e-15 * np.abs(xj).max()


def test_chebyshev_vcycle_converges_and_is_symmetric():
    """With equal pre- and post-smoothing degrees the V-cycle is a symmetric operator
    (the smoother's polynomial in D^{-1} A is self-adjoint in the A inner product, and
    its adjoint is the same sweep order), and the cycle converges fast on 3D Poisson."""
    A = synth.poisson3d(8)
    H = amg.hierarchy(A, coarse_size=20, smoother="chebyshev", nu1=2, nu2=2)
    n = A.n
    E = np.stack([amg.vcycle(H, e, np.zeros(n)) for e in np.eye(n)], axis=1)
    assert np.abs(E - E.T).max() <= 1e-12 * np.abs(E).max()
    b = np.random.default_rng(2).uniform(-1, 1, n)
    r = amg.solve(H, b, rtol=1e-10, maxit=30)
    assert r.converged and r.iterations <= 10
