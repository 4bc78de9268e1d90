"""Pins for the oracle's SpMV (Alg. 1 / Eq. (2)) and HEC layout (Sec. 2.1), and for the generators."""
import os

import numpy as np
import pytest

import oracle as O
from paper_1606_00545_amd import synth
from tests._mats import from_dense, random_sparse, to_dense

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("n,density", [(1, 1.0), (7, 0.3), (33, 0.2), (64, 0.05)])
def test_spmv_matches_dense_product(n, density):
    rng = np.random.default_rng(n)
    A = random_sparse(n, density, rng, dominant=False)
    D = to_dense(A.n, A.Ap, A.Aj, A.Ax)
    x = rng.standard_normal(n)
    y0 = rng.standard_normal(n)
    for alpha, beta in [(1.0, 0.0), (-1.0, 1.0), (2.5, -0.75)]:
        y = O.csr_spmv(n, A.Ap, A.Aj, A.Ax, x, alpha, beta, y0)
        ref = alpha * (D @ x) + beta * y0
        assert np.allclose(y, ref, rtol=1e-14, atol=1e-14 * np.abs(D).sum())


def test_spmv_beta_zero_ignores_y():
    rng = np.random.default_rng(0)
    A = random_sparse(20, 0.2, rng)
    y0 = np.full(20, np.nan)
    y = O.csr_spmv(20, A.Ap, A.Aj, A.Ax, np.ones(20), 1.0, 0.0, y0)
    assert np.isfinite(y).all()


def test_spmv_empty_rows_and_zero_size():
    D = np.zeros((4, 4))
    D[1, 2] = 3.0
    A = from_dense(D)
    y = O.csr_spmv(4, A.Ap, A.Aj, A.Ax, np.array([1.0, 2.0, 5.0, 7.0]))
    assert list(y) == [0.0, 15.0, 0.0, 0.0]
    y = O.csr_spmv(0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0), np.zeros(0))
    assert y.size == 0


@pytest.mark.parametrize("dim,m", [(1, 50), (2, 16), (3, 7)])
def test_spmv_poisson_closed_form_eigenpairs(dim, m):
    """Dirichlet Poisson: lambda = sum_d (2 - 2 cos(j_d pi h)), v = product of sines, h = 1/(m+1)."""
    if dim == 1:
        D = 2 * np.eye(m) - np.eye(m, k=1) - np.eye(m, k=-1)
        A = from_dense(D)
    elif dim == 2:
        A = synth.poisson2d(m)
    else:
        A = synth.poisson3d(m)
    h = 1.0 / (m + 1)
    idx = np.arange(1, m + 1)
    rng = np.random.default_rng(dim)
    for _ in range(3):
        js = rng.integers(1, m + 1, size=dim)
        s = [np.sin(idx * j * np.pi * h) for j in js]
        v = s[0]
        for k in range(1, dim):
            v = np.kron(s[k], v)  # x fastest: cell = x + m*(y + m*z)
        lam = sum(2.0 - 2.0 * np.cos(j * np.pi * h) for j in js)
        Av = O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, v)
        assert np.linalg.norm(Av - lam * v) / np.linalg.norm(v) < 1e-13


def test_generator_reproduces_paper_poisson_sizes():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "paper_sizes.txt")) if not l.startswith("#")]
    for m, n, nnz, mb in (map(int, r) for r in rows if r):
        A = synth.poisson3d(m)
        assert A.n == n and A.nnz == nnz
        if mb > 0:
            assert round((12 * A.nnz + 4 * (A.n + 1)) / 2 ** 20) == mb
        assert (A.Ax != 0).all()


@pytest.mark.parametrize("width", [-1, 0, 1, 3, 5, 100])
def test_hec_reassembles_to_the_input(width):
    rng = np.random.default_rng(7)
    A = random_sparse(300, 0.02, rng, dominant=False)
    lens = np.diff(A.Ap)
    h = O.hec_from_csr(A.n, A.Ap, A.Aj, A.Ax, width)
    K_expect = min(20 if width < 0 else width, lens.max())
    assert h.K == K_expect
    assert h.ld % 256 == 0 and h.ld >= A.n and h.ld - A.n < 256
    assert h.ell_col.size == h.K * h.ld
    nnz_ell = int(np.minimum(lens, h.K).sum())
    assert nnz_ell + h.rem_col.size == A.nnz
    for i in range(A.n):
        a = slice(A.Ap[i], A.Ap[i + 1])
        L = lens[i]
        k = min(L, h.K)
        got_c = [h.ell_col[s * h.ld + i] for s in range(k)] + list(h.rem_col[h.rem_ptr[i]:h.rem_ptr[i + 1]])
        got_v = [h.ell_val[s * h.ld + i] for s in range(k)] + list(h.rem_val[h.rem_ptr[i]:h.rem_ptr[i + 1]])
        assert got_c == list(A.Aj[a]) and got_v == list(A.Ax[a])
        for s in range(k, h.K):  # padding of a real row: value 0, own column
            assert h.ell_col[s * h.ld + i] == i and h.ell_val[s * h.ld + i] == 0.0
    for i in range(A.n, h.ld):
        for s in range(h.K):
            assert h.ell_col[s * h.ld + i] == 0 and h.ell_val[s * h.ld + i] == 0.0


def test_hec_hand_example():
    """A 3x3 example worked by hand with ELL width 2 (ld = 256).

    row 0: (0,1.) (2,2.)          -> ELL both, no remainder
    row 1: (0,3.) (1,4.) (2,5.)   -> ELL (0,3.) (1,4.), remainder (2,5.)
    row 2: (2,6.)                 -> ELL (2,6.) + padding (col 2, 0.)
    """
    D = np.array([[1.0, 0, 2.0], [3.0, 4.0, 5.0], [0, 0, 6.0]])
    A = from_dense(D)
    h = O.hec_from_csr(3, A.Ap, A.Aj, A.Ax, 2)
    assert (h.K, h.ld) == (2, 256)
    assert list(h.ell_col[0:3]) == [0, 0, 2] and list(h.ell_val[0:3]) == [1.0, 3.0, 6.0]
    assert list(h.ell_col[256:259]) == [2, 1, 2] and list(h.ell_val[256:259]) == [2.0, 4.0, 0.0]
    assert list(h.rem_ptr) == [0, 0, 1, 1]
    assert list(h.rem_col) == [2] and list(h.rem_val) == [5.0]
    x = np.array([1.0, 10.0, 100.0])
    assert list(O.csr_spmv(3, A.Ap, A.Aj, A.Ax, x)) == [201.0, 543.0, 600.0]


def test_hec_stencil_has_empty_remainder():
    A = synth.poisson3d(6)
    h = O.hec_from_csr(A.n, A.Ap, A.Aj, A.Ax)
    assert h.K == 7 and h.rem_col.size == 0 and (h.rem_ptr == 0).all()


def test_hec_zero_rows():
    h = O.hec_from_csr(0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    assert h.K == 0 and h.ld == 0 and h.rem_ptr.tolist() == [0]


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_threaded_csr_spmv_equals_the_serial_one(threads):
    """The all-cores CPU figure's product sums every row as the serial oracle does."""
    rng = np.random.default_rng(12)
    A, xt = synth.workload_diffusion3d(17, sigma=2.0, seed=3)
    y0 = rng.uniform(-1, 1, A.n)
    for alpha, beta in ((1.0, 0.0), (-1.0, 1.0), (0.5, -2.0)):
        ys = O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, xt, alpha, beta, y0)
        yp = O.csr_spmv_omp(A.n, A.Ap, A.Aj, A.Ax, xt, threads, alpha, beta, y0)
        assert np.array_equal(ys.view(np.uint64), yp.view(np.uint64))
