"""Small matrices built inside the tests (tridiagonal, random sparse, dense-from-CSR helpers)."""
import numpy as np

from paper_1606_00545_amd.synth import CSR


def from_dense(D):
    n = D.shape[0]
    Ap = [0]
    Aj = []
    Ax = []
    for i in range(n):
        for j in range(n):
            if D[i, j] != 0.0:
                Aj.append(j)
                Ax.append(D[i, j])
        Ap.append(len(Aj))
    return CSR(n, np.array(Ap, np.int32), np.array(Aj, np.int32), np.array(Ax, np.float64))


def from_pattern(P, V):
    """CSR with the boolean pattern P and values V (explicit zeros allowed)."""
    n = P.shape[0]
    Ap = [0]
    Aj = []
    Ax = []
    for i in range(n):
        for j in range(n):
            if P[i, j]:
                Aj.append(j)
                Ax.append(V[i, j])
        Ap.append(len(Aj))
    return CSR(n, np.array(Ap, np.int32), np.array(Aj, np.int32), np.array(Ax, np.float64))


def to_dense(n, Ap, Aj, Ax):
    D = np.zeros((n, n))
    for i in range(n):
        for e in range(Ap[i], Ap[i + 1]):
            D[i, Aj[e]] = Ax[e]
    return D


def tridiag(n, rng):
    D = np.zeros((n, n))
    for i in range(n):
        D[i, i] = 4.0 + rng.random()
        if i > 0:
            D[i, i - 1] = -1.0 + 0.5 * rng.random()
        if i < n - 1:
            D[i, i + 1] = -1.0 + 0.5 * rng.random()
    return from_dense(D)


def random_sparse(n, density, rng, dominant=True, sym_pattern=False):
    P = rng.random((n, n)) < density
    if sym_pattern:
        P = P | P.T
    np.fill_diagonal(P, True)
    V = rng.standard_normal((n, n))
    if dominant:
        V[np.arange(n), np.arange(n)] = 1.0 + (np.abs(V) * P).sum(1)
    return from_pattern(P, V)


def identity_factor(n):
    import oracle as O
    return O.Factor(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32),
                    np.ones(n), np.zeros(n, np.int32))


def poisson2d_positive(m, pairs, rng):
    """2D 5-point Poisson (m x m) plus `pairs` symmetric positive couplings between random
    points at most two cells apart, each added to both diagonals as well: a symmetric,
    diagonally dominant (so SPD) matrix that is not an M-matrix."""
    n = m * m
    D = np.zeros((n, n))
    for y in range(m):
        for x in range(m):
            i = x + m * y
            D[i, i] = 4.0
            for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                if 0 <= x + dx < m and 0 <= y + dy < m:
                    D[i, x + dx + m * (y + dy)] = -1.0
    for _ in range(pairs):
        x, y = rng.integers(0, m, 2)
        dx, dy = rng.integers(-2, 3, 2)
        if (dx, dy) == (0, 0) or not (0 <= x + dx < m and 0 <= y + dy < m):
            continue
        i, j = x + m * y, x + dx + m * (y + dy)
        if D[i, j] != 0.0:
            continue
        v = float(rng.uniform(0.1, 0.6))
        D[i, j] = D[j, i] = v
        D[i, i] += v
        D[j, j] += v
    return from_dense(D)
