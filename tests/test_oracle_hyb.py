"""Pins of the oracle's ELL and HYB layouts (Sec. 2.1).

The HYB width rule is pinned by closed forms on row-length distributions chosen
so that the count of rows with at least K entries is known exactly; the layouts
by reassembly (the ELL part and the COO triplets give back A entry for entry, in
row order) and by the plain-ELL case (a width at least the longest row leaves
nothing over)."""
import numpy as np
import pytest

import oracle as O
from paper_1606_00545_amd import synth
from tests._mats import random_sparse


def _lengths_matrix(lens, seed=0):
    """A CSR matrix whose row i has lens[i] entries (diagonal first, then the next columns)."""
    n = len(lens)
    Ap = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    rng = np.random.default_rng(seed)
    Aj = np.concatenate([np.sort((i + np.arange(L)) % n) for i, L in enumerate(lens)]).astype(np.int32)
    return synth.CSR(n, Ap, Aj, rng.uniform(-1, 1, Ap[-1]))


def test_width_rule_closed_form_cyclic_lengths():
    # row i has (i % 10) + 1 entries: 900 (11 - k) rows hold k or more; need max(4096, 3000) = 4096
    A = _lengths_matrix([(i % 10) + 1 for i in range(9000)])
    assert O.hyb_width(A.n, A.Ap) == 6  # 900 * 5 = 4500 >= 4096 > 900 * 4 = 3600


def test_width_rule_small_matrices_are_all_coo():
    # fewer than 4096 rows: no width has 4096 rows holding it
    for A in (synth.poisson2d(40), synth.poisson3d(12), random_sparse(777, 0.01, np.random.default_rng(1))):
        assert O.hyb_width(A.n, A.Ap) == 0


def test_width_rule_on_3d_poisson_grids():
    # m^3 7-point grid: (m-2)^3 rows hold 7 entries, (m-2)^3 + 6 (m-2)^2 at least 6,
    # plus 12 (m-2) at least 5, plus 8 corners at least 4
    def counts(m):
        c7 = (m - 2) ** 3
        c6 = c7 + 6 * (m - 2) ** 2
        c5 = c6 + 12 * (m - 2)
        return {7: c7, 6: c6, 5: c5, 4: c5 + 8}
    for m in (16, 17, 20, 24):
        n, need = m ** 3, max(4096, m ** 3 // 3)
        want = max(k for k, c in counts(m).items() if c >= need)
        assert O.hyb_width(n, synth.poisson3d(m).Ap) == want
    assert O.hyb_width(16 ** 3, synth.poisson3d(16).Ap) == 4   # 4096 rows, only all rows reach 4096
    assert O.hyb_width(20 ** 3, synth.poisson3d(20).Ap) == 7   # 5832 interior rows >= 4096: plain ELL


@pytest.mark.parametrize("make", [
    lambda: synth.powerlaw_random(9000, np.random.default_rng(3), lmax=300),
    lambda: _lengths_matrix([(i % 10) + 1 for i in range(9000)]),
    lambda: synth.lognormal_tpfa((21, 17, 13), 2.0, np.random.default_rng(4)),
    lambda: random_sparse(500, 0.02, np.random.default_rng(5), dominant=False),
])
def test_hyb_reassembles_the_matrix(make):
    A = make()
    H = O.hyb_from_csr(A.n, A.Ap, A.Aj, A.Ax)
    K, ld = H.ell.K, H.ell.ld
    assert K == O.hyb_width(A.n, A.Ap)
    got = {}
    col = H.ell.ell_col.reshape(K, ld) if K else np.zeros((0, ld), np.int32)
    val = H.ell.ell_val.reshape(K, ld) if K else np.zeros((0, ld))
    lens = np.diff(A.Ap)
    for i in range(A.n):
        for s in range(min(K, lens[i])):
            got[(i, int(col[s, i]))] = val[s, i]
    assert (np.diff(H.coo_row) >= 0).all(), "COO rows not ascending"
    for r, c, v in zip(H.coo_row, H.coo_col, H.coo_val):
        assert (int(r), int(c)) not in got
        got[(int(r), int(c))] = v
    want = {(i, int(A.Aj[e])): A.Ax[e] for i in range(A.n) for e in range(A.Ap[i], A.Ap[i + 1])}
    assert got == want
    # each row's entries keep their column order across the two parts
    for i in range(0, A.n, max(1, A.n // 50)):
        cols = [int(col[s, i]) for s in range(min(K, lens[i]))] + list(H.coo_col[H.coo_row == i])
        assert cols == list(A.Aj[A.Ap[i]:A.Ap[i + 1]])


def test_plain_ell_leaves_no_remainder():
    A = synth.powerlaw_random(3000, np.random.default_rng(6), lmax=64)
    maxrow = int(np.diff(A.Ap).max())
    H = O.hec_from_csr(A.n, A.Ap, A.Aj, A.Ax, maxrow)
    assert H.K == maxrow and H.rem_col.size == 0
    x = np.random.default_rng(7).uniform(-1, 1, A.n)
    # the slab's padding (value 0) adds nothing: slab product equals the CSR product bit for bit
    val, col = H.ell_val.reshape(H.K, H.ld), H.ell_col.reshape(H.K, H.ld)
    y = np.zeros(A.n)
    for s in range(H.K):
        y = y + val[s, :A.n] * x[col[s, :A.n]]
    assert np.array_equal(y, O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, x))
