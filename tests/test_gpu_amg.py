"""AMG (Sec. 2.8, Alg. 5) against the oracle: the hierarchy level by level
(C/F splitting, interpolation and Galerkin operators identical: the setup takes
the same steps in the same order of operations), and V-cycle solves (cycle
counts within one of the oracle's, FP64 residual at the tolerance, solution
close to the oracle's), with the damped Jacobi and the Chebyshev smoother; edge
cases: one level, a matrix at most the coarse size, zero right-hand side, maxit
reached, bad options, a zero diagonal."""
import numpy as np
import pytest

from oracle import amg as OA
from paper_1606_00545_amd import hec, synth
from tests._gpu import dev, empty, host
from tests._mats import from_dense, poisson2d_positive

pytestmark = pytest.mark.gpu


def _cases():
    yield "poisson1d_1000", lambda: synth.poisson1d(1000), {}
    yield "poisson2d_40", lambda: synth.poisson2d(40), {}
    yield "poisson3d_20", lambda: synth.poisson3d(20), {}
    yield "tpfa3d_17x13x11", lambda: synth.lognormal_tpfa((17, 13, 11), 2.0, np.random.default_rng(1)), {}
    yield "tpfa2d_61x45_theta05", lambda: synth.lognormal_tpfa((61, 45), 1.5, np.random.default_rng(2)), \
        {"theta": 0.5}
    yield "poisson3d_16_two_levels", lambda: synth.poisson3d(16), {"max_levels": 2, "nu1": 1, "nu2": 2}
    yield "aniso3d_14", lambda: synth.lognormal_tpfa((14, 14, 14), 1.0, np.random.default_rng(3), zscale=0.01), \
        {"omega": 0.8}
    # not M-matrices: positive off-diagonal couplings reach the beta weights and the lumping
    # of direct interpolation
    yield "nonm_worked_5", _worked_non_m, {"coarse_size": 1}
    yield "poisson2d_40_positive", lambda: poisson2d_positive(40, 300, np.random.default_rng(7)), {}


def _worked_non_m():
    D = 4.0 * np.eye(5) - np.eye(5, k=1) - np.eye(5, k=-1)
    for (i, j), v in {(0, 3): 0.5, (2, 4): 0.3, (0, 4): 0.05}.items():
        D[i, j] = D[j, i] = v
    return from_dense(D)


CASES = {c[0]: c[1:] for c in _cases()}


@pytest.fixture(scope="module")
def built():
    cache = {}

    def get(name):
        if name not in cache:
            mk, opt = CASES[name]
            A = mk()
            H = OA.hierarchy(A, **opt)
            G = hec.amg_setup(A, **opt)
            cache[name] = (A, opt, H, G)
        return cache[name]
    return get


@pytest.mark.parametrize("name", list(CASES))
def test_hierarchy_matches_oracle(built, name):
    A, opt, H, G = built(name)
    info = hec.amg_info(G)
    assert info["levels"] == len(H.levels)
    for l, lev in enumerate(H.levels):
        g = hec.amg_export_level(G, l)
        M = lev.A
        Ap, Aj, Ax = g["A"]
        assert info["n"][l] == M.shape[0]
        assert np.array_equal(Ap, M.indptr) and np.array_equal(Aj, M.indices)
        assert np.array_equal(Ax, M.data), f"level {l}: A values"
        if l + 1 < len(H.levels):
            assert np.array_equal(g["cf"], lev.cf), f"level {l}: C/F splitting"
            Pp, Pj, Px = g["P"]
            assert np.array_equal(Pp, lev.P.indptr) and np.array_equal(Pj, lev.P.indices)
            assert np.array_equal(Px, lev.P.data), f"level {l}: P values"


@pytest.mark.parametrize("name", list(CASES))
def test_solve_matches_oracle(built, name):
    A, opt, H, G = built(name)
    xt = np.random.default_rng(5).uniform(-1, 1, A.n)
    b = H.levels[0].A @ xt
    ro = OA.solve(H, b, rtol=1e-8, maxit=200)
    x = empty(A.n)
    inf = hec.amg_solve(G, dev(b), x, maxit=200, rtol=1e-8)
    xg = host(x)
    rr = np.linalg.norm(b - H.levels[0].A @ xg) / np.linalg.norm(b)
    print(f"{name}: levels {len(H.levels)} cycles gpu {inf['iterations']} oracle {ro.iterations} res {rr:.2e}")
    assert inf["status"] == hec.OK and ro.converged
    assert rr <= 1e-8 and abs(inf["rel_res_true"] - rr) <= 1e-10
    assert abs(inf["iterations"] - ro.iterations) <= 1
    assert np.linalg.norm(xg - ro.x) <= 1e-6 * np.linalg.norm(ro.x)


@pytest.mark.parametrize("nu", [(3, 3), (0, 2), (1, 0)])
def test_one_cycle_matches_oracle_closely(nu):
    """One V-cycle from x = 0 against the oracle's, also without pre-smoothing (the
    coarse iterates are zeroed) and with a single one (the first sweep from zero)."""
    A = synth.poisson3d(16)
    H = OA.hierarchy(A, nu1=nu[0], nu2=nu[1])
    G = hec.amg_setup(A, nu1=nu[0], nu2=nu[1])
    b = np.random.default_rng(6).uniform(-1, 1, A.n)
    x = empty(A.n)
    inf = hec.amg_solve(G, dev(b), x, maxit=1, rtol=0.0, check=False)
    assert inf["status"] == hec.NOT_CONVERGED and inf["iterations"] == 1
    xo = OA.vcycle(H, b, np.zeros(A.n))
    assert np.linalg.norm(host(x) - xo) <= 1e-12 * np.linalg.norm(xo)


CHEB_CASES = ["poisson2d_40", "poisson3d_20", "tpfa3d_17x13x11", "aniso3d_14", "poisson2d_40_positive"]


@pytest.mark.parametrize("name", CHEB_CASES)
@pytest.mark.parametrize("lower", [0.3, 0.05])
def test_chebyshev_solve_matches_oracle(name, lower):
    mk, opt = CASES[name]
    A = mk()
    opt = dict(opt, smoother="chebyshev", cheb_lower=lower)
    H = OA.hierarchy(A, **opt)
    G = hec.amg_setup(A, **opt)
    xt = np.random.default_rng(5).uniform(-1, 1, A.n)
    b = H.levels[0].A @ xt
    ro = OA.solve(H, b, rtol=1e-8, maxit=200)
    x = empty(A.n)
    inf = hec.amg_solve(G, dev(b), x, maxit=200, rtol=1e-8)
    xg = host(x)
    rr = np.linalg.norm(b - H.levels[0].A @ xg) / np.linalg.norm(b)
    print(f"{name} chebyshev [{lower}, 1]: cycles gpu {inf['iterations']} oracle {ro.iterations} res {rr:.2e}")
    assert inf["status"] == hec.OK and ro.converged
    assert rr <= 1e-8 and abs(inf["iterations"] - ro.iterations) <= 1
    assert np.linalg.norm(xg - ro.x) <= 1e-6 * np.linalg.norm(ro.x)


@pytest.mark.parametrize("nu", [(3, 3), (0, 2), (1, 0), (2, 5)])
def test_chebyshev_one_cycle_matches_oracle_closely(nu):
    """One V-cycle with Chebyshev smoothing from x = 0 against the oracle's: every level's
    sweeps, from a zero iterate below level 0, and degree 1 (a single weighted step)."""
    A = synth.lognormal_tpfa((18, 16, 14), 2.0, np.random.default_rng(11))
    H = OA.hierarchy(A, nu1=nu[0], nu2=nu[1], smoother="chebyshev")
    G = hec.amg_setup(A, nu1=nu[0], nu2=nu[1], smoother="chebyshev")
    b = np.random.default_rng(6).uniform(-1, 1, A.n)
    x = empty(A.n)
    inf = hec.amg_solve(G, dev(b), x, maxit=1, rtol=0.0, check=False)
    assert inf["status"] == hec.NOT_CONVERGED and inf["iterations"] == 1
    xo = OA.vcycle(H, b, np.zeros(A.n))
    assert np.linalg.norm(host(x) - xo) <= 1e-12 * np.linalg.norm(xo)


@pytest.mark.parametrize("smoother", ["jacobi", "chebyshev"])
@pytest.mark.parametrize("nu", [(3, 3), (2, 1), (0, 2)])
def test_graph_replays_equal_eager_cycles(nu, smoother):
    """The recorded cycle, replayed many times with other device work and
    synchronisations in between, gives bit for bit what launching every cycle gives."""
    import torch
    A = synth.lognormal_tpfa((23, 19, 17), 2.0, np.random.default_rng(8))
    Gg = hec.amg_setup(A, nu1=nu[0], nu2=nu[1], use_graph=True, smoother=smoother)
    Ge = hec.amg_setup(A, nu1=nu[0], nu2=nu[1], use_graph=False, smoother=smoother)
    for rep in range(4):
        b = np.random.default_rng(20 + rep).uniform(-1, 1, A.n)
        xe, xg = empty(A.n), empty(A.n)
        ie = hec.amg_solve(Ge, dev(b), xe, maxit=3 + rep, rtol=0.0, check=False)
        junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
        junk.mul_(3.0).sum().item()
        ig = hec.amg_solve(Gg, dev(b), xg, maxit=3 + rep, rtol=0.0, check=False)
        torch.cuda.synchronize()
        assert ie["iterations"] == ig["iterations"] == 3 + rep
        assert np.array_equal(host(xe).view(np.uint64), host(xg).view(np.uint64)), rep
        assert ie["rel_res_true"] == ig["rel_res_true"]


def test_edge_cases():
    # a diagonal matrix: no strong connection, one level, solved exactly by its inverse
    d = np.arange(1.0, 301.0)
    D = from_dense(np.diag(d))
    G = hec.amg_setup(D)
    assert hec.amg_info(G)["levels"] == 1
    x = empty(300)
    inf = hec.amg_solve(G, dev(np.ones(300)), x)
    assert inf["iterations"] == 1 and np.allclose(host(x), 1.0 / d, rtol=1e-14, atol=0)
    # at most coarse_size rows: one level, direct
    A = synth.poisson2d(7)
    G = hec.amg_setup(A, coarse_size=64)
    assert hec.amg_info(G)["levels"] == 1
    b = np.random.default_rng(7).uniform(-1, 1, A.n)
    x = empty(A.n)
    assert hec.amg_solve(G, dev(b), x)["iterations"] == 1
    # zero right-hand side: x = 0 at once
    A = synth.poisson2d(30)
    G = hec.amg_setup(A)
    x = dev(np.full(A.n, 7.0))
    inf = hec.amg_solve(G, dev(np.zeros(A.n)), x)
    assert inf["iterations"] == 0 and not host(x).any()
    # bad options and a zero diagonal
    for kw in ({"theta": 0.0}, {"max_levels": 0}, {"omega": 2.0}, {"nu1": -1}, {"coarse_size": 0},
               {"smoother": "chebyshev", "cheb_lower": 0.0}, {"smoother": "chebyshev", "cheb_lower": 1.0}):
        kw = dict(kw)
        with pytest.raises(hec.HecError) as e:
            hec.amg_setup(A, **kw)
        assert e.value.code == hec.INVALID_ARG
    Z = np.diag(np.ones(5))
    Z[2, 2] = 0.0
    Z[2, 3] = Z[3, 2] = -1.0
    with pytest.raises(hec.HecError) as e:
        hec.amg_setup(from_dense(Z))
    assert e.value.code == hec.ZERO_PIVOT
