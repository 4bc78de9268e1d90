"""Batched small-system GMRES (one persistent launch, one workgroup per system,
replayed from a hipGraph) against the oracle, and its independence of the batch.

Parity is judged as for the single-system solver: FP64 true residual computed with
the oracle's SpMV, distance to the oracle's GMRES solution, iteration counts. A
system's result must be bit-identical alone, in any batch, with or without the
graph, and across graph replays with other work in between."""
import numpy as np
import pytest

import oracle as O
from paper_1606_00545_amd import hec, synth
from tests._gpu import dev, empty, host

pytestmark = pytest.mark.gpu


def _systems():
    """(name, A, k) small systems covering 2D/3D stencils, ILU(0)/ILU(1), a HEC
    remainder (rows longer than the ELL width) and a single row."""
    out = [
        ("poisson2d_8", synth.poisson2d(8), 0),
        ("poisson2d_64", synth.poisson2d(64), 0),
        ("tpfa2d_45x31", synth.lognormal_tpfa((45, 31), 2.0, np.random.default_rng(31)), 0),
        ("tpfa3d_12x11x10_k1", synth.lognormal_tpfa((12, 11, 10), 1.5, np.random.default_rng(32)), 1),
        ("tpfa3d_20_k0", synth.lognormal_tpfa((20, 20, 20), 2.0, np.random.default_rng(33)), 0),
        ("powerlaw_3000", synth.powerlaw_random(3000, np.random.default_rng(34), lmax=64), 0),
        ("tpfa2d_90x91", synth.lognormal_tpfa((90, 91), 1.0, np.random.default_rng(35)), 0),
        ("single", synth.CSR(1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([3.0])), 0),
    ]
    return out


@pytest.fixture(scope="module")
def prepared():
    items = []
    for i, (name, A, k) in enumerate(_systems()):
        xt = np.random.default_rng(100 + i).uniform(-1, 1, A.n)
        b = O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, xt)
        Mh = hec.hec_from_csr(A, keep_f32=True)
        F = hec.ilu_factor(A, k=k, keep_f32=True)
        lv = hec.level_schedule(F)
        items.append(dict(name=name, A=A, k=k, b=b, bd=dev(b), Mh=Mh, F=F, lv=lv))
    return items


def _solve(B, items, precision=0, rtol=1e-8, maxit=10000, check=True):
    xs = [empty(it["A"].n) for it in items]
    infos = hec.gmres_solve_batched(B, [(it["Mh"], it["F"], it["lv"], it["bd"], x) for it, x in zip(items, xs)],
                                    maxit=maxit, rtol=rtol, precision=precision, check=check)
    return [host(x) for x in xs], infos


def _rel_res(A, x, b):
    return np.linalg.norm(b - O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, x)) / np.linalg.norm(b)


def test_batch_fp64_matches_oracle(prepared):
    B = hec.Batch(len(prepared), restart=30, max_n=8192)
    xs, infos = _solve(B, prepared)
    for it, x, inf in zip(prepared, xs, infos):
        A, b = it["A"], it["b"]
        Fo = O.iluk(A.n, A.Ap, A.Aj, A.Ax, it["k"])
        ro = O.gmres(A, Fo, b, restart=30, rtol=1e-8)
        rr = _rel_res(A, x, b)
        dx = np.linalg.norm(x - ro.x) / np.linalg.norm(ro.x)
        print(f"{it['name']}: n={A.n} it gpu={inf['iterations']} oracle={ro.iterations} res={rr:.2e} dx={dx:.2e}")
        assert inf["status"] == hec.OK and rr <= 1e-8
        assert abs(inf["rel_res_true"] - rr) <= 1e-10
        assert abs(inf["iterations"] - ro.iterations) <= max(2, ro.iterations // 10)
        assert dx < 1e-4
    B.close()


def test_batch_independent_of_composition_and_graph(prepared):
    import torch
    full = hec.Batch(len(prepared), restart=30, max_n=8192, use_graph=True)
    eager = hec.Batch(len(prepared), restart=30, max_n=8192, use_graph=False)
    ref, _ = _solve(eager, prepared)
    # graph replays: the whole batch, reversed subsets, single systems, with other work between replays
    orders = [list(range(len(prepared))), list(range(len(prepared)))[::-1], [3, 1], [5], [0, 2, 4, 6, 7]]
    for rep, order in enumerate(orders):
        junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
        junk.mul_(2.0).sum().item()
        xs, infos = _solve(full, [prepared[i] for i in order])
        for i, x in zip(order, xs):
            assert np.array_equal(x.view(np.uint64), ref[i].view(np.uint64)), (rep, prepared[i]["name"])
        torch.cuda.synchronize()
    # alone, in a context sized for one system
    one = hec.Batch(1, restart=30, max_n=8192)
    for i in (1, 5):
        xs, _ = _solve(one, [prepared[i]])
        assert np.array_equal(xs[0].view(np.uint64), ref[i].view(np.uint64))
    for B in (full, eager, one):
        B.close()


def test_batch_mixed_precision_reaches_tolerance(prepared):
    B = hec.Batch(len(prepared), restart=30, max_n=8192)
    xs, infos = _solve(B, prepared, precision=1)
    for it, x, inf in zip(prepared, xs, infos):
        rr = _rel_res(it["A"], x, it["b"])
        print(f"mixed {it['name']}: it={inf['iterations']} ir={inf['ir_steps']} res={rr:.2e}")
        assert inf["status"] == hec.OK and rr <= 1e-8
        if it["A"].n > 1:
            assert inf["ir_steps"] >= 1
    B.close()


def test_batch_edge_cases(prepared):
    B = hec.Batch(4, restart=30, max_n=4096)
    it = prepared[1]  # 64 x 64 Poisson, n = 4096
    # zero right-hand side: x = 0 at once
    z = empty(it["A"].n)
    z.zero_()
    x = empty(it["A"].n)
    infos = hec.gmres_solve_batched(B, [(it["Mh"], it["F"], it["lv"], z, x)])
    assert infos[0]["status"] == hec.OK and infos[0]["iterations"] == 0 and not host(x).any()
    # maxit = 0: not converged, reported per system
    x = empty(it["A"].n)
    infos = hec.gmres_solve_batched(B, [(it["Mh"], it["F"], it["lv"], it["bd"], x)], maxit=0, check=False)
    assert infos[0]["status"] == hec.NOT_CONVERGED and infos[0]["iterations"] == 0
    # empty batch
    assert hec.gmres_solve_batched(B, []) == []
    # a system larger than max_n, a count above capacity, a restart other than the context's
    big = prepared[6]
    with pytest.raises(hec.HecError):
        hec.gmres_solve_batched(B, [(big["Mh"], big["F"], big["lv"], big["bd"], empty(big["A"].n))])
    with pytest.raises(hec.HecError):
        hec.gmres_solve_batched(B, [(it["Mh"], it["F"], it["lv"], it["bd"], empty(it["A"].n))] * 5)
    with pytest.raises(hec.HecError):
        hec.Batch(2, restart=33)
    with pytest.raises(hec.HecError):
        hec.Batch(2, max_n=hec.BATCH_MAX_N + 1)
    B.close()
