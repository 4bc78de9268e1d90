"""GPU serving: continuous batching over streams with memory admission, and the
batched persistent launch for small systems.

Every request's result must be the same alone and in a mix (bitwise: all
reductions have a fixed order that depends only on the request's own size),
admission must respect the memory budget, and every request must converge."""
import numpy as np
import pytest

import oracle as O
from paper_1606_00545_amd import serve, synth

pytestmark = pytest.mark.gpu


def _requests(precisions=(0,)):
    out = []
    specs = [(2, 40, 0.5), (3, 14, 2.0), (2, 90, 3.0), (3, 22, 1.0), (2, 61, 2.5), (3, 9, 0.7), (3, 30, 1.5)]
    rid = 0
    for prec in precisions:
        for dim, m, sig in specs:
            rng = np.random.default_rng(7000 + rid)
            A = synth.lognormal_tpfa((m,) * dim, sig, rng)
            xt = synth.uniform_vector(A.n, rng)
            b = O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, xt)
            out.append(serve.Request(rid, A, b, precision=prec, rtol=1e-8, arrival=0.0))
            rid += 1
    return out


def _rel_res(A, x, b):
    return np.linalg.norm(b - O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, x)) / np.linalg.norm(b)


def test_results_identical_alone_and_in_the_mix():
    reqs = _requests(precisions=(0, 1))
    alone = {}
    for r in reqs:  # one at a time, one slot
        res = serve.Server(slots=1).run([r])
        assert len(res) == 1
        alone[r.rid] = res[0].x
    srv = serve.Server(slots=6)
    mixed = {res.rid: res for res in srv.run(reqs)}
    assert not srv.errors and len(mixed) == len(reqs)
    assert srv.peak_inflight > 1  # the requests really overlapped
    for r in reqs:
        got = mixed[r.rid]
        assert got.info["status"] == 0
        assert np.array_equal(got.x.view(np.uint64), alone[r.rid].view(np.uint64)), r.rid
        assert _rel_res(r.A, got.x, r.b) <= 1e-8


@pytest.mark.parametrize("precision", [0, 1])
def test_admission_respects_the_memory_budget(precision):
    """Admission reserves the estimate; once the handles exist the reservation becomes the
    library-reported footprint (plus the workspace estimate). The estimate bounds what the
    library reports after the solve (workspace included), and the reported bytes in flight
    never exceed the budget."""
    reqs = _requests(precisions=(precision,))
    fps = [serve.footprint_bytes(r.A.n, r.A.nnz, precision=precision) for r in reqs]
    budget = max(fps) + min(fps)  # at most the largest and the smallest together
    srv = serve.Server(slots=6, mem_budget=budget)
    res = srv.run(reqs)
    assert not srv.errors and len(res) == len(reqs)
    assert srv.peak_mem <= budget and srv.peak_reported <= budget
    for r, fp in zip(reqs, fps):
        assert 0 < srv.reported[r.rid] <= fp, (r.rid, srv.reported[r.rid], fp)
        got = next(x for x in res if x.rid == r.rid)
        assert _rel_res(r.A, got.x, r.b) <= 1e-8


def test_arrivals_over_time_and_latency():
    reqs = _requests()
    for k, r in enumerate(reqs):
        r.arrival = 0.01 * k
    srv = serve.Server(slots=3)
    res = srv.run(reqs)
    assert len(res) == len(reqs)
    for x in res:
        assert x.admitted >= x.arrival - 1e-3 and x.done >= x.admitted and x.latency > 0
    st = serve.latency_stats(res)
    assert st["p99_ms"] >= st["p50_ms"] > 0


def test_batched_route_identical_alone_and_in_the_mix():
    """Small systems go to the batched launch; large ones keep their own streams."""
    reqs = _requests(precisions=(0, 1))
    small = [r for r in reqs if r.A.n <= 4096]
    assert 2 <= len(small) < len(reqs)
    alone = {}
    for r in reqs:
        srv = serve.Server(slots=1, batch_max_n=4096, batch_capacity=8)
        res = srv.run([r])
        assert len(res) == 1 and not srv.errors
        assert len(srv.batches) == (1 if r.A.n <= 4096 else 0)
        alone[r.rid] = res[0].x
    srv = serve.Server(slots=6, batch_max_n=4096, batch_capacity=8, batch_wait=0.5, batch_target=4)
    got = {res.rid: res for res in srv.run(reqs)}
    assert not srv.errors and len(got) == len(reqs)
    assert max(srv.batches) > 1  # several small systems shared a launch
    for r in reqs:
        g = got[r.rid]
        assert g.info["status"] == 0
        assert np.array_equal(g.x.view(np.uint64), alone[r.rid].view(np.uint64)), r.rid
        assert _rel_res(r.A, g.x, r.b) <= 1e-8
