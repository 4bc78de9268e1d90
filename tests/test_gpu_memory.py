"""Device memory at the boundary: every buffer the library allocates goes through the hooks
of hec_set_allocator (here counting wrappers around torch's caching allocator), the
footprint the library reports for a system equals what the hooks handed out for it, all of
it comes back when the handles are destroyed, and results do not depend on the allocator.
Vectors too short for the system are refused by the binding before any library call."""
import numpy as np
import pytest

import oracle as O
from paper_1606_00545_amd import hec, synth
from tests._gpu import dev, empty, host

pytestmark = pytest.mark.gpu


class Counting:
    def __init__(self):
        self.live = {}
        self.calls = 0

    def alloc(self, nbytes, stream):
        p = hec._torch_alloc(nbytes, stream)
        self.live[p] = nbytes
        self.calls += 1
        return p

    def free(self, ptr, nbytes, stream):
        assert self.live.pop(ptr) == nbytes
        hec._torch_free(ptr, nbytes, stream)

    @property
    def bytes(self):
        return sum(self.live.values())


@pytest.fixture
def counting():
    c = Counting()
    hec.set_allocator(c.alloc, c.free)
    yield c
    hec.use_torch_allocator()


def _system():
    A, xt = synth.workload_diffusion3d(20, sigma=2.0, seed=7)
    return A, O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, xt)


def test_footprint_equals_the_memory_handed_out(counting):
    A, b = _system()
    Mh = hec.hec_from_csr(A, keep_f32=True)
    F = hec.ilu_factor(A, k=1, keep_f32=True)
    lv = hec.level_schedule(F)
    assert counting.bytes == hec.footprint(Mh, F, lv) > 0
    x = empty(A.n)
    hec.gmres_solve(Mh, F, lv, dev(b), x, precision=1, rtol=1e-10)  # caches the solver workspace on Mh
    hec.bicgstab_solve(Mh, F, lv, dev(b), x)
    ws = counting.bytes
    assert ws == hec.footprint(Mh, F, lv)
    assert hec.footprint(Mh) + hec.footprint(None, F) + hec.footprint(None, None, lv) == ws
    for h in (Mh, F, lv):
        h.close()
    assert counting.bytes == 0 and not counting.live


def test_batch_and_amg_memory_comes_back(counting):
    A = synth.poisson2d(40)
    G = hec.amg_setup(A)
    assert counting.bytes > 0
    G.close()
    assert counting.bytes == 0
    B = hec.Batch(4, restart=30, max_n=2048)
    assert counting.bytes >= 4 * 63 * 2048 * 8
    B.close()
    assert counting.bytes == 0


def test_results_do_not_depend_on_the_allocator():
    A, b = _system()
    outs = []
    for mode in ("default", "torch"):
        if mode == "default":
            hec.set_allocator(None, None)  # hipMallocAsync / hipFreeAsync
        else:
            hec.use_torch_allocator()
        Mh = hec.hec_from_csr(A)
        F = hec.ilu_factor(A, k=0)
        lv = hec.level_schedule(F)
        x = empty(A.n)
        hec.gmres_solve(Mh, F, lv, dev(b), x)
        outs.append(host(x))
        for h in (Mh, F, lv):
            h.close()
    hec.use_torch_allocator()
    assert np.array_equal(outs[0].view(np.uint64), outs[1].view(np.uint64))


def test_short_or_misplaced_vectors_are_refused_before_the_call():
    import torch
    A, b = _system()
    Mh = hec.hec_from_csr(A)
    F = hec.ilu_factor(A, k=0)
    lv = hec.level_schedule(F)
    short = empty(A.n - 1)
    good = empty(A.n)
    with pytest.raises(ValueError):
        hec.hec_spmv(Mh, short, good)
    with pytest.raises(ValueError):
        hec.hec_spmv(Mh, good, short)
    with pytest.raises(ValueError):
        hec.trsv_levels(F, lv, short, good)
    with pytest.raises(ValueError):
        hec.gmres_solve(Mh, F, lv, dev(b), short)
    with pytest.raises(ValueError):
        hec.bicgstab_solve(Mh, F, lv, dev(b[:-1]), good)
    with pytest.raises(ValueError):
        hec.cg_solve(Mh, F, lv, torch.from_numpy(b), good)  # a host tensor
    with pytest.raises(ValueError):
        hec.gmres_solve(Mh, F, lv, dev(b).to(torch.float32), good)
