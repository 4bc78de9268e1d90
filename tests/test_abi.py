"""The C-ABI library loads, exports every entry point of include/hec.h, and rejects
malformed input on the host before any device work (no GPU needed)."""
import os
import re

import numpy as np
import pytest

from paper_1606_00545_amd import hec, synth
from paper_1606_00545_amd.synth import CSR

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            src = re.sub(r"^\s*typedef[^;]*;", "", src, flags=re.M)  # function-pointer types
            names |= set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", src, flags=re.M))
    return names


def test_every_declared_symbol_is_exported():
    L = hec.load()
    declared = _declared()
    assert {"hec_from_csr", "hec_spmv", "ilu_factor", "level_schedule", "trsv_levels", "gmres_solve",
            "bicgstab_solve"} <= declared
    for name in declared:
        assert hasattr(L, name), name
    assert set(hec.EXPORTED) == declared


def _bad(A, **kw):
    return CSR(A.n, kw.get("Ap", A.Ap), kw.get("Aj", A.Aj), kw.get("Ax", A.Ax))


@pytest.mark.parametrize("entry", ["hec_from_csr", "ilu_factor"])
def test_malformed_csr_is_rejected_on_the_host(entry):
    A = synth.poisson2d(5)
    f = getattr(hec, entry)
    Aj = A.Aj.copy()
    Aj[1], Aj[2] = Aj[2], Aj[1]          # unsorted row
    Aj2 = A.Aj.copy()
    Aj2[1] = Aj2[0]                      # duplicate column
    Aj3 = A.Aj.copy()
    Aj3[-1] = A.n                        # out of range
    Ap = A.Ap.copy()
    Ap[3] = Ap[2] - 1                    # decreasing row pointer
    for bad in (_bad(A, Aj=Aj), _bad(A, Aj=Aj2), _bad(A, Aj=Aj3), _bad(A, Ap=Ap)):
        with pytest.raises(hec.HecError) as e:
            f(bad)
        assert e.value.code == hec.INVALID_ARG


def test_ilu_requires_a_stored_diagonal():
    Ap = np.array([0, 2, 3], np.int32)
    Aj = np.array([0, 1, 0], np.int32)   # row 1 has no diagonal
    Ax = np.array([1.0, 2.0, 3.0])
    with pytest.raises(hec.HecError) as e:
        hec.ilu_factor(CSR(2, Ap, Aj, Ax))
    assert e.value.code == hec.INVALID_ARG and "diagonal" in str(e.value)


def test_bad_arguments():
    A = synth.poisson2d(3)
    with pytest.raises(hec.HecError) as e:
        hec.ilu_factor(A, k=-1)
    assert e.value.code == hec.INVALID_ARG
    L = hec.load()
    assert L.hec_from_csr(-1, None, None, None, -1, 0, None, None) == hec.INVALID_ARG
    assert L.hec_spmv(None, 0, 1.0, None, 0, 0.0, None, 0, None) == hec.INVALID_ARG
    assert L.trsv_levels(None, None, 3, 0, None, None, None) == hec.INVALID_ARG
    assert L.gmres_solve(None, None, None, None, None, None, None, None) == hec.INVALID_ARG
    assert b"null" in L.hec_last_error()


def test_device_memory_only_through_the_allocator_hooks():
    """Every device allocation of the library goes through dev_alloc / dev_free (which call the
    hooks of hec_set_allocator, or hipMallocAsync / hipFreeAsync by default): no other call
    site allocates or frees device memory."""
    csrc = os.path.join(ROOT, "paper_1606_00545_amd", "csrc")
    calls = {}
    for fn in sorted(os.listdir(csrc)):
        src = open(os.path.join(csrc, fn)).read()
        src = re.sub(r"//[^\n]*", "", src)
        for api in ("hipMalloc", "hipMallocAsync", "hipMallocManaged", "hipExtMallocWithFlags", "hipMallocPitch",
                    "hipFree", "hipFreeAsync", "hipMallocFromPoolAsync"):
            k = len(re.findall(rf"\b{api}\s*\(", src))
            if k:
                calls[(fn, api)] = k
    assert calls == {("hec_matrix.hip", "hipMallocAsync"): 1, ("hec_matrix.hip", "hipFreeAsync"): 1}


def test_set_allocator_rejects_a_single_hook():
    L = hec.load()
    code = L.hec_set_allocator(hec._ALLOC_FN(lambda c, n, s: None), hec._FREE_FN(), None)
    assert code == hec.INVALID_ARG
    hec.set_allocator(None, None)  # the library default
    hec.use_torch_allocator()      # the binding's default


def test_trsv_kernel_switch_arguments():
    """hec_set_trsv_grid takes 0 or 1 only (host-side check, no device work)."""
    L = hec.load()
    assert L.hec_set_trsv_grid(2) == hec.INVALID_ARG
    assert L.hec_set_trsv_grid(-1) == hec.INVALID_ARG
    assert L.hec_set_trsv_grid(1) == hec.OK
    assert L.levels_grid(None, None) == hec.INVALID_ARG


def test_every_binding_declares_its_argument_types():
    """Handles are 64-bit pointers: an entry point bound without argument types would pass
    them through ctypes' default int conversion, truncated."""
    L = hec.load()
    for name in hec.EXPORTED:
        if name != "hec_last_error":
            assert getattr(L, name).argtypes is not None, name
