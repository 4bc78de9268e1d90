"""Helpers for the GPU tests: host <-> device copies through torch (plumbing only)."""
import numpy as np


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def empty(n, dtype="f64"):
    import torch
    return torch.empty(n, dtype=torch.float64 if dtype == "f64" else torch.float32, device="cuda")


def abs_product(A, x):
    """(|A| |x|) row by row, for componentwise error bounds."""
    import scipy.sparse as sp
    S = sp.csr_matrix((np.abs(A.Ax), A.Aj, A.Ap), shape=(A.n, A.n))
    return S @ np.abs(x)
