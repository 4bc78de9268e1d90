"""FP64 CPU oracle (test infrastructure only).

A thin ctypes wrapper over ``liboracle.so`` (built from ``oracle.c`` with
``gcc -O3 -ffp-contract=off``). Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product path never
does. It shares no code with the GPU library.

Functions, each following the passage cited in ``oracle.c``:

* :func:`csr_spmv`        -- Alg. 1 / Eq. (2); :func:`csr_spmv_omp` the same on several
  threads (the benchmark's all-cores CPU figure)
* :func:`hec_from_csr`    -- Sec. 2.1 HEC layout (ELL slab + CSR remainder)
* :func:`iluk`            -- Sec. 2.4, Eq. (9)-(10), Alg. 2 (ILU(k), in place)
* :func:`level_schedule`  -- Sec. 2.6, Eq. (11), Alg. 3
* :func:`trsv_lower`, :func:`trsv_upper` -- Sec. 2.6 substitution
* :func:`gmres`           -- Sec. 2.7 restarted right-preconditioned GMRES(m)
* :func:`bicgstab`        -- Sec. 2.7, Alg. 4
* :func:`cg`              -- Sec. 2.7 preconditioned conjugate gradient
* :func:`ras_blocks`, :func:`ras_factor`, :func:`ras_apply` -- Sec. 2.5 restricted
  additive Schwarz (sequence partition, overlap layers, per-block ILU(k), restricted
  solve), written out block by block from the definition
* :func:`hyb_width`, :func:`hyb_from_csr` -- Sec. 2.1 HYB layout (ELL + COO)
* ``oracle.amg`` -- Sec. 2.8, Alg. 5: Ruge-Stueben setup and the V-cycle (plain numpy)
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "oracle.c")

OK, INVALID, NOMEM, ZERO_PIVOT, BREAKDOWN, NOT_CONVERGED = range(6)


def build_command(out: str = LIB_PATH):
    return ["gcc", "-O3", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC", "-fopenmp",
            "-shared", "-o", out, SRC_PATH, "-lm"]


def build() -> str:
    import subprocess
    subprocess.run(build_command(), check=True)
    return LIB_PATH


_lib = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = C.POINTER(C.c_int)
_dp = C.POINTER(C.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        L.orc_csr_spmv.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_double, _f64p, C.c_double, _f64p]
        L.orc_csr_spmv.restype = None
        L.orc_csr_spmv_omp.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_double, _f64p, C.c_double, _f64p,
                                       C.c_int]
        L.orc_csr_spmv_omp.restype = None
        L.orc_hec_sizes.argtypes = [C.c_int, _i32p, C.c_int, _ip, _ip, C.POINTER(C.c_long)]
        L.orc_hec_fill.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_int, C.c_int,
                                   _i32p, _f64p, _i32p, _i32p, _f64p]
        L.orc_iluk.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_int,
                               C.POINTER(_ip), C.POINTER(_ip), C.POINTER(_dp), C.POINTER(_ip)]
        L.orc_iluk.restype = C.c_int
        L.orc_free.argtypes = [C.c_void_p]
        L.orc_level_schedule.argtypes = [C.c_int, _i32p, _i32p, C.c_int, _i32p, _i32p, _i32p]
        L.orc_level_schedule.restype = C.c_int
        L.orc_trsv_lower.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, _f64p]
        L.orc_trsv_upper.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, _f64p]
        L.orc_gmres.argtypes = [C.c_int, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p, _f64p, _f64p,
                                C.c_int, C.c_int, C.c_double, _ip, _dp, C.c_void_p, C.c_void_p, _ip]
        L.orc_gmres.restype = C.c_int
        L.orc_bicgstab.argtypes = [C.c_int, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p, _f64p, _f64p,
                                   C.c_int, C.c_double, _ip, _dp, _ip]
        L.orc_bicgstab.restype = C.c_int
        L.orc_cg.argtypes = L.orc_bicgstab.argtypes[:-1]
        L.orc_cg.restype = C.c_int
        _lib = L
    return _lib


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def csr_spmv(n, Ap, Aj, Ax, x, alpha=1.0, beta=0.0, y=None):
    """y = alpha*A*x + beta*y (Alg. 1 / Eq. (2)). Returns y (a new array if y is None)."""
    y = np.zeros(n) if y is None else _f64(y).copy()
    lib().orc_csr_spmv(n, _i32(Ap), _i32(Aj), _f64(Ax), alpha, _f64(x), beta, y)
    return y


def csr_spmv_omp(n, Ap, Aj, Ax, x, nthreads, alpha=1.0, beta=0.0, y=None):
    """csr_spmv with the rows shared among nthreads OpenMP threads (same result bit for bit)."""
    y = np.zeros(n) if y is None else _f64(y).copy()
    lib().orc_csr_spmv_omp(n, _i32(Ap), _i32(Aj), _f64(Ax), alpha, _f64(x), beta, y, int(nthreads))
    return y


@dataclass
class HEC:
    n: int
    K: int
    ld: int
    ell_col: np.ndarray
    ell_val: np.ndarray
    rem_ptr: np.ndarray
    rem_col: np.ndarray
    rem_val: np.ndarray


def hec_from_csr(n, Ap, Aj, Ax, ell_width=-1) -> HEC:
    """HEC arrays of Sec. 2.1 (column-major ELL slab, CSR remainder)."""
    L = lib()
    K = C.c_int()
    ld = C.c_int()
    nr = C.c_long()
    Ap = _i32(Ap)
    L.orc_hec_sizes(n, Ap, ell_width, C.byref(K), C.byref(ld), C.byref(nr))
    K, ld, nr = K.value, ld.value, nr.value
    ell_col = np.empty(max(K * ld, 1), np.int32)
    ell_val = np.empty(max(K * ld, 1), np.float64)
    rem_ptr = np.empty(n + 1, np.int32)
    rem_col = np.empty(max(nr, 1), np.int32)
    rem_val = np.empty(max(nr, 1), np.float64)
    L.orc_hec_fill(n, Ap, _i32(Aj), _f64(Ax), K, ld, ell_col, ell_val, rem_ptr, rem_col, rem_val)
    return HEC(n, K, ld, ell_col[:K * ld], ell_val[:K * ld], rem_ptr, rem_col[:nr], rem_val[:nr])


def hyb_width(n, Ap):
    """ELL width of the HYB format (Sec. 2.1's ELL + COO, after Bell and Garland):
    the largest K such that at least max(4096, n // 3) rows hold K or more entries,
    0 when no K qualifies. A plain count over the row lengths."""
    lens = np.diff(np.asarray(Ap, np.int64))
    need = max(4096, n // 3)
    K = 0
    for k in range(1, int(lens.max(initial=0)) + 1):
        if int((lens >= k).sum()) >= need:
            K = k
    return K


@dataclass
class HYB:
    """HYB form (Sec. 2.1): the ELL part of width K as in HEC, the rest as COO
    (row, column, value) triplets in row order."""
    ell: HEC
    coo_row: np.ndarray
    coo_col: np.ndarray
    coo_val: np.ndarray


def hyb_from_csr(n, Ap, Aj, Ax, ell_width=None) -> HYB:
    """HYB arrays: the ELL part of hec_from_csr with the HYB width (or ell_width),
    and the remaining entries of every row as COO triplets, rows ascending, each
    row's entries in column order."""
    K = hyb_width(n, Ap) if ell_width is None else ell_width
    H = hec_from_csr(n, Ap, Aj, Ax, K)
    rows = np.repeat(np.arange(n, dtype=np.int32), np.diff(H.rem_ptr))
    return HYB(H, rows, H.rem_col.copy(), H.rem_val.copy())


@dataclass
class Factor:
    """In-place ILU(k) factor: L strict lower (unit diagonal implied), U upper with diagonal."""
    n: int
    LUp: np.ndarray
    LUj: np.ndarray
    LUx: np.ndarray
    LUlev: np.ndarray


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


def iluk(n, Ap, Aj, Ax, k) -> Factor:
    """ILU(k) of Alg. 2 / Eq. (9)-(10)."""
    L = lib()
    pp, pj, plev = _ip(), _ip(), _ip()
    px = _dp()
    st = L.orc_iluk(n, _i32(Ap), _i32(Aj), _f64(Ax), k, C.byref(pp), C.byref(pj), C.byref(px), C.byref(plev))
    if st != OK:
        raise OracleError(st, "iluk")
    LUp = np.ctypeslib.as_array(pp, shape=(n + 1,)).copy()
    nnz = int(LUp[-1])
    if nnz:
        LUj = np.ctypeslib.as_array(pj, shape=(nnz,)).copy()
        LUx = np.ctypeslib.as_array(px, shape=(nnz,)).copy()
        LUlev = np.ctypeslib.as_array(plev, shape=(nnz,)).copy()
    else:
        LUj = np.empty(0, np.int32); LUx = np.empty(0); LUlev = np.empty(0, np.int32)
    for p in (pp, pj, px, plev):
        L.orc_free(C.cast(p, C.c_void_p))
    return Factor(n, LUp, LUj, LUx, LUlev)


@dataclass
class Levels:
    nlev: int
    lev: np.ndarray
    level_ptr: np.ndarray
    perm: np.ndarray


def level_schedule(n, Lp, Lj, which: str) -> Levels:
    """Eq. (11) levels of the 'lower' or 'upper' triangle of a CSR pattern, plus Alg. 3's grouping."""
    w = {"lower": 0, "upper": 1}[which]
    lev = np.zeros(max(n, 1), np.int32)
    lptr = np.zeros(n + 1, np.int32)
    perm = np.zeros(max(n, 1), np.int32)
    nlev = lib().orc_level_schedule(n, _i32(Lp), _i32(Lj), w, lev, lptr, perm)
    return Levels(nlev, lev[:n], lptr[:nlev + 1], perm[:n])


def trsv_lower(F: Factor, b):
    y = np.zeros(F.n)
    lib().orc_trsv_lower(F.n, F.LUp, F.LUj, F.LUx, _f64(b), y)
    return y


def trsv_upper(F: Factor, y):
    x = np.zeros(F.n)
    lib().orc_trsv_upper(F.n, F.LUp, F.LUj, F.LUx, _f64(y), x)
    return x


@dataclass
class SolveResult:
    status: int
    x: np.ndarray
    iterations: int
    rel_res: float
    restarts: int = 0
    # GMRES with arnoldi=True: the last cycle's basis V ((steps+1) x n, or steps x n when
    # the cycle stopped on convergence) and its Hessenberg matrix before the rotations
    # ((restart+1) x restart)
    V: np.ndarray = None
    Hbar: np.ndarray = None
    steps: int = 0


def gmres(A, F: Factor, b, x0=None, restart=30, maxit=10000, rtol=1e-8, arnoldi=False) -> SolveResult:
    """Restarted right-preconditioned GMRES(m) with MGS (Sec. 2.7). A has .n/.Ap/.Aj/.Ax."""
    x = np.zeros(A.n) if x0 is None else _f64(x0).copy()
    it = C.c_int()
    rr = C.c_double()
    steps = C.c_int(0)
    V = np.zeros((restart + 1, A.n)) if arnoldi else None
    H = np.zeros((restart + 1, restart)) if arnoldi else None
    st = lib().orc_gmres(A.n, _i32(A.Ap), _i32(A.Aj), _f64(A.Ax), F.LUp, F.LUj, F.LUx, _f64(b), x,
                         restart, maxit, rtol, C.byref(it), C.byref(rr),
                         V.ctypes.data if arnoldi else None, H.ctypes.data if arnoldi else None,
                         C.byref(steps))
    return SolveResult(st, x, it.value, rr.value, 0, V, H, steps.value)


def bicgstab(A, F: Factor, b, x0=None, maxit=10000, rtol=1e-8) -> SolveResult:
    """Preconditioned BiCGSTAB, Alg. 4."""
    x = np.zeros(A.n) if x0 is None else _f64(x0).copy()
    it = C.c_int()
    rr = C.c_double()
    rs = C.c_int()
    st = lib().orc_bicgstab(A.n, _i32(A.Ap), _i32(A.Aj), _f64(A.Ax), F.LUp, F.LUj, F.LUx, _f64(b), x,
                            maxit, rtol, C.byref(it), C.byref(rr), C.byref(rs))
    return SolveResult(st, x, it.value, rr.value, rs.value)


def cg(A, F: Factor, b, x0=None, maxit=10000, rtol=1e-8) -> SolveResult:
    """Preconditioned conjugate gradient (Sec. 2.7), M = LU symmetric positive definite."""
    x = np.zeros(A.n) if x0 is None else _f64(x0).copy()
    it = C.c_int()
    rr = C.c_double()
    st = lib().orc_cg(A.n, _i32(A.Ap), _i32(A.Aj), _f64(A.Ax), F.LUp, F.LUj, F.LUx, _f64(b), x,
                      maxit, rtol, C.byref(it), C.byref(rr))
    return SolveResult(st, x, it.value, rr.value)


# ---------------------------------------------------------------- Sec. 2.5: restricted additive Schwarz

@dataclass
class RasBlock:
    rows: np.ndarray      # the system rows the block owns (a contiguous range)
    ext: np.ndarray       # the extended block, ascending system rows
    factor: Factor        # ILU(k) of A restricted to ext x ext


def ras_blocks(n, Ap, Aj, nblocks, overlap):
    """Sec. 2.5: sequence partition into nblocks contiguous blocks of ceil(n/nblocks)
    rows, each extended by `overlap` layers of neighbours (rows reached through the
    stored entries of the rows added by the previous layer). Returns [(own, ext)]."""
    R = -(-n // nblocks)
    out = []
    for s0 in range(0, n, R):
        own = np.arange(s0, min(n, s0 + R))
        ext = set(own.tolist())
        frontier = list(own)
        for _ in range(overlap):
            nxt = []
            for i in frontier:
                for e in range(Ap[i], Ap[i + 1]):
                    j = int(Aj[e])
                    if j not in ext:
                        ext.add(j)
                        nxt.append(j)
            frontier = nxt
        out.append((own, np.array(sorted(ext), dtype=np.int64)))
    return out


def _submatrix(A, ext):
    """CSR of A restricted to rows and columns `ext` (ascending), local numbering."""
    loc = {int(j): t for t, j in enumerate(ext)}
    Ap, Aj, Ax = [0], [], []
    for i in ext:
        for e in range(A.Ap[i], A.Ap[i + 1]):
            j = int(A.Aj[e])
            if j in loc:
                Aj.append(loc[j])
                Ax.append(A.Ax[e])
        Ap.append(len(Aj))
    return len(ext), np.array(Ap, np.int32), np.array(Aj, np.int32), np.array(Ax, np.float64)


def ras_factor(A, nblocks, overlap, k=0):
    """Sec. 2.5 + Sec. 2.4: ILU(k) of each extended diagonal block of A (entries of A
    outside the extended blocks dropped)."""
    blocks = []
    for own, ext in ras_blocks(A.n, A.Ap, A.Aj, nblocks, overlap):
        nb, bp, bj, bx = _submatrix(A, ext)
        blocks.append(RasBlock(own, ext, iluk(nb, bp, bj, bx, k)))
    return blocks


def ras_apply(blocks, r):
    """The restricted additive Schwarz preconditioner solve: every block solves its
    own ILU system on r restricted to its extended rows (Eq. (7)-(8)), and keeps only
    the rows it owns."""
    r = _f64(r)
    z = np.zeros(r.size)
    for B in blocks:
        zb = trsv_upper(B.factor, trsv_lower(B.factor, r[B.ext]))
        keep = np.searchsorted(B.ext, B.rows)
        z[B.rows] = zb[keep]
    return z
