"""Python binding of the HEC / ILU(k) / level-schedule Krylov library (``libhec.so``).

Argument marshalling only: every call goes straight to the C ABI declared in
``include/hec.h``, with the same names. Host CSR arrays are numpy arrays;
vectors are torch CUDA tensors (device memory and streams come from PyTorch).
There is no fallback: if ``libhec.so`` is missing or cannot be loaded, every
call raises.
"""
from __future__ import annotations

import ctypes as C
import os
import sys
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhec.so")

OK, INVALID_ARG, NOMEM, ZERO_PIVOT, BREAKDOWN, NOT_CONVERGED, HIP_ERROR, TIMEOUT = range(8)
F64, F32 = 0, 1
KEEP_F32 = 1
COO_REMAINDER = 2   # hec_from_csr flag: remainder as COO (HYB = ELL + COO)
WIDTH_HYB = -2      # hec_from_csr ell_width: the HYB width rule
LOWER, UPPER, LU = 1, 2, 3

EXPORTED = ("hec_from_csr", "hec_info", "hec_export", "hec_spmv", "hec_destroy",
            "ilu_factor", "ilu_factor_ras", "ilu_info", "ilu_ras_export", "ilu_export", "ilu_destroy",
            "level_schedule", "levels_info", "levels_export", "levels_destroy",
            "trsv_levels", "gmres_solve", "bicgstab_solve", "cg_solve",
            "batch_create", "batch_destroy", "gmres_solve_batched",
            "amg_setup", "amg_info", "amg_export_level", "amg_solve", "amg_destroy",
            "hec_set_allocator", "hec_footprint", "gmres_solve_noalloc", "hec_set_spin_limit", "levels_check",
            "hec_set_trsv_grid", "levels_grid", "hec_last_error")
BATCH_MAX_N = 8192
NOALLOC_MAX_N = 16384


class HecError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: status {code}: {msg}")
        self.code = code


class SolveOpts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("maxit", C.c_int32), ("precision", C.c_int32),
                ("x0_zero", C.c_int32), ("rtol", C.c_double), ("ir_rtol", C.c_double),
                ("inner_rtol", C.c_double)]


class AmgOpts(C.Structure):
    _fields_ = [("theta", C.c_double), ("max_levels", C.c_int32), ("coarse_size", C.c_int32),
                ("omega", C.c_double), ("nu1", C.c_int32), ("nu2", C.c_int32), ("use_graph", C.c_int32),
                ("smoother", C.c_int32), ("cheb_lower", C.c_double)]


SMOOTHERS = {"jacobi": 0, "chebyshev": 1}


class SolveInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("restarts", C.c_int32),
                ("ir_steps", C.c_int32), ("rel_res_true", C.c_double), ("rel_res_est", C.c_double),
                ("seconds", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_vp = C.c_void_p
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)


def load(path: str = LIB_PATH):
    """Load libhec.so (raises OSError if it is missing: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"{path} not found: build it with `python -m paper_1606_00545_amd.build`")
    # One HIP runtime per process: torch ships its own libamdhip64.so.7. Loading
    # torch first makes the dynamic linker bind libhec.so to that same runtime
    # (same soname), so torch's device pointers and streams are valid here.
    import torch  # noqa: F401
    L = C.CDLL(path)
    L.hec_last_error.restype = C.c_char_p
    L.hec_from_csr.argtypes = [C.c_int32, _vp, _vp, _vp, C.c_int32, C.c_uint32, _vp, C.POINTER(_vp)]
    L.hec_info.argtypes = [_vp, _i32p, _i32p, _i32p, _i64p, _i64p]
    L.hec_export.argtypes = [_vp] + [_vp] * 7
    L.hec_spmv.argtypes = [_vp, C.c_int, C.c_double, _vp, C.c_int, C.c_double, _vp, C.c_int, _vp]
    L.hec_destroy.argtypes = [_vp]
    L.ilu_factor.argtypes = [C.c_int32, _vp, _vp, _vp, C.c_int32, C.c_uint32, _vp, C.POINTER(_vp)]
    L.ilu_factor_ras.argtypes = [C.c_int32, _vp, _vp, _vp, C.c_int32, C.c_int32, C.c_int32, C.c_uint32, _vp,
                                 C.POINTER(_vp)]
    L.ilu_info.argtypes = [_vp, _i32p, _i64p]
    L.ilu_ras_export.argtypes = [_vp, _i32p, _i32p, _vp, _vp, _vp]
    L.ilu_export.argtypes = [_vp, _vp, _vp, _vp]
    L.ilu_destroy.argtypes = [_vp]
    L.level_schedule.argtypes = [_vp, _vp, C.POINTER(_vp)]
    L.levels_info.argtypes = [_vp, _i32p, _i32p, _i32p]
    L.levels_export.argtypes = [_vp, _vp, _vp, _vp, _vp]
    L.levels_destroy.argtypes = [_vp]
    L.trsv_levels.argtypes = [_vp, _vp, C.c_uint32, C.c_int, _vp, _vp, _vp]
    L.gmres_solve.argtypes = [_vp, _vp, _vp, _vp, _vp, C.POINTER(SolveOpts), C.POINTER(SolveInfo), _vp]
    L.bicgstab_solve.argtypes = L.gmres_solve.argtypes
    L.cg_solve.argtypes = L.gmres_solve.argtypes
    L.gmres_solve_noalloc.argtypes = L.gmres_solve.argtypes
    L.batch_create.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.POINTER(_vp)]
    L.batch_destroy.argtypes = [_vp]
    L.gmres_solve_batched.argtypes = [_vp, C.c_int32, _vp, _vp, _vp, _vp, _vp, C.POINTER(SolveOpts),
                                      _vp, _vp]
    L.amg_setup.argtypes = [C.c_int32, _vp, _vp, _vp, C.POINTER(AmgOpts), _vp, C.POINTER(_vp)]
    L.amg_info.argtypes = [_vp, _i32p, _vp, _vp, _vp]
    L.amg_export_level.argtypes = [_vp, C.c_int32] + [_vp] * 7
    L.amg_solve.argtypes = [_vp, _vp, _vp, C.c_int32, C.c_double, _vp, C.POINTER(SolveInfo)]
    L.amg_destroy.argtypes = [_vp]
    L.hec_set_allocator.argtypes = [_ALLOC_FN, _FREE_FN, _vp]
    L.hec_footprint.argtypes = [_vp, _vp, _vp, _i64p]
    L.hec_set_spin_limit.argtypes = [C.c_int64]
    L.levels_check.argtypes = [_vp, _vp]
    L.hec_set_trsv_grid.argtypes = [C.c_int32]
    L.levels_grid.argtypes = [_vp, _i32p]
    for name in EXPORTED:
        if name != "hec_last_error":
            getattr(L, name).restype = C.c_int
    _lib = L
    use_torch_allocator()
    return L


# ---------------------------------------------------------------- device memory

_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
_hooks = None  # the ctypes callbacks in force (kept alive while the library may call them)


def set_allocator(alloc=None, free=None):
    """hec_set_allocator: `alloc(nbytes, stream) -> int` (0 on failure) and `free(ptr, nbytes,
    stream)` serve every device buffer the library allocates from now on; None, None restores
    the library's default (hipMallocAsync / hipFreeAsync)."""
    global _hooks
    L = load()
    if alloc is None and free is None:
        _check(L.hec_set_allocator(_ALLOC_FN(), _FREE_FN(), None), "hec_set_allocator")
        _hooks = None
        return

    def _a(ctx, nbytes, stream):
        try:
            return alloc(int(nbytes), int(stream or 0)) or None
        except Exception as e:  # the library reports NOMEM; the reason is kept for the message
            _alloc_errors.append(f"{type(e).__name__}: {e}")
            del _alloc_errors[:-4]
            return None

    def _f(ctx, ptr, nbytes, stream):
        free(int(ptr), int(nbytes), int(stream or 0))

    hooks = (_ALLOC_FN(_a), _FREE_FN(_f))
    _check(L.hec_set_allocator(hooks[0], hooks[1], None), "hec_set_allocator")
    _hooks = hooks  # buffers made by earlier hooks keep their own (module-level references below)
    _all_hooks.append(hooks)


_all_hooks = []  # every callback pair ever set: buffers are freed by the hooks that made them
_alloc_errors = []  # the last exceptions raised by an allocation hook


def _torch_hooks():
    """alloc / free through torch's caching allocator. The torch functions are bound
    here, not looked up per call: handles released while the interpreter shuts down
    (when imports no longer work) still reach them; once shutdown has begun a free is
    skipped, since the process's memory goes with it."""
    import torch
    alloc = torch.cuda.caching_allocator_alloc
    delete = torch.cuda.caching_allocator_delete
    finalizing = sys.is_finalizing

    def _alloc(nbytes, stream):
        return alloc(nbytes, stream=stream)

    def _free(ptr, nbytes, stream):
        if not finalizing():
            delete(ptr)

    return _alloc, _free


def _torch_alloc(nbytes, stream):
    return _torch_hooks()[0](nbytes, stream)


def _torch_free(ptr, nbytes, stream):
    _torch_hooks()[1](ptr, nbytes, stream)


def use_torch_allocator():
    """Route the library's device memory through torch's caching allocator."""
    set_allocator(*_torch_hooks())


def set_spin_limit(polls: int = -1):
    """hec_set_spin_limit: polls a device-side wait of the triangular solves makes before
    it gives up (negative: the default)."""
    _check(load().hec_set_spin_limit(int(polls)), "hec_set_spin_limit")


def set_trsv_grid(enable: bool = True):
    """hec_set_trsv_grid: schedules built after the call get wavefront plans where they
    apply (True, the default) or level-blocked plans only (False)."""
    _check(load().hec_set_trsv_grid(1 if enable else 0), "hec_set_trsv_grid")


def levels_grid(lv) -> bool:
    """levels_grid: whether lv carries wavefront plans for its triangles."""
    g = C.c_int32()
    _check(load().levels_grid(lv.ptr, C.byref(g)), "levels_grid")
    return bool(g.value)


def levels_check(lv, stream=None):
    """levels_check: synchronises the stream; raises HecError(TIMEOUT) if a wait of lv's
    triangular solves gave up since the last check."""
    _check(load().levels_check(lv.ptr, _stream(stream)), "levels_check")


def footprint(A=None, M=None, lv=None) -> int:
    """hec_footprint: device bytes held by a matrix (its solver workspace included), a
    factor and a schedule."""
    out = C.c_int64()
    _check(load().hec_footprint(A.ptr if A else None, M.ptr if M else None, lv.ptr if lv else None,
                                C.byref(out)), "hec_footprint")
    return out.value


def _check(code: int, where: str):
    if code != OK:
        msg = load().hec_last_error().decode()
        if code == NOMEM and _alloc_errors:
            msg += f" (allocation hook: {_alloc_errors[-1]})"
            _alloc_errors.clear()
        raise HecError(code, where, msg)


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def _dev(t, n, dtype=None, what="vector"):
    """Device pointer of a contiguous torch tensor of at least n elements on the current
    device (checked here, before any library call: a short vector would make the
    kernels read and write past its end)."""
    import torch
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{what} must be a contiguous CUDA tensor")
    if t.device.index != torch.cuda.current_device():
        raise ValueError(f"{what} is on {t.device}, the current device is cuda:{torch.cuda.current_device()}")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{what}: expected {dtype}, got {t.dtype}")
    if t.numel() < n:
        raise ValueError(f"{what} has {t.numel()} elements, the system has {n} rows")
    return t.data_ptr()


def _dtype_code(t):
    import torch
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise ValueError(f"unsupported dtype {t.dtype}")


def _csr(A):
    n = int(A.n)
    Ap = np.ascontiguousarray(A.Ap, dtype=np.int32)
    Aj = np.ascontiguousarray(A.Aj, dtype=np.int32)
    Ax = np.ascontiguousarray(A.Ax, dtype=np.float64)
    return n, Ap, Aj, Ax


class _Handle:
    _destroy = None

    def __init__(self, ptr):
        self.ptr = ptr

    def close(self):
        if self.ptr:
            getattr(load(), self._destroy)(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Matrix(_Handle):
    _destroy = "hec_destroy"

    def __init__(self, ptr):
        super().__init__(ptr)
        n = C.c_int32()
        _check(load().hec_info(ptr, C.byref(n), None, None, None, None), "hec_info")
        self.n = n.value


class Factor(_Handle):
    _destroy = "ilu_destroy"

    def __init__(self, ptr):
        super().__init__(ptr)
        n_sys = C.c_int32()
        _check(load().ilu_ras_export(ptr, C.byref(n_sys), None, None, None, None), "ilu_ras_export")
        self.n = n_sys.value  # the system size (rows of the vectors it is applied to)


class Levels(_Handle):
    _destroy = "levels_destroy"

    def __init__(self, ptr):
        super().__init__(ptr)
        n = C.c_int32()
        _check(load().levels_info(ptr, C.byref(n), None, None), "levels_info")
        self.n = n.value


class Amg(_Handle):
    _destroy = "amg_destroy"

    def __init__(self, ptr):
        super().__init__(ptr)
        self.n = amg_info(self)["n"][0]


class Batch(_Handle):
    """Context of gmres_solve_batched: up to `capacity` systems of at most `max_n` rows."""
    _destroy = "batch_destroy"

    def __init__(self, capacity: int, restart: int = 30, max_n: int = BATCH_MAX_N, use_graph: bool = True):
        h = _vp()
        _check(load().batch_create(capacity, restart, max_n, int(use_graph), C.byref(h)), "batch_create")
        super().__init__(h.value)
        self.capacity, self.restart, self.max_n = capacity, restart, max_n


# ---------------------------------------------------------------- HEC matrix

def hec_from_csr(A, ell_width: int = -1, keep_f32: bool = False, coo: bool = False, stream=None) -> Matrix:
    """HEC (default), plain ELL (ell_width >= longest row), CSR (ell_width = 0) or HYB
    (coo=True, usually with ell_width=WIDTH_HYB) form of A on the device."""
    n, Ap, Aj, Ax = _csr(A)
    out = _vp()
    flags = (KEEP_F32 if keep_f32 else 0) | (COO_REMAINDER if coo else 0)
    _check(load().hec_from_csr(n, Ap.ctypes.data, Aj.ctypes.data, Ax.ctypes.data, ell_width,
                               flags, _stream_or_null(stream), C.byref(out)),
           "hec_from_csr")
    return Matrix(out.value)


def _stream_or_null(stream):
    """Setup calls accept a stream; None means the legacy default stream (no torch needed)."""
    if stream is None:
        return None
    return getattr(stream, "cuda_stream", stream)


def hec_info(M: Matrix) -> dict:
    n, K, ld = C.c_int32(), C.c_int32(), C.c_int32()
    nnz, nr = C.c_int64(), C.c_int64()
    _check(load().hec_info(M.ptr, C.byref(n), C.byref(K), C.byref(ld), C.byref(nnz), C.byref(nr)), "hec_info")
    return {"n": n.value, "K": K.value, "ld": ld.value, "nnz": nnz.value, "nnz_rem": nr.value}


def hec_export(M: Matrix, f32: bool = False) -> dict:
    d = hec_info(M)
    slab = d["K"] * d["ld"]
    out = {"ell_col": np.empty(slab, np.int32), "ell_val": np.empty(slab, np.float64),
           "rem_ptr": np.empty(d["n"] + 1, np.int32), "rem_col": np.empty(d["nnz_rem"], np.int32),
           "rem_val": np.empty(d["nnz_rem"], np.float64)}
    if f32:
        out["ell_val32"] = np.empty(slab, np.float32)
        out["rem_val32"] = np.empty(d["nnz_rem"], np.float32)
    p = lambda k: out[k].ctypes.data if k in out else None
    _check(load().hec_export(M.ptr, p("ell_col"), p("ell_val"), p("rem_ptr"), p("rem_col"), p("rem_val"),
                             p("ell_val32"), p("rem_val32")), "hec_export")
    out.update(d)
    return out


def hec_spmv(M: Matrix, x, y, alpha: float = 1.0, beta: float = 0.0, vals: int = F64, stream=None):
    """y = alpha*A*x + beta*y on the device (asynchronous on the stream)."""
    _check(load().hec_spmv(M.ptr, vals, alpha, _dev(x, M.n, what="x"), _dtype_code(x), beta,
                           _dev(y, M.n, what="y"), _dtype_code(y), _stream(stream)), "hec_spmv")
    return y


# ---------------------------------------------------------------- ILU(k) + levels

def ilu_factor(A, k: int = 0, keep_f32: bool = False, stream=None) -> Factor:
    n, Ap, Aj, Ax = _csr(A)
    out = _vp()
    _check(load().ilu_factor(n, Ap.ctypes.data, Aj.ctypes.data, Ax.ctypes.data, k, KEEP_F32 if keep_f32 else 0,
                             _stream_or_null(stream), C.byref(out)), "ilu_factor")
    return Factor(out.value)


def ilu_factor_ras(A, nblocks: int, overlap: int = 0, k: int = 0, keep_f32: bool = False, stream=None) -> Factor:
    """Restricted additive Schwarz ILU(k): nblocks contiguous blocks, `overlap` neighbour layers."""
    n, Ap, Aj, Ax = _csr(A)
    out = _vp()
    _check(load().ilu_factor_ras(n, Ap.ctypes.data, Aj.ctypes.data, Ax.ctypes.data, k, nblocks, overlap,
                                 KEEP_F32 if keep_f32 else 0, _stream_or_null(stream), C.byref(out)),
           "ilu_factor_ras")
    return Factor(out.value)


def ilu_ras_export(M: Factor) -> dict:
    nf = ilu_info(M)["n"]
    n_sys, nb = C.c_int32(), C.c_int32()
    _check(load().ilu_ras_export(M.ptr, C.byref(n_sys), C.byref(nb), None, None, None), "ilu_ras_export")
    bs = np.empty(nb.value + 1, np.int32)
    ext = np.empty(nf, np.int32)
    own = np.empty(n_sys.value, np.int32)
    _check(load().ilu_ras_export(M.ptr, None, None, bs.ctypes.data, ext.ctypes.data, own.ctypes.data),
           "ilu_ras_export")
    return {"n_sys": n_sys.value, "nblocks": nb.value, "block_start": bs, "ext_row": ext, "own": own}


def ilu_info(M: Factor) -> dict:
    n, nnz = C.c_int32(), C.c_int64()
    _check(load().ilu_info(M.ptr, C.byref(n), C.byref(nnz)), "ilu_info")
    return {"n": n.value, "nnz": nnz.value}


def ilu_export(M: Factor):
    d = ilu_info(M)
    LUp = np.empty(d["n"] + 1, np.int32)
    LUj = np.empty(d["nnz"], np.int32)
    LUx = np.empty(d["nnz"], np.float64)
    _check(load().ilu_export(M.ptr, LUp.ctypes.data, LUj.ctypes.data, LUx.ctypes.data), "ilu_export")
    return LUp, LUj, LUx


def level_schedule(M: Factor, stream=None) -> Levels:
    out = _vp()
    _check(load().level_schedule(M.ptr, _stream_or_null(stream), C.byref(out)), "level_schedule")
    return Levels(out.value)


def levels_info(lv: Levels) -> dict:
    n, a, b = C.c_int32(), C.c_int32(), C.c_int32()
    _check(load().levels_info(lv.ptr, C.byref(n), C.byref(a), C.byref(b)), "levels_info")
    return {"n": n.value, "nlev_lower": a.value, "nlev_upper": b.value}


def levels_export(lv: Levels) -> dict:
    d = levels_info(lv)
    out = {"lower_ptr": np.empty(d["nlev_lower"] + 1, np.int32), "lower_perm": np.empty(d["n"], np.int32),
           "upper_ptr": np.empty(d["nlev_upper"] + 1, np.int32), "upper_perm": np.empty(d["n"], np.int32)}
    _check(load().levels_export(lv.ptr, out["lower_ptr"].ctypes.data, out["lower_perm"].ctypes.data,
                                out["upper_ptr"].ctypes.data, out["upper_perm"].ctypes.data), "levels_export")
    out.update(d)
    return out


def trsv_levels(M: Factor, lv: Levels, b, x, which: int = LU, stream=None):
    """x = L^{-1} b, U^{-1} b or U^{-1} L^{-1} b on the device (asynchronous)."""
    prec = _dtype_code(b)
    if _dtype_code(x) != prec:
        raise ValueError("b and x must have the same dtype")
    _check(load().trsv_levels(M.ptr, lv.ptr, which, prec, _dev(b, lv.n, what="b"), _dev(x, lv.n, what="x"),
                              _stream(stream)), "trsv_levels")
    return x


# ---------------------------------------------------------------- solvers

def _opts(restart, maxit, rtol, precision, x0_zero, ir_rtol, inner_rtol):
    return SolveOpts(restart, maxit, precision, 1 if x0_zero else 0, rtol, ir_rtol, inner_rtol)


def gmres_solve(A: Matrix, M: Factor, lv: Levels, b, x, restart: int = 30, maxit: int = 10000,
                rtol: float = 1e-8, precision: int = 0, x0_zero: bool = True, ir_rtol: float = 0.0,
                inner_rtol: float = 1e-4, stream=None, check: bool = True) -> dict:
    import torch
    o = _opts(restart, maxit, rtol, precision, x0_zero, ir_rtol, inner_rtol)
    info = SolveInfo()
    code = load().gmres_solve(A.ptr, M.ptr, lv.ptr, _dev(b, A.n, torch.float64, "b"), _dev(x, A.n, torch.float64, "x"),
                              C.byref(o), C.byref(info), _stream(stream))
    if check and code != OK:
        _check(code, "gmres_solve")
    return info.as_dict()


def gmres_solve_noalloc(A: Matrix, M: Factor, lv: Levels, b, x, restart: int = 30, maxit: int = 10000,
                        rtol: float = 1e-8, x0_zero: bool = True, stream=None, check: bool = True) -> dict:
    """gmres_solve (FP64) with the library's static scratch as workspace: allocates nothing."""
    import torch
    o = _opts(restart, maxit, rtol, 0, x0_zero, 0.0, 0.0)
    info = SolveInfo()
    code = load().gmres_solve_noalloc(A.ptr, M.ptr, lv.ptr, _dev(b, A.n, torch.float64, "b"),
                                      _dev(x, A.n, torch.float64, "x"), C.byref(o), C.byref(info), _stream(stream))
    if check and code != OK:
        _check(code, "gmres_solve_noalloc")
    return info.as_dict()


def bicgstab_solve(A: Matrix, M: Factor, lv: Levels, b, x, maxit: int = 10000, rtol: float = 1e-8,
                   x0_zero: bool = True, stream=None, check: bool = True) -> dict:
    import torch
    o = _opts(1, maxit, rtol, 0, x0_zero, 0.0, 0.0)
    info = SolveInfo()
    code = load().bicgstab_solve(A.ptr, M.ptr, lv.ptr, _dev(b, A.n, torch.float64, "b"), _dev(x, A.n, torch.float64, "x"),
                                 C.byref(o), C.byref(info), _stream(stream))
    if check and code != OK:
        _check(code, "bicgstab_solve")
    return info.as_dict()


def cg_solve(A: Matrix, M: Factor, lv: Levels, b, x, maxit: int = 10000, rtol: float = 1e-8,
             x0_zero: bool = True, stream=None, check: bool = True) -> dict:
    import torch
    o = _opts(1, maxit, rtol, 0, x0_zero, 0.0, 0.0)
    info = SolveInfo()
    code = load().cg_solve(A.ptr, M.ptr, lv.ptr, _dev(b, A.n, torch.float64, "b"), _dev(x, A.n, torch.float64, "x"),
                           C.byref(o), C.byref(info), _stream(stream))
    if check and code != OK:
        _check(code, "cg_solve")
    return info.as_dict()


def gmres_solve_batched(B: Batch, systems, maxit: int = 10000, rtol: float = 1e-8, precision: int = 0,
                        x0_zero: bool = True, ir_rtol: float = 0.0, inner_rtol: float = 1e-4, stream=None,
                        check: bool = True) -> list:
    """GMRES(B.restart) on every (A, M, lv, b, x) of `systems` in one launch; returns one info dict each."""
    import torch
    count = len(systems)
    o = _opts(B.restart, maxit, rtol, precision, x0_zero, ir_rtol, inner_rtol)
    arr = lambda vals: (_vp * max(1, count))(*vals)
    A = arr([s[0].ptr for s in systems])
    M = arr([s[1].ptr for s in systems])
    lv = arr([s[2].ptr for s in systems])
    b = arr([_dev(s[3], s[0].n, torch.float64, "b") for s in systems])
    x = arr([_dev(s[4], s[0].n, torch.float64, "x") for s in systems])
    infos = (SolveInfo * max(1, count))()
    code = load().gmres_solve_batched(B.ptr, count, A, M, lv, b, x, C.byref(o), infos, _stream(stream))
    if check and code != OK:
        _check(code, "gmres_solve_batched")
    return [infos[i].as_dict() for i in range(count)]


# ------------------------------------------------------------------ AMG (Sec. 2.8)

def amg_setup(A, theta: float = 0.25, max_levels: int = 8, coarse_size: int = 64, omega: float = 2.0 / 3.0,
              nu1: int = 3, nu2: int = 3, use_graph: bool = True, smoother: str = "jacobi",
              cheb_lower: float = 0.3, stream=None) -> Amg:
    """smoother: "jacobi" (damped, weight omega) or "chebyshev" (polynomial of degree nu1 /
    nu2 in D^{-1} A on [cheb_lower * lmax, lmax])."""
    n, Ap, Aj, Ax = _csr(A)
    if smoother not in SMOOTHERS:
        raise ValueError(f"smoother must be one of {sorted(SMOOTHERS)}")
    o = AmgOpts(theta, max_levels, coarse_size, omega, nu1, nu2, 1 if use_graph else 0, SMOOTHERS[smoother],
                cheb_lower)
    out = _vp()
    _check(load().amg_setup(n, Ap.ctypes.data, Aj.ctypes.data, Ax.ctypes.data, C.byref(o),
                            _stream_or_null(stream), C.byref(out)), "amg_setup")
    return Amg(out.value)


def amg_info(H: Amg) -> dict:
    nl = C.c_int32()
    _check(load().amg_info(H.ptr, C.byref(nl), None, None, None), "amg_info")
    n = np.zeros(nl.value, np.int32)
    nnz = np.zeros(nl.value, np.int64)
    nnzp = np.zeros(nl.value, np.int64)
    _check(load().amg_info(H.ptr, C.byref(nl), n.ctypes.data, nnz.ctypes.data, nnzp.ctypes.data), "amg_info")
    return {"levels": nl.value, "n": n.tolist(), "nnz": nnz.tolist(), "nnz_p": nnzp.tolist()}


def amg_export_level(H: Amg, level: int) -> dict:
    d = amg_info(H)
    n, nnz, nnzp = d["n"][level], d["nnz"][level], d["nnz_p"][level]
    cf = np.zeros(n, np.int8)
    Ap, Aj, Ax = np.zeros(n + 1, np.int32), np.zeros(max(nnz, 1), np.int32), np.zeros(max(nnz, 1))
    coarsest = level == d["levels"] - 1
    Pp = np.zeros(n + 1, np.int32)
    Pj, Px = np.zeros(max(nnzp, 1), np.int32), np.zeros(max(nnzp, 1))
    _check(load().amg_export_level(H.ptr, level, None if coarsest else cf.ctypes.data, Ap.ctypes.data,
                                   Aj.ctypes.data, Ax.ctypes.data, None if coarsest else Pp.ctypes.data,
                                   Pj.ctypes.data, Px.ctypes.data), "amg_export_level")
    out = {"A": (Ap, Aj[:nnz], Ax[:nnz])}
    if not coarsest:
        out.update(cf=cf, P=(Pp, Pj[:nnzp], Px[:nnzp]))
    return out


def amg_solve(H: Amg, b, x, maxit: int = 100, rtol: float = 1e-8, stream=None, check: bool = True) -> dict:
    import torch
    info = SolveInfo()
    code = load().amg_solve(H.ptr, _dev(b, H.n, torch.float64, "b"), _dev(x, H.n, torch.float64, "x"), maxit, rtol,
                            _stream(stream),
                            C.byref(info))
    if check and code != OK:
        _check(code, "amg_solve")
    return info.as_dict()
