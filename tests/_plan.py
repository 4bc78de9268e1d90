"""ctypes access to the host build of the triangular-solve planner (libhecplan.so)."""
import ctypes as C
import os

import numpy as np

from paper_1606_00545_amd import build as hipbuild

META = ("n", "nlev", "K", "KC", "ldq", "nparts", "nss", "W", "S", "D64", "D32", "blocked",
        "lds64", "lds32", "kSub", "kPad", "NS")
ARRAYS = ("level_ptr", "perm", "lev", "part_ss", "part_pos", "ss_pos", "ss_need", "grow", "part_of", "pos",
          "chunks", "enc", "src", "psrc")
LDS_MAX = 160 * 1024 - 256  # what the GPU library passes on gfx950 (160 KiB per workgroup, less a margin)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(hipbuild.PLAN_LIB):
            hipbuild.build_plan()
        L = C.CDLL(hipbuild.PLAN_LIB)
        ip = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        L.hecplan_make.restype = C.c_void_p
        L.hecplan_make.argtypes = [C.c_int32, ip, ip, ip, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                   C.c_int32, C.c_int64, C.c_int32, C.c_void_p, C.c_int32, C.c_int32, C.c_int32]
        L.hecplan_meta.argtypes = [C.c_void_p, np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")]
        L.hecplan_array.restype = C.c_int64
        L.hecplan_array.argtypes = [C.c_void_p, C.c_char_p, C.c_void_p]
        L.hecplan_free.argtypes = [C.c_void_p]
        L.hecplan_detect_grid.argtypes = [C.c_int32, ip, ip, ip]
        L.hecplan_grid_make.restype = C.c_void_p
        L.hecplan_grid_make.argtypes = [C.c_int32, ip, ip, ip, C.c_int32, C.c_int32, C.c_int32, C.c_int32]
        L.hecplan_grid_meta.argtypes = [C.c_void_p, np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")]
        L.hecplan_grid_src.restype = C.c_int64
        L.hecplan_grid_src.argtypes = [C.c_void_p, C.c_void_p]
        L.hecplan_grid_free.argtypes = [C.c_void_p]
        _lib = L
    return _lib


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def detect_grid(A):
    out = np.zeros(3, np.int32)
    lib().hecplan_detect_grid(A.n, _i32(A.Ap), _i32(A.Aj), out)
    return tuple(int(v) for v in out)


def diag_positions(F):
    d = np.empty(F.n, np.int32)
    for i in range(F.n):
        row = F.LUj[F.LUp[i]:F.LUp[i + 1]]
        d[i] = F.LUp[i] + int(np.searchsorted(row, i))
        assert F.LUj[d[i]] == i
    return d


def make_plan(F, upper, grid=(0, 0, 0), has_f32=True, lds_max=LDS_MAX, flat=False, blocks=None, solvers=0,
              tile=0):
    """Plan of one triangle of the factor F (oracle Factor) as a dict of meta values and arrays
    (solvers: solver wavefronts per workgroup for wide levels, 0: the library's default;
    tile: grid tile side, 0: the planner's choice)."""
    L = lib()
    diag = diag_positions(F)
    bl = None if blocks is None else _i32(blocks)
    h = L.hecplan_make(F.n, _i32(F.LUp), _i32(F.LUj), diag, grid[0], grid[1], grid[2], int(upper),
                       int(has_f32), lds_max, int(flat), None if bl is None else bl.ctypes.data,
                       0 if bl is None else bl.size, solvers, tile)
    assert h, "planner failed"
    try:
        meta = np.zeros(17, np.int64)
        L.hecplan_meta(h, meta)
        P = {k: int(v) for k, v in zip(META, meta)}
        for name in ARRAYS:
            m = L.hecplan_array(h, name.encode(), None)
            a = np.empty(max(m, 0), np.int32)
            if m > 0:
                L.hecplan_array(h, name.encode(), a.ctypes.data_as(C.c_void_p))
            P[name] = a
    finally:
        L.hecplan_free(h)
    P["diag"] = diag
    return P


GRID_META = ("NA", "NB", "NC", "sa", "sb", "sc", "PA", "PB", "S", "ncoef", "TA", "TB")


def make_grid_plan(F, upper, grid):
    """Wavefront plan of one triangle of F on the grid (nx, ny, nz) as a dict, or None when
    the planner gives none."""
    L = lib()
    diag = diag_positions(F)
    h = L.hecplan_grid_make(F.n, _i32(F.LUp), _i32(F.LUj), diag, grid[0], grid[1], grid[2], int(upper))
    if not h:
        return None
    try:
        meta = np.zeros(12, np.int64)
        L.hecplan_grid_meta(h, meta)
        G = {k: int(v) for k, v in zip(GRID_META, meta)}
        m = L.hecplan_grid_src(h, None)
        G["src"] = np.empty(m, np.int32)
        L.hecplan_grid_src(h, G["src"].ctypes.data_as(C.c_void_p))
    finally:
        L.hecplan_grid_free(h)
    return G
