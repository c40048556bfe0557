"""Oracle: a plain serial CPU Delaunay tetrahedralization with exact predicates.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the GPU library.

The C sources (plain C99, one core) follow the paper's Algorithm 1 (Sec. 2.1) with the
exact predicates of Sec. 2.4 and the ghost tetrahedra of Sec. 2.6; see ``oracle.h``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SOURCES = ["exact.c", "predicates.c", "moore.c", "delaunay.c"]
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, E_ARG, E_INPUT, E_DEGENERATE, E_NOMEM = 0, 1, 2, 3, 4
ORDERS = {"brio": 0, "random": 1, "reverse": 2, "input": 3}


class OracleStats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "orient_calls", "orient_exact", "orient_zero",
        "insphere_calls", "insphere_exact", "insphere_zero",
        "walk_steps", "cavity_tets", "boundary_facets", "max_cavity", "duplicates",
        "inserted")]

    def as_dict(self):
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


def build(verbose: bool = False) -> str:
    """Compile the oracle into oracle/liboracle.so with gcc (always recompiles)."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu99", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-Wall", "-o", tmp] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        c_dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_orient3d_batch.argtypes = [c_dp, ctypes.c_int64, ctypes.c_void_p]
        L.oracle_insphere_batch.argtypes = [c_dp, ctypes.c_int64, ctypes.c_void_p]
        L.oracle_insphere_sos_batch.argtypes = [c_dp, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
        L.oracle_moore_level.argtypes = [ctypes.c_int64]
        L.oracle_moore_level.restype = ctypes.c_int
        L.oracle_moore_keys.argtypes = [c_dp, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p]
        L.oracle_moore_index.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.oracle_moore_index.restype = ctypes.c_uint64
        L.oracle_brio_levels.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]
        L.oracle_brio_levels.restype = ctypes.c_int
        L.oracle_stable_sort.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
        L.oracle_delaunay.argtypes = [c_dp, ctypes.c_int64, ctypes.c_int, ctypes.c_uint64,
                                      ctypes.POINTER(ctypes.POINTER(ctypes.c_int32)),
                                      ctypes.POINTER(ctypes.POINTER(ctypes.c_int64)),
                                      ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(OracleStats)]
        L.oracle_delaunay.restype = ctypes.c_int
        L.oracle_free.argtypes = [ctypes.c_void_p]
        _lib = L
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def orient3d(pts: np.ndarray) -> np.ndarray:
    """Exact signs of orient3d for k x 4 x 3 points."""
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 4, 3)
    out = np.empty(len(pts), dtype=np.int8)
    lib().oracle_orient3d_batch(_dptr(pts), len(pts), out.ctypes.data)
    return out


def insphere(pts: np.ndarray) -> np.ndarray:
    """Exact signs of the (unperturbed) lifted 5x5 determinant for k x 5 x 3 points."""
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 5, 3)
    out = np.empty(len(pts), dtype=np.int8)
    lib().oracle_insphere_batch(_dptr(pts), len(pts), out.ctypes.data)
    return out


def insphere_sos(pts: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """Signs of the perturbed lifted determinant (-1 = inside) for k x 5 x 3 points."""
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 5, 3)
    idx = np.ascontiguousarray(idx, dtype=np.int64).reshape(-1, 5)
    out = np.empty(len(pts), dtype=np.int8)
    lib().oracle_insphere_sos_batch(_dptr(pts), idx.ctypes.data, len(pts), out.ctypes.data)
    return out


def moore_level(n: int) -> int:
    return int(lib().oracle_moore_level(int(n)))


def moore_index(cell, m: int) -> int:
    c = np.ascontiguousarray(cell, dtype=np.uint32)
    return int(lib().oracle_moore_index(c.ctypes.data, int(m)))


def moore_keys(xyz: np.ndarray, m: int) -> np.ndarray:
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    out = np.empty(len(xyz), dtype=np.uint64)
    lib().oracle_moore_keys(_dptr(xyz), len(xyz), int(m), out.ctypes.data)
    return out


def brio_levels(n: int, seed: int):
    lev = np.empty(max(int(n), 1), dtype=np.uint8)
    cum = np.zeros(64, dtype=np.int64)
    L = lib().oracle_brio_levels(int(n), int(seed), lev.ctypes.data, cum.ctypes.data)
    return lev[: int(n)], cum[:L]


def stable_sort(keys: np.ndarray) -> np.ndarray:
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    perm = np.empty(len(keys), dtype=np.int64)
    lib().oracle_stable_sort(keys.ctypes.data, len(keys), perm.ctypes.data)
    return perm


def sort_reference(xyz: np.ndarray, seed: int, m: int | None = None):
    """Sorted order of the points by (BRIO level, Moore index on the grid of level m), ties
    by input index; m defaults to the level of the point count.  The keys returned are
    level << 3m | Moore index when that fits 64 bits, else the Moore index alone."""
    n = len(xyz)
    m = moore_level(n) if m is None else int(m)
    lev, cum = brio_levels(n, seed)
    moore = moore_keys(xyz, m)
    if 3 * m + 8 <= 64:
        keys = (lev.astype(np.uint64) << np.uint64(3 * m)) | moore
        return keys, stable_sort(keys), m, cum
    # level first, then the Moore index, ties by input index (lexsort is stable)
    return moore, np.lexsort((moore, lev)).astype(np.int64), m, cum


def delaunay(xyz: np.ndarray, order: str = "brio", seed: int = 0):
    """Returns (rc, tets[T,4] int32, nbrs[T,4] int64, stats dict)."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    pt = ctypes.POINTER(ctypes.c_int32)()
    pn = ctypes.POINTER(ctypes.c_int64)()
    nt = ctypes.c_int64(0)
    st = OracleStats()
    rc = lib().oracle_delaunay(_dptr(xyz), len(xyz), ORDERS[order], int(seed),
                               ctypes.byref(pt), ctypes.byref(pn), ctypes.byref(nt), ctypes.byref(st))
    T = int(nt.value)
    if rc != OK:
        return rc, np.zeros((0, 4), np.int32), np.zeros((0, 4), np.int64), st.as_dict()
    tets = np.ctypeslib.as_array(pt, shape=(T * 4,)).copy().reshape(T, 4) if T else np.zeros((0, 4), np.int32)
    nbrs = np.ctypeslib.as_array(pn, shape=(T * 4,)).copy().reshape(T, 4) if T else np.zeros((0, 4), np.int64)
    lib().oracle_free(ctypes.cast(pt, ctypes.c_void_p))
    lib().oracle_free(ctypes.cast(pn, ctypes.c_void_p))
    return rc, tets, nbrs, st.as_dict()


def canonical(tets: np.ndarray) -> np.ndarray:
    """Each tetrahedron's four indices sorted, rows sorted lexicographically."""
    q = np.sort(np.asarray(tets, dtype=np.int64).reshape(-1, 4), axis=1)
    if len(q) == 0:
        return q
    order = np.lexsort((q[:, 3], q[:, 2], q[:, 1], q[:, 0]))
    return q[order]
