"""Host-side whole-output check of a large tetrahedralization (see fullcheck.c): I1, I2, no
folds and I7 on every tetrahedron and facet with the oracle's exact predicates, then the
hull (few facets) and vertex coverage in numpy.  Test infrastructure."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libfullcheck.so")
CODES = {1: "vertex index out of range or repeated", 2: "non-positive tetrahedron (I1)",
         3: "neighbour index out of range", 4: "neighbour link not mirrored on a shared facet (I2)",
         5: "neighbours overlap (fold)", 6: "facet not locally Delaunay (I7)"}
_lib = None


def build(verbose=False):
    srcs = [os.path.join(HERE, "fullcheck.c"), os.path.join(ROOT, "oracle", "predicates.c"),
            os.path.join(ROOT, "oracle", "exact.c")]
    cmd = ["gcc", "-O2", "-std=gnu99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-Wall", "-o", LIB + ".tmp"] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        L.fullcheck.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]
        L.fullcheck.restype = ctypes.c_int
        _lib = L
    return _lib


def check_all_facets(xyz, tets, nbrs):
    """Runs fullcheck.c; returns (tetrahedra, interior facets, hull facets).  Raises
    AssertionError naming the first failure."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tets = np.ascontiguousarray(tets, dtype=np.uint32)
    nbrs = np.ascontiguousarray(nbrs, dtype=np.int64)
    assert tets.shape == nbrs.shape and tets.shape[1:] == (4,)
    counts = np.zeros(3, dtype=np.int64)
    where = ctypes.c_int64(-1)
    rc = lib().fullcheck(xyz.ctypes.data, len(xyz), tets.ctypes.data, nbrs.ctypes.data, len(tets),
                         counts.ctypes.data, ctypes.byref(where))
    assert rc == 0, f"{CODES.get(rc, rc)} at tetrahedron {where.value}"
    return tuple(int(c) for c in counts)


def check_hull_and_vertices(xyz, tets, nbrs, oracle, n_expect=None, chunk=1 << 26):
    """The faces without neighbour form one closed, locally convex surface (V - E + F = 2,
    every hull edge on exactly two hull facets, exact orient3d across each hull edge), and
    every point index below n_expect is a vertex."""
    from validators import check_hull_convex
    t_idx, j_idx = [], []
    for s in range(0, len(nbrs), chunk):
        a, b = np.nonzero(nbrs[s:s + chunk] < 0)
        t_idx.append(a + s)
        j_idx.append(b)
    t_idx, j_idx = np.concatenate(t_idx), np.concatenate(j_idx)
    sub_t = np.asarray(tets[t_idx], dtype=np.int64)
    sub_n = np.zeros((len(t_idx), 4), dtype=np.int64)
    sub_n[np.arange(len(t_idx)), j_idx] = -1
    H = check_hull_convex(xyz, sub_t, sub_n, oracle)
    rest = np.array([[k for k in range(4) if k != j] for j in range(4)])
    faces = np.sort(sub_t[np.arange(len(t_idx))[:, None], rest[j_idx]], axis=1)
    V = len(np.unique(faces))
    E = len(np.unique(np.sort(faces[:, [[0, 1], [0, 2], [1, 2]]], axis=2).reshape(-1, 2), axis=0))
    assert V - E + H == 2, f"hull surface: V - E + F = {V - E + H}"
    if n_expect is not None:
        seen = np.zeros(int(n_expect), dtype=bool)
        for s in range(0, len(tets), chunk):
            seen[np.asarray(tets[s:s + chunk]).reshape(-1)] = True
        assert bool(seen.all()), f"{int((~seen).sum())} points are not vertices"
    return H
