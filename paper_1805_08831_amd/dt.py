"""Thin ctypes binding of libdt.so (include/dt.h).  Argument marshalling only: every step
of the triangulation runs in the library's HIP kernels.  PyTorch, when given, only supplies
device memory (tensor.data_ptr()) and the stream."""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdt.so")

DT_OK, DT_E_ARG, DT_E_INPUT, DT_E_DEGENERATE, DT_E_CAPACITY, DT_E_INCOMPLETE, DT_E_DEVICE, DT_E_INTERNAL = range(8)
ERROR_NAMES = {0: "DT_OK", 1: "DT_E_ARG", 2: "DT_E_INPUT", 3: "DT_E_DEGENERATE", 4: "DT_E_CAPACITY",
               5: "DT_E_INCOMPLETE", 6: "DT_E_DEVICE", 7: "DT_E_INTERNAL"}


class DTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class dt_options(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("stream", ctypes.c_void_p), ("round_size", ctypes.c_uint32),
                ("cavity_cap", ctypes.c_uint32), ("capacity_tets", ctypes.c_uint64), ("seed", ctypes.c_uint64),
                ("max_rounds", ctypes.c_uint32), ("timing", ctypes.c_int), ("round_fraction", ctypes.c_double),
                ("lanes_per_insert", ctypes.c_uint32), ("scheduler", ctypes.c_int), ("log_points", ctypes.c_int),
                ("index_bits", ctypes.c_int), ("adaptive_curve", ctypes.c_int), ("subdet_cache", ctypes.c_int), ("walk_cap", ctypes.c_uint32),
                ("large_lanes", ctypes.c_uint32), ("graph_rounds", ctypes.c_int)]

DT_SCHED_PLAIN, DT_SCHED_LEARNED = 0, 1
NFEAT, NHID, NOUT = 16, 64, 3
NPARAM = NFEAT * NHID + NHID + NHID * NHID + NHID + NHID * NOUT + NOUT


_STAT_U64 = ["points", "vertices", "duplicates", "tets", "rounds", "attempts", "inserted", "conflicts",
             "overflows", "walk_steps", "cavity_tets", "boundary_facets", "orient_calls", "orient_exact",
             "insphere_calls", "insphere_exact", "perturbed"]


class dt_stats(ctypes.Structure):
    _fields_ = ([(n, ctypes.c_uint64) for n in _STAT_U64] +
                [("ms_total", ctypes.c_double), ("ms_sort", ctypes.c_double), ("ms_insert", ctypes.c_double),
                 ("cavity_launches", ctypes.c_uint64), ("ball_launches", ctypes.c_uint64),
                 ("ms_cavity_kernel", ctypes.c_double), ("ms_ball_kernel", ctypes.c_double),
                 ("cavity_units", ctypes.c_uint64), ("ball_units", ctypes.c_uint64),
                 ("sched_fallbacks", ctypes.c_uint64), ("index_bits", ctypes.c_uint64),
                 ("dropped_slots", ctypes.c_uint64), ("deferred", ctypes.c_uint64),
                 ("walk_caps", ctypes.c_uint64), ("timed_attempts", ctypes.c_uint64),
                 ("timed_insertions", ctypes.c_uint64), ("graph_rounds", ctypes.c_uint64)])

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


_lib = None


def lib():
    """Load libdt.so; fails loudly when the HIP library has not been built."""
    global _lib
    if _lib is None:
        # One HIP runtime per process: when PyTorch is installed its bundled runtime (same
        # soname as ROCm's) is loaded first so that the library binds to it and device
        # pointers and streams are shared with torch.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1805_08831_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, u64, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
        L.dt_default_options.argtypes = [ctypes.POINTER(dt_options)]
        L.dt_default_options.restype = None
        L.dt_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(dt_options)]
        L.dt_insert_points.argtypes = [vp, vp, u64]
        L.dt_get_tets.argtypes = [vp, vp, vp, ctypes.POINTER(u64)]
        L.dt_clear.argtypes = [vp]
        L.dt_destroy.argtypes = [vp]
        L.dt_get_stats.argtypes = [vp, ctypes.POINTER(dt_stats)]
        L.dt_last_error.argtypes = [vp]
        L.dt_last_error.restype = ctypes.c_char_p
        L.dt_insert_batch.argtypes = [vp, vp, vp, ctypes.c_uint32]
        L.dt_get_tets_batch.argtypes = [vp, ctypes.c_uint32, vp, vp, ctypes.POINTER(u64)]
        L.dt_autotune.argtypes = [vp, vp, u64, ctypes.POINTER(dt_options), ctypes.POINTER(ctypes.c_double)]
        L.dt_autotune_reset.argtypes = [vp]
        L.dt_get_point_log.argtypes = [vp, vp, vp, vp, ctypes.POINTER(u64)]
        L.dt_train_model.argtypes = [vp, vp, vp, vp, u64, ctypes.c_uint32, ctypes.c_float, u64, vp,
                                     ctypes.POINTER(ctypes.c_size_t)]
        L.dt_load_model.argtypes = [vp, vp, ctypes.c_size_t]
        L.dt_debug_mlp.argtypes = [vp, vp, u64, vp]
        L.dt_debug_mlp_grad.argtypes = [vp, vp, vp, vp, ctypes.c_uint32, vp, vp]
        L.dt_debug_sort.argtypes = [vp, vp, u64, vp, vp, ctypes.POINTER(i32)]
        L.dt_debug_predicates.argtypes = [vp, i32, vp, vp, u64, vp]
        L.dt_debug_set_round_counter.argtypes = [vp, u64]
        L.dt_debug_widen_at.argtypes = [vp, u64]
        L.dt_triangulate_noalloc.argtypes = [i32, vp, vp, u64, vp, vp, ctypes.POINTER(u64)]
        L.dt_refine.argtypes = [vp, ctypes.c_double, ctypes.c_uint32, vp, ctypes.POINTER(ctypes.c_uint32),
                                ctypes.POINTER(u64)]
        L.dt_get_points.argtypes = [vp, vp, ctypes.POINTER(u64)]
        for f in ("dt_create", "dt_insert_points", "dt_get_tets", "dt_clear", "dt_destroy", "dt_get_stats",
                  "dt_insert_batch", "dt_get_tets_batch", "dt_autotune", "dt_autotune_reset", "dt_get_point_log",
                  "dt_train_model",
                  "dt_load_model", "dt_debug_mlp", "dt_debug_mlp_grad", "dt_debug_sort", "dt_debug_predicates",
                  "dt_debug_set_round_counter", "dt_debug_widen_at", "dt_triangulate_noalloc", "dt_refine",
                  "dt_get_points"):
            getattr(L, f).restype = i32
        _lib = L
    return _lib


def _ptr(x):
    """Address of a numpy array or torch tensor (contiguous), or None."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("array is not C-contiguous")
        return x.ctypes.data
    if not x.is_contiguous():
        raise ValueError("tensor is not contiguous")
    return x.data_ptr()


def _dtype(x):
    return str(x.dtype).replace("torch.", "")


def _numel(x):
    return int(x.size) if isinstance(x, np.ndarray) else int(x.numel())


def _points(xyz, n=None):
    """Checks an n x 3 float64 point buffer (the library reads 24 n bytes from it) and
    returns (address, n)."""
    if _dtype(xyz) != "float64":
        raise ValueError(f"points must be float64, got {xyz.dtype}")
    if n is None:
        if len(xyz.shape) != 2 or int(xyz.shape[1]) != 3:
            raise ValueError(f"points must have shape (n, 3), got {tuple(xyz.shape)}")
        n = int(xyz.shape[0])
    if _numel(xyz) < 3 * int(n):
        raise ValueError(f"{int(n)} points need {3 * int(n)} values, the buffer holds {_numel(xyz)}")
    return _ptr(xyz), int(n)


def _out(buf, dtypes, count, what):
    """Checks an output buffer of at least `count` elements of one of `dtypes`."""
    if buf is None:
        return None
    if _dtype(buf) not in dtypes:
        raise ValueError(f"{what} must be {' or '.join(dtypes)}, got {buf.dtype}")
    if _numel(buf) < count:
        raise ValueError(f"{what} holds {_numel(buf)} elements, {count} needed")
    return _ptr(buf)


# --------------------------------------------------------------------- C-ABI mirror

def dt_default_options():
    o = dt_options()
    lib().dt_default_options(ctypes.byref(o))
    return o


def dt_create(opt=None):
    h = ctypes.c_void_p()
    rc = lib().dt_create(ctypes.byref(h), ctypes.byref(opt) if opt is not None else None)
    if rc != DT_OK:
        raise DTError(rc, "dt_create failed")
    return h


def _check(ctx, rc):
    if rc != DT_OK:
        raise DTError(rc, lib().dt_last_error(ctx).decode())


def dt_insert_points(ctx, xyz, n=None):
    p, n = _points(xyz, n)
    _check(ctx, lib().dt_insert_points(ctx, p, n))


_TET_TYPES, _NBR_TYPES = ("int32", "uint32"), ("int64",)


def dt_get_tets(ctx, tets=None, nbrs=None, capacity=0):
    num = ctypes.c_uint64(capacity)
    pt = _out(tets, _TET_TYPES, 4 * int(capacity), "tets")
    pn = _out(nbrs, _NBR_TYPES, 4 * int(capacity), "nbrs")
    _check(ctx, lib().dt_get_tets(ctx, pt, pn, ctypes.byref(num)))
    return int(num.value)


def dt_insert_batch(ctx, xyz, offsets):
    """offsets: host array of num_clouds + 1 uint64 (numpy)."""
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    if len(off) < 2:
        raise ValueError("offsets must hold num_clouds + 1 >= 2 entries")
    p, _ = _points(xyz, int(off[-1]))
    _check(ctx, lib().dt_insert_batch(ctx, p, off.ctypes.data, int(len(off) - 1)))


def dt_get_tets_batch(ctx, cloud, tets=None, nbrs=None, capacity=0):
    num = ctypes.c_uint64(capacity)
    pt = _out(tets, _TET_TYPES, 4 * int(capacity), "tets")
    pn = _out(nbrs, _NBR_TYPES, 4 * int(capacity), "nbrs")
    _check(ctx, lib().dt_get_tets_batch(ctx, int(cloud), pt, pn, ctypes.byref(num)))
    return int(num.value)


def dt_autotune(ctx, xyz):
    """Returns (chosen dt_options, ms of the chosen configuration on the sample)."""
    best, ms = dt_options(), ctypes.c_double(0.0)
    p, n = _points(xyz)
    _check(ctx, lib().dt_autotune(ctx, p, n, ctypes.byref(best), ctypes.byref(ms)))
    return best, float(ms.value)


def dt_autotune_reset(ctx):
    _check(ctx, lib().dt_autotune_reset(ctx))


def dt_get_point_log(ctx):
    """(features[n,16] f32, cost[n] f32, bucket[n] u8) of the last logged insertion."""
    num = ctypes.c_uint64(0)
    _check(ctx, lib().dt_get_point_log(ctx, None, None, None, ctypes.byref(num)))
    n = int(num.value)
    f = np.empty((n, NFEAT), dtype=np.float32)
    c = np.empty(n, dtype=np.float32)
    b = np.empty(n, dtype=np.uint8)
    _check(ctx, lib().dt_get_point_log(ctx, f.ctypes.data, c.ctypes.data, b.ctypes.data, ctypes.byref(num)))
    return f, c, b


def dt_train_model(ctx, features, cost, bucket, epochs=4, lr=1e-3, seed=1):
    """Trains (and loads) a model; returns its bytes."""
    f = np.ascontiguousarray(features, dtype=np.float32)
    c = np.ascontiguousarray(cost, dtype=np.float32)
    b = np.ascontiguousarray(bucket, dtype=np.uint8)
    size = ctypes.c_size_t(0)
    _check(ctx, lib().dt_train_model(ctx, f.ctypes.data, c.ctypes.data, b.ctypes.data, len(c), 0, 0.0, 0, None,
                                     ctypes.byref(size)))
    buf = ctypes.create_string_buffer(size.value)
    _check(ctx, lib().dt_train_model(ctx, f.ctypes.data, c.ctypes.data, b.ctypes.data, len(c), int(epochs),
                                     float(lr), int(seed), buf, ctypes.byref(size)))
    return bytes(buf.raw[:size.value])


def dt_load_model(ctx, model):
    buf = ctypes.create_string_buffer(model, len(model))
    _check(ctx, lib().dt_load_model(ctx, buf, len(model)))


def dt_debug_mlp(ctx, features):
    f = np.ascontiguousarray(features, dtype=np.float32)
    out = np.empty((len(f), NOUT), dtype=np.float32)
    _check(ctx, lib().dt_debug_mlp(ctx, f.ctypes.data, len(f), out.ctypes.data))
    return out


def dt_debug_mlp_grad(ctx, features, cost, bucket):
    f = np.ascontiguousarray(features, dtype=np.float32)
    c = np.ascontiguousarray(cost, dtype=np.float32)
    b = np.ascontiguousarray(bucket, dtype=np.uint8)
    g = np.empty(NPARAM, dtype=np.float32)
    loss = np.zeros(1, dtype=np.float32)
    _check(ctx, lib().dt_debug_mlp_grad(ctx, f.ctypes.data, c.ctypes.data, b.ctypes.data, len(c), g.ctypes.data,
                                        loss.ctypes.data))
    return g, float(loss[0])


def dt_clear(ctx):
    _check(ctx, lib().dt_clear(ctx))


def dt_destroy(ctx):
    lib().dt_destroy(ctx)


def dt_get_stats(ctx):
    s = dt_stats()
    _check(ctx, lib().dt_get_stats(ctx, ctypes.byref(s)))
    return s.as_dict()


def dt_debug_sort(ctx, xyz):
    p, n = _points(xyz)
    keys = np.empty(n, dtype=np.uint64)
    perm = np.empty(n, dtype=np.uint32)
    m = ctypes.c_int(0)
    _check(ctx, lib().dt_debug_sort(ctx, p, n, keys.ctypes.data, perm.ctypes.data, ctypes.byref(m)))
    return keys, perm, int(m.value)


def dt_debug_set_round_counter(ctx, rounds):
    _check(ctx, lib().dt_debug_set_round_counter(ctx, int(rounds)))


def dt_triangulate_noalloc(xyz, tets=None, nbrs=None, capacity=0, device=0, stream=None):
    """The no-allocation entry point: triangulates xyz (n x 3 float64, host or device) with
    the library's static scratch memory; fills tets / nbrs (may be None) and returns T."""
    p, n = _points(xyz)
    _out(tets, _TET_TYPES, 4 * int(capacity), "tets")
    _out(nbrs, _NBR_TYPES, 4 * int(capacity), "nbrs")
    cnt = ctypes.c_uint64(int(capacity))
    rc = lib().dt_triangulate_noalloc(int(device), stream, p, n, _ptr(tets), _ptr(nbrs), ctypes.byref(cnt))
    if rc != DT_OK:
        raise DTError(rc, f"dt_triangulate_noalloc returned {ERROR_NAMES.get(rc, rc)} (needs {cnt.value} tetrahedra)")
    return int(cnt.value)


def dt_refine(ctx, h, max_steps=100):
    """Refinement steps (see dt.h); returns (points inserted, [(candidates, kept) per step])."""
    counts = np.zeros(2 * int(max_steps), dtype=np.uint32)
    ns = ctypes.c_uint32(0)
    ins = ctypes.c_uint64(0)
    _check(ctx, lib().dt_refine(ctx, float(h), int(max_steps), counts.ctypes.data, ctypes.byref(ns), ctypes.byref(ins)))
    k = int(ns.value)
    return int(ins.value), [(int(counts[2 * i]), int(counts[2 * i + 1])) for i in range(k)]


def dt_get_points(ctx):
    """(n, 3) float64 coordinates of every inserted point, by global input index."""
    n = ctypes.c_uint64(0)
    _check(ctx, lib().dt_get_points(ctx, None, ctypes.byref(n)))
    out = np.empty((int(n.value), 3), dtype=np.float64)
    _check(ctx, lib().dt_get_points(ctx, out.ctypes.data, ctypes.byref(n)))
    return out


def dt_debug_widen_at(ctx, slots):
    _check(ctx, lib().dt_debug_widen_at(ctx, int(slots)))


def dt_debug_predicates(ctx, kind, pts, idx=None):
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    k = int(pts.shape[0])
    npts = 4 if int(kind) == 0 else 5
    if pts.size != 3 * npts * k:
        raise ValueError(f"kind {kind} needs {npts} points (x, y, z) per record, {3 * npts * k} values")
    out = np.empty(k, dtype=np.int8)
    idx = None if idx is None else np.ascontiguousarray(idx, dtype=np.int64)
    if idx is not None and idx.size != 5 * k:
        raise ValueError("idx must hold 5 input indices per record")
    _check(ctx, lib().dt_debug_predicates(ctx, int(kind), pts.ctypes.data, _ptr(idx), k, out.ctypes.data))
    return out


# --------------------------------------------------------------------- convenience class

class Triangulation:
    """One library context.  `insert` takes an (n, 3) float64 numpy array or torch tensor
    (host or device); `tets` returns (tets[T,4] uint32, nbrs[T,4] int64)."""

    def __init__(self, device=0, stream=None, round_size=0, cavity_cap=0, capacity_tets=0, seed=0x5EED,
                 max_rounds=0, timing=False, round_fraction=0.0, lanes_per_insert=0, scheduler=0, log_points=False,
                 index_bits=0, adaptive_curve=False, subdet_cache=False, walk_cap=0, large_lanes=0,
                 graph_rounds=False):
        o = dt_default_options()
        o.device, o.round_size, o.cavity_cap = int(device), int(round_size), int(cavity_cap)
        o.capacity_tets, o.seed, o.max_rounds = int(capacity_tets), int(seed), int(max_rounds)
        o.timing, o.round_fraction = int(timing), float(round_fraction)
        o.lanes_per_insert = int(lanes_per_insert)
        o.scheduler, o.log_points = int(scheduler), int(bool(log_points))
        o.index_bits = int(index_bits)
        o.adaptive_curve = int(bool(adaptive_curve))
        o.subdet_cache = int(bool(subdet_cache))
        o.walk_cap = int(walk_cap)
        o.large_lanes = int(large_lanes)
        o.graph_rounds = int(bool(graph_rounds))
        o.stream = stream
        self.ctx = dt_create(o)

    def insert(self, xyz):
        if isinstance(xyz, np.ndarray):
            xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        dt_insert_points(self.ctx, xyz)

    def insert_batch(self, xyz, offsets):
        """Independent clouds: cloud k is xyz[offsets[k]:offsets[k+1]]."""
        if isinstance(xyz, np.ndarray):
            xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        dt_insert_batch(self.ctx, xyz, offsets)

    def tets_batch(self, cloud):
        """(tets[T,4] uint32, nbrs[T,4] int64) of one cloud, in its local indices."""
        T = dt_get_tets_batch(self.ctx, cloud)
        tets = np.empty((T, 4), dtype=np.uint32)
        nbrs = np.empty((T, 4), dtype=np.int64)
        dt_get_tets_batch(self.ctx, cloud, tets, nbrs, T)
        return tets, nbrs

    def autotune_reset(self):
        dt_autotune_reset(self.ctx)

    def autotune(self, xyz):
        """Picks lanes per insertion, round fraction and cavity cap for the sample's size
        class (see dt.h)."""
        if isinstance(xyz, np.ndarray):
            xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        best, ms = dt_autotune(self.ctx, xyz)
        return {"lanes_per_insert": best.lanes_per_insert, "round_fraction": best.round_fraction,
                "cavity_cap": best.cavity_cap, "large_lanes": best.large_lanes, "ms": ms}

    def num_tets(self):
        return dt_get_tets(self.ctx)

    def tets(self, device_tensors=False):
        T = dt_get_tets(self.ctx)
        if device_tensors:
            import torch
            tets = torch.empty((T, 4), dtype=torch.int32, device="cuda")
            nbrs = torch.empty((T, 4), dtype=torch.int64, device="cuda")
        else:
            tets = np.empty((T, 4), dtype=np.uint32)
            nbrs = np.empty((T, 4), dtype=np.int64)
        dt_get_tets(self.ctx, tets, nbrs, T)
        return tets, nbrs

    def stats(self):
        return dt_get_stats(self.ctx)

    def clear(self):
        dt_clear(self.ctx)

    def close(self):
        if self.ctx is not None:
            dt_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
