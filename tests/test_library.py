"""CPU checks of the HIP library: it builds, loads without a GPU, and exports every entry point
that include/dt.h declares; host-side logic that needs no device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1805_08831_amd", "libdt.so")


def declared_functions():
    src = open(os.path.join(ROOT, "include", "dt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return re.findall(r"^\s*(?:[A-Za-z_][\w\s\*]*?)\b(dt_\w+)\s*\(", src, re.M)


@pytest.fixture(scope="module")
def libdt():
    if not os.path.exists(LIB):
        from paper_1805_08831_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_exports_every_declared_symbol(libdt):
    names = declared_functions()
    assert len(names) >= 10
    for n in ["dt_create", "dt_insert_points", "dt_get_tets", "dt_destroy"]:
        assert n in names
    missing = [n for n in names if not hasattr(libdt, n)]
    assert not missing, missing


def test_default_options_and_argument_errors(libdt):
    from paper_1805_08831_amd import dt
    o = dt.dt_options()
    dt.lib().dt_default_options(ctypes.byref(o))
    assert o.device == 0 and o.seed == 0x5EED and o.round_size == 0 and o.stream is None
    # NULL arguments are rejected before any device work
    assert dt.lib().dt_create(None, None) == dt.DT_E_ARG
    assert dt.lib().dt_insert_points(None, None, 0) == dt.DT_E_ARG
    assert dt.lib().dt_get_tets(None, None, None, None) == dt.DT_E_ARG
    assert dt.lib().dt_destroy(None) == dt.DT_E_ARG
    assert dt.lib().dt_last_error(None) == b"no context"
    # invalid options are rejected before any device work
    h = ctypes.c_void_p()
    for field, bad in [("lanes_per_insert", 5), ("lanes_per_insert", 128), ("round_fraction", -1.0),
                       ("large_lanes", 128), ("graph_rounds", 2)]:
        o2 = dt.dt_options()
        dt.lib().dt_default_options(ctypes.byref(o2))
        setattr(o2, field, bad)
        assert dt.lib().dt_create(ctypes.byref(h), ctypes.byref(o2)) == dt.DT_E_ARG, field


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1805_08831_amd import dt
    monkeypatch.setattr(dt, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(dt, "_lib", None)
    with pytest.raises(RuntimeError):
        dt.lib()


def test_every_entry_point_rejects_a_null_context(libdt):
    """Each entry point that takes a context returns DT_E_ARG for NULL, touching nothing."""
    from paper_1805_08831_amd import dt
    L = dt.lib()
    n = None
    calls = {
        "dt_insert_points": (n, n, 0),
        "dt_insert_batch": (n, n, n, 0),
        "dt_get_tets": (n, n, n, n),
        "dt_get_tets_batch": (n, 0, n, n, n),
        "dt_autotune": (n, n, 0, n, n),
        "dt_autotune_reset": (n,),
        "dt_get_point_log": (n, n, n, n, n),
        "dt_train_model": (n, n, n, n, 0, 0, 0.0, 0, n, n),
        "dt_load_model": (n, n, 0),
        "dt_debug_mlp": (n, n, 0, n),
        "dt_debug_mlp_grad": (n, n, n, n, 0, n, n),
        "dt_debug_sort": (n, n, 0, n, n, n),
        "dt_debug_predicates": (n, 0, n, n, 0, n),
        "dt_debug_set_round_counter": (n, 0),
        "dt_debug_widen_at": (n, 0),
        "dt_refine": (n, 0.1, 10, n, n, n),
        "dt_get_points": (n, n, n),
        "dt_clear": (n,),
        "dt_destroy": (n,),
        "dt_get_stats": (n, n),
    }
    assert set(calls) | {"dt_default_options", "dt_create", "dt_last_error", "dt_triangulate_noalloc"} == \
        set(declared_functions())
    for name, args in calls.items():
        assert getattr(L, name)(*args) == dt.DT_E_ARG, name
    # the context-free entry point checks its arguments before touching a device
    assert L.dt_triangulate_noalloc(0, None, None, 0, None, None, None) == dt.DT_E_ARG
    assert L.dt_triangulate_noalloc(-1, None, None, 0, None, None, None) == dt.DT_E_ARG


def test_create_without_a_device_fails_cleanly(libdt):
    """With valid options, dt_create either succeeds (a GPU is present) or returns
    DT_E_DEVICE with the handle cleared; it never returns a half-built context."""
    from paper_1805_08831_amd import dt
    o = dt.dt_options()
    dt.lib().dt_default_options(ctypes.byref(o))
    o.device = 0
    h = ctypes.c_void_p(1)
    rc = dt.lib().dt_create(ctypes.byref(h), ctypes.byref(o))
    if rc == dt.DT_OK:
        assert h.value
        assert dt.lib().dt_destroy(h) == dt.DT_OK
    else:
        assert rc == dt.DT_E_DEVICE and not h.value


def test_binding_checks_buffers_before_the_library(libdt):
    """The binding rejects buffers the library would read or write out of bounds (wrong
    dtype, shape or size, or not contiguous) with ValueError, before any library call; valid
    buffers reach the library (here with no context: DT_E_ARG)."""
    import torch
    from paper_1805_08831_amd import dt
    bad_points = [np.zeros((5, 3), np.float32), np.zeros((5, 2)), np.zeros((3, 5))[:, :3],
                  torch.zeros((5, 3), dtype=torch.float32), np.zeros((5, 3, 1))]
    for x in bad_points:
        with pytest.raises(ValueError):
            dt.dt_insert_points(None, x)
        with pytest.raises(ValueError):
            dt.dt_autotune(None, x)
    with pytest.raises(ValueError):
        dt.dt_insert_points(None, np.zeros(9), n=4)
    with pytest.raises(ValueError):
        dt.dt_insert_batch(None, np.zeros((10, 3)), [0, 5, 11])
    with pytest.raises(ValueError):
        dt.dt_insert_batch(None, np.zeros((10, 3)), [0])
    for t, nb in [(np.zeros((3, 4), np.int64), None), (np.zeros((2, 4), np.int32), None),
                  (None, np.zeros((3, 4), np.int32)), (None, np.zeros((2, 4), np.int64)),
                  (torch.zeros((3, 4), dtype=torch.float32), None), (np.zeros((4, 3), np.int32).T, None)]:
        with pytest.raises(ValueError):
            dt.dt_get_tets(None, t, nb, 3)
        with pytest.raises(ValueError):
            dt.dt_get_tets_batch(None, 0, t, nb, 3)
    with pytest.raises(ValueError):
        dt.dt_debug_predicates(None, 1, np.zeros((4, 12)))
    with pytest.raises(ValueError):
        dt.dt_debug_predicates(None, 2, np.zeros((4, 15)), np.zeros((4, 4), np.int64))
    # accepted forms: (n, 3) float64 arrays and tensors, flat or 2-D 4-byte and 8-byte
    # outputs of at least 4 * capacity elements, offset views
    good = [lambda: dt.dt_insert_points(None, np.zeros((5, 3))),
            lambda: dt.dt_insert_points(None, torch.zeros((5, 3), dtype=torch.float64)),
            lambda: dt.dt_insert_points(None, np.zeros((10, 3))[2:7]),
            lambda: dt.dt_insert_batch(None, np.zeros((10, 3)), np.array([0, 4, 10], np.uint64)),
            lambda: dt.dt_get_tets(None),
            lambda: dt.dt_get_tets(None, np.zeros((3, 4), np.uint32), np.zeros((3, 4), np.int64), 3),
            lambda: dt.dt_get_tets(None, torch.zeros(13, dtype=torch.int32)[1:13],
                                   torch.zeros(13, dtype=torch.int64)[1:13], 3),
            lambda: dt.dt_get_tets(None, torch.zeros((4, 4), dtype=torch.int32), None, 3),
            lambda: dt.dt_get_tets_batch(None, 0, np.zeros((3, 4), np.uint32), np.zeros((3, 4), np.int64), 3),
            lambda: dt.dt_debug_predicates(None, 0, np.zeros((4, 12))),
            lambda: dt.dt_debug_predicates(None, 2, np.zeros((4, 15)), np.zeros((4, 5), np.int64))]
    for call in good:
        with pytest.raises(dt.DTError) as e:
            call()
        assert e.value.code == dt.DT_E_ARG
