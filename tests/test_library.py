"""CPU checks of the HIP library: it builds, loads without a GPU, and exports every entry point
that include/dt.h declares; host-side logic that needs no device."""
import ctypes
import os
import re

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
    for field, bad in [("lanes_per_insert", 5), ("lanes_per_insert", 32), ("round_fraction", -1.0)]:
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
        "dt_get_point_log": (n, n, n, n, n),
        "dt_train_model": (n, n, n, n, 0, 0, 0.0, 0, n, n),
        "dt_load_model": (n, n, 0),
        "dt_debug_mlp": (n, n, 0, n),
        "dt_debug_mlp_grad": (n, n, n, n, 0, n, n),
        "dt_debug_sort": (n, n, 0, n, n, n),
        "dt_debug_predicates": (n, 0, n, n, 0, n),
        "dt_clear": (n,),
        "dt_destroy": (n,),
        "dt_get_stats": (n, n),
    }
    assert set(calls) | {"dt_default_options", "dt_create", "dt_last_error"} == set(declared_functions())
    for name, args in calls.items():
        assert getattr(L, name)(*args) == dt.DT_E_ARG, name


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
