"""The no-allocation entry point (dt_triangulate_noalloc, static scratch memory) through the C
ABI, against the allocating entry points (dt_insert_points + dt_get_tets) on the same inputs:
the triangulation is unique, so the canonical tetrahedra must be equal.  Two calls in a row,
the second smaller, then host buffers, a degenerate input, the size limit and n = 0."""
import ctypes

import numpy as np
import pytest

from synth import uniform_points
from test_gpu import dtlib, mix_small, say  # noqa: F401  (fixture)
from validators import check_invariants

pytestmark = pytest.mark.gpu


def _allocating(dtlib, oracle_mod, xyz):
    with dtlib.Triangulation() as tri:
        tri.insert(xyz)
        t, _ = tri.tets()
    return oracle_mod.canonical(t.astype(np.int64))


def _noalloc_device(dtlib, xyz):
    import torch
    d = torch.from_numpy(xyz).cuda()
    stream = torch.cuda.current_stream().cuda_stream
    torch.cuda.synchronize()
    T = dtlib.dt_triangulate_noalloc(d, stream=stream)
    t = torch.full((T, 4), -1, dtype=torch.int32, device="cuda")
    nb = torch.full((T, 4), -2, dtype=torch.int64, device="cuda")
    assert dtlib.dt_triangulate_noalloc(d, t, nb, T, stream=stream) == T
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.int64), nb.cpu().numpy()


def test_noalloc_matches_the_allocating_path(dtlib, oracle_mod):
    say("no-alloc: 65536 points (the limit), then 20000 points")
    for n, seed in ((65536, 301), (20000, 302)):
        xyz = uniform_points(n, seed)
        t, nb = _noalloc_device(dtlib, xyz)
        a, b = oracle_mod.canonical(t), _allocating(dtlib, oracle_mod, xyz)
        say(f"n={n}: {len(a)} tetrahedra without allocation, {len(b)} with")
        assert a.shape == b.shape and np.array_equal(a, b)
        check_invariants(xyz, t, nb, oracle_mod, expect_vertices=np.arange(n), exact_volume=n < 30000)


def test_noalloc_host_buffers_and_degenerate_input(dtlib, oracle_mod):
    say("no-alloc: host buffers, MIX input")
    xyz = mix_small(303, 6000)
    T = dtlib.dt_triangulate_noalloc(xyz)
    t = np.full((T, 4), 7, dtype=np.uint32)
    nb = np.zeros((T, 4), dtype=np.int64)
    assert dtlib.dt_triangulate_noalloc(xyz, t, nb, T) == T
    assert np.array_equal(oracle_mod.canonical(t.astype(np.int64)), _allocating(dtlib, oracle_mod, xyz))
    check_invariants(xyz, t.astype(np.int64), nb, oracle_mod, expect_vertices=np.arange(len(xyz)))


def test_noalloc_limits(dtlib):
    say("no-alloc: size limit, empty input, small output buffer")
    L = dtlib.lib()
    cnt = ctypes.c_uint64(0)
    big = np.zeros((4, 3))
    assert L.dt_triangulate_noalloc(0, None, big.ctypes.data, 65537, None, None, ctypes.byref(cnt)) == \
        dtlib.DT_E_CAPACITY
    assert dtlib.dt_triangulate_noalloc(np.zeros((0, 3))) == 0
    xyz = uniform_points(1000, 304)
    T = dtlib.dt_triangulate_noalloc(xyz)
    small = np.zeros((T - 1, 4), dtype=np.uint32)
    with pytest.raises(dtlib.DTError) as e:
        dtlib.dt_triangulate_noalloc(xyz, small, None, T - 1)
    assert e.value.code == dtlib.DT_E_ARG
    # still usable afterwards
    assert dtlib.dt_triangulate_noalloc(xyz) == T
