"""Edge cases of the C ABI on the GPU that need no kernel of their own: empty inserts
(n = 0 inserts nothing) and exports of an empty context, before and around a real insert."""
import numpy as np
import pytest

from synth import uniform_points
from test_gpu import assert_parity, dtlib, say  # noqa: F401  (fixture)

pytestmark = pytest.mark.gpu


def test_empty_inserts(dtlib, oracle_mod):
    say("empty inserts and empty exports")
    with dtlib.Triangulation() as tri:
        tri.insert(np.zeros((0, 3)))
        assert tri.num_tets() == 0
        t, nb = tri.tets()
        assert t.shape == (0, 4) and nb.shape == (0, 4)
        assert tri.stats()["points"] == 0
        xyz = uniform_points(1000, 71)
        tri.insert(xyz)
        t1, _ = tri.tets()
        tri.insert(np.zeros((0, 3)))  # nothing changes
        t2, _ = tri.tets()
        assert np.array_equal(t1, t2)
        assert tri.stats()["points"] == 1000
        assert_parity(oracle_mod, xyz, t2.astype(np.int64), "after empty inserts")


def test_size_limits(dtlib, oracle_mod):
    """2^30 points per call (and per batch) is refused with DT_E_CAPACITY before the points
    are read; the context stays usable."""
    import ctypes
    say("size limits")
    small = np.zeros((4, 3))
    with dtlib.Triangulation() as tri:
        rc = dtlib.lib().dt_insert_points(tri.ctx, small.ctypes.data, 1 << 30)
        assert rc == dtlib.DT_E_CAPACITY
        off = np.array([0, 1 << 30], dtype=np.uint64)
        rc = dtlib.lib().dt_insert_batch(tri.ctx, small.ctypes.data, off.ctypes.data, ctypes.c_uint32(1))
        assert rc == dtlib.DT_E_CAPACITY
        assert tri.num_tets() == 0
        xyz = uniform_points(500, 72)
        tri.insert(xyz)
        t, _ = tri.tets()
        assert_parity(oracle_mod, xyz, t.astype(np.int64), "after refused calls")
