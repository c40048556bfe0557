"""GPU parity of the pool with 64-bit adjacency codes (dt_options.index_bits = 64), the layout
of pools beyond 2^30 tetrahedron slots: every launch variant, degenerate inputs, batches,
and a pool with 32-bit codes widened in the middle of an insertion, each against the oracle."""
import itertools

import numpy as np
import pytest

from synth import batch_clouds, uniform_points
from test_gpu import assert_parity, dtlib, gpu_dt, mix_small, say, sphere50  # noqa: F401  (fixture)
from validators import check_invariants

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("opts", [dict(), dict(lanes_per_insert=4), dict(lanes_per_insert=16), dict(lanes_per_insert=32),
                                  dict(lanes_per_insert=64), dict(cavity_cap=12),
                                  dict(lanes_per_insert=4, cavity_cap=200), dict(cavity_cap=2048),
                                  dict(capacity_tets=4096), dict(round_size=64), dict(large_lanes=64, cavity_cap=12)])
def test_wide_codes_launch_options(dtlib, oracle_mod, opts):
    say(f"64-bit codes, options {opts}")
    xyz = mix_small(52, 4000)
    tets, nbrs, st = gpu_dt(dtlib, xyz, index_bits=64, **opts)
    assert st["index_bits"] == 64
    assert_parity(oracle_mod, xyz, tets, f"wide {opts}")
    check_invariants(xyz, tets, nbrs, oracle_mod, expect_vertices=np.arange(len(xyz)))


@pytest.mark.parametrize("case", ["uniform", "lattice6", "sphere", "cube"])
def test_wide_codes_inputs(dtlib, oracle_mod, case):
    say(f"64-bit codes, {case}")
    xyz = {
        "uniform": uniform_points(50000, 93),
        "lattice6": np.array(list(itertools.product(np.arange(6.0) / 8, repeat=3))),
        "sphere": sphere50(),
        "cube": np.array(list(itertools.product([0.0, 1.0], repeat=3))),
    }[case]
    xyz = np.random.default_rng(12).permutation(xyz)
    tets, nbrs, st = gpu_dt(dtlib, xyz, index_bits=64)
    assert st["index_bits"] == 64
    assert_parity(oracle_mod, xyz, tets, case)
    check_invariants(xyz, tets, nbrs, oracle_mod, expect_vertices=np.arange(len(xyz)))


def test_pool_widened_during_an_insert(dtlib, oracle_mod):
    """An automatic pool starts with 32-bit codes and is widened when it grows past the
    threshold (lowered for the test): records converted between rounds, pending candidates
    kept; then an append and an export."""
    say("pool widened mid-insert")
    xyz = uniform_points(20000, 94)
    more = uniform_points(5000, 95)
    with dtlib.Triangulation(capacity_tets=4096) as tri:
        dtlib.dt_debug_widen_at(tri.ctx, 40000)
        tri.insert(xyz)
        st = tri.stats()
        assert st["index_bits"] == 64
        t, nb = tri.tets()
        assert_parity(oracle_mod, xyz, t.astype(np.int64), "widened")
        check_invariants(xyz, t.astype(np.int64), nb, oracle_mod, expect_vertices=np.arange(len(xyz)))
        tri.insert(more)
        both = np.vstack([xyz, more])
        t, _ = tri.tets()
        assert_parity(oracle_mod, both, t.astype(np.int64), "widened, then appended")
    with dtlib.Triangulation(capacity_tets=4096) as tri:  # below the threshold: stays narrow
        tri.insert(uniform_points(2000, 96))
        assert tri.stats()["index_bits"] == 32


def test_index_bits_32_refuses_a_pool_beyond_its_codes(dtlib, oracle_mod):
    """index_bits = 32 with a pool request past 2^30 - 1 slots is refused before any
    allocation; the context stays usable."""
    say("index_bits 32 limit")
    with dtlib.Triangulation(index_bits=32, capacity_tets=1 << 31) as tri:
        with pytest.raises(dtlib.DTError) as e:
            tri.insert(uniform_points(1000, 97))
        assert e.value.code == dtlib.DT_E_CAPACITY
    with dtlib.Triangulation(index_bits=32) as tri:
        xyz = uniform_points(1000, 97)
        tri.insert(xyz)
        assert tri.stats()["index_bits"] == 32
        t, _ = tri.tets()
        assert_parity(oracle_mod, xyz, t.astype(np.int64), "32-bit codes")


def test_wide_codes_batch(dtlib, oracle_mod):
    say("64-bit codes, batch of 30 clouds")
    xyz, off = batch_clouds(30, seed_base=7200, nmin=4, nmax=3000)
    with dtlib.Triangulation(index_bits=64) as tri:
        tri.insert_batch(xyz, off)
        assert tri.stats()["index_bits"] == 64
        for k in range(30):
            t, nb = tri.tets_batch(k)
            pts = xyz[off[k]:off[k + 1]]
            assert_parity(oracle_mod, pts, t.astype(np.int64), f"cloud {k}")
            if k % 10 == 0:
                check_invariants(pts, t.astype(np.int64), nb, oracle_mod, expect_vertices=np.arange(len(pts)))
