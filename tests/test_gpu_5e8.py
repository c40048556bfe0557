"""5e8 uniform points (seed 5008): the largest configuration, with 64-bit adjacency codes
(about 3.4e9 tetrahedra, 220 GB of tetrahedron pool).  The oracle cannot run at this size, so
a sub-box placed by seed 5009 (side 0.126, about 1e6 points) is compared with the oracle: a
tetrahedron whose circumball lies inside a box B belongs to the tetrahedralization of all
points iff it belongs to that of the points in B.  Every point must be a vertex.

Needs most of one MI355X's memory and about 80 GB of host memory, and takes minutes: it runs
only with DT_TEST_5E8=1 in the environment."""
import os

import numpy as np
import pytest

from synth import uniform_points
from test_gpu import dtlib, say  # noqa: F401  (fixture)
from test_gpu_fullsize import _in_box

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(os.environ.get("DT_TEST_5E8") != "1",
                                 reason="5e8 points need a whole MI355X and minutes: set DT_TEST_5E8=1")]


def test_uniform_5e8_subbox(dtlib, oracle_mod):
    import torch
    n = 500_000_000
    say("5e8 uniform points (seed 5008): generating")
    xyz = uniform_points(n, 5008)
    d = torch.from_numpy(xyz).cuda()
    torch.cuda.synchronize()
    say("triangulating")
    with dtlib.Triangulation(device=0, stream=torch.cuda.current_stream().cuda_stream) as tri:
        tri.insert(d)
        del d
        torch.cuda.empty_cache()
        st = tri.stats()
        T = tri.num_tets()
        say(f"{T} tetrahedra, {st['rounds']} rounds, index_bits {st['index_bits']}, "
            f"dropped slots {st['dropped_slots']}")
        assert st["index_bits"] == 64 and T > 6.7 * n
        t = np.empty((T, 4), dtype=np.uint32)
        assert dtlib.dt_get_tets(tri.ctx, t, None, T) == T
    say("exported; classifying")
    lo = 0.05 + 0.8 * uniform_points(1, 5009)[0]
    side = 0.126
    hi = lo + side
    inb = np.all((xyz >= lo) & (xyz < hi), axis=1)
    sub_idx = np.nonzero(inb)[0]
    m = torch.from_numpy(inb).cuda()
    seen = torch.zeros(n, dtype=torch.bool, device="cuda")
    keep = []
    chunk = 1 << 26
    for s in range(0, T, chunk):
        q = torch.from_numpy(t[s:s + chunk].view(np.int32)).cuda().long()
        seen[q.reshape(-1)] = True
        keep.append(q[m[q].all(dim=1)].cpu().numpy())
        del q
    assert int(seen.sum()) == n, "a point is not a vertex"
    g = np.concatenate(keep)
    del t
    g = g[_in_box(xyz, g, lo, hi)]
    say(f"sub-box [{lo}, {hi}): {len(sub_idx)} points, {len(g)} GPU tetrahedra with the ball inside")
    rc, ot, _, _ = oracle_mod.delaunay(xyz[sub_idx])
    assert rc == 0
    o = sub_idx[ot.astype(np.int64)]
    o = o[_in_box(xyz, o, lo, hi)]
    a, b = oracle_mod.canonical(g), oracle_mod.canonical(o)
    say(f"oracle: {len(b)} tetrahedra with the ball inside")
    assert len(a) > 0.5 * 6.5 * len(sub_idx)
    assert a.shape == b.shape and np.array_equal(a, b)
