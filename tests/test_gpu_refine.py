"""GPU Delaunay refinement (dt_refine, paper Sec. 4) against the refinement oracle's stored
results (tests/golden/refine_golden.txt, written by make_refine_golden.py from the oracle
alone): the same steps (candidates and kept points per step), the same final point set bit
for bit, and the same tetrahedralization."""
import hashlib
import os

import numpy as np
import pytest

from synth import cluster_points, shell_points, uniform_points
from test_gpu import dtlib, say  # noqa: F401  (fixture)
from validators import check_invariants

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "refine_golden.txt")


def _cases():
    out = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        left, right = line.split("|")
        kind, n, seed, h = left.split()
        npts, steps, ht, hp = right.split()
        out.append((kind, int(n), int(seed), float(h), int(npts),
                    [tuple(int(x) for x in s.split("/")) for s in steps.split(";")], ht, hp))
    return out


@pytest.mark.parametrize("case", _cases(), ids=lambda c: f"{c[0]}-{c[1]}-{c[3]}")
def test_refine_matches_the_oracle(dtlib, oracle_mod, case):
    kind, n, seed, h, npts, steps, ht, hp = case
    say(f"refine {kind} n={n} seed={seed} h={h}")
    xyz = (uniform_points(n, seed) if kind == "uniform" else shell_points(n, seed) if kind == "shell"
           else cluster_points(n, seed, clusters=4))
    with dtlib.Triangulation() as tri:
        tri.insert(xyz)
        added, got_steps = dtlib.dt_refine(tri.ctx, h)
        pts = dtlib.dt_get_points(tri.ctx)
        t, nb = tri.tets()
    say(f"steps {got_steps}, {added} points added")
    assert got_steps == steps
    assert len(pts) == npts and added == npts - n
    assert np.array_equal(pts[:n], xyz)
    assert hashlib.sha256(np.ascontiguousarray(pts).tobytes()).hexdigest() == hp
    canon = oracle_mod.canonical(t.astype(np.int64)).astype(np.int64)
    assert hashlib.sha256(canon.tobytes()).hexdigest() == ht
    if npts < 5000:
        check_invariants(pts, t.astype(np.int64), nb, oracle_mod, expect_vertices=np.arange(npts))


FULLSIZE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "refine_fullsize_golden.txt")


def test_refine_benchmark_size(dtlib, oracle_mod):
    """The benchmark's refinement workload (2.5e5 uniform points, seed 4007, h = 0.0064; about
    1.5e6 final points) against the oracle's stored result for it
    (tests/golden/refine_fullsize_golden.txt, written by make_refine_golden.py --fullsize from
    the oracle alone): the same passes (candidates and kept points), the same final points bit
    for bit and the same tetrahedra; and, by what holds at any size, every added point lies
    at least 0.7 h from every other vertex."""
    from scipy.spatial import cKDTree
    rows = [l.split("|") for l in open(FULLSIZE) if l.strip() and not l.startswith("#")]
    (kind, n, seed, h), (npts, steps, ht, hp) = rows[0][0].split(), rows[0][1].split()
    n, seed, h, npts = int(n), int(seed), float(h), int(npts)
    steps = [tuple(int(x) for x in st.split("/")) for st in steps.split(";")]
    assert (kind, n, seed, h) == ("uniform", 250_000, 4007, 0.0064)
    say(f"refine uniform n={n} seed={seed} h={h}")
    xyz = uniform_points(n, seed)
    with dtlib.Triangulation() as tri:
        tri.insert(xyz)
        added, got_steps = dtlib.dt_refine(tri.ctx, h)
        pts = dtlib.dt_get_points(tri.ctx)
        t, _ = tri.tets()
    say(f"steps {got_steps}, {added} points added, {len(t)} tetrahedra")
    assert got_steps == steps
    assert len(pts) == npts and added == npts - n
    assert np.array_equal(pts[:n], xyz)
    assert hashlib.sha256(np.ascontiguousarray(pts).tobytes()).hexdigest() == hp
    canon = oracle_mod.canonical(t.astype(np.int64)).astype(np.int64)
    assert hashlib.sha256(canon.tobytes()).hexdigest() == ht
    d, _ = cKDTree(pts).query(pts[n:], k=2)
    assert d[:, 1].min() >= 0.7 * h * (1 - 1e-12)
