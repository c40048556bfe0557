"""The seeded input generators (CPU): splitmix64 against its published outputs, the
counter layout, and the recipe of each workload (ranges, distinctness, sizes)."""
import numpy as np

from synth import batch_clouds, cluster_points, lattice_points, mix_points, shell_points, uniform_points
from synth.generators import splitmix64

GAMMA = 0x9E3779B97F4A7C15


def test_splitmix64_published_outputs():
    """Vigna's splitmix64 from state 0 returns e220a8397b1dcdaf, 6e789e6aa1b965f4,
    06c45d188009454f: the finaliser of the counters 0, gamma and 2 gamma."""
    c = np.array([0, GAMMA, (2 * GAMMA) % 2 ** 64], dtype=np.uint64)
    assert [int(v) for v in splitmix64(c)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_uniform_grid_prefix_and_streams():
    a = uniform_points(1000, 7)
    assert a.shape == (1000, 3) and a.dtype == np.float64
    assert np.all((a >= 0.0) & (a < 1.0))
    assert np.all(np.floor(a * 2.0 ** 53) == a * 2.0 ** 53)  # on the 2^-53 grid
    # counter-based: a prefix is the same points, another seed other points
    assert np.array_equal(uniform_points(10, 7), a[:10])
    assert not np.array_equal(uniform_points(10, 8), a[:10])
    # coordinate 0 of point 0 is draw 0 of stream 0 of the seed
    x = int(splitmix64(np.array([7 << 40], dtype=np.uint64))[0])
    assert a[0, 0] == (x >> 11) * 2.0 ** -53


def test_lattice_nodes_distinct_and_dyadic():
    side = 10
    p = lattice_points(side ** 3, 3, side=side)
    assert len(np.unique(p, axis=0)) == side ** 3  # all nodes, none twice
    q = p * 512.0 + (side - 1)
    assert np.all(q == np.round(q)) and np.all(q % 2 == 0) and q.min() == 0 and q.max() == 2 * (side - 1)
    sub = lattice_points(300, 3, side=side)
    assert len(np.unique(sub, axis=0)) == 300
    assert np.array_equal(lattice_points(300, 3, side=side), sub)


def test_shell_and_clusters():
    s = shell_points(20000, 5)
    r = np.linalg.norm(s, axis=1)
    assert np.all(np.abs(r - 1.0) <= 1e-4 * (1 + 1e-9))
    assert abs(np.mean(s[:, 2])) < 0.05  # directions roughly uniform
    c = cluster_points(5000, 5, clusters=50)
    assert c.shape == (5000, 3) and np.all(np.isfinite(c))
    # 100 points per cluster, each cluster tight (sigma <= 0.05) around a centre in r <= 0.9
    for k in range(0, 50, 7):
        blk = c[100 * k:100 * (k + 1)]
        cen = blk.mean(axis=0)
        assert np.linalg.norm(cen) < 0.9 + 0.05
        assert np.all(blk.std(axis=0) < 0.08)


def test_mix_is_the_three_parts_shuffled():
    m = mix_points(4, 500, 400, 300, side=20)
    parts = np.vstack([lattice_points(500, 4, side=20), cluster_points(400, 4), shell_points(300, 4)])
    assert m.shape == (1200, 3)
    a = m[np.lexsort(m.T[::-1])]
    b = parts[np.lexsort(parts.T[::-1])]
    assert np.array_equal(a, b)
    assert not np.array_equal(m, parts)


def test_batch_clouds_recipe():
    pts, off = batch_clouds(16, seed_base=3000)
    sizes = np.diff(off.astype(np.int64))
    assert off[0] == 0 and off[-1] == len(pts) and len(off) == 17
    assert np.all((sizes >= 1000) & (sizes <= 200000))
    for c in range(16):
        p = pts[int(off[c]):int(off[c + 1])]
        lo, hi = p.min(axis=0), p.max(axis=0)
        assert np.all(lo >= -10.0) and np.all(lo <= 10.0)
        ext = hi - lo
        assert np.all(ext <= 10.0) and np.all(ext >= 0.1 * 0.98)
    # cloud c is seeded by seed_base + c alone
    p3, o3 = batch_clouds(4, seed_base=3003)
    assert np.array_equal(p3[:int(o3[1])], pts[int(off[3]):int(off[4])])
