"""GPU parity: the HIP library, called through its C ABI, against the oracle.

The triangulation is unique (perturbed Delaunay), so parity is bit-exact equality of the
canonically sorted vertex quadruples; the invariants (orientation, adjacency, Euler
characteristic, vertex coverage, volume, local Delaunay) are checked on the GPU output too.
"""
import itertools
import sys

import numpy as np
import pytest

from synth import batch_clouds, cluster_points, lattice_points, shell_points, uniform_points
from validators import check_invariants

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dtlib():
    from paper_1805_08831_amd import dt
    dt.lib()
    return dt


def gpu_dt(dtlib, xyz, **opts):
    with dtlib.Triangulation(**opts) as tri:
        tri.insert(np.ascontiguousarray(xyz, dtype=np.float64))
        tets, nbrs = tri.tets()
        return tets.astype(np.int64), nbrs, tri.stats()


def oracle_dt(oracle_mod, xyz):
    rc, tets, nbrs, st = oracle_mod.delaunay(xyz)
    assert rc == 0
    return tets, nbrs, st


def assert_parity(oracle_mod, xyz, tets_gpu, label):
    ref_tets, _, _ = oracle_dt(oracle_mod, xyz)
    a, b = oracle_mod.canonical(tets_gpu), oracle_mod.canonical(ref_tets)
    assert a.shape == b.shape, f"{label}: {a.shape} vs {b.shape}"
    assert np.array_equal(a, b), f"{label}: quadruples differ"


def sphere50():
    return np.array([(x, y, z) for x in range(-8, 8) for y in range(-8, 8) for z in range(-8, 8)
                     if x * x + y * y + z * z == 50], dtype=np.float64) / 8.0


def mix_small(seed, n_each):
    return np.random.default_rng(seed).permutation(np.vstack([
        lattice_points(n_each, seed, side=int(np.ceil((1.05 * n_each) ** (1 / 3))) + 1),
        cluster_points(n_each, seed, clusters=5), shell_points(n_each, seed)]))


# ------------------------------------------------------------------ predicates

def test_predicates_match_oracle(dtlib, oracle_mod):
    say("predicates")
    rng = np.random.default_rng(7)
    cases4, cases5, idx5 = [], [], []
    for s in range(2000):
        cases4.append(uniform_points(4, 10000 + s))
        cases5.append(uniform_points(5, 20000 + s))
    lat = lattice_points(120, 3, side=5)
    sph = sphere50()
    cube = np.array(list(itertools.product([0.0, 1.0], repeat=3)))
    for _ in range(2000):
        cases4.append(lat[rng.choice(len(lat), 4, replace=False)])
        src = [lat, sph, cube][rng.integers(3)]
        cases5.append(src[rng.choice(len(src), 5, replace=False)])
    for s in range(500):  # near-degenerate: a point on the plane of three, nudged
        p = uniform_points(3, 30000 + s)
        u, v = rng.random(2)
        q = p[0] + u * (p[1] - p[0]) + v * (p[2] - p[0])
        q[0] = np.nextafter(q[0], np.inf if s % 2 else -np.inf)
        cases4.append(np.vstack([p, q]))
    # wide exponent spread
    for s in range(300):
        c = uniform_points(5, 40000 + s) * (2.0 ** rng.integers(-100, 100, size=(5, 1)))
        cases5.append(c)
        cases4.append(c[:4])
    p4, p5 = np.array(cases4), np.array(cases5)
    ctx = dtlib.dt_create()
    try:
        o4 = dtlib.dt_debug_predicates(ctx, 0, p4.reshape(len(p4), -1))
        assert np.array_equal(o4, oracle_mod.orient3d(p4))
        o5 = dtlib.dt_debug_predicates(ctx, 1, p5.reshape(len(p5), -1))
        assert np.array_equal(o5, oracle_mod.insphere(p5))
        # perturbed: rows abcd must be positive
        ori = oracle_mod.orient3d(p5[:, :4])
        keep = ori != 0
        q5 = p5[keep].copy()
        neg = ori[keep] < 0
        q5[neg, 0], q5[neg, 1] = p5[keep][neg, 1], p5[keep][neg, 0]
        idx = np.array([rng.permutation(10 ** 6)[:5] for _ in range(len(q5))])
        s5 = dtlib.dt_debug_predicates(ctx, 2, q5.reshape(len(q5), -1), idx)
        assert np.array_equal(s5, oracle_mod.insphere_sos(q5, idx))
        assert np.count_nonzero(oracle_mod.insphere(q5) == 0) > 100
    finally:
        dtlib.dt_destroy(ctx)


def test_exact_stage_widths_match_oracle(dtlib, oracle_mod):
    """Near-degenerate orient3d and insphere cases whose coordinates span 2^-s .. 1, for s
    around 26 bits: the integer stage's fixed-width form in registers takes spreads up to 26
    bits and the general form the wider ones; both must give the oracle's signs."""
    say("exact stage widths")
    rng = np.random.default_rng(11)
    cases4, cases5 = [], []
    for s in (20, 24, 25, 26, 27, 28, 32, 40):
        for k in range(150):
            p = uniform_points(3, 50000 + 1000 * s + k) + 0.25
            p[k % 3, k % 2] = np.ldexp(0.5 + 0.5 * rng.random(), -s)  # one tiny coordinate
            u, v = rng.random(2)
            q = p[0] + u * (p[1] - p[0]) + v * (p[2] - p[0])
            q[1] = np.nextafter(q[1], np.inf if k % 2 else -np.inf)
            cases4.append(np.vstack([p, q]))
            a = uniform_points(4, 60000 + 1000 * s + k) + 0.25
            a[k % 4, 2] = np.ldexp(0.5 + 0.5 * rng.random(), -s)
            # a fifth point on the circumsphere of the four, up to rounding
            A = 2.0 * (a[1:] - a[0])
            bvec = (a[1:] ** 2).sum(1) - (a[0] ** 2).sum()
            c = np.linalg.solve(A, bvec)
            d = rng.normal(size=3)
            e = c + np.linalg.norm(a[0] - c) * d / np.linalg.norm(d)
            cases5.append(np.vstack([a, e]))
    p4, p5 = np.array(cases4), np.array(cases5)
    want4, want5 = oracle_mod.orient3d(p4), oracle_mod.insphere(p5)
    ctx = dtlib.dt_create()
    try:
        assert np.array_equal(dtlib.dt_debug_predicates(ctx, 0, p4.reshape(len(p4), -1)), want4)
        assert np.array_equal(dtlib.dt_debug_predicates(ctx, 1, p5.reshape(len(p5), -1)), want5)
    finally:
        dtlib.dt_destroy(ctx)
    # both signs occur: the cases are near, not on, the degenerate configurations
    assert set(np.unique(want4)) >= {-1, 1} and set(np.unique(want5)) >= {-1, 1}


# ------------------------------------------------------------------ sort

@pytest.mark.parametrize("kind,n", [("uniform", 1017), ("uniform", 100000), ("mix", 30000)])
def test_sort_matches_oracle(dtlib, oracle_mod, kind, n):
    say(f"sort {kind} {n}")
    xyz = uniform_points(n, 1001) if kind == "uniform" else mix_small(5, n // 3)
    ctx = dtlib.dt_create()
    try:
        keys, perm, m = dtlib.dt_debug_sort(ctx, xyz)
    finally:
        dtlib.dt_destroy(ctx)
    rkeys, rperm, rm, _ = oracle_mod.sort_reference(xyz, 0x5EED)
    assert m == rm
    assert np.array_equal(keys, rkeys)
    assert np.array_equal(perm.astype(np.int64), rperm)


@pytest.mark.parametrize("kind,n", [("uniform", 20000), ("mix", 30000)])
def test_adaptive_curve_sort_matches_oracle(dtlib, oracle_mod, kind, n):
    """The adaptive curve: the same definition on the grid of 21 levels."""
    say(f"adaptive sort {kind} {n}")
    xyz = uniform_points(n, 1002) if kind == "uniform" else mix_small(6, n // 3)
    o = dtlib.dt_default_options()
    o.adaptive_curve = 1
    ctx = dtlib.dt_create(o)
    try:
        keys, perm, m = dtlib.dt_debug_sort(ctx, xyz)
    finally:
        dtlib.dt_destroy(ctx)
    rkeys, rperm, rm, _ = oracle_mod.sort_reference(xyz, 0x5EED, m=21)
    assert m == rm == 21
    assert np.array_equal(keys, rkeys)
    assert np.array_equal(perm.astype(np.int64), rperm)


@pytest.mark.parametrize("case", ["uniform", "mix", "lattice6", "sphere", "widened"])
def test_subdet_cache_keeps_result(dtlib, oracle_mod, case):
    """Cached sub-determinants (Sec. 2.4): the cavity search's insphere as a dot product with a
    filter bound of its own; undecided signs go to the exact predicates.  Same triangulation;
    the pool grows (the cache is copied) and is widened in one case."""
    say(f"sub-determinant cache, {case}")
    xyz = {
        "uniform": lambda: uniform_points(30000, 401),
        "mix": lambda: mix_small(402, 6000),
        "lattice6": lambda: np.random.default_rng(3).permutation(
            np.array(list(itertools.product(np.arange(6.0) / 8, repeat=3)))),
        "sphere": lambda: sphere50(),
        "widened": lambda: uniform_points(20000, 403),
    }[case]()
    opts = dict(subdet_cache=True)
    if case in ("uniform", "widened"):
        opts["capacity_tets"] = 4096  # grows several times
    with dtlib.Triangulation(**opts) as tri:
        if case == "widened":
            dtlib.dt_debug_widen_at(tri.ctx, 40000)
        tri.insert(np.ascontiguousarray(xyz, dtype=np.float64))
        t, nb = tri.tets()
        st = tri.stats()
    assert_parity(oracle_mod, xyz, t.astype(np.int64), f"subdet cache {case}")
    if case == "widened":
        assert st["index_bits"] == 64
    if len(xyz) < 10000:
        check_invariants(xyz, t.astype(np.int64), nb, oracle_mod, expect_vertices=np.arange(len(xyz)))


def test_adaptive_curve_keeps_result(dtlib, oracle_mod):
    say("adaptive curve triangulation")
    xyz = mix_small(53, 6000)
    tets, nbrs, st = gpu_dt(dtlib, xyz, adaptive_curve=True)
    assert_parity(oracle_mod, xyz, tets, "adaptive curve")


# ------------------------------------------------------------------ triangulations

@pytest.mark.parametrize("n,seed", [(4, 1), (5, 2), (6, 3), (8, 4), (12, 5), (33, 6), (100, 7), (1000, 8),
                                    (4999, 9), (20000, 10)])
def test_uniform_small(dtlib, oracle_mod, n, seed):
    say(f"uniform n={n} seed={seed}")
    xyz = uniform_points(n, seed)
    tets, nbrs, st = gpu_dt(dtlib, xyz)
    assert_parity(oracle_mod, xyz, tets, f"uniform {n}")
    check_invariants(xyz, tets, nbrs, oracle_mod, expect_vertices=np.arange(n))


def test_uniform_1e5(dtlib, oracle_mod):
    """1e5 i.i.d. uniform points, seed 1001: exact match with the oracle."""
    say("uniform 1e5")
    xyz = uniform_points(100000, 1001)
    tets, nbrs, st = gpu_dt(dtlib, xyz)
    assert_parity(oracle_mod, xyz, tets, "uniform 1e5")
    check_invariants(xyz, tets, nbrs, oracle_mod, expect_vertices=np.arange(len(xyz)))
    say(f"stats {st}")


@pytest.mark.parametrize("case", ["cube", "cube_center", "lattice3", "lattice6", "sphere", "coplanar_hull"])
def test_degenerate_sets(dtlib, oracle_mod, case):
    say(f"degenerate {case}")
    cube = np.array(list(itertools.product([0.0, 1.0], repeat=3)))
    grid = np.array([[x, y, 0.0] for x in range(4) for y in range(4)])
    xyz = {
        "cube": cube,
        "cube_center": np.vstack([cube, [[0.5, 0.5, 0.5]]]),
        "lattice3": np.array(list(itertools.product([0.0, 0.5, 1.0], repeat=3))),
        "lattice6": np.array(list(itertools.product(np.arange(6.0) / 8, repeat=3))),
        "sphere": sphere50(),
        "coplanar_hull": np.vstack([grid, [[1.5, 1.5, 1.0], [0.5, 2.5, 0.75], [2.5, 0.5, 1.25]]]),
    }[case]
    xyz = np.random.default_rng(11).permutation(xyz)
    tets, nbrs, st = gpu_dt(dtlib, xyz)
    assert_parity(oracle_mod, xyz, tets, case)
    check_invariants(xyz, tets, nbrs, oracle_mod, expect_vertices=np.arange(len(xyz)))


@pytest.mark.parametrize("n_each", [3000, 20000])
def test_mix(dtlib, oracle_mod, n_each):
    say(f"mix {n_each}")
    xyz = mix_small(21, n_each)
    tets, nbrs, st = gpu_dt(dtlib, xyz)
    assert_parity(oracle_mod, xyz, tets, "mix")
    check_invariants(xyz, tets, nbrs, oracle_mod, expect_vertices=np.arange(len(xyz)))
    assert st["insphere_exact"] > 0 and st["perturbed"] > 0


def test_errors(dtlib):
    say("errors")
    cases = {
        "coplanar": (np.c_[uniform_points(100, 3)[:, :2], np.zeros(100)], dtlib.DT_E_DEGENERATE),
        "three": (uniform_points(3, 3), dtlib.DT_E_DEGENERATE),
        "nan": (np.where(np.arange(30).reshape(10, 3) == 7, np.nan, uniform_points(10, 4)), dtlib.DT_E_INPUT),
        "huge": (np.where(np.arange(30).reshape(10, 3) == 5, 1e300, uniform_points(10, 4)), dtlib.DT_E_INPUT),
        "tiny": (np.where(np.arange(30).reshape(10, 3) == 5, 1e-300, uniform_points(10, 4)), dtlib.DT_E_INPUT),
    }
    for name, (xyz, code) in cases.items():
        with dtlib.Triangulation() as tri:
            with pytest.raises(dtlib.DTError) as e:
                tri.insert(np.ascontiguousarray(xyz))
            assert e.value.code == code, name
            assert tri.num_tets() == 0


def test_duplicates_within_and_across_calls(dtlib, oracle_mod):
    say("duplicates")
    xyz = uniform_points(3000, 31)
    dup = np.vstack([xyz[[5]], xyz, xyz[[7, 100, 7, 2999]]])  # index 0 duplicates index 6
    tets, nbrs, st = gpu_dt(dtlib, dup)
    assert_parity(oracle_mod, dup, tets, "duplicates")
    assert st["duplicates"] == 5
    assert 6 not in set(tets.reshape(-1).tolist())
    # across calls: the second call repeats points of the first
    with dtlib.Triangulation() as tri:
        tri.insert(xyz[:2000])
        tri.insert(np.vstack([xyz[2000:], xyz[:10]]))
        t2, n2 = tri.tets()
    assert_parity(oracle_mod, np.vstack([xyz, xyz[:10]]), t2.astype(np.int64), "duplicates across calls")


def test_append_and_clear(dtlib, oracle_mod):
    say("append")
    xyz = uniform_points(30000, 41)
    with dtlib.Triangulation() as tri:
        for a, b in [(0, 7), (7, 5000), (5000, 5001), (5001, 30000)]:
            tri.insert(xyz[a:b])
        t, nb = tri.tets()
        assert_parity(oracle_mod, xyz, t.astype(np.int64), "append")
        check_invariants(xyz, t.astype(np.int64), nb, oracle_mod, expect_vertices=np.arange(len(xyz)))
        tri.clear()
        other = uniform_points(5000, 42)
        tri.insert(other)
        t, nb = tri.tets()
        assert_parity(oracle_mod, other, t.astype(np.int64), "after clear")


@pytest.mark.parametrize("opts", [dict(cavity_cap=4), dict(cavity_cap=12), dict(round_size=64),
                                  dict(round_size=1 << 16), dict(round_fraction=2.0), dict(seed=99),
                                  dict(lanes_per_insert=4), dict(lanes_per_insert=16),
                                  dict(lanes_per_insert=32), dict(lanes_per_insert=64),
                                  dict(lanes_per_insert=4, cavity_cap=200),
                                  dict(cavity_cap=2048), dict(lanes_per_insert=16, cavity_cap=1500),
                                  dict(capacity_tets=4096), dict(walk_cap=1), dict(walk_cap=3),
                                  dict(walk_cap=0xFFFFFFFF), dict(large_lanes=64, cavity_cap=4),
                                  dict(large_lanes=256, cavity_cap=4), dict(large_lanes=64, cavity_cap=12)])
def test_launch_options_do_not_change_result(dtlib, oracle_mod, opts):
    say(f"options {opts}")
    xyz = mix_small(51, 4000)
    tets, nbrs, st = gpu_dt(dtlib, xyz, **opts)
    assert_parity(oracle_mod, xyz, tets, str(opts))
    if opts.get("cavity_cap") == 4:
        assert st["overflows"] > 0
    if "capacity_tets" in opts:  # the pool grew several times between rounds
        assert len(tets) > 4 * opts["capacity_tets"]
    if opts.get("walk_cap") in (1, 3):  # walks stopped and resumed in later rounds
        assert st["walk_caps"] > 0
    if opts.get("walk_cap") == 0xFFFFFFFF:
        assert st["walk_caps"] == 0


def test_round_limit(dtlib):
    say("round limit")
    with dtlib.Triangulation(max_rounds=1) as tri:
        with pytest.raises(dtlib.DTError) as e:
            tri.insert(uniform_points(20000, 5))
        assert e.value.code == dtlib.DT_E_INCOMPLETE


def test_device_buffers_through_torch(dtlib, oracle_mod):
    """Device input and device outputs (the benchmark's path)."""
    say("device buffers")
    import torch
    xyz = uniform_points(50000, 61)
    d = torch.from_numpy(xyz).cuda()
    torch.cuda.synchronize()
    with dtlib.Triangulation(stream=torch.cuda.current_stream().cuda_stream) as tri:
        tri.insert(d)
        t, nb = tri.tets(device_tensors=True)
        torch.cuda.synchronize()
        t = t.cpu().numpy().astype(np.int64)
        nb = nb.cpu().numpy()
    assert_parity(oracle_mod, xyz, t, "device buffers")
    check_invariants(xyz, t, nb, oracle_mod, expect_vertices=np.arange(len(xyz)))
    # device buffers that are not 16-byte aligned (views one element in) give the same output
    with dtlib.Triangulation(stream=torch.cuda.current_stream().cuda_stream) as tri:
        tri.insert(d)
        T = dtlib.dt_get_tets(tri.ctx)
        bt = torch.full((T + 1, 4), -7, dtype=torch.int32, device="cuda")
        bn = torch.full((T + 1, 4), -7, dtype=torch.int64, device="cuda")
        vt = bt.view(-1)[1:1 + 4 * T]
        vn = bn.view(-1)[1:1 + 4 * T]
        assert vt.data_ptr() % 16 and vn.data_ptr() % 16
        assert dtlib.dt_get_tets(tri.ctx, vt, vn, T) == T
        t2, nb2 = tri.tets(device_tensors=True)  # aligned, same context: same order
        torch.cuda.synchronize()
        assert np.array_equal(vt.cpu().numpy().reshape(T, 4), t2.cpu().numpy())
        assert np.array_equal(vn.cpu().numpy().reshape(T, 4), nb2.cpu().numpy())
        assert bt.view(-1)[0].item() == -7 and bn.view(-1)[0].item() == -7


# ------------------------------------------------------------------ batches of clouds

def _concat(clouds):
    off = np.concatenate([[0], np.cumsum([len(c) for c in clouds])]).astype(np.uint64)
    return np.ascontiguousarray(np.vstack(clouds), dtype=np.float64), off


def test_batch_clouds_match_oracle(dtlib, oracle_mod):
    """Many independent clouds in one call: each equals the oracle run on that cloud alone."""
    say("batch: 40 clouds of 4 .. 3000 points in random boxes")
    xyz, off = batch_clouds(40, seed_base=7000, nmin=4, nmax=3000)
    with dtlib.Triangulation() as tri:
        tri.insert_batch(xyz, off)
        for k in range(40):
            pts = xyz[off[k]:off[k + 1]]
            t, nb = tri.tets_batch(k)
            assert_parity(oracle_mod, pts, t.astype(np.int64), f"cloud {k}")
            if k % 8 == 0:
                check_invariants(pts, t.astype(np.int64), nb, oracle_mod, expect_vertices=np.arange(len(pts)))
        assert tri.stats()["points"] == int(off[-1])


def test_batch_mixed_clouds(dtlib, oracle_mod):
    """Clouds sharing coordinates stay independent; duplicates are removed within a cloud;
    a cospherical lattice and a lone tetrahedron; no dt_insert_points on a batch."""
    say("batch: shared coordinates, duplicates, lattice, single tetrahedron")
    a = uniform_points(500, 11)
    dups = np.vstack([uniform_points(300, 12), uniform_points(300, 12)[:50]])
    clouds = [a, a.copy(), dups, lattice_points(216, 5, side=6),
              np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.float64)]
    xyz, off = _concat(clouds)
    with dtlib.Triangulation() as tri:
        tri.insert_batch(xyz, off)
        for k, pts in enumerate(clouds):
            t, _ = tri.tets_batch(k)
            assert_parity(oracle_mod, pts, t.astype(np.int64), f"cloud {k}")
        assert tri.stats()["duplicates"] == 50
        with pytest.raises(dtlib.DTError) as e:
            tri.insert(uniform_points(10, 1))
        assert e.value.code == dtlib.DT_E_ARG
        tri.clear()
        tri.insert(uniform_points(1000, 13))
        t, _ = tri.tets_batch(0)
        assert_parity(oracle_mod, uniform_points(1000, 13), t.astype(np.int64), "single cloud after clear")


def test_batch_export_to_unaligned_device_buffers(dtlib, oracle_mod):
    """dt_get_tets_batch into device buffers that are not 16-byte aligned goes through the
    staging buffers and must give what the aligned export gives."""
    say("batch: export into unaligned device buffers")
    import torch
    xyz, off = batch_clouds(6, seed_base=7100, nmin=500, nmax=3000)
    with dtlib.Triangulation(stream=torch.cuda.current_stream().cuda_stream) as tri:
        tri.insert_batch(xyz, off)
        for k in range(6):
            T = dtlib.dt_get_tets_batch(tri.ctx, k)
            bt = torch.full((T + 1, 4), -7, dtype=torch.int32, device="cuda")
            bn = torch.full((T + 1, 4), -7, dtype=torch.int64, device="cuda")
            vt = bt.view(-1)[1:1 + 4 * T]
            vn = bn.view(-1)[1:1 + 4 * T]
            assert vt.data_ptr() % 16 and vn.data_ptr() % 16
            assert dtlib.dt_get_tets_batch(tri.ctx, k, vt, vn, T) == T
            torch.cuda.synchronize()
            t, nb = tri.tets_batch(k)
            assert np.array_equal(vt.cpu().numpy().reshape(T, 4), t.astype(np.int32))
            assert np.array_equal(vn.cpu().numpy().reshape(T, 4), nb)
            assert bt.view(-1)[0].item() == -7 and bn.view(-1)[0].item() == -7
            assert_parity(oracle_mod, xyz[off[k]:off[k + 1]], t.astype(np.int64), f"cloud {k}")


def test_claim_stamps_across_the_round_counter_wrap(dtlib, oracle_mod):
    """Claim stamps take the low 32 bits of the round counter; the rounds of this insert
    cross the wrap (the library resets the claim words there), and the result is unchanged."""
    say("round counter wrap")
    xyz = uniform_points(30000, 81)
    with dtlib.Triangulation() as tri:
        tri.insert(uniform_points(2000, 80))  # claims left in the pool by earlier rounds
        tri.clear()
        dtlib.dt_debug_set_round_counter(tri.ctx, (1 << 32) - 7)
        tri.insert(xyz)
        assert tri.stats()["rounds"] > 7
        t, nb = tri.tets()
        assert_parity(oracle_mod, xyz, t.astype(np.int64), "across the wrap")


def test_batch_degenerate_cloud(dtlib):
    say("batch: a coplanar cloud is reported by index")
    flat = np.array([[x, y, 0.0] for x in range(3) for y in range(3)], dtype=np.float64)
    xyz, off = _concat([uniform_points(100, 3), flat])
    with dtlib.Triangulation() as tri:
        with pytest.raises(dtlib.DTError) as e:
            tri.insert_batch(xyz, off)
        assert e.value.code == dtlib.DT_E_DEGENERATE and "cloud 1" in str(e.value)


def test_autotune_keeps_results(dtlib, oracle_mod):
    say("autotune at two sizes, then triangulations of sizes near each and between them")
    with dtlib.Triangulation() as tri:
        for size, seed in ((20000, 31), (3000, 33)):
            best = tri.autotune(uniform_points(size, seed))
            assert best["lanes_per_insert"] in (0, 8, 16, 32) and best["cavity_cap"] in (64, 128)
            assert best["large_lanes"] in (64, 256)
            assert best["round_fraction"] in (0.0, 3 / 64, 3 / 32) and best["ms"] > 0
            assert tri.stats()["points"] == 0
        for n, seed in ((5000, 32), (2500, 34), (40000, 35)):
            xyz = uniform_points(n, seed)
            tri.insert(xyz)
            t, _ = tri.tets()
            assert_parity(oracle_mod, xyz, t.astype(np.int64), f"tuned, {n} points")
            tri.clear()
        tri.autotune_reset()
        xyz = uniform_points(4000, 36)
        tri.insert(xyz)
        t, _ = tri.tets()
        assert_parity(oracle_mod, xyz, t.astype(np.int64), "after the reset")


# ------------------------------------------------------------------ learned scheduler

def _bf16(a):
    """fp32 -> bf16 (round to nearest even) -> fp32: the kernels' weight copies."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return (u & 0xFFFFFFFF).astype(np.uint32).view(np.float32)


def _unpack(model, F=16, H=64, O=3):
    hdr = np.frombuffer(model[:24], dtype=np.uint32)
    assert tuple(hdr[2:6]) == (F, H, O, F * H + H + H * H + H + H * O + O)
    w = np.frombuffer(model[32:], dtype=np.float32)
    out, o = [], 0
    for shape in [(F, H), (H,), (H, H), (H,), (H, O), (O,)]:
        k = int(np.prod(shape))
        out.append(w[o:o + k].reshape(shape))
        o += k
    return out


def _synthetic_samples(n, seed):
    rng = np.random.default_rng(seed)
    f = rng.normal(size=(n, 16)).astype(np.float32)
    cost = (0.5 * f[:, 0] - 0.3 * f[:, 3] + 0.2 * f[:, 5] * f[:, 6] + 1.0).astype(np.float32)
    bucket = (f[:, 1] + 0.5 * f[:, 2] > 0).astype(np.uint8)
    return f, cost, bucket


def test_mlp_matches_cpu_reference(dtlib):
    """The BF16-weight / FP32-accumulate inference and training-gradient kernels against
    PyTorch CPU float32 with the same bf16-rounded weights; training fits a known target."""
    import torch
    say("mlp: inference and gradient vs CPU reference, training fit")
    f, cost, bucket = _synthetic_samples(16384, 5)
    with dtlib.Triangulation() as tri:
        model = dtlib.dt_train_model(tri.ctx, f, cost, bucket, epochs=40, lr=3e-3, seed=7)
        ps = [torch.tensor(_bf16(p)).requires_grad_(True) for p in _unpack(model)]

        def forward(x):
            h1 = torch.relu(x @ ps[0] + ps[1])
            h2 = torch.relu(h1 @ ps[2] + ps[3])
            return h2 @ ps[4] + ps[5]

        y = dtlib.dt_debug_mlp(tri.ctx, f[:2048])
        np.testing.assert_allclose(y, forward(torch.tensor(f[:2048])).detach().numpy(), rtol=1e-4, atol=1e-4)
        n = 3000
        g, loss = dtlib.dt_debug_mlp_grad(tri.ctx, f[:n], cost[:n], bucket[:n])
        out = forward(torch.tensor(f[:n]))
        ref = ((out[:, 0] - torch.tensor(cost[:n])) ** 2).mean() + \
            torch.nn.functional.cross_entropy(out[:, 1:3], torch.tensor(bucket[:n]).long())
        ref.backward()
        gr = torch.cat([p.grad.reshape(-1) for p in ps]).numpy()
        np.testing.assert_allclose(g, gr, rtol=2e-3, atol=2e-6)
        assert abs(loss / n - ref.item()) < 1e-3 * (1.0 + ref.item())
        yall = dtlib.dt_debug_mlp(tri.ctx, f)
        assert np.corrcoef(yall[:, 0], cost)[0, 1] > 0.9
        assert ((yall[:, 2] > yall[:, 1]) == (bucket == 1)).mean() > 0.9


def test_learned_scheduler_keeps_result(dtlib, oracle_mod):
    """Trained on the log of a plain run (another seed); the learned order gives the same
    triangulation as the oracle."""
    say("learned scheduler: train on a plain MIX log, run MIX of another seed")
    train = mix_small(61, 5000)
    with dtlib.Triangulation(log_points=True) as tri:
        tri.insert(train)
        f, c, b = dtlib.dt_get_point_log(tri.ctx)
        assert f.shape == (len(train), 16) and np.isfinite(f).all()
        # every point but the 4 of the initial tetrahedron took at least one attempt
        assert (c < 1.0).sum() == 4 and c.mean() > 1.0
        model = dtlib.dt_train_model(tri.ctx, f, c, b, epochs=4, seed=3)
    xyz = mix_small(62, 7000)
    # without a model the learned scheduler falls back to the plain order
    with dtlib.Triangulation(scheduler=dtlib.DT_SCHED_LEARNED) as tri:
        tri.insert(xyz)
        assert tri.stats()["sched_fallbacks"] == 1
        t, _ = tri.tets()
        assert_parity(oracle_mod, xyz, t.astype(np.int64), "learned scheduler without a model")
    with dtlib.Triangulation(scheduler=dtlib.DT_SCHED_LEARNED) as tri:
        dtlib.dt_load_model(tri.ctx, model)
        tri.insert(xyz)
        t, nb = tri.tets()
        assert_parity(oracle_mod, xyz, t.astype(np.int64), "learned scheduler")
        check_invariants(xyz, t.astype(np.int64), nb, oracle_mod, expect_vertices=None)


@pytest.mark.parametrize("timing", [0, 1, 2])
def test_timing_modes(dtlib, oracle_mod, timing):
    """Timing 1 times both insertion kernels of every round, 2 the cavity kernel of rounds of
    at least 32768 candidates (none at this size), 0 neither; the result is the same."""
    say(f"timing {timing}")
    xyz = uniform_points(30000, 41)
    with dtlib.Triangulation(timing=timing) as tri:
        tri.insert(xyz)
        t, _ = tri.tets()
        st = tri.stats()
    assert_parity(oracle_mod, xyz, t.astype(np.int64), f"timing {timing}")
    if timing == 1:
        assert 0 < st["cavity_launches"] <= st["rounds"] and st["ms_cavity_kernel"] > 0
        assert st["ball_launches"] == st["cavity_launches"] and st["ms_ball_kernel"] > 0
        assert st["timed_insertions"] == st["inserted"] and st["timed_attempts"] == st["attempts"]
    else:
        assert st["cavity_launches"] == 0 and st["ball_launches"] == 0 and st["timed_insertions"] == 0


def test_timing_large_rounds(dtlib):
    """Timing 2 on 2e6 points times the rounds of at least 32768 candidates: some but not all
    rounds, the counts of their insertions and attempts; the output equals an untimed run's."""
    from canon import canonical_hash
    say("timing 2 on 2e6 points")
    xyz = uniform_points(2_000_000, 43)
    out = {}
    for timing in (0, 2):
        with dtlib.Triangulation(timing=timing) as tri:
            tri.insert(xyz)
            t, _ = tri.tets()
            out[timing] = (canonical_hash(t), tri.stats())
    assert out[0][0] == out[2][0]
    st = out[2][1]
    assert 0 < st["cavity_launches"] < st["rounds"] and st["ms_cavity_kernel"] > 0 and st["ball_launches"] == 0
    assert 0 < st["timed_insertions"] < st["inserted"] and st["timed_insertions"] <= st["timed_attempts"]


@pytest.mark.parametrize("case", ["mix", "lanes16", "wide", "grown", "batch", "large"])
def test_graph_rounds_keep_result(dtlib, oracle_mod, case):
    """Regular rounds launched as one HIP graph each (dt_options.graph_rounds) give the
    oracle's result: with drains of overflowed candidates between graph rounds (small cavity
    cap), with 16 lanes, on a pool of 64-bit codes, across pool growth, for a batch of clouds,
    and on 2e6 points (graphs of both lane counts, compared with the separate launches)."""
    from canon import canonical_hash
    say(f"graph rounds: {case}")
    if case == "batch":
        xyz, off = batch_clouds(24, seed_base=7300, nmin=4, nmax=3000)
        with dtlib.Triangulation(graph_rounds=True) as tri:
            tri.insert_batch(xyz, off)
            assert tri.stats()["graph_rounds"] > 0
            for k in range(0, 24, 3):
                t, _ = tri.tets_batch(k)
                assert_parity(oracle_mod, xyz[off[k]:off[k + 1]], t.astype(np.int64), f"cloud {k}")
        return
    if case == "large":
        xyz = uniform_points(2_000_000, 47)
        out = {}
        for graph in (False, True):
            with dtlib.Triangulation(graph_rounds=graph) as tri:
                tri.insert(xyz)
                t, _ = tri.tets()
                out[graph] = (canonical_hash(t), tri.stats())
        assert out[True][0] == out[False][0]
        assert out[True][1]["graph_rounds"] > 0 and out[False][1]["graph_rounds"] == 0
        return
    opts = {"mix": dict(cavity_cap=12), "lanes16": dict(lanes_per_insert=16), "wide": dict(index_bits=64),
            "grown": dict(capacity_tets=4096)}[case]
    xyz = mix_small(53, 4000) if case in ("mix", "grown") else uniform_points(60000, 59)
    tets, nbrs, st = gpu_dt(dtlib, xyz, graph_rounds=True, **opts)
    assert_parity(oracle_mod, xyz, tets, case)
    assert 0 < st["graph_rounds"] <= st["rounds"]
    if case == "mix":
        assert st["overflows"] > 0
    if case == "grown":
        assert len(tets) > 4 * 4096
