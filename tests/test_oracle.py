"""Pins for the oracle (CPU only): exact rational arithmetic, the eps-polynomial of the
symbolic perturbation, brute force on tiny inputs, invariants, order independence, and
the Moore-curve / BRIO definitions."""
import itertools
import os
from fractions import Fraction

import numpy as np
import pytest

from synth import cluster_points, lattice_points, shell_points, uniform_points
from validators import (brute_force_dt, check_adjacency, check_hull_convex, check_invariants,
                        check_volume_exact, det_exact, euler_counts, insphere_exact,
                        insphere_perturbed_poly, lifted_rows, orient3d_exact,
                        perturbed_sign_int, _int_scale)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
rng = np.random.default_rng(12345)


def sphere50_points():
    """All integer points with x^2 + y^2 + z^2 = 50 (84 cospherical points)."""
    pts = []
    for x in range(-8, 8):
        for y in range(-8, 8):
            for z in range(-8, 8):
                if x * x + y * y + z * z == 50:
                    pts.append((x, y, z))
    return np.array(pts, dtype=np.float64)


def nudge(x, k):
    return np.nextafter(x, np.inf) if k > 0 else (np.nextafter(x, -np.inf) if k < 0 else x)


# ------------------------------------------------------------------ orient3d / insphere

def test_orient3d_matches_rational(oracle_mod):
    cases = [uniform_points(4, s) for s in range(200)]
    # near-degenerate: 4th point on the plane of the first three, nudged by an ulp
    for s in range(150):
        p = uniform_points(3, 500 + s)
        u, v = rng.random(2)
        q = p[0] + u * (p[1] - p[0]) + v * (p[2] - p[0])
        q = np.array([nudge(q[0], int(rng.integers(-1, 2))), q[1], nudge(q[2], int(rng.integers(-1, 2)))])
        cases.append(np.vstack([p, q]))
    # exactly degenerate: lattice quadruples
    lat = lattice_points(100, 7, side=5)
    for _ in range(150):
        cases.append(lat[rng.choice(len(lat), 4, replace=False)])
    pts = np.array(cases)
    got = oracle_mod.orient3d(pts)
    want = np.array([orient3d_exact(*c) for c in cases])
    assert np.array_equal(got, want)
    assert np.count_nonzero(want == 0) > 10


def test_insphere_matches_rational(oracle_mod):
    cases = [uniform_points(5, 1000 + s) for s in range(150)]
    sph = sphere50_points() / 8.0
    for _ in range(150):  # cospherical, some nudged by an ulp
        c = sph[rng.choice(len(sph), 5, replace=False)].copy()
        k = int(rng.integers(-1, 2))
        j = int(np.flatnonzero(c[4])[0])  # nudge a non-zero coordinate (stay in range)
        c[4, j] = nudge(c[4, j], k)
        cases.append(c)
    lat = lattice_points(60, 9, side=4)
    for _ in range(100):
        cases.append(lat[rng.choice(len(lat), 5, replace=False)])
    pts = np.array(cases)
    got = oracle_mod.insphere(pts)
    want = np.array([insphere_exact(c) for c in cases])
    assert np.array_equal(got, want)
    assert np.count_nonzero(want == 0) > 20


# ------------------------------------------------------------------ the accepted domain's edges
# Coordinates are 0 or have magnitude in [2^-120, 2^120).  The exact stage turns every
# coordinate into an integer multiple of 2^-(120 + 52), so one determinant can hold terms
# 2^239 apart; these cases put such extremes into one call, with exact zeros and one-ulp
# nudges, and compare with rational arithmetic.

_WIDE_RNG = np.random.default_rng(2024)


def _wide(shape, lo=-120, hi=119):
    """Coordinates sign * (1 + u) * 2^e, e uniform in [lo, hi] (inside the accepted domain)."""
    m = 1.0 + _WIDE_RNG.random(shape)
    e = _WIDE_RNG.integers(lo, hi + 1, size=shape)
    sgn = np.where(_WIDE_RNG.random(shape) < 0.5, -1.0, 1.0)
    out = np.ldexp(sgn * m, e)
    return np.where(np.abs(out) >= 2.0 ** 120, np.ldexp(sgn * 1.5, 119), out)


def _scaled(points, k):
    return np.ldexp(np.asarray(points, dtype=np.float64), k)


def _wide_orient_cases():
    cases = [_wide((4, 3)) for _ in range(120)]
    # the extremes only: every coordinate is +-2^-120, +-2^119 or 0
    ext = np.array([2.0 ** -120, -2.0 ** -120, 2.0 ** 119, -2.0 ** 119, 0.0])
    cases += [ext[_WIDE_RNG.integers(0, 5, size=(4, 3))] for _ in range(80)]
    # coplanar: equal z (any x, y spread) -> exactly 0; one z nudged by an ulp -> tiny
    for t in range(120):
        c = _wide((4, 3))
        c[:, 2] = c[0, 2]
        if t % 2:
            k = int(_WIDE_RNG.integers(0, 4))
            c[k, 2] = nudge(c[k, 2], 1 if t % 4 == 1 else -1)
        cases.append(c)
    # a small plane far from the origin: lattice quadruples scaled by 2^-110 and 2^100
    lat = lattice_points(100, 7, side=5)
    for t in range(80):
        q = lat[_WIDE_RNG.choice(len(lat), 4, replace=False)]
        q = _scaled(q, -110 if t % 2 else 100)
        if t % 3 == 0:
            q[3, 0] = nudge(q[3, 0], 1) if q[3, 0] != 0 else 2.0 ** -120
        cases.append(q)
    return np.array(cases)


def test_orient3d_matches_rational_at_the_domain_edges(oracle_mod):
    pts = _wide_orient_cases()
    assert np.all((pts == 0) | ((np.abs(pts) >= 2.0 ** -120) & (np.abs(pts) < 2.0 ** 120)))
    got = oracle_mod.orient3d(pts)
    want = np.array([orient3d_exact(*c) for c in pts])
    assert np.array_equal(got, want)
    assert np.count_nonzero(want == 0) > 40 and np.count_nonzero(want != 0) > 200


def _wide_insphere_cases():
    cases = [_wide((5, 3)) for _ in range(100)]
    ext = np.array([2.0 ** -120, -2.0 ** -120, 2.0 ** 119, -2.0 ** 119, 0.0])
    cases += [ext[_WIDE_RNG.integers(0, 5, size=(5, 3))] for _ in range(60)]
    sph = sphere50_points() / 8.0
    for t in range(160):
        # cospherical at scales 2^-115 .. 2^115 (exact), some nudged by an ulp
        k = int(_WIDE_RNG.integers(-115, 116))
        c = _scaled(sph[_WIDE_RNG.choice(len(sph), 5, replace=False)], k)
        if t % 2:
            j = int(np.flatnonzero(c[4])[0])
            c[4, j] = nudge(c[4, j], 1 if t % 4 == 1 else -1)
        cases.append(c)
    for t in range(60):
        # a tiny sphere next to a huge coordinate: the sum rounds, the rational reference
        # takes the doubles as they are
        c = _scaled(sph[_WIDE_RNG.choice(len(sph), 5, replace=False)], -100)
        c[:, 0] += 2.0 ** int(_WIDE_RNG.integers(-60, 110))
        cases.append(c)
    return np.array(cases)


def test_insphere_matches_rational_at_the_domain_edges(oracle_mod):
    pts = _wide_insphere_cases()
    assert np.all((pts == 0) | ((np.abs(pts) >= 2.0 ** -120) & (np.abs(pts) < 2.0 ** 120)))
    got = oracle_mod.insphere(pts)
    want = np.array([insphere_exact(c) for c in pts])
    assert np.array_equal(got, want)
    assert np.count_nonzero(want == 0) > 60 and np.count_nonzero(want != 0) > 150


def test_perturbed_insphere_matches_eps_polynomial_at_the_domain_edges(oracle_mod):
    """The perturbation cascade on degenerate sets scaled to the domain's edges and on
    mixed-magnitude points, against the eps-polynomial."""
    sph = sphere50_points() / 8.0
    cube = np.array(list(itertools.product([0.0, 1.0], repeat=3)))
    lat = lattice_points(64, 3, side=4)
    pts, idxs = [], []
    trial = 0
    while len(pts) < 150:
        src = [sph, cube, lat][trial % 3]
        k = [-117, 116, int(_WIDE_RNG.integers(-110, 110))][trial % 3]
        trial += 1
        c = _scaled(src[_WIDE_RNG.choice(len(src), 5, replace=False)], k)
        if trial % 5 == 0:
            c[4] = _wide((3,))  # a fifth point of any magnitude
        if orient3d_exact(*c[:4]) == 0:
            continue
        c[:4] = _positive(c[:4])
        pts.append(c)
        idxs.append(_WIDE_RNG.permutation(1000)[:5])
    pts, idxs = np.array(pts), np.array(idxs)
    got = oracle_mod.insphere_sos(pts, idxs)
    want = np.array([insphere_perturbed_poly(p, i) for p, i in zip(pts, idxs)])
    assert np.all(want != 0)
    assert np.array_equal(got, want)
    raw = np.array([insphere_exact(p) for p in pts])
    assert np.count_nonzero(raw == 0) > 30


def test_bruteforce_at_the_domain_edges(oracle_mod):
    """Whole triangulations at the edges of the domain: a cospherical set scaled by 2^-117,
    a lattice scaled by 2^116, and a mixed cloud (a few points of magnitude 2^100 around a
    cluster of magnitude 2^-100), each against brute force."""
    sph = sphere50_points() / 8.0
    xyz = _scaled(sph[np.random.default_rng(3).choice(len(sph), 12, replace=False)], -117)
    assert np.array_equal(_oracle_canon(oracle_mod, xyz)[0], brute_force_dt(xyz))
    xyz = _scaled(np.random.default_rng(4).permutation(
        np.array(list(itertools.product([0.0, 0.5, 1.0], repeat=3))))[:16], 116)
    canon, tets, nbrs = _oracle_canon(oracle_mod, xyz)
    assert np.array_equal(canon, brute_force_dt(xyz))
    check_invariants(xyz, tets, nbrs, oracle_mod, expect_vertices=np.arange(16))
    big = _scaled(np.array(list(itertools.product([-1.0, 1.0], repeat=3))), 100)
    small = _scaled(uniform_points(8, 91) - 0.5, -100)
    xyz = np.random.default_rng(5).permutation(np.vstack([big, small]))
    canon, tets, nbrs = _oracle_canon(oracle_mod, xyz)
    assert np.array_equal(canon, brute_force_dt(xyz))
    check_invariants(xyz, tets, nbrs, oracle_mod, expect_vertices=np.arange(16))


def test_insphere_closed_forms(oracle_mod):
    """Hand-worked determinant values (tests/golden/insphere_closed_forms.txt)."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "insphere_closed_forms.txt"))
            if l.strip() and not l.startswith("#")]
    base = [[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]]
    for ex, ey, ez, val in rows:
        e = [float(ex), float(ey), float(ez)]
        det = det_exact(lifted_rows(base + [e]))
        assert det == Fraction(val)
        got = int(oracle_mod.insphere(np.array(base + [e]))[0])
        assert got == (det > 0) - (det < 0)
    assert int(oracle_mod.orient3d(np.array(base, dtype=float))[0]) == 1


def _positive(quad):
    q = np.array(quad)
    if orient3d_exact(*q) < 0:
        q[[0, 1]] = q[[1, 0]]
    return q


def test_perturbed_insphere_matches_eps_polynomial(oracle_mod):
    """The oracle's perturbation against the eps-polynomial of the definition."""
    sph = sphere50_points() / 8.0
    cube = np.array(list(itertools.product([0.0, 1.0], repeat=3)))
    lat = lattice_points(64, 3, side=4)
    sets = [sph, cube, lat]
    pts, idxs = [], []
    for trial in range(240):
        src = sets[trial % 3]
        sel = rng.choice(len(src), 5, replace=False)
        c = src[sel].copy()
        if orient3d_exact(*c[:4]) == 0:
            continue
        c[:4] = _positive(c[:4])
        idx = rng.permutation(1000)[:5]
        pts.append(c)
        idxs.append(idx)
    pts, idxs = np.array(pts), np.array(idxs)
    got = oracle_mod.insphere_sos(pts, idxs)
    want = np.array([insphere_perturbed_poly(p, i) for p, i in zip(pts, idxs)])
    assert np.all(want != 0)
    assert np.array_equal(got, want)
    # many of these were exact zeros before the perturbation
    raw = np.array([insphere_exact(p) for p in pts])
    assert np.count_nonzero(raw == 0) > 40


def test_ghost_rule_is_intrinsic(oracle_mod):
    """Reading R4: for p coplanar with a hull facet abc, the decision falls to the perturbed
    insphere of (a, b, c, x, p) with x the finite neighbour's apex; its sign must not depend
    on x (position on the inner side, or input index).  Cube faces (p on the circumcircle of
    abc: the perturbation decides), generic points of the plane, and tilted lattice planes."""
    r = np.random.default_rng(77)
    lat = lattice_points(216, 9, side=6)
    cases = []
    sq = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], dtype=np.float64)
    for _ in range(40):
        cases.append(sq[r.permutation(4)])  # three corners of a square face and the fourth
    for _ in range(40):
        abc = np.c_[r.integers(-8, 9, size=(3, 2)) / 8.0, np.zeros(3)]
        p = np.array([r.integers(-8, 9) / 8.0, r.integers(-8, 9) / 8.0, 0.0])
        cases.append(np.vstack([abc, p]))
    while len(cases) < 200:  # coplanar lattice quadruples in tilted planes
        q = lat[r.choice(len(lat), 4, replace=False)]
        if oracle_mod.orient3d(q[None])[0] == 0:
            cases.append(q)
    checked, ties = 0, 0
    for q in cases:
        a, b, c, p = q
        if oracle_mod.orient3d(np.array([[a, b, c, p]]))[0] != 0:
            continue
        n = np.cross(b - a, c - a)
        if not np.any(n):
            continue  # collinear facet
        signs = []
        base = 100 + r.permutation(1000)[:5]  # indices of a, b, c, (x), p; only x's varies below
        srt = np.sort(base[[0, 1, 2, 4]])
        for k in range(6):
            x = a + n * (0.25 + r.random() * 3) + (b - a) * r.normal() + (c - a) * r.normal()
            abcx = np.array([a, b, c, x])  # x is on the side of (b - a) x (c - a): positive
            assert oracle_mod.orient3d(abcx[None])[0] > 0
            idx = base.copy()
            # the apex's index: before, after or between the others in the index order
            mid = (int(srt[1]) + int(srt[2])) // 2
            idx[3] = [int(srt[0]) - 1 - k, int(srt[-1]) + 1 + k,
                      mid if mid not in (srt[1], srt[2]) else int(srt[-1]) + 50 + k][k % 3]
            signs.append(oracle_mod.insphere_sos(np.vstack([abcx, p])[None], idx[None])[0])
        assert len(set(signs)) == 1 and signs[0] != 0, (q, signs)
        checked += 1
        ties += int(oracle_mod.insphere(np.vstack([abcx, p])[None])[0] == 0)
    assert checked > 150 and ties > 40  # many decided by the perturbation alone


def test_bruteforce_cofactor_sign_matches_eps_polynomial():
    """The brute-force helper's tie-break agrees with the eps-polynomial definition."""
    cube = np.array(list(itertools.product([0.0, 1.0], repeat=3)))
    P = _int_scale(cube)
    for quad in itertools.combinations(range(8), 4):
        q = list(quad)
        if orient3d_exact(*cube[q]) == 0:
            continue
        if orient3d_exact(*cube[q]) < 0:
            q[0], q[1] = q[1], q[0]
        for e in range(8):
            if e in quad:
                continue
            idx = list(rng.permutation(8))
            a = perturbed_sign_int(P, q, e, idx)
            b = insphere_perturbed_poly(cube[q + [e]], [idx[v] for v in q + [e]])
            assert a == b


# ------------------------------------------------------------------ brute force

def _oracle_canon(oracle_mod, xyz, order="brio"):
    rc, tets, nbrs, st = oracle_mod.delaunay(xyz, order=order)
    assert rc == 0
    return oracle_mod.canonical(tets), tets, nbrs


@pytest.mark.parametrize("n,seed", [(4, 1), (5, 2), (5, 3), (6, 4), (8, 5), (10, 6), (12, 7), (12, 8),
                                    (20, 60), (32, 72), (40, 80)])
def test_bruteforce_uniform(oracle_mod, n, seed):
    xyz = uniform_points(n, seed)
    canon, tets, nbrs = _oracle_canon(oracle_mod, xyz)
    assert np.array_equal(canon, brute_force_dt(xyz))


def test_bruteforce_cube_corners(oracle_mod):
    cube = np.array(list(itertools.product([0.0, 1.0], repeat=3)))
    for perm_seed in range(4):
        perm = np.random.default_rng(perm_seed).permutation(8)
        xyz = cube[perm]
        canon, tets, nbrs = _oracle_canon(oracle_mod, xyz)
        assert np.array_equal(canon, brute_force_dt(xyz))
        assert len(canon) in (5, 6)
        check_invariants(xyz, tets, nbrs, oracle_mod, expect_vertices=np.arange(8))


def test_bruteforce_cospherical(oracle_mod):
    sph = sphere50_points() / 8.0
    for s in range(3):
        xyz = sph[np.random.default_rng(40 + s).choice(len(sph), 12, replace=False)]
        canon, tets, nbrs = _oracle_canon(oracle_mod, xyz)
        assert np.array_equal(canon, brute_force_dt(xyz))


def test_bruteforce_coplanar_hull(oracle_mod):
    """3x3 grid in the plane z = 0 plus points above: coplanar and cocircular hull."""
    grid = np.array([[x, y, 0.0] for x in range(3) for y in range(3)])
    top = np.array([[0.5, 0.5, 1.0], [1.5, 1.0, 0.75], [1.0, 1.75, 1.25]])
    for s in range(3):
        xyz = np.random.default_rng(s).permutation(np.vstack([grid, top]))
        canon, tets, nbrs = _oracle_canon(oracle_mod, xyz)
        assert np.array_equal(canon, brute_force_dt(xyz))
        check_invariants(xyz, tets, nbrs, oracle_mod, expect_vertices=np.arange(len(xyz)))


def test_bruteforce_lattice_40(oracle_mod):
    """40 distinct nodes of a 4^3 lattice: co-spherical everywhere, the perturbation decides."""
    xyz = lattice_points(40, 5, side=4)
    canon, tets, nbrs = _oracle_canon(oracle_mod, xyz)
    assert np.array_equal(canon, brute_force_dt(xyz))
    check_invariants(xyz, tets, nbrs, oracle_mod, expect_vertices=np.arange(40))


def test_bruteforce_lattice_3x3x3(oracle_mod):
    xyz = np.random.default_rng(5).permutation(
        np.array(list(itertools.product([0.0, 0.5, 1.0], repeat=3))))
    canon, tets, nbrs = _oracle_canon(oracle_mod, xyz)
    assert np.array_equal(canon, brute_force_dt(xyz))
    check_invariants(xyz, tets, nbrs, oracle_mod, expect_vertices=np.arange(27))


def test_hull_convexity_check_rejects_a_concave_complex(oracle_mod):
    """The I4 check on its own: two tetrahedra glued on a facet, with the segment between
    their apexes missing that facet, form a valid closed complex (I1-I3 hold) whose hull is
    not convex; every oracle output above passes the check."""
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [2, 2, 1], [2, 2, -1]], dtype=np.float64)
    tets = np.array([[0, 1, 2, 3], [0, 1, 2, 4]])
    for t in tets:
        if oracle_mod.orient3d(xyz[t][None])[0] < 0:
            t[[1, 2]] = t[[2, 1]]
    assert np.all(oracle_mod.orient3d(xyz[tets]) > 0)
    nbrs = np.full((2, 4), -1)
    nbrs[0, list(tets[0]).index(3)] = 1
    nbrs[1, list(tets[1]).index(4)] = 0
    check_adjacency(tets, nbrs)
    V, E, F, T, Vh, Eh, Fh = euler_counts(tets, nbrs)
    assert V - E + F - T == 1 and Vh - Eh + Fh == 2
    with pytest.raises(AssertionError, match="not locally convex"):
        check_hull_convex(xyz, tets, nbrs, oracle_mod)
    # the Delaunay tetrahedralization of the same points is convex
    rc, t2, n2, _ = oracle_mod.delaunay(xyz)
    assert rc == 0 and check_hull_convex(xyz, t2, n2, oracle_mod) == 6


def test_exact_volume_check_rejects_a_folded_complex(oracle_mod):
    """The exact I6 check on its own: two positive tetrahedra glued on a facet with both apexes
    on the same side pass I1-I3, but the facet does not cancel in the divergence sum."""
    # (off the origin: a facet whose plane holds the origin adds nothing to the divergence sum)
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0.25, 0.25, 1], [0.125, 0.25, 2]], dtype=np.float64) + 0.5
    tets = np.array([[0, 1, 2, 3], [0, 1, 2, 4]])
    assert np.all(oracle_mod.orient3d(xyz[tets]) > 0)
    nbrs = np.full((2, 4), -1)
    nbrs[0, 3] = 1
    nbrs[1, 3] = 0
    check_adjacency(tets, nbrs)
    V, E, F, T, Vh, Eh, Fh = euler_counts(tets, nbrs)
    assert V - E + F - T == 1 and Vh - Eh + Fh == 2
    with pytest.raises(AssertionError, match="different volumes"):
        check_volume_exact(xyz, tets, nbrs, oracle_mod)
    rc, t2, n2, _ = oracle_mod.delaunay(xyz)
    assert rc == 0 and check_volume_exact(xyz, t2, n2, oracle_mod) > 0


# ------------------------------------------------------------------ edge cases

def test_input_domain_boundaries(oracle_mod):
    """Accepted coordinates: 0, or magnitude in [2^-120, 2^120).  The edges of the interval,
    one ulp either side, in either sign."""
    base = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [0.25, 0.25, 0.25]], dtype=np.float64)
    big, tiny = 2.0 ** 120, 2.0 ** -120
    cases = [(np.nextafter(big, 0), True), (big, False), (tiny, True), (np.nextafter(tiny, 0), False),
             (np.inf, False), (np.nan, False)]
    for v, ok in cases:
        for sign in (1.0, -1.0):
            x = base.copy()
            x[4, 1] = sign * v
            rc = oracle_mod.delaunay(x)[0]
            assert (rc == oracle_mod.OK) == ok and (ok or rc == oracle_mod.E_INPUT), (v, sign, rc)


def test_errors_and_duplicates(oracle_mod):
    assert oracle_mod.delaunay(np.zeros((3, 3)))[0] == oracle_mod.E_DEGENERATE
    plane = np.c_[uniform_points(50, 3)[:, :2], np.zeros(50)]
    assert oracle_mod.delaunay(plane)[0] == oracle_mod.E_DEGENERATE
    line = np.outer(np.arange(10.0), [1.0, 2.0, 3.0])
    assert oracle_mod.delaunay(line)[0] == oracle_mod.E_DEGENERATE
    bad = uniform_points(10, 4)
    bad[3, 1] = np.nan
    assert oracle_mod.delaunay(bad)[0] == oracle_mod.E_INPUT
    big = uniform_points(10, 4)
    big[2, 2] = 1e300
    assert oracle_mod.delaunay(big)[0] == oracle_mod.E_INPUT
    # duplicates: representative is the lowest index, result as without the copies
    xyz = uniform_points(300, 5)
    dup = np.vstack([xyz, xyz[[7, 100, 7, 299]]])
    rc, tets, nbrs, st = oracle_mod.delaunay(dup)
    assert rc == 0 and st["duplicates"] == 4
    canon_dup = oracle_mod.canonical(tets)
    canon = _oracle_canon(oracle_mod, xyz)[0]
    assert np.array_equal(canon_dup, canon)
    # a duplicate placed before its twin: the lower index wins
    dup2 = np.vstack([xyz[[5]], xyz])
    canon2 = oracle_mod.canonical(oracle_mod.delaunay(dup2)[1])
    assert 0 in canon2 and 6 not in canon2


# ------------------------------------------------------------------ order independence

def _mix_small(seed):
    return np.random.default_rng(seed).permutation(np.vstack([
        lattice_points(700, seed, side=10), cluster_points(700, seed, clusters=5),
        shell_points(700, seed)]))


@pytest.mark.parametrize("kind", ["uniform", "lattice", "mix"])
def test_order_independence(oracle_mod, kind):
    xyz = {"uniform": lambda: uniform_points(3000, 11),
           "lattice": lambda: lattice_points(300, 12, side=7),
           "mix": lambda: _mix_small(13)}[kind]()
    ref = _oracle_canon(oracle_mod, xyz, "brio")[0]
    for order in ("random", "reverse", "input"):
        assert np.array_equal(_oracle_canon(oracle_mod, xyz, order)[0], ref), order


@pytest.mark.parametrize("kind", ["uniform", "mix"])
def test_invariants(oracle_mod, kind):
    xyz = uniform_points(20000, 21) if kind == "uniform" else _mix_small(22)
    rc, tets, nbrs, st = oracle_mod.delaunay(xyz)
    assert rc == 0
    info = check_invariants(xyz, tets, nbrs, oracle_mod, expect_vertices=np.arange(len(xyz)))
    if kind == "uniform":
        # sanity, not a pin: a little more than 6 tetrahedra per point (paper Sec. 2.2)
        assert 6.0 < len(tets) / len(xyz) < 7.0
        assert st["insphere_exact"] == 0
    else:
        assert st["insphere_zero"] > 0


# ------------------------------------------------------------------ Moore curve, BRIO

@pytest.mark.parametrize("m", [1, 2, 3, 4, 5])
def test_moore_curve_closed_and_adjacent(oracle_mod, m):
    n = 1 << m
    cells = np.array(list(itertools.product(range(n), repeat=3)), dtype=np.uint32)
    keys = np.array([oracle_mod.moore_index(c, m) for c in cells], dtype=np.int64)
    assert np.array_equal(np.sort(keys), np.arange(n ** 3))
    path = cells[np.argsort(keys)].astype(np.int64)
    step = np.abs(np.diff(np.vstack([path, path[:1]]), axis=0)).sum(axis=1)
    assert np.all(step == 1)  # consecutive cells share a face, last back to first


def test_moore_level(oracle_mod):
    assert oracle_mod.moore_level(1e5) == 6
    assert oracle_mod.moore_level(1e7) == 8
    assert oracle_mod.moore_level(1e8) == 9
    assert oracle_mod.moore_level(2) == 1


@pytest.mark.parametrize("m", [2, 5])
def test_moore_keys_cells_by_construction(oracle_mod, m):
    """Points placed at the centres of known cells of a 2^m grid; two corner points fix the
    bounding box to [0, 2^m] on the long axes, so each point's cell is known without the
    quantisation formula.  The short y axis (half the extent) shares the long axes' scale."""
    g = 1 << m
    r = np.random.default_rng(m)
    cells = np.stack([r.integers(0, g, 500), r.integers(0, g // 2, 500), r.integers(0, g, 500)], axis=1)
    xyz = np.vstack([cells + 0.5, [[0.0, 0.0, 0.0], [g, g / 2, g]]])
    keys = oracle_mod.moore_keys(xyz, m)
    want = [oracle_mod.moore_index(c, m) for c in cells]
    assert np.array_equal(keys[:500], np.array(want, dtype=np.uint64))
    # the low corner is cell (0, 0, 0); the high corner sits on the grid's far faces and
    # belongs to the last cell along x and z, and to cell g/2 along y
    assert keys[500] == oracle_mod.moore_index([0, 0, 0], m)
    assert keys[501] == oracle_mod.moore_index([g - 1, g // 2, g - 1], m)


def test_stable_sort_is_numpy_stable_argsort(oracle_mod):
    """The oracle's sort is the stable sort: equal keys keep the input order."""
    r = np.random.default_rng(7)
    for n, hi in [(1, 5), (1000, 7), (50000, 1 << 40), (50000, 100)]:
        keys = r.integers(0, hi, size=n, dtype=np.uint64)
        assert np.array_equal(oracle_mod.stable_sort(keys), np.argsort(keys, kind="stable"))
    keys = np.array([2 ** 64 - 1, 0, 2 ** 63, 2 ** 63 - 1, 0], dtype=np.uint64)
    assert list(oracle_mod.stable_sort(keys)) == [1, 4, 3, 2, 0]


def test_sort_reference_is_level_major_moore_order(oracle_mod):
    """The insertion order: BRIO levels in turn (sizes as the level table gives them), each
    level along the Moore curve, ties by input index."""
    xyz = uniform_points(40000, 31)
    keys, perm, m, cum = oracle_mod.sort_reference(xyz, 5)
    assert np.array_equal(np.sort(perm), np.arange(len(xyz)))
    lev = (keys >> np.uint64(3 * m)).astype(np.int64)
    mk = keys & np.uint64((1 << (3 * m)) - 1)
    assert np.array_equal(mk, oracle_mod.moore_keys(xyz, m))
    lv, _ = oracle_mod.brio_levels(len(xyz), 5)
    assert np.array_equal(lev, lv.astype(np.int64))
    sl, sk = lev[perm], mk[perm]
    assert np.all(np.diff(sl) >= 0)
    same = sl[1:] == sl[:-1]
    assert np.all(sk[1:][same] >= sk[:-1][same])
    tie = same & (sk[1:] == sk[:-1])
    assert np.all(perm[1:][tie] > perm[:-1][tie])
    assert list(cum) == [2048, 14336, 40000]


def test_brio_rounds_match_paper_table(oracle_mod):
    lines = [l.split() for l in open(os.path.join(GOLDEN, "brio_rounds_1e6.txt"))
             if l.strip() and not l.startswith("#")]
    n = int(lines[0][1])
    want = [int(v) for v in lines[1][1:]]
    lev, cum = oracle_mod.brio_levels(n, 77)
    assert list(cum) == want
    counts = np.cumsum(np.bincount(lev, minlength=len(cum)))
    for c, w in zip(counts, want):
        assert abs(c - w) <= 6 * np.sqrt(w) + 1
    assert counts[-1] == n
