"""Pins for the refinement oracle (CPU): the circumcentre against exact rational arithmetic,
the hull test against scipy's Delaunay, the greedy filter against brute force, a closed form
on the cube, and the final-state properties the rule implies."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

from synth import cluster_points, shell_points, uniform_points
from validators import check_invariants


@pytest.fixture(scope="module")
def R(oracle_mod):
    from oracle import refine
    return refine


def _exact_circumcentre(q):
    """Solve 2 (p_i - a) . x = |p_i|^2 - |a|^2 (i = b, c, d) in rationals (Cramer)."""
    F = [[Fraction(float(v)) for v in r] for r in q]
    a = F[0]
    M = [[2 * (F[i][k] - a[k]) for k in range(3)] for i in (1, 2, 3)]
    rhs = [sum(F[i][k] * F[i][k] - a[k] * a[k] for k in range(3)) for i in (1, 2, 3)]

    def det(m):
        return (m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0])
                + m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]))
    D = det(M)
    out = []
    for k in range(3):
        Mk = [row[:] for row in M]
        for i in range(3):
            Mk[i][k] = rhs[i]
        out.append(det(Mk) / D)
    return out


def test_circumcentre_matches_exact_rationals(R, oracle_mod):
    xyz = uniform_points(400, 5)
    rc, tets, _, _ = oracle_mod.delaunay(xyz)
    assert rc == 0
    pick = tets[np.random.default_rng(1).choice(len(tets), 150, replace=False)]
    cc, r2 = R.circumcentres(xyz, pick)
    for q, c, rr in zip(pick, cc, r2):
        ex = _exact_circumcentre(xyz[q])
        scale = max(1.0, max(abs(float(v)) for v in ex))
        assert max(abs(c[k] - float(ex[k])) for k in range(3)) <= 1e-9 * scale
        d2 = [sum((float(ex[k]) - xyz[v][k]) ** 2 for k in range(3)) for v in q]
        assert abs(rr - d2[0]) <= 1e-8 * d2[0]
        assert max(d2) - min(d2) <= 1e-9 * max(d2)  # the exact centre is equidistant


def test_strictly_inside_matches_scipy(R, oracle_mod):
    from scipy.spatial import Delaunay
    xyz = uniform_points(300, 6)
    rc, tets, nbrs, _ = oracle_mod.delaunay(xyz)
    f = R.hull_facets(xyz, tets, nbrs)
    q = np.random.default_rng(2).random((4000, 3)) * 1.2 - 0.1
    got = R.strictly_inside(q, xyz, f)
    ref = Delaunay(xyz).find_simplex(q) >= 0
    # away from the hull surface the two agree exactly; count both sides
    from scipy.spatial import ConvexHull
    eq = ConvexHull(xyz).equations
    margin = np.min(np.abs(q @ eq[:, :3].T + eq[:, 3]), axis=1) > 1e-9
    assert np.array_equal(got[margin], ref[margin])
    assert got.sum() > 1000 and (~got).sum() > 1000
    # points on the hull (its vertices) are not strictly inside
    assert not R.strictly_inside(xyz[np.unique(f)], xyz, f).any()


def test_greedy_filter_matches_brute_force(R):
    r = np.random.default_rng(3)
    h = 0.1
    verts = r.random((60, 3))
    cand = r.random((400, 3))
    order = r.permutation(400)
    got = R.greedy_filter(cand, order, verts, h)
    lim = (0.7 * h) * (0.7 * h)
    kept = []
    for i in order:
        if min(R.sq_dist(verts, cand[i])) < lim:
            continue
        if any(R.sq_dist(cand[j], cand[i]) < lim for j in kept):
            continue
        kept.append(i)
    assert list(got) == kept
    assert 20 < len(kept) < 400


@pytest.mark.parametrize("h,inserted", [(0.5, 1), (0.6, 1), (0.7, 0)])
def test_cube_closed_form(R, h, inserted):
    """Unit cube corners: every Delaunay tetrahedron has circumradius sqrt(3)/2 and centre
    (1/2, 1/2, 1/2).  For h = 0.5 and 0.6 (r / h > 1.4) the centre is inserted once; the new
    tetrahedra (centre + half a face) have their circumcentres outside the cube, so refinement
    stops with 9 points and 12 tetrahedra.  For h = 0.7 (r / h = 1.237) nothing is inserted."""
    cube = np.array(list(itertools.product([0.0, 1.0], repeat=3)))
    pts, tets, nbrs, steps = R.refine(cube, h)
    assert len(pts) == 8 + inserted
    if inserted:
        assert np.array_equal(pts[8], [0.5, 0.5, 0.5])
        assert len(tets) == 12 and steps[0][1] == 1 and steps[-1] == (0, 0)
    else:
        assert steps == [(0, 0)]


def test_lattice_closed_form(R, oracle_mod):
    """5 x 5 x 5 lattice, spacing 1/4 (co-spherical everywhere).  Each of the 64 cells has
    circumradius sqrt(3)/8 = 0.2165.  h = 0.2 (r / h = 1.08) inserts nothing.  h = 0.12
    (r / h = 1.80) proposes the centre of every cell six times (once per tetrahedron of the
    cell) and keeps it once: centres are 1/4 apart and sqrt(3)/8 from the corners, both above
    0.7 h.  The lattice plus the centres is body-centred cubic, whose Delaunay tetrahedra have
    circumradius sqrt(5)/16 = 0.1398 (r / h = 1.16); the tetrahedra on a hull face have their
    circumcentres outside the hull.  So refinement stops with exactly the 64 centres added."""
    lat = np.array(list(itertools.product(np.arange(5.0) / 4, repeat=3)))
    pts, tets, nbrs, steps = R.refine(lat, 0.2)
    assert len(pts) == 125 and steps == [(0, 0)]
    pts, tets, nbrs, steps = R.refine(lat, 0.12)
    assert steps == [(384, 64), (0, 0)]
    centres = np.array(list(itertools.product((np.arange(4.0) + 0.5) / 4, repeat=3)))
    got = pts[125:]
    assert len(got) == 64
    assert np.array_equal(got[np.lexsort(got.T[::-1])], centres[np.lexsort(centres.T[::-1])])
    check_invariants(pts, tets, nbrs, oracle_mod, expect_vertices=np.arange(len(pts)))


@pytest.mark.parametrize("kind,h", [("uniform", 0.08), ("uniform", 0.05), ("clusters", 0.03), ("shell", 0.15)])
def test_refined_mesh_properties(R, oracle_mod, kind, h):
    """What the rule fixes at the end: the result is the Delaunay tetrahedralization of its
    points (I1-I7); no inserted point is closer than 0.7 h to another vertex; every
    tetrahedron still larger than 1.4 h with its circumcentre strictly inside the hull has a
    vertex closer than 0.7 h to that circumcentre (so the filter alone stopped it)."""
    from scipy.spatial import cKDTree
    xyz = (uniform_points(600, 7) if kind == "uniform" else shell_points(300, 21) if kind == "shell"
           else cluster_points(800, 8, clusters=4))
    pts, tets, nbrs, steps = R.refine(xyz, h)
    n0 = len(xyz)
    assert len(pts) > n0 + 50 and steps[-1][1] == 0
    check_invariants(pts, tets, nbrs, oracle_mod, expect_vertices=np.arange(len(pts)))
    tree = cKDTree(pts)
    d, _ = tree.query(pts[n0:], k=2)
    assert np.all(d[:, 1] >= 0.7 * h * (1 - 1e-12))
    cc, r2 = R.circumcentres(pts, tets)
    big = r2 > (1.4 * h) ** 2
    f = R.hull_facets(pts, tets, nbrs)
    big &= R.strictly_inside(cc, pts, f) if big.any() else big
    if big.any():
        dn, _ = tree.query(cc[big])
        assert np.all(dn < 0.7 * h * (1 + 1e-12))
    # the hull is the input's: inserted points are strictly inside it
    f0 = R.hull_facets(xyz, *oracle_mod.delaunay(xyz)[1:3])
    assert R.strictly_inside(pts[n0:], xyz, f0).all()


def test_refine_matches_stored_results(R):
    """Regression: the oracle reproduces tests/golden/refine_golden.txt, which
    tests/golden/make_refine_golden.py wrote from this oracle.  A change to the oracle's
    arithmetic must come with a rewritten file and the passage that justifies it."""
    import os
    import sys
    here = os.path.dirname(os.path.abspath(__file__))
    sys.path.insert(0, os.path.join(here, "golden"))
    import make_refine_golden as mk
    rows = [l.split("|") for l in open(os.path.join(here, "golden", "refine_golden.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == len(mk.CASES)
    for (lhs, rhs), case in zip(rows, mk.CASES):
        kind, n, seed, h = lhs.split()
        assert (kind, int(n), int(seed), float(h)) == case
        npts, steps, ht, hp = rhs.split()
        assert mk.run_case(*case) == (int(npts), steps, ht, hp)


def _filter_in_rounds(R, cand, order, vertices, h):
    """The filter as parallel rounds (the form a GPU would run): drop candidates too close to a
    vertex; then, each round, every undecided candidate whose lower-ranked conflicting
    candidates are all decided is kept iff none of them was kept.  Returns (kept in rank
    order, rounds)."""
    from scipy.spatial import cKDTree
    lim = (0.7 * h) * (0.7 * h)
    rank = np.empty(len(cand), dtype=np.int64)
    rank[order] = np.arange(len(order))
    near = cKDTree(vertices).query_ball_point(cand, 0.7 * h * 1.000001)
    alive = np.array([not (nb and np.any(R.sq_dist(vertices[nb], cand[i]) < lim)) for i, nb in enumerate(near)])
    tree = cKDTree(cand)
    lower = []
    for i in range(len(cand)):
        nb = [j for j in tree.query_ball_point(cand[i], 0.7 * h * 1.000001)
              if j != i and alive[j] and rank[j] < rank[i] and R.sq_dist(cand[j], cand[i]) < lim]
        lower.append(nb)
    state = np.where(alive, 0, -1)  # 0 undecided, 1 kept, -1 dropped
    rounds = 0
    while np.any(state == 0):
        rounds += 1
        ready = [i for i in np.nonzero(state == 0)[0] if all(state[j] != 0 for j in lower[i])]
        new = {i: (1 if all(state[j] != 1 for j in lower[i]) else -1) for i in ready}
        for i, v in new.items():
            state[i] = v
    kept = [i for i in order if state[i] == 1]
    return kept, rounds


def test_filter_rounds_equal_greedy(R, oracle_mod):
    """The parallel-round form of the filter keeps exactly the greedy filter's candidates, for
    random ranks and for the Moore-curve ranks the oracle uses; a few rounds suffice."""
    r = np.random.default_rng(5)
    for h, k, moore in [(0.1, 600, False), (0.05, 3000, False), (0.05, 3000, True)]:
        verts = r.random((200, 3))
        cand = r.random((k, 3))
        if moore:
            order = np.argsort(oracle_mod.moore_keys(cand, oracle_mod.moore_level(k)), kind="stable")
        else:
            order = r.permutation(k)
        kept, rounds = _filter_in_rounds(R, cand, order, verts, h)
        assert kept == list(R.greedy_filter(cand, order, verts, h))
        assert 1 <= rounds < 20
