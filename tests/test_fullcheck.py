"""CPU tests of the whole-output checker (fullcheck.c) used at the benchmark's full sizes: it
accepts the oracle's outputs, and rejects broken ones and valid triangulations that are not
the perturbed Delaunay tetrahedralization."""
import itertools

import numpy as np
import pytest

import fullcheck
from synth import lattice_points, mix_points, uniform_points


@pytest.fixture(scope="module")
def fc():
    fullcheck.build()
    return fullcheck


@pytest.mark.parametrize("kind", ["uniform", "lattice", "mix"])
def test_accepts_oracle_outputs(fc, oracle_mod, kind):
    xyz = {"uniform": lambda: uniform_points(30000, 3), "lattice": lambda: lattice_points(3000, 4, side=16),
           "mix": lambda: mix_points(5, 8000, 6000, 6000)}[kind]()
    rc, t, nb, _ = oracle_mod.delaunay(xyz)
    assert rc == 0
    T, interior, hull = fc.check_all_facets(xyz, t, nb)
    assert T == len(t) and 2 * interior + hull == 4 * T
    assert fc.check_hull_and_vertices(xyz, t, nb, oracle_mod, n_expect=len(xyz)) == hull


def test_rejects_broken_outputs(fc, oracle_mod):
    xyz = uniform_points(5000, 6)
    rc, t, nb, _ = oracle_mod.delaunay(xyz)
    k = len(t) // 2
    j = int(np.nonzero(nb[k] >= 0)[0][0])
    broken = []
    a = t.copy(); a[k, [0, 1]] = a[k, [1, 0]]; broken.append((a, nb))          # orientation
    b = nb.copy(); b[k, j] = (b[k, j] + 1) % len(t); broken.append((t, b))      # wrong link
    c = t.copy(); c[k, 0] = len(xyz); broken.append((c, nb))                    # index range
    d = nb.copy(); d[k, j] = -1; broken.append((t, d))                         # half link
    for tt, nn in broken:
        with pytest.raises(AssertionError):
            fc.check_all_facets(xyz, tt, nn)


def test_rejects_a_valid_triangulation_that_is_not_the_perturbed_one(fc, oracle_mod):
    """The eight cube corners are cospherical: each index order has its own perturbed
    Delaunay tetrahedralization.  The oracle's output for one order, read with the points
    numbered in another order, is still a valid triangulation; where the two results differ
    the checker must find a facet that is not locally Delaunay (I7)."""
    cube = np.array(list(itertools.product([0.0, 1.0], repeat=3)))
    rng = np.random.default_rng(0)
    rejected = 0
    for _ in range(12):
        p, q = rng.permutation(8), rng.permutation(8)
        _, tp, nbp, _ = oracle_mod.delaunay(cube[p])
        _, tq, _, _ = oracle_mod.delaunay(cube[q])
        # tp in the numbering of q: point p[i] of the cube is index i in order p
        inv_q = np.argsort(q)
        relabeled = inv_q[p[tp]]
        same = np.array_equal(oracle_mod.canonical(relabeled), oracle_mod.canonical(tq))
        if same:
            fc.check_all_facets(cube[q], relabeled, nbp)
        else:
            with pytest.raises(AssertionError, match="I7"):
                fc.check_all_facets(cube[q], relabeled, nbp)
            rejected += 1
    assert rejected >= 3
