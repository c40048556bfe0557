"""Oracle for Delaunay refinement by circumcentre insertion (paper, Sec. 4: points at the
circumcentres of tetrahedra whose circumradius r exceeds 1.4 h, filtered so that no edge
shorter than 0.7 h is created, inserted in large sets).

TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls it.  Plain numpy on top of
the serial triangulation of this package; slow and meant for small clouds.

Readings (the paper gives the rule, not these details):

* Domain: the convex hull of the input cloud (no boundary recovery).  A circumcentre is a
  candidate only if it lies strictly inside the hull: exact orient3d > 0 against every hull
  facet, the facet ordered with its tetrahedron's fourth vertex on the positive side.
  Inserted points are strictly inside, so the hull facets never change.
* Size: one constant h.  A tetrahedron is refined when r^2 > (1.4 h)^2, with the
  circumcentre and r^2 evaluated in fp64 by the fixed formula of `circumcentres`, which takes
  the four vertices in ascending input index (so the rounded values depend on the
  tetrahedron only, not on how a triangulation stores it).
* Filter: the candidates of a step are taken in the order of their Moore key (the input
  cloud's grid) and then of their tetrahedron's sorted vertex indices.  A candidate is kept
  iff its squared distance (fp64, fixed formula) to every current vertex and to every
  candidate kept before it in this step is at least (0.7 h)^2.  This stands for the paper's
  discarding of close points along the curve plus the cavity that aborts when one of its
  vertices is too close: the nearest vertex of a new point is adjacent to it in the new
  triangulation, so it is a vertex of the cavity, and the abort is the nearest-vertex test.
* Steps: triangulate the current points, collect and filter the candidates, append the kept
  ones (in filter order, so their input indices follow it); stop after a step that keeps
  none.  The result is the Delaunay tetrahedralization of the final point set.
"""
from __future__ import annotations

import numpy as np

from . import canonical, delaunay, moore_keys, moore_level, orient3d

GROW, FILTER = 1.4, 0.7


def circumcentres(xyz: np.ndarray, tets: np.ndarray):
    """fp64 circumcentre c and squared radius |c - a|^2 of each tetrahedron, its vertices
    (a, b, c, d) in ascending input index: with u = b - a, v = c - a, w = d - a,
    c - a = (|u|^2 (v x w) + |v|^2 (w x u) + |w|^2 (u x v)) / (2 u . (v x w)),
    evaluated left to right as written, no fused operations."""
    p = np.asarray(xyz, dtype=np.float64)[np.sort(np.asarray(tets, dtype=np.int64), axis=1)]
    a = p[:, 0]
    u, v, w = p[:, 1] - a, p[:, 2] - a, p[:, 3] - a

    def cross(x, y):
        return np.stack([x[:, 1] * y[:, 2] - x[:, 2] * y[:, 1],
                         x[:, 2] * y[:, 0] - x[:, 0] * y[:, 2],
                         x[:, 0] * y[:, 1] - x[:, 1] * y[:, 0]], axis=1)

    def dot(x, y):
        return x[:, 0] * y[:, 0] + x[:, 1] * y[:, 1] + x[:, 2] * y[:, 2]

    vw, wu, uv = cross(v, w), cross(w, u), cross(u, v)
    den = 2.0 * dot(u, vw)
    num = dot(u, u)[:, None] * vw + dot(v, v)[:, None] * wu + dot(w, w)[:, None] * uv
    off = num / den[:, None]
    return a + off, dot(off, off)


def sq_dist(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Squared distance, (dx dx + dy dy) + dz dz in fp64."""
    d = np.asarray(x, dtype=np.float64) - np.asarray(y, dtype=np.float64)
    return d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1] + d[..., 2] * d[..., 2]


def hull_facets(xyz, tets, nbrs):
    """Facets without neighbour, ordered so that the fourth vertex of the tetrahedron is on
    the positive side (exact orient3d)."""
    tets = np.asarray(tets, dtype=np.int64)
    t_idx, j_idx = np.nonzero(np.asarray(nbrs) < 0)
    rest = np.array([[k for k in range(4) if k != j] for j in range(4)])
    f = tets[t_idx[:, None], rest[j_idx]].copy()
    s = orient3d(np.asarray(xyz)[np.concatenate([f, tets[t_idx, j_idx][:, None]], axis=1)])
    f[s < 0] = f[s < 0][:, [0, 2, 1]]
    return f


def strictly_inside(q, xyz, facets, quads_per_batch=1 << 19):
    """Exact test: q is on the positive side of every oriented hull facet."""
    q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
    P = np.asarray(xyz, dtype=np.float64)[facets]  # H, 3, 3
    out = np.ones(len(q), dtype=bool)
    chunk = max(1, quads_per_batch // max(len(P), 1))
    for s in range(0, len(q), chunk):
        qq = q[s:s + chunk]
        quad = np.concatenate([np.broadcast_to(P[None], (len(qq),) + P.shape),
                               np.broadcast_to(qq[:, None, None, :], (len(qq), len(P), 1, 3))], axis=2)
        sign = orient3d(quad.reshape(-1, 4, 3)).reshape(len(qq), len(P))
        out[s:s + chunk] = np.all(sign > 0, axis=1)
    return out


def greedy_filter(cand, order, vertices, h):
    """Indices (into cand) kept by the filter, in filter order."""
    from scipy.spatial import cKDTree
    lim = (FILTER * h) * (FILTER * h)
    reach = FILTER * h * (1.0 + 1e-6)
    tree = cKDTree(vertices)
    near_v = tree.query_ball_point(cand[order], reach)
    # grid cells a little wider than the threshold, so that two candidates closer than it
    # always fall in neighbouring cells despite the rounding of c / cell
    cell = FILTER * h * (1.0 + 1e-9)
    grid = {}
    kept = []
    for k, i in enumerate(order):
        c = cand[i]
        if near_v[k] and np.any(sq_dist(vertices[near_v[k]], c) < lim):
            continue
        g = tuple(np.floor(c / cell).astype(np.int64))
        close = False
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    for j in grid.get((g[0] + dx, g[1] + dy, g[2] + dz), ()):
                        if sq_dist(cand[j], c) < lim:
                            close = True
                            break
                    if close:
                        break
                if close:
                    break
            if close:
                break
        if close:
            continue
        grid.setdefault(g, []).append(i)
        kept.append(i)
    return np.array(kept, dtype=np.int64)


def refine(xyz: np.ndarray, h: float, max_steps: int = 100):
    """Returns (points, tets, nbrs, steps): the final point set (the input first, then the
    inserted points in insertion order), its Delaunay tetrahedralization and, per step,
    (candidates, kept)."""
    pts = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    n0 = len(pts)
    m = moore_level(n0)
    grow = (GROW * h) * (GROW * h)
    rc, tets, nbrs, _ = delaunay(pts)
    if rc != 0:
        raise ValueError(f"input not triangulable (code {rc})")
    facets = hull_facets(pts, tets, nbrs)
    steps = []
    for _ in range(max_steps):
        cc, r2 = circumcentres(pts, tets)
        bad = np.nonzero(r2 > grow)[0]
        inside = strictly_inside(cc[bad], pts, facets) if len(bad) else np.zeros(0, dtype=bool)
        cand_t = bad[inside]
        cand = cc[cand_t]
        if len(cand) == 0:
            steps.append((0, 0))
            break
        # Moore keys in the input cloud's grid: the candidates lie in its box
        keys = moore_keys(np.vstack([pts[:n0], cand]), m)[n0:]
        q = np.sort(np.asarray(tets, dtype=np.int64)[cand_t], axis=1)
        order = np.lexsort((q[:, 3], q[:, 2], q[:, 1], q[:, 0], keys))
        kept = greedy_filter(cand, order, pts, h)
        steps.append((len(cand), len(kept)))
        if len(kept) == 0:
            break
        pts = np.vstack([pts, cand[kept]])
        rc, tets, nbrs, _ = delaunay(pts)
        if rc != 0:
            raise RuntimeError(f"triangulation failed during refinement (code {rc})")
    return pts, tets, nbrs, steps


__all__ = ["circumcentres", "sq_dist", "hull_facets", "strictly_inside", "greedy_filter", "refine",
           "canonical"]
