"""Independent checks of a tetrahedralization: exact rational determinants, brute force,
and the invariants that, by Delaunay's lemma, certify a triangulation as the (perturbed)
Delaunay tetrahedralization.  Test infrastructure.
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np

# ---------------------------------------------------------------- exact determinants

def det_exact(M):
    """Determinant of a square matrix of ints/Fractions by Gaussian elimination."""
    A = [[Fraction(x) for x in row] for row in M]
    n = len(A)
    det = Fraction(1)
    for c in range(n):
        piv = next((r for r in range(c, n) if A[r][c] != 0), None)
        if piv is None:
            return Fraction(0)
        if piv != c:
            A[c], A[piv] = A[piv], A[c]
            det = -det
        det *= A[c][c]
        for r in range(c + 1, n):
            f = A[r][c] / A[c][c]
            if f:
                for k in range(c, n):
                    A[r][k] -= f * A[c][k]
    return det


def frac_pt(p):
    return [Fraction(float(v)) for v in p]


def orient3d_exact(a, b, c, d) -> int:
    """sign of (b-a).((c-a)x(d-a)) in exact rational arithmetic."""
    a, b, c, d = map(frac_pt, (a, b, c, d))
    u = [b[k] - a[k] for k in range(3)]
    v = [c[k] - a[k] for k in range(3)]
    w = [d[k] - a[k] for k in range(3)]
    det = (u[0] * (v[1] * w[2] - v[2] * w[1]) - u[1] * (v[0] * w[2] - v[2] * w[0])
           + u[2] * (v[0] * w[1] - v[1] * w[0]))
    return (det > 0) - (det < 0)


def lifted_rows(pts):
    rows = []
    for p in pts:
        p = frac_pt(p)
        rows.append([p[0], p[1], p[2], p[0] ** 2 + p[1] ** 2 + p[2] ** 2, Fraction(1)])
    return rows


def insphere_exact(pts) -> int:
    """sign of the 5x5 determinant with rows (x, y, z, |p|^2, 1), rows in the given order."""
    d = det_exact(lifted_rows(pts))
    return (d > 0) - (d < 0)


# ε-polynomials: dict power -> Fraction

def _pmul(p, q):
    r = {}
    for i, a in p.items():
        for j, b in q.items():
            r[i + j] = r.get(i + j, 0) + a * b
    return r


def _padd(p, q, s=1):
    r = dict(p)
    for j, b in q.items():
        r[j] = r.get(j, 0) + s * b
    return r


def _perm_sign(perm):
    s, seen = 1, [False] * len(perm)
    for i in range(len(perm)):
        if not seen[i]:
            j, L = i, 0
            while not seen[j]:
                seen[j] = True
                j = perm[j]
                L += 1
            if L % 2 == 0:
                s = -s
    return s


def insphere_perturbed_poly(pts, idx) -> int:
    """Sign of det(rows (x, y, z, |p|^2 + eps^delta_i, 1)) as eps -> 0+, delta_i strictly
    decreasing in the input index (largest index = smallest exponent), by full Leibniz
    expansion over polynomials in eps.  Returns the sign of the lowest-order non-zero
    coefficient (0 only if the polynomial vanishes identically)."""
    order = sorted(range(5), key=lambda r: -idx[r])
    delta = {r: k + 1 for k, r in enumerate(order)}
    rows = lifted_rows(pts)
    M = [[{0: x} for x in row] for row in rows]
    for r in range(5):
        M[r][3] = {0: rows[r][3], delta[r]: Fraction(1)}
    total = {}
    for perm in itertools.permutations(range(5)):
        term = {0: Fraction(_perm_sign(perm))}
        for r in range(5):
            term = _pmul(term, M[r][perm[r]])
        total = _padd(total, term)
    for k in sorted(total):
        if total[k] != 0:
            return 1 if total[k] > 0 else -1
    return 0


# ---------------------------------------------------------------- brute force

def _int_scale(xyz):
    """Exact integer coordinates: all doubles times a common power of two."""
    xyz = np.asarray(xyz, dtype=np.float64)
    fr = [Fraction(float(v)) for v in xyz.reshape(-1)]
    den = 1
    for f in fr:
        den = max(den, f.denominator)
    return [[int(fr[3 * i + k] * den) for k in range(3)] for i in range(len(xyz))]


def _det_int(M):
    """Integer determinant by fraction-free Bareiss elimination."""
    A = [list(r) for r in M]
    n = len(A)
    sign, prev = 1, 1
    for k in range(n - 1):
        if A[k][k] == 0:
            piv = next((r for r in range(k + 1, n) if A[r][k] != 0), None)
            if piv is None:
                return 0
            A[k], A[piv] = A[piv], A[k]
            sign = -sign
        for i in range(k + 1, n):
            for j in range(k + 1, n):
                A[i][j] = (A[i][j] * A[k][k] - A[i][k] * A[k][j]) // prev
        prev = A[k][k]
    return sign * A[n - 1][n - 1]


def _lift_int(p):
    return [p[0], p[1], p[2], p[0] * p[0] + p[1] * p[1] + p[2] * p[2], 1]


def perturbed_sign_int(P, quad, e, idx):
    """Perturbed insphere sign for integer points, rows quad + [e]: the cofactors of the
    lifted column taken from the largest index down (textbook cofactor signs)."""
    rows = [_lift_int(P[v]) for v in list(quad) + [e]]
    d = _det_int(rows)
    if d != 0:
        return 1 if d > 0 else -1
    ids = [idx[v] for v in list(quad) + [e]]
    for r in sorted(range(5), key=lambda r: -ids[r]):
        minor = [[rows[i][j] for j in range(5) if j != 3] for i in range(5) if i != r]
        c = (-1) ** (r + 3) * _det_int(minor)
        if c != 0:
            return 1 if c > 0 else -1
    return 0


def brute_force_dt(xyz, idx=None):
    """All positively oriented 4-subsets whose perturbed circumsphere is empty, as sorted
    quads (rows sorted).  O(n^5): tiny inputs only."""
    n = len(xyz)
    idx = list(range(n)) if idx is None else list(idx)
    P = _int_scale(xyz)
    out = []
    for quad in itertools.combinations(range(n), 4):
        a, b, c, d = (P[q] for q in quad)
        u = [b[k] - a[k] for k in range(3)]
        v = [c[k] - a[k] for k in range(3)]
        w = [d[k] - a[k] for k in range(3)]
        o = (u[0] * (v[1] * w[2] - v[2] * w[1]) - u[1] * (v[0] * w[2] - v[2] * w[0])
             + u[2] * (v[0] * w[1] - v[1] * w[0]))
        if o == 0:
            continue
        q = list(quad)
        if o < 0:
            q[0], q[1] = q[1], q[0]
        if all(perturbed_sign_int(P, q, e, idx) > 0 for e in range(n) if e not in quad):
            out.append(sorted(idx[x] for x in quad))
    out.sort()
    return np.array(out, dtype=np.int64).reshape(-1, 4)


# ---------------------------------------------------------------- invariants

def check_adjacency(tets, nbrs):
    """I2: every neighbour link is mutual and across the same three vertices; returns the
    number of hull facets."""
    tets = np.asarray(tets, dtype=np.int64)
    nbrs = np.asarray(nbrs, dtype=np.int64)
    T = len(tets)
    assert nbrs.shape == (T, 4)
    assert np.all((nbrs >= -1) & (nbrs < T))
    faces = np.sort(np.stack([np.delete(tets, j, axis=1) for j in range(4)], axis=1), axis=2)  # T,4,3
    t_idx, j_idx = np.nonzero(nbrs >= 0)
    s = nbrs[t_idx, j_idx]
    f = faces[t_idx, j_idx]
    match = np.all(faces[s] == f[:, None, :], axis=2)  # K,4
    assert np.all(match.sum(axis=1) == 1), "neighbour does not share the facet"
    k = np.argmax(match, axis=1)
    assert np.all(nbrs[s, k] == t_idx), "neighbour link not mutual"
    return int(np.count_nonzero(nbrs < 0))


def euler_counts(tets, nbrs):
    tets = np.asarray(tets, dtype=np.int64)
    V = len(np.unique(tets))
    e = np.sort(tets[:, list(itertools.combinations(range(4), 2))], axis=2).reshape(-1, 2)
    E = len(np.unique(e, axis=0))
    f = np.sort(np.stack([np.delete(tets, j, axis=1) for j in range(4)], axis=1), axis=2).reshape(-1, 3)
    F = len(np.unique(f, axis=0))
    hull = np.sort(np.stack([np.delete(tets, j, axis=1) for j in range(4)], axis=1), axis=2)[np.asarray(nbrs) < 0]
    Vh = len(np.unique(hull))
    Eh = len(np.unique(np.sort(hull[:, [[0, 1], [0, 2], [1, 2]]], axis=2).reshape(-1, 2), axis=0))
    return V, E, F, len(tets), Vh, Eh, len(hull)


def hull_facets(xyz, tets, nbrs, oracle):
    """The facets without neighbour, (H, 3) vertex indices, each ordered so that the fourth
    vertex of its tetrahedron is on the positive side (exact orient3d > 0)."""
    tets = np.asarray(tets, dtype=np.int64)
    t_idx, j_idx = np.nonzero(np.asarray(nbrs) < 0)
    rest = np.array([[k for k in range(4) if k != j] for j in range(4)])
    f = tets[t_idx[:, None], rest[j_idx]].copy()
    inner = tets[t_idx, j_idx]
    s = oracle.orient3d(np.asarray(xyz, dtype=np.float64)[np.concatenate([f, inner[:, None]], axis=1)])
    assert np.all(s != 0), "flat tetrahedron on the hull"
    neg = s < 0
    tmp = f[neg, 1].copy()
    f[neg, 1] = f[neg, 2]
    f[neg, 2] = tmp
    return f


def check_volume_exact(xyz, tets, nbrs, oracle):
    """I6, exact: with the coordinates scaled to integers, six times the summed volume of the
    tetrahedra (the sum of their orient3d determinants) equals the divergence-theorem volume of
    the hull facets, -sum det(a, b, c) over the facets ordered as in hull_facets.  The identity
    holds for a complex whose shared facets cancel; two positive tetrahedra folded over a
    shared facet break it, unless that facet's plane holds the origin (the reference point of
    the divergence sum)."""
    P = np.empty((len(xyz), 3), dtype=object)
    P[:, :] = _int_scale(xyz)
    t = np.asarray(tets, dtype=np.int64)
    a = P[t[:, 0]]
    u, v, w = P[t[:, 1]] - a, P[t[:, 2]] - a, P[t[:, 3]] - a
    vol6 = (u[:, 0] * (v[:, 1] * w[:, 2] - v[:, 2] * w[:, 1]) - u[:, 1] * (v[:, 0] * w[:, 2] - v[:, 2] * w[:, 0])
            + u[:, 2] * (v[:, 0] * w[:, 1] - v[:, 1] * w[:, 0]))
    f = hull_facets(xyz, tets, nbrs, oracle)
    A, B, C = P[f[:, 0]], P[f[:, 1]], P[f[:, 2]]
    div6 = (A[:, 0] * (B[:, 1] * C[:, 2] - B[:, 2] * C[:, 1]) - A[:, 1] * (B[:, 0] * C[:, 2] - B[:, 2] * C[:, 0])
            + A[:, 2] * (B[:, 0] * C[:, 1] - B[:, 1] * C[:, 0]))
    total, hull = int(vol6.sum()), -int(div6.sum())
    assert total == hull, "tetrahedra and hull facets enclose different volumes"
    return total


def check_hull_convex(xyz, tets, nbrs, oracle):
    """I4: the hull is locally convex.  Each hull facet is oriented with its tetrahedron's
    fourth vertex on the inner side (exact orient3d > 0); across every hull edge, the far
    vertex of the other hull facet must lie on the inner side of this one or in its plane."""
    xyz = np.asarray(xyz, dtype=np.float64)
    f = hull_facets(xyz, tets, nbrs, oracle)
    H = len(f)
    # hull edges: (sorted vertex pair, facet, far vertex of the facet)
    E = np.stack([np.sort(np.stack([f[:, k], f[:, (k + 1) % 3]], axis=1), axis=1) for k in range(3)],
                 axis=1).reshape(-1, 2)
    W = np.stack([f[:, (k + 2) % 3] for k in range(3)], axis=1).reshape(-1)
    face = np.repeat(np.arange(H), 3)
    order = np.lexsort((E[:, 1], E[:, 0]))
    assert len(order) % 2 == 0
    a, b = order[0::2], order[1::2]
    assert np.all(E[a] == E[b]), "a hull edge is not shared by exactly two hull facets"
    if len(a) > 1:
        assert np.all(np.any(E[a[1:]] != E[a[:-1]], axis=1)), "a hull edge is shared by more than two facets"
    for x, y in ((a, b), (b, a)):
        q = np.concatenate([f[face[x]], W[y][:, None]], axis=1)
        assert np.all(oracle.orient3d(xyz[q]) >= 0), "hull not locally convex"
    return H


def check_invariants(xyz, tets, nbrs, oracle, expect_vertices=None, local_delaunay=True,
                     chunk=1 << 20, exact_volume=True):
    """I1 orientation, I2 adjacency, I3 Euler characteristic, I4 local convexity of the hull,
    I5 vertex coverage, I6 volume, I7 local Delaunay (perturbed).  Raises AssertionError on
    failure."""
    xyz = np.asarray(xyz, dtype=np.float64)
    tets = np.asarray(tets, dtype=np.int64)
    nbrs = np.asarray(nbrs, dtype=np.int64)
    T = len(tets)
    assert T > 0
    # I1: exact positive orientation
    for s in range(0, T, chunk):
        o = oracle.orient3d(xyz[tets[s:s + chunk]])
        assert np.all(o > 0), "non-positive tetrahedron"
    # I2
    check_adjacency(tets, nbrs)
    # I3
    V, E, F, TT, Vh, Eh, Fh = euler_counts(tets, nbrs)
    assert V - E + F - TT == 1, "Euler characteristic of the complex"
    assert Vh - Eh + Fh == 2, "Euler characteristic of the hull surface"
    # I4
    check_hull_convex(xyz, tets, nbrs, oracle)
    # I5
    if expect_vertices is not None:
        assert np.array_equal(np.unique(tets), np.sort(np.asarray(expect_vertices)))
    # I6: exact, the tetrahedra against the hull facets of the output; then the summed volumes
    # against an independent hull (tolerance: float)
    if exact_volume:
        check_volume_exact(xyz, tets, nbrs, oracle)
    p = xyz[tets]
    vol = np.einsum("ij,ij->i", p[:, 1] - p[:, 0], np.cross(p[:, 2] - p[:, 0], p[:, 3] - p[:, 0])).sum() / 6.0
    try:
        from scipy.spatial import ConvexHull
        hv = ConvexHull(xyz[np.unique(tets)]).volume
        assert abs(vol - hv) <= 1e-9 * max(hv, 1e-300), (vol, hv)
    except ImportError:  # pragma: no cover
        pass
    # I7: each interior facet is locally Delaunay under the perturbation
    if local_delaunay:
        t_idx, j_idx = np.nonzero(nbrs >= 0)
        sel = nbrs[t_idx, j_idx] > t_idx
        t_idx, j_idx = t_idx[sel], j_idx[sel]
        s_idx = nbrs[t_idx, j_idx]
        # apex of s opposite the shared facet
        in_t = (tets[s_idx][:, :, None] == tets[t_idx][:, None, :]).any(axis=2)
        apex = tets[s_idx][~in_t]
        assert len(apex) == len(s_idx)
        for s in range(0, len(t_idx), chunk):
            q = np.concatenate([tets[t_idx[s:s + chunk]], apex[s:s + chunk, None]], axis=1)
            sign = oracle.insphere_sos(xyz[q], q)
            assert np.all(sign > 0), "facet not locally Delaunay"
    return dict(V=V, E=E, F=F, T=TT, hull_facets=Fh)
