/*
 * Whole-output check of a tetrahedralization, for outputs too large for the Python
 * validators.  TEST INFRASTRUCTURE ONLY: it links the oracle's exact predicates
 * (oracle/predicates.c, oracle/exact.c) and runs on the host, one OpenMP thread per core.
 *
 * For every tetrahedron t (vertex input indices tets[4t..], neighbours nbrs[4t..], facet j
 * opposite vertex j, -1 on the hull) it checks:
 *   I1  orient3d(t) > 0, exactly (the four indices distinct and in range);
 *   I2  each neighbour s holds t exactly once among its neighbours, on the facet that has
 *       the same three vertices;
 *   fold  across each interior facet the apex of s lies strictly on the other side of the
 *       facet from t's own vertex (the two tetrahedra do not overlap);
 *   I7  each interior facet is locally Delaunay under the symbolic perturbation: the apex of
 *       s is outside the circumsphere of t (perturbed insphere > 0, input index = point index).
 * With the hull facets forming one locally convex closed surface (checked by the caller on
 * the few hull facets) and every point a vertex, Delaunay's lemma makes such an output the
 * unique perturbed Delaunay tetrahedralization.
 */
#include <stdint.h>
#include <stdlib.h>

#include "../oracle/oracle.h"

enum {
    FC_OK = 0,
    FC_VERTEX = 1,    /* vertex index out of range or repeated */
    FC_ORIENT = 2,    /* I1 */
    FC_NBR_RANGE = 3, /* neighbour index out of range */
    FC_MIRROR = 4,    /* I2 */
    FC_FOLD = 5,      /* overlapping neighbours */
    FC_DELAUNAY = 6   /* I7 */
};

/* counts[0] tetrahedra, [1] interior facets checked (once each), [2] hull facets.
   Returns FC_OK or the first failure code found; *where = its tetrahedron. */
int fullcheck(const double *xyz, int64_t n, const uint32_t *tets, const int64_t *nbrs, int64_t T,
              int64_t *counts, int64_t *where) {
    int code = FC_OK;
    int64_t first = -1, interior = 0, hull = 0;
#pragma omp parallel for schedule(dynamic, 4096) reduction(+ : interior, hull)
    for (int64_t t = 0; t < T; ++t) {
        int bad = FC_OK;
        const uint32_t *v = tets + 4 * t;
        for (int a = 0; a < 4 && !bad; ++a) {
            if ((int64_t)v[a] >= n) bad = FC_VERTEX;
            for (int b = 0; b < a && !bad; ++b)
                if (v[a] == v[b]) bad = FC_VERTEX;
        }
        const double *p[4];
        if (!bad) {
            for (int a = 0; a < 4; ++a) p[a] = xyz + 3 * (int64_t)v[a];
            if (or_orient3d(p[0], p[1], p[2], p[3], NULL) <= 0) bad = FC_ORIENT;
        }
        for (int j = 0; j < 4 && !bad; ++j) {
            const int64_t s = nbrs[4 * t + j];
            if (s < 0) {
                hull++;
                continue;
            }
            if (s >= T || s == t) {
                bad = FC_NBR_RANGE;
                break;
            }
            const uint32_t *w = tets + 4 * s;
            int k = -1, links = 0;
            for (int q = 0; q < 4; ++q)
                if (nbrs[4 * s + q] == t) {
                    k = q;
                    links++;
                }
            if (links != 1) {
                bad = FC_MIRROR;
                break;
            }
            /* the apex w[k] is not a vertex of t; t's other three vertices are in s */
            for (int a = 0; a < 4 && !bad; ++a)
                if (v[a] == w[k]) bad = FC_MIRROR;
            for (int a = 0; a < 4 && !bad; ++a) {
                if (a == j) continue;
                int found = 0;
                for (int q = 0; q < 4; ++q)
                    if (q != k && w[q] == v[a]) found = 1;
                if (!found) bad = FC_MIRROR;
            }
            if (bad || s < t) continue; /* each interior facet once, from its lower tetrahedron */
            interior++;
            if ((int64_t)w[k] >= n) {
                bad = FC_VERTEX;
                break;
            }
            const double *e = xyz + 3 * (int64_t)w[k];
            const double *f[4] = {p[0], p[1], p[2], p[3]};
            f[j] = e;
            if (or_orient3d(f[0], f[1], f[2], f[3], NULL) >= 0) {
                bad = FC_FOLD;
                break;
            }
            const double *q5[5] = {p[0], p[1], p[2], p[3], e};
            const int64_t idx[5] = {v[0], v[1], v[2], v[3], w[k]};
            if (or_insphere_sos(q5, idx, NULL) <= 0) bad = FC_DELAUNAY;
        }
        if (bad) {
#pragma omp critical
            {
                if (code == FC_OK || t < first) {
                    code = bad;
                    first = t;
                }
            }
        }
    }
    counts[0] = T;
    counts[1] = interior;
    counts[2] = hull;
    *where = first;
    return code;
}
