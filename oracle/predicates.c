/*
 * Oracle: filtered orient3d / insphere and the symbolic perturbation (paper, Sec. 2.4).
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Step 1 evaluates the determinant in fp64 in the translated form printed in Sec. 2.4
 * (rows p - a).  Step 2 is a dynamic filter: every monomial of the expansion passes
 * through at most 8 (orient3d) or 19 (insphere) roundings, so the computed value is
 * within gamma_19 < 2.2e-15 of the exact one relative to the sum of the monomials'
 * absolute values (the "permanent", computed alongside).  The oracle accepts the fp64
 * sign only when |det| exceeds 1e-14 (orient3d) or 1e-13 (insphere) times the permanent,
 * a deliberately wide margin.  Otherwise step 3 recomputes the sign exactly (exact.c).
 * Step 4, for an exact zero of insphere, is the symbolic perturbation.
 */
#include <math.h>
#include <stdint.h>

#include "oracle.h"

int or_coord_ok(double x) {
    if (!isfinite(x)) return 0;
    if (x == 0.0) return 1;
    double ax = fabs(x);
    return ax >= ldexp(1.0, -OR_COORD_EXP) && ax < ldexp(1.0, OR_COORD_EXP);
}

int or_orient3d(const double *a, const double *b, const double *c, const double *d,
                oracle_stats *st) {
    if (st) st->orient_calls++;
    double ux = b[0] - a[0], uy = b[1] - a[1], uz = b[2] - a[2];
    double vx = c[0] - a[0], vy = c[1] - a[1], vz = c[2] - a[2];
    double wx = d[0] - a[0], wy = d[1] - a[1], wz = d[2] - a[2];
    double det = ux * (vy * wz - vz * wy) + uy * (vz * wx - vx * wz) + uz * (vx * wy - vy * wx);
    double perm = fabs(ux) * (fabs(vy * wz) + fabs(vz * wy)) +
                  fabs(uy) * (fabs(vz * wx) + fabs(vx * wz)) +
                  fabs(uz) * (fabs(vx * wy) + fabs(vy * wx));
    if (fabs(det) > 1e-14 * perm) return det > 0 ? 1 : -1;
    if (st) st->orient_exact++;
    int s = or_orient3d_exact(a, b, c, d);
    if (s == 0 && st) st->orient_zero++;
    return s;
}

static double det3_fp(const double m[3][3], double *perm) {
    /* Leibniz formula, terms accumulated left to right */
    double t0 = m[0][0] * m[1][1] * m[2][2];
    double t1 = m[0][1] * m[1][2] * m[2][0];
    double t2 = m[0][2] * m[1][0] * m[2][1];
    double t3 = m[0][0] * m[1][2] * m[2][1];
    double t4 = m[0][2] * m[1][1] * m[2][0];
    double t5 = m[0][1] * m[1][0] * m[2][2];
    *perm = fabs(t0) + fabs(t1) + fabs(t2) + fabs(t3) + fabs(t4) + fabs(t5);
    return t0 + t1 + t2 - t3 - t4 - t5;
}

int or_insphere_raw(const double *a, const double *b, const double *c, const double *d,
                    const double *e, oracle_stats *st) {
    if (st) st->insphere_calls++;
    const double *p[4] = {b, c, d, e};
    double m[4][4];
    for (int r = 0; r < 4; ++r) {
        for (int k = 0; k < 3; ++k) m[r][k] = p[r][k] - a[k];
        m[r][3] = m[r][0] * m[r][0] + m[r][1] * m[r][1] + m[r][2] * m[r][2];
    }
    double det = 0.0, perm = 0.0;
    for (int row = 0; row < 4; ++row) {
        double sub[3][3], pm;
        int rr = 0;
        for (int i = 0; i < 4; ++i) {
            if (i == row) continue;
            for (int j = 0; j < 3; ++j) sub[rr][j] = m[i][j];
            rr++;
        }
        double dm = det3_fp((const double(*)[3])sub, &pm);
        double term = m[row][3] * dm;
        det += ((row + 3) % 2 == 0) ? term : -term;
        perm += m[row][3] * pm;
    }
    if (fabs(det) > 1e-13 * perm) return det > 0 ? 1 : -1;
    if (st) st->insphere_exact++;
    int s = or_insphere_exact(a, b, c, d, e);
    if (s == 0 && st) st->insphere_zero++;
    return s;
}

/*
 * Sign of the perturbed insphere determinant for rows p[0..4] (a,b,c,d,e, abcd positive).
 * When the unperturbed value is zero: the determinant is linear in the lifted column, so
 * the perturbed value is sum_r eps^delta(r) * C(r), C(r) the cofactor of row r in that
 * column, equal to (-1)^r * orient3d(the other four rows, in order) for 0-based r.  The
 * dominant power belongs to the largest input index, so rows are tried from the largest
 * index down and the first non-zero cofactor decides.
 */
int or_insphere_sos(const double *p[5], const int64_t idx[5], oracle_stats *st) {
    int s = or_insphere_raw(p[0], p[1], p[2], p[3], p[4], st);
    if (s != 0) return s;
    int order[5] = {0, 1, 2, 3, 4};
    for (int i = 0; i < 5; ++i)
        for (int j = i + 1; j < 5; ++j)
            if (idx[order[j]] > idx[order[i]]) { int t = order[i]; order[i] = order[j]; order[j] = t; }
    for (int q = 0; q < 5; ++q) {
        int r = order[q];
        const double *o[4];
        int k = 0;
        for (int i = 0; i < 5; ++i)
            if (i != r) o[k++] = p[i];
        int c = or_orient3d(o[0], o[1], o[2], o[3], st);
        if (c != 0) return (r % 2 == 0) ? c : -c;
    }
    return 0; /* only reachable when a,b,c,d are coplanar */
}

void oracle_orient3d_batch(const double *pts, int64_t k, int8_t *out) {
    for (int64_t i = 0; i < k; ++i) {
        const double *q = pts + 12 * i;
        out[i] = (int8_t)or_orient3d(q, q + 3, q + 6, q + 9, 0);
    }
}

void oracle_insphere_batch(const double *pts, int64_t k, int8_t *out) {
    for (int64_t i = 0; i < k; ++i) {
        const double *q = pts + 15 * i;
        out[i] = (int8_t)or_insphere_raw(q, q + 3, q + 6, q + 9, q + 12, 0);
    }
}

void oracle_insphere_sos_batch(const double *pts, const int64_t *idx, int64_t k, int8_t *out) {
    for (int64_t i = 0; i < k; ++i) {
        const double *q = pts + 15 * i;
        const double *p[5] = {q, q + 3, q + 6, q + 9, q + 12};
        out[i] = (int8_t)or_insphere_sos(p, idx + 5 * i, 0);
    }
}
