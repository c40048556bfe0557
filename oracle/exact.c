/*
 * Oracle: exact signs of the orient3d and insphere determinants (paper, Sec. 2.4).
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Every finite double is M * 2^E with an integer |M| < 2^53.  The coordinates of one
 * call are scaled by 2^-Emin, Emin the smallest exponent among them, which turns each
 * into an exact integer; the determinant is then evaluated by its textbook expansion in
 * signed big integers (base 2^32 limbs).  No rounding happens anywhere, so the sign is
 * exact.  With every coordinate 0 or of magnitude in [2^-120, 2^120) the scaled
 * integers have at most 292 bits and the 4x4 lifted determinant at most 1472 bits, well
 * inside the 2048-bit capacity used here.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define BI_L 64

typedef struct {
    int n;   /* number of used limbs; 0 means the value zero */
    int neg; /* sign flag, only meaningful when n > 0 */
    uint32_t d[BI_L];
} bi;

static void bi_trim(bi *r) {
    while (r->n > 0 && r->d[r->n - 1] == 0) r->n--;
    if (r->n == 0) r->neg = 0;
}

static void bi_from(bi *r, int64_t m, int shift) {
    memset(r, 0, sizeof(*r));
    if (m == 0) return;
    r->neg = m < 0;
    uint64_t mag = m < 0 ? (uint64_t)(-m) : (uint64_t)m;
    int limb = shift / 32, bit = shift % 32;
    /* mag < 2^53 so mag << bit fits in 85 bits: three limbs */
    uint64_t lo = mag << bit;
    uint64_t hi = bit ? (mag >> (64 - bit)) : 0;
    if (limb + 3 > BI_L) abort();
    r->d[limb] = (uint32_t)lo;
    r->d[limb + 1] = (uint32_t)(lo >> 32);
    r->d[limb + 2] = (uint32_t)hi;
    r->n = limb + 3;
    bi_trim(r);
}

static int cmp_mag(const bi *a, const bi *b) {
    if (a->n != b->n) return a->n < b->n ? -1 : 1;
    for (int i = a->n - 1; i >= 0; --i)
        if (a->d[i] != b->d[i]) return a->d[i] < b->d[i] ? -1 : 1;
    return 0;
}

/* r = |a| + |b| (sign left to the caller) */
static void add_mag(bi *r, const bi *a, const bi *b) {
    int n = a->n > b->n ? a->n : b->n;
    uint64_t carry = 0;
    bi t;
    memset(&t, 0, sizeof(t));
    for (int i = 0; i < n; ++i) {
        uint64_t s = carry;
        if (i < a->n) s += a->d[i];
        if (i < b->n) s += b->d[i];
        t.d[i] = (uint32_t)s;
        carry = s >> 32;
    }
    if (carry) {
        if (n >= BI_L) abort();
        t.d[n++] = (uint32_t)carry;
    }
    t.n = n;
    *r = t;
}

/* r = |a| - |b| with |a| >= |b| */
static void sub_mag(bi *r, const bi *a, const bi *b) {
    int64_t borrow = 0;
    bi t;
    memset(&t, 0, sizeof(t));
    for (int i = 0; i < a->n; ++i) {
        int64_t s = (int64_t)a->d[i] - borrow - (i < b->n ? (int64_t)b->d[i] : 0);
        borrow = s < 0;
        if (s < 0) s += ((int64_t)1 << 32);
        t.d[i] = (uint32_t)s;
    }
    t.n = a->n;
    *r = t;
}

/* r = a + sb * b with sb = +1 or -1 */
static void bi_addsub(bi *r, const bi *a, const bi *b, int sb) {
    int bneg = b->n ? (b->neg ^ (sb < 0)) : 0;
    if (b->n == 0) { *r = *a; return; }
    if (a->n == 0) { *r = *b; r->neg = bneg; return; }
    if (a->neg == bneg) {
        int s = a->neg;
        add_mag(r, a, b);
        r->neg = s;
    } else if (cmp_mag(a, b) >= 0) {
        int s = a->neg;
        sub_mag(r, a, b);
        r->neg = s;
    } else {
        sub_mag(r, b, a);
        r->neg = bneg;
    }
    bi_trim(r);
}

static void bi_mul(bi *r, const bi *a, const bi *b) {
    bi t;
    memset(&t, 0, sizeof(t));
    if (a->n == 0 || b->n == 0) { *r = t; return; }
    if (a->n + b->n > BI_L) abort();
    for (int i = 0; i < a->n; ++i) {
        uint64_t carry = 0;
        for (int j = 0; j < b->n; ++j) {
            uint64_t cur = (uint64_t)a->d[i] * b->d[j] + t.d[i + j] + carry;
            t.d[i + j] = (uint32_t)cur;
            carry = cur >> 32;
        }
        t.d[i + b->n] = (uint32_t)carry;
    }
    t.n = a->n + b->n;
    t.neg = a->neg ^ b->neg;
    bi_trim(&t);
    *r = t;
}

static int bi_sign(const bi *a) { return a->n == 0 ? 0 : (a->neg ? -1 : 1); }

/* x = m * 2^e with |m| < 2^53 an integer; x == 0 gives m = 0 */
static void split_double(double x, int64_t *m, int *e) {
    if (x == 0.0) { *m = 0; *e = 0; return; }
    int k;
    double f = frexp(x, &k);
    *m = (int64_t)ldexp(f, 53);
    *e = k - 53;
}

/* Scale `cnt` doubles to exact integers sharing the smallest exponent. */
static void to_integers(const double *v, int cnt, bi *out) {
    int64_t m[15];
    int e[15], emin = 1 << 30;
    for (int i = 0; i < cnt; ++i) {
        split_double(v[i], &m[i], &e[i]);
        if (m[i] != 0 && e[i] < emin) emin = e[i];
    }
    for (int i = 0; i < cnt; ++i) bi_from(&out[i], m[i], m[i] ? e[i] - emin : 0);
}

/* determinant of a 3x3 matrix by the Leibniz formula */
static void det3(bi *r, const bi m[3][3]) {
    static const int perm[6][3] = {{0, 1, 2}, {1, 2, 0}, {2, 0, 1}, {0, 2, 1}, {2, 1, 0}, {1, 0, 2}};
    static const int sgn[6] = {1, 1, 1, -1, -1, -1};
    bi acc, t;
    memset(&acc, 0, sizeof(acc));
    for (int p = 0; p < 6; ++p) {
        bi_mul(&t, &m[0][perm[p][0]], &m[1][perm[p][1]]);
        bi_mul(&t, &t, &m[2][perm[p][2]]);
        bi_addsub(&acc, &acc, &t, sgn[p]);
    }
    *r = acc;
}

/* determinant of a 4x4 matrix by cofactor expansion along the last column */
static void det4(bi *r, const bi m[4][4]) {
    bi acc, minor_det, t;
    memset(&acc, 0, sizeof(acc));
    for (int row = 0; row < 4; ++row) {
        bi sub[3][3];
        int rr = 0;
        for (int i = 0; i < 4; ++i) {
            if (i == row) continue;
            for (int j = 0; j < 3; ++j) sub[rr][j] = m[i][j];
            rr++;
        }
        det3(&minor_det, (const bi(*)[3])sub);
        bi_mul(&t, &m[row][3], &minor_det);
        /* cofactor sign (-1)^(row + 3) */
        bi_addsub(&acc, &acc, &t, ((row + 3) % 2 == 0) ? 1 : -1);
    }
    *r = acc;
}

int or_orient3d_exact(const double *a, const double *b, const double *c, const double *d) {
    double v[12];
    for (int k = 0; k < 3; ++k) { v[k] = a[k]; v[3 + k] = b[k]; v[6 + k] = c[k]; v[9 + k] = d[k]; }
    bi X[12];
    to_integers(v, 12, X);
    bi m[3][3], r;
    for (int row = 0; row < 3; ++row)
        for (int k = 0; k < 3; ++k) bi_addsub(&m[row][k], &X[3 * (row + 1) + k], &X[k], -1);
    det3(&r, (const bi(*)[3])m);
    return bi_sign(&r);
}

int or_insphere_exact(const double *a, const double *b, const double *c, const double *d,
                      const double *e) {
    double v[15];
    const double *p[5] = {a, b, c, d, e};
    for (int i = 0; i < 5; ++i)
        for (int k = 0; k < 3; ++k) v[3 * i + k] = p[i][k];
    bi X[15];
    to_integers(v, 15, X);
    /* rows (p - a, |p - a|^2) for p = b, c, d, e: the translated form of the 5x5 */
    bi m[4][4], t;
    for (int row = 0; row < 4; ++row) {
        bi lift;
        memset(&lift, 0, sizeof(lift));
        for (int k = 0; k < 3; ++k) {
            bi_addsub(&m[row][k], &X[3 * (row + 1) + k], &X[k], -1);
            bi_mul(&t, &m[row][k], &m[row][k]);
            bi_addsub(&lift, &lift, &t, 1);
        }
        m[row][3] = lift;
    }
    bi r;
    det4(&r, (const bi(*)[4])m);
    return bi_sign(&r);
}

int or_collinear_exact(const double *a, const double *b, const double *c) {
    double v[9];
    for (int k = 0; k < 3; ++k) { v[k] = a[k]; v[3 + k] = b[k]; v[6 + k] = c[k]; }
    bi X[9], u[3], w[3], t1, t2, cr;
    to_integers(v, 9, X);
    for (int k = 0; k < 3; ++k) {
        bi_addsub(&u[k], &X[3 + k], &X[k], -1);
        bi_addsub(&w[k], &X[6 + k], &X[k], -1);
    }
    for (int k = 0; k < 3; ++k) {
        int i = (k + 1) % 3, j = (k + 2) % 3;
        bi_mul(&t1, &u[i], &w[j]);
        bi_mul(&t2, &u[j], &w[i]);
        bi_addsub(&cr, &t1, &t2, -1);
        if (bi_sign(&cr) != 0) return 0;
    }
    return 1;
}
