/*
 * Driver for the oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (CPU
 * only): runs the serial triangulation in every insertion order on tiny, uniform, duplicate,
 * lattice, co-spherical, coplanar, collinear, wide-exponent, one-ulp-nudged, NaN and thin
 * shell inputs, plus the batch predicates, Moore keys, sort and BRIO levels, and checks each
 * call's return code.  Any sanitizer report aborts the run.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static uint64_t rs = 88172645463325252ull;
static double u01(void) {  /* xorshift64 */
    rs ^= rs << 13;
    rs ^= rs >> 7;
    rs ^= rs << 17;
    return (double)(rs >> 11) * 0x1.0p-53;
}

static int failures = 0;

static void run(const char *name, const double *xyz, int64_t n, int want_rc) {
    for (int order = 0; order < 4; ++order) {
        int32_t *t = NULL;
        int64_t *nb = NULL, T = 0;
        oracle_stats s;
        memset(&s, 0, sizeof s);
        int rc = oracle_delaunay(xyz, n, order, 5, &t, &nb, &T, &s);
        if (rc != want_rc || (rc == 0) != (T > 0)) {
            printf("FAIL %s n=%lld order=%d rc=%d T=%lld\n", name, (long long)n, order, rc, (long long)T);
            failures++;
        }
        if (t) oracle_free(t);
        if (nb) oracle_free(nb);
    }
    printf("%-10s n=%-6lld rc=%d\n", name, (long long)n, want_rc);
}

int main(void) {
    const int64_t N = 30000;
    double *x = malloc(sizeof(double) * 3 * N);
    if (!x) return 2;
    for (int64_t n = 0; n <= 8; ++n) {
        for (int64_t i = 0; i < 3 * n; ++i) x[i] = u01();
        run("tiny", x, n, n < 4 ? 3 : 0);
    }
    for (int64_t i = 0; i < 3 * N; ++i) x[i] = u01();
    run("uniform", x, N, 0);
    memcpy(x + 3 * 1000, x, sizeof(double) * 3 * 1000);
    run("dups", x, 5000, 0);
    int64_t k = 0;
    for (int a = 0; a < 12; ++a)
        for (int b = 0; b < 12; ++b)
            for (int c = 0; c < 12; ++c, ++k) {
                x[3 * k] = a;
                x[3 * k + 1] = b;
                x[3 * k + 2] = c;
            }
    run("lattice", x, k, 0);
    k = 0;
    for (int a = -8; a < 8; ++a)
        for (int b = -8; b < 8; ++b)
            for (int c = -8; c < 8; ++c)
                if (a * a + b * b + c * c == 50) {
                    x[3 * k] = a;
                    x[3 * k + 1] = b;
                    x[3 * k + 2] = c;
                    k++;
                }
    run("sphere50", x, k, 0);
    for (int64_t i = 0; i < 200; ++i) {
        x[3 * i] = u01();
        x[3 * i + 1] = u01();
        x[3 * i + 2] = 0.5;
    }
    run("coplanar", x, 200, 3);
    for (int64_t i = 0; i < 50; ++i) {
        x[3 * i] = (double)i;
        x[3 * i + 1] = 2.0 * i;
        x[3 * i + 2] = 3.0 * i;
    }
    run("collinear", x, 50, 3);
    for (int64_t i = 0; i < 3 * 3000; ++i) x[i] = ldexp(u01() - 0.5, (int)(u01() * 60) - 30);
    run("wide", x, 3000, 0);
    k = 0;
    for (int a = 0; a < 8; ++a)
        for (int b = 0; b < 8; ++b)
            for (int c = 0; c < 8; ++c, ++k) {
                x[3 * k] = a + 1;
                x[3 * k + 1] = b + 1;
                x[3 * k + 2] = c + 1;
                if (u01() < 0.3) x[3 * k + (k % 3)] = nextafter(x[3 * k + (k % 3)], 1e9);
            }
    run("nudged", x, k, 0);
    for (int64_t i = 0; i < 30; ++i) x[i] = u01();
    x[7] = NAN;
    run("nan", x, 10, 2);
    for (int64_t i = 0; i < 5000; ++i) {
        double a = u01() * 6.283185307179586, z = 2 * u01() - 1, r = sqrt(1 - z * z);
        double rr = 1 + 1e-4 * u01();
        x[3 * i] = rr * r * cos(a);
        x[3 * i + 1] = rr * r * sin(a);
        x[3 * i + 2] = rr * z;
    }
    run("shell", x, 5000, 0);

    int8_t out[200];
    int64_t idx[5 * 200];
    for (int i = 0; i < 5 * 200; ++i) idx[i] = i;
    for (int64_t i = 0; i < 3 * 5 * 200; ++i) x[i] = floor(u01() * 3);
    oracle_orient3d_batch(x, 200, out);
    oracle_insphere_batch(x, 200, out);
    oracle_insphere_sos_batch(x, idx, 200, out);
    static uint64_t keys[1000];
    static int64_t perm[1000], cum[64];
    static uint8_t lev[1000];
    for (int i = 0; i < 3000; ++i) x[i] = u01();
    oracle_moore_keys(x, 1000, oracle_moore_level(1000), keys);
    oracle_stable_sort(keys, 1000, perm);
    oracle_brio_levels(1000, 3, lev, cum);
    free(x);
    printf(failures ? "failures: %d\n" : "done\n", failures);
    return failures ? 1 : 0;
}
