/*
 * Oracle for the Delaunay tetrahedralization: plain, slow, serial CPU code.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls it; only the tests,
 * the package's smoke check and the benchmark's CPU-baseline leg load it.  It shares no
 * code with the GPU path.
 *
 * Conventions (paper, Sec. 2.2 and Sec. 2.4):
 *   orient3d(a,b,c,d) = (b-a) . ((c-a) x (d-a)); a stored tetrahedron has orient3d > 0;
 *   facet i of a tetrahedron is the one opposite its i-th vertex.
 *   insphere(a,b,c,d,e) = det of the 5x5 matrix with rows (x, y, z, |p|^2, 1) for
 *   a,b,c,d,e in that order; for a positive tetrahedron abcd, e is strictly inside the
 *   circumsphere iff the determinant is negative.
 * Symbolic perturbation (reading of Sec. 2.4 item 3): the lifted coordinate of point i is
 * |p_i|^2 + eps^(delta_i) with delta strictly decreasing in the input index, so the
 * highest index dominates; orient3d is never perturbed.
 *
 * What pins each part (tests, CPU only): the predicate signs against exact rational
 * determinants; the perturbation against the eps-polynomial of its definition, and the ghost
 * rule's tie-break against its independence of the apex; Moore keys by brute-force curve
 * properties and cells placed by construction; the sort against a library stable sort; the
 * level sizes against the paper's table of insertion steps; the triangulation against
 * brute-force enumeration on tiny inputs and invariants I1-I7 on larger ones.  The work
 * counters in oracle_stats are reported only: parity unpinned.
 */
#ifndef DT_ORACLE_H
#define DT_ORACLE_H
#include <stdint.h>

#define OR_OK 0
#define OR_E_ARG 1
#define OR_E_INPUT 2
#define OR_E_DEGENERATE 3
#define OR_E_NOMEM 4

/* Coordinates must be 0 or have magnitude in [2^-120, 2^120). */
#define OR_COORD_EXP 120

typedef struct {
    int64_t orient_calls, orient_exact, orient_zero;
    int64_t insphere_calls, insphere_exact, insphere_zero;
    int64_t walk_steps, cavity_tets, boundary_facets, max_cavity, duplicates;
    int64_t inserted;
} oracle_stats;

/* exact.c: signs of determinants evaluated in exact integer arithmetic */
int or_orient3d_exact(const double *a, const double *b, const double *c, const double *d);
int or_insphere_exact(const double *a, const double *b, const double *c, const double *d,
                      const double *e);
int or_collinear_exact(const double *a, const double *b, const double *c);

/* predicates.c: filtered predicates, perturbation and the ghost rule */
int or_orient3d(const double *a, const double *b, const double *c, const double *d,
                oracle_stats *st);
int or_insphere_raw(const double *a, const double *b, const double *c, const double *d,
                    const double *e, oracle_stats *st);
int or_insphere_sos(const double *p[5], const int64_t idx[5], oracle_stats *st);
int or_coord_ok(double x);

/* batch entry points used by the tests */
void oracle_orient3d_batch(const double *pts, int64_t k, int8_t *out);
void oracle_insphere_batch(const double *pts, int64_t k, int8_t *out);
void oracle_insphere_sos_batch(const double *pts, const int64_t *idx, int64_t k, int8_t *out);

/* moore.c: Moore-curve keys and BRIO levels (space-filling order of Sec. 2.3) */
int oracle_moore_level(int64_t n);
void oracle_moore_keys(const double *xyz, int64_t n, int m, uint64_t *keys);
uint64_t oracle_moore_index(const uint32_t cell[3], int m);
int oracle_brio_levels(int64_t n, uint64_t seed, uint8_t *level, int64_t *cum);
void oracle_stable_sort(const uint64_t *keys, int64_t n, int64_t *perm);

/* delaunay.c: serial Bowyer-Watson (Algorithm 1) */
enum { OR_ORDER_BRIO = 0, OR_ORDER_RANDOM = 1, OR_ORDER_REVERSE = 2, OR_ORDER_INPUT = 3 };
int oracle_delaunay(const double *xyz, int64_t n, int order, uint64_t seed, int32_t **tets,
                    int64_t **nbrs, int64_t *ntets, oracle_stats *st);
void oracle_free(void *p);

#endif
