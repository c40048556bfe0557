/*
 * Oracle: serial Bowyer-Watson insertion (paper, Sec. 2.1, Algorithm 1, Eq. (1)).
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Plain serial C on one core.
 *
 *   1. reject non-finite or out-of-range coordinates; drop exact duplicates, keeping the
 *      lowest input index of each group;
 *   2. Init: the first point in input order, then the first point distinct from it, the
 *      first not collinear with both, the first not coplanar with the three; one positive
 *      tetrahedron plus four ghost tetrahedra (Sec. 2.6);
 *   3. the remaining points in the requested order (BRIO levels with Morton order inside
 *      each level, a random permutation, reverse or input order; the result does not
 *      depend on it);
 *   4. per point: Walk (cross any facet from which the point is visible, i.e. where the
 *      facet and the point have negative volume; a ghost start steps to its finite
 *      neighbour, entering a ghost stops), Cavity (breadth-first search over tetrahedra
 *      whose perturbed circumsphere contains the point; ghosts by the half-space plus
 *      circumdisk rule of Sec. 2.6), DelaunayBall (one new tetrahedron per cavity boundary
 *      facet, glued to the outer tetrahedron and, through a hash map over the boundary
 *      edges, to each other; freed slots are reused first).
 * Output: every finite tetrahedron (input indices, positive orientation) and the index
 * of the finite tetrahedron across each facet, -1 on the convex hull.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define GHOST (-1)

typedef struct {
    const double *xyz;
    int32_t *v;    /* 4 per tetrahedron: input index or GHOST */
    int64_t *nb;   /* 4 per tetrahedron: 4 * neighbour + facet in the neighbour */
    int64_t *mark; /* breadth-first-search stamp */
    uint8_t *dead;
    int64_t cap, count;
    int64_t *freel;
    int64_t nfree, capfree;
    oracle_stats *st;
} mesh_t;

static const double *P(const mesh_t *m, int32_t i) { return m->xyz + 3 * (int64_t)i; }

static int grow(mesh_t *m) {
    int64_t nc = m->cap ? 2 * m->cap : 1024;
    int32_t *v = realloc(m->v, sizeof(int32_t) * 4 * nc);
    if (!v) return 0;
    m->v = v;
    int64_t *nb = realloc(m->nb, sizeof(int64_t) * 4 * nc);
    if (!nb) return 0;
    m->nb = nb;
    int64_t *mk = realloc(m->mark, sizeof(int64_t) * nc);
    if (!mk) return 0;
    m->mark = mk;
    uint8_t *dd = realloc(m->dead, nc);
    if (!dd) return 0;
    m->dead = dd;
    for (int64_t t = m->cap; t < nc; ++t) { m->mark[t] = -1; m->dead[t] = 1; }
    m->cap = nc;
    return 1;
}

static int64_t alloc_tet(mesh_t *m) {
    if (m->nfree > 0) return m->freel[--m->nfree];
    if (m->count == m->cap && !grow(m)) return -1;
    return m->count++;
}

static int free_tet(mesh_t *m, int64_t t) {
    if (m->nfree == m->capfree) {
        int64_t nc = m->capfree ? 2 * m->capfree : 1024;
        int64_t *f = realloc(m->freel, sizeof(int64_t) * nc);
        if (!f) return 0;
        m->freel = f;
        m->capfree = nc;
    }
    m->dead[t] = 1;
    m->freel[m->nfree++] = t;
    return 1;
}

static int ghost_pos(const mesh_t *m, int64_t t) {
    for (int k = 0; k < 4; ++k)
        if (m->v[4 * t + k] == GHOST) return k;
    return -1;
}

/* Finite facet of a ghost, ordered so that orient3d(f0, f1, f2, x) > 0 for x outside. */
static void ghost_face(const mesh_t *m, int64_t t, int k, int32_t f[3]) {
    int q = 0;
    for (int i = 0; i < 4; ++i)
        if (i != k) f[q++] = m->v[4 * t + i];
    if ((3 - k) % 2 == 1) { int32_t s = f[0]; f[0] = f[1]; f[1] = s; }
}

/* perturbed "p strictly inside the circumsphere of finite tetrahedron t" */
static int finite_inside(const mesh_t *m, int64_t t, int32_t p) {
    const double *pts[5];
    int64_t idx[5];
    for (int i = 0; i < 4; ++i) { idx[i] = m->v[4 * t + i]; pts[i] = P(m, m->v[4 * t + i]); }
    idx[4] = p;
    pts[4] = P(m, p);
    return or_insphere_sos(pts, idx, m->st) < 0;
}

/* Sec. 2.6: the open half-space beyond the hull facet, plus the facet's circumdisk,
 * decided by the finite neighbour's perturbed insphere */
static int tet_inside(const mesh_t *m, int64_t t, int32_t p) {
    int k = ghost_pos(m, t);
    if (k < 0) return finite_inside(m, t, p);
    int32_t f[3];
    ghost_face(m, t, k, f);
    int o = or_orient3d(P(m, f[0]), P(m, f[1]), P(m, f[2]), P(m, p), m->st);
    if (o != 0) return o > 0;
    int64_t nt = m->nb[4 * t + k] >> 2;
    return finite_inside(m, nt, p);
}

/* orient3d of tetrahedron t with its vertex j replaced by point p */
static int orient_replace(const mesh_t *m, int64_t t, int j, int32_t p) {
    const double *q[4];
    for (int i = 0; i < 4; ++i) q[i] = P(m, i == j ? p : m->v[4 * t + i]);
    return or_orient3d(q[0], q[1], q[2], q[3], m->st);
}

static int64_t walk(mesh_t *m, int64_t t, int32_t p) {
    if (ghost_pos(m, t) >= 0) t = m->nb[4 * t + ghost_pos(m, t)] >> 2;
    for (int64_t steps = 0;; ++steps) {
        if (steps > 4 * m->count + 1000) abort(); /* a visibility walk cannot cycle */
        int moved = 0;
        for (int j = 0; j < 4; ++j) {
            if (orient_replace(m, t, j, p) < 0) {
                int64_t nt = m->nb[4 * t + j] >> 2;
                if (m->st) m->st->walk_steps++;
                t = nt;
                moved = 1;
                break;
            }
        }
        if (!moved || ghost_pos(m, t) >= 0) return t;
    }
}

typedef struct { int64_t key; int64_t code; int64_t gen; } edge_slot;

typedef struct {
    int64_t *cav, *bnd, *outer; /* cavity tetrahedra; boundary (4c+f); outer (4u+j) */
    int64_t ccap, bcap;
    edge_slot *tab;
    int64_t tcap, gen;
} work_t;

static int push64(int64_t **arr, int64_t *cap, int64_t n, int64_t val) {
    if (n == *cap) {
        int64_t nc = *cap ? 2 * *cap : 256;
        int64_t *a = realloc(*arr, sizeof(int64_t) * nc);
        if (!a) return 0;
        *arr = a;
        *cap = nc;
    }
    (*arr)[n] = val;
    return 1;
}

static int insert_point(mesh_t *m, work_t *w, int64_t *last, int32_t p, int64_t stamp) {
    int64_t t = walk(m, *last, p);
    if (ghost_pos(m, t) < 0) {
        const double *pp = P(m, p);
        for (int i = 0; i < 4; ++i) {
            const double *q = P(m, m->v[4 * t + i]);
            if (q[0] == pp[0] && q[1] == pp[1] && q[2] == pp[2]) {
                if (m->st) m->st->duplicates++;
                return 1;
            }
        }
    }
    /* Cavity: breadth-first search; mark 2*stamp = inside, 2*stamp+1 = outside */
    int64_t nc = 0, nbnd = 0, bcap_o = w->bcap;
    m->mark[t] = 2 * stamp;
    if (!push64(&w->cav, &w->ccap, nc++, t)) return 0;
    for (int64_t qi = 0; qi < nc; ++qi) {
        int64_t c = w->cav[qi];
        for (int f = 0; f < 4; ++f) {
            int64_t code = m->nb[4 * c + f];
            int64_t u = code >> 2;
            int in;
            if (m->mark[u] == 2 * stamp) continue;
            if (m->mark[u] == 2 * stamp + 1) {
                in = 0;
            } else {
                in = tet_inside(m, u, p);
                m->mark[u] = 2 * stamp + (in ? 0 : 1);
            }
            if (in) {
                if (!push64(&w->cav, &w->ccap, nc++, u)) return 0;
            } else {
                bcap_o = w->bcap;
                if (!push64(&w->bnd, &w->bcap, nbnd, 4 * c + f)) return 0;
                if (w->bcap != bcap_o) {
                    int64_t *o = realloc(w->outer, sizeof(int64_t) * w->bcap);
                    if (!o) return 0;
                    w->outer = o;
                }
                w->outer[nbnd++] = code;
            }
        }
    }
    if (m->st) {
        m->st->cavity_tets += nc;
        m->st->boundary_facets += nbnd;
        if (nc > m->st->max_cavity) m->st->max_cavity = nc;
        m->st->inserted++;
    }
    /* DT <- DT \ C */
    for (int64_t i = 0; i < nc; ++i)
        if (!free_tet(m, w->cav[i])) return 0;
    /* edge hash table of at least 4 * (number of boundary facets) slots */
    int64_t need = 16;
    while (need < 4 * nbnd) need *= 2;
    if (need > w->tcap) {
        edge_slot *tb = realloc(w->tab, sizeof(edge_slot) * need);
        if (!tb) return 0;
        w->tab = tb;
        for (int64_t i = w->tcap; i < need; ++i) w->tab[i].gen = -1;
        w->tcap = need;
    }
    int64_t mask = need - 1, gen = ++w->gen;
    /* DT <- DT u B */
    int64_t tnew = -1;
    for (int64_t k = 0; k < nbnd; ++k) {
        int64_t u = w->outer[k] >> 2;
        int j = (int)(w->outer[k] & 3);
        tnew = alloc_tet(m);
        if (tnew < 0) return 0;
        int32_t vv[4];
        for (int i = 0; i < 4; ++i) vv[i] = m->v[4 * u + i];
        vv[j] = p;
        int a = (j + 1) % 4, b = (j + 2) % 4;
        int32_t s = vv[a]; vv[a] = vv[b]; vv[b] = s;
        for (int i = 0; i < 4; ++i) m->v[4 * tnew + i] = vv[i];
        m->dead[tnew] = 0;
        m->mark[tnew] = -1;
        m->nb[4 * tnew + j] = 4 * u + j;
        m->nb[4 * u + j] = 4 * tnew + j;
        for (int q = 0; q < 4; ++q) {
            if (q == j) continue;
            int32_t e[2];
            int ne = 0;
            for (int i = 0; i < 4; ++i)
                if (i != q && i != j) e[ne++] = vv[i];
            int64_t lo = e[0] < e[1] ? e[0] : e[1], hi = e[0] < e[1] ? e[1] : e[0];
            int64_t key = (lo + 1) * ((int64_t)1 << 32) + (hi + 1);
            uint64_t h = (uint64_t)key * 0x9E3779B97F4A7C15ull;
            int64_t pos = (int64_t)(h >> 20) & mask;
            for (;;) {
                edge_slot *sl = &w->tab[pos];
                if (sl->gen != gen) {
                    sl->gen = gen;
                    sl->key = key;
                    sl->code = 4 * tnew + q;
                    break;
                }
                if (sl->key == key) {
                    m->nb[4 * tnew + q] = sl->code;
                    m->nb[sl->code] = 4 * tnew + q;
                    sl->key = INT64_MIN; /* consumed; keep the probe chain intact */
                    break;
                }
                pos = (pos + 1) & mask;
            }
        }
    }
    *last = tnew;
    return 1;
}

/* order helpers */
static const double *g_xyz;
static uint64_t *g_key;
static int cmp_coords(const void *pa, const void *pb) {
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    for (int k = 0; k < 3; ++k) {
        double x = g_xyz[3 * a + k], y = g_xyz[3 * b + k];
        if (x != y) return x < y ? -1 : 1;
    }
    return a < b ? -1 : (a > b);
}
static int cmp_key(const void *pa, const void *pb) {
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    if (g_key[a] != g_key[b]) return g_key[a] < g_key[b] ? -1 : 1;
    return a < b ? -1 : (a > b);
}
static uint64_t spread3(uint64_t x) { /* 21 bits -> every third bit */
    uint64_t r = 0;
    for (int i = 0; i < 21; ++i) r |= ((x >> i) & 1ull) << (3 * i);
    return r;
}
static uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int oracle_delaunay(const double *xyz, int64_t n, int order, uint64_t seed, int32_t **tets,
                    int64_t **nbrs, int64_t *ntets, oracle_stats *st) {
    *tets = 0;
    *nbrs = 0;
    *ntets = 0;
    if (n < 0 || (n > 0 && !xyz) || n >= ((int64_t)1 << 31)) return OR_E_ARG;
    for (int64_t i = 0; i < 3 * n; ++i)
        if (!or_coord_ok(xyz[i])) return OR_E_INPUT;
    int rc = OR_E_NOMEM;
    mesh_t m;
    memset(&m, 0, sizeof(m));
    m.xyz = xyz;
    m.st = st;
    work_t w;
    memset(&w, 0, sizeof(w));
    int64_t *idx = malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    uint8_t *dup = calloc(n > 0 ? n : 1, 1);
    uint64_t *key = malloc(sizeof(uint64_t) * (n > 0 ? n : 1));
    uint8_t *lev = malloc(n > 0 ? n : 1);
    if (!idx || !dup || !key || !lev) goto out;
    /* 1. duplicates: sort by coordinates, keep the lowest index of each equal group */
    for (int64_t i = 0; i < n; ++i) idx[i] = i;
    g_xyz = xyz;
    qsort(idx, (size_t)n, sizeof(int64_t), cmp_coords);
    for (int64_t i = 1; i < n; ++i) {
        const double *a = xyz + 3 * idx[i - 1], *b = xyz + 3 * idx[i];
        if (a[0] == b[0] && a[1] == b[1] && a[2] == b[2]) {
            dup[idx[i]] = 1;
            if (st) st->duplicates++;
        }
    }
    /* 2. Init */
    int64_t in[4] = {-1, -1, -1, -1};
    for (int64_t i = 0; i < n; ++i) {
        if (dup[i]) continue;
        const double *p = xyz + 3 * i;
        if (in[0] < 0) { in[0] = i; continue; }
        if (in[1] < 0) { in[1] = i; continue; } /* not a duplicate, hence distinct */
        if (in[2] < 0) {
            if (!or_collinear_exact(xyz + 3 * in[0], xyz + 3 * in[1], p)) in[2] = i;
            continue;
        }
        if (or_orient3d(xyz + 3 * in[0], xyz + 3 * in[1], xyz + 3 * in[2], p, st) != 0) {
            in[3] = i;
            break;
        }
    }
    if (in[3] < 0) { rc = OR_E_DEGENERATE; goto out; }
    if (or_orient3d(xyz + 3 * in[0], xyz + 3 * in[1], xyz + 3 * in[2], xyz + 3 * in[3], st) < 0) {
        int64_t s = in[0]; in[0] = in[1]; in[1] = s;
    }
    for (int i = 0; i < 5; ++i)
        if (alloc_tet(&m) < 0) goto out;
    for (int i = 0; i < 4; ++i) m.v[i] = (int32_t)in[i];
    for (int j = 0; j < 4; ++j) {
        /* ghost j: tetrahedron 0 with vertex j replaced by G, two entries swapped */
        int64_t g = 1 + j;
        int32_t vv[4];
        for (int i = 0; i < 4; ++i) vv[i] = m.v[i];
        vv[j] = GHOST;
        int a = (j + 1) % 4, b = (j + 2) % 4;
        int32_t s = vv[a]; vv[a] = vv[b]; vv[b] = s;
        for (int i = 0; i < 4; ++i) m.v[4 * g + i] = vv[i];
        m.nb[4 * g + j] = j;
        m.nb[j] = 4 * g + j;
    }
    for (int t = 0; t < 5; ++t) { m.dead[t] = 0; m.mark[t] = -1; }
    /* glue the ghosts to each other through their shared facets */
    for (int g1 = 1; g1 < 5; ++g1)
        for (int f1 = 0; f1 < 4; ++f1) {
            if (m.v[4 * g1 + f1] == GHOST) continue;
            for (int g2 = g1 + 1; g2 < 5; ++g2)
                for (int f2 = 0; f2 < 4; ++f2) {
                    if (m.v[4 * g2 + f2] == GHOST) continue;
                    int same = 1;
                    for (int i = 0; i < 4 && same; ++i) {
                        if (i == f1) continue;
                        int found = 0;
                        for (int k = 0; k < 4; ++k)
                            if (k != f2 && m.v[4 * g2 + k] == m.v[4 * g1 + i]) found = 1;
                        same = found;
                    }
                    if (same) {
                        m.nb[4 * g1 + f1] = 4 * g2 + f2;
                        m.nb[4 * g2 + f2] = 4 * g1 + f1;
                    }
                }
        }
    /* 3. insertion order */
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; ++i)
        if (!dup[i] && i != in[0] && i != in[1] && i != in[2] && i != in[3]) idx[cnt++] = i;
    if (order == OR_ORDER_BRIO || order == OR_ORDER_RANDOM) {
        if (order == OR_ORDER_BRIO) {
            int64_t cum[64];
            oracle_brio_levels(n, seed, lev, cum);
            double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
            for (int64_t i = 0; i < n; ++i)
                for (int k = 0; k < 3; ++k) {
                    if (xyz[3 * i + k] < lo[k]) lo[k] = xyz[3 * i + k];
                    if (xyz[3 * i + k] > hi[k]) hi[k] = xyz[3 * i + k];
                }
            for (int64_t i = 0; i < n; ++i) {
                uint64_t code = 0;
                for (int k = 0; k < 3; ++k) {
                    double ext = hi[k] - lo[k];
                    double t = ext > 0 ? (xyz[3 * i + k] - lo[k]) / ext * 2097151.0 : 0.0;
                    code |= spread3((uint64_t)t) << k;
                }
                key[i] = ((uint64_t)lev[i] << 58) | (code >> 5);
            }
        } else {
            for (int64_t i = 0; i < n; ++i) key[i] = mix64(seed * 0x2545F4914F6CDD1Dull + (uint64_t)i);
        }
        g_key = key;
        qsort(idx, (size_t)cnt, sizeof(int64_t), cmp_key);
    } else if (order == OR_ORDER_REVERSE) {
        for (int64_t i = 0; i < cnt / 2; ++i) {
            int64_t s = idx[i]; idx[i] = idx[cnt - 1 - i]; idx[cnt - 1 - i] = s;
        }
    }
    /* 4. insertions */
    int64_t last = 0;
    for (int64_t i = 0; i < cnt; ++i)
        if (!insert_point(&m, &w, &last, (int32_t)idx[i], i)) goto out;
    /* output */
    {
        int64_t *map = malloc(sizeof(int64_t) * m.count);
        if (!map) goto out;
        int64_t T = 0;
        for (int64_t t = 0; t < m.count; ++t)
            map[t] = (!m.dead[t] && ghost_pos(&m, t) < 0) ? T++ : -1;
        int32_t *ot = malloc(sizeof(int32_t) * 4 * (T ? T : 1));
        int64_t *on = malloc(sizeof(int64_t) * 4 * (T ? T : 1));
        if (!ot || !on) { free(map); free(ot); free(on); goto out; }
        for (int64_t t = 0; t < m.count; ++t) {
            if (map[t] < 0) continue;
            for (int i = 0; i < 4; ++i) {
                ot[4 * map[t] + i] = m.v[4 * t + i];
                on[4 * map[t] + i] = map[m.nb[4 * t + i] >> 2];
            }
        }
        free(map);
        *tets = ot;
        *nbrs = on;
        *ntets = T;
        rc = OR_OK;
    }
out:
    free(idx); free(dup); free(key); free(lev);
    free(m.v); free(m.nb); free(m.mark); free(m.dead); free(m.freel);
    free(w.cav); free(w.bnd); free(w.outer); free(w.tab);
    return rc;
}

void oracle_free(void *p) { free(p); }
