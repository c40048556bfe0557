/*
 * Oracle: Moore-curve keys and BRIO levels (paper, Sec. 2.1 "Sort" and Sec. 2.3).
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Grid: m = the smallest m >= 1 with 2^(3m) >= n (capped at 21), i.e. ceil(log2(n)/3);
 * the bounding box is made cubic with one scale s = 2^m / (largest extent) and the cell
 * of coordinate x along an axis is min(2^m - 1, floor((x - min) * s)).
 *
 * Hilbert curve: Hamilton's construction ("Compact Hilbert indices", 2006).  The curve of
 * a cube entered at corner e and heading first along axis d (state (e, d)) visits the
 * eight octants in the order l = T^{-1}(gray(w)), w = 0..7, with T_{e,d}(l) =
 * rotate_right(l xor e, d + 1); sub-cube w gets the state (e xor rotate_left(entry(w), d+1),
 * d + dir(w) + 1 mod 3) with entry(w) = gray(2 floor((w-1)/2)) and dir(w) the number of
 * trailing one bits of w-1 (w even) or of w (w odd), modulo 3.  The curve of state (e, d)
 * starts in corner e and ends in corner e xor 2^d.
 *
 * Moore curve: the closed variant.  The top-level octants are visited in Gray-code order
 * gray(0..7) (a cycle of face-adjacent octants) and octant w holds the Hilbert curve of
 * state (e_w, d_w).  The states are the first, in lexicographic order of
 * (e_0, d_0, ..., d_7), that chain every exit cell to the next entry cell and the last
 * exit back to the first entry; this search runs here from that definition.
 *
 * BRIO (Sec. 2.1 "Sort", cumulative round sizes of the per-step table of Sec. 3.4):
 * level k holds the points whose hash falls below cum_k / n, cum_k = min(n, 2048 * 7^k).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#include "oracle.h"

static unsigned rotl3(unsigned x, unsigned r) { r %= 3; return r ? (((x << r) | (x >> (3 - r))) & 7u) : x; }
static unsigned rotr3(unsigned x, unsigned r) { r %= 3; return r ? (((x >> r) | (x << (3 - r))) & 7u) : x; }
static unsigned gray(unsigned i) { return i ^ (i >> 1); }
static unsigned gray_inv(unsigned g) {
    unsigned i = g;
    for (unsigned s = 1; (g >> s) != 0; ++s) i ^= g >> s;
    return i;
}
static unsigned trailing_ones(unsigned i) {
    unsigned c = 0;
    while (i & 1u) { c++; i >>= 1; }
    return c;
}
static unsigned entry_corner(unsigned w) { return w == 0 ? 0 : gray(2 * ((w - 1) / 2)); }
static unsigned inner_dir(unsigned w) {
    if (w == 0) return 0;
    return (w % 2 == 0 ? trailing_ones(w - 1) : trailing_ones(w)) % 3;
}

static int moore_ready = 0;
static unsigned moore_e[8], moore_d[8];

static void moore_search(void) {
    for (unsigned e0 = 0; e0 < 8; ++e0) {
        for (unsigned code = 0; code < 6561; ++code) { /* 3^8 choices, d_0 most significant */
            unsigned ds[8], c = code;
            for (int w = 7; w >= 0; --w) { ds[w] = c % 3; c /= 3; }
            unsigned e = e0, es[8];
            int ok = 1;
            for (unsigned w = 0; w < 8 && ok; ++w) {
                es[w] = e;
                unsigned x = e ^ (1u << ds[w]);
                unsigned A = gray(w), B = gray((w + 1) % 8), diff = A ^ B;
                unsigned axis = diff == 1 ? 0 : (diff == 2 ? 1 : 2);
                if (((x >> axis) & 1u) != ((B >> axis) & 1u)) ok = 0;
                e = x ^ (1u << axis);
            }
            if (ok && e == e0) {
                for (int w = 0; w < 8; ++w) { moore_e[w] = es[w]; moore_d[w] = ds[w]; }
                moore_ready = 1;
                return;
            }
        }
    }
    abort();
}

uint64_t oracle_moore_index(const uint32_t cell[3], int m) {
    if (!moore_ready) moore_search();
    unsigned o = 0;
    for (int k = 0; k < 3; ++k) o |= ((cell[k] >> (m - 1)) & 1u) << k;
    unsigned w = gray_inv(o);
    uint64_t h = w;
    unsigned e = moore_e[w], d = moore_d[w];
    for (int i = m - 2; i >= 0; --i) {
        unsigned l = 0;
        for (int k = 0; k < 3; ++k) l |= ((cell[k] >> i) & 1u) << k;
        l = rotr3(l ^ e, d + 1);
        unsigned ww = gray_inv(l);
        e = e ^ rotl3(entry_corner(ww), d + 1);
        d = (d + inner_dir(ww) + 1) % 3;
        h = (h << 3) | ww;
    }
    return h;
}

int oracle_moore_level(int64_t n) {
    int m = 1;
    while (m < 21 && ((int64_t)1 << (3 * m)) < n) m++;
    return m;
}

void oracle_moore_keys(const double *xyz, int64_t n, int m, uint64_t *keys) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) {
            double v = xyz[3 * i + k];
            if (v < lo[k]) lo[k] = v;
            if (v > hi[k]) hi[k] = v;
        }
    double ext = 0.0;
    for (int k = 0; k < 3; ++k)
        if (hi[k] - lo[k] > ext) ext = hi[k] - lo[k];
    double cells = ldexp(1.0, m);
    double s = ext > 0.0 ? cells / ext : 0.0;
    uint32_t top = (uint32_t)((1u << m) - 1u);
    for (int64_t i = 0; i < n; ++i) {
        uint32_t c[3];
        for (int k = 0; k < 3; ++k) {
            double t = floor((xyz[3 * i + k] - lo[k]) * s);
            c[k] = t >= (double)top ? top : (uint32_t)t;
        }
        keys[i] = oracle_moore_index(c, m);
    }
}

static uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* level[i] for every point, cum[0..L-1] the cumulative sizes; returns L */
int oracle_brio_levels(int64_t n, uint64_t seed, uint8_t *level, int64_t *cum) {
    int L = 0;
    int64_t size = 2048;
    for (;;) {
        cum[L] = size < n ? size : n;
        L++;
        if (size >= n) break;
        size *= 7;
    }
    uint64_t salt = mix64(seed ^ 0x5851F42D4C957F2Dull);
    for (int64_t i = 0; i < n; ++i) {
        uint64_t u = mix64(salt + (uint64_t)i) >> 11; /* 53 uniform bits */
        int k = 0;
        while (k < L - 1 &&
               !((unsigned __int128)u * (uint64_t)n < ((unsigned __int128)(uint64_t)cum[k] << 53)))
            k++;
        level[i] = (uint8_t)k;
    }
    return L;
}

static const uint64_t *sort_keys;
static int cmp_idx(const void *pa, const void *pb) {
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    if (sort_keys[a] != sort_keys[b]) return sort_keys[a] < sort_keys[b] ? -1 : 1;
    return a < b ? -1 : (a > b);
}

void oracle_stable_sort(const uint64_t *keys, int64_t n, int64_t *perm) {
    for (int64_t i = 0; i < n; ++i) perm[i] = i;
    sort_keys = keys;
    qsort(perm, (size_t)n, sizeof(int64_t), cmp_idx);
}
