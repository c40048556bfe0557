// Exact geometric predicates on the GPU (paper Sec. 2.4 "Implementation details").
//
//   orient3d(a,b,c,d) = (b-a).((c-a)x(d-a))                       (Sec. 2.4)
//   insphere(a,b,c,d,e) = det of rows (x, y, z, |p|^2, 1), a..e    (Sec. 2.4, 5x5 form)
//                       = det of rows (p-e, |p-e|^2) for p = a,b,c,d (translated form)
//   For orient3d(a,b,c,d) > 0, e is strictly inside the circumsphere iff insphere < 0.
//
// Stage 1: fp64 evaluation in a fixed order plus a semi-static filter.  Every monomial of
// the expansion passes through at most 8 (orient3d) or 16 (insphere) roundings, so with the
// unit roundoff u = 2^-53 the absolute error is below gamma_k times the sum of the
// monomials' magnitudes.  With M the largest magnitude of the computed coordinate
// differences, that sum is at most 6 M^3 (orient3d: six products of three differences) and
// 72 M^5 (insphere: 4 lifted terms of 3 squares times 6 products of three differences).
// gamma_8 * 6 < 2^-46 and gamma_16 * 72 < 2^-42 leave a margin of more than two for the
// rounding of the differences and of M^k itself; the filter uses 2^-46 M^3 and 2^-41 M^5.
// Inputs are restricted to 0 or |x| in [2^-120, 2^120): every difference and product then
// stays a multiple of 2^(-172 k) at degree k <= 5, far above the underflow threshold, and
// far below overflow.
//
// Stage 2a (when the filter cannot decide): the same fp64 evaluation is repeated with an
// exactness certificate.  The rounding error of each product p = fl(x y) is fma(x, y, -p),
// and that of each sum or difference is the remainder of Knuth's TwoSum; both are computed
// without rounding.  If every one is zero, no operation rounded and the fp64 value is the
// exact determinant, zero included.  This decides the degenerate configurations of inputs
// with few significant bits (points of a lattice with a power-of-two spacing) without the
// integer stage.  The input range above keeps every intermediate out of the subnormals.
//
// Stage 2b (when the certificate fails): the coordinates are scaled by a common power
// of two into exact integers and the same determinant is evaluated in two's-complement
// multi-limb integers modulo 2^(32 W).  W is chosen from the exponent spread of the call
// so that every true intermediate value fits; the result is then exact.  This replaces
// the floating-point expansion arithmetic of the CPU implementation: its exact stage
// needs expansions of up to thousands of doubles per lane, while the integer form is
// bounded by the exponent spread (at most 47 limbs here) and needs no branches.
//
// Stage 3: symbolic perturbation for an exact zero of insphere (Sec. 2.4 item 3): the
// lifted coordinate of the point with input index i is |p_i|^2 + eps^delta_i, delta
// strictly decreasing in i.  The determinant is linear in that column, so its perturbed
// sign is the sign of the first non-zero cofactor (-1)^r orient3d(other four rows),
// rows r taken by decreasing input index.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dtk {

struct P3 {
    double x, y, z;
};

// per-thread predicate counters
struct PredStats {
    uint32_t orient = 0, orient_exact = 0, insphere = 0, insphere_exact = 0, perturbed = 0;
};

// ------------------------------------------------------------------ exact integers

constexpr int LIMBS_MAX = 48;

struct Dyadic {
    long long m;  // |m| < 2^53
    int e;        // value = m * 2^e
};

__device__ inline Dyadic split_dyadic(double x) {
    unsigned long long b = (unsigned long long)__double_as_longlong(x);
    int ex = (int)((b >> 52) & 0x7FF);
    if (ex == 0) return {0, 0};  // zero (subnormals are outside the accepted range)
    long long m = (long long)((b & 0xFFFFFFFFFFFFFull) | (1ull << 52));
    if (b >> 63) m = -m;
    return {m, ex - 1075};
}

// r (w limbs) = m * 2^sh, two's complement
__device__ inline void ei_set(uint32_t *r, int w, long long m, int sh) {
    for (int i = 0; i < w; ++i) r[i] = 0;
    unsigned long long mag = m < 0 ? (unsigned long long)(-m) : (unsigned long long)m;
    int q = sh >> 5, s = sh & 31;
    unsigned long long lo = mag << s;
    unsigned long long hi = s ? (mag >> (64 - s)) : 0ull;
    if (q < w) r[q] = (uint32_t)lo;
    if (q + 1 < w) r[q + 1] = (uint32_t)(lo >> 32);
    if (q + 2 < w) r[q + 2] = (uint32_t)hi;
    if (m < 0) {
        unsigned long long c = 1;
        for (int i = 0; i < w; ++i) {
            unsigned long long t = (unsigned long long)(uint32_t)~r[i] + c;
            r[i] = (uint32_t)t;
            c = t >> 32;
        }
    }
}

__device__ inline uint32_t ei_get(const uint32_t *a, int wa, int k) {
    return k < wa ? a[k] : ((a[wa - 1] >> 31) ? 0xFFFFFFFFu : 0u);
}

// r = a + s*b (s = +1/-1) modulo 2^(32 w); operands sign-extended
__device__ inline void ei_addsub(uint32_t *r, int w, const uint32_t *a, int wa, const uint32_t *b,
                                 int wb, bool sub) {
    unsigned long long c = sub ? 1ull : 0ull;
    for (int i = 0; i < w; ++i) {
        uint32_t bi = ei_get(b, wb, i);
        if (sub) bi = ~bi;
        unsigned long long t = (unsigned long long)ei_get(a, wa, i) + bi + c;
        r[i] = (uint32_t)t;
        c = t >> 32;
    }
}

// r = a * b modulo 2^(32 w); r must not alias a or b
__device__ inline void ei_mul(uint32_t *r, int w, const uint32_t *a, int wa, const uint32_t *b,
                              int wb) {
    for (int i = 0; i < w; ++i) r[i] = 0;
    for (int i = 0; i < w; ++i) {
        uint32_t ai = ei_get(a, wa, i);
        if (ai == 0) continue;
        unsigned long long c = 0;
        for (int j = 0; i + j < w; ++j) {
            unsigned long long t = (unsigned long long)ai * ei_get(b, wb, j) + r[i + j] + c;
            r[i + j] = (uint32_t)t;
            c = t >> 32;
        }
    }
}

__device__ inline int ei_sign(const uint32_t *a, int w) {
    if (a[w - 1] >> 31) return -1;
    for (int i = 0; i < w; ++i)
        if (a[i]) return 1;
    return 0;
}

// Scale `cnt` coordinates to exact integers with a common exponent; returns the number of
// bits of the largest magnitude (the exponent spread plus 53).
__device__ inline int ei_load(const double *v, int cnt, uint32_t (*X)[12], int wx) {
    Dyadic d[15];
    int emin = 1 << 20, emax = -(1 << 20);
    for (int i = 0; i < cnt; ++i) {
        d[i] = split_dyadic(v[i]);
        if (d[i].m != 0) {
            emin = min(emin, d[i].e);
            emax = max(emax, d[i].e);
        }
    }
    if (emax < emin) emin = emax = 0;
    for (int i = 0; i < cnt; ++i) ei_set(X[i], wx, d[i].m, d[i].m ? d[i].e - emin : 0);
    return emax - emin + 54;
}

// ------------------------------------------------------------------ exact integers, fixed width
// The same integer arithmetic with widths fixed at compile time, for inputs whose exponent
// spread is small (every coordinate an integer of at most SMALL_BITS bits after the common
// scaling): with every loop unrolled the limbs stay in registers.  The general routines
// above index their limbs with run-time widths, which puts them in per-lane scratch memory,
// where each limb operation waits on a memory round trip.

constexpr int SMALL_BITS = 80;

template <int WA>
__device__ __forceinline__ uint32_t fx_at(const uint32_t (&a)[WA], int k) {
    return k < WA ? a[k] : (uint32_t)((int32_t)a[WA - 1] >> 31);
}

// r = a - b or a + b modulo 2^(32 W); r may alias a
template <int W, int WA, int WB>
__device__ __forceinline__ void fx_addsub(uint32_t (&r)[W], const uint32_t (&a)[WA], const uint32_t (&b)[WB],
                                          bool sub) {
    unsigned long long c = sub ? 1ull : 0ull;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        const uint32_t bi = sub ? ~fx_at(b, i) : fx_at(b, i);
        const unsigned long long t = (unsigned long long)fx_at(a, i) + bi + c;
        r[i] = (uint32_t)t;
        c = t >> 32;
    }
}

// r = a * b modulo 2^(32 W); r must not alias a or b
template <int W, int WA, int WB>
__device__ __forceinline__ void fx_mul(uint32_t (&r)[W], const uint32_t (&a)[WA], const uint32_t (&b)[WB]) {
#pragma unroll
    for (int i = 0; i < W; ++i) r[i] = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        const uint32_t ai = fx_at(a, i);
        unsigned long long c = 0;
#pragma unroll
        for (int j = 0; i + j < W; ++j) {
            const unsigned long long t = (unsigned long long)ai * fx_at(b, j) + r[i + j] + c;
            r[i + j] = (uint32_t)t;
            c = t >> 32;
        }
    }
}

template <int W>
__device__ __forceinline__ int fx_sign(const uint32_t (&a)[W]) {
    if (a[W - 1] >> 31) return -1;
    uint32_t any = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) any |= a[i];
    return any ? 1 : 0;
}

// the N coordinates as three-limb integers m 2^(e - emin); false when the spread needs more
// than SMALL_BITS bits
template <int N>
__device__ __forceinline__ bool fx_load(const double (&v)[N], uint32_t (&X)[N][3]) {
    Dyadic d[N];
    int emin = 1 << 20, emax = -(1 << 20);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        d[i] = split_dyadic(v[i]);
        if (d[i].m != 0) {
            emin = min(emin, d[i].e);
            emax = max(emax, d[i].e);
        }
    }
    if (emax < emin) emin = emax = 0;
    if (emax - emin + 54 > SMALL_BITS) return false;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const unsigned long long mag = d[i].m < 0 ? (unsigned long long)(-d[i].m) : (unsigned long long)d[i].m;
        const int sh = d[i].m ? d[i].e - emin : 0;  // 0 .. SMALL_BITS - 54
        const unsigned long long lo = mag << sh;
        const uint32_t hi = sh ? (uint32_t)(mag >> (64 - sh)) : 0u;
        uint32_t r[3] = {(uint32_t)lo, (uint32_t)(lo >> 32), hi};
        if (d[i].m < 0) {
            unsigned long long c = 1;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const unsigned long long t = (unsigned long long)(uint32_t)~r[k] + c;
                r[k] = (uint32_t)t;
                c = t >> 32;
            }
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) X[i][k] = r[k];
    }
    return true;
}

// exact sign of orient3d for coordinates within SMALL_BITS (false: not within)
__device__ __forceinline__ bool orient3d_small(P3 a, P3 b, P3 c, P3 d, int *sign) {
    const double v[12] = {a.x, a.y, a.z, b.x, b.y, b.z, c.x, c.y, c.z, d.x, d.y, d.z};
    uint32_t X[12][3];
    if (!fx_load(v, X)) return false;
    // widths for SMALL_BITS = 80: differences 4 limbs, 2x2 minors 7, 3x3 determinant 9
    uint32_t D[9][4];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) fx_addsub(D[3 * r + k], X[3 * (r + 1) + k], X[k], true);
    uint32_t acc[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) acc[i] = 0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int i = q, j = (q + 1) % 3, k = (q + 2) % 3;
        uint32_t t1[7], t2[7], m[7], t3[9];
        fx_mul(t1, D[3 + j], D[6 + k]);
        fx_mul(t2, D[3 + k], D[6 + j]);
        fx_addsub(m, t1, t2, true);
        fx_mul(t3, D[i], m);
        fx_addsub(acc, acc, t3, false);
    }
    *sign = fx_sign(acc);
    return true;
}

// the common exponent of the N values (the smallest dyadic exponent of a non-zero one); false
// when the spread needs more than SMALL_BITS bits
template <int N>
__device__ __forceinline__ bool fx_range(const double (&v)[N], int *emin_out) {
    int emin = 1 << 20, emax = -(1 << 20);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const int ex = (int)(((unsigned long long)__double_as_longlong(v[i]) >> 52) & 0x7FF);
        if (ex != 0) {
            emin = min(emin, ex - 1075);
            emax = max(emax, ex - 1075);
        }
    }
    if (emax < emin) emin = emax = 0;
    *emin_out = emin;
    return emax - emin + 54 <= SMALL_BITS;
}

// x as a three-limb integer scaled by 2^-emin (the spread checked by fx_range)
__device__ __forceinline__ void fx_int(double x, int emin, uint32_t (&r)[3]) {
    const Dyadic d = split_dyadic(x);
    const unsigned long long mag = d.m < 0 ? (unsigned long long)(-d.m) : (unsigned long long)d.m;
    const int sh = d.m ? d.e - emin : 0;
    const unsigned long long lo = mag << sh;
    r[0] = (uint32_t)lo;
    r[1] = (uint32_t)(lo >> 32);
    r[2] = sh ? (uint32_t)(mag >> (64 - sh)) : 0u;
    if (d.m < 0) {
        unsigned long long c = 1;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const unsigned long long t = (unsigned long long)(uint32_t)~r[k] + c;
            r[k] = (uint32_t)t;
            c = t >> 32;
        }
    }
}

// exact sign of the lifted determinant (translated by e) for coordinates within SMALL_BITS.
// With rows p - e (p = a, b, c, d), the six 2x2 minors of their x and y columns serve all four
// 3x3 determinants, as in the fp64 filter.
__device__ __forceinline__ bool insphere_small(P3 a, P3 b, P3 c, P3 d, P3 e, int *sign) {
    const double v[15] = {a.x, a.y, a.z, b.x, b.y, b.z, c.x, c.y, c.z, d.x, d.y, d.z, e.x, e.y, e.z};
    int emin;
    if (!fx_range(v, &emin)) return false;
    // widths for SMALL_BITS = 80: differences 4 limbs, minors and lifts 7, 3x3 determinants 9,
    // the final sum 14
    uint32_t Dx[4][4], Dy[4][4], Dz[4][4];
    {
        uint32_t E[3][3];
#pragma unroll
        for (int k = 0; k < 3; ++k) fx_int(v[12 + k], emin, E[k]);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            uint32_t X[3];
            fx_int(v[3 * r], emin, X);
            fx_addsub(Dx[r], X, E[0], true);
            fx_int(v[3 * r + 1], emin, X);
            fx_addsub(Dy[r], X, E[1], true);
            fx_int(v[3 * r + 2], emin, X);
            fx_addsub(Dz[r], X, E[2], true);
        }
    }
    uint32_t L[4][7];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        uint32_t t[7];
        fx_mul(L[r], Dx[r], Dx[r]);
        fx_mul(t, Dy[r], Dy[r]);
        fx_addsub(L[r], L[r], t, false);
        fx_mul(t, Dz[r], Dz[r]);
        fx_addsub(L[r], L[r], t, false);
    }
    // minors m(p, q) = p_x q_y - q_x p_y for the pairs 01 02 03 12 13 23
    uint32_t M[6][7];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int p = k < 3 ? 0 : (k < 5 ? 1 : 2);
        const int q = k < 3 ? k + 1 : (k < 5 ? k - 1 : 3);
        uint32_t t1[7], t2[7];
        fx_mul(t1, Dx[p], Dy[q]);
        fx_mul(t2, Dx[q], Dy[p]);
        fx_addsub(M[k], t1, t2, true);
    }
    // det = l_d det3(a,b,c) - l_c det3(a,b,d) + l_b det3(a,c,d) - l_a det3(b,c,d), with
    // det3(p,q,s) = p_z m(q,s) - q_z m(p,s) + s_z m(p,q)
    uint32_t acc[14];
#pragma unroll
    for (int i = 0; i < 14; ++i) acc[i] = 0;
#pragma unroll
    for (int row = 0; row < 4; ++row) {
        const int p = row == 0 ? 1 : 0, q = row <= 1 ? 2 : 1, s = row <= 2 ? 3 : 2;
        // pair indices of (q, s), (p, s), (p, q)
        const int mqs = q == 1 ? 3 + (s - 2) : (q == 2 ? 5 : 0), mps = p == 0 ? s - 1 : 3 + (s - 2),
                  mpq = p == 0 ? q - 1 : 3;
        uint32_t det3[9], t[9];
        fx_mul(det3, Dz[p], M[mqs]);
        fx_mul(t, Dz[q], M[mps]);
        fx_addsub(det3, det3, t, true);
        fx_mul(t, Dz[s], M[mpq]);
        fx_addsub(det3, det3, t, false);
        uint32_t prod[14];
        fx_mul(prod, L[row], det3);
        fx_addsub(acc, acc, prod, row == 0 || row == 2);
    }
    *sign = fx_sign(acc);
    return true;
}

// exact sign of orient3d(a,b,c,d)
__device__ __noinline__ int orient3d_exact(P3 a, P3 b, P3 c, P3 d) {
    int sign;
    if (orient3d_small(a, b, c, d, &sign)) return sign;
    double v[12] = {a.x, a.y, a.z, b.x, b.y, b.z, c.x, c.y, c.z, d.x, d.y, d.z};
    uint32_t X[12][12];
    // coordinates: bits <= 53 + 239 + 1 (sign) -> at most 10 limbs
    int bits = ei_load(v, 12, X, 10);
    int w1 = (bits + 1 + 31) / 32 + 1;        // differences
    int w2 = (2 * bits + 3 + 31) / 32 + 1;    // 2x2 minors
    int w3 = (3 * bits + 6 + 31) / 32 + 1;    // 3x3 determinant
    w1 = min(w1, 12);
    w2 = min(w2, 24);
    w3 = min(w3, 36);
    uint32_t D[9][12];  // u = b-a, v = c-a, w = d-a
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) ei_addsub(D[3 * r + k], w1, X[3 * (r + 1) + k], 10, X[k], 10, true);
    // det = u.(v x w) = ux (vy wz - vz wy) + uy (vz wx - vx wz) + uz (vx wy - vy wx)
    uint32_t t1[24], t2[24], m[24], t3[36], acc[36];
    for (int i = 0; i < w3; ++i) acc[i] = 0;
    const int cyc[3][3] = {{0, 1, 2}, {1, 2, 0}, {2, 0, 1}};
    for (int q = 0; q < 3; ++q) {
        int i = cyc[q][0], j = cyc[q][1], k = cyc[q][2];
        ei_mul(t1, w2, D[3 + j], w1, D[6 + k], w1);
        ei_mul(t2, w2, D[3 + k], w1, D[6 + j], w1);
        ei_addsub(m, w2, t1, w2, t2, w2, true);
        ei_mul(t3, w3, D[i], w1, m, w2);
        ei_addsub(acc, w3, acc, w3, t3, w3, false);
    }
    return ei_sign(acc, w3);
}

// exact sign of the lifted determinant, translated by e
__device__ __noinline__ int insphere_exact(P3 a, P3 b, P3 c, P3 d, P3 e) {
    int sign;
    if (insphere_small(a, b, c, d, e, &sign)) return sign;
    double v[15] = {a.x, a.y, a.z, b.x, b.y, b.z, c.x, c.y, c.z, d.x, d.y, d.z, e.x, e.y, e.z};
    uint32_t X[15][12];
    int bits = ei_load(v, 15, X, 10);
    int w1 = min((bits + 1 + 31) / 32 + 1, 11);          // differences
    int w2 = min((2 * bits + 4 + 31) / 32 + 1, 21);      // minors and lifts
    int w3 = min((3 * bits + 7 + 31) / 32 + 1, 31);      // 3x3 determinants
    int w5 = min((5 * bits + 14 + 31) / 32 + 1, 48);     // final sum
    uint32_t D[12][11];  // rows p - e for p = a, b, c, d
    for (int r = 0; r < 4; ++r)
        for (int k = 0; k < 3; ++k) ei_addsub(D[3 * r + k], w1, X[3 * r + k], 10, X[12 + k], 10, true);
    // D = l_d det3(a,b,c) - l_c det3(a,b,d) + l_b det3(a,c,d) - l_a det3(b,c,d)
    const int others[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
    const bool neg[4] = {true, false, true, false};  // rows a, b, c, d
    uint32_t t1[21], t2[21], m[21], lift[21], tz[31], det3[31], prod[48], acc[48];
    for (int i = 0; i < w5; ++i) acc[i] = 0;
    for (int row = 0; row < 4; ++row) {
        int p = others[row][0], q = others[row][1], s = others[row][2];
        // det3(p,q,s) = p_z m(q,s) - q_z m(p,s) + s_z m(p,q),  m(x,y) = x_x y_y - y_x x_y
        for (int i = 0; i < w3; ++i) det3[i] = 0;
        const int zr[3] = {p, q, s};
        const int mr[3][2] = {{q, s}, {p, s}, {p, q}};
        for (int z = 0; z < 3; ++z) {
            int x0 = mr[z][0], y0 = mr[z][1];
            ei_mul(t1, w2, D[3 * x0 + 0], w1, D[3 * y0 + 1], w1);
            ei_mul(t2, w2, D[3 * y0 + 0], w1, D[3 * x0 + 1], w1);
            ei_addsub(m, w2, t1, w2, t2, w2, true);
            ei_mul(tz, w3, D[3 * zr[z] + 2], w1, m, w2);
            ei_addsub(det3, w3, det3, w3, tz, w3, z == 1);
        }
        for (int i = 0; i < w2; ++i) lift[i] = 0;
        for (int k = 0; k < 3; ++k) {
            ei_mul(t1, w2, D[3 * row + k], w1, D[3 * row + k], w1);
            ei_addsub(lift, w2, lift, w2, t1, w2, false);
        }
        ei_mul(prod, w5, lift, w2, det3, w3);
        ei_addsub(acc, w5, acc, w5, prod, w5, neg[row]);
    }
    return ei_sign(acc, w5);
}

// exact test of collinearity of a, b, c (cross product of b-a and c-a is zero)
__device__ __noinline__ bool collinear_exact(P3 a, P3 b, P3 c) {
    double v[9] = {a.x, a.y, a.z, b.x, b.y, b.z, c.x, c.y, c.z};
    uint32_t X[9][12];
    int bits = ei_load(v, 9, X, 10);
    int w1 = min((bits + 1 + 31) / 32 + 1, 12);
    int w2 = min((2 * bits + 3 + 31) / 32 + 1, 24);
    uint32_t U[3][12], V[3][12], t1[24], t2[24], cr[24];
    for (int k = 0; k < 3; ++k) {
        ei_addsub(U[k], w1, X[3 + k], 10, X[k], 10, true);
        ei_addsub(V[k], w1, X[6 + k], 10, X[k], 10, true);
    }
    for (int k = 0; k < 3; ++k) {
        int i = (k + 1) % 3, j = (k + 2) % 3;
        ei_mul(t1, w2, U[i], w1, V[j], w1);
        ei_mul(t2, w2, U[j], w1, V[i], w1);
        ei_addsub(cr, w2, t1, w2, t2, w2, true);
        if (ei_sign(cr, w2) != 0) return false;
    }
    return true;
}

// ------------------------------------------------------------------ certified fp64

// a - b, clearing ok unless it is exact (TwoSum remainder zero)
__device__ __forceinline__ double c_sub(double a, double b, bool &ok) {
    const double x = a - b;
    const double bv = a - x;
    const double av = x + bv;
    const double r = (a - av) + (bv - b);
    ok = ok && r == 0.0;
    return x;
}

__device__ __forceinline__ double c_add(double a, double b, bool &ok) {
    const double x = a + b;
    const double bv = x - a;
    const double av = x - bv;
    const double r = (a - av) + (b - bv);
    ok = ok && r == 0.0;
    return x;
}

__device__ __forceinline__ double c_mul(double a, double b, bool &ok) {
    const double p = a * b;
    ok = ok && fma(a, b, -p) == 0.0;
    return p;
}

// sign of orient3d if the fp64 evaluation is certified exact, else 2
__device__ __noinline__ int orient3d_cert(P3 a, P3 b, P3 c, P3 d) {
    bool ok = true;
    const double ux = c_sub(b.x, a.x, ok), uy = c_sub(b.y, a.y, ok), uz = c_sub(b.z, a.z, ok);
    const double vx = c_sub(c.x, a.x, ok), vy = c_sub(c.y, a.y, ok), vz = c_sub(c.z, a.z, ok);
    const double wx = c_sub(d.x, a.x, ok), wy = c_sub(d.y, a.y, ok), wz = c_sub(d.z, a.z, ok);
    const double m0 = c_sub(c_mul(vy, wz, ok), c_mul(vz, wy, ok), ok);
    const double m1 = c_sub(c_mul(vz, wx, ok), c_mul(vx, wz, ok), ok);
    const double m2 = c_sub(c_mul(vx, wy, ok), c_mul(vy, wx, ok), ok);
    const double det = c_add(c_add(c_mul(ux, m0, ok), c_mul(uy, m1, ok), ok), c_mul(uz, m2, ok), ok);
    if (!ok) return 2;
    return det > 0.0 ? 1 : (det < 0.0 ? -1 : 0);
}

// sign of the unperturbed lifted determinant (translated form) if certified exact, else 2
__device__ __noinline__ int insphere_cert(P3 a, P3 b, P3 c, P3 d, P3 e) {
    bool ok = true;
    const double ax = c_sub(a.x, e.x, ok), ay = c_sub(a.y, e.y, ok), az = c_sub(a.z, e.z, ok);
    const double bx = c_sub(b.x, e.x, ok), by = c_sub(b.y, e.y, ok), bz = c_sub(b.z, e.z, ok);
    const double cx = c_sub(c.x, e.x, ok), cy = c_sub(c.y, e.y, ok), cz = c_sub(c.z, e.z, ok);
    const double dx = c_sub(d.x, e.x, ok), dy = c_sub(d.y, e.y, ok), dz = c_sub(d.z, e.z, ok);
    if (!ok) return 2;
    const double ab = c_sub(c_mul(ax, by, ok), c_mul(bx, ay, ok), ok);
    const double ac = c_sub(c_mul(ax, cy, ok), c_mul(cx, ay, ok), ok);
    const double ad = c_sub(c_mul(ax, dy, ok), c_mul(dx, ay, ok), ok);
    const double bc = c_sub(c_mul(bx, cy, ok), c_mul(cx, by, ok), ok);
    const double bd = c_sub(c_mul(bx, dy, ok), c_mul(dx, by, ok), ok);
    const double cd = c_sub(c_mul(cx, dy, ok), c_mul(dx, cy, ok), ok);
    const double abc = c_add(c_sub(c_mul(az, bc, ok), c_mul(bz, ac, ok), ok), c_mul(cz, ab, ok), ok);
    const double abd = c_add(c_sub(c_mul(az, bd, ok), c_mul(bz, ad, ok), ok), c_mul(dz, ab, ok), ok);
    const double acd = c_add(c_sub(c_mul(az, cd, ok), c_mul(cz, ad, ok), ok), c_mul(dz, ac, ok), ok);
    const double bcd = c_add(c_sub(c_mul(bz, cd, ok), c_mul(cz, bd, ok), ok), c_mul(dz, bc, ok), ok);
    const double la = c_add(c_add(c_mul(ax, ax, ok), c_mul(ay, ay, ok), ok), c_mul(az, az, ok), ok);
    const double lb = c_add(c_add(c_mul(bx, bx, ok), c_mul(by, by, ok), ok), c_mul(bz, bz, ok), ok);
    const double lc = c_add(c_add(c_mul(cx, cx, ok), c_mul(cy, cy, ok), ok), c_mul(cz, cz, ok), ok);
    const double ld = c_add(c_add(c_mul(dx, dx, ok), c_mul(dy, dy, ok), ok), c_mul(dz, dz, ok), ok);
    const double det = c_add(c_sub(c_mul(ld, abc, ok), c_mul(lc, abd, ok), ok),
                             c_sub(c_mul(lb, acd, ok), c_mul(la, bcd, ok), ok), ok);
    if (!ok) return 2;
    return det > 0.0 ? 1 : (det < 0.0 ? -1 : 0);
}

// ------------------------------------------------------------------ filtered predicates

// sign of orient3d, or 2 when the fp64 filter cannot decide
__device__ __forceinline__ int orient3d_filter(P3 a, P3 b, P3 c, P3 d) {
    const double ux = b.x - a.x, uy = b.y - a.y, uz = b.z - a.z;
    const double vx = c.x - a.x, vy = c.y - a.y, vz = c.z - a.z;
    const double wx = d.x - a.x, wy = d.y - a.y, wz = d.z - a.z;
    const double det = ux * (vy * wz - vz * wy) + uy * (vz * wx - vx * wz) + uz * (vx * wy - vy * wx);
    double M = fmax(fmax(fmax(fabs(ux), fabs(uy)), fmax(fabs(uz), fabs(vx))),
                    fmax(fmax(fabs(vy), fabs(vz)), fmax(fmax(fabs(wx), fabs(wy)), fabs(wz))));
    const double bound = (M * M) * M * 0x1p-46;
    if (det > bound) return 1;
    if (-det > bound) return -1;
    if (M == 0.0) return 0;
    return 2;
}

__device__ __forceinline__ int orient3d(P3 a, P3 b, P3 c, P3 d, PredStats &st) {
    st.orient++;
    int s = orient3d_filter(a, b, c, d);
    if (s != 2) return s;
    st.orient_exact++;
    s = orient3d_cert(a, b, c, d);
    if (s != 2) return s;
    return orient3d_exact(a, b, c, d);
}

// sign of the unperturbed lifted determinant, or 2 when the filter cannot decide
__device__ __forceinline__ int insphere_filter(P3 a, P3 b, P3 c, P3 d, P3 e) {
    const double ax = a.x - e.x, ay = a.y - e.y, az = a.z - e.z;
    const double bx = b.x - e.x, by = b.y - e.y, bz = b.z - e.z;
    const double cx = c.x - e.x, cy = c.y - e.y, cz = c.z - e.z;
    const double dx = d.x - e.x, dy = d.y - e.y, dz = d.z - e.z;
    // 2x2 minors m(p,q) = p_x q_y - q_x p_y
    const double ab = ax * by - bx * ay, ac = ax * cy - cx * ay, ad = ax * dy - dx * ay;
    const double bc = bx * cy - cx * by, bd = bx * dy - dx * by, cd = cx * dy - dx * cy;
    // 3x3 determinants det3(p,q,s) = p_z m(q,s) - q_z m(p,s) + s_z m(p,q)
    const double abc = az * bc - bz * ac + cz * ab;
    const double abd = az * bd - bz * ad + dz * ab;
    const double acd = az * cd - cz * ad + dz * ac;
    const double bcd = bz * cd - cz * bd + dz * bc;
    const double la = ax * ax + ay * ay + az * az;
    const double lb = bx * bx + by * by + bz * bz;
    const double lc = cx * cx + cy * cy + cz * cz;
    const double ld = dx * dx + dy * dy + dz * dz;
    const double det = (ld * abc - lc * abd) + (lb * acd - la * bcd);
    const double M = fmax(fmax(fmax(fmax(fabs(ax), fabs(ay)), fmax(fabs(az), fabs(bx))),
                               fmax(fmax(fabs(by), fabs(bz)), fmax(fabs(cx), fabs(cy)))),
                          fmax(fmax(fabs(cz), fabs(dx)), fmax(fabs(dy), fabs(dz))));
    const double M2 = M * M;
    const double bound = (M2 * M2) * M * 0x1p-41;
    if (det > bound) return 1;
    if (-det > bound) return -1;
    if (M == 0.0) return 0;
    return 2;
}

__device__ __forceinline__ int insphere_raw(P3 a, P3 b, P3 c, P3 d, P3 e, PredStats &st) {
    st.insphere++;
    int s = insphere_filter(a, b, c, d, e);
    if (s != 2) return s;
    st.insphere_exact++;
    s = insphere_cert(a, b, c, d, e);
    if (s != 2) return s;
    return insphere_exact(a, b, c, d, e);
}

// sign of the perturbed lifted determinant of rows (a,b,c,d,e) with perturbation keys
// key[0..4] (input indices); requires orient3d(a,b,c,d) > 0.  -1 means e is inside.
__device__ __noinline__ int insphere_perturbed_tail(P3 a, P3 b, P3 c, P3 d, P3 e, const unsigned long long *key,
                                                    PredStats *st) {
    P3 p[5] = {a, b, c, d, e};
    bool used[5] = {false, false, false, false, false};
    for (int q = 0; q < 5; ++q) {
        int r = -1;
        for (int i = 0; i < 5; ++i)
            if (!used[i] && (r < 0 || key[i] > key[r])) r = i;
        used[r] = true;
        P3 o[4];
        int k = 0;
        for (int i = 0; i < 5; ++i)
            if (i != r) o[k++] = p[i];
        int s = orient3d(o[0], o[1], o[2], o[3], *st);
        if (s != 0) return (r & 1) ? -s : s;
    }
    return 1;  // unreachable: row e's cofactor is orient3d(a,b,c,d) > 0
}

// Perturbed insphere with the keys supplied by `keys(k)` (called only when the unperturbed
// determinant is zero), k = 0..4 for rows a..e.
template <class Keys>
__device__ __forceinline__ int insphere_perturbed(P3 a, P3 b, P3 c, P3 d, P3 e, Keys keys, PredStats &st) {
    int s = insphere_raw(a, b, c, d, e, st);
    if (s != 0) return s;
    st.perturbed++;
    unsigned long long key[5];
    for (int k = 0; k < 5; ++k) key[k] = keys(k);
    return insphere_perturbed_tail(a, b, c, d, e, key, &st);
}

// ------------------------------------------------------------------ cached sub-determinants

// Sec. 2.4 caches four sub-determinants per tetrahedron so that insphere becomes a dot
// product.  For a positive tetrahedron (a, b, c, d) with u = b - a, v = c - a, w = d - a and
// the lifts |u|^2, |v|^2, |w|^2, the lifted 5x5 determinant with a fifth point e is
// det = x . C with x = (e - a, |e - a|^2) and C = (-M1, M2, -M3, M4), Mk the 3x3 minor of
// [u |u|^2; v |v|^2; w |w|^2] without column k (M4 = orient3d(a, b, c, d)).  The record also
// keeps m, the largest magnitude of the nine rounded differences, which the filter's error
// bound needs; a query then reads a and the record, not b, c and d.
struct SubD {
    double c[4];
    double m;
};

__device__ __forceinline__ double det3r(double p0, double p1, double p2, double q0, double q1, double q2, double r0,
                                        double r1, double r2) {
    return p0 * (q1 * r2 - q2 * r1) - p1 * (q0 * r2 - q2 * r0) + p2 * (q0 * r1 - q1 * r0);
}

__device__ __forceinline__ SubD subdets(P3 a, P3 b, P3 c, P3 d) {
    const double ux = b.x - a.x, uy = b.y - a.y, uz = b.z - a.z;
    const double vx = c.x - a.x, vy = c.y - a.y, vz = c.z - a.z;
    const double wx = d.x - a.x, wy = d.y - a.y, wz = d.z - a.z;
    const double lu = ux * ux + uy * uy + uz * uz, lv = vx * vx + vy * vy + vz * vz, lw = wx * wx + wy * wy + wz * wz;
    SubD r;
    r.c[0] = -det3r(uy, uz, lu, vy, vz, lv, wy, wz, lw);
    r.c[1] = det3r(ux, uz, lu, vx, vz, lv, wx, wz, lw);
    r.c[2] = -det3r(ux, uy, lu, vx, vy, lv, wx, wy, lw);
    r.c[3] = det3r(ux, uy, uz, vx, vy, vz, wx, wy, wz);
    r.m = fmax(fmax(fmax(fabs(ux), fabs(uy)), fmax(fabs(uz), fabs(vx))),
               fmax(fmax(fmax(fabs(vy), fabs(vz)), fmax(fabs(wx), fabs(wy))), fabs(wz)));
    return r;
}

// Sign of the lifted determinant of (a, b, c, d, e) from the cached record of (a, b, c, d), or
// 2 when the fp64 filter cannot decide.  Error bound: each cached minor's monomials (two
// rounded differences and one rounded lift) carry at most 13 roundings, so with M the largest
// magnitude of the rounded differences b - a, c - a, d - a, e - a, |C1..3| <= 18 M^4 and
// |C4| <= 6 M^3 are off by at most gamma_13 of that; the query's differences add one rounding
// and its lift five; the dot product seven.  The sum stays below 1400 u M^5 < 2^-42 M^5; the
// filter uses 2^-40 M^5.
__device__ __forceinline__ int insphere_cached(const SubD &C, P3 a, P3 e) {
    const double x0 = e.x - a.x, x1 = e.y - a.y, x2 = e.z - a.z;
    const double x3 = x0 * x0 + x1 * x1 + x2 * x2;
    const double det = ((x0 * C.c[0] + x1 * C.c[1]) + x2 * C.c[2]) + x3 * C.c[3];
    const double M = fmax(fmax(C.m, fabs(x0)), fmax(fabs(x1), fabs(x2)));
    const double M2 = M * M;
    const double bound = (M2 * M2) * M * 0x1p-40;
    if (det > bound) return 1;
    if (-det > bound) return -1;
    return 2;
}

// filtered orient2d-free collinearity test used only by the initial tetrahedron search
__device__ __forceinline__ bool collinear(P3 a, P3 b, P3 c) {
    double ux = b.x - a.x, uy = b.y - a.y, uz = b.z - a.z;
    double vx = c.x - a.x, vy = c.y - a.y, vz = c.z - a.z;
    double c0a = uy * vz, c0b = uz * vy, c1a = uz * vx, c1b = ux * vz, c2a = ux * vy, c2b = uy * vx;
    // each component has 4 roundings: error < gamma_4/(1-gamma_4) * (|a|+|b|) < 2^-50 (..)
    if (fabs(c0a - c0b) > (fabs(c0a) + fabs(c0b)) * 0x1p-50) return false;
    if (fabs(c1a - c1b) > (fabs(c1a) + fabs(c1b)) * 0x1p-50) return false;
    if (fabs(c2a - c2b) > (fabs(c2a) + fabs(c2b)) * 0x1p-50) return false;
    return collinear_exact(a, b, c);
}

}  // namespace dtk
