// Delaunay refinement by circumcentre insertion (paper Sec. 4: the mesh generator inserts
// the circumcentres of tetrahedra larger than the size field, discarding points that would
// make short edges, in large concurrent sets through the same Delaunay kernel).
//
// One step over the current triangulation (the host driver in dt_capi.hip loops the steps):
//   k_circum     : every live finite tetrahedron with r^2 > (1.4 h)^2 proposes its
//                  circumcentre (one fixed fp64 formula, vertices in ascending input index,
//                  no contraction), with its sorted vertex indices as the tie-break; a
//                  tetrahedron unchanged since the last pass and not larger then is skipped;
//   k_inside     : the candidate is kept only strictly inside the convex hull: exact
//                  orient3d against every hull facet (the facets of the ghost tetrahedra);
//   (sort)       : candidates ordered by the Moore key of the point in the input's grid,
//                  then by the sorted vertex indices (radix sorts, dt_sort.hip);
//   k_near_vertex: a candidate closer than 0.7 h to a vertex is dropped (vertex grid of
//                  cells wider than 0.7 h, sorted cell keys, 9 rows of 3 cells);
//   k_filter_round: the greedy filter along that order (keep a candidate iff no kept earlier
//                  candidate is closer than 0.7 h) as rounds: a candidate is decided once every
//                  earlier candidate near it is, so each round decides at least the lowest
//                  undecided one and the result is the greedy one.
// The kept points are then inserted in filter order by the ordinary insertion rounds.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "dt_internal.h"
#include "dt_predicates.h"

namespace dtk {

// the facets of the ghost tetrahedra: (a, b, c) vertex records with the hull's interior on
// the negative side of orient3d(a, b, c, .)
template <class R>
__global__ void k_hull_facets(const R *__restrict__ T, uint32_t count, uint4 *__restrict__ facets,
                              uint32_t *__restrict__ nfacets) {
    const uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (t >= count) return;
    const uint4 w = T[t].v;
    if (w.x == DEAD || w.w != GHOST) return;
    facets[atomicAdd(nfacets, 1u)] = make_uint4(w.x, w.y, w.z, 0u);
}

// Slot of this thread in a list appended to by the threads with `want` set: one atomic per
// block, whose NW waves all call it (LDS: NW + 1 words).  Candidates are sparse but spread
// over the whole pool, and one counter takes about one atomic per 12 ns, so per-wave appends
// from a pass over ten million slots serialize for most of a millisecond.
template <int NW>
__device__ __forceinline__ uint32_t block_append(bool want, uint32_t *count, uint32_t *s_tmp) {
    const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x >> 6;
    const unsigned long long m = __ballot(want);
    if (lane == 0) s_tmp[wid] = (uint32_t)__popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < NW; ++w) {
            const uint32_t c = s_tmp[w];
            s_tmp[w] = t;
            t += c;
        }
        s_tmp[NW] = t ? atomicAdd(count, t) : 0u;
    }
    __syncthreads();
    const uint32_t r = s_tmp[NW] + s_tmp[wid] + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
    __syncthreads();  // s_tmp may be reused after
    return r;
}

__device__ __forceinline__ double dot3(const double *x, const double *y) {
    return x[0] * y[0] + x[1] * y[1] + x[2] * y[2];
}

__device__ __forceinline__ void cross3(const double *x, const double *y, double *r) {
    r[0] = x[1] * y[2] - x[2] * y[1];
    r[1] = x[2] * y[0] - x[0] * y[2];
    r[2] = x[0] * y[1] - x[1] * y[0];
}

// Circumcentre and squared radius of the tetrahedron with vertices p[0..3] (ascending input
// index): u = p1 - p0, v = p2 - p0, w = p3 - p0,
// off = (|u|^2 (v x w) + |v|^2 (w x u) + |w|^2 (u x v)) / (2 u . (v x w)), centre p0 + off,
// r^2 = off . off; every sum left to right (the library is compiled without contraction).
__device__ __forceinline__ void circumcentre(const double p[4][3], double *cc, double *r2) {
    double u[3], v[3], w[3], vw[3], wu[3], uv[3], off[3];
    for (int k = 0; k < 3; ++k) {
        u[k] = p[1][k] - p[0][k];
        v[k] = p[2][k] - p[0][k];
        w[k] = p[3][k] - p[0][k];
    }
    cross3(v, w, vw);
    cross3(w, u, wu);
    cross3(u, v, uv);
    const double den = 2.0 * dot3(u, vw);
    const double uu = dot3(u, u), vv = dot3(v, v), ww = dot3(w, w);
    for (int k = 0; k < 3; ++k) {
        const double num = uu * vw[k] + vv * wu[k] + ww * uv[k];
        off[k] = num / den;
        cc[k] = p[0][k] + off[k];
    }
    *r2 = dot3(off, off);
}

// live finite tetrahedra with r^2 > grow: candidate (circumcentre, sorted vertex input indices)
constexpr int CIRCUM_BLOCK = 1024;

template <class R>
__global__ __launch_bounds__(CIRCUM_BLOCK) void k_circum(const R *__restrict__ T, const Vert *__restrict__ V, uint32_t count, double grow,
                         uint4 *__restrict__ prev, uint8_t *__restrict__ pbig, uint32_t known,
                         double *__restrict__ cc, uint4 *__restrict__ q, uint32_t *__restrict__ src, uint32_t cap,
                         uint32_t *__restrict__ ncand) {
    const uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    uint4 w = make_uint4(DEAD, 0u, 0u, 0u);
    if (t < count) w = T[t].v;
    const bool live = w.x != DEAD && w.w != GHOST;
    // a slot holding the same four vertices as at the last pass holds the same tetrahedron
    // (a destroyed tetrahedron never returns: a later point lies inside its circumsphere);
    // one that was not larger than 1.4 h then is not now, and its vertices are not read
    bool keep_small = false;
    if (t < count) {
        if (t < known) {
            const uint4 pw = prev[t];
            keep_small = live && pw.x == w.x && pw.y == w.y && pw.z == w.z && pw.w == w.w && pbig[t] == 0;
        }
        prev[t] = w;
    }
    double c[3] = {0.0, 0.0, 0.0}, r2 = 0.0;
    uint32_t rec[4] = {w.x, w.y, w.z, w.w}, id[4] = {0u, 0u, 0u, 0u};
    if (live && !keep_small) {
        // the four records, read once, in ascending input index (insertion sort of four)
        double p[4][3];
        for (int k = 0; k < 4; ++k) {
            const Vert r = V[rec[k]];
            id[k] = (uint32_t)r.idx;
            p[k][0] = r.x;
            p[k][1] = r.y;
            p[k][2] = r.z;
        }
        for (int i = 1; i < 4; ++i)
            for (int j = i; j > 0 && id[j - 1] > id[j]; --j) {
                uint32_t x = id[j]; id[j] = id[j - 1]; id[j - 1] = x;
                x = rec[j]; rec[j] = rec[j - 1]; rec[j - 1] = x;
                for (int k = 0; k < 3; ++k) {
                    const double y = p[j][k]; p[j][k] = p[j - 1][k]; p[j - 1][k] = y;
                }
            }
        circumcentre(p, c, &r2);
    }
    const bool want = live && !keep_small && r2 > grow;
    if (t < count) pbig[t] = want ? 1 : 0;
    __shared__ uint32_t s_tmp[CIRCUM_BLOCK / 64 + 1];
    const uint32_t i = block_append<CIRCUM_BLOCK / 64>(want, ncand, s_tmp);
    if (!want || i >= cap) return;  // the host sizes cap to the live tetrahedra
    cc[3 * (size_t)i] = c[0];
    cc[3 * (size_t)i + 1] = c[1];
    cc[3 * (size_t)i + 2] = c[2];
    q[i] = make_uint4(id[0], id[1], id[2], id[3]);
    // a vertex of the tetrahedron: within its circumradius of the candidate, where the
    // candidate's insertion starts its walk
    src[i] = rec[0];
}

// strictly inside the hull: orient3d(a, b, c, x) < 0 for every hull facet.  k_inside_box
// takes the candidates in the inner box (a box whose corners were found strictly inside; the
// hull is convex) as inside without a test and lists the others, so that k_inside runs the
// facet tests over a compact list (the candidates come in slot order, which is spatially
// mixed: nearly every block would hold one outside the box).  The fp64 filter decides almost
// every test; a candidate it leaves undecided on some facet gets flag 2 and k_inside_exact
// settles it with the exact predicate (kept out of this kernel, whose registers it would
// take).  Candidates found inside are appended (compacted) to cc2 / q2 / src2.  The facets'
// corners pass through LDS in tiles shared by the block's candidates.
constexpr uint32_t INSIDE_TILE = 512;  // facets per tile: 512 x 9 doubles = 36 KB

__device__ __forceinline__ void inside_append(uint32_t i, bool in, P3 x, const uint4 *__restrict__ q,
                                              const uint32_t *__restrict__ src, double *__restrict__ cc2,
                                              uint4 *__restrict__ q2, uint32_t *__restrict__ src2,
                                              uint32_t *__restrict__ nin) {
    __shared__ uint32_t s_tmp[256 / 64 + 1];
    const uint32_t j = block_append<256 / 64>(in, nin, s_tmp);
    if (!in) return;
    cc2[3 * (size_t)j] = x.x;
    cc2[3 * (size_t)j + 1] = x.y;
    cc2[3 * (size_t)j + 2] = x.z;
    q2[j] = q[i];
    src2[j] = src[i];
}

__global__ __launch_bounds__(256) void k_inside_box(const double *__restrict__ cc, const uint4 *__restrict__ q,
                                                    const uint32_t *__restrict__ src, uint32_t k, InnerBox box,
                                                    uint8_t *__restrict__ flag, uint32_t *__restrict__ rest,
                                                    uint32_t *__restrict__ nrest, double *__restrict__ cc2,
                                                    uint4 *__restrict__ q2, uint32_t *__restrict__ src2,
                                                    uint32_t *__restrict__ nin) {
    __shared__ uint32_t s_tmp[256 / 64 + 1];
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    P3 x = {0.0, 0.0, 0.0};
    if (i < k) x = {cc[3 * (size_t)i], cc[3 * (size_t)i + 1], cc[3 * (size_t)i + 2]};
    const bool boxed = i < k && x.x >= box.lo[0] && x.x <= box.hi[0] && x.y >= box.lo[1] && x.y <= box.hi[1] &&
                       x.z >= box.lo[2] && x.z <= box.hi[2];
    if (i < k) flag[i] = 0;
    const uint32_t j = block_append<256 / 64>(i < k && !boxed, nrest, s_tmp);
    if (i < k && !boxed) rest[j] = i;
    inside_append(i, boxed, x, q, src, cc2, q2, src2, nin);
}

// lanes per listed candidate in k_inside, each testing every INSIDE_LANES-th facet: the list
// is short (the candidates near the hull), so one lane per candidate would leave most of the
// chip idle through the long facet loop
constexpr uint32_t INSIDE_LANES = 4;

__device__ __forceinline__ bool lanes_and(bool v) {
    int t = v ? 1 : 0;
    for (uint32_t m = 1; m < INSIDE_LANES; m <<= 1) t &= __shfl_xor(t, (int)m);
    return t != 0;
}

__device__ __forceinline__ bool lanes_or(bool v) {
    int t = v ? 1 : 0;
    for (uint32_t m = 1; m < INSIDE_LANES; m <<= 1) t |= __shfl_xor(t, (int)m);
    return t != 0;
}

__global__ __launch_bounds__(256) void k_inside(const Vert *__restrict__ V, const uint4 *__restrict__ facets,
                                                uint32_t nf, const double *__restrict__ cc,
                                                const uint4 *__restrict__ q, const uint32_t *__restrict__ src,
                                                const uint32_t *__restrict__ rest, const uint32_t *__restrict__ nrest,
                                                uint8_t *__restrict__ flag, double *__restrict__ cc2,
                                                uint4 *__restrict__ q2, uint32_t *__restrict__ src2,
                                                uint32_t *__restrict__ nin) {
    constexpr uint32_t PER_BLOCK = 256 / INSIDE_LANES;
    __shared__ double s_f[INSIDE_TILE][9];
    const uint32_t n = *nrest;
    if (blockIdx.x * PER_BLOCK >= n) return;  // the whole block: the list is shorter
    const uint32_t r = blockIdx.x * PER_BLOCK + threadIdx.x / INSIDE_LANES, l = threadIdx.x % INSIDE_LANES;
    const uint32_t i = r < n ? rest[r] : 0u;
    P3 x = {0.0, 0.0, 0.0};
    if (r < n) x = {cc[3 * (size_t)i], cc[3 * (size_t)i + 1], cc[3 * (size_t)i + 2]};
    // the sign of each facet decides on its own (inside iff negative on all; a facet the
    // filter leaves open matters only if none is decided non-negative), so the lanes split
    // the facets and combine at the end
    bool in = r < n, unsure = false;
    for (uint32_t f0 = 0; f0 < nf; f0 += INSIDE_TILE) {
        const uint32_t nt = min(INSIDE_TILE, nf - f0);
        // also the barrier before the tile is overwritten (the loop bounds are the block's)
        if (__syncthreads_or(in) == 0) break;
        for (uint32_t j = threadIdx.x; j < nt; j += blockDim.x) {
            const uint4 fa = facets[f0 + j];
            const Vert a = V[fa.x], b = V[fa.y], c = V[fa.z];
            s_f[j][0] = a.x; s_f[j][1] = a.y; s_f[j][2] = a.z;
            s_f[j][3] = b.x; s_f[j][4] = b.y; s_f[j][5] = b.z;
            s_f[j][6] = c.x; s_f[j][7] = c.y; s_f[j][8] = c.z;
        }
        __syncthreads();
        for (uint32_t j = l; j < nt && in; j += INSIDE_LANES) {
            const int o = orient3d_filter({s_f[j][0], s_f[j][1], s_f[j][2]}, {s_f[j][3], s_f[j][4], s_f[j][5]},
                                          {s_f[j][6], s_f[j][7], s_f[j][8]}, x);
            if (o == 2) unsure = true;
            else in = o < 0;
        }
        in = lanes_and(in);  // a lane that found the candidate outside stops the others
    }
    unsure = lanes_or(unsure);
    if (r < n && l == 0) flag[i] = in && unsure ? 2 : 0;
    inside_append(i, l == 0 && in && !unsure, x, q, src, cc2, q2, src2, nin);
}

// the candidates k_inside left undecided, with exact orient3d
__global__ __launch_bounds__(256) void k_inside_exact(const Vert *__restrict__ V, const uint4 *__restrict__ facets,
                                                      uint32_t nf, const double *__restrict__ cc,
                                                      const uint4 *__restrict__ q, const uint32_t *__restrict__ src,
                                                      uint32_t k, const uint8_t *__restrict__ flag,
                                                      double *__restrict__ cc2, uint4 *__restrict__ q2,
                                                      uint32_t *__restrict__ src2, uint32_t *__restrict__ nin) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    bool in = i < k && flag[i] == 2;
    P3 x = {0.0, 0.0, 0.0};
    if (in) {
        x = {cc[3 * (size_t)i], cc[3 * (size_t)i + 1], cc[3 * (size_t)i + 2]};
        PredStats st;
        for (uint32_t f = 0; f < nf && in; ++f) {
            const uint4 fa = facets[f];
            const Vert a = V[fa.x], b = V[fa.y], c = V[fa.z];
            in = orient3d({a.x, a.y, a.z}, {b.x, b.y, b.z}, {c.x, c.y, c.z}, x, st) < 0;
        }
    }
    inside_append(i, in, x, q, src, cc2, q2, src2, nin);
}

// sort keys in the order of perm: (q.z, q.w) (which = 0), (q.x, q.y) (which = 1), or the
// candidate's Moore key (which = 2)
__global__ void k_order_keys(const uint4 *__restrict__ q, const unsigned long long *__restrict__ moore,
                             const uint32_t *__restrict__ perm, uint32_t k, int which, int bits,
                             unsigned long long *__restrict__ keys, uint32_t *__restrict__ vals) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= k) return;
    const uint32_t i = perm ? perm[j] : j;
    const uint4 r = q[i];
    unsigned long long key;
    if (which == 0) key = ((unsigned long long)r.z << bits) | r.w;
    else if (which == 1) key = ((unsigned long long)r.x << bits) | r.y;
    else key = moore[i];
    keys[j] = key;
    vals[j] = i;
}

// ---- grids of cells wider than the filter distance

struct Grid {
    double lo[3];
    double cell;   // edge length, a little above 0.7 h
    uint64_t g;    // cells per axis
};

__device__ __forceinline__ long long cell_of(const Grid &G, double x, int k) {
    return (long long)floor((x - G.lo[k]) / G.cell);
}

__device__ __forceinline__ unsigned long long cell_key(const Grid &G, long long cx, long long cy, long long cz) {
    return (unsigned long long)cx + G.g * ((unsigned long long)cy + G.g * (unsigned long long)cz);
}

// cell key of each point (x at stride 3, or a vertex record)
__global__ void k_cell_keys_xyz(Grid G, const double *__restrict__ x, uint32_t n, unsigned long long *__restrict__ keys,
                                uint32_t *__restrict__ vals) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    keys[i] = cell_key(G, cell_of(G, x[3 * (size_t)i], 0), cell_of(G, x[3 * (size_t)i + 1], 1),
                       cell_of(G, x[3 * (size_t)i + 2], 2));
    vals[i] = i;
}

__global__ void k_cell_keys_vert(Grid G, const Vert *__restrict__ V, uint32_t n, unsigned long long *__restrict__ keys,
                                 uint32_t *__restrict__ vals) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Vert r = V[i];
    keys[i] = cell_key(G, cell_of(G, r.x, 0), cell_of(G, r.y, 1), cell_of(G, r.z, 2));
    vals[i] = i;
}

// first position in sorted keys[0, n) with keys[pos] >= key
__device__ __forceinline__ uint32_t lower_bound(const unsigned long long *keys, uint32_t n, unsigned long long key) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (keys[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// squared distance as the oracle takes it: (dx dx + dy dy) + dz dz
__device__ __forceinline__ double sq_dist(double ax, double ay, double az, double bx, double by, double bz) {
    const double dx = ax - bx, dy = ay - by, dz = az - bz;
    return dx * dx + dy * dy + dz * dz;
}

// The candidates in filter order: rank r is candidate perm[r]; ccr and srcr (rank order) get
// its point and its tetrahedron's vertex record; status 0 (undecided) unless a vertex is
// closer than the limit (2: dropped).
__global__ void k_near_vertex(Grid G, const Vert *__restrict__ V, const unsigned long long *__restrict__ vkeys,
                              const uint32_t *__restrict__ vidx, uint32_t nv, const double *__restrict__ cc,
                              const uint32_t *__restrict__ src, const uint32_t *__restrict__ perm, uint32_t k,
                              double lim, double *__restrict__ ccr, uint32_t *__restrict__ srcr,
                              uint8_t *__restrict__ status) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= k) return;
    const uint32_t i = perm[r];
    srcr[r] = src[i];
    const double x = cc[3 * (size_t)i], y = cc[3 * (size_t)i + 1], z = cc[3 * (size_t)i + 2];
    ccr[3 * (size_t)r] = x;
    ccr[3 * (size_t)r + 1] = y;
    ccr[3 * (size_t)r + 2] = z;
    const long long cx = cell_of(G, x, 0), cy = cell_of(G, y, 1), cz = cell_of(G, z, 2);
    bool close = false;
    for (long long dz = -1; dz <= 1 && !close; ++dz)
        for (long long dy = -1; dy <= 1 && !close; ++dy) {
            const long long yy = cy + dy, zz = cz + dz;
            if (yy < 0 || zz < 0 || yy >= (long long)G.g || zz >= (long long)G.g) continue;
            const long long x0 = cx > 0 ? cx - 1 : 0, x1 = cx + 1 < (long long)G.g ? cx + 1 : (long long)G.g - 1;
            uint32_t a = lower_bound(vkeys, nv, cell_key(G, x0, yy, zz));
            const unsigned long long kend = cell_key(G, x1, yy, zz);
            for (; a < nv && vkeys[a] <= kend && !close; ++a) {
                const Vert v = V[vidx[a]];
                close = sq_dist(v.x, v.y, v.z, x, y, z) < lim;
            }
        }
    status[r] = close ? 2 : 0;
}

// The earlier candidates (rank below r) closer than the limit: the three cells around the
// point in each of the 9 rows of cells about it, found by binary search over the candidates'
// sorted cell keys.  f(o) is called for each; returning false stops the search.
template <class F>
__device__ __forceinline__ void near_earlier(const Grid &G, const unsigned long long *__restrict__ ckeys,
                                             const uint32_t *__restrict__ crank, uint32_t k,
                                             const double *__restrict__ ccr, double lim, uint32_t r, F &&f) {
    const double x = ccr[3 * (size_t)r], y = ccr[3 * (size_t)r + 1], z = ccr[3 * (size_t)r + 2];
    const long long cx = cell_of(G, x, 0), cy = cell_of(G, y, 1), cz = cell_of(G, z, 2);
    for (long long dz = -1; dz <= 1; ++dz)
        for (long long dy = -1; dy <= 1; ++dy) {
            const long long yy = cy + dy, zz = cz + dz;
            if (yy < 0 || zz < 0 || yy >= (long long)G.g || zz >= (long long)G.g) continue;
            const long long x0 = cx > 0 ? cx - 1 : 0, x1 = cx + 1 < (long long)G.g ? cx + 1 : (long long)G.g - 1;
            uint32_t a = lower_bound(ckeys, k, cell_key(G, x0, yy, zz));
            const unsigned long long kend = cell_key(G, x1, yy, zz);
            for (; a < k && ckeys[a] <= kend; ++a) {
                const uint32_t o = crank[a];
                if (o >= r) continue;
                if (sq_dist(ccr[3 * (size_t)o], ccr[3 * (size_t)o + 1], ccr[3 * (size_t)o + 2], x, y, z) < lim &&
                    !f(o))
                    return;
            }
        }
}

// The list every filter round reads, built once per pass (it depends on the points and their
// order only): for each candidate still undecided, the earlier candidates closer than the
// limit that the vertex test did not drop, up to NEAR_MAX of them, stored as near[j * k + r];
// nnear[r] = their number, NEAR_MAX + 1 when there are more (that candidate searches the
// grid in every round instead).
constexpr uint32_t NEAR_MAX = FILTER_NEAR_MAX;

__global__ __launch_bounds__(256) void k_filter_near(Grid G, const unsigned long long *__restrict__ ckeys,
                                                     const uint32_t *__restrict__ crank, uint32_t k,
                                                     const double *__restrict__ ccr, double lim,
                                                     const uint8_t *__restrict__ status, uint32_t *__restrict__ near,
                                                     uint8_t *__restrict__ nnear) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= k) return;
    uint32_t c = 0;
    if (status[r] == 0)
        near_earlier(G, ckeys, crank, k, ccr, lim, r, [&](uint32_t o) {
            if (status[o] == 2) return true;  // dropped by a vertex: never counts
            if (c < NEAR_MAX) near[(size_t)c * k + r] = o;
            ++c;
            return c <= NEAR_MAX;
        });
    nnear[r] = (uint8_t)c;
}

// One round of the greedy filter over the candidates in rank order.  Candidate r (not yet
// decided) looks at the earlier candidates r' < r closer than the limit that are not dropped:
// any kept one drops r; none undecided keeps r; otherwise r waits.  Decisions never change,
// and a decision reads only earlier ranks, so reading a neighbour decided in this same round
// or the round before gives the same result.  *undecided becomes non-zero if any is left.
__global__ __launch_bounds__(256) void k_filter_round(Grid G, const unsigned long long *__restrict__ ckeys,
                                                      const uint32_t *__restrict__ crank, uint32_t k,
                                                      const double *__restrict__ ccr, double lim,
                                                      const uint32_t *__restrict__ near,
                                                      const uint8_t *__restrict__ nnear, uint8_t *status,
                                                      uint32_t *__restrict__ undecided) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    bool pending = false;
    if (r < k && __hip_atomic_load(&status[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
        bool kept_near = false;
        const uint32_t c = nnear[r];
        if (c <= NEAR_MAX) {
            for (uint32_t j = 0; j < c && !kept_near; ++j) {
                const uint8_t so = __hip_atomic_load(&status[near[(size_t)j * k + r]], __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
                if (so == 1) kept_near = true;
                else if (so == 0) pending = true;
            }
        } else {
            near_earlier(G, ckeys, crank, k, ccr, lim, r, [&](uint32_t o) {
                const uint8_t so = __hip_atomic_load(&status[o], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (so == 1) kept_near = true;
                else if (so == 0) pending = true;
                return !kept_near;
            });
        }
        if (kept_near) {
            pending = false;
            __hip_atomic_store(&status[r], (uint8_t)2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if (!pending) {
            __hip_atomic_store(&status[r], (uint8_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    // one flag per block: the host only asks whether any candidate is left undecided (one
    // counter takes about one atomic per 12 ns, and a first round leaves many)
    if (__syncthreads_or(pending) && threadIdx.x == 0) atomicOr(undecided, 1u);
}

// kept candidates in rank order: flag for the scan, then the points at their scanned positions
__global__ void k_kept_flags(const uint8_t *__restrict__ status, uint32_t k, uint32_t *__restrict__ flags) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < k) flags[r] = status[r] == 1 ? 1u : 0u;
}

__global__ void k_kept_points(const uint8_t *__restrict__ status, const uint32_t *__restrict__ pos, uint32_t k,
                              const double *__restrict__ ccr, const uint32_t *__restrict__ srcr,
                              double *__restrict__ out, uint32_t *__restrict__ hint) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= k || status[r] != 1) return;
    const uint32_t j = pos[r];
    for (int c = 0; c < 3; ++c) out[3 * (size_t)j + c] = ccr[3 * (size_t)r + c];
    hint[j] = srcr[r];
}

// bounding box of the vertex records [0, n): per-block partial boxes, then one thread folds
// them into the cloud's grid origin and cubic scale 2^m / (largest extent)
__global__ void k_vert_box(const Vert *__restrict__ V, uint32_t n, double *__restrict__ partial) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const Vert r = V[i];
        const double x[3] = {r.x, r.y, r.z};
        for (int k = 0; k < 3; ++k) {
            lo[k] = fmin(lo[k], x[k]);
            hi[k] = fmax(hi[k], x[k]);
        }
    }
    __shared__ double sh[6][256];
    for (int k = 0; k < 3; ++k) {
        sh[k][threadIdx.x] = lo[k];
        sh[3 + k][threadIdx.x] = hi[k];
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 3; ++k) {
                sh[k][threadIdx.x] = fmin(sh[k][threadIdx.x], sh[k][threadIdx.x + w]);
                sh[3 + k][threadIdx.x] = fmax(sh[3 + k][threadIdx.x], sh[3 + k][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) partial[6 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void k_box_final(const double *__restrict__ partial, uint32_t nb, uint32_t m, Cloud *__restrict__ cl) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (uint32_t b = 0; b < nb; ++b)
        for (int k = 0; k < 3; ++k) {
            lo[k] = fmin(lo[k], partial[6 * b + k]);
            hi[k] = fmax(hi[k], partial[6 * b + 3 + k]);
        }
    double ext = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double e = hi[k] - lo[k];
        if (e > ext) ext = e;
    }
    Cloud c{};
    c.lo = 0;
    c.hi = 0;
    c.m = m;
    c.box[0] = lo[0];
    c.box[1] = lo[1];
    c.box[2] = lo[2];
    c.box[3] = ext > 0.0 ? ldexp(1.0, (int)m) / ext : 0.0;
    *cl = c;
}

// ---- launch wrappers

static inline uint32_t blocks256(uint64_t n) { return (uint32_t)((n + 255) / 256); }

hipError_t launch_hull_facets(const void *T, bool wide, uint32_t count, uint4 *facets, uint32_t *nfacets,
                              hipStream_t s) {
    if (count == 0) return hipSuccess;
    if (wide) k_hull_facets<<<blocks256(count), 256, 0, s>>>((const TetW *)T, count, facets, nfacets);
    else k_hull_facets<<<blocks256(count), 256, 0, s>>>((const Tet *)T, count, facets, nfacets);
    return hipGetLastError();
}

hipError_t launch_circum(const void *T, bool wide, const Vert *V, uint32_t count, double grow, uint4 *prev,
                         uint8_t *pbig, uint32_t known, double *cc, uint4 *q, uint32_t *src, uint32_t cap,
                         uint32_t *ncand, hipStream_t s) {
    if (count == 0) return hipSuccess;
    const uint32_t nb = (uint32_t)((count + CIRCUM_BLOCK - 1) / CIRCUM_BLOCK);
    if (wide)
        k_circum<<<nb, CIRCUM_BLOCK, 0, s>>>((const TetW *)T, V, count, grow, prev, pbig, known, cc, q, src, cap,
                                             ncand);
    else
        k_circum<<<nb, CIRCUM_BLOCK, 0, s>>>((const Tet *)T, V, count, grow, prev, pbig, known, cc, q, src, cap,
                                             ncand);
    return hipGetLastError();
}

hipError_t launch_inside(const Vert *V, const uint4 *facets, uint32_t nf, const double *cc, const uint4 *q,
                         const uint32_t *src, uint32_t k, const InnerBox &box, uint32_t *rest, uint32_t *nrest,
                         uint8_t *flag, double *cc2, uint4 *q2, uint32_t *src2, uint32_t *nin, hipStream_t s) {
    if (k == 0) return hipSuccess;
    k_inside_box<<<blocks256(k), 256, 0, s>>>(cc, q, src, k, box, flag, rest, nrest, cc2, q2, src2, nin);
    k_inside<<<(uint32_t)(((uint64_t)k + 256 / INSIDE_LANES - 1) / (256 / INSIDE_LANES)), 256, 0, s>>>(
        V, facets, nf, cc, q, src, rest, nrest, flag, cc2, q2, src2, nin);
    k_inside_exact<<<blocks256(k), 256, 0, s>>>(V, facets, nf, cc, q, src, k, flag, cc2, q2, src2, nin);
    return hipGetLastError();
}

hipError_t launch_order_keys(const uint4 *q, const unsigned long long *moore, const uint32_t *perm, uint32_t k,
                             int which, int bits, unsigned long long *keys, uint32_t *vals, hipStream_t s) {
    if (k == 0) return hipSuccess;
    k_order_keys<<<blocks256(k), 256, 0, s>>>(q, moore, perm, k, which, bits, keys, vals);
    return hipGetLastError();
}

hipError_t launch_cell_keys(const double *lo, double cell, uint64_t g, const double *xyz, const Vert *V, uint32_t n,
                            unsigned long long *keys, uint32_t *vals, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const Grid G = {{lo[0], lo[1], lo[2]}, cell, g};
    if (V) k_cell_keys_vert<<<blocks256(n), 256, 0, s>>>(G, V, n, keys, vals);
    else k_cell_keys_xyz<<<blocks256(n), 256, 0, s>>>(G, xyz, n, keys, vals);
    return hipGetLastError();
}

hipError_t launch_near_vertex(const double *lo, double cell, uint64_t g, const Vert *V, const unsigned long long *vkeys,
                              const uint32_t *vidx, uint32_t nv, const double *cc, const uint32_t *src,
                              const uint32_t *perm, uint32_t k, double lim, double *ccr, uint32_t *srcr,
                              uint8_t *status, hipStream_t s) {
    if (k == 0) return hipSuccess;
    const Grid G = {{lo[0], lo[1], lo[2]}, cell, g};
    k_near_vertex<<<blocks256(k), 256, 0, s>>>(G, V, vkeys, vidx, nv, cc, src, perm, k, lim, ccr, srcr, status);
    return hipGetLastError();
}

hipError_t launch_filter_near(const double *lo, double cell, uint64_t g, const unsigned long long *ckeys,
                              const uint32_t *crank, uint32_t k, const double *ccr, double lim, const uint8_t *status,
                              uint32_t *near, uint8_t *nnear, hipStream_t s) {
    if (k == 0) return hipSuccess;
    const Grid G = {{lo[0], lo[1], lo[2]}, cell, g};
    k_filter_near<<<blocks256(k), 256, 0, s>>>(G, ckeys, crank, k, ccr, lim, status, near, nnear);
    return hipGetLastError();
}

hipError_t launch_filter_round(const double *lo, double cell, uint64_t g, const unsigned long long *ckeys,
                               const uint32_t *crank, uint32_t k, const double *ccr, double lim, const uint32_t *near,
                               const uint8_t *nnear, uint8_t *status, uint32_t *undecided, hipStream_t s) {
    if (k == 0) return hipSuccess;
    const Grid G = {{lo[0], lo[1], lo[2]}, cell, g};
    k_filter_round<<<blocks256(k), 256, 0, s>>>(G, ckeys, crank, k, ccr, lim, near, nnear, status, undecided);
    return hipGetLastError();
}

hipError_t launch_kept(const uint8_t *status, uint32_t k, uint32_t *flags, const uint32_t *pos, const double *ccr,
                       const uint32_t *srcr, double *out, uint32_t *hint, int phase, hipStream_t s) {
    if (k == 0) return hipSuccess;
    if (phase == 0) k_kept_flags<<<blocks256(k), 256, 0, s>>>(status, k, flags);
    else k_kept_points<<<blocks256(k), 256, 0, s>>>(status, pos, k, ccr, srcr, out, hint);
    return hipGetLastError();
}

hipError_t launch_vert_box(const Vert *V, uint32_t n, uint32_t m, double *partial, uint32_t nblocks, Cloud *cl,
                           hipStream_t s) {
    k_vert_box<<<nblocks, 256, 0, s>>>(V, n, partial);
    k_box_final<<<1, 64, 0, s>>>(partial, nblocks, m, cl);
    return hipGetLastError();
}

}  // namespace dtk
