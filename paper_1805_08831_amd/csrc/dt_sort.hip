// Point ingest and spatial sort (paper Sec. 2.1 "Sort", Sec. 2.3).
//
// validate + bounding box -> Moore key and BRIO level per point -> stable LSD radix sort of
// (Moore index, input index) -> 32-byte vertex records in Moore order -> BRIO level of
// each record and the level-major order of the records (a one-pass counting sort) -> exact
// duplicate removal by hashing.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "dt_internal.h"

namespace dtk {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ bool coord_ok(double x) {
    // 0, or finite with |x| in [2^-120, 2^120)
    double a = fabs(x);
    return a == 0.0 || (a >= 0x1p-120 && a < 0x1p120);
}

// exclusive scan across a 256-thread block; returns the prefix, *total the block sum
__device__ uint32_t block_scan_256(uint32_t v, uint32_t *total) {
    __shared__ uint32_t wsum[4];
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int w = 0; w < 4; ++w) {
        if (w < wave) before += wsum[w];
        all += wsum[w];
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}

// ------------------------------------------------------------------ validate + bbox

__global__ void k_validate_bbox(const double *__restrict__ xyz, uint64_t n, double *__restrict__ blocks,
                                uint32_t *__restrict__ err) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    bool ok = true;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        for (int k = 0; k < 3; ++k) {
            double v = xyz[3 * i + k];
            ok = ok && coord_ok(v);
            lo[k] = fmin(lo[k], v);
            hi[k] = fmax(hi[k], v);
        }
    }
    if (!ok) atomicOr(err, ERR_INPUT);
    __shared__ double s[6][256];
    for (int k = 0; k < 3; ++k) {
        s[k][threadIdx.x] = lo[k];
        s[3 + k][threadIdx.x] = hi[k];
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 3; ++k) {
                s[k][threadIdx.x] = fmin(s[k][threadIdx.x], s[k][threadIdx.x + w]);
                s[3 + k][threadIdx.x] = fmax(s[3 + k][threadIdx.x], s[3 + k][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) blocks[6 * blockIdx.x + threadIdx.x] = s[threadIdx.x][0];
}

__global__ void k_bbox_final(const double *__restrict__ blocks, int nb, double *__restrict__ out) {
    if (threadIdx.x >= 6) return;
    int k = threadIdx.x;
    double v = k < 3 ? INFINITY : -INFINITY;
    for (int b = 0; b < nb; ++b) v = k < 3 ? fmin(v, blocks[6 * b + k]) : fmax(v, blocks[6 * b + k]);
    out[k] = v;
}

hipError_t launch_validate_bbox(const double *xyz, uint64_t n, double *bbox_blocks, int nblocks,
                                double *bbox_out, uint32_t *err, hipStream_t s) {
    k_validate_bbox<<<nblocks, 256, 0, s>>>(xyz, n, bbox_blocks, err);
    k_bbox_final<<<1, 64, 0, s>>>(bbox_blocks, nblocks, bbox_out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Moore key + level

// Hilbert sub-curve transitions (Hamilton): entry corner and direction of sub-cube w
__device__ __forceinline__ unsigned rot_left3(unsigned x, unsigned r) { return ((x << r) | (x >> (3 - r))) & 7u; }
__device__ __forceinline__ unsigned rot_right3(unsigned x, unsigned r) { return ((x >> r) | (x << (3 - r))) & 7u; }

__host__ __device__ constexpr unsigned gray3(unsigned i) { return i ^ (i >> 1); }
__host__ __device__ constexpr unsigned ones_below(unsigned i) { return (i & 1u) ? 1u + ones_below(i >> 1) : 0u; }
__host__ __device__ constexpr unsigned hil_entry(unsigned w) { return w == 0 ? 0u : gray3(2u * ((w - 1u) / 2u)); }
__host__ __device__ constexpr unsigned hil_dir(unsigned w) {
    return w == 0 ? 0u : ((w % 2u == 0u ? ones_below(w - 1u) : ones_below(w)) % 3u);
}

// packed per-octant Moore states: bits [5w, 5w+3) entry corner, [5w+3, 5w+5) direction
static unsigned long long g_moore_states = 0;

static unsigned long long moore_states() {
    if (g_moore_states) return g_moore_states;
    // the first (e0, d0..d7) in lexicographic order chaining the 8 Hilbert sub-curves, in
    // Gray-code octant order, into a closed curve (exit cell of octant w face-adjacent to
    // the entry cell of octant w+1, octant 7 back to octant 0)
    for (unsigned e0 = 0; e0 < 8; ++e0)
        for (unsigned code = 0; code < 6561u; ++code) {
            unsigned d[8], c = code;
            for (int w = 7; w >= 0; --w) { d[w] = c % 3u; c /= 3u; }
            unsigned e = e0, es[8];
            bool ok = true;
            for (unsigned w = 0; w < 8 && ok; ++w) {
                es[w] = e;
                unsigned exitc = e ^ (1u << d[w]);
                unsigned nxt = gray3((w + 1u) & 7u), axis_bit = gray3(w) ^ nxt;
                unsigned axis = axis_bit == 1u ? 0u : (axis_bit == 2u ? 1u : 2u);
                if (((exitc >> axis) & 1u) != ((nxt >> axis) & 1u)) ok = false;
                e = exitc ^ (1u << axis);
            }
            if (ok && e == e0) {
                unsigned long long packed = 0;
                for (int w = 0; w < 8; ++w)
                    packed |= (unsigned long long)(es[w] | (d[w] << 3)) << (5 * w);
                g_moore_states = packed | (1ull << 63);
                return g_moore_states;
            }
        }
    return 0;
}

__device__ __forceinline__ unsigned long long moore_index(unsigned cx, unsigned cy, unsigned cz, int m,
                                                          unsigned long long states) {
    unsigned o = ((cx >> (m - 1)) & 1u) | (((cy >> (m - 1)) & 1u) << 1) | (((cz >> (m - 1)) & 1u) << 2);
    unsigned w = o ^ (o >> 1) ^ (o >> 2);  // position of octant o in the Gray-code cycle
    unsigned long long h = w;
    unsigned st = (unsigned)(states >> (5 * w)) & 31u;
    unsigned e = st & 7u, d = st >> 3;
    for (int i = m - 2; i >= 0; --i) {
        unsigned l = ((cx >> i) & 1u) | (((cy >> i) & 1u) << 1) | (((cz >> i) & 1u) << 2);
        l = rot_right3(l ^ e, (d + 1u) % 3u);
        unsigned ww = l ^ (l >> 1) ^ (l >> 2);
        e ^= rot_left3(hil_entry(ww), (d + 1u) % 3u);
        d = (d + hil_dir(ww) + 1u) % 3u;
        h = (h << 3) | ww;
    }
    return h;
}

__global__ void k_keys(const double *__restrict__ xyz, uint64_t n, const double *__restrict__ bbox, int m,
                       unsigned long long salt, const uint64_t *__restrict__ cum, int L,
                       unsigned long long states, unsigned long long *__restrict__ keys,
                       uint32_t *__restrict__ vals) {
    uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double ext = 0.0;
    for (int k = 0; k < 3; ++k) {
        double e = bbox[3 + k] - bbox[k];
        if (e > ext) ext = e;
    }
    double cells = ldexp(1.0, m);
    double sc = ext > 0.0 ? cells / ext : 0.0;
    unsigned top = (1u << m) - 1u, c[3];
    for (int k = 0; k < 3; ++k) {
        double t = floor((xyz[3 * i + k] - bbox[k]) * sc);
        c[k] = t >= (double)top ? top : (unsigned)t;
    }
    unsigned long long key = moore_index(c[0], c[1], c[2], m, states);
    // BRIO level: 53 uniform bits u; level = first k with u * n < cum_k * 2^53
    unsigned long long u = mix64(salt + i) >> 11;
    int lev = 0;
    while (lev < L - 1) {
        unsigned long long lo = u * n, hi = __umul64hi(u, n);
        unsigned long long clo = (unsigned long long)cum[lev] << 53, chi = (unsigned long long)cum[lev] >> 11;
        bool less = hi < chi || (hi == chi && lo < clo);
        if (less) break;
        ++lev;
    }
    keys[i] = ((unsigned long long)lev << (3 * m)) | key;
    vals[i] = (uint32_t)i;
}

hipError_t launch_keys(const double *xyz, uint64_t n, const double *bbox, int m, uint64_t salt,
                       const uint64_t *cum, int L, unsigned long long *keys, uint32_t *vals, hipStream_t s) {
    unsigned long long st = moore_states();
    if (!st) return hipErrorUnknown;
    if (n == 0) return hipSuccess;
    k_keys<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(xyz, n, bbox, m, salt, cum, L, st, keys, vals);
    return hipGetLastError();
}

// BRIO level of the point at each Moore-sorted position (src[i] = its index within the
// call), as the key of a stable counting sort that yields the level-major order of the
// positions; vals[i] = base + i
__global__ void k_levels(const uint32_t *__restrict__ src, uint64_t n, uint64_t base,
                         unsigned long long salt, const uint64_t *__restrict__ cum, int L,
                         unsigned long long *__restrict__ keys, uint32_t *__restrict__ vals) {
    uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const unsigned long long u = mix64(salt + (unsigned long long)src[i]) >> 11;
    int lev = 0;
    while (lev < L - 1) {
        unsigned long long lo = u * n, hi = __umul64hi(u, n);
        unsigned long long clo = (unsigned long long)cum[lev] << 53, chi = (unsigned long long)cum[lev] >> 11;
        if (hi < chi || (hi == chi && lo < clo)) break;
        ++lev;
    }
    keys[i] = (unsigned long long)lev;
    vals[i] = (uint32_t)(base + i);
}

hipError_t launch_levels(const uint32_t *src, uint64_t n, uint64_t base, uint64_t salt, const uint64_t *cum,
                         int L, unsigned long long *keys, uint32_t *vals, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_levels<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(src, n, base, salt, cum, L, keys, vals);
    return hipGetLastError();
}

// Walk anchor of every record of level k >= 1: the record of the nearest non-empty lower
// level that precedes it on the curve (else that level's first record).  lord lists each
// level's positions in increasing order; anchor is indexed by position - base.
__global__ void k_anchor(const uint32_t *__restrict__ lord, const uint32_t *__restrict__ start, int L,
                         uint64_t base, uint64_t n, uint32_t *__restrict__ anchor) {
    const uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (j >= n) return;
    int k = 0;
    while (k + 1 < L && start[k + 1] <= j) ++k;
    const uint32_t p = lord[j];
    int kk = k - 1;
    while (kk >= 0 && start[kk + 1] == start[kk]) --kk;
    if (kk < 0) {
        anchor[p - base] = 0xFFFFFFFFu;
        return;
    }
    uint32_t lo = start[kk], hi = start[kk + 1];  // last entry < p in [lo, hi), else lo
    uint32_t res = lo;
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (lord[mid] < p) {
            res = mid;
            lo = mid + 1;
        } else {
            hi = mid;
        }
    }
    anchor[p - base] = lord[res];
}

hipError_t launch_anchor(const uint32_t *lord, const uint32_t *start, int L, uint64_t base, uint64_t n,
                         uint32_t *anchor, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_anchor<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(lord, start, L, base, n, anchor);
    return hipGetLastError();
}

// ------------------------------------------------------------------ scan

constexpr int SCAN_TILE = 1024;  // 256 threads x 4 items

size_t scan_tmp_entries(uint64_t n) { return (size_t)((n + SCAN_TILE - 1) / SCAN_TILE) + 1; }

__global__ void k_scan_reduce(const uint32_t *__restrict__ in, uint64_t n, uint32_t *__restrict__ sums) {
    uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
    uint32_t v = 0;
    for (int k = 0; k < 4; ++k) {
        uint64_t e = base + threadIdx.x * 4 + k;
        if (e < n) v += in[e];
    }
    uint32_t tot;
    block_scan_256(v, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void k_scan_sums(uint32_t *__restrict__ sums, uint64_t nb, uint32_t *__restrict__ total) {
    uint32_t carry = 0;
    for (uint64_t base = 0; base < nb; base += 256) {
        uint64_t e = base + threadIdx.x;
        uint32_t v = e < nb ? sums[e] : 0, tot;
        uint32_t ex = block_scan_256(v, &tot);
        if (e < nb) sums[e] = carry + ex;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

__global__ void k_scan_apply(const uint32_t *__restrict__ in, uint32_t *__restrict__ out, uint64_t n,
                             const uint32_t *__restrict__ sums) {
    uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
    uint32_t v[4], s = 0;
    for (int k = 0; k < 4; ++k) {
        uint64_t e = base + threadIdx.x * 4 + k;
        v[k] = e < n ? in[e] : 0;
        s += v[k];
    }
    uint32_t tot;
    uint32_t ex = block_scan_256(s, &tot) + sums[blockIdx.x];
    for (int k = 0; k < 4; ++k) {
        uint64_t e = base + threadIdx.x * 4 + k;
        if (e < n) out[e] = ex;
        ex += v[k];
    }
}

hipError_t exclusive_scan_u32(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *tmp, uint32_t *total,
                              hipStream_t s) {
    uint64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 0) nb = 1;
    k_scan_reduce<<<(unsigned)nb, 256, 0, s>>>(in, n, tmp);
    k_scan_sums<<<1, 256, 0, s>>>(tmp, nb, total);
    k_scan_apply<<<(unsigned)nb, 256, 0, s>>>(in, out, n, tmp);
    return hipGetLastError();
}

// ------------------------------------------------------------------ LSD radix sort

constexpr int RS_ITEMS = 8;
constexpr int RS_TILE = 256 * RS_ITEMS;

size_t radix_hist_entries(uint64_t n) { return 256 * (size_t)((n + RS_TILE - 1) / RS_TILE + 1); }

__global__ void k_rs_hist(const unsigned long long *__restrict__ keys, uint64_t n, int shift,
                          uint32_t *__restrict__ hist, uint32_t nblocks) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    uint64_t base = (uint64_t)blockIdx.x * RS_TILE;
    for (int it = 0; it < RS_ITEMS; ++it) {
        uint64_t e = base + it * 256 + threadIdx.x;
        if (e < n) atomicAdd(&h[(keys[e] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// stable scatter: the tile is processed in its index order (it, thread); equal digits keep
// their order through per-wave match masks and per-wave digit counts
__global__ void k_rs_scatter(const unsigned long long *__restrict__ kin, const uint32_t *__restrict__ vin,
                             unsigned long long *__restrict__ kout, uint32_t *__restrict__ vout, uint64_t n,
                             int shift, const uint32_t *__restrict__ offsets, uint32_t nblocks) {
    __shared__ uint32_t off[256];
    __shared__ uint32_t wt[4][256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    off[threadIdx.x] = offsets[threadIdx.x * nblocks + blockIdx.x];
    for (int w = 0; w < 4; ++w) wt[w][threadIdx.x] = 0;
    __syncthreads();
    uint64_t base = (uint64_t)blockIdx.x * RS_TILE;
    const unsigned long long lt = (1ull << lane) - 1ull;
    for (int it = 0; it < RS_ITEMS; ++it) {
        uint64_t e = base + it * 256 + threadIdx.x;
        bool valid = e < n;
        unsigned long long key = valid ? kin[e] : 0ull;
        uint32_t val = valid ? vin[e] : 0u;
        unsigned d = (unsigned)(key >> shift) & 255u;
        unsigned long long mask = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            bool bit = (d >> b) & 1u;
            unsigned long long bb = __ballot(valid && bit);
            mask &= bit ? bb : ~bb;
        }
        unsigned rank = (unsigned)__popcll(mask & lt);
        if (valid && rank == 0) wt[wave][d] = (unsigned)__popcll(mask);
        __syncthreads();
        if (valid) {
            uint32_t pre = 0;
            for (int w = 0; w < wave; ++w) pre += wt[w][d];
            uint32_t pos = off[d] + pre + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        off[threadIdx.x] += wt[0][threadIdx.x] + wt[1][threadIdx.x] + wt[2][threadIdx.x] + wt[3][threadIdx.x];
        for (int w = 0; w < 4; ++w) wt[w][threadIdx.x] = 0;
        __syncthreads();
    }
}

hipError_t radix_sort_pairs(unsigned long long *keys, uint32_t *vals, unsigned long long *keys_tmp,
                            uint32_t *vals_tmp, uint32_t *hist, uint32_t *scan_tmp, uint64_t n, int nbits,
                            hipStream_t s, bool *swapped) {
    *swapped = false;
    if (n <= 1 || nbits <= 0) return hipSuccess;
    uint32_t nb = (uint32_t)((n + RS_TILE - 1) / RS_TILE);
    unsigned long long *ka = keys, *kb = keys_tmp;
    uint32_t *va = vals, *vb = vals_tmp;
    for (int shift = 0; shift < nbits; shift += 8) {
        k_rs_hist<<<nb, 256, 0, s>>>(ka, n, shift, hist, nb);
        hipError_t e = exclusive_scan_u32(hist, hist, 256ull * nb, scan_tmp, nullptr, s);
        if (e != hipSuccess) return e;
        k_rs_scatter<<<nb, 256, 0, s>>>(ka, va, kb, vb, n, shift, hist, nb);
        unsigned long long *tk = ka; ka = kb; kb = tk;
        uint32_t *tv = va; va = vb; vb = tv;
        *swapped = !*swapped;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ permutation, levels, anchors

__global__ void k_permute(const double *__restrict__ xyz, const uint32_t *__restrict__ vals, uint64_t n,
                          uint64_t base, uint64_t idx_offset, Vert *__restrict__ V, uint32_t *__restrict__ vtet,
                          uint8_t *__restrict__ dup) {
    uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t src = vals[i];
    Vert v;
    v.x = xyz[3ull * src + 0];
    v.y = xyz[3ull * src + 1];
    v.z = xyz[3ull * src + 2];
    v.idx = idx_offset + src;
    V[base + i] = v;
    vtet[base + i] = NONE;
    dup[base + i] = 0;
}

hipError_t launch_permute(const double *xyz, const uint32_t *vals, uint64_t n, uint64_t base, uint64_t idx_offset,
                          Vert *V, uint32_t *vtet, uint8_t *dup, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_permute<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(xyz, vals, n, base, idx_offset, V, vtet, dup);
    return hipGetLastError();
}

__global__ void k_level_hist(const unsigned long long *__restrict__ keys, uint64_t n, int shift,
                             uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[64];
    if (threadIdx.x < 64) h[threadIdx.x] = 0;
    __syncthreads();
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        atomicAdd(&h[(keys[i] >> shift) & 63u], 1u);
    __syncthreads();
    if (threadIdx.x < 64 && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

hipError_t launch_level_hist(const unsigned long long *keys, uint64_t n, int shift, uint32_t *hist, hipStream_t s) {
    unsigned nb = (unsigned)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
    if (nb == 0) return hipSuccess;
    k_level_hist<<<nb, 256, 0, s>>>(keys, n, shift, hist);
    return hipGetLastError();
}

// ------------------------------------------------------------------ duplicates

__device__ __forceinline__ unsigned long long coord_hash(double x, double y, double z) {
    // -0.0 and +0.0 are equal coordinates: hash them alike
    if (x == 0.0) x = 0.0;
    if (y == 0.0) y = 0.0;
    if (z == 0.0) z = 0.0;
    unsigned long long h = mix64((unsigned long long)__double_as_longlong(x));
    h = mix64(h ^ (unsigned long long)__double_as_longlong(y));
    return mix64(h ^ (unsigned long long)__double_as_longlong(z));
}

// table entry: (global input index << 32) | sorted position; all equal points end in one
// slot, which keeps the smallest input index (atomicMin)
__global__ void k_dedupe_insert(const Vert *__restrict__ V, uint64_t base, uint64_t n,
                                unsigned long long *__restrict__ table, uint64_t tmask) {
    uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    Vert v = V[base + i];
    unsigned long long mine = (v.idx << 32) | (unsigned long long)(base + i);
    uint64_t h = coord_hash(v.x, v.y, v.z) & tmask;
    for (;;) {
        unsigned long long cur = table[h];
        if (cur == ~0ull) {
            cur = atomicCAS(&table[h], ~0ull, mine);
            if (cur == ~0ull) return;
        }
        Vert w = V[(uint32_t)cur];
        if (w.x == v.x && w.y == v.y && w.z == v.z) {
            atomicMin(&table[h], mine);
            return;
        }
        h = (h + 1) & tmask;
    }
}

__global__ void k_dedupe_resolve(const Vert *__restrict__ V, uint64_t base, uint64_t n,
                                 const unsigned long long *__restrict__ table, uint64_t tmask,
                                 uint8_t *__restrict__ dup, uint32_t *__restrict__ ndup) {
    uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    Vert v = V[base + i];
    uint64_t h = coord_hash(v.x, v.y, v.z) & tmask;
    for (;;) {
        unsigned long long cur = table[h];
        if (cur == ~0ull) return;  // unreachable: the point's own slot precedes any empty one
        Vert w = V[(uint32_t)cur];
        if (w.x == v.x && w.y == v.y && w.z == v.z) {
            if ((uint32_t)cur != (uint32_t)(base + i)) {
                dup[base + i] = 1;
                atomicAdd(ndup, 1u);
            }
            return;
        }
        h = (h + 1) & tmask;
    }
}

hipError_t launch_dedupe(const Vert *V, uint64_t base, uint64_t n, unsigned long long *table, uint64_t tsize,
                         uint8_t *dup, uint32_t *ndup, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipError_t e = hipMemsetAsync(table, 0xFF, tsize * sizeof(unsigned long long), s);
    if (e != hipSuccess) return e;
    unsigned nb = (unsigned)((n + 255) / 256);
    k_dedupe_insert<<<nb, 256, 0, s>>>(V, base, n, table, tsize - 1);
    k_dedupe_resolve<<<nb, 256, 0, s>>>(V, base, n, table, tsize - 1, dup, ndup);
    return hipGetLastError();
}

}  // namespace dtk
