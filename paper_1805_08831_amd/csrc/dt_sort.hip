// Point ingest and spatial sort (paper Sec. 2.1 "Sort", Sec. 2.3).
//
// validate + bounding box of each cloud -> (cloud, Moore index) key per point -> stable LSD
// radix sort of (key, input index) -> 32-byte vertex records in curve order -> BRIO level of
// each record within its cloud and the level-major order of the records (a counting sort) ->
// exact duplicate removal by hashing, within each cloud.
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

// one block per chunk of one cloud: validity of the coordinates and the chunk's box
__global__ void k_chunk_bbox(const double *__restrict__ xyz, const uint64_t *__restrict__ ch_start,
                             const uint64_t *__restrict__ ch_end, double *__restrict__ partial,
                             uint32_t *__restrict__ err) {
    const uint64_t b = ch_start[blockIdx.x], e = ch_end[blockIdx.x];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    bool ok = true;
    for (uint64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
        for (int k = 0; k < 3; ++k) {
            const double v = xyz[3 * i + k];
            ok = ok && coord_ok(v);
            lo[k] = fmin(lo[k], v);
            hi[k] = fmax(hi[k], v);
        }
    }
    if (!ok) atomicOr(err, ERR_INPUT);
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

// one thread per cloud: its box from its chunks; the grid origin and the cubic scale
// 2^m / (largest extent)
__global__ void k_cloud_box(const double *__restrict__ partial, const uint32_t *__restrict__ cloud_ch,
                            uint32_t nclouds, Cloud *__restrict__ clouds) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nclouds) return;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (uint32_t j = cloud_ch[c]; j < cloud_ch[c + 1]; ++j)
        for (int k = 0; k < 3; ++k) {
            lo[k] = fmin(lo[k], partial[6 * j + k]);
            hi[k] = fmax(hi[k], partial[6 * j + 3 + k]);
        }
    double ext = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double e = hi[k] - lo[k];
        if (e > ext) ext = e;
    }
    const double cells = ldexp(1.0, (int)clouds[c].m);
    clouds[c].box[0] = lo[0];
    clouds[c].box[1] = lo[1];
    clouds[c].box[2] = lo[2];
    clouds[c].box[3] = ext > 0.0 ? cells / ext : 0.0;
}

hipError_t launch_cloud_bbox(const double *xyz, const uint64_t *ch_start, const uint64_t *ch_end,
                             uint32_t nchunks, double *partial, const uint32_t *cloud_ch, uint32_t nclouds,
                             Cloud *clouds, uint32_t *err, hipStream_t s) {
    if (nchunks) k_chunk_bbox<<<nchunks, 256, 0, s>>>(xyz, ch_start, ch_end, partial, err);
    k_cloud_box<<<(nclouds + 255) / 256, 256, 0, s>>>(partial, cloud_ch, nclouds, clouds);
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

// cloud of input point i: the last c with off[c] <= i
__device__ __forceinline__ uint32_t cloud_of(const uint64_t *__restrict__ off, uint32_t nclouds, uint64_t i) {
    uint32_t lo = 0, hi = nclouds;  // off[lo] <= i < off[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (off[mid] <= i) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ void k_keys(const double *__restrict__ xyz, uint64_t n, const uint64_t *__restrict__ off,
                       uint32_t nclouds, const Cloud *__restrict__ clouds, int shift, unsigned long long states,
                       unsigned long long *__restrict__ keys, uint32_t *__restrict__ vals) {
    uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t c = cloud_of(off, nclouds, i);
    const Cloud cl = clouds[c];
    const int m = (int)cl.m;
    const unsigned top = (1u << m) - 1u;
    unsigned cell[3];
    for (int k = 0; k < 3; ++k) {
        const double t = floor((xyz[3 * i + k] - cl.box[k]) * cl.box[3]);
        cell[k] = t >= (double)top ? top : (unsigned)t;
    }
    keys[i] = ((unsigned long long)c << shift) | moore_index(cell[0], cell[1], cell[2], m, states);
    vals[i] = (uint32_t)i;
}

hipError_t launch_keys(const double *xyz, uint64_t n, const uint64_t *off, uint32_t nclouds, const Cloud *clouds,
                       int shift, unsigned long long *keys, uint32_t *vals, hipStream_t s) {
    unsigned long long st = moore_states();
    if (!st) return hipErrorUnknown;
    if (n == 0) return hipSuccess;
    k_keys<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(xyz, n, off, nclouds, clouds, shift, st, keys, vals);
    return hipGetLastError();
}

// BRIO level of the point at each curve-ordered position, within its cloud (src[i] = its
// input index within the call; the cloud of the record is in the upper half of its idx), as
// the key of a stable counting sort that yields the level-major order of the positions;
// vals[i] = base + i
__global__ void k_levels(const uint32_t *__restrict__ src, const Vert *__restrict__ V, uint64_t n, uint64_t base,
                         const uint64_t *__restrict__ off, const Cloud *__restrict__ clouds,
                         unsigned long long salt, unsigned long long *__restrict__ keys,
                         uint32_t *__restrict__ vals, uint8_t *__restrict__ lev_out) {
    uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t c = (uint32_t)(V[base + i].idx >> 32);
    const unsigned long long local = (unsigned long long)src[i] - off[c];
    const unsigned long long nc = clouds[c].hi - clouds[c].lo;
    const unsigned long long u = mix64(salt + local) >> 11;
    const int lev = brio_level(u, nc);
    keys[i] = (unsigned long long)lev;
    vals[i] = (uint32_t)(base + i);
    if (lev_out) lev_out[i] = (uint8_t)lev;
}

hipError_t launch_levels(const uint32_t *src, const Vert *V, uint64_t n, uint64_t base, const uint64_t *off,
                         const Cloud *clouds, uint64_t salt, unsigned long long *keys, uint32_t *vals,
                         uint8_t *lev_out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_levels<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(src, V, n, base, off, clouds, salt, keys, vals, lev_out);
    return hipGetLastError();
}

// Walk anchor of every record of level k >= 1: the record of the nearest non-empty lower
// level that precedes it on the curve, or else follows it, if that record is in the same
// cloud.  lord lists each level's positions in increasing order; anchor is indexed by
// position - base.
__global__ void k_anchor(const uint32_t *__restrict__ lord, const uint32_t *__restrict__ start, int L,
                         const Vert *__restrict__ V, uint64_t base, uint64_t n, uint32_t *__restrict__ anchor) {
    const uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (j >= n) return;
    int k = 0;
    while (k + 1 < L && start[k + 1] <= j) ++k;
    const uint32_t p = lord[j];
    int kk = k - 1;
    while (kk >= 0 && start[kk + 1] == start[kk]) --kk;
    uint32_t res = 0xFFFFFFFFu;
    if (kk >= 0) {
        const uint32_t b = start[kk], e = start[kk + 1];
        uint32_t lo = b, hi = e, pos = b;  // last entry < p in [b, e), else b
        while (lo < hi) {
            const uint32_t mid = lo + (hi - lo) / 2;
            if (lord[mid] < p) {
                pos = mid;
                lo = mid + 1;
            } else {
                hi = mid;
            }
        }
        const uint32_t cp = (uint32_t)(V[p].idx >> 32);
        if ((uint32_t)(V[lord[pos]].idx >> 32) == cp) res = lord[pos];
        else if (pos + 1 < e && (uint32_t)(V[lord[pos + 1]].idx >> 32) == cp) res = lord[pos + 1];
    }
    anchor[p - base] = res;
}

hipError_t launch_anchor(const uint32_t *lord, const uint32_t *start, int L, const Vert *V, uint64_t base,
                         uint64_t n, uint32_t *anchor, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_anchor<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(lord, start, L, V, base, n, anchor);
    return hipGetLastError();
}

// Walk anchors given by the caller: input point i of the call (record base + j with input
// index idx_offset + i) starts its walk near record hint[i], an inserted vertex.
__global__ void k_hint_anchor(const Vert *__restrict__ V, uint64_t base, uint64_t n, uint64_t idx_offset,
                              const uint32_t *__restrict__ hint, uint32_t *__restrict__ anchor) {
    const uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (j >= n) return;
    const uint64_t i = (uint32_t)V[base + j].idx - idx_offset;
    anchor[j] = i < n ? hint[i] : 0xFFFFFFFFu;
}

hipError_t launch_hint_anchor(const Vert *V, uint64_t base, uint64_t n, uint64_t idx_offset, const uint32_t *hint,
                              uint32_t *anchor, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_hint_anchor<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(V, base, n, idx_offset, hint, anchor);
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

// The same sort in one block when the keys fit one tile (n <= RS_TILE): each digit pass is the
// tile's histogram, its scan and the stable scatter above, and the passes alternate between
// the two buffers as radix_sort_pairs does, so the result and its buffer are the same.  Short
// lists (the late refinement passes) then take one launch instead of five per digit.
__global__ __launch_bounds__(256) void k_rs_small(unsigned long long *ka, uint32_t *va, unsigned long long *kb,
                                                  uint32_t *vb, uint32_t n, int nbits) {
    __shared__ uint32_t off[256];
    __shared__ uint32_t wt[4][256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned long long lt = (1ull << lane) - 1ull;
    for (int shift = 0; shift < nbits; shift += 8) {
        off[threadIdx.x] = 0;
        for (int w = 0; w < 4; ++w) wt[w][threadIdx.x] = 0;
        __syncthreads();
        for (int it = 0; it < RS_ITEMS; ++it) {
            const uint32_t e = it * 256 + threadIdx.x;
            if (e < n) atomicAdd(&off[(ka[e] >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t t = 0;
            for (int d = 0; d < 256; ++d) {
                const uint32_t c = off[d];
                off[d] = t;
                t += c;
            }
        }
        __syncthreads();
        for (int it = 0; it < RS_ITEMS; ++it) {
            const uint32_t e = it * 256 + threadIdx.x;
            const bool valid = e < n;
            const unsigned long long key = valid ? ka[e] : 0ull;
            const uint32_t val = valid ? va[e] : 0u;
            const unsigned d = (unsigned)(key >> shift) & 255u;
            unsigned long long mask = __ballot(valid);
            for (int b = 0; b < 8; ++b) {
                const bool bit = (d >> b) & 1u;
                const unsigned long long bb = __ballot(valid && bit);
                mask &= bit ? bb : ~bb;
            }
            const unsigned rank = (unsigned)__popcll(mask & lt);
            if (valid && rank == 0) wt[wave][d] = (unsigned)__popcll(mask);
            __syncthreads();
            if (valid) {
                uint32_t pre = 0;
                for (int w = 0; w < wave; ++w) pre += wt[w][d];
                const uint32_t pos = off[d] + pre + rank;
                kb[pos] = key;
                vb[pos] = val;
            }
            __syncthreads();
            off[threadIdx.x] += wt[0][threadIdx.x] + wt[1][threadIdx.x] + wt[2][threadIdx.x] + wt[3][threadIdx.x];
            for (int w = 0; w < 4; ++w) wt[w][threadIdx.x] = 0;
            __syncthreads();
        }
        unsigned long long *tk = ka;
        ka = kb;
        kb = tk;
        uint32_t *tv = va;
        va = vb;
        vb = tv;
        // the block's stores of this pass are what the next pass reads (the barriers above
        // order them within the block)
    }
}

hipError_t radix_sort_pairs_any(unsigned long long *keys, uint32_t *vals, unsigned long long *keys_tmp,
                                uint32_t *vals_tmp, uint32_t *hist, uint32_t *scan_tmp, uint64_t n, int nbits,
                                hipStream_t s, bool *swapped) {
    if (n > (uint64_t)RS_TILE)
        return radix_sort_pairs(keys, vals, keys_tmp, vals_tmp, hist, scan_tmp, n, nbits, s, swapped);
    *swapped = false;
    if (n <= 1 || nbits <= 0) return hipSuccess;
    k_rs_small<<<1, 256, 0, s>>>(keys, vals, keys_tmp, vals_tmp, (uint32_t)n, nbits);
    *swapped = ((nbits + 7) / 8) % 2 == 1;
    return hipGetLastError();
}

// ------------------------------------------------------------------ permutation, levels, anchors

__global__ void k_permute(const double *__restrict__ xyz, const uint32_t *__restrict__ vals,
                          const unsigned long long *__restrict__ skeys, int shift, uint64_t n, uint64_t base,
                          uint64_t idx_offset, Vert *__restrict__ V, uint32_t *__restrict__ vtet,
                          uint8_t *__restrict__ dup) {
    uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t src = vals[i];
    Vert v;
    v.x = xyz[3ull * src + 0];
    v.y = xyz[3ull * src + 1];
    v.z = xyz[3ull * src + 2];
    v.idx = ((skeys[i] >> shift) << 32) | (idx_offset + src);
    V[base + i] = v;
    if (vtet) vtet[base + i] = NONE;
    if (dup) dup[base + i] = 0;
}

hipError_t launch_permute(const double *xyz, const uint32_t *vals, const unsigned long long *skeys, int shift,
                          uint64_t n, uint64_t base, uint64_t idx_offset, Vert *V, uint32_t *vtet, uint8_t *dup,
                          hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_permute<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(xyz, vals, skeys, shift, n, base, idx_offset, V, vtet,
                                                          dup);
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
    // smallest input index first (the cloud id in the upper half of idx is shifted out)
    unsigned long long mine = (v.idx << 32) | (unsigned long long)(base + i);
    uint64_t h = coord_hash(v.x, v.y, v.z) & tmask;
    for (;;) {
        unsigned long long cur = table[h];
        if (cur == ~0ull) {
            cur = atomicCAS(&table[h], ~0ull, mine);
            if (cur == ~0ull) return;
        }
        Vert w = V[(uint32_t)cur];
        if (w.x == v.x && w.y == v.y && w.z == v.z && (w.idx >> 32) == (v.idx >> 32)) {
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
        if (w.x == v.x && w.y == v.y && w.z == v.z && (w.idx >> 32) == (v.idx >> 32)) {
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
