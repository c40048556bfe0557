// Concurrent Bowyer-Watson insertion rounds (paper Sec. 2.1 Algorithm 1, Sec. 2.5, Sec. 2.6;
// concurrency rules of Sec. 3.2).
//
// A round is two kernels over the round's candidate points:
//   k_cavity_g : Walk (visibility walk, Sec. 2.1) from a live tetrahedron of an already
//              inserted neighbour on the space-filling curve, then Cavity (breadth-first
//              search by perturbed insphere, ghosts by the half-space + circumdisk rule of
//              Sec. 2.6), by a group of lanes per insertion.  The attempt claims every
//              tetrahedron it touches, once it has tested it, with atomicMin on the
//              tetrahedron's 64-bit claim word: its stamp S = (round part, 2 rank) for cavity
//              tetrahedra, S + 1 for tetrahedra found outside.  Meeting a lower claim that
//              excludes it ends the attempt (one search step later).
//   k_ball   : an attempt wins iff no lower attempt claimed a tetrahedron of its cavity
//              (either way) or has one of its outer tetrahedra in its cavity, so the cavities
//              of winners are disjoint from each other and from each other's adjacent
//              tetrahedra (rules 1a-1c and 2 of Sec. 3.2); the lowest rank in a
//              round always wins, so every round makes progress.  A winner builds
//              DelaunayBall (Sec. 2.5): one tetrahedron per boundary facet, glued a priori to
//              the outer tetrahedron, and glued to its three sibling tetrahedra through an
//              LDS table of boundary edges (pivoting around each boundary edge through copies
//              of the cavity tetrahedra for large balls).  Freed
//              slots are reused in later rounds (Sec. 2.5 end, Sec. 3.6).
// Then k_compact queues losers for the next round with their rank, and overflowing
// cavities for rounds with larger per-insertion buffers.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstdlib>

#include "dt_internal.h"
#include "dt_predicates.h"

namespace dtk {

constexpr uint32_t WALK_LIMIT = 1u << 20;

__device__ __forceinline__ P3 vpos(const Vert *V, uint32_t v) {
    Vert r = V[v];
    return {r.x, r.y, r.z};
}

// neighbour code of facet f of tetrahedron t, as an lvalue
__device__ __forceinline__ uint32_t &nref(Tet *T, uint32_t t, uint32_t f) {
    return reinterpret_cast<uint32_t *>(&T[t].n)[f];
}
__device__ __forceinline__ unsigned long long &nref(TetW *T, uint32_t t, uint32_t f) {
    return T[t].n.c[f];
}

// slot and facet of an adjacency code 4 t + f
template <class C>
__device__ __forceinline__ uint32_t code_slot(C code) {
    return (uint32_t)(code >> 2);
}
template <class C>
__device__ __forceinline__ int code_facet(C code) {
    return (int)(code & 3u);
}
template <class K>
__device__ __forceinline__ typename K::code make_code(uint32_t slot, uint32_t f) {
    return ((typename K::code)slot << 2) | (typename K::code)f;
}

__device__ __forceinline__ unsigned wave_sum(unsigned v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ void add_stat(unsigned long long *stat, int id, unsigned v) {
    unsigned s = wave_sum(v);
    if ((threadIdx.x & 63) == 0 && s)
        atomicAdd(&stat[((size_t)id * STAT_SPREAD + (blockIdx.x % STAT_SPREAD)) * STAT_PAD], (unsigned long long)s);
}

// Reserves v units of the counter *count per thread with one atomic per block (the block is
// NW waves; every thread must call it): returns the first unit of this thread's range.
// tmp: NW + 1 words of LDS the block does not use meanwhile.
template <int NW = 4>
__device__ __forceinline__ uint32_t block_reserve(uint32_t v, uint32_t *count, uint32_t *tmp) {
    uint32_t *s_wave = tmp, &s_base = tmp[NW];
    const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x >> 6;
    uint32_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= (uint32_t)o) x += y;
    }
    if (lane == 63) s_wave[wid] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < NW; ++w) {
            const uint32_t c = s_wave[w];
            s_wave[w] = t;
            t += c;
        }
        s_base = t ? atomicAdd(count, t) : 0u;
    }
    __syncthreads();
    const uint32_t r = s_base + s_wave[wid] + x - v;
    __syncthreads();  // tmp may be reused after the call
    return r;
}

// Orders a tetrahedron built from outer tetrahedron vertices w (w[j] replaced by the new
// point): one transposition restores positive orientation; a ghost vertex is then moved to
// slot 3 by an even permutation.  Returns the slot of the new point.
__device__ __forceinline__ int orient_new_tet(uint32_t w[4], int j) {
    int a = (j + 1) & 3, b = (j + 2) & 3;
    uint32_t t = w[a]; w[a] = w[b]; w[b] = t;
    int pf = j;
    int g = -1;
    for (int i = 0; i < 3; ++i)
        if (w[i] == GHOST) g = i;
    if (g >= 0) {
        int x = -1, y = -1;
        for (int i = 0; i < 3; ++i)
            if (i != g) { if (x < 0) x = i; else y = i; }
        t = w[g]; w[g] = w[3]; w[3] = t;
        t = w[x]; w[x] = w[y]; w[y] = t;
        if (pf == 3) pf = g;
        else if (pf == x) pf = y;
        else if (pf == y) pf = x;
    }
    return pf;
}

// ------------------------------------------------------------------ initial tetrahedron

// One block per cloud: the first four affinely independent distinct points of the cloud's
// records (any choice gives the same triangulation), positively oriented, plus the four
// ghosts (each holds G in slot 3, its finite facet facing outward), at slots
// first_slot + 5 c .. + 4.
static_assert(sizeof(SubD) == 40, "the host sizes the sub-determinant cache at 40 bytes per tetrahedron");

template <class K>
__global__ void k_init(const Vert *__restrict__ V, Cloud *__restrict__ clouds, uint32_t first_slot,
                       const uint8_t *__restrict__ dup, typename K::Rec *__restrict__ T, uint32_t *__restrict__ vtet,
                       Ctr *__restrict__ ctr, SubD *__restrict__ subd) {
    using code = typename K::code;
    __shared__ uint32_t sel[4];
    __shared__ uint32_t best;
    PredStats st;
    const uint32_t c = blockIdx.x;
    const uint32_t base = clouds[c].lo, n = clouds[c].hi - clouds[c].lo;
    for (int stage = 0; stage < 4; ++stage) {
        if (threadIdx.x == 0) best = NONE;
        __syncthreads();
        for (uint32_t chunk = 0; chunk < n; chunk += blockDim.x) {
            uint32_t i = chunk + threadIdx.x;
            bool ok = i < n && !dup[base + i];
            for (int s = 0; s < stage && ok; ++s) ok = sel[s] != base + i;
            if (ok && stage == 2) ok = !collinear(vpos(V, sel[0]), vpos(V, sel[1]), vpos(V, base + i));
            if (ok && stage == 3)
                ok = orient3d(vpos(V, sel[0]), vpos(V, sel[1]), vpos(V, sel[2]), vpos(V, base + i), st) != 0;
            if (ok) atomicMin(&best, i);
            __syncthreads();
            if (best != NONE) break;
            __syncthreads();
        }
        if (best == NONE) {
            if (threadIdx.x == 0) {
                atomicOr(&ctr->error, ERR_DEGENERATE);
                atomicMin(&ctr->bad_cloud, c);
            }
            return;
        }
        if (threadIdx.x == 0) sel[stage] = base + best;
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    uint32_t v[4] = {sel[0], sel[1], sel[2], sel[3]};
    if (orient3d(vpos(V, v[0]), vpos(V, v[1]), vpos(V, v[2]), vpos(V, v[3]), st) < 0) {
        uint32_t t = v[0]; v[0] = v[1]; v[1] = t;
    }
    const uint32_t s0 = first_slot + 5 * c;
    uint32_t TV[5][4];
    code N[5][4];
    for (int k = 0; k < 4; ++k) TV[0][k] = v[k];
    for (int j = 0; j < 4; ++j) {
        uint32_t w[4] = {v[0], v[1], v[2], v[3]};
        w[j] = GHOST;
        orient_new_tet(w, j);  // G ends in slot 3: finite facet (w0,w1,w2) faces outward
        for (int k = 0; k < 4; ++k) TV[1 + j][k] = w[k];
        N[0][j] = make_code<K>(s0 + 1u + j, 3u);
        N[1 + j][3] = make_code<K>(s0, (uint32_t)j);
    }
    // ghost-ghost adjacencies: facets through G with the same three vertices
    for (int g1 = 1; g1 < 5; ++g1)
        for (int f1 = 0; f1 < 3; ++f1)
            for (int g2 = 1; g2 < 5; ++g2) {
                if (g2 == g1) continue;
                for (int f2 = 0; f2 < 3; ++f2) {
                    int same = 0;
                    for (int i = 0; i < 4; ++i) {
                        if (i == f1) continue;
                        for (int k = 0; k < 4; ++k)
                            if (k != f2 && TV[g2][k] == TV[g1][i]) same++;
                    }
                    if (same == 3) N[g1][f1] = make_code<K>(s0 + (uint32_t)g2, (uint32_t)f2);
                }
            }
    for (int t = 0; t < 5; ++t) {
        typename K::Rec &r = T[s0 + t];
        r.v = make_uint4(TV[t][0], TV[t][1], TV[t][2], TV[t][3]);
        for (int f = 0; f < 4; ++f) nref(T, s0 + t, f) = N[t][f];
        r.claim = ~0ull;
        r.spare[0] = 0;
    }
    for (int k = 0; k < 4; ++k) vtet[v[k]] = s0;
    if (subd) subd[s0] = subdets(vpos(V, v[0]), vpos(V, v[1]), vpos(V, v[2]), vpos(V, v[3]));
    clouds[c].any_live = s0;
}

hipError_t launch_init(const Vert *V, Cloud *clouds, uint32_t nclouds, uint32_t first_slot, const uint8_t *dup,
                       void *T, bool wide, uint32_t *vtet, Ctr *ctr, void *subd, hipStream_t s) {
    if (nclouds == 0) return hipSuccess;
    if (wide)
        k_init<Wide><<<nclouds, 256, 0, s>>>(V, clouds, first_slot, dup, (TetW *)T, vtet, ctr, (SubD *)subd);
    else
        k_init<Narrow><<<nclouds, 256, 0, s>>>(V, clouds, first_slot, dup, (Tet *)T, vtet, ctr, (SubD *)subd);
    return hipGetLastError();
}

// ------------------------------------------------------------------ candidate fill

// Ranks: level k owns ranks [rank_base[k], rank_base[k] + 2^bits[k]); local rank l maps to
// the level position q = bitreverse(l) (lord lists each level's records in curve order), so
// any window of consecutive ranks is spread evenly along the level's points.  Within an
// aligned block of 2^w local ranks the positions form an arithmetic progression in the
// order of bitreverse_w of the rank's low bits: thread s takes l = a + bitreverse_w(s), so
// the block's candidates come out in curve order.  A wave appends its valid candidates
// with one atomic, in thread order.
// Round-start and round-end kernels append to shared list counters with one atomic per
// 1024-thread block: one address takes about one atomic per 12 ns, so per-wave appends from
// a large round serialize for several microseconds.
constexpr int FILL_BLOCK = 1024;

__global__ __launch_bounds__(FILL_BLOCK) void k_fill(FillPlan plan, const uint32_t *__restrict__ lvl_start, const uint32_t *__restrict__ lvl_size,
                       const uint32_t *__restrict__ lvl_bits, const unsigned long long *__restrict__ rank_base,
                       const uint32_t *__restrict__ lord, const uint8_t *__restrict__ dup,
                       const uint32_t *__restrict__ vtet, uint32_t *__restrict__ cand_pt,
                       uint32_t *__restrict__ cand_rank, uint32_t *__restrict__ ncand) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    bool ok = t < plan.off[plan.nblk];
    uint32_t p = 0, r = 0;
    if (ok) {
        uint32_t j = 0;
        while (j + 1 < plan.nblk && plan.off[j + 1] <= t) ++j;
        const uint32_t s = t - plan.off[j], w = plan.w[j], k = plan.lvl[j];
        const uint32_t local = plan.a[j] + (w ? (__brev(s) >> (32 - w)) : 0u);
        const uint32_t bits = lvl_bits[k];
        const uint32_t q = bits ? (__brev(local) >> (32 - bits)) : 0u;
        ok = q < lvl_size[k];
        if (ok) {
            p = lord[lvl_start[k] + q];
            ok = !dup[p] && vtet[p] == NONE;
            r = (uint32_t)(rank_base[k] + local);
        }
    }
    __shared__ uint32_t s_tmp[FILL_BLOCK / 64 + 1];
    const uint32_t pos = block_reserve<FILL_BLOCK / 64>(ok ? 1u : 0u, ncand, s_tmp);
    if (ok) {
        cand_pt[pos] = p;
        cand_rank[pos] = r;
    }
}

hipError_t launch_fill_list(const FillPlan &plan, const uint32_t *lvl_start, const uint32_t *lvl_size,
                            const uint32_t *lvl_bits, const unsigned long long *rank_base, const uint32_t *lord,
                            const uint8_t *dup, const uint32_t *vtet, uint32_t *cand_pt, uint32_t *cand_rank,
                            uint32_t *ncand, hipStream_t s) {
    const uint32_t count = plan.off[plan.nblk];
    if (count == 0) return hipSuccess;
    k_fill<<<(count + FILL_BLOCK - 1) / FILL_BLOCK, FILL_BLOCK, 0, s>>>(plan, lvl_start, lvl_size, lvl_bits, rank_base, lord, dup, vtet,
                                               cand_pt, cand_rank, ncand);
    return hipGetLastError();
}

// ------------------------------------------------------------------ walk + cavity + claim


// Predicates of the cavity kernel.  FULL decides every sign exactly (filter, certified fp64,
// integers, perturbation).  Without FULL only the fp64 filter runs, and a sign it cannot
// decide (an exact zero included, which needs the perturbation) comes back as UNDECIDED: the
// attempt then stops before claiming anything on that step and is run again by the FULL
// kernel in the same round.  The exact stages (and their registers and scratch) stay out of
// the kernel that does almost all the work.
constexpr int UNDECIDED = 2;

template <bool FULL>
__device__ __forceinline__ int cav_orient(P3 a, P3 b, P3 c, P3 d, PredStats &st) {
    if (FULL) return orient3d(a, b, c, d, st);
    st.orient++;
    return orient3d_filter(a, b, c, d);
}

// -1: e strictly inside the (perturbed) circumsphere of the positive tetrahedron abcd
template <bool FULL, class Keys>
__device__ __forceinline__ int cav_insphere(P3 a, P3 b, P3 c, P3 d, P3 e, Keys keys, PredStats &st) {
    if (FULL) return insphere_perturbed(a, b, c, d, e, keys, st);
    st.insphere++;
    const int s = insphere_filter(a, b, c, d, e);
    return s == 0 ? UNDECIDED : s;
}

// perturbed "P strictly inside the circumsphere of finite tetrahedron w": -1 inside, 1
// outside, UNDECIDED
template <bool FULL>
__device__ __forceinline__ int finite_inside(const Vert *V, uint4 w, P3 P, unsigned long long pidx,
                                             PredStats &st) {
    const uint32_t ids[4] = {w.x, w.y, w.z, w.w};
    const int s = cav_insphere<FULL>(vpos(V, w.x), vpos(V, w.y), vpos(V, w.z), vpos(V, w.w), P,
                                     [&](int k) { return k < 4 ? V[ids[k]].idx : pidx; }, st);
    return s == UNDECIDED ? s : (s < 0 ? -1 : 1);
}

// Sec. 2.6: a ghost (a,b,c,G) contains the open half-space beyond abc and abc's circumdisk;
// -1 inside, 1 outside, UNDECIDED
template <class K, bool FULL>
__device__ __forceinline__ int tet_inside(const typename K::Rec *T, const Vert *V, uint32_t u, P3 P,
                                          unsigned long long pidx, PredStats &st) {
    uint4 w = T[u].v;
    if (w.w != GHOST) return finite_inside<FULL>(V, w, P, pidx, st);
    int o = cav_orient<FULL>(vpos(V, w.x), vpos(V, w.y), vpos(V, w.z), P, st);
    if (o == UNDECIDED) return o;
    if (o != 0) return o > 0 ? -1 : 1;
    uint32_t x = code_slot(comp(T[u].n, 3));
    return finite_inside<FULL>(V, T[x].v, P, pidx, st);
}

// ------------------------------------------------------------------ walk + cavity + claim

// Sizes of the cavity kernel's per-insertion state: a queue of CAPL cavity tetrahedra and a
// set of HM entries holding the attempt's own cavity and outer tetrahedra.  Regular rounds
// keep both in LDS at (128, 256) with 4 to 64 lanes per insertion; rounds for large
// cavities use (1024, 2048) with 64 lanes, and beyond that the same 64-lane search keeps
// both in global memory (the candidate's cavity buffer and its part of the ball scratch).
constexpr uint32_t LCAPC = 128;
constexpr uint32_t BIG_CAPC = 1024, BIG_HM = 2048;

template <class E>
__device__ __forceinline__ constexpr E mem_empty() {
    return ~(E)0;
}

// open addressing in a power-of-two table of hm entries, (t << 1 | kind) per entry
__device__ __forceinline__ uint32_t mem_hash(uint32_t t, uint32_t hm) {
    return (t * 2654435761u) >> (32 - __builtin_ctz(hm));
}

// kind of tetrahedron t in the set (0 cavity, 1 outer) or -1; a set in global memory is
// read at device scope, past any vector L1 copy, since other lanes fill it by atomics
template <bool GLOBAL, class E>
__device__ __forceinline__ int mem_find(E *mem, uint32_t hm, uint32_t t) {
    uint32_t h = mem_hash(t, hm);
    for (uint32_t probe = 0; probe < hm; ++probe) {
        const E e =
            GLOBAL ? __hip_atomic_load(&mem[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : mem[h];
        if (e == mem_empty<E>()) return -1;
        if ((e >> 1) == (E)t) return (int)(e & 1u);
        h = (h + 1) & (hm - 1);
    }
    return -1;
}

// adds t with `kind`: 1 if this call added it (its entry is then mem[*at]), 0 if it was
// there, -1 if the set is full
template <class E>
__device__ __forceinline__ int mem_insert(E *mem, uint32_t hm, uint32_t t, uint32_t kind, uint32_t *at) {
    uint32_t h = mem_hash(t, hm);
    const E e = ((E)t << 1) | (E)kind;
    for (uint32_t probe = 0; probe < hm; ++probe) {
        const E old = atomicCAS(&mem[h], mem_empty<E>(), e);
        if (old == mem_empty<E>()) {
            *at = h;
            return 1;
        }
        if ((old >> 1) == (E)t) return 0;
        h = (h + 1) & (hm - 1);
    }
    return -1;
}

// Orders the accesses of one group (all in one wave) to its queue and set where other lanes
// consume them: the hardware processes one wave's LDS requests in order, so LDS needs only a
// compiler barrier; global memory also waits for the wave's outstanding accesses.
template <bool GLOBAL>
__device__ __forceinline__ void lane_fence() {
    if (GLOBAL) __threadfence_block();
    __asm__ volatile("" ::: "memory");
}

// Walk (Sec. 2.3) and cavity search (Sec. 2.4) of one candidate per group of GS lanes
// (4, 8, 16, 32 or 64): the walk tests the four facets of the current tetrahedron on four lanes
// at once, and the cavity search expands GS / 4 cavity tetrahedra (four facets each) per
// step, appending cavity and boundary entries by ballot prefix counts.  Control flow is
// uniform within each group.  Cavity entries hold (tetrahedron << 2 | facet it was entered
// through), which is skipped when the tetrahedron is expanded.
//
// Claims: every neighbour examined is tested first and then claimed once, with S if it is
// inside (S is the attempt's stamp: round, then rank) and S + 1 if it is outside.  A lower
// value returned on an inside tetrahedron, or a lower even value (a lower attempt's cavity)
// on an outside one, loses the attempt.  The attempt's own tetrahedra are tracked in the
// set, so each is claimed and tested once.  GLOBAL keeps queue and set in global memory
// (any capC).
//
// FULL = false: filter-only predicates; an attempt meeting a sign the filter cannot decide
// ends with ST_FULL and is listed for the FULL kernel.  DEFER: the kernel runs the listed
// candidates (a.defer[0 .. *a.ndefer_ptr)) instead of the round's list, grid-stride.
template <class K, int GS, uint32_t CAPL, uint32_t HM, bool GLOBAL, bool FULL, bool DEFER>
__global__ __launch_bounds__(256) void k_cavity_g(RoundArgs a) {
    using code = typename K::code;
    using E = typename K::set_t;
    constexpr uint32_t GPB = 256 / GS;  // insertions per 256-thread block
    constexpr uint32_t NP = GS / 4;     // cavity tetrahedra expanded per step
    // LDS queue entries: (slot of the tetrahedron's entry in the set << 2 | facet it was
    // entered through), 16 bits; the global queue holds (tetrahedron << 2 | facet)
    __shared__ uint16_t s_cav[GPB][GLOBAL ? 1 : CAPL];
    __shared__ E s_mem[GPB][GLOBAL ? 1 : HM];
    typename K::Rec *const T = static_cast<typename K::Rec *>(a.T);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t gl = threadIdx.x & (GS - 1);
    const uint32_t gi = threadIdx.x / GS;
    const uint32_t gbase = lane & ~(uint32_t)(GS - 1);
    const unsigned long long gmask = GS == 64 ? ~0ull : (((1ull << (GS & 63)) - 1ull) << gbase);
    const unsigned long long below = gmask & ((1ull << lane) - 1ull);
    const uint32_t ncand = DEFER ? *a.ndefer_ptr : *a.ncand_ptr;
    const uint32_t stride = a.stride;
    PredStats st;
    unsigned steps = 0, attempt = 0;
    // one candidate per group; the deferred pass strides over its short list
    for (uint32_t j = blockIdx.x * GPB + gi; j < ncand; j += DEFER ? gridDim.x * GPB : ncand) {
        const uint32_t i = DEFER ? a.defer[j] : j;
        uint8_t status = ST_NONE;
        const uint32_t p = a.cand_pt[i];
        const unsigned long long S = a.round_hi | (2ull * a.cand_rank[i]);
        const Vert pv = a.V[p];
        const P3 P = {pv.x, pv.y, pv.z};
        const bool clocked = !FULL && !DEFER && a.clk != nullptr;
        const unsigned long long tc0 = clocked ? (unsigned long long)wall_clock64() : 0ull;
        // start: near the nearest inserted point among GS / 2 records on either side of p on
        // the curve (in p's cloud), one probe per lane; else near the point's anchor (a
        // record of a lower level); else the cloud's known live tetrahedron.  A record's
        // hint is a tetrahedron incident to it: the ball kernel renews the hints of all
        // vertices of the tetrahedra it builds, which include every vertex of a removed one.
        Cloud *cl = &a.clouds[pv.idx >> 32];
        const uint32_t clo = cl->lo, chi = cl->hi;
        const uint32_t d = (gl >> 1) + 1;
        const uint32_t hp = (gl & 1) ? p + d : p - d;
        const bool inr = (gl & 1) ? (p + d < a.vhi) : (p >= a.vlo + d);
        const uint32_t ht = inr && hp >= clo && hp < chi ? a.vtet[hp] : NONE;
        const uint32_t q = a.anchor[p - a.vlo];
        const uint32_t tq = q != NONE ? a.vtet[q] : NONE;
        const uint32_t tl = a.lastt[p - a.vlo];
        const unsigned long long hm = __ballot(ht != NONE) & gmask;
        uint32_t t = hm ? __shfl(ht, __ffsll((long long)hm) - 1) : tq;
        // the learned scheduler predicts the anchor to be the closer start
        if (a.wbucket && tq != NONE && a.wbucket[p - a.vlo]) t = tq;
        if (t == NONE) t = cl->any_live;
        // a retry starts where the last attempt located p: that tetrahedron, or the one the
        // ball of a winner built in its slot, is near p unless the slot went to another
        // cloud of the call
        uint4 w;
        bool from_last = false;
        if (tl != NONE) {
            w = T[tl].v;
            from_last = w.x != DEAD && (!a.multi || (a.V[w.x].idx >> 32) == (pv.idx >> 32));
        }
        if (from_last) {
            t = tl;
        } else {
            w = T[t].v;
        }
        if (w.x == DEAD) {
            t = cl->any_live;
            w = T[t].v;
        }
        if (w.w == GHOST) {
            t = code_slot(comp(T[t].n, 3));
            w = T[t].v;
        }
        // Walk: lane j < 4 tests facet j.  The walk moves through a facet whose sign is
        // negative; a facet the filter cannot decide is not crossed.  If the walk stops at a
        // tetrahedron with such a facet (p within rounding of its plane), that tetrahedron
        // still starts the cavity when the filter puts p strictly inside its circumsphere
        // (the cavity is connected, any of its tetrahedra starts it); else the FULL kernel
        // runs the attempt.
        int entry = -1;
        bool in_ghost = false, unsure = false;
        const int jl = (int)(gl & 3u);
        unsigned ws = 0;  // steps of this walk
        for (;;) {
            const P3 q0 = vpos(a.V, w.x), q1 = vpos(a.V, w.y), q2 = vpos(a.V, w.z), q3 = vpos(a.V, w.w);
            const typename K::code4 nn = T[t].n;
            int o = 1;
            if (gl < 4 && jl != entry)
                o = cav_orient<FULL>(jl == 0 ? P : q0, jl == 1 ? P : q1, jl == 2 ? P : q2, jl == 3 ? P : q3, st);
            const unsigned bits = (unsigned)((__ballot(o < 0) & gmask) >> gbase) & 0xFu;
            if (!bits) {
                unsure = !FULL && (__ballot(o == UNDECIDED) & gmask);
                break;
            }
            const unsigned rot = (p + ws) & 3u;
            const unsigned rb = ((bits >> rot) | (bits << (4u - rot))) & 0xFu;
            const int moved = (int)(((unsigned)__ffs(rb) - 1u + rot) & 3u);
            const code cd = comp(nn, moved);
            t = code_slot(cd);
            entry = code_facet(cd);
            w = T[t].v;
            if (++ws > WALK_LIMIT) {
                status = ST_ERROR;
                break;
            }
            if (w.w == GHOST) {
                in_ghost = true;
                break;
            }
            if (!FULL && ws >= a.walk_cap) {
                status = ST_WALK;
                break;
            }
        }
        steps += ws;
        if (gl == 0 && status != ST_ERROR) a.lastt[p - a.vlo] = t;
        const unsigned long long tc1 = clocked ? (unsigned long long)wall_clock64() : 0ull;
        unsigned cav_steps = 0;
        if (status == ST_NONE && !in_ghost) {
            // p equal to a vertex of its containing tetrahedron: lane j < 4 compares vertex j
            bool same = false;
            if (gl < 4) {
                const P3 v = vpos(a.V, comp(w, jl));
                same = v.x == P.x && v.y == P.y && v.z == P.z;
            }
            if (__ballot(same) & gmask) status = ST_DUP;
        }
        if (!FULL && unsure && status == ST_NONE && !in_ghost) {
            const int si = gl == 0 ? finite_inside<FULL>(a.V, w, P, pv.idx, st) : -1;
            if (__ballot(si != -1) & gmask) status = ST_FULL;
        }
        uint32_t ncav = 0, nbnd = 0;
        const uint32_t capL = GLOBAL ? a.capC : min(a.capC, CAPL), capF = a.capF;
        uint32_t *bnd = a.bnd + (size_t)i * a.capF;
        code *outc = static_cast<code *>(a.outc) + (size_t)i * a.capF;
        code *cavg = static_cast<code *>(a.cav) + (size_t)i * a.capC;
        uint16_t *cavl = s_cav[gi];
        // the set in global memory: hms entries (a power of two, at most 16 capC bytes) of
        // the candidate's part of the ball scratch, which the ball kernel uses only later
        const uint32_t hms = GLOBAL ? a.hmg : HM;
        E *mem = GLOBAL ? reinterpret_cast<E *>(a.scr_v + (size_t)i * a.capC) : s_mem[gi];
        if (status == ST_NONE) {
            // Cavity.  Step k expands cavity tetrahedra k0 .. k0 + NP - 1, lane (slot, facet)
            // = (gl / 4, gl % 4).
            for (uint32_t h = gl; h < hms; h += GS) mem[h] = mem_empty<E>();
            lane_fence<GLOBAL>();
            // each step's claims are checked at the next step (or after the last), once that
            // step's loads are in flight, so that the atomics' latency overlaps them; the
            // walk's tetrahedron is inside, its claim is checked with the first step's
            bool pneed = gl == 0, pinside = true;
            unsigned long long po1 = ~0ull;
            if (gl == 0) {
                po1 = atomicMin(&T[t].claim, S);
                uint32_t at = 0;
                mem_insert(mem, hms, t, 0u, &at);
                if (GLOBAL) cavg[0] = make_code<K>(t, 0u);
                else cavl[0] = (uint16_t)(at << 2);
            }
            ncav = 1;
            lane_fence<GLOBAL>();
            for (uint32_t k0 = 0, nproc = 0; k0 < ncav && status == ST_NONE; k0 += nproc) {
                nproc = min(NP, ncav - k0);  // entries expanded in this step
                ++cav_steps;
                const uint32_t slot = k0 + (gl >> 2);
                const int f = jl;
                const bool lv = slot < k0 + nproc;
                code cd = 0u;
                if (lv) {
                    if (GLOBAL) {
                        cd = cavg[slot];
                    } else {
                        const uint32_t q = cavl[slot];
                        cd = make_code<K>((uint32_t)(mem[q >> 2] >> 1), q & 3u);
                    }
                }
                const uint32_t c = code_slot(cd);
                const int pf = slot == 0 ? -1 : code_facet(cd);
                const bool act = lv && f != pf;
                uint4 cv = make_uint4(0u, 0u, 0u, 0u), uw = cv;
                typename K::code4 cn{};
                if (lv) {
                    cv = T[c].v;
                    cn = T[c].n;
                }
                // the previous step's claims: a lower claim on a tetrahedron of this cavity,
                // or a lower cavity claim (even) on one outside it, loses the attempt
                if (__ballot(pneed && po1 < S && (pinside || !(po1 & 1ull))) & gmask) {
                    status = ST_CONFLICT;
                    break;
                }
                const code ncode = comp(cn, f);
                const uint32_t u = code_slot(ncode);
                const int kind = act ? mem_find<GLOBAL>(mem, hms, u) : -1;  // 0: in this cavity, 1: outside it
                const bool need = act && kind < 0;
                if (need) uw = T[u].v;
                bool inside = false, undecided = false;
                if (need) {
                    const bool cghost = cv.w == GHOST;
                    const uint32_t apex = comp(uw, code_facet(ncode));
                    if (!cghost && apex != GHOST) {
                        // u = facet f of c + apex; c with vertex f replaced by the apex and
                        // two entries swapped is positively oriented
                        const uint32_t cid[4] = {cv.x, cv.y, cv.z, cv.w};
                        uint32_t rid[4];
#pragma unroll
                        for (int m = 0; m < 4; ++m) rid[m] = m == f ? apex : cid[m];
                        const int sa = (f + 1) & 3, sb = (f + 2) & 3;
                        uint32_t r2[4];
#pragma unroll
                        for (int m = 0; m < 4; ++m) r2[m] = m == sa ? rid[sb] : (m == sb ? rid[sa] : rid[m]);
                        int si;
                        if (!FULL && a.subd) {
                            // cached sub-determinants of u (its stored vertex order is positive too,
                            // an even permutation of r2, so the sign is the same)
                            st.insphere++;
                            si = insphere_cached(static_cast<const SubD *>(a.subd)[u], vpos(a.V, uw.x), P);
                        } else {
                            si = cav_insphere<FULL>(vpos(a.V, r2[0]), vpos(a.V, r2[1]), vpos(a.V, r2[2]),
                                                    vpos(a.V, r2[3]), P,
                                                    [&](int kk) { return kk < 4 ? a.V[r2[kk]].idx : pv.idx; }, st);
                        }
                        inside = si < 0;
                        undecided = si == UNDECIDED;
                    } else if (!cghost) {
                        // u is the ghost beyond facet f of the finite cavity tetrahedron c:
                        // inside iff p is beyond the facet, or on it (then c decides: inside)
                        const P3 c0 = vpos(a.V, cv.x), c1 = vpos(a.V, cv.y), c2 = vpos(a.V, cv.z),
                                 c3 = vpos(a.V, cv.w);
                        const int so = cav_orient<FULL>(f == 0 ? P : c0, f == 1 ? P : c1, f == 2 ? P : c2,
                                                        f == 3 ? P : c3, st);
                        inside = so <= 0;
                        undecided = so == UNDECIDED;
                    } else {
                        const int si = tet_inside<K, FULL>(T, a.V, u, P, pv.idx, st);
                        inside = si < 0;
                        undecided = si == UNDECIDED;
                    }
                }
                // a sign the filter could not decide: no claim on this step, the FULL kernel
                // runs the attempt again
                if (!FULL && (__ballot(undecided) & gmask)) {
                    status = ST_FULL;
                    break;
                }
                // the one claim of u: S if inside, S + 1 if outside (a tetrahedron reached
                // through several facets in this step gets the same claim from each lane)
                unsigned long long o1 = ~0ull;
                if (need) o1 = atomicMin(&T[u].claim, inside ? S : S + 1);
                // record u in the set; a tetrahedron reached through several facets in this
                // step is queued (if inside) by the lane that records it
                int ins = 0;
                uint32_t at = 0;
                if (need) ins = mem_insert(mem, hms, u, inside ? 0u : 1u, &at);
                const bool first_in = ins == 1 && inside;
                const bool outside = (act && kind == 1) || (need && !inside);  // boundary facet (c, f)
                const unsigned long long mi = __ballot(first_in) & gmask;
                const unsigned long long mo = __ballot(outside) & gmask;
                const uint32_t ni = (uint32_t)__popcll(mi), no = (uint32_t)__popcll(mo);
                if (ncav + ni > capL || nbnd + no > capF || (__ballot(ins < 0) & gmask)) {
                    status = ST_OVERFLOW;
                    break;
                }
                if (first_in) {
                    const uint32_t pos = ncav + (uint32_t)__popcll(mi & below);
                    if (GLOBAL) cavg[pos] = ncode;
                    else cavl[pos] = (uint16_t)((at << 2) | (uint32_t)code_facet(ncode));
                }
                if (outside) {
                    // boundary facet: (local index of c) << 2 | f, and the outer tetrahedron
                    const uint32_t pos = nbnd + (uint32_t)__popcll(mo & below);
                    bnd[pos] = (slot << 2) | (uint32_t)f;
                    outc[pos] = ncode;
                }
                ncav += ni;
                nbnd += no;
                pneed = need;
                pinside = inside;
                po1 = o1;
                lane_fence<GLOBAL>();
            }
            if (status == ST_NONE && (__ballot(pneed && po1 < S && (pinside || !(po1 & 1ull))) & gmask))
                status = ST_CONFLICT;
            if (status == ST_NONE) status = ST_CAND;
        }
        if (!GLOBAL && status == ST_CAND)
            for (uint32_t k = gl; k < ncav; k += GS) {
                const uint32_t q = cavl[k];
                cavg[k] = make_code<K>((uint32_t)(mem[q >> 2] >> 1), q & 3u);
            }
        if (clocked && gl == 0) {
            unsigned long long *r = a.clk + 8ull * i;
            r[0] = tc0;
            r[1] = tc1;
            r[2] = (unsigned long long)wall_clock64();
            r[3] = (unsigned long long)min(ws, 0xFFFFu) | ((unsigned long long)min(cav_steps, 0xFFFFu) << 16) |
                   ((unsigned long long)min(ncav, 0xFFFFu) << 32) | ((unsigned long long)status << 48);
        }
        if (gl == 0) {
            a.status[i] = status;
            a.cnt[i] = ncav;
            a.cnt[stride + i] = nbnd;
            if (!FULL && status == ST_FULL) a.defer[atomicAdd(a.ndefer_ptr, 1u)] = i;
            else attempt++;  // a deferred attempt is counted by the FULL kernel
        }
    }
    if (gl != 0) steps = 0;
    add_stat(a.stat, STAT_ATTEMPTS, attempt);
    add_stat(a.stat, STAT_WALK, steps);
    add_stat(a.stat, STAT_ORIENT, st.orient);
    add_stat(a.stat, STAT_ORIENT_EXACT, st.orient_exact);
    add_stat(a.stat, STAT_INSPHERE, st.insphere);
    add_stat(a.stat, STAT_INSPHERE_EXACT, st.insphere_exact);
    add_stat(a.stat, STAT_PERTURBED, st.perturbed);
}

// Walk and cavity search of one candidate per 256-thread block, for rounds of large
// cavities (exact predicates throughout).  The four waves walk the same path independently
// (the walk reads nothing that changes during the kernel, so they arrive at the same
// tetrahedron); the cavity search then expands 64 cavity tetrahedra per step, thread
// (slot, facet) = (tid / 4, tid % 4), with block-wide prefix counts for the appends and a
// barrier between steps.  Queue and set are in LDS (CAPL and HM entries) or, with GLOBAL, in
// global memory as in k_cavity_g.  Claims, set and status follow k_cavity_g.
template <class K, uint32_t CAPL, uint32_t HM, bool GLOBAL>
__global__ __launch_bounds__(256) void k_cavity_b(RoundArgs a) {
    using code = typename K::code;
    using E = typename K::set_t;
    __shared__ uint16_t s_cav[GLOBAL ? 1 : CAPL];
    __shared__ E s_mem[GLOBAL ? 1 : HM];
    __shared__ uint32_t s_cnt[2][4];
    __shared__ int s_flag;
    typename K::Rec *const T = static_cast<typename K::Rec *>(a.T);
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u, wid = tid >> 6;
    const unsigned long long below = (1ull << lane) - 1ull;
    const uint32_t i = blockIdx.x;
    if (i >= *a.ncand_ptr) return;  // uniform over the block
    PredStats st;
    uint8_t status = ST_NONE;
    const uint32_t p = a.cand_pt[i];
    const unsigned long long S = a.round_hi | (2ull * a.cand_rank[i]);
    const Vert pv = a.V[p];
    const P3 P = {pv.x, pv.y, pv.z};
    // start as in k_cavity_g, probing 32 records on either side of p
    Cloud *cl = &a.clouds[pv.idx >> 32];
    const uint32_t clo = cl->lo, chi = cl->hi;
    const uint32_t d = (lane >> 1) + 1;
    const uint32_t hp = (lane & 1) ? p + d : p - d;
    const bool inr = (lane & 1) ? (p + d < a.vhi) : (p >= a.vlo + d);
    const uint32_t ht = inr && hp >= clo && hp < chi ? a.vtet[hp] : NONE;
    const uint32_t q = a.anchor[p - a.vlo];
    const uint32_t tq = q != NONE ? a.vtet[q] : NONE;
    const uint32_t tl = a.lastt[p - a.vlo];
    const unsigned long long hmask = __ballot(ht != NONE);
    uint32_t t = hmask ? __shfl(ht, __ffsll((long long)hmask) - 1) : tq;
    if (a.wbucket && tq != NONE && a.wbucket[p - a.vlo]) t = tq;
    if (t == NONE) t = cl->any_live;
    uint4 w;
    bool from_last = false;
    if (tl != NONE) {
        w = T[tl].v;
        from_last = w.x != DEAD && (!a.multi || (a.V[w.x].idx >> 32) == (pv.idx >> 32));
    }
    if (from_last) {
        t = tl;
    } else {
        w = T[t].v;
    }
    if (w.x == DEAD) {
        t = cl->any_live;
        w = T[t].v;
    }
    if (w.w == GHOST) {
        t = code_slot(comp(T[t].n, 3));
        w = T[t].v;
    }
    // walk: lane j < 4 of each wave tests facet j
    int entry = -1;
    bool in_ghost = false;
    const int jl = (int)(lane & 3u);
    unsigned ws = 0;
    for (;;) {
        const P3 q0 = vpos(a.V, w.x), q1 = vpos(a.V, w.y), q2 = vpos(a.V, w.z), q3 = vpos(a.V, w.w);
        const typename K::code4 nn = T[t].n;
        int o = 1;
        if (lane < 4 && jl != entry)
            o = cav_orient<true>(jl == 0 ? P : q0, jl == 1 ? P : q1, jl == 2 ? P : q2, jl == 3 ? P : q3, st);
        const unsigned bits = (unsigned)__ballot(o < 0) & 0xFu;
        if (!bits) break;
        const unsigned rot = (p + ws) & 3u;
        const unsigned rb = ((bits >> rot) | (bits << (4u - rot))) & 0xFu;
        const int moved = (int)(((unsigned)__ffs(rb) - 1u + rot) & 3u);
        const code cd = comp(nn, moved);
        t = code_slot(cd);
        entry = code_facet(cd);
        w = T[t].v;
        if (++ws > WALK_LIMIT) {
            status = ST_ERROR;
            break;
        }
        if (w.w == GHOST) {
            in_ghost = true;
            break;
        }
    }
    if (tid == 0 && status != ST_ERROR) a.lastt[p - a.vlo] = t;
    const uint32_t walk_or = st.orient, walk_orx = st.orient_exact;
    if (status == ST_NONE && !in_ghost) {
        bool same = false;
        if (lane < 4) {
            const P3 v = vpos(a.V, comp(w, jl));
            same = v.x == P.x && v.y == P.y && v.z == P.z;
        }
        if (__ballot(same)) status = ST_DUP;
    }
    uint32_t ncav = 0, nbnd = 0;
    const uint32_t capL = GLOBAL ? a.capC : min(a.capC, CAPL), capF = a.capF;
    uint32_t *bnd = a.bnd + (size_t)i * a.capF;
    code *outc = static_cast<code *>(a.outc) + (size_t)i * a.capF;
    code *cavg = static_cast<code *>(a.cav) + (size_t)i * a.capC;
    const uint32_t hms = GLOBAL ? a.hmg : HM;
    E *mem = GLOBAL ? reinterpret_cast<E *>(a.scr_v + (size_t)i * a.capC) : s_mem;
    if (status == ST_NONE) {
        for (uint32_t h = tid; h < hms; h += 256) mem[h] = mem_empty<E>();
        if (GLOBAL) __threadfence_block();
        __syncthreads();
        bool pneed = tid == 0, pinside = true;
        unsigned long long po1 = ~0ull;
        if (tid == 0) {
            po1 = atomicMin(&T[t].claim, S);
            uint32_t at = 0;
            mem_insert(mem, hms, t, 0u, &at);
            if (GLOBAL) cavg[0] = make_code<K>(t, 0u);
            else s_cav[0] = (uint16_t)(at << 2);
        }
        ncav = 1;
        if (GLOBAL) __threadfence_block();
        __syncthreads();
        for (uint32_t k0 = 0, nproc = 0; k0 < ncav && status == ST_NONE; k0 += nproc) {
            nproc = min(64u, ncav - k0);
            const uint32_t slot = k0 + (tid >> 2);
            const int f = (int)(tid & 3u);
            const bool lv = slot < k0 + nproc;
            code cd = 0u;
            if (lv) {
                if (GLOBAL) {
                    cd = cavg[slot];
                } else {
                    const uint32_t qe = s_cav[slot];
                    cd = make_code<K>((uint32_t)(mem[qe >> 2] >> 1), qe & 3u);
                }
            }
            const uint32_t c = code_slot(cd);
            const int pf = slot == 0 ? -1 : code_facet(cd);
            const bool act = lv && f != pf;
            uint4 cv = make_uint4(0u, 0u, 0u, 0u), uw = cv;
            typename K::code4 cn{};
            if (lv) {
                cv = T[c].v;
                cn = T[c].n;
            }
            // the previous step's claims (as in k_cavity_g)
            if (__syncthreads_or(pneed && po1 < S && (pinside || !(po1 & 1ull)))) {
                status = ST_CONFLICT;
                break;
            }
            const code ncode = comp(cn, f);
            const uint32_t u = code_slot(ncode);
            const int kind = act ? mem_find<GLOBAL>(mem, hms, u) : -1;
            const bool need = act && kind < 0;
            if (need) uw = T[u].v;
            bool inside = false;
            if (need) {
                const bool cghost = cv.w == GHOST;
                const uint32_t apex = comp(uw, code_facet(ncode));
                if (!cghost && apex != GHOST) {
                    const uint32_t cid[4] = {cv.x, cv.y, cv.z, cv.w};
                    uint32_t rid[4];
#pragma unroll
                    for (int m = 0; m < 4; ++m) rid[m] = m == f ? apex : cid[m];
                    const int sa = (f + 1) & 3, sb = (f + 2) & 3;
                    uint32_t r2[4];
#pragma unroll
                    for (int m = 0; m < 4; ++m) r2[m] = m == sa ? rid[sb] : (m == sb ? rid[sa] : rid[m]);
                    inside = cav_insphere<true>(vpos(a.V, r2[0]), vpos(a.V, r2[1]), vpos(a.V, r2[2]),
                                                vpos(a.V, r2[3]), P,
                                                [&](int kk) { return kk < 4 ? a.V[r2[kk]].idx : pv.idx; }, st) < 0;
                } else if (!cghost) {
                    const P3 c0 = vpos(a.V, cv.x), c1 = vpos(a.V, cv.y), c2 = vpos(a.V, cv.z), c3 = vpos(a.V, cv.w);
                    inside = cav_orient<true>(f == 0 ? P : c0, f == 1 ? P : c1, f == 2 ? P : c2, f == 3 ? P : c3,
                                              st) <= 0;
                } else {
                    inside = tet_inside<K, true>(T, a.V, u, P, pv.idx, st) < 0;
                }
            }
            unsigned long long o1 = ~0ull;
            if (need) o1 = atomicMin(&T[u].claim, inside ? S : S + 1);
            int ins = 0;
            uint32_t at = 0;
            if (need) ins = mem_insert(mem, hms, u, inside ? 0u : 1u, &at);
            const bool first_in = ins == 1 && inside;
            const bool outside = (act && kind == 1) || (need && !inside);
            const unsigned long long mi = __ballot(first_in), mo = __ballot(outside);
            const unsigned long long mf = __ballot(ins < 0);
            if (lane == 0) {
                s_cnt[0][wid] = (uint32_t)__popcll(mi);
                s_cnt[1][wid] = (uint32_t)__popcll(mo);
            }
            if (tid == 0) s_flag = 0;
            __syncthreads();
            if (lane == 0 && mf) s_flag = 1;
            uint32_t bi = 0, bo = 0, ni = 0, no = 0;
#pragma unroll
            for (uint32_t v = 0; v < 4; ++v) {
                if (v < wid) {
                    bi += s_cnt[0][v];
                    bo += s_cnt[1][v];
                }
                ni += s_cnt[0][v];
                no += s_cnt[1][v];
            }
            __syncthreads();
            if (ncav + ni > capL || nbnd + no > capF || s_flag) {
                status = ST_OVERFLOW;
                break;
            }
            if (first_in) {
                const uint32_t pos = ncav + bi + (uint32_t)__popcll(mi & below);
                if (GLOBAL) cavg[pos] = ncode;
                else s_cav[pos] = (uint16_t)((at << 2) | (uint32_t)code_facet(ncode));
            }
            if (outside) {
                const uint32_t pos = nbnd + bo + (uint32_t)__popcll(mo & below);
                bnd[pos] = (slot << 2) | (uint32_t)f;
                outc[pos] = ncode;
            }
            ncav += ni;
            nbnd += no;
            pneed = need;
            pinside = inside;
            po1 = o1;
            if (GLOBAL) __threadfence_block();
            __syncthreads();
        }
        if (status == ST_NONE && __syncthreads_or(pneed && po1 < S && (pinside || !(po1 & 1ull))))
            status = ST_CONFLICT;
        if (status == ST_NONE) status = ST_CAND;
    }
    if (!GLOBAL && status == ST_CAND)
        for (uint32_t k = tid; k < ncav; k += 256) {
            const uint32_t qe = s_cav[k];
            cavg[k] = make_code<K>((uint32_t)(mem[qe >> 2] >> 1), qe & 3u);
        }
    if (tid == 0) {
        a.status[i] = status;
        a.cnt[i] = ncav;
        a.cnt[a.stride + i] = nbnd;
    }
    add_stat(a.stat, STAT_ATTEMPTS, tid == 0 ? 1u : 0u);
    add_stat(a.stat, STAT_WALK, tid == 0 ? ws : 0u);
    // the four waves repeated the walk's orientation tests: wave 0's count them
    add_stat(a.stat, STAT_ORIENT, wid == 0 ? st.orient : st.orient - walk_or);
    add_stat(a.stat, STAT_ORIENT_EXACT, wid == 0 ? st.orient_exact : st.orient_exact - walk_orx);
    add_stat(a.stat, STAT_INSPHERE, st.insphere);
    add_stat(a.stat, STAT_INSPHERE_EXACT, st.insphere_exact);
    add_stat(a.stat, STAT_PERTURBED, st.perturbed);
}

// Winner test, slot reservation and DelaunayBall (Sec. 2.5), GL lanes per candidate, all in
// one wave.  An attempt wins iff no lower attempt touched a tetrahedron of its cavity (the
// claim word still holds its stamp) and the lowest claim on each of its outer tetrahedra is
// an outer claim (a lower attempt with that tetrahedron in its cavity then loses on it);
// winners of one round therefore have disjoint cavities, and no cavity meets another
// winner's outer tetrahedra, so winners build concurrently without further coordination
// (claim words are only written by the cavity kernel, so the test of one candidate is not
// affected by the building of another).
//
// The ball takes the cavity's own slots (and F - C more when it is larger).  The
// tetrahedron on boundary facet f of cavity tetrahedron k is k with vertex f replaced by p
// (the cavity is star-shaped from p, so p lies on v_f's side of the facet and the
// orientation is kept; a ghost vertex stays in slot 3), glued a priori to the outer
// tetrahedron.  Its other three facets pass through p and one edge of its boundary facet;
// the cavity boundary is a closed surface, so each edge lies on exactly two boundary
// facets, and the two new tetrahedra on them are the siblings.  They are paired through a
// hash table of edges in LDS.  Balls too large for the table pair siblings by pivoting
// around the edge through copies of the cavity tetrahedra instead.
constexpr uint32_t HT = 128;             // edge table entries per candidate
constexpr uint32_t HT_MAX_FACETS = 64;   // balls up to this size use the table (load <= 3/4)
constexpr unsigned long long HT_EMPTY = ~0ull;
// threads per block of the ball kernel: the slot reservation is one atomic per block on one
// counter, so larger blocks contend less (at the cost of LDS occupancy)
constexpr int BALL_BLOCK = 1024;

// orders the memory accesses of one group (all in one wave) across phases
__device__ __forceinline__ void group_fence() {
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint32_t edge_hash(unsigned long long key) {
    return (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> 57);  // 7 bits: HT = 128
}

template <class K, int GL, int BS>
__global__ __launch_bounds__(BS) void k_ball(RoundArgs a) {
    using code = typename K::code;
    constexpr code LOC_BOUNDARY = (code)1 << (8 * sizeof(code) - 1);
    constexpr uint32_t GPB = BS / GL;
    // edge table: key = the edge's two vertices; value = (boundary facet b << 2 | facet q of
    // b's new tetrahedron) for the two new tetrahedra on the edge; the slot of b's new
    // tetrahedron is in s_slot[b] (b < HT_MAX_FACETS on this path)
    __shared__ unsigned long long s_key[GPB][HT];
    __shared__ uint16_t s_val[GPB][HT][2];
    __shared__ uint32_t s_slot[GPB][HT_MAX_FACETS];
    typename K::Rec *const T = static_cast<typename K::Rec *>(a.T);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t gl = threadIdx.x % GL;
    const uint32_t gi = threadIdx.x / GL;
    const uint32_t gbase = lane & ~(uint32_t)(GL - 1);
    const unsigned long long gmask = GL == 64 ? ~0ull : (((1ull << (GL & 63)) - 1ull) << gbase);
    const uint32_t i = blockIdx.x * GPB + gi;
    const uint32_t ncand = *a.ncand_ptr;
    const uint32_t stride = a.stride, capC = a.capC, capF = a.capF;
    unsigned cav_w = 0, bnd_w = 0;
    const unsigned long long tb0 = a.clk ? (unsigned long long)wall_clock64() : 0ull;
    const bool cand = i < ncand && a.status[i] == ST_CAND;
    uint32_t p = 0, nc = 0, nb = 0;
    unsigned long long S = 0;
    const code *cavl = static_cast<const code *>(a.cav) + (size_t)i * capC;
    const uint32_t *bl = a.bnd + (size_t)i * capF;
    code *ol = static_cast<code *>(a.outc) + (size_t)i * capF;
    uint4 *sv = a.scr_v + (size_t)i * capC;
    typename K::code4 *sn = static_cast<typename K::code4 *>(a.scr_n) + (size_t)i * capC;
    bool ok = true;
    if (cand) {
        p = a.cand_pt[i];
        S = a.round_hi | (2ull * a.cand_rank[i]);
        nc = a.cnt[i];
        nb = a.cnt[stride + i];
        // winner test
        // cavity tetrahedra: no lower claim; outer tetrahedra: the lowest claim is an outer
        // one (any lower attempt with it in its cavity then loses on that claim)
        for (uint32_t k = gl; k < nc; k += GL) ok &= T[code_slot(cavl[k])].claim == S;
        for (uint32_t k = gl; k < nb; k += GL) ok &= (T[code_slot(ol[k])].claim & 1ull) != 0;
    }
    const bool win = cand && (__ballot(!ok) & gmask) == 0;
    // slot reservation by each winner's first lane, one atomic per block: the F - C extra
    // slots are units of fl_take (units below fl_n are free-list entries of earlier rounds,
    // the rest are fresh pool slots from tet_count on); C - F surplus cavity slots are freed
    const bool leader = win && gl == 0;
    const uint32_t need = leader && nb > nc ? nb - nc : 0u;
    const uint32_t u0 = block_reserve<BS / 64>(need, &a.ctr->fl_take, &s_slot[0][0]);
    const uint32_t fln = a.ctr->fl_n, tc0 = a.ctr->tet_count;
    const bool full = need && u0 + need > fln && (uint64_t)tc0 + (u0 + need - fln) > a.tcap;
    if (full) {
        // pool full: give the units back (pool slots inside the pool are marked free) and
        // retry next round after the host has grown the pool
        uint32_t give = 0;
        for (uint32_t k = 0; k < need; ++k) {
            const uint32_t u = u0 + k;
            if (u < fln || (uint64_t)tc0 + (u - fln) < a.tcap) ++give;
        }
        const uint32_t g0 = atomicAdd(&a.ctr->fl_next, give);
        uint32_t q = 0;
        for (uint32_t k = 0; k < need; ++k) {
            const uint32_t u = u0 + k;
            uint32_t slot = NONE;
            if (u < fln) {
                slot = a.fl_cur[u];
            } else if ((uint64_t)tc0 + (u - fln) < a.tcap) {
                slot = tc0 + (u - fln);
                T[slot].v.x = DEAD;
            }
            // a slot that does not fit the free list stays free and unused (k_roll counts it)
            if (slot != NONE && (uint64_t)g0 + q < a.flcap) a.fl_next[g0 + q] = slot;
            if (slot != NONE) ++q;
        }
        atomicOr(&a.ctr->error, ERR_POOL);
    }
    const bool lbuilt = leader && !full;
    const uint32_t fb = lbuilt && nc > nb ? atomicAdd(&a.ctr->fl_next, nc - nb) : 0u;  // rare
    if (cand && gl == 0) a.status[i] = lbuilt ? ST_WON : ST_CONFLICT;
    const bool built = __shfl((int)lbuilt, (int)gbase) != 0;
    const uint32_t g_u0 = __shfl(u0, (int)gbase), g_fb = __shfl(fb, (int)gbase);
    const unsigned long long tb1 = a.clk ? (unsigned long long)wall_clock64() : 0ull;
    unsigned long long tb2 = tb1;
    if (built) {
        const bool table = nb <= HT_MAX_FACETS;
        // A: copies of the cavity tetrahedra (vertices; for the pivot also the neighbours and
        // the local index in the spare word); the edge table is cleared
        for (uint32_t k = gl; k < nc; k += GL) {
            const uint32_t c = code_slot(cavl[k]);
            sv[k] = T[c].v;
            if (!table) {
                sn[k] = T[c].n;
                T[c].spare[0] = k;
            }
        }
        if (table)
            for (uint32_t h = gl; h < HT; h += GL) s_key[gi][h] = HT_EMPTY;
        group_fence();
        if (a.clk) tb2 = (unsigned long long)wall_clock64();
        if (!table) {
            // B (pivot only): facets between two cavity tetrahedra -> local codes
            for (uint32_t task = gl; task < 4 * nc; task += GL) {
                const uint32_t k = task >> 2;
                const int f = (int)(task & 3u);
                const code cd = comp(sn[k], f);
                const uint32_t nt = code_slot(cd);
                if (T[nt].claim == S)  // only this winner's cavity tetrahedra hold S
                    reinterpret_cast<code *>(&sn[k])[f] = make_code<K>((uint32_t)T[nt].spare[0], code_facet(cd));
            }
            group_fence();
        }
        // C: one new tetrahedron per boundary facet (k, f): k with v_f replaced by p
        for (uint32_t b = gl; b < nb; b += GL) {
            uint32_t slot;
            if (b < nc) {
                slot = code_slot(cavl[b]);
            } else {
                const uint32_t u = g_u0 + (b - nc);
                slot = u < fln ? a.fl_cur[u] : tc0 + (u - fln);
            }
            const uint32_t bc = bl[b];  // local index of the cavity tetrahedron << 2 | facet
            const uint32_t kb = bc >> 2;
            const int f = (int)(bc & 3u);
            const code oc = ol[b];
            const uint4 cw = sv[kb];
            uint32_t wv[4] = {cw.x, cw.y, cw.z, cw.w};
            wv[f] = p;
            T[slot].v = make_uint4(wv[0], wv[1], wv[2], wv[3]);
            if (a.subd && wv[3] != GHOST)
                static_cast<SubD *>(a.subd)[slot] =
                    subdets(vpos(a.V, wv[0]), vpos(a.V, wv[1]), vpos(a.V, wv[2]), vpos(a.V, wv[3]));
            const code me = make_code<K>(slot, (uint32_t)f);
            nref(T, slot, f) = oc;                            // facet opposite p: the outer tetrahedron
            nref(T, code_slot(oc), code_facet(oc)) = me;      // and back
            ol[b] = me;
            // vertex hints: the cavity boundary's vertices from every new tetrahedron on them,
            // the new point (vertex f of each) from the first only
            for (int q = 0; q < 4; ++q)
                if (wv[q] != GHOST && (q != f || b == 0)) a.vtet[wv[q]] = slot;
            if (table) {
                // the three facets through p: facet q holds p and the edge of the boundary
                // facet without vertex q
                for (int q = 0; q < 4; ++q) {
                    if (q == f) continue;
                    uint32_t e0 = NONE, e1 = NONE;
                    for (int r = 0; r < 4; ++r)
                        if (r != q && r != f) {
                            if (e0 == NONE) e0 = wv[r];
                            else e1 = wv[r];
                        }
                    const unsigned long long key = e0 < e1 ? ((unsigned long long)e0 << 32) | e1
                                                           : ((unsigned long long)e1 << 32) | e0;
                    uint32_t h = edge_hash(key);
                    bool placed = false;
                    for (uint32_t probe = 0; probe < HT && !placed; ++probe) {
                        const unsigned long long old = atomicCAS(&s_key[gi][h], HT_EMPTY, key);
                        if (old == HT_EMPTY || old == key) {
                            s_val[gi][h][old == HT_EMPTY ? 0 : 1] = (uint16_t)((b << 2) | (uint32_t)q);
                            placed = true;
                        }
                        h = (h + 1) & (HT - 1);
                    }
                    if (!placed) atomicOr(&a.ctr->error, ERR_WALK);
                }
                s_slot[gi][b] = slot;
            } else {
                reinterpret_cast<code *>(&sn[kb])[f] = LOC_BOUNDARY | (code)b;
            }
        }
        group_fence();
        // D: the three siblings of each new tetrahedron
        if (table) {
            for (uint32_t b = gl; b < nb; b += GL) {
                const code me = ol[b];
                const uint32_t slot = code_slot(me);
                const int f = code_facet(me);
                const uint4 cw = sv[bl[b] >> 2];
                uint32_t wv[4] = {cw.x, cw.y, cw.z, cw.w};
                wv[f] = p;
                for (int q = 0; q < 4; ++q) {
                    if (q == f) continue;
                    uint32_t e0 = NONE, e1 = NONE;
                    for (int r = 0; r < 4; ++r)
                        if (r != q && r != f) {
                            if (e0 == NONE) e0 = wv[r];
                            else e1 = wv[r];
                        }
                    const unsigned long long key = e0 < e1 ? ((unsigned long long)e0 << 32) | e1
                                                           : ((unsigned long long)e1 << 32) | e0;
                    const uint32_t mine = (b << 2) | (uint32_t)q;
                    uint32_t h = edge_hash(key), res = NONE;
                    for (uint32_t probe = 0; probe < HT; ++probe) {
                        if (s_key[gi][h] == key) {
                            const uint32_t v0 = s_val[gi][h][0], v1 = s_val[gi][h][1];
                            res = v0 == mine ? v1 : v0;
                            break;
                        }
                        h = (h + 1) & (HT - 1);
                    }
                    if (res == NONE) atomicOr(&a.ctr->error, ERR_WALK);
                    else nref(T, slot, q) = make_code<K>(s_slot[gi][res >> 2], res & 3u);
                }
            }
        } else {
            for (uint32_t task = gl; task < 3 * nb; task += GL) {
                const uint32_t b = task / 3, qi = task - 3 * b;
                const code me = ol[b];
                const uint32_t slot = code_slot(me);
                const int pf = code_facet(me);
                const int q = (pf + 1 + (int)qi) & 3;  // the three facets through p
                const uint32_t kb = bl[b] >> 2;
                const uint4 cw = sv[kb];
                const uint32_t c4[4] = {cw.x, cw.y, cw.z, cw.w};
                uint32_t e[2];
                int ne = 0;
                for (int r = 0; r < 4; ++r)
                    if (r != q && r != pf) e[ne++] = c4[r];
                uint32_t k = kb;
                int f = pf;
                code res = 0;
                bool found = false;
                for (uint32_t guard = 0; guard <= nc + 1; ++guard) {
                    const uint4 cv = sv[k];
                    const uint32_t v4[4] = {cv.x, cv.y, cv.z, cv.w};
                    int xpos = -1;
                    for (int m = 0; m < 4; ++m)
                        if (m != f && v4[m] != e[0] && v4[m] != e[1]) xpos = m;
                    if (xpos < 0) break;
                    const code lc = comp(sn[k], xpos);
                    if (lc & LOC_BOUNDARY) {
                        // boundary facet (k, xpos): its new tetrahedron has p at xpos, and
                        // the facet through p, e0, e1 is opposite its vertex f
                        res = make_code<K>(code_slot(ol[(size_t)(lc & ~LOC_BOUNDARY)]), (uint32_t)f);
                        found = true;
                        break;
                    }
                    k = code_slot(lc);
                    f = code_facet(lc);
                    if (k >= nc) break;
                }
                if (!found) atomicOr(&a.ctr->error, ERR_WALK);
                else nref(T, slot, q) = res;
            }
        }
        // E: cavity slots beyond the ball's size are freed.  The cloud's known live
        // tetrahedron stays live unless it is one of them (the other cavity slots hold the
        // new tetrahedra): then it moves to the ball's first tetrahedron.  Only this rare
        // case writes it, so winners do not all store to one address.
        if (nc > nb) {
            Cloud *cl = &a.clouds[a.V[p].idx >> 32];
            const uint32_t live = cl->any_live;
            for (uint32_t k = nb + gl; k < nc; k += GL) {
                const uint32_t c = code_slot(cavl[k]);
                T[c].v.x = DEAD;
                // a slot that does not fit the free list stays free and unused (k_roll counts it)
                if ((uint64_t)g_fb + (k - nb) < a.flcap) a.fl_next[g_fb + (k - nb)] = c;
                if (c == live) cl->any_live = code_slot(cavl[0]);
            }
        }
        if (gl == 0) {
            cav_w = nc;
            bnd_w = nb;
        }
    }
    if (a.clk && cand && gl == 0) {
        unsigned long long *r = a.clk + 8ull * i + 4;
        r[0] = tb0;
        r[1] = tb1;
        r[2] = built ? tb2 : 0ull;
        r[3] = built ? (unsigned long long)wall_clock64() : 0ull;
    }
    add_stat(a.stat, STAT_CAV_TETS, cav_w);
    add_stat(a.stat, STAT_BND_FACETS, bnd_w);
}

// ------------------------------------------------------------------ round end

__global__ __launch_bounds__(FILL_BLOCK) void k_compact(RoundArgs a) {
    constexpr int NW = FILL_BLOCK / 64;
    __shared__ uint32_t s_tmp[NW + 1];
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t ncand = *a.ncand_ptr;
    const uint8_t s = i < ncand ? a.status[i] : (uint8_t)ST_NONE;
    // ST_FULL left by a round whose exact pass was not launched: the attempt retries
    const bool again = i < ncand && (s == ST_CONFLICT || s == ST_CAND || s == ST_WALK || s == ST_FULL);
    const bool ovf = i < ncand && s == ST_OVERFLOW;
    if (a.log_att && i < ncand) atomicAdd(&a.log_att[a.cand_pt[i] - a.vlo], 1u);
    const uint32_t pn = block_reserve<NW>(again ? 1u : 0u, a.nnext_ptr, s_tmp);
    const uint32_t po = block_reserve<NW>(ovf ? 1u : 0u, a.novf_ptr, s_tmp);
    if (again) {
        a.next_pt[pn] = a.cand_pt[i];
        a.next_rank[pn] = a.cand_rank[i];
    }
    if (ovf) {
        a.ovf_pt[po] = a.cand_pt[i];
        a.ovf_rank[po] = a.cand_rank[i];
    }
    // the round's counts: one atomic per block and counter
    block_reserve<NW>(again ? 1u : 0u, &a.ctr->conflicts, s_tmp);
    block_reserve<NW>(ovf ? 1u : 0u, &a.ctr->overflows, s_tmp);
    block_reserve<NW>(i < ncand && s == ST_WON ? 1u : 0u, &a.ctr->won, s_tmp);
    block_reserve<NW>(i < ncand && s == ST_DUP ? 1u : 0u, &a.ctr->dups, s_tmp);
    block_reserve<NW>(i < ncand && s == ST_WALK ? 1u : 0u, &a.ctr->walk_caps, s_tmp);
    const bool bad = i < ncand && !(again || ovf || s == ST_WON || s == ST_DUP);
    if (bad) atomicOr(&a.ctr->error, ERR_WALK);
}

// carry the unused part of this round's free list behind the slots freed this round (as far
// as the list holds them; k_roll counts the rest)
__global__ void k_freelist_carry(RoundArgs a) {
    const uint32_t fln = a.ctr->fl_n, take = a.ctr->fl_take, nxt = min(a.ctr->fl_next, a.flcap);
    if (take >= fln) return;
    const uint32_t left = min(fln - take, a.flcap - nxt);
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < left; k += gridDim.x * blockDim.x)
        a.fl_next[nxt + k] = a.fl_cur[take + k];
}

// Round end: statistics summed, the pool's counters advanced.  With `snap` (pinned host
// memory), the counters are then written there and `seq` (host memory too) is set to `tag`
// after them with a release at system scope: the host waits for that value instead of for a
// copy and an event.
__global__ void k_roll(Ctr *ctr, uint32_t *consumed, uint32_t tcap, uint32_t flcap, const unsigned long long *stat,
                       Ctr *snap, unsigned long long *seq, unsigned long long tag) {
    const uint32_t t = threadIdx.x;
    if (t < NSTAT) {
        unsigned long long sum = 0;
        for (int k = 0; k < STAT_SPREAD; ++k) sum += stat[((size_t)t * STAT_SPREAD + k) * STAT_PAD];
        unsigned long long *dst[NSTAT] = {&ctr->attempts, &ctr->walk_steps, &ctr->orient, &ctr->orient_exact,
                                         &ctr->insphere, &ctr->insphere_exact, &ctr->perturbed,
                                         &ctr->cav_tets, &ctr->bnd_facets};
        *dst[t] = sum;
    }
    __syncthreads();
    if (t == 0) {
    const uint32_t fln = ctr->fl_n, take = ctr->fl_take;
    if (take > fln) {
        // units beyond the free list were fresh pool slots (beyond the pool: never used)
        const unsigned long long tc = (unsigned long long)ctr->tet_count + (take - fln);
        ctr->tet_count = tc > tcap ? tcap : (uint32_t)tc;
    }
    const uint32_t left = take < fln ? fln - take : 0u;
    const uint32_t nxt = min(ctr->fl_next, flcap), keep = min(left, flcap - nxt);
    ctr->dropped += (ctr->fl_next - nxt) + (left - keep);
    ctr->deferred += ctr->ndefer;
    ctr->ndefer = 0;
    ctr->fl_n = nxt + keep;
    ctr->fl_take = 0;
    ctr->fl_next = 0;
    *consumed = 0;  // the list this round read from is empty now
    }
    if (!snap) return;
    __threadfence_block();
    __syncthreads();
    static_assert(sizeof(Ctr) % sizeof(uint32_t) == 0, "the snapshot is copied in words");
    const uint32_t *src = reinterpret_cast<const uint32_t *>(ctr);
    uint32_t *dst = reinterpret_cast<uint32_t *>(snap);
    for (uint32_t k = t; k < sizeof(Ctr) / sizeof(uint32_t); k += blockDim.x) dst[k] = src[k];
    __threadfence_system();
    __syncthreads();
    if (t == 0) __hip_atomic_store(seq, tag, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// The exact-predicate pass: 16 lanes per attempt (its attempts are whole walks and cavity
// searches with the exact stages), grid-stride over the attempts the filter pass handed on
// with up to 16384 of them in flight
constexpr uint32_t EXACT_LANES = 16;
constexpr uint32_t DEFER_BLOCKS = 1024;

template <class K>
static hipError_t launch_round_k(const RoundArgs &a, uint32_t max_cand, uint32_t lanes, uint32_t large_lanes,
                                 bool exact, hipStream_t s, hipEvent_t *ev) {
    constexpr uint32_t LHM = K::LHM;
    if (ev) hipEventRecord(ev[0], s);
    // regular rounds: the filter-only kernel over the round's list, then the exact kernel over
    // the attempts it handed on (a short grid-stride pass; nothing to do for most rounds);
    // rounds for large cavities use exact predicates throughout
    const uint32_t dgrid = std::min<uint32_t>((max_cand + 256 / EXACT_LANES - 1) / (256 / EXACT_LANES), DEFER_BLOCKS);
    const bool blk = large_lanes != 64;
    if (blk && a.capC > BIG_CAPC) {
        if (a.hmg < 4096 || (a.hmg & (a.hmg - 1)) || (uint64_t)a.hmg * sizeof(typename K::set_t) > 16ull * a.capC)
            return hipErrorInvalidValue;
        k_cavity_b<K, 1, 1, true><<<max_cand, 256, 0, s>>>(a);
    } else if (blk && a.capC > LCAPC) {
        k_cavity_b<K, BIG_CAPC, BIG_HM, false><<<max_cand, 256, 0, s>>>(a);
    } else if (a.capC > BIG_CAPC) {
        // the set takes hmg entries of the candidate's 16 capC bytes of ball scratch
        if (a.hmg < 4096 || (a.hmg & (a.hmg - 1)) || (uint64_t)a.hmg * sizeof(typename K::set_t) > 16ull * a.capC)
            return hipErrorInvalidValue;
        k_cavity_g<K, 64, 1, 1, true, true, false><<<(max_cand + 3) / 4, 256, 0, s>>>(a);
    } else if (a.capC > LCAPC) {
        k_cavity_g<K, 64, BIG_CAPC, BIG_HM, false, true, false><<<(max_cand + 3) / 4, 256, 0, s>>>(a);
    } else if (lanes == 4) {
        k_cavity_g<K, 4, LCAPC, LHM, false, false, false><<<(max_cand + 63) / 64, 256, 0, s>>>(a);
        if (exact) k_cavity_g<K, EXACT_LANES, LCAPC, LHM, false, true, true><<<dgrid, 256, 0, s>>>(a);
    } else if (lanes == 8) {
        k_cavity_g<K, 8, LCAPC, LHM, false, false, false><<<(max_cand + 31) / 32, 256, 0, s>>>(a);
        if (exact) k_cavity_g<K, EXACT_LANES, LCAPC, LHM, false, true, true><<<dgrid, 256, 0, s>>>(a);
    } else if (lanes == 32) {
        k_cavity_g<K, 32, LCAPC, LHM, false, false, false><<<(max_cand + 7) / 8, 256, 0, s>>>(a);
        if (exact) k_cavity_g<K, EXACT_LANES, LCAPC, LHM, false, true, true><<<dgrid, 256, 0, s>>>(a);
    } else if (lanes == 64) {
        k_cavity_g<K, 64, LCAPC, LHM, false, false, false><<<(max_cand + 3) / 4, 256, 0, s>>>(a);
        if (exact) k_cavity_g<K, EXACT_LANES, LCAPC, LHM, false, true, true><<<dgrid, 256, 0, s>>>(a);
    } else {
        k_cavity_g<K, 16, LCAPC, LHM, false, false, false><<<(max_cand + 15) / 16, 256, 0, s>>>(a);
        if (exact) k_cavity_g<K, EXACT_LANES, LCAPC, LHM, false, true, true><<<dgrid, 256, 0, s>>>(a);
    }
    if (ev) hipEventRecord(ev[1], s);
    // rounds for large cavities build large balls (their siblings found by pivoting), and
    // short rounds wait on their slowest candidate: a wavefront per candidate
    if (a.capC > LCAPC || lanes == 64)
        k_ball<K, 64, BALL_BLOCK><<<(max_cand + BALL_BLOCK / 64 - 1) / (BALL_BLOCK / 64), BALL_BLOCK, 0, s>>>(a);
    else
        k_ball<K, 16, BALL_BLOCK><<<(max_cand + BALL_BLOCK / 16 - 1) / (BALL_BLOCK / 16), BALL_BLOCK, 0, s>>>(a);
    if (ev && ev[2]) hipEventRecord(ev[2], s);
    return hipGetLastError();
}

hipError_t launch_round(const RoundArgs &a, bool wide, uint32_t max_cand, uint32_t lanes, uint32_t large_lanes,
                        bool exact, hipStream_t s, hipEvent_t *ev) {
    if (max_cand == 0) return hipSuccess;
    return wide ? launch_round_k<Wide>(a, max_cand, lanes, large_lanes, exact, s, ev)
                : launch_round_k<Narrow>(a, max_cand, lanes, large_lanes, exact, s, ev);
}

hipError_t launch_round_end(const RoundArgs &a, uint32_t max_cand, hipStream_t s, Ctr *snap,
                            unsigned long long *seq, unsigned long long tag) {
    if (max_cand) k_compact<<<(max_cand + FILL_BLOCK - 1) / FILL_BLOCK, FILL_BLOCK, 0, s>>>(a);
    k_freelist_carry<<<256, 256, 0, s>>>(a);
    k_roll<<<1, 64, 0, s>>>(a.ctr, const_cast<uint32_t *>(a.ncand_ptr), a.tcap, a.flcap, a.stat, snap, seq, tag);
    return hipGetLastError();
}

// ------------------------------------------------------------------ graph-launched rounds

namespace {

template <class K>
void *cavity_filter_kernel(uint32_t lanes) {
    constexpr uint32_t LHM = K::LHM;
    switch (lanes) {
    case 4: return (void *)k_cavity_g<K, 4, LCAPC, LHM, false, false, false>;
    case 8: return (void *)k_cavity_g<K, 8, LCAPC, LHM, false, false, false>;
    case 32: return (void *)k_cavity_g<K, 32, LCAPC, LHM, false, false, false>;
    case 64: return (void *)k_cavity_g<K, 64, LCAPC, LHM, false, false, false>;
    default: return (void *)k_cavity_g<K, 16, LCAPC, LHM, false, false, false>;
    }
}

int lanes_index(uint32_t lanes) {
    switch (lanes) {
    case 4: return 0;
    case 8: return 1;
    case 32: return 3;
    case 64: return 4;
    default: return 2;
    }
}

}  // namespace

// The kernels and grids are those of launch_fill_list, launch_round (regular rounds) and
// launch_round_end; an empty fill plan runs one block that appends nothing.
hipError_t launch_round_graph(RoundGraph *graphs, const FillPlan &plan, const FillArgs &fa, const RoundArgs &a,
                              bool wide, uint32_t max_cand, uint32_t lanes, Ctr *snap, unsigned long long *seq,
                              unsigned long long tag, hipStream_t s) {
    if (max_cand == 0 || a.capC > LCAPC) return hipErrorInvalidValue;
    const uint32_t L = lanes == 4 || lanes == 8 || lanes == 32 || lanes == 64 ? lanes : 16u;
    RoundGraph &g = graphs[(wide ? 5 : 0) + lanes_index(L)];
    const uint32_t fill_count = plan.off[plan.nblk];
    const uint32_t gl_ball = L == 64 ? 64u : 16u;
    void *k_cav = wide ? cavity_filter_kernel<Wide>(L) : cavity_filter_kernel<Narrow>(L);
    void *k_exact = wide ? (void *)k_cavity_g<Wide, EXACT_LANES, LCAPC, Wide::LHM, false, true, true>
                         : (void *)k_cavity_g<Narrow, EXACT_LANES, LCAPC, Narrow::LHM, false, true, true>;
    void *k_b = wide ? (gl_ball == 64 ? (void *)k_ball<Wide, 64, BALL_BLOCK> : (void *)k_ball<Wide, 16, BALL_BLOCK>)
                     : (gl_ball == 64 ? (void *)k_ball<Narrow, 64, BALL_BLOCK> : (void *)k_ball<Narrow, 16, BALL_BLOCK>);
    // arguments (copied into the graph when set)
    FillPlan pl = plan;
    FillArgs f = fa;
    RoundArgs ra = a;
    Ctr *ctr = a.ctr;
    uint32_t *consumed = const_cast<uint32_t *>(a.ncand_ptr);
    uint32_t tcap = a.tcap, flcap = a.flcap;
    const unsigned long long *stat = a.stat;
    void *fill_args[] = {&pl, &f.lvl_start, &f.lvl_size, &f.lvl_bits, &f.rank_base, &f.lord, &f.dup, &f.vtet,
                         &f.cand_pt, &f.cand_rank, &f.ncand};
    void *round_args[] = {&ra};
    void *roll_args[] = {&ctr, &consumed, &tcap, &flcap, &stat, &snap, &seq, &tag};
    hipKernelNodeParams p[7] = {};
    auto set = [&](int k, void *fn, uint32_t grid, uint32_t block, void **args) {
        p[k].func = fn;
        p[k].gridDim = dim3(grid ? grid : 1u);
        p[k].blockDim = dim3(block);
        p[k].sharedMemBytes = 0;
        p[k].kernelParams = args;
        p[k].extra = nullptr;
    };
    const uint32_t gpb = 256 / L;
    set(0, (void *)k_fill, (fill_count + FILL_BLOCK - 1) / FILL_BLOCK, FILL_BLOCK, fill_args);
    set(1, k_cav, (max_cand + gpb - 1) / gpb, 256, round_args);
    set(2, k_exact, std::min<uint32_t>((max_cand + 256 / EXACT_LANES - 1) / (256 / EXACT_LANES), DEFER_BLOCKS), 256, round_args);
    set(3, k_b, (max_cand + BALL_BLOCK / gl_ball - 1) / (BALL_BLOCK / gl_ball), BALL_BLOCK, round_args);
    set(4, (void *)k_compact, (max_cand + FILL_BLOCK - 1) / FILL_BLOCK, FILL_BLOCK, round_args);
    set(5, (void *)k_freelist_carry, 256, 256, round_args);
    set(6, (void *)k_roll, 1, 64, roll_args);
    hipError_t e;
    if (!g.exec) {
        if ((e = hipGraphCreate(&g.graph, 0)) != hipSuccess) return e;
        for (int k = 0; k < 7; ++k) {
            e = hipGraphAddKernelNode(&g.node[k], g.graph, k ? &g.node[k - 1] : nullptr, k ? 1 : 0, &p[k]);
            if (e != hipSuccess) return e;
        }
        if ((e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0)) != hipSuccess) {
            g.exec = nullptr;
            return e;
        }
    } else {
        for (int k = 0; k < 7; ++k)
            if ((e = hipGraphExecKernelNodeSetParams(g.exec, g.node[k], &p[k])) != hipSuccess) return e;
    }
    return hipGraphLaunch(g.exec, s);
}

void destroy_round_graphs(RoundGraph *graphs) {
    for (int k = 0; k < ROUND_GRAPH_SHAPES; ++k) {
        if (graphs[k].exec) hipGraphExecDestroy(graphs[k].exec);
        if (graphs[k].graph) hipGraphDestroy(graphs[k].graph);
        graphs[k] = RoundGraph{};
    }
}

// Claim words back to the empty value (above every stamp), for the round after the round
// counter's low 32 bits wrap.  A fill kernel rather than a strided memset.
template <class R>
__global__ void k_reset_claims(R *__restrict__ T, uint32_t tcap) {
    for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < tcap; t += (uint64_t)gridDim.x * blockDim.x)
        T[t].claim = ~0ull;
}

hipError_t launch_reset_claims(void *T, bool wide, uint32_t tcap, hipStream_t s) {
    if (tcap == 0) return hipSuccess;
    if (wide) k_reset_claims<<<2048, 256, 0, s>>>((TetW *)T, tcap);
    else k_reset_claims<<<2048, 256, 0, s>>>((Tet *)T, tcap);
    return hipGetLastError();
}

// A pool with 32-bit codes copied into one with 64-bit codes (the code 4 t + f is the same
// number in either width).
__global__ void k_widen(const Tet *__restrict__ src, TetW *__restrict__ dst, uint32_t count) {
    const uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (t >= count) return;
    const Tet r = src[t];
    TetW w;
    w.v = r.v;
    w.n.c[0] = r.n.x;
    w.n.c[1] = r.n.y;
    w.n.c[2] = r.n.z;
    w.n.c[3] = r.n.w;
    w.claim = r.claim;
    w.spare[0] = r.spare[0];
    dst[t] = w;
}

hipError_t launch_widen(const void *src, void *dst, uint32_t count, hipStream_t s) {
    if (count == 0) return hipSuccess;
    k_widen<<<(uint32_t)(((uint64_t)count + 255) / 256), 256, 0, s>>>((const Tet *)src, (TetW *)dst, count);
    return hipGetLastError();
}

// ------------------------------------------------------------------ output

// Per-cloud output.  The live finite tetrahedra are sorted by the cloud of their vertices
// (keys: cloud, or nclouds for ghosts and free slots); cloud c owns sorted positions
// [toff[c], toff[c + 1]); map[t] is the sorted position of tetrahedron t.
template <class R>
__global__ void k_tet_cloud(const R *__restrict__ T, const Vert *__restrict__ V, uint32_t count, uint32_t nclouds,
                            unsigned long long *__restrict__ keys, uint32_t *__restrict__ vals) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const uint4 w = T[t].v;
    keys[t] = (w.x != DEAD && w.w != GHOST) ? (V[w.x].idx >> 32) : (unsigned long long)nclouds;
    vals[t] = t;
}

__global__ void k_seg_bounds(const unsigned long long *__restrict__ keys, uint32_t count, uint32_t nclouds,
                             uint32_t *__restrict__ toff) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= count) return;
    const unsigned long long k = keys[j];
    if (j == 0 || keys[j - 1] != k) toff[k < nclouds ? k : nclouds] = j;
}

__global__ void k_tet_map(const uint32_t *__restrict__ sorted, uint32_t nlive, uint32_t *__restrict__ map) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < nlive) map[sorted[j]] = j;
}

template <class R>
__global__ void k_output_cloud(const R *__restrict__ T, const Vert *__restrict__ V, const uint32_t *__restrict__ sorted,
                               const uint32_t *__restrict__ map, uint32_t tb, uint32_t te, uint64_t vbase,
                               uint32_t *__restrict__ tets, int64_t *__restrict__ nbrs) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= te - tb) return;
    const uint32_t t = sorted[tb + j];
    const uint4 w = T[t].v;
    if (tets) {
        const uint32_t wv[4] = {w.x, w.y, w.z, w.w};
        for (int k = 0; k < 4; ++k) tets[4 * (size_t)j + k] = (uint32_t)((uint32_t)V[wv[k]].idx - vbase);
    }
    if (nbrs) {
        const auto nn = T[t].n;
        for (int k = 0; k < 4; ++k) {
            const uint32_t nt = code_slot(comp(nn, k));
            nbrs[4 * (size_t)j + k] = T[nt].v.w == GHOST ? -1 : (int64_t)map[nt] - (int64_t)tb;
        }
    }
}

hipError_t launch_tet_cloud(const void *T, bool wide, const Vert *V, uint32_t count, uint32_t nclouds,
                            unsigned long long *keys, uint32_t *vals, hipStream_t s) {
    if (count == 0) return hipSuccess;
    if (wide) k_tet_cloud<<<(uint32_t)(((uint64_t)count + 255) / 256), 256, 0, s>>>((const TetW *)T, V, count, nclouds, keys, vals);
    else k_tet_cloud<<<(uint32_t)(((uint64_t)count + 255) / 256), 256, 0, s>>>((const Tet *)T, V, count, nclouds, keys, vals);
    return hipGetLastError();
}

hipError_t launch_seg_bounds(const unsigned long long *keys, uint32_t count, uint32_t nclouds, uint32_t *toff,
                             hipStream_t s) {
    if (count == 0) return hipSuccess;
    k_seg_bounds<<<(uint32_t)(((uint64_t)count + 255) / 256), 256, 0, s>>>(keys, count, nclouds, toff);
    return hipGetLastError();
}

hipError_t launch_tet_map(const uint32_t *sorted, uint32_t nlive, uint32_t *map, hipStream_t s) {
    if (nlive == 0) return hipSuccess;
    k_tet_map<<<(uint32_t)(((uint64_t)nlive + 255) / 256), 256, 0, s>>>(sorted, nlive, map);
    return hipGetLastError();
}

hipError_t launch_output_cloud(const void *T, bool wide, const Vert *V, const uint32_t *sorted, const uint32_t *map,
                               uint32_t tb, uint32_t te, uint64_t vbase, uint32_t *tets, int64_t *nbrs, hipStream_t s) {
    if (te <= tb) return hipSuccess;
    if (wide)
        k_output_cloud<<<(te - tb + 255) / 256, 256, 0, s>>>((const TetW *)T, V, sorted, map, tb, te, vbase, tets, nbrs);
    else
        k_output_cloud<<<(te - tb + 255) / 256, 256, 0, s>>>((const Tet *)T, V, sorted, map, tb, te, vbase, tets, nbrs);
    return hipGetLastError();
}

// Export.  The live finite tetrahedra are numbered in slot order through a bit set: one
// 64-bit word per 64 slots (one wavefront's ballot), and an exclusive scan of the words'
// population counts.  The output index of live slot t is pre[t / 64] plus the live bits
// below t in its word, so the export needs 12 bytes per 64 slots instead of a per-slot map,
// and the neighbour lookups read from this small array, which stays in the caches.
template <class R>
__global__ void k_live_bits(const R *__restrict__ T, uint32_t count, unsigned long long *__restrict__ bits,
                            uint32_t *__restrict__ wcnt) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    bool live = false;
    if (t < count) {
        const uint4 w = T[t].v;
        live = w.x != DEAD && w.w != GHOST;
    }
    const unsigned long long m = __ballot(live);
    const uint32_t word = t >> 6;
    if ((threadIdx.x & 63u) == 0 && word < ((uint64_t)count + 63) / 64) {
        bits[word] = m;
        wcnt[word] = (uint32_t)__popcll(m);
    }
}

__device__ __forceinline__ bool is_live(const unsigned long long *bits, uint32_t t) {
    return (bits[t >> 6] >> (t & 63u)) & 1ull;
}

__device__ __forceinline__ uint32_t out_index(const unsigned long long *bits, const uint32_t *pre, uint32_t t) {
    return pre[t >> 6] + (uint32_t)__popcll(bits[t >> 6] & ((1ull << (t & 63u)) - 1ull));
}

// input index of each vertex record as a compact 4-byte array
__global__ void k_out_vid(const Vert *__restrict__ V, uint32_t nv, uint32_t *__restrict__ vid) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nv) vid[t] = (uint32_t)V[t].idx;
}

// slots [t0, t1): live tetrahedron t goes to output row out_index(t) - obase
template <class R>
__global__ void k_output(const R *__restrict__ T, const uint32_t *__restrict__ vid,
                         const unsigned long long *__restrict__ bits, const uint32_t *__restrict__ pre, uint32_t t0,
                         uint32_t t1, uint32_t obase, uint32_t *__restrict__ tets, int64_t *__restrict__ nbrs) {
    const uint64_t tt = (uint64_t)t0 + blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (tt >= t1) return;
    const uint32_t t = (uint32_t)tt;
    if (!is_live(bits, t)) return;
    const uint32_t o = out_index(bits, pre, t) - obase;
    if (tets) {
        const uint4 w = T[t].v;
        const uint4 out = make_uint4(vid[w.x], vid[w.y], vid[w.z], vid[w.w]);
        *reinterpret_cast<uint4 *>(tets + 4 * (size_t)o) = out;
    }
    if (nbrs) {
        const auto nn = T[t].n;
        const uint32_t nt[4] = {code_slot(comp(nn, 0)), code_slot(comp(nn, 1)), code_slot(comp(nn, 2)),
                                code_slot(comp(nn, 3))};
        long long m[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) m[k] = is_live(bits, nt[k]) ? (long long)out_index(bits, pre, nt[k]) : -1ll;
        longlong2 *dst = reinterpret_cast<longlong2 *>(nbrs + 4 * (size_t)o);
        dst[0] = make_longlong2(m[0], m[1]);
        dst[1] = make_longlong2(m[2], m[3]);
    }
}

hipError_t launch_live_bits(const void *T, bool wide, uint32_t count, unsigned long long *bits, uint32_t *wcnt,
                            hipStream_t s) {
    if (count == 0) return hipSuccess;
    const uint32_t nb = (uint32_t)(((uint64_t)count + 255) / 256);
    if (wide) k_live_bits<<<nb, 256, 0, s>>>((const TetW *)T, count, bits, wcnt);
    else k_live_bits<<<nb, 256, 0, s>>>((const Tet *)T, count, bits, wcnt);
    return hipGetLastError();
}

hipError_t launch_out_vid(const Vert *V, uint32_t nv, uint32_t *vid, hipStream_t s) {
    if (nv == 0) return hipSuccess;
    k_out_vid<<<(nv + 255) / 256, 256, 0, s>>>(V, nv, vid);
    return hipGetLastError();
}

hipError_t launch_output(const void *T, bool wide, const uint32_t *vid, const unsigned long long *bits,
                         const uint32_t *pre, uint32_t t0, uint32_t t1, uint32_t obase, uint32_t *tets, int64_t *nbrs,
                         hipStream_t s) {
    if (t1 <= t0) return hipSuccess;
    const uint32_t nb = (uint32_t)(((uint64_t)(t1 - t0) + 255) / 256);
    if (wide) k_output<<<nb, 256, 0, s>>>((const TetW *)T, vid, bits, pre, t0, t1, obase, tets, nbrs);
    else k_output<<<nb, 256, 0, s>>>((const Tet *)T, vid, bits, pre, t0, t1, obase, tets, nbrs);
    return hipGetLastError();
}

__global__ void k_points_out(const Vert *__restrict__ V, uint32_t nv, double *__restrict__ xyz) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nv) return;
    const Vert v = V[r];
    const size_t i = (uint32_t)v.idx;
    xyz[3 * i] = v.x;
    xyz[3 * i + 1] = v.y;
    xyz[3 * i + 2] = v.z;
}

hipError_t launch_points_out(const Vert *V, uint32_t nv, double *xyz, hipStream_t s) {
    if (nv == 0) return hipSuccess;
    k_points_out<<<(uint32_t)(((uint64_t)nv + 255) / 256), 256, 0, s>>>(V, nv, xyz);
    return hipGetLastError();
}

// ------------------------------------------------------------------ predicate test hook

__global__ void k_predicates(int kind, const double *__restrict__ pts, const int64_t *__restrict__ idx, uint64_t k,
                             int8_t *__restrict__ out) {
    const uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (r >= k) return;
    PredStats st;
    const int np = kind == 0 ? 4 : 5;
    P3 q[5];
    for (int j = 0; j < np; ++j) q[j] = {pts[3 * (np * r + j)], pts[3 * (np * r + j) + 1], pts[3 * (np * r + j) + 2]};
    int s;
    if (kind == 0) s = orient3d(q[0], q[1], q[2], q[3], st);
    else if (kind == 1) s = insphere_raw(q[0], q[1], q[2], q[3], q[4], st);
    else
        s = insphere_perturbed(q[0], q[1], q[2], q[3], q[4],
                               [&](int k) { return (unsigned long long)idx[5 * r + k]; }, st);
    out[r] = (int8_t)s;
}

hipError_t launch_predicates(int kind, const double *pts, const int64_t *idx, uint64_t k, int8_t *out, hipStream_t s) {
    if (k == 0) return hipSuccess;
    k_predicates<<<(unsigned)((k + 255) / 256), 256, 0, s>>>(kind, pts, idx, k, out);
    return hipGetLastError();
}

}  // namespace dtk
