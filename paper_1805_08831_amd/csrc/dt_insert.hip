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

#include "dt_internal.h"
#include "dt_predicates.h"

namespace dtk {

constexpr uint32_t WALK_LIMIT = 1u << 20;

__device__ __forceinline__ P3 vpos(const Vert *V, uint32_t v) {
    Vert r = V[v];
    return {r.x, r.y, r.z};
}

__device__ __forceinline__ uint32_t comp(uint4 q, int k) {
    return k == 0 ? q.x : (k == 1 ? q.y : (k == 2 ? q.z : q.w));
}

// neighbour code of facet f of tetrahedron t, as a 4-byte lvalue
__device__ __forceinline__ uint32_t &nref(Tet *T, uint32_t t, uint32_t f) {
    return reinterpret_cast<uint32_t *>(&T[t].n)[f];
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
__global__ void k_init(const Vert *__restrict__ V, Cloud *__restrict__ clouds, uint32_t first_slot,
                       const uint8_t *__restrict__ dup, Tet *__restrict__ T, uint32_t *__restrict__ vtet,
                       Ctr *__restrict__ ctr) {
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
    uint32_t TV[5][4], N[5][4];
    for (int k = 0; k < 4; ++k) TV[0][k] = v[k];
    for (int j = 0; j < 4; ++j) {
        uint32_t w[4] = {v[0], v[1], v[2], v[3]};
        w[j] = GHOST;
        orient_new_tet(w, j);  // G ends in slot 3: finite facet (w0,w1,w2) faces outward
        for (int k = 0; k < 4; ++k) TV[1 + j][k] = w[k];
        N[0][j] = ((s0 + 1u + j) << 2) | 3u;
        N[1 + j][3] = (s0 << 2) | (uint32_t)j;
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
                    if (same == 3) N[g1][f1] = ((s0 + (uint32_t)g2) << 2) | (uint32_t)f2;
                }
            }
    for (int t = 0; t < 5; ++t) {
        Tet r;
        r.v = make_uint4(TV[t][0], TV[t][1], TV[t][2], TV[t][3]);
        r.n = make_uint4(N[t][0], N[t][1], N[t][2], N[t][3]);
        r.claim = ~0ull;
        r.spare[0] = r.spare[1] = r.spare[2] = 0;
        T[s0 + t] = r;
    }
    for (int k = 0; k < 4; ++k) vtet[v[k]] = s0;
    clouds[c].any_live = s0;
}

hipError_t launch_init(const Vert *V, Cloud *clouds, uint32_t nclouds, uint32_t first_slot, const uint8_t *dup,
                       Tet *T, uint32_t *vtet, Ctr *ctr, hipStream_t s) {
    if (nclouds == 0) return hipSuccess;
    k_init<<<nclouds, 256, 0, s>>>(V, clouds, first_slot, dup, T, vtet, ctr);
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


// perturbed "P strictly inside the circumsphere of finite tetrahedron w"
__device__ __forceinline__ bool finite_inside(const Vert *V, uint4 w, P3 P, unsigned long long pidx,
                                              PredStats &st) {
    const uint32_t ids[4] = {w.x, w.y, w.z, w.w};
    return insphere_perturbed(vpos(V, w.x), vpos(V, w.y), vpos(V, w.z), vpos(V, w.w), P,
                              [&](int k) { return k < 4 ? V[ids[k]].idx : pidx; }, st) < 0;
}

// Sec. 2.6: a ghost (a,b,c,G) contains the open half-space beyond abc and abc's circumdisk
__device__ __forceinline__ bool tet_inside(const RoundArgs &a, uint32_t u, P3 P, unsigned long long pidx,
                                           PredStats &st) {
    uint4 w = a.T[u].v;
    if (w.w != GHOST) return finite_inside(a.V, w, P, pidx, st);
    int o = orient3d(vpos(a.V, w.x), vpos(a.V, w.y), vpos(a.V, w.z), P, st);
    if (o != 0) return o > 0;
    uint32_t x = a.T[u].n.w >> 2;
    return finite_inside(a.V, a.T[x].v, P, pidx, st);
}

// ------------------------------------------------------------------ walk + cavity + claim

// Sizes of the cavity kernel's per-insertion state: a queue of CAPL cavity tetrahedra and a
// set of HM entries holding the attempt's own cavity and outer tetrahedra.  Regular rounds
// keep both in LDS at (128, 256) with 4 to 64 lanes per insertion; rounds for large
// cavities use (1024, 2048) with 64 lanes, and beyond that the same 64-lane search keeps
// both in global memory (the candidate's cavity buffer and its part of the ball scratch).
constexpr uint32_t LCAPC = 128, LHM = 256;
constexpr uint32_t BIG_CAPC = 1024, BIG_HM = 2048;
constexpr uint32_t MEM_EMPTY = 0xFFFFFFFFu;

// open addressing in a power-of-two table of hm entries, (t << 1 | kind) per entry
__device__ __forceinline__ uint32_t mem_hash(uint32_t t, uint32_t hm) {
    return (t * 2654435761u) >> (32 - __builtin_ctz(hm));
}

// kind of tetrahedron t in the set (0 cavity, 1 outer) or -1; a set in global memory is
// read at device scope, past any vector L1 copy, since other lanes fill it by atomics
template <bool GLOBAL>
__device__ __forceinline__ int mem_find(uint32_t *mem, uint32_t hm, uint32_t t) {
    uint32_t h = mem_hash(t, hm);
    for (uint32_t probe = 0; probe < hm; ++probe) {
        const uint32_t e =
            GLOBAL ? __hip_atomic_load(&mem[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : mem[h];
        if (e == MEM_EMPTY) return -1;
        if ((e >> 1) == t) return (int)(e & 1u);
        h = (h + 1) & (hm - 1);
    }
    return -1;
}

// adds t with `kind`: 1 if this call added it (its entry is then mem[*at]), 0 if it was
// there, -1 if the set is full
__device__ __forceinline__ int mem_insert(uint32_t *mem, uint32_t hm, uint32_t t, uint32_t kind, uint32_t *at) {
    uint32_t h = mem_hash(t, hm);
    const uint32_t e = (t << 1) | kind;
    for (uint32_t probe = 0; probe < hm; ++probe) {
        const uint32_t old = atomicCAS(&mem[h], MEM_EMPTY, e);
        if (old == MEM_EMPTY) {
            *at = h;
            return 1;
        }
        if ((old >> 1) == t) return 0;
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
// (4, 8, 16 or 64): the walk tests the four facets of the current tetrahedron on four lanes
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
template <int GS, uint32_t CAPL, uint32_t HM, bool GLOBAL>
__global__ __launch_bounds__(256) void k_cavity_g(RoundArgs a) {
    constexpr uint32_t GPB = 256 / GS;  // insertions per 256-thread block
    constexpr uint32_t NP = GS / 4;     // cavity tetrahedra expanded per step
    // LDS queue entries: (slot of the tetrahedron's entry in the set << 2 | facet it was
    // entered through), 16 bits; the global queue holds (tetrahedron << 2 | facet)
    __shared__ uint16_t s_cav[GPB][GLOBAL ? 1 : CAPL];
    __shared__ uint32_t s_mem[GPB][GLOBAL ? 1 : HM];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t gl = threadIdx.x & (GS - 1);
    const uint32_t gi = threadIdx.x / GS;
    const uint32_t gbase = lane & ~(uint32_t)(GS - 1);
    const unsigned long long gmask = GS == 64 ? ~0ull : (((1ull << (GS & 63)) - 1ull) << gbase);
    const unsigned long long below = gmask & ((1ull << lane) - 1ull);
    const uint32_t i = blockIdx.x * GPB + gi;
    const uint32_t ncand = *a.ncand_ptr;
    const uint32_t stride = a.stride;
    PredStats st;
    unsigned steps = 0, attempt = 0;
    if (i < ncand) {
        uint8_t status = ST_NONE;
        const uint32_t p = a.cand_pt[i];
        const unsigned long long S = a.round_hi | (2ull * a.cand_rank[i]);
        const Vert pv = a.V[p];
        const P3 P = {pv.x, pv.y, pv.z};
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
        const unsigned long long hm = __ballot(ht != NONE) & gmask;
        uint32_t t = hm ? __shfl(ht, __ffsll((long long)hm) - 1) : tq;
        // the learned scheduler predicts the anchor to be the closer start
        if (a.wbucket && tq != NONE && a.wbucket[p - a.vlo]) t = tq;
        if (t == NONE) t = cl->any_live;
        uint4 w = a.T[t].v;
        if (w.x == DEAD) {
            t = cl->any_live;
            w = a.T[t].v;
        }
        if (w.w == GHOST) {
            t = a.T[t].n.w >> 2;
            w = a.T[t].v;
        }
        // Walk: lane j < 4 tests facet j
        int entry = -1;
        bool in_ghost = false;
        const int jl = (int)(gl & 3u);
        for (;;) {
            const P3 q0 = vpos(a.V, w.x), q1 = vpos(a.V, w.y), q2 = vpos(a.V, w.z), q3 = vpos(a.V, w.w);
            const uint4 nn = a.T[t].n;
            int o = 1;
            if (gl < 4 && jl != entry)
                o = orient3d(jl == 0 ? P : q0, jl == 1 ? P : q1, jl == 2 ? P : q2, jl == 3 ? P : q3, st);
            const unsigned bits = (unsigned)((__ballot(o < 0) & gmask) >> gbase) & 0xFu;
            if (!bits) break;
            const unsigned rot = (p + steps) & 3u;
            const unsigned rb = ((bits >> rot) | (bits << (4u - rot))) & 0xFu;
            const int moved = (int)(((unsigned)__ffs(rb) - 1u + rot) & 3u);
            const uint32_t code = comp(nn, moved);
            t = code >> 2;
            entry = (int)(code & 3u);
            w = a.T[t].v;
            if (++steps > WALK_LIMIT) {
                status = ST_ERROR;
                break;
            }
            if (w.w == GHOST) {
                in_ghost = true;
                break;
            }
        }
        if (status == ST_NONE && !in_ghost) {
            // p equal to a vertex of its containing tetrahedron: lane j < 4 compares vertex j
            bool same = false;
            if (gl < 4) {
                const P3 v = vpos(a.V, comp(w, jl));
                same = v.x == P.x && v.y == P.y && v.z == P.z;
            }
            if (__ballot(same) & gmask) status = ST_DUP;
        }
        uint32_t ncav = 0, nbnd = 0;
        const uint32_t capL = GLOBAL ? a.capC : min(a.capC, CAPL), capF = a.capF;
        uint32_t *bnd = a.bnd + (size_t)i * a.capF;
        uint32_t *outc = a.outc + (size_t)i * a.capF;
        uint32_t *cavg = a.cav + (size_t)i * a.capC;
        uint16_t *cavl = s_cav[gi];
        // the set in global memory: hms (a power of two, at most 4 capC) words of the
        // candidate's part of the ball scratch, which the ball kernel uses only later
        const uint32_t hms = GLOBAL ? a.hmg : HM;
        uint32_t *mem = GLOBAL ? reinterpret_cast<uint32_t *>(a.scr_v + (size_t)i * a.capC) : s_mem[gi];
        if (status == ST_NONE) {
            // Cavity.  Step k expands cavity tetrahedra k0 .. k0 + NP - 1, lane (slot, facet)
            // = (gl / 4, gl % 4).
            for (uint32_t h = gl; h < hms; h += GS) mem[h] = MEM_EMPTY;
            lane_fence<GLOBAL>();
            // each step's claims are checked at the next step (or after the last), once that
            // step's loads are in flight, so that the atomics' latency overlaps them; the
            // walk's tetrahedron is inside, its claim is checked with the first step's
            bool pneed = gl == 0, pinside = true;
            unsigned long long po1 = ~0ull;
            if (gl == 0) {
                po1 = atomicMin(&a.T[t].claim, S);
                uint32_t at = 0;
                mem_insert(mem, hms, t, 0u, &at);
                if (GLOBAL) cavg[0] = t << 2;
                else cavl[0] = (uint16_t)(at << 2);
            }
            ncav = 1;
            lane_fence<GLOBAL>();
            for (uint32_t k0 = 0, nproc = 0; k0 < ncav && status == ST_NONE; k0 += nproc) {
                nproc = min(NP, ncav - k0);  // entries expanded in this step
                const uint32_t slot = k0 + (gl >> 2);
                const int f = jl;
                const bool lv = slot < k0 + nproc;
                uint32_t code = 0u;
                if (lv) {
                    if (GLOBAL) {
                        code = cavg[slot];
                    } else {
                        const uint32_t q = cavl[slot];
                        code = ((mem[q >> 2] >> 1) << 2) | (q & 3u);
                    }
                }
                const uint32_t c = code >> 2;
                const int pf = slot == 0 ? -1 : (int)(code & 3u);
                const bool act = lv && f != pf;
                uint4 cv = make_uint4(0u, 0u, 0u, 0u), cn = cv, uw = cv;
                if (lv) {
                    cv = a.T[c].v;
                    cn = a.T[c].n;
                }
                // the previous step's claims: a lower claim on a tetrahedron of this cavity,
                // or a lower cavity claim (even) on one outside it, loses the attempt
                if (__ballot(pneed && po1 < S && (pinside || !(po1 & 1ull))) & gmask) {
                    status = ST_CONFLICT;
                    break;
                }
                const uint32_t ncode = comp(cn, f);
                const uint32_t u = ncode >> 2;
                const int kind = act ? mem_find<GLOBAL>(mem, hms, u) : -1;  // 0: in this cavity, 1: outside it
                const bool need = act && kind < 0;
                if (need) uw = a.T[u].v;
                bool inside = false;
                if (need) {
                    const bool cghost = cv.w == GHOST;
                    const uint32_t apex = comp(uw, (int)(ncode & 3u));
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
                        inside = insphere_perturbed(vpos(a.V, r2[0]), vpos(a.V, r2[1]), vpos(a.V, r2[2]),
                                                    vpos(a.V, r2[3]), P,
                                                    [&](int kk) { return kk < 4 ? a.V[r2[kk]].idx : pv.idx; },
                                                    st) < 0;
                    } else if (!cghost) {
                        // u is the ghost beyond facet f of the finite cavity tetrahedron c:
                        // inside iff p is beyond the facet, or on it (then c decides: inside)
                        const P3 c0 = vpos(a.V, cv.x), c1 = vpos(a.V, cv.y), c2 = vpos(a.V, cv.z),
                                 c3 = vpos(a.V, cv.w);
                        inside = orient3d(f == 0 ? P : c0, f == 1 ? P : c1, f == 2 ? P : c2, f == 3 ? P : c3, st) <= 0;
                    } else {
                        inside = tet_inside(a, u, P, pv.idx, st);
                    }
                }
                // the one claim of u: S if inside, S + 1 if outside (a tetrahedron reached
                // through several facets in this step gets the same claim from each lane)
                unsigned long long o1 = ~0ull;
                if (need) o1 = atomicMin(&a.T[u].claim, inside ? S : S + 1);
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
                    else cavl[pos] = (uint16_t)((at << 2) | (ncode & 3u));
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
                cavg[k] = ((mem[q >> 2] >> 1) << 2) | (q & 3u);
            }
        if (gl == 0) {
            a.status[i] = status;
            a.cnt[i] = ncav;
            a.cnt[stride + i] = nbnd;
            attempt = 1;
        } else {
            steps = 0;
        }
    }
    add_stat(a.stat, STAT_ATTEMPTS, attempt);
    add_stat(a.stat, STAT_WALK, steps);
    add_stat(a.stat, STAT_ORIENT, st.orient);
    add_stat(a.stat, STAT_ORIENT_EXACT, st.orient_exact);
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
constexpr uint32_t LOC_BOUNDARY = 0x80000000u;
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

template <int GL, int BS>
__global__ __launch_bounds__(BS) void k_ball(RoundArgs a) {
    constexpr uint32_t GPB = BS / GL;
    __shared__ unsigned long long s_key[GPB][HT];
    __shared__ uint32_t s_val[GPB][HT][2];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t gl = threadIdx.x % GL;
    const uint32_t gi = threadIdx.x / GL;
    const uint32_t gbase = lane & ~(uint32_t)(GL - 1);
    const unsigned long long gmask = GL == 64 ? ~0ull : (((1ull << (GL & 63)) - 1ull) << gbase);
    const uint32_t i = blockIdx.x * GPB + gi;
    const uint32_t ncand = *a.ncand_ptr;
    const uint32_t stride = a.stride, capC = a.capC, capF = a.capF;
    unsigned cav_w = 0, bnd_w = 0;
    const bool cand = i < ncand && a.status[i] == ST_CAND;
    uint32_t p = 0, nc = 0, nb = 0;
    unsigned long long S = 0;
    const uint32_t *cavl = a.cav + (size_t)i * capC;
    const uint32_t *bl = a.bnd + (size_t)i * capF;
    uint32_t *ol = a.outc + (size_t)i * capF;
    uint4 *sv = a.scr_v + (size_t)i * capC;
    uint4 *sn = a.scr_n + (size_t)i * capC;
    bool ok = true;
    if (cand) {
        p = a.cand_pt[i];
        S = a.round_hi | (2ull * a.cand_rank[i]);
        nc = a.cnt[i];
        nb = a.cnt[stride + i];
        // winner test
        // cavity tetrahedra: no lower claim; outer tetrahedra: the lowest claim is an outer
        // one (any lower attempt with it in its cavity then loses on that claim)
        for (uint32_t k = gl; k < nc; k += GL) ok &= a.T[cavl[k] >> 2].claim == S;
        for (uint32_t k = gl; k < nb; k += GL) ok &= (a.T[ol[k] >> 2].claim & 1ull) != 0;
    }
    const bool win = cand && (__ballot(!ok) & gmask) == 0;
    // slot reservation by each winner's first lane, one atomic per block: the F - C extra
    // slots are units of fl_take (units below fl_n are free-list entries of earlier rounds,
    // the rest are fresh pool slots from tet_count on); C - F surplus cavity slots are freed
    const bool leader = win && gl == 0;
    const uint32_t need = leader && nb > nc ? nb - nc : 0u;
    const uint32_t u0 = block_reserve<BS / 64>(need, &a.ctr->fl_take, &s_val[0][0][0]);
    const uint32_t fln = a.ctr->fl_n, tc0 = a.ctr->tet_count;
    const bool full = need && u0 + need > fln && tc0 + (u0 + need - fln) > a.tcap;
    if (full) {
        // pool full: give the units back (pool slots inside the pool are marked free) and
        // retry next round after the host has grown the pool
        uint32_t give = 0;
        for (uint32_t k = 0; k < need; ++k) {
            const uint32_t u = u0 + k;
            if (u < fln || tc0 + (u - fln) < a.tcap) ++give;
        }
        const uint32_t g0 = atomicAdd(&a.ctr->fl_next, give);
        uint32_t q = 0;
        for (uint32_t k = 0; k < need; ++k) {
            const uint32_t u = u0 + k;
            if (u < fln) {
                a.fl_next[g0 + q++] = a.fl_cur[u];
            } else if (tc0 + (u - fln) < a.tcap) {
                a.T[tc0 + (u - fln)].v.x = DEAD;
                a.fl_next[g0 + q++] = tc0 + (u - fln);
            }
        }
        atomicOr(&a.ctr->error, ERR_POOL);
    }
    const bool lbuilt = leader && !full;
    const uint32_t fb = lbuilt && nc > nb ? atomicAdd(&a.ctr->fl_next, nc - nb) : 0u;  // rare
    if (cand && gl == 0) a.status[i] = lbuilt ? ST_WON : ST_CONFLICT;
    const bool built = __shfl((int)lbuilt, (int)gbase) != 0;
    const uint32_t g_u0 = __shfl(u0, (int)gbase), g_fb = __shfl(fb, (int)gbase);
    if (built) {
        const bool table = nb <= HT_MAX_FACETS;
        // A: copies of the cavity tetrahedra (vertices; for the pivot also the neighbours and
        // the local index in the spare word); the edge table is cleared
        for (uint32_t k = gl; k < nc; k += GL) {
            const uint32_t c = cavl[k] >> 2;
            sv[k] = a.T[c].v;
            if (!table) {
                sn[k] = a.T[c].n;
                a.T[c].spare[0] = k;
            }
        }
        if (table)
            for (uint32_t h = gl; h < HT; h += GL) s_key[gi][h] = HT_EMPTY;
        group_fence();
        if (!table) {
            // B (pivot only): facets between two cavity tetrahedra -> local codes
            for (uint32_t task = gl; task < 4 * nc; task += GL) {
                const uint32_t k = task >> 2;
                const int f = (int)(task & 3u);
                const uint32_t code = comp(sn[k], f);
                const uint32_t nt = code >> 2;
                if (a.T[nt].claim == S)  // only this winner's cavity tetrahedra hold S
                    reinterpret_cast<uint32_t *>(&sn[k])[f] = ((uint32_t)a.T[nt].spare[0] << 2) | (code & 3u);
            }
            group_fence();
        }
        // C: one new tetrahedron per boundary facet (k, f): k with v_f replaced by p
        for (uint32_t b = gl; b < nb; b += GL) {
            uint32_t slot;
            if (b < nc) {
                slot = cavl[b] >> 2;
            } else {
                const uint32_t u = g_u0 + (b - nc);
                slot = u < fln ? a.fl_cur[u] : tc0 + (u - fln);
            }
            const uint32_t bc = bl[b];  // local index of the cavity tetrahedron << 2 | facet
            const uint32_t kb = bc >> 2;
            const int f = (int)(bc & 3u);
            const uint32_t oc = ol[b];
            const uint4 cw = sv[kb];
            uint32_t wv[4] = {cw.x, cw.y, cw.z, cw.w};
            wv[f] = p;
            a.T[slot].v = make_uint4(wv[0], wv[1], wv[2], wv[3]);
            const uint32_t me = (slot << 2) | (uint32_t)f;
            nref(a.T, slot, f) = oc;           // facet opposite p: the outer tetrahedron
            nref(a.T, oc >> 2, oc & 3u) = me;  // and back
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
                            s_val[gi][h][old == HT_EMPTY ? 0 : 1] = (slot << 2) | (uint32_t)q;
                            placed = true;
                        }
                        h = (h + 1) & (HT - 1);
                    }
                    if (!placed) atomicOr(&a.ctr->error, ERR_WALK);
                }
            } else {
                reinterpret_cast<uint32_t *>(&sn[kb])[f] = LOC_BOUNDARY | b;
            }
        }
        group_fence();
        // D: the three siblings of each new tetrahedron
        if (table) {
            for (uint32_t b = gl; b < nb; b += GL) {
                const uint32_t me = ol[b];
                const uint32_t slot = me >> 2;
                const int f = (int)(me & 3u);
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
                    const uint32_t mine = (slot << 2) | (uint32_t)q;
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
                    nref(a.T, slot, q) = res;
                }
            }
        } else {
            for (uint32_t task = gl; task < 3 * nb; task += GL) {
                const uint32_t b = task / 3, qi = task - 3 * b;
                const uint32_t me = ol[b];
                const uint32_t slot = me >> 2;
                const int pf = (int)(me & 3u);
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
                uint32_t res = 0;
                bool found = false;
                for (uint32_t guard = 0; guard <= nc + 1; ++guard) {
                    const uint4 cv = sv[k];
                    const uint32_t v4[4] = {cv.x, cv.y, cv.z, cv.w};
                    int xpos = -1;
                    for (int m = 0; m < 4; ++m)
                        if (m != f && v4[m] != e[0] && v4[m] != e[1]) xpos = m;
                    if (xpos < 0) break;
                    const uint32_t lc = comp(sn[k], xpos);
                    if (lc & LOC_BOUNDARY) {
                        // boundary facet (k, xpos): its new tetrahedron has p at xpos, and
                        // the facet through p, e0, e1 is opposite its vertex f
                        res = (ol[lc & ~LOC_BOUNDARY] & ~3u) | (uint32_t)f;
                        found = true;
                        break;
                    }
                    k = lc >> 2;
                    f = (int)(lc & 3u);
                    if (k >= nc) break;
                }
                if (!found) atomicOr(&a.ctr->error, ERR_WALK);
                nref(a.T, slot, q) = res;
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
                const uint32_t c = cavl[k] >> 2;
                a.T[c].v.x = DEAD;
                a.fl_next[g_fb + (k - nb)] = c;
                if (c == live) cl->any_live = cavl[0] >> 2;
            }
        }
        if (gl == 0) {
            cav_w = nc;
            bnd_w = nb;
        }
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
    const bool again = i < ncand && (s == ST_CONFLICT || s == ST_CAND);
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
    const bool bad = i < ncand && !(again || ovf || s == ST_WON || s == ST_DUP);
    if (bad) atomicOr(&a.ctr->error, ERR_WALK);
}

// carry the unused part of this round's free list behind the slots freed this round
__global__ void k_freelist_carry(RoundArgs a) {
    const uint32_t fln = a.ctr->fl_n, take = a.ctr->fl_take, nxt = a.ctr->fl_next;
    if (take >= fln) return;
    const uint32_t left = fln - take;
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < left; k += gridDim.x * blockDim.x)
        a.fl_next[nxt + k] = a.fl_cur[take + k];
}

__global__ void k_roll(Ctr *ctr, uint32_t *consumed, uint32_t tcap, const unsigned long long *stat) {
    const uint32_t t = threadIdx.x;
    if (t < NSTAT) {
        unsigned long long sum = 0;
        for (int k = 0; k < STAT_SPREAD; ++k) sum += stat[((size_t)t * STAT_SPREAD + k) * STAT_PAD];
        unsigned long long *dst[NSTAT] = {&ctr->attempts, &ctr->walk_steps, &ctr->orient, &ctr->orient_exact,
                                         &ctr->insphere, &ctr->insphere_exact, &ctr->perturbed,
                                         &ctr->cav_tets, &ctr->bnd_facets};
        *dst[t] = sum;
    }
    if (t != 0) return;
    const uint32_t fln = ctr->fl_n, take = ctr->fl_take;
    if (take > fln) {
        // units beyond the free list were fresh pool slots (beyond the pool: never used)
        const unsigned long long tc = (unsigned long long)ctr->tet_count + (take - fln);
        ctr->tet_count = tc > tcap ? tcap : (uint32_t)tc;
    }
    const uint32_t left = take < fln ? fln - take : 0u;
    ctr->fl_n = ctr->fl_next + left;
    ctr->fl_take = 0;
    ctr->fl_next = 0;
    *consumed = 0;  // the list this round read from is empty now
}

hipError_t launch_round(const RoundArgs &a, uint32_t max_cand, uint32_t lanes, hipStream_t s, hipEvent_t *ev) {
    if (max_cand == 0) return hipSuccess;
    const unsigned nb = (max_cand + 255) / 256;
    if (ev) hipEventRecord(ev[0], s);
    if (a.capC > BIG_CAPC) {
        // the set takes hmg words of the candidate's 4 capC words of ball scratch
        if (a.hmg < 4096 || (a.hmg & (a.hmg - 1)) || a.hmg > 4ull * a.capC) return hipErrorInvalidValue;
        k_cavity_g<64, 1, 1, true><<<(max_cand + 3) / 4, 256, 0, s>>>(a);
    } else if (a.capC > LCAPC) {
        k_cavity_g<64, BIG_CAPC, BIG_HM, false><<<(max_cand + 3) / 4, 256, 0, s>>>(a);
    } else if (lanes == 4) {
        k_cavity_g<4, LCAPC, LHM, false><<<(max_cand + 63) / 64, 256, 0, s>>>(a);
    } else if (lanes == 8) {
        k_cavity_g<8, LCAPC, LHM, false><<<(max_cand + 31) / 32, 256, 0, s>>>(a);
    } else if (lanes == 64) {
        k_cavity_g<64, LCAPC, LHM, false><<<(max_cand + 3) / 4, 256, 0, s>>>(a);
    } else {
        k_cavity_g<16, LCAPC, LHM, false><<<(max_cand + 15) / 16, 256, 0, s>>>(a);
    }
    if (ev) hipEventRecord(ev[1], s);
    k_ball<16, BALL_BLOCK><<<(max_cand + BALL_BLOCK / 16 - 1) / (BALL_BLOCK / 16), BALL_BLOCK, 0, s>>>(a);
    if (ev) hipEventRecord(ev[2], s);
    return hipGetLastError();
}

hipError_t launch_round_end(const RoundArgs &a, uint32_t max_cand, hipStream_t s) {
    if (max_cand) k_compact<<<(max_cand + FILL_BLOCK - 1) / FILL_BLOCK, FILL_BLOCK, 0, s>>>(a);
    k_freelist_carry<<<256, 256, 0, s>>>(a);
    k_roll<<<1, 64, 0, s>>>(a.ctr, const_cast<uint32_t *>(a.ncand_ptr), a.tcap, a.stat);
    return hipGetLastError();
}

// Claim words back to the empty value (above every stamp), for the round after the round
// counter's low 32 bits wrap.  A fill kernel rather than a strided memset.
__global__ void k_reset_claims(Tet *__restrict__ T, uint32_t tcap) {
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < tcap; t += gridDim.x * blockDim.x)
        T[t].claim = ~0ull;
}

hipError_t launch_reset_claims(Tet *T, uint32_t tcap, hipStream_t s) {
    if (tcap == 0) return hipSuccess;
    k_reset_claims<<<2048, 256, 0, s>>>(T, tcap);
    return hipGetLastError();
}

// ------------------------------------------------------------------ output

__global__ void k_out_flags(const Tet *__restrict__ T, uint32_t count, uint32_t *__restrict__ flags) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const uint4 w = T[t].v;
    flags[t] = (w.x != DEAD && w.w != GHOST) ? 1u : 0u;
}

// Per-cloud output.  The live finite tetrahedra are sorted by the cloud of their vertices
// (keys: cloud, or nclouds for ghosts and free slots); cloud c owns sorted positions
// [toff[c], toff[c + 1]); map[t] is the sorted position of tetrahedron t.
__global__ void k_tet_cloud(const Tet *__restrict__ T, const Vert *__restrict__ V, uint32_t count, uint32_t nclouds,
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

__global__ void k_output_cloud(const Tet *__restrict__ T, const Vert *__restrict__ V, const uint32_t *__restrict__ sorted,
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
        const uint4 nn = T[t].n;
        const uint32_t nv[4] = {nn.x, nn.y, nn.z, nn.w};
        for (int k = 0; k < 4; ++k) {
            const uint32_t nt = nv[k] >> 2;
            nbrs[4 * (size_t)j + k] = T[nt].v.w == GHOST ? -1 : (int64_t)map[nt] - (int64_t)tb;
        }
    }
}

hipError_t launch_tet_cloud(const Tet *T, const Vert *V, uint32_t count, uint32_t nclouds, unsigned long long *keys,
                            uint32_t *vals, hipStream_t s) {
    if (count == 0) return hipSuccess;
    k_tet_cloud<<<(count + 255) / 256, 256, 0, s>>>(T, V, count, nclouds, keys, vals);
    return hipGetLastError();
}

hipError_t launch_seg_bounds(const unsigned long long *keys, uint32_t count, uint32_t nclouds, uint32_t *toff,
                             hipStream_t s) {
    if (count == 0) return hipSuccess;
    k_seg_bounds<<<(count + 255) / 256, 256, 0, s>>>(keys, count, nclouds, toff);
    return hipGetLastError();
}

hipError_t launch_tet_map(const uint32_t *sorted, uint32_t nlive, uint32_t *map, hipStream_t s) {
    if (nlive == 0) return hipSuccess;
    k_tet_map<<<(nlive + 255) / 256, 256, 0, s>>>(sorted, nlive, map);
    return hipGetLastError();
}

hipError_t launch_output_cloud(const Tet *T, const Vert *V, const uint32_t *sorted, const uint32_t *map, uint32_t tb,
                               uint32_t te, uint64_t vbase, uint32_t *tets, int64_t *nbrs, hipStream_t s) {
    if (te <= tb) return hipSuccess;
    k_output_cloud<<<(te - tb + 255) / 256, 256, 0, s>>>(T, V, sorted, map, tb, te, vbase, tets, nbrs);
    return hipGetLastError();
}

hipError_t launch_output_flags(const Tet *T, uint32_t count, uint32_t *flags, hipStream_t s) {
    if (count == 0) return hipSuccess;
    k_out_flags<<<(count + 255) / 256, 256, 0, s>>>(T, count, flags);
    return hipGetLastError();
}

// Output position of each slot: map[t] (the exclusive scan of the live flags) for live finite
// tetrahedra, NONE for ghosts and free slots; and the input index of each vertex record as a
// compact 4-byte array.  The export kernel then gathers from these two small arrays (which
// stay in the last-level caches far better than 64-byte tetrahedron rows and 32-byte vertex
// records) instead of from the tetrahedron and vertex pools.
__global__ void k_out_map(const uint32_t *__restrict__ flags, uint32_t count, uint32_t *__restrict__ map,
                          const Vert *__restrict__ V, uint32_t nv, uint32_t *__restrict__ vid) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count && !flags[t]) map[t] = NONE;
    if (t < nv) vid[t] = (uint32_t)V[t].idx;
}

__global__ void k_output(const Tet *__restrict__ T, const uint32_t *__restrict__ vid,
                         const uint32_t *__restrict__ map, uint32_t count, uint32_t *__restrict__ tets,
                         int64_t *__restrict__ nbrs) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const uint32_t o = map[t];
    if (o == NONE) return;
    if (tets) {
        const uint4 w = T[t].v;
        const uint4 out = make_uint4(vid[w.x], vid[w.y], vid[w.z], vid[w.w]);
        *reinterpret_cast<uint4 *>(tets + 4 * (size_t)o) = out;
    }
    if (nbrs) {
        const uint4 nn = T[t].n;
        const uint32_t m[4] = {map[nn.x >> 2], map[nn.y >> 2], map[nn.z >> 2], map[nn.w >> 2]};
        longlong2 *dst = reinterpret_cast<longlong2 *>(nbrs + 4 * (size_t)o);
        dst[0] = make_longlong2(m[0] == NONE ? -1ll : (long long)m[0], m[1] == NONE ? -1ll : (long long)m[1]);
        dst[1] = make_longlong2(m[2] == NONE ? -1ll : (long long)m[2], m[3] == NONE ? -1ll : (long long)m[3]);
    }
}

hipError_t launch_output(const Tet *T, const Vert *V, uint32_t nv, const uint32_t *flags, uint32_t *map,
                         uint32_t *vid, uint32_t count, uint32_t *tets, int64_t *nbrs, hipStream_t s) {
    if (count == 0) return hipSuccess;
    const uint32_t m = count > nv ? count : nv;
    k_out_map<<<(m + 255) / 256, 256, 0, s>>>(flags, count, map, V, nv, vid);
    k_output<<<(count + 255) / 256, 256, 0, s>>>(T, vid, map, count, tets, nbrs);
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
