// Concurrent Bowyer-Watson insertion rounds (paper Sec. 2.1 Algorithm 1, Sec. 2.5, Sec. 2.6;
// concurrency rules of Sec. 3.2).
//
// One thread per candidate point.  A round is three kernels:
//   k_cavity : Walk (visibility walk, Sec. 2.1) from a live tetrahedron of an already
//              inserted neighbour on the space-filling curve, then Cavity (breadth-first search by perturbed insphere,
//              ghosts by the half-space + circumdisk rule of Sec. 2.6).  Every tetrahedron
//              the search touches is claimed with atomicMin on 64-bit claim words:
//              stamp S = (round part, 2 rank) for cavity tetrahedra, S + 1 for tetrahedra
//              found outside.  Meeting a lower stamp ends the attempt at once.
//   k_ball   : an attempt wins iff every tetrahedron it touched still holds its stamp, so
//              the cavities of winners are disjoint from each other and from each other's
//              adjacent tetrahedra (rules 1a-1c and 2 of Sec. 3.2); the lowest rank in a
//              round always wins, so every round makes progress.  A winner builds
//              DelaunayBall (Sec. 2.5): one tetrahedron per boundary facet, glued a priori to
//              the outer tetrahedron, and glued to its three sibling tetrahedra by pivoting
//              around each boundary edge through the (still intact) cavity tetrahedra.  Freed
//              slots are reused in later rounds (Sec. 2.5 end, Sec. 3.6).
//   k_compact: losers are queued for the next round with their rank; overflowing
//              cavities are queued for a round with larger per-insertion buffers.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dt_internal.h"
#include "dt_predicates.h"

namespace dtk {

constexpr uint32_t WALK_LIMIT = 1u << 20;
constexpr int HINT_RANGE = 4;

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

__device__ __forceinline__ void add_stat(unsigned long long *dst, unsigned v) {
    unsigned s = wave_sum(v);
    if ((threadIdx.x & 63) == 0 && s) atomicAdd(dst, (unsigned long long)s);
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

__global__ void k_init(const Vert *__restrict__ V, uint32_t base, uint32_t n, const uint8_t *__restrict__ dup,
                       Tet *__restrict__ T, uint32_t *__restrict__ vtet,
                       Ctr *__restrict__ ctr) {
    __shared__ uint32_t sel[4];
    __shared__ uint32_t best;
    PredStats st;
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
            if (threadIdx.x == 0) atomicOr(&ctr->error, ERR_DEGENERATE);
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
    uint32_t TV[5][4], N[5][4];
    for (int k = 0; k < 4; ++k) TV[0][k] = v[k];
    for (int j = 0; j < 4; ++j) {
        uint32_t w[4] = {v[0], v[1], v[2], v[3]};
        w[j] = GHOST;
        orient_new_tet(w, j);  // G ends in slot 3: finite facet (w0,w1,w2) faces outward
        for (int k = 0; k < 4; ++k) TV[1 + j][k] = w[k];
        N[0][j] = ((1u + j) << 2) | 3u;
        N[1 + j][3] = (0u << 2) | (uint32_t)j;
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
                    if (same == 3) N[g1][f1] = ((uint32_t)g2 << 2) | (uint32_t)f2;
                }
            }
    for (int t = 0; t < 5; ++t) {
        Tet r;
        r.v = make_uint4(TV[t][0], TV[t][1], TV[t][2], TV[t][3]);
        r.n = make_uint4(N[t][0], N[t][1], N[t][2], N[t][3]);
        r.any = r.cav = ~0ull;
        r.spare[0] = r.spare[1] = 0;
        T[t] = r;
    }
    for (int k = 0; k < 4; ++k) {
        vtet[v[k]] = 0;
        ctr->init[k] = v[k];
    }
    ctr->tet_count = 5;
    ctr->any_live = 0;
}

hipError_t launch_init(const Vert *V, uint32_t base, uint32_t n, const uint8_t *dup, Tet *T, uint32_t *vtet,
                       Ctr *ctr, hipStream_t s) {
    k_init<<<1, 256, 0, s>>>(V, base, n, dup, T, vtet, ctr);
    return hipGetLastError();
}

// ------------------------------------------------------------------ candidate fill

// Ranks: level k owns ranks [rank_base[k], rank_base[k] + 2^bits[k]); rank r maps to the
// level position bitreverse(r - rank_base[k]) (lord lists each level's records in Moore
// order), so any window of consecutive ranks is spread evenly along the level's points.
__global__ void k_fill(const uint32_t *__restrict__ lvl_start, const uint32_t *__restrict__ lvl_size,
                       const uint32_t *__restrict__ lvl_bits, const unsigned long long *__restrict__ rank_base, int L,
                       const uint32_t *__restrict__ lord, unsigned long long first_rank, uint32_t count,
                       const uint8_t *__restrict__ dup,
                       const uint32_t *__restrict__ vtet, uint32_t *__restrict__ cand_pt,
                       uint32_t *__restrict__ cand_rank, uint32_t *__restrict__ ncand) {
    uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    unsigned long long r = first_rank + t;
    int k = 0;
    while (k + 1 < L && rank_base[k + 1] <= r) ++k;
    uint32_t local = (uint32_t)(r - rank_base[k]);
    uint32_t bits = lvl_bits[k];
    uint32_t q = bits ? (__brev(local) >> (32 - bits)) : 0u;
    if (q >= lvl_size[k]) return;
    uint32_t p = lord[lvl_start[k] + q];
    if (dup[p] || vtet[p] != NONE) return;
    uint32_t pos = atomicAdd(ncand, 1u);
    cand_pt[pos] = p;
    cand_rank[pos] = (uint32_t)r;
}

hipError_t launch_fill_list(const uint32_t *lvl_start, const uint32_t *lvl_size, const uint32_t *lvl_bits,
                            const unsigned long long *rank_base, int L, const uint32_t *lord,
                            unsigned long long first_rank, uint32_t count, const uint8_t *dup,
                            const uint32_t *vtet, uint32_t *cand_pt, uint32_t *cand_rank, uint32_t *ncand,
                            hipStream_t s) {
    if (count == 0) return hipSuccess;
    k_fill<<<(count + 255) / 256, 256, 0, s>>>(lvl_start, lvl_size, lvl_bits, rank_base, L, lord, first_rank,
                                               count, dup, vtet, cand_pt, cand_rank, ncand);
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

__global__ __launch_bounds__(256) void k_cavity(RoundArgs a) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t ncand = *a.ncand_ptr;
    const uint32_t stride = a.stride;
    PredStats st;
    unsigned steps = 0, attempt = 0;
    if (i < ncand) {
        attempt = 1;
        uint8_t status = ST_NONE;
        const uint32_t p = a.cand_pt[i];
        const unsigned long long S = a.round_hi | (2ull * a.cand_rank[i]);
        const Vert pv = a.V[p];
        const P3 P = {pv.x, pv.y, pv.z};
        // start: a live tetrahedron near the nearest inserted point among the HINT_RANGE
        // records on either side on the curve, else near the point's anchor (a record of
        // a lower level), else any live tetrahedron
        uint32_t t = NONE;
        for (int d = 1; d <= HINT_RANGE && t == NONE; ++d) {
            if (p >= a.vlo + d) t = a.vtet[p - d];
            if (t == NONE && p + d < a.vhi) t = a.vtet[p + d];
        }
        if (t == NONE) {
            const uint32_t q = a.anchor[p - a.vlo];
            if (q != NONE) t = a.vtet[q];
        }
        if (t == NONE) t = a.ctr->any_live;
        uint4 w = a.T[t].v;
        if (w.x == DEAD) {
            t = a.ctr->any_live;
            w = a.T[t].v;
        }
        if (w.w == GHOST) {
            t = a.T[t].n.w >> 2;
            w = a.T[t].v;
        }
        // Walk.  The current tetrahedron's vertex ids and positions are kept; after crossing
        // a facet only the apex of the next tetrahedron is fetched.
        int entry = -1;
        bool in_ghost = false;
        uint32_t id[4] = {w.x, w.y, w.z, w.w};
        P3 q[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) q[k] = vpos(a.V, id[k]);
        for (;;) {
            const uint4 nn = a.T[t].n;
            int moved = -1;
            const int rot = (int)((p + steps) & 3u);
            for (int jj = 0; jj < 4; ++jj) {
                const int j = (jj + rot) & 3;
                if (j == entry) continue;
                int o;
                if (j == 0) o = orient3d(P, q[1], q[2], q[3], st);
                else if (j == 1) o = orient3d(q[0], P, q[2], q[3], st);
                else if (j == 2) o = orient3d(q[0], q[1], P, q[3], st);
                else o = orient3d(q[0], q[1], q[2], P, st);
                if (o < 0) {
                    moved = j;
                    break;
                }
            }
            if (moved < 0) break;
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
            const uint32_t id2[4] = {w.x, w.y, w.z, w.w};
            P3 q2[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                q2[k] = q[0];
#pragma unroll
                for (int m = 1; m < 4; ++m)
                    if (id[m] == id2[k]) q2[k] = q[m];
            }
            // the apex (opposite the entry facet) is the one new vertex
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (k == entry) q2[k] = vpos(a.V, id2[k]);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                id[k] = id2[k];
                q[k] = q2[k];
            }
        }
        if (status == ST_NONE && !in_ghost) {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (q[k].x == P.x && q[k].y == P.y && q[k].z == P.z) status = ST_DUP;
        }
        uint32_t ncav = 0, nbnd = 0;
        if (status == ST_NONE) {
            // Cavity: breadth-first search; cav entries hold (tetrahedron << 2 | facet it was
            // entered through), which is skipped when the tetrahedron is expanded.
            // Claims: T[t].any = min stamp of every attempt touching t, S for this cavity's
            // tetrahedra and S + 1 for those found outside (so the parity tells the kind);
            // T[t].cav = min stamp of the attempts with t in their cavity.  All neighbours of
            // a cavity tetrahedron are claimed tentatively (S + 1) and fetched together; a
            // neighbour of a finite cavity tetrahedron c shares the facet's three vertices
            // with c, so only its apex vertex is fetched.
            {
                const unsigned long long o0 = atomicMin(&a.T[t].any, S);
                if (o0 < S) {
                    status = ST_CONFLICT;
                } else {
                    atomicMin(&a.T[t].cav, S);
                    a.cav[(size_t)i * a.capC] = t << 2;
                    ncav = 1;
                }
            }
            for (uint32_t k = 0; k < ncav && status == ST_NONE; ++k) {
                const uint32_t code = a.cav[(size_t)i * a.capC + k];
                const uint32_t c = code >> 2;
                const int pf = k == 0 ? -1 : (int)(code & 3u);
                const uint4 cv = a.T[c].v;
                const uint4 cn = a.T[c].n;
                const bool cghost = cv.w == GHOST;
                unsigned long long o1[4];
                uint4 uw[4];
#pragma unroll
                for (int f = 0; f < 4; ++f) {
                    o1[f] = S;
                    if (f == pf) continue;
                    const uint32_t u = comp(cn, f) >> 2;
                    o1[f] = atomicMin(&a.T[u].any, S + 1);
                    uw[f] = a.T[u].v;
                }
                P3 cw[4];
                if (!cghost) {
#pragma unroll
                    for (int m = 0; m < 4; ++m) cw[m] = vpos(a.V, comp(cv, m));
                }
#pragma unroll
                for (int f = 0; f < 4; ++f) {
                    if (status != ST_NONE) break;
                    const unsigned long long o = o1[f];
                    if (o == S) continue;  // already in this cavity, or the parent: internal facet
                    if (o < S && !(o & 1ull)) {
                        // a lower attempt has this neighbour in its cavity: this one loses
                        status = ST_CONFLICT;
                        break;
                    }
                    const uint32_t ncode = comp(cn, f);
                    const uint32_t u = ncode >> 2;
                    bool inside = false;
                    if (o != S + 1) {
                        const uint32_t apex = comp(uw[f], (int)(ncode & 3u));
                        if (!cghost && apex != GHOST) {
                            // u = facet f of c + apex; c with vertex f replaced by the apex and
                            // two entries swapped is positively oriented
                            P3 r[4] = {cw[0], cw[1], cw[2], cw[3]};
                            uint32_t rid[4] = {cv.x, cv.y, cv.z, cv.w};
                            r[f] = vpos(a.V, apex);
                            rid[f] = apex;
                            const P3 tmp = r[(f + 1) & 3];
                            r[(f + 1) & 3] = r[(f + 2) & 3];
                            r[(f + 2) & 3] = tmp;
                            const uint32_t tid = rid[(f + 1) & 3];
                            rid[(f + 1) & 3] = rid[(f + 2) & 3];
                            rid[(f + 2) & 3] = tid;
                            inside = insphere_perturbed(r[0], r[1], r[2], r[3], P,
                                                        [&](int kk) { return kk < 4 ? a.V[rid[kk]].idx : pv.idx; },
                                                        st) < 0;
                        } else if (!cghost) {
                            // u is the ghost beyond facet f of the finite cavity tetrahedron c:
                            // inside iff p is beyond the facet, or on it (then c decides: inside)
                            P3 r[4] = {cw[0], cw[1], cw[2], cw[3]};
                            r[f] = P;
                            inside = orient3d(r[0], r[1], r[2], r[3], st) <= 0;
                        } else {
                            inside = tet_inside(a, u, P, pv.idx, st);
                        }
                        if (inside && o < S) {
                            // a lower attempt touched a tetrahedron of this cavity
                            status = ST_CONFLICT;
                            break;
                        }
                    }
                    if (inside) {
                        atomicMin(&a.T[u].any, S);
                        atomicMin(&a.T[u].cav, S);
                        if (ncav == a.capC) {
                            status = ST_OVERFLOW;
                            break;
                        }
                        a.cav[(size_t)i * a.capC + ncav] = ncode;
                        ++ncav;
                    } else {
                        if (nbnd == a.capF) {
                            status = ST_OVERFLOW;
                            break;
                        }
                        a.bnd[(size_t)i * a.capF + nbnd] = (c << 2) | (uint32_t)f;
                        a.outc[(size_t)i * a.capF + nbnd] = ncode;
                        ++nbnd;
                    }
                }
            }
            if (status == ST_NONE) status = ST_CAND;
        }
        a.status[i] = status;
        a.cnt[i] = ncav;
        a.cnt[stride + i] = nbnd;
    }
    add_stat(&a.ctr->attempts, attempt);
    add_stat(&a.ctr->walk_steps, steps);
    add_stat(&a.ctr->orient, st.orient);
    add_stat(&a.ctr->orient_exact, st.orient_exact);
    add_stat(&a.ctr->insphere, st.insphere);
    add_stat(&a.ctr->insphere_exact, st.insphere_exact);
    add_stat(&a.ctr->perturbed, st.perturbed);
}

// ------------------------------------------------------------------ check + DelaunayBall

// Winner test and slot reservation, one thread per candidate.  An attempt wins iff it still
// holds the lowest claim on every tetrahedron of its cavity (any) and no lower attempt
// has one of its outer tetrahedra in its cavity (cav).  Winners of one round therefore
// have disjoint cavities, and no cavity meets another winner's outer tetrahedra.
__global__ __launch_bounds__(256) void k_check(RoundArgs a) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t ncand = *a.ncand_ptr;
    const uint32_t stride = a.stride;
    if (i >= ncand || a.status[i] != ST_CAND) return;
    const unsigned long long S = a.round_hi | (2ull * a.cand_rank[i]);
    const uint32_t nc = a.cnt[i], nb = a.cnt[stride + i];
    bool win = true;
    for (uint32_t k = 0; k < nc; ++k) win &= a.T[a.cav[(size_t)i * a.capC + k] >> 2].any == S;
    for (uint32_t k = 0; k < nb; ++k) win &= a.T[a.outc[(size_t)i * a.capF + k] >> 2].cav > S;
    if (!win) {
        a.status[i] = ST_CONFLICT;
        return;
    }
    // the ball reuses the cavity's slots; F - C more come from the free list of earlier
    // rounds, then from the bump pointer; C - F surplus cavity slots are freed
    const uint32_t need = nb > nc ? nb - nc : 0u;
    const uint32_t take = need ? atomicAdd(&a.ctr->fl_take, need) : 0u;
    const uint32_t fln = a.ctr->fl_n;
    const uint32_t from_fl = fln > take ? min(need, fln - take) : 0u;
    const uint32_t rest = need - from_fl;
    const uint32_t bump = rest ? atomicAdd(&a.ctr->tet_count, rest) : 0u;
    if (rest && bump + rest > a.tcap) {
        // pool full: give the slots back (those inside the pool are marked free) and
        // retry next round after the host has grown the pool
        uint32_t give = from_fl;
        for (uint32_t k = 0; k < rest; ++k)
            if (bump + k < a.tcap) ++give;
        const uint32_t fb = atomicAdd(&a.ctr->fl_next, give);
        uint32_t q = 0;
        for (uint32_t k = 0; k < from_fl; ++k) a.fl_next[fb + q++] = a.fl_cur[take + k];
        for (uint32_t k = 0; k < rest; ++k)
            if (bump + k < a.tcap) {
                a.T[bump + k].v.x = DEAD;
                a.fl_next[fb + q++] = bump + k;
            }
        atomicOr(&a.ctr->error, ERR_POOL);
        a.status[i] = ST_CONFLICT;
        return;
    }
    a.status[i] = ST_WON;
    a.w_take[i] = take;
    a.w_bump[i] = bump;
    a.w_free[i] = nc > nb ? atomicAdd(&a.ctr->fl_next, nc - nb) : 0u;
    a.winners[atomicAdd(&a.ctr->nwin, 1u)] = i;
}

// ------------------------------------------------------------------ 16 lanes per insertion

constexpr int GS = 16;              // lanes per insertion
constexpr int GPB = 256 / GS;       // insertions per 256-thread block
constexpr uint32_t LCAPC = 128;     // cavity tetrahedra held in LDS per insertion
constexpr uint32_t LCAPF = 224;     // boundary facets held in LDS per insertion

// keeps the compiler from moving LDS accesses across a point where other lanes of the
// same wave consume them (the hardware processes one wave's LDS requests in order)
__device__ __forceinline__ void lane_fence() { __asm__ volatile("" ::: "memory"); }

// Same computation as k_cavity, with 16 lanes cooperating on one insertion: the walk
// tests the four facets of the current tetrahedron on four lanes at once, and the cavity
// search expands four cavity tetrahedra (four facets each) per step.  Cavity and boundary
// lists live in LDS and are appended by ballot prefix counts.  Control flow is uniform
// within each group of 16 lanes.
__global__ __launch_bounds__(256) void k_cavity16(RoundArgs a) {
    __shared__ uint32_t s_cav[GPB][LCAPC];
    __shared__ uint32_t s_bnd[GPB][LCAPF];
    __shared__ uint32_t s_out[GPB][LCAPF];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t gl = threadIdx.x & (GS - 1);
    const uint32_t gi = threadIdx.x / GS;
    const uint32_t gbase = lane & ~(uint32_t)(GS - 1);
    const unsigned long long gmask = 0xFFFFull << gbase;
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
        // start: near the nearest inserted point among 8 records on either side of p on the
        // curve, one probe per lane; else near the point's anchor (a record of a lower
        // level); else any live tetrahedron
        const uint32_t d = (gl >> 1) + 1;
        const bool inr = (gl & 1) ? (p + d < a.vhi) : (p >= a.vlo + d);
        const uint32_t ht = inr ? a.vtet[(gl & 1) ? p + d : p - d] : NONE;
        const uint32_t q = a.anchor[p - a.vlo];
        const unsigned long long hm = __ballot(ht != NONE) & gmask;
        uint32_t t = hm ? __shfl(ht, __ffsll((long long)hm) - 1) : (q != NONE ? a.vtet[q] : NONE);
        if (t == NONE) t = a.ctr->any_live;
        uint4 w = a.T[t].v;
        if (w.x == DEAD) {
            t = a.ctr->any_live;
            w = a.T[t].v;
        }
        if (w.w == GHOST) {
            t = a.T[t].n.w >> 2;
            w = a.T[t].v;
        }
        // Walk: lane j < 4 tests facet j
        int entry = -1;
        bool in_ghost = false;
        P3 q0, q1, q2, q3;
        const int jl = (int)(gl & 3u);
        for (;;) {
            q0 = vpos(a.V, w.x);
            q1 = vpos(a.V, w.y);
            q2 = vpos(a.V, w.z);
            q3 = vpos(a.V, w.w);
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
            if ((q0.x == P.x && q0.y == P.y && q0.z == P.z) || (q1.x == P.x && q1.y == P.y && q1.z == P.z) ||
                (q2.x == P.x && q2.y == P.y && q2.z == P.z) || (q3.x == P.x && q3.y == P.y && q3.z == P.z))
                status = ST_DUP;
        }
        uint32_t ncav = 0, nbnd = 0;
        const uint32_t capC = a.capC, capF = a.capF;
        if (status == ST_NONE) {
            // Cavity (same claims as k_cavity): step k expands cavity tetrahedra
            // k0 .. k0+3, lane (slot, facet) = (gl / 4, gl % 4)
            unsigned long long o0 = 0;
            if (gl == 0) o0 = atomicMin(&a.T[t].any, S);
            o0 = __shfl(o0, (int)gbase);
            if (o0 < S) {
                status = ST_CONFLICT;
            } else {
                if (gl == 0) {
                    atomicMin(&a.T[t].cav, S);
                    s_cav[gi][0] = t << 2;
                }
                ncav = 1;
            }
            lane_fence();
            for (uint32_t k0 = 0, nproc = 0; k0 < ncav && status == ST_NONE; k0 += nproc) {
                nproc = min(4u, ncav - k0);  // entries expanded in this step
                const uint32_t slot = k0 + (gl >> 2);
                const int f = jl;
                const bool lv = slot < k0 + nproc;
                const uint32_t code = lv ? s_cav[gi][slot] : 0u;
                const uint32_t c = code >> 2;
                const int pf = slot == 0 ? -1 : (int)(code & 3u);
                const bool act = lv && f != pf;
                uint4 cv = make_uint4(0u, 0u, 0u, 0u), cn = cv, uw = cv;
                if (lv) {
                    cv = a.T[c].v;
                    cn = a.T[c].n;
                }
                const uint32_t ncode = comp(cn, f);
                const uint32_t u = ncode >> 2;
                unsigned long long o1 = S;
                if (act) {
                    o1 = atomicMin(&a.T[u].any, S + 1);
                    uw = a.T[u].v;
                }
                const bool lower_cav = act && o1 < S && !(o1 & 1ull);
                const bool need = act && o1 != S && !lower_cav;
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
                const bool conflict = lower_cav || (inside && o1 < S);
                if (__ballot(conflict) & gmask) {
                    status = ST_CONFLICT;
                    break;
                }
                // a tetrahedron reached through several facets in this step is added once
                bool first = inside;
                for (int m = 0; m < GS; ++m) {
                    const uint32_t um = __shfl(u, (int)gbase + m);
                    const int im = __shfl((int)inside, (int)gbase + m);
                    if ((uint32_t)m < gl && im && um == u) first = false;
                }
                const bool outside = need && !inside;
                const unsigned long long mi = __ballot(first) & gmask;
                const unsigned long long mo = __ballot(outside) & gmask;
                const uint32_t ni = (uint32_t)__popcll(mi), no = (uint32_t)__popcll(mo);
                if (ncav + ni > capC || nbnd + no > capF) {
                    status = ST_OVERFLOW;
                    break;
                }
                if (first) {
                    s_cav[gi][ncav + __popcll(mi & below)] = ncode;
                    atomicMin(&a.T[u].any, S);
                    atomicMin(&a.T[u].cav, S);
                }
                if (outside) {
                    const uint32_t pos = nbnd + (uint32_t)__popcll(mo & below);
                    s_bnd[gi][pos] = (c << 2) | (uint32_t)f;
                    s_out[gi][pos] = ncode;
                }
                ncav += ni;
                nbnd += no;
                lane_fence();
            }
            if (status == ST_NONE) status = ST_CAND;
        }
        if (status == ST_CAND) {
            for (uint32_t k = gl; k < ncav; k += GS) a.cav[(size_t)i * capC + k] = s_cav[gi][k];
            for (uint32_t k = gl; k < nbnd; k += GS) {
                a.bnd[(size_t)i * capF + k] = s_bnd[gi][k];
                a.outc[(size_t)i * capF + k] = s_out[gi][k];
            }
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
    add_stat(&a.ctr->attempts, attempt);
    add_stat(&a.ctr->walk_steps, steps);
    add_stat(&a.ctr->orient, st.orient);
    add_stat(&a.ctr->orient_exact, st.orient_exact);
    add_stat(&a.ctr->insphere, st.insphere);
    add_stat(&a.ctr->insphere_exact, st.insphere_exact);
    add_stat(&a.ctr->perturbed, st.perturbed);
}

// DelaunayBall, GL lanes per winner (Sec. 2.5).  The cavity tetrahedra are first copied to
// the winner's scratch area and their facets resolved to local codes (another cavity
// tetrahedron, or the new tetrahedron on that boundary facet); the new tetrahedra take the cavity's own slots
// (and F - C more when the ball is larger), each glued a priori to its outer tetrahedron;
// finally each new tetrahedron finds its three siblings by pivoting around boundary edges
// through the scratch copies.  Reusing the cavity's slots keeps the tetrahedra of a region
// together in memory.
constexpr uint32_t LOC_BOUNDARY = 0x80000000u;

template <int GL>
__global__ __launch_bounds__(256) void k_build_t(RoundArgs a) {
    constexpr uint32_t WPB = 256 / GL;
    const uint32_t nwin = a.ctr->nwin;
    const uint32_t stride = a.stride;
    const uint32_t fln = a.ctr->fl_n;
    const uint32_t gl = threadIdx.x % GL;
    const uint32_t gi = threadIdx.x / GL;
    const uint32_t capC = a.capC, capF = a.capF;
    unsigned cav_w = 0, bnd_w = 0;
    for (uint32_t base = blockIdx.x * WPB; base < nwin; base += gridDim.x * WPB) {
        const uint32_t w = base + gi;
        const bool act = w < nwin;
        const uint32_t i = act ? a.winners[w] : 0u;
        const uint32_t p = act ? a.cand_pt[i] : 0u;
        const unsigned long long S = act ? (a.round_hi | (2ull * a.cand_rank[i])) : 0ull;
        const uint32_t nc = act ? a.cnt[i] : 0u, nb = act ? a.cnt[stride + i] : 0u;
        const uint32_t take = act ? a.w_take[i] : 0u, bump = act ? a.w_bump[i] : 0u;
        const uint32_t extra = nb > nc ? nb - nc : 0u;
        const uint32_t from_fl = fln > take ? min(extra, fln - take) : 0u;
        const uint32_t *cavl = a.cav + (size_t)i * capC;
        uint32_t *bl = a.bnd + (size_t)i * capF;
        uint32_t *ol = a.outc + (size_t)i * capF;
        uint4 *sv = a.scr_v + (size_t)i * capC;
        uint4 *sn = a.scr_n + (size_t)i * capC;
        // A: copies of the cavity tetrahedra; each records its local index in its spare word
        for (uint32_t k = gl; k < nc; k += GL) {
            const uint32_t c = cavl[k] >> 2;
            sv[k] = a.T[c].v;
            sn[k] = a.T[c].n;
            a.T[c].spare[0] = k;
        }
        __syncthreads();
        // B: facets between two cavity tetrahedra -> (local index << 2 | facet), found by the
        // claim word (only this cavity's tetrahedra hold S); the other facets are boundary
        // facets and are rewritten in C.  C: the ball, in the cavity's slots first; the copy
        // of each boundary facet names its new tetrahedron (LOC_BOUNDARY | slot).  C never
        // writes the claim or spare words.
        for (uint32_t task = gl; task < 4 * nc; task += GL) {
            const uint32_t k = task >> 2;
            const int f = (int)(task & 3u);
            const uint32_t code = comp(sn[k], f);
            const uint32_t nt = code >> 2;
            if (a.T[nt].any == S)
                reinterpret_cast<uint32_t *>(&sn[k])[f] = ((uint32_t)a.T[nt].spare[0] << 2) | (code & 3u);
        }
        __syncthreads();
        for (uint32_t b = gl; b < nb; b += GL) {
            uint32_t slot;
            if (b < nc) {
                slot = cavl[b] >> 2;
            } else {
                const uint32_t e = b - nc;
                slot = e < from_fl ? a.fl_cur[take + e] : bump + (e - from_fl);
            }
            const uint32_t bc = bl[b];
            const uint32_t kb = (uint32_t)a.T[bc >> 2].spare[0];
            const uint32_t oc = ol[b];
            const uint32_t u = oc >> 2;
            const int j = (int)(oc & 3u);
            const uint4 uw = a.T[u].v;
            uint32_t wv[4] = {uw.x, uw.y, uw.z, uw.w};
            wv[j] = p;
            const int pf = orient_new_tet(wv, j);
            a.T[slot].v = make_uint4(wv[0], wv[1], wv[2], wv[3]);
            const uint32_t me = (slot << 2) | (uint32_t)pf;
            nref(a.T, slot, pf) = oc;  // facet opposite p: the outer tetrahedron
            nref(a.T, u, j) = me;      // and back
            reinterpret_cast<uint32_t *>(&sn[kb])[bc & 3u] = LOC_BOUNDARY | slot;
            ol[b] = me;
            bl[b] = (kb << 2) | (bc & 3u);
            for (int q = 0; q < 4; ++q)
                if (wv[q] != GHOST) a.vtet[wv[q]] = slot;
            if (b == 0) a.ctr->any_live = slot;
        }
        __syncthreads();
        // D: siblings by pivoting around the boundary edges through the copies
        for (uint32_t task = gl; task < 3 * nb; task += GL) {
            const uint32_t b = task / 3, qi = task - 3 * b;
            const uint32_t me = ol[b];
            const uint32_t slot = me >> 2;
            const int pf = (int)(me & 3u);
            const int q = (pf + 1 + (int)qi) & 3;  // the three facets through p
            const uint4 sw = a.T[slot].v;
            const uint32_t wv[4] = {sw.x, sw.y, sw.z, sw.w};
            uint32_t e[2];
            int ne = 0;
            for (int r = 0; r < 4; ++r)
                if (r != q && r != pf) e[ne++] = wv[r];
            uint32_t k = bl[b] >> 2;
            int f = (int)(bl[b] & 3u);
            uint32_t res = 0;
            bool ok = false;
            for (uint32_t guard = 0; guard <= nc + 1; ++guard) {
                const uint4 cv = sv[k];
                const uint32_t v4[4] = {cv.x, cv.y, cv.z, cv.w};
                int xpos = -1;
                for (int m = 0; m < 4; ++m)
                    if (m != f && v4[m] != e[0] && v4[m] != e[1]) xpos = m;
                if (xpos < 0) break;
                const uint32_t lc = comp(sn[k], xpos);
                if (lc & LOC_BOUNDARY) {
                    const uint32_t s2 = lc & ~LOC_BOUNDARY;
                    const uint4 nv = a.T[s2].v;
                    const uint32_t w2[4] = {nv.x, nv.y, nv.z, nv.w};
                    int q2 = -1;
                    for (int m = 0; m < 4; ++m)
                        if (w2[m] != e[0] && w2[m] != e[1] && w2[m] != p) q2 = m;
                    if (q2 >= 0) {
                        res = (s2 << 2) | (uint32_t)q2;
                        ok = true;
                    }
                    break;
                }
                k = lc >> 2;
                f = (int)(lc & 3u);
                if (k >= nc) break;
            }
            if (!ok) atomicOr(&a.ctr->error, ERR_WALK);
            nref(a.T, slot, q) = res;
        }
        __syncthreads();
        // E: cavity slots beyond the ball's size are freed
        const uint32_t fb = act ? a.w_free[i] : 0u;
        for (uint32_t k = nb + gl; k < nc; k += GL) {
            const uint32_t c = cavl[k] >> 2;
            a.T[c].v.x = DEAD;
            a.fl_next[fb + (k - nb)] = c;
        }
        if (gl == 0) {
            cav_w += nc;
            bnd_w += nb;
        }
        __syncthreads();
    }
    add_stat(&a.ctr->cav_tets, cav_w);
    add_stat(&a.ctr->bnd_facets, bnd_w);
}

// ------------------------------------------------------------------ round end

__global__ void k_compact(RoundArgs a) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t ncand = *a.ncand_ptr;
    if (i >= ncand) return;
    const uint8_t s = a.status[i];
    if (s == ST_CONFLICT || s == ST_CAND) {
        const uint32_t pos = atomicAdd(a.nnext_ptr, 1u);
        a.next_pt[pos] = a.cand_pt[i];
        a.next_rank[pos] = a.cand_rank[i];
        atomicAdd(&a.ctr->conflicts, 1u);
    } else if (s == ST_OVERFLOW) {
        const uint32_t pos = atomicAdd(a.novf_ptr, 1u);
        a.ovf_pt[pos] = a.cand_pt[i];
        a.ovf_rank[pos] = a.cand_rank[i];
        atomicAdd(&a.ctr->overflows, 1u);
    } else if (s == ST_WON) {
        atomicAdd(&a.ctr->won, 1u);
    } else if (s == ST_DUP) {
        atomicAdd(&a.ctr->dups, 1u);
    } else {
        atomicOr(&a.ctr->error, ERR_WALK);
    }
}

// carry the unused part of this round's free list behind the slots freed this round
__global__ void k_freelist_carry(RoundArgs a) {
    const uint32_t fln = a.ctr->fl_n, take = a.ctr->fl_take, nxt = a.ctr->fl_next;
    if (take >= fln) return;
    const uint32_t left = fln - take;
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < left; k += gridDim.x * blockDim.x)
        a.fl_next[nxt + k] = a.fl_cur[take + k];
}

__global__ void k_roll(Ctr *ctr, uint32_t *consumed, uint32_t tcap) {
    const uint32_t left = ctr->fl_take < ctr->fl_n ? ctr->fl_n - ctr->fl_take : 0u;
    if (ctr->tet_count > tcap) ctr->tet_count = tcap;  // slots beyond the pool were never used
    ctr->fl_n = ctr->fl_next + left;
    ctr->fl_take = 0;
    ctr->fl_next = 0;
    ctr->nwin = 0;
    *consumed = 0;  // the list this round read from is empty now
}

bool round_fits_lds(uint32_t capC, uint32_t capF) { return capC <= LCAPC && capF <= LCAPF; }

hipError_t launch_round(const RoundArgs &a, uint32_t max_cand, hipStream_t s, hipEvent_t *ev) {
    if (max_cand == 0) return hipSuccess;
    const unsigned nb = (max_cand + 255) / 256;
    const bool grouped = round_fits_lds(a.capC, a.capF);
    if (ev) hipEventRecord(ev[0], s);
    if (grouped) k_cavity16<<<(max_cand + GPB - 1) / GPB, 256, 0, s>>>(a);
    else k_cavity<<<nb, 256, 0, s>>>(a);
    if (ev) hipEventRecord(ev[1], s);
    k_check<<<nb, 256, 0, s>>>(a);
    if (grouped) {
        const unsigned gb = (max_cand + GPB - 1) / GPB;
        k_build_t<16><<<gb < 4096u ? gb : 4096u, 256, 0, s>>>(a);
    } else {
        const unsigned gb = (max_cand + 3) / 4;
        k_build_t<64><<<gb < 4096u ? gb : 4096u, 256, 0, s>>>(a);
    }
    if (ev) hipEventRecord(ev[2], s);
    return hipGetLastError();
}

hipError_t launch_round_end(const RoundArgs &a, uint32_t max_cand, bool big, hipStream_t s) {
    (void)big;
    if (max_cand) k_compact<<<(max_cand + 255) / 256, 256, 0, s>>>(a);
    k_freelist_carry<<<256, 256, 0, s>>>(a);
    k_roll<<<1, 1, 0, s>>>(a.ctr, const_cast<uint32_t *>(a.ncand_ptr), a.tcap);
    return hipGetLastError();
}

// ------------------------------------------------------------------ output

__global__ void k_out_flags(const Tet *__restrict__ T, uint32_t count, uint32_t *__restrict__ flags) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const uint4 w = T[t].v;
    flags[t] = (w.x != DEAD && w.w != GHOST) ? 1u : 0u;
}

hipError_t launch_output_flags(const Tet *T, uint32_t count, uint32_t *flags, hipStream_t s) {
    if (count == 0) return hipSuccess;
    k_out_flags<<<(count + 255) / 256, 256, 0, s>>>(T, count, flags);
    return hipGetLastError();
}

__global__ void k_output(const Tet *__restrict__ T, const Vert *__restrict__ V,
                         const uint32_t *__restrict__ map, uint32_t count, uint32_t *__restrict__ tets,
                         int64_t *__restrict__ nbrs) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const uint4 w = T[t].v;
    if (w.x == DEAD || w.w == GHOST) return;
    const uint32_t o = map[t];
    if (tets) {
        tets[4 * (size_t)o + 0] = (uint32_t)V[w.x].idx;
        tets[4 * (size_t)o + 1] = (uint32_t)V[w.y].idx;
        tets[4 * (size_t)o + 2] = (uint32_t)V[w.z].idx;
        tets[4 * (size_t)o + 3] = (uint32_t)V[w.w].idx;
    }
    if (nbrs) {
        const uint4 nn = T[t].n;
        for (int k = 0; k < 4; ++k) {
            const uint32_t nt = comp(nn, k) >> 2;
            nbrs[4 * (size_t)o + k] = T[nt].v.w == GHOST ? -1 : (int64_t)map[nt];
        }
    }
}

hipError_t launch_output(const Tet *T, const Vert *V, const uint32_t *map, uint32_t count, uint32_t *tets,
                         int64_t *nbrs, hipStream_t s) {
    if (count == 0) return hipSuccess;
    k_output<<<(count + 255) / 256, 256, 0, s>>>(T, V, map, count, tets, nbrs);
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
