// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dtk {

constexpr uint32_t GHOST = 0xFFFFFFFFu;  // ghost vertex id (paper Sec. 2.6); always slot 3
constexpr uint32_t DEAD = 0xFFFFFFFEu;   // first vertex slot of a freed tetrahedron
constexpr uint32_t NONE = 0xFFFFFFFFu;   // "no tetrahedron" in the vertex -> tetrahedron hints
constexpr uint32_t MAX_TETS = (1u << 30) - 1;         // 32-bit codes: 4 t + f must fit 32 bits
constexpr uint32_t MAX_TETS_WIDE = 0xFFFFFFF0u;       // 64-bit codes: slots stay 32-bit indices

// A vertex record: 32 bytes so that one aligned fetch brings a whole vertex (Sec. 2.2,
// Listing 1); `idx` holds the global input index (the key of the symbolic perturbation).
struct __align__(32) Vert {
    double x, y, z;
    unsigned long long idx;
};

// One tetrahedron: 64 bytes, so that a visit touches one cache line.  Facet j is opposite
// v[j]; n[j] = 4 t' + f' names the neighbour across it (Sec. 2.2, adjacency code).  The
// claim word of the concurrent rounds lives in the same record.
struct __align__(64) Tet {
    uint4 v;                    // vertex ids (ghost in slot 3); v.x = DEAD once freed
    uint4 n;                    // neighbour codes
    unsigned long long claim;   // lowest claim of the attempts touching it this round:
                                // stamp S (in the attempt's cavity) or S + 1 (outside it)
    unsigned long long spare[3];
};

// The same record with 64-bit neighbour codes, for pools beyond 2^30 slots (the paper's own
// 3e9-tetrahedron scale, Sec. 3.7): still 64 bytes, one line per visit.
struct Codes4W {
    unsigned long long c[4];
};
struct __align__(64) TetW {
    uint4 v;
    Codes4W n;
    unsigned long long claim;
    unsigned long long spare[1];
};
static_assert(sizeof(Tet) == 64 && sizeof(TetW) == 64, "one tetrahedron is one 64-byte record");

// Layout of the tetrahedron pool and its adjacency codes: 32-bit codes (pools below 2^30
// slots) or 64-bit codes.  Slots are 32-bit indices in both.
struct Narrow {
    using Rec = Tet;
    using code = uint32_t;
    using code4 = uint4;
    using set_t = uint32_t;                // cavity-set entry (slot << 1 | kind)
    static constexpr uint32_t LHM = 256;   // regular cavity set entries in LDS
};
struct Wide {
    using Rec = TetW;
    using code = unsigned long long;
    using code4 = Codes4W;
    using set_t = unsigned long long;
    static constexpr uint32_t LHM = 128;   // same LDS bytes as the narrow set
};

__host__ __device__ __forceinline__ uint32_t comp(uint4 q, int k) {
    return k == 0 ? q.x : (k == 1 ? q.y : (k == 2 ? q.z : q.w));
}
__host__ __device__ __forceinline__ unsigned long long comp(const Codes4W &q, int k) {
    return k == 0 ? q.c[0] : (k == 1 ? q.c[1] : (k == 2 ? q.c[2] : q.c[3]));
}

// candidate status after a round
enum : uint8_t {
    ST_NONE = 0,
    ST_CAND = 1,      // cavity built and claimed, waiting for the check
    ST_CONFLICT = 2,  // met a claim of a lower-ranked insertion
    ST_OVERFLOW = 3,  // cavity larger than this round's per-insertion buffer
    ST_DUP = 4,       // exact duplicate of a vertex already in the mesh
    ST_WON = 5,       // inserted
    ST_ERROR = 6,     // walk did not terminate (never expected)
    ST_FULL = 7,      // a sign the fp64 filter could not decide: run again with exact predicates
    ST_WALK = 8       // walk stopped at the round's cap: retried next round from where it stopped
};

enum : uint32_t {
    ERR_WALK = 1u,
    ERR_CAPACITY = 2u,
    ERR_INPUT = 4u,
    ERR_DEGENERATE = 8u,
    ERR_POOL = 16u  // not an error: the tetrahedron pool filled up during a round
};

// Work statistics accumulated by the round kernels.  Each is spread over STAT_SPREAD
// counters 128 bytes apart (block b adds to counter b % STAT_SPREAD), so that concurrent
// waves do not serialize on one address; k_roll sums them into Ctr.
enum : int {
    STAT_ATTEMPTS = 0, STAT_WALK, STAT_ORIENT, STAT_ORIENT_EXACT, STAT_INSPHERE, STAT_INSPHERE_EXACT,
    STAT_PERTURBED, STAT_CAV_TETS, STAT_BND_FACETS, NSTAT
};
constexpr int STAT_SPREAD = 64;
constexpr int STAT_PAD = 16;  // u64 words per counter (128 bytes)
constexpr size_t STAT_WORDS = (size_t)NSTAT * STAT_SPREAD * STAT_PAD;

// Device-resident counters of the round driver.
struct Ctr {
    uint32_t list_count[4];  // lengths of the candidate lists (two normal, two overflow)
    uint32_t fl_n;       // free slots available this round
    uint32_t fl_take;    // slot units taken this round: unit u < fl_n is free-list entry u,
                         // unit u >= fl_n is pool slot tet_count + (u - fl_n)
    uint32_t fl_next;    // slots freed this round
    uint32_t tet_count;  // bump pointer of the tetrahedron pool
    uint32_t won;        // insertions so far (this and the other counters below: since the
    uint32_t conflicts;  // last clear), conflicts,
    uint32_t overflows;  // cavity buffer overflows,
    uint32_t dups;       // duplicates found
    uint32_t error;      // ERR_* flags
    uint32_t init[4];    // sorted positions of the initial tetrahedron's vertices
    uint32_t bad_cloud;  // first cloud found degenerate by the initial-tetrahedron search
    uint32_t any_live;   // some live tetrahedron (walk start of last resort)
    uint32_t chunk;      // length of a list slice processed as one round
    uint32_t dropped;    // freed slots that did not fit the free list (left unused)
    uint32_t ndefer;     // candidates of this round handed to the exact-predicate pass
    uint32_t deferred;   // such candidates since the last clear
    uint32_t walk_caps;  // attempts stopped at the walk cap since the last clear
    unsigned long long walk_steps, cav_tets, bnd_facets;
    unsigned long long orient, orient_exact, insphere, insphere_exact, perturbed;
    unsigned long long attempts;
};

// learned scheduler: MLP NFEAT -> NHID -> NHID -> NOUT
constexpr int NFEAT = 16, NHID = 64, NOUT = 3;
constexpr int NPARAM = NFEAT * NHID + NHID + NHID * NHID + NHID + NHID * NOUT + NOUT;

// One independent point cloud of a call (a single-cloud call is a batch of one).  Its vertex
// records are [lo, hi) in curve order; the cloud id is stored in the upper 32 bits of each
// record's idx.
struct Cloud {
    uint32_t lo, hi;     // vertex records of this call belonging to the cloud
    uint32_t any_live;   // a live tetrahedron of the cloud's mesh (walk start of last resort)
    uint32_t m;          // Moore level of the cloud's cubic grid
    double box[4];       // grid origin (x, y, z) and scale 2^m / largest extent
};

// Arguments of one insertion round.  The pool and the code buffers are typed by the
// kernels' layout (Narrow or Wide): T is K::Rec[tcap], cav and outc are K::code arrays,
// scr_n is a K::code4 array.
struct RoundArgs {
    const Vert *V;
    void *T;                     // tetrahedron pool
    uint32_t *vtet;              // vertex -> a live tetrahedron containing it
    uint32_t vlo, vhi;           // vertex records of the current call
    const uint32_t *anchor;      // walk anchor of each record of the call (a lower-level record
                                 // of the same cloud), indexed by record - vlo
    uint32_t *lastt;             // where the record's last attempt located it (NONE before the
                                 // first), indexed by record - vlo: the start of its next walk
    uint32_t multi;              // 1: the call has several clouds (slots move between them)
    uint32_t walk_cap;           // filter pass: walk steps after which an attempt stops (ST_WALK)
    Cloud *clouds;               // the call's clouds (walk bounds, live tetrahedron)
    uint32_t *log_att;           // if set: attempts per record of the call (record - vlo)
    const uint8_t *wbucket;      // if set: 1 = start the walk at the anchor (record - vlo)
    const uint32_t *cand_pt;     // current candidate list
    const uint32_t *cand_rank;
    uint32_t *next_pt;           // losers for the next round
    uint32_t *next_rank;
    uint32_t *ovf_pt;            // overflowed candidates
    uint32_t *ovf_rank;
    const uint32_t *ncand_ptr;   // device count of the current list
    uint32_t *nnext_ptr;         // device count of the next list
    uint32_t *novf_ptr;          // device count of the overflow list
    void *subd;                  // if set: [tcap] cached sub-determinants (SubD) of each finite tetrahedron
    uint32_t *defer;             // [stride] candidates handed to the exact-predicate pass
    uint32_t *ndefer_ptr;        // device count of them (reset at the round's end)
    void *cav;                   // [stride][capC] cavity tetrahedra (code 4 t + entry facet)
    uint32_t *bnd;               // [stride][capF] boundary facets (4 c + f, c in the cavity)
    void *outc;                  // [stride][capF] outer codes, then new tetrahedra
    uint32_t *cnt;               // [2][stride] cavity size, boundary size
    uint8_t *status;             // [stride]
    uint4 *scr_v;                // [stride][capC] vertex copies of the winners' cavity tetrahedra
    void *scr_n;                 // [stride][capC] their neighbour codes (pivoting balls)
    uint32_t *fl_cur;            // free list consumed this round
    uint32_t *fl_next;           // free list filled this round
    uint32_t flcap;              // entries of each free list (slots freed beyond it are dropped)
    Ctr *ctr;
    unsigned long long *stat;    // [NSTAT][STAT_SPREAD][STAT_PAD] work statistics
    uint32_t stride, capC, capF, tcap;
    uint32_t hmg;                // capC > 1024: entries of the cavity set in global memory
    unsigned long long round_hi;  // (0xFFFFFFFF - round) << 32: newer rounds claim lower
    // if set (trace mode): [stride][8] per attempt.  Filter pass: wall clock (100 MHz) at its
    // start, at the walk's end and at its end, then walk steps | cavity steps << 16 | cavity
    // size << 32 | status << 48.  Ball kernel: clock at its start, after the winner test and
    // slot reservation, after the cavity copies and at its end.
    unsigned long long *clk;
};

// New candidates of one round: a window of ranks split into aligned power-of-two blocks,
// block j covering local ranks a[j] .. a[j] + 2^w[j] of level lvl[j]; threads off[j] ..
// off[j+1] handle block j, in the order of the records on the curve.
constexpr int FILL_BLOCKS = 48;
struct FillPlan {
    uint32_t nblk;
    uint32_t lvl[FILL_BLOCKS], a[FILL_BLOCKS], w[FILL_BLOCKS], off[FILL_BLOCKS + 1];
};

// ---- launch wrappers (dt_sort.hip) ----
// Validation and per-cloud bounding boxes: chunk j covers input points [ch_start[j],
// ch_end[j]) of cloud ch_cloud[j]; cloud c owns chunks [cloud_ch[c], cloud_ch[c + 1]).
hipError_t launch_cloud_bbox(const double *xyz, const uint64_t *ch_start, const uint64_t *ch_end,
                             uint32_t nchunks, double *partial, const uint32_t *cloud_ch, uint32_t nclouds,
                             Cloud *clouds, uint32_t *err, hipStream_t s);
// keys[i] = cloud << shift | Moore index of point i in its cloud's grid; vals[i] = i
hipError_t launch_keys(const double *xyz, uint64_t n, const uint64_t *off, uint32_t nclouds, const Cloud *clouds,
                       int shift, unsigned long long *keys, uint32_t *vals, hipStream_t s);
hipError_t radix_sort_pairs(unsigned long long *keys, uint32_t *vals, unsigned long long *keys_tmp,
                            uint32_t *vals_tmp, uint32_t *hist, uint32_t *scan_tmp, uint64_t n,
                            int nbits, hipStream_t s, bool *swapped);
// the same, in one block (one launch) when n fits one tile of the multi-block form
hipError_t radix_sort_pairs_any(unsigned long long *keys, uint32_t *vals, unsigned long long *keys_tmp,
                                uint32_t *vals_tmp, uint32_t *hist, uint32_t *scan_tmp, uint64_t n, int nbits,
                                hipStream_t s, bool *swapped);
size_t radix_hist_entries(uint64_t n);
hipError_t launch_permute(const double *xyz, const uint32_t *vals, const unsigned long long *skeys, int shift,
                          uint64_t n, uint64_t base, uint64_t idx_offset, Vert *V, uint32_t *vtet, uint8_t *dup,
                          hipStream_t s);
hipError_t launch_level_hist(const unsigned long long *keys, uint64_t n, int shift, uint32_t *hist,
                             hipStream_t s);
hipError_t launch_levels(const uint32_t *src, const Vert *V, uint64_t n, uint64_t base, const uint64_t *off,
                         const Cloud *clouds, uint64_t salt, unsigned long long *keys, uint32_t *vals,
                         uint8_t *lev_out, hipStream_t s);
hipError_t launch_hint_anchor(const Vert *V, uint64_t base, uint64_t n, uint64_t idx_offset, const uint32_t *hint,
                              uint32_t *anchor, hipStream_t s);
hipError_t launch_anchor(const uint32_t *lord, const uint32_t *start, int L, const Vert *V, uint64_t base,
                         uint64_t n, uint32_t *anchor, hipStream_t s);
hipError_t launch_dedupe(const Vert *V, uint64_t base, uint64_t n, unsigned long long *table,
                         uint64_t tsize, uint8_t *dup, uint32_t *ndup, hipStream_t s);
hipError_t exclusive_scan_u32(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *tmp,
                              uint32_t *total, hipStream_t s);
size_t scan_tmp_entries(uint64_t n);
// the level of point i (local index li in a cloud of n points): first k with u n < cum_k 2^53
__device__ __forceinline__ int brio_level(unsigned long long u, unsigned long long n) {
    unsigned long long size = 2048;
    int lev = 0;
    for (;;) {
        const unsigned long long cum = size < n ? size : n;
        if (cum >= n) return lev;
        // u * n < cum * 2^53, in 128 bits
        const unsigned long long lo = u * n, hi = __umul64hi(u, n);
        const unsigned long long clo = cum << 53, chi = cum >> 11;
        if (hi < chi || (hi == chi && lo < clo)) return lev;
        ++lev;
        size *= 7;
    }
}

// ---- launch wrappers (dt_learn.hip) ----
hipError_t launch_features(const Vert *V, uint64_t base, uint64_t n, const Cloud *clouds, const uint32_t *anchor,
                           const uint8_t *level, int L, float *feat, hipStream_t s);
hipError_t launch_mlp_infer(const uint16_t *wbf, const float *feat, uint64_t n, float *y, hipStream_t s);
hipError_t launch_to_bf16(const float *w, uint16_t *wbf, hipStream_t s);
hipError_t launch_mlp_grad(const uint16_t *wbf, const float *feat, const float *cost, const uint8_t *bucket,
                           uint64_t b0, uint32_t nb, float *grad, float *loss, hipStream_t s);
hipError_t launch_adam(float *w, float *grad, float *m1, float *m2, uint16_t *wbf, float lr, int t, hipStream_t s);
hipError_t launch_learned_keys(const float *y, const uint8_t *level, uint64_t n, uint64_t base, float thr,
                               unsigned long long *keys, uint32_t *vals, uint8_t *wbucket, hipStream_t s);
hipError_t launch_labels(const Vert *V, uint64_t base, uint64_t n, const Cloud *clouds, const uint32_t *anchor,
                         const uint8_t *level, const uint32_t *attempts, float *cost, uint8_t *bucket,
                         hipStream_t s);

// ---- launch wrappers (dt_insert.hip) ----
// initial tetrahedron and four ghosts of each cloud c at slots 5 c0 + 5 c .. + 4 (c0: first)
// Every wrapper that touches the pool takes `wide`: the pool holds TetW records with 64-bit
// codes (true) or Tet records with 32-bit codes (false).
hipError_t launch_init(const Vert *V, Cloud *clouds, uint32_t nclouds, uint32_t first_slot, const uint8_t *dup,
                       void *T, bool wide, uint32_t *vtet, Ctr *ctr, void *subd, hipStream_t s);
hipError_t launch_fill_list(const FillPlan &plan, const uint32_t *lvl_start, const uint32_t *lvl_size,
                            const uint32_t *lvl_bits, const unsigned long long *rank_base, const uint32_t *lord,
                            const uint8_t *dup, const uint32_t *vtet, uint32_t *cand_pt, uint32_t *cand_rank,
                            uint32_t *ncand, hipStream_t s);
// exact: launch the exact-predicate pass after the filter pass of a regular round (without
// it, attempts the filter hands on retry in the next round)
hipError_t launch_round(const RoundArgs &a, bool wide, uint32_t max_cand, uint32_t lanes, uint32_t large_lanes,
                        bool exact, hipStream_t s, hipEvent_t *ev);
hipError_t launch_round_end(const RoundArgs &a, uint32_t max_cand, hipStream_t s, Ctr *snap,
                            unsigned long long *seq, unsigned long long tag);
// A regular round (cavity buffers of the regular size) as one HIP graph: the fill, the two
// cavity passes, the DelaunayBall kernel and the three round-end kernels as a chain of kernel
// nodes.  The graph is built and instantiated once per launch shape (pool layout, lanes per
// insertion); each later round of that shape only updates the nodes' arguments and grids.
struct FillArgs {
    const uint32_t *lvl_start, *lvl_size, *lvl_bits;
    const unsigned long long *rank_base;
    const uint32_t *lord;
    const uint8_t *dup;
    const uint32_t *vtet;
    uint32_t *cand_pt, *cand_rank, *ncand;
};
struct RoundGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t node[7] = {};
};
constexpr int ROUND_GRAPH_SHAPES = 10;  // pool layout (2) x lanes per insertion (4, 8, 16, 32, 64)
hipError_t launch_round_graph(RoundGraph *graphs, const FillPlan &plan, const FillArgs &fa, const RoundArgs &a,
                              bool wide, uint32_t max_cand, uint32_t lanes, Ctr *snap, unsigned long long *seq,
                              unsigned long long tag, hipStream_t s);
void destroy_round_graphs(RoundGraph *graphs);
hipError_t launch_reset_claims(void *T, bool wide, uint32_t tcap, hipStream_t s);
// copies `count` Tet records into TetW records
hipError_t launch_widen(const void *src, void *dst, uint32_t count, hipStream_t s);
// export: live bit set (one word per 64 slots) with per-word counts, input index per vertex
// record, and the output rows of live slots [t0, t1) at out_index - obase
hipError_t launch_live_bits(const void *T, bool wide, uint32_t count, unsigned long long *bits, uint32_t *wcnt,
                            hipStream_t s);
hipError_t launch_out_vid(const Vert *V, uint32_t nv, uint32_t *vid, hipStream_t s);
hipError_t launch_output(const void *T, bool wide, const uint32_t *vid, const unsigned long long *bits,
                         const uint32_t *pre, uint32_t t0, uint32_t t1, uint32_t obase, uint32_t *tets, int64_t *nbrs,
                         hipStream_t s);
// grouping of the live finite tetrahedra by cloud (see dt_get_tets_batch)
hipError_t launch_tet_cloud(const void *T, bool wide, const Vert *V, uint32_t count, uint32_t nclouds,
                            unsigned long long *keys, uint32_t *vals, hipStream_t s);
hipError_t launch_seg_bounds(const unsigned long long *keys, uint32_t count, uint32_t nclouds, uint32_t *toff,
                             hipStream_t s);
hipError_t launch_tet_map(const uint32_t *sorted, uint32_t nlive, uint32_t *map, hipStream_t s);
hipError_t launch_output_cloud(const void *T, bool wide, const Vert *V, const uint32_t *sorted, const uint32_t *map,
                               uint32_t tb, uint32_t te, uint64_t vbase, uint32_t *tets, int64_t *nbrs, hipStream_t s);
hipError_t launch_predicates(int kind, const double *pts, const int64_t *idx, uint64_t k, int8_t *out,
                             hipStream_t s);
// coordinates of every vertex record at its input index (single-cloud contexts)
hipError_t launch_points_out(const Vert *V, uint32_t nv, double *xyz, hipStream_t s);

// ---- launch wrappers (dt_refine.hip): circumcentre refinement steps
hipError_t launch_hull_facets(const void *T, bool wide, uint32_t count, uint4 *facets, uint32_t *nfacets,
                              hipStream_t s);
// prev / pbig (count entries): each slot's vertices and "larger than 1.4 h" at the last pass,
// valid for the first `known` slots; rewritten for the next pass
hipError_t launch_circum(const void *T, bool wide, const Vert *V, uint32_t count, double grow, uint4 *prev,
                         uint8_t *pbig, uint32_t known, double *cc, uint4 *q, uint32_t *src, uint32_t cap,
                         uint32_t *ncand, hipStream_t s);
// a closed axis-aligned box whose eight corners are strictly inside the convex hull, so every
// point of it is (the hull is convex); lo > hi on an axis for none
struct InnerBox {
    double lo[3], hi[3];
};
// candidates in `box` are inside without the facet tests; the others are listed in rest[k]
// (*nrest zero on entry) for them
hipError_t launch_inside(const Vert *V, const uint4 *facets, uint32_t nf, const double *cc, const uint4 *q,
                         const uint32_t *src, uint32_t k, const InnerBox &box, uint32_t *rest, uint32_t *nrest,
                         uint8_t *flag, double *cc2, uint4 *q2, uint32_t *src2, uint32_t *nin, hipStream_t s);
hipError_t launch_order_keys(const uint4 *q, const unsigned long long *moore, const uint32_t *perm, uint32_t k,
                             int which, int bits, unsigned long long *keys, uint32_t *vals, hipStream_t s);
hipError_t launch_cell_keys(const double *lo, double cell, uint64_t g, const double *xyz, const Vert *V, uint32_t n,
                            unsigned long long *keys, uint32_t *vals, hipStream_t s);
hipError_t launch_near_vertex(const double *lo, double cell, uint64_t g, const Vert *V, const unsigned long long *vkeys,
                              const uint32_t *vidx, uint32_t nv, const double *cc, const uint32_t *src,
                              const uint32_t *perm, uint32_t k, double lim, double *ccr, uint32_t *srcr,
                              uint8_t *status, hipStream_t s);
// the filter rounds' lists of close earlier candidates: near[8 * k], nnear[k]
constexpr uint32_t FILTER_NEAR_MAX = 8;
hipError_t launch_filter_near(const double *lo, double cell, uint64_t g, const unsigned long long *ckeys,
                              const uint32_t *crank, uint32_t k, const double *ccr, double lim, const uint8_t *status,
                              uint32_t *near, uint8_t *nnear, hipStream_t s);
hipError_t launch_filter_round(const double *lo, double cell, uint64_t g, const unsigned long long *ckeys,
                               const uint32_t *crank, uint32_t k, const double *ccr, double lim, const uint32_t *near,
                               const uint8_t *nnear, uint8_t *status, uint32_t *undecided, hipStream_t s);
hipError_t launch_kept(const uint8_t *status, uint32_t k, uint32_t *flags, const uint32_t *pos, const double *ccr,
                       const uint32_t *srcr, double *out, uint32_t *hint, int phase, hipStream_t s);
hipError_t launch_vert_box(const Vert *V, uint32_t n, uint32_t m, double *partial, uint32_t nblocks, Cloud *cl,
                           hipStream_t s);

}  // namespace dtk
