// Host driver and C ABI of the library (include/dt.h).
//
// dt_insert_points: validate + bounding box -> Moore keys -> radix sort -> vertex records
// in Moore order -> BRIO levels and the level-major order of the records -> duplicates ->
// initial tetrahedron (first call) -> insertion rounds until every point of the call is
// inserted (paper Algorithm 1, with the sequential loop replaced by rounds of concurrent
// insertions).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dt.h"
#include "dt_internal.h"

using namespace dtk;

namespace {

constexpr uint32_t DEFAULT_ROUND_MAX = 1u << 20;
constexpr uint32_t DEFAULT_CAVITY_CAP = 128;
constexpr uint32_t DEFAULT_LANES = 16;
constexpr double DEFAULT_ROUND_FRACTION = 1.0 / 16.0;
constexpr uint32_t DEFAULT_WALK_CAP = 16;
constexpr uint32_t DEFAULT_LARGE_LANES = 256;
// automatic lanes: rounds of fewer candidates than this use 64 lanes per insertion; with the
// automatic round fraction they take 1.5 times the usual share of the mesh's vertices
constexpr uint32_t SMALL_ROUND = 32768;
constexpr double SHORT_ROUND_FRACTION_SCALE = 1.5;
constexpr uint32_t ROUND_MIN = 256;
constexpr uint32_t DRAIN_SLICE = 4096;  // candidates per round when draining overflowed cavities
constexpr uint32_t EXPORT_CHUNK = 1u << 24;  // slots per staged export launch (a multiple of 64)
constexpr size_t TET_BYTES = 64;               // one tetrahedron record, either layout
constexpr size_t SUBD_BYTES = 40;              // its cached sub-determinants (dt_options.subdet_cache)
// entries of each free list: slots freed while it is full stay unused (the pool has room for
// them); in practice a round frees far fewer
constexpr uint64_t FREE_LIST_MAX = 1ull << 26;
// calls with more points release the sort's temporaries before the rounds
constexpr uint64_t BIG_CALL_POINTS = 1ull << 27;
// learned order: where the points above the median training cost needed COSTLY_ATTEMPTS
// attempts or more on average, rounds over the costly halves take COSTLY_ROUND_SCALE of the
// usual size (fewer of these conflict-heavy points at once)
constexpr uint32_t COSTLY_ATTEMPTS = 3;
constexpr double COSTLY_ROUND_SCALE = 0.5;

uint64_t host_mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int moore_level(uint64_t n) {
    int m = 1;
    while (m < 21 && (1ull << (3 * m)) < n) ++m;
    return m;
}

// cumulative BRIO sizes 2048 * 7^k, capped at n
std::vector<uint64_t> brio_cum(uint64_t n) {
    std::vector<uint64_t> cum;
    uint64_t size = 2048;
    for (;;) {
        cum.push_back(std::min(size, n));
        if (size >= n) break;
        size *= 7;
    }
    return cum;
}

template <class T>
struct DevBuf {
    T *p = nullptr;
    size_t cap = 0;  // elements
};

}  // namespace

struct dt_ctx {
    dt_options opt{};
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err = "no error";

    uint64_t npoints = 0;  // points passed so far (global input indices)
    uint64_t nv = 0;       // vertex records in V
    bool have_mesh = false;
    uint64_t round_counter = 0;  // monotonic over the context's lifetime
    uint64_t mesh_vertices = 0;
    int fl_idx = 0;
    int list_idx = 0;
    int ovf_idx = 0;

    DevBuf<Vert> V;
    DevBuf<uint32_t> vtet, anchor, lastt;
    DevBuf<uint8_t> dup;
    uint32_t tcap = 0;
    void *T = nullptr;       // Tet[tcap] (32-bit codes) or TetW[tcap] (64-bit codes)
    void *subd = nullptr;    // dt_options.subdet_cache: SubD[tcap], the cached sub-determinants
    bool wide = false;       // the pool's layout
    uint64_t narrow_max = MAX_TETS;  // growth past this widens an automatic pool
    uint32_t flcap = 0;      // entries of each free list
    uint32_t *fl[2] = {nullptr, nullptr};

    uint32_t list_cap = 0;
    uint32_t *lpt[4] = {}, *lrank[4] = {};
    size_t bufC = 0, bufF = 0;
    uint32_t capC = 0, capF = 0;
    uint32_t lanes = 8;  // lanes per insertion of the cavity kernel
    bool lanes_auto = true;  // lanes_per_insert 0: 64 lanes in rounds below SMALL_ROUND
    // exact-predicate pass: launched in the regular rounds once the call's filter passes have
    // handed on an attempt (counted in Ctr::deferred, which stood at deferred_base when the
    // call began); inputs whose fp64 filter decides everything never launch it
    bool exact_needed = false;
    unsigned long long deferred_base = 0;
    uint32_t large_lanes = 256;  // the same in rounds for large cavities (64 or 256)
    double frac = 0;     // round size as a fraction of the mesh's vertices
    bool frac_auto = true;  // round_fraction 0: short rounds take SHORT_ROUND_FRACTION_SCALE times more
    uint32_t call_clouds = 1;  // clouds of the insertion call in progress
    // dt_autotune's choices by size class (floor(log2 n) of the sample): an insertion takes
    // the choice of the nearest tuned class; without any, the options decide
    struct Tuned {
        bool set = false;
        uint32_t lanes = 0, cap = 0, large = 0;
        double frac = 0;
        double ms = 0;
    } tuned[64];
    uint32_t *defer = nullptr;             // candidates handed to the exact-predicate pass
    void *cav = nullptr, *outc = nullptr;  // adjacency codes (4 or 8 bytes each)
    uint32_t *bnd = nullptr, *cnt = nullptr;
    uint4 *scr_v = nullptr;
    void *scr_n = nullptr;
    uint8_t *status = nullptr;
    bool buf_wide = false;  // code width the round buffers were sized for

    Ctr *ctr = nullptr;
    Ctr *hctr = nullptr;   // pinned: the counters after the last completed round (one of hring)
    Ctr *hring = nullptr;  // three pinned snapshots: the host's and one per round in flight
    // pinned ring: the round-end kernel writes each snapshot there and then sets hseq[slot]
    // to the round's tag (else a copy and an event per round)
    bool ring_direct = false;
    unsigned long long *hseq = nullptr;
    unsigned long long tag_counter = 0;
    unsigned long long slot_tag[3] = {0, 0, 0};
    unsigned long long *stat = nullptr;  // spread work statistics (summed into ctr each round)

    // per-call scratch
    DevBuf<double> staging;
    DevBuf<unsigned long long> keys, keys_tmp, table;
    DevBuf<uint32_t> vals, vals_tmp, hist, scan_tmp, small;
    DevBuf<uint64_t> small64;
    // output scratch
    DevBuf<unsigned long long> obits;  // export: live bit set, one word per 64 slots
    DevBuf<uint32_t> owcnt, opre, otets, ovid;
    DevBuf<int64_t> onbrs;

    hipEvent_t ev[3][3] = {};   // per snapshot slot: kernel timing events of its round
    hipEvent_t evdone[3] = {};  // per snapshot slot: its copy has landed
    uint32_t slot_cand[3] = {}, slot_capC[3] = {};
    bool slot_timed[3] = {};  // the round in the slot recorded timing events
    bool grow_pending = false;  // a round found the pool full: grow before the next one
    dt_stats st{};
    uint32_t trace_prev_won = 0, trace_prev_conf = 0, trace_prev_ovf = 0;
    uint64_t trace_rounds = 0;
    unsigned long long trace_prev_att = 0, trace_prev_walk = 0, trace_prev_cav = 0, trace_prev_ins = 0;
    const uint32_t *lord = nullptr;  // level-major order of the current call's vertex records
    // clouds of the current call (one for dt_insert_points)
    uint32_t nclouds = 0;
    bool batch = false;                  // the context holds a dt_insert_batch result
    DevBuf<Cloud> clouds;
    DevBuf<uint64_t> off, ch_start, ch_end;
    DevBuf<uint32_t> cloud_ch;
    DevBuf<double> partial;
    std::vector<uint64_t> h_off;         // input offsets of the clouds (nclouds + 1)
    // per-cloud output index (batch): tetrahedra grouped by cloud
    bool out_index = false;
    DevBuf<unsigned long long> okeys;
    DevBuf<uint32_t> osorted, omap2;
    std::vector<uint64_t> h_toff;
    const uint32_t *osorted_live = nullptr;
    // learned scheduler: per-record level, attempts log, walk bucket, features, predictions;
    // the model (fp32 master weights, bf16 copy, Adam moments)
    DevBuf<uint8_t> lev, wbucket;
    DevBuf<uint32_t> log_att;
    DevBuf<float> feat, ypred;
    bool have_model = false, logged = false;
    bool learned_active = false;  // this call runs the learned order (scheduler set and a model loaded)
    float thr = 0.0f;
    float costly_scale = 1.0f;
    uint64_t log_base = 0, log_n = 0;
    DevBuf<float> w32, m1, m2, grad, loss;
    DevBuf<uint16_t> wbf;
    // scratch of dt_debug_sort (kept apart from the mesh's own buffers)
    DevBuf<Vert> dbgV;
    DevBuf<Cloud> dbg_cloud;
    // DT_TRACE=1 in the environment: one line per round on stderr; DT_TRACE=2 adds the
    // distribution of the filter pass's per-attempt clocks (walk, cavity, launch span)
    int trace = 0;
    unsigned long long *clk[3] = {nullptr, nullptr, nullptr};  // per snapshot slot
    uint32_t clk_cap[3] = {0, 0, 0};
    std::vector<unsigned long long> clk_host;
    // Device memory source: hipMalloc, or (no-allocation entry point) a bump arena carved
    // from the library's static scratch array, reset at every call; then nothing is freed,
    // events are not used (rounds complete by stream synchronization) and the counters'
    // host copies are static memory.
    // refinement (dt_refine): candidates, their ordering, grids and the kept points
    DevBuf<double> rf_cc, rf_cc2, rf_ccr, rf_pts, rf_partial;
    DevBuf<uint4> rf_q, rf_q2, rf_facets;
    DevBuf<unsigned long long> rf_moore, rf_k0, rf_k1;
    DevBuf<uint32_t> rf_v0, rf_v1, rf_ctr, rf_flags, rf_pos;
    DevBuf<uint32_t> rf_src, rf_src2, rf_srcr, rf_hint, rf_rest, rf_near;  // candidates' tetrahedron vertex records
    RoundGraph graphs[ROUND_GRAPH_SHAPES];              // graph-launched rounds, one per launch shape
    DevBuf<uint8_t> rf_status, rf_flag, rf_pbig, rf_nnear;
    DevBuf<uint4> rf_prev;  // each slot's vertices at the last refinement pass
    DevBuf<Cloud> rf_cloud;
    DevBuf<uint64_t> rf_off;
    unsigned char *arena = nullptr;
    size_t arena_size = 0, arena_used = 0;
    DevBuf<Ctr> ctrbuf;                          // counters and statistics in the arena
    DevBuf<unsigned long long> statbuf;
    uint32_t round_cap = DEFAULT_ROUND_MAX;  // candidates per round buffer (smaller in the arena)
    uint32_t export_chunk = EXPORT_CHUNK;    // slots per staged export launch
};

namespace {

int fail(dt_ctx *c, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

#define HIPCHK(x)                                                                          \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess) return fail(c, DT_E_DEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

// Device memory of the context: hipMalloc, or the next 256-byte aligned piece of the arena.
hipError_t dev_alloc(dt_ctx *c, void **p, size_t bytes) {
    if (!c->arena) return hipMalloc(p, bytes);
    const size_t off = (c->arena_used + 255) & ~(size_t)255;
    if (off > c->arena_size || bytes > c->arena_size - off) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    *p = c->arena + off;
    c->arena_used = off + bytes;
    return hipSuccess;
}

void dev_free(dt_ctx *c, void *p) {
    if (!c->arena && p) hipFree(p);
}

template <class T>
int ensure(dt_ctx *c, DevBuf<T> &b, size_t n, bool keep = false) {
    if (b.cap >= n && b.p) return DT_OK;
    size_t cap = std::max<size_t>(n, 1);
    if (b.cap) cap = std::max(cap, b.cap + b.cap / 2);
    T *p = nullptr;
    if (dev_alloc(c, (void **)&p, cap * sizeof(T)) != hipSuccess) {
        hipGetLastError();
        return fail(c, DT_E_CAPACITY, "device allocation of %zu bytes failed", cap * sizeof(T));
    }
    if (keep && b.p && b.cap) HIPCHK(hipMemcpyAsync(p, b.p, b.cap * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
    if (b.p) {
        HIPCHK(hipStreamSynchronize(c->stream));
        dev_free(c, b.p);
    }
    b.p = p;
    b.cap = cap;
    return DT_OK;
}

bool is_device_ptr(const void *p) {
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice;
}

int sync_ctr(dt_ctx *c) {
    HIPCHK(hipMemcpyAsync(c->hctr, c->ctr, sizeof(Ctr), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return DT_OK;
}

int realloc_code_buffers(dt_ctx *c);

// Grows (or first allocates) the tetrahedron pool to at least `need` slots.  A pool with
// 32-bit codes that must pass 2^30 slots is widened to 64-bit codes on the way when the
// options allow it (index_bits 0); the records are converted on the device.
int grow_tets(dt_ctx *c, uint64_t need) {
    bool wide = c->wide;
    if (!wide && need > c->narrow_max) {
        if (c->opt.index_bits == 32)
            return fail(c, DT_E_CAPACITY, "more than %u tetrahedra needed with 32-bit adjacency codes "
                                          "(dt_options.index_bits = 64 or 0 lifts the limit)", MAX_TETS);
        wide = true;
    }
    const uint64_t max_tets = wide ? MAX_TETS_WIDE : MAX_TETS;
    if (need > max_tets) return fail(c, DT_E_CAPACITY, "more than %llu tetrahedra needed", (unsigned long long)max_tets);
    uint64_t cap = std::max<uint64_t>(need, (uint64_t)c->tcap + c->tcap / 2);
    cap = std::min<uint64_t>(cap, max_tets);
    const uint32_t flcap = (uint32_t)std::min<uint64_t>(cap, FREE_LIST_MAX);
    void *T = nullptr, *sd = nullptr;
    uint32_t *f0 = nullptr, *f1 = nullptr;
    bool ok = dev_alloc(c, &T, cap * TET_BYTES) == hipSuccess &&
              dev_alloc(c, (void **)&f0, (size_t)flcap * sizeof(uint32_t)) == hipSuccess &&
              dev_alloc(c, (void **)&f1, (size_t)flcap * sizeof(uint32_t)) == hipSuccess &&
              (!c->opt.subdet_cache || dev_alloc(c, &sd, cap * SUBD_BYTES) == hipSuccess);
    if (!ok) {
        hipGetLastError();
        dev_free(c, T); dev_free(c, f0); dev_free(c, f1); dev_free(c, sd);
        return fail(c, DT_E_CAPACITY, "device allocation for %llu tetrahedra failed", (unsigned long long)cap);
    }
    // claim words start above every stamp
    HIPCHK(hipMemsetAsync(T, 0xFF, cap * TET_BYTES, c->stream));
    if (c->tcap) {
        uint64_t used = c->hctr->tet_count;
        if (wide && !c->wide) HIPCHK(launch_widen(c->T, T, (uint32_t)used, c->stream));
        else HIPCHK(hipMemcpyAsync(T, c->T, used * TET_BYTES, hipMemcpyDeviceToDevice, c->stream));
        uint64_t nf = std::min<uint64_t>(c->hctr->fl_n, flcap);
        HIPCHK(hipMemcpyAsync(c->fl_idx == 0 ? f0 : f1, c->fl[c->fl_idx], nf * sizeof(uint32_t),
                              hipMemcpyDeviceToDevice, c->stream));
        if (sd && c->subd) HIPCHK(hipMemcpyAsync(sd, c->subd, used * SUBD_BYTES, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        dev_free(c, c->T); dev_free(c, c->fl[0]); dev_free(c, c->fl[1]); dev_free(c, c->subd);
    }
    c->T = T; c->fl[0] = f0; c->fl[1] = f1;
    c->subd = sd;
    c->tcap = (uint32_t)cap;
    c->flcap = flcap;
    const bool widened = wide && !c->wide;
    c->wide = wide;
    // the code buffers of the rounds follow the pool's code width (the candidate lists, which
    // may hold pending candidates, are kept)
    if (widened && c->cav) return realloc_code_buffers(c);
    return DT_OK;
}

// cavity and outer lists and neighbour copies for the pool's code width
int realloc_code_buffers(dt_ctx *c) {
    HIPCHK(hipStreamSynchronize(c->stream));
    dev_free(c, c->cav); dev_free(c, c->outc); dev_free(c, c->scr_n);
    c->cav = c->outc = c->scr_n = nullptr;
    const size_t cb = c->wide ? sizeof(unsigned long long) : sizeof(uint32_t);
    if (dev_alloc(c, &c->cav, c->bufC * cb) != hipSuccess || dev_alloc(c, &c->outc, c->bufF * cb) != hipSuccess ||
        dev_alloc(c, &c->scr_n, c->bufC * 4 * cb) != hipSuccess) {
        hipGetLastError();
        return fail(c, DT_E_CAPACITY, "round buffers for %u insertions do not fit", c->list_cap);
    }
    c->buf_wide = c->wide;
    return DT_OK;
}

int ensure_round_buffers(dt_ctx *c, uint32_t rmax) {
    if (c->list_cap >= rmax && c->cav && c->bufC == (size_t)c->list_cap * c->capC &&
        c->bufF == (size_t)c->list_cap * c->capF && c->buf_wide == c->wide)
        return DT_OK;
    rmax = std::max(rmax, c->list_cap);
    for (int k = 0; k < 4; ++k) {
        dev_free(c, c->lpt[k]);
        dev_free(c, c->lrank[k]);
        c->lpt[k] = c->lrank[k] = nullptr;
    }
    dev_free(c, c->cav); dev_free(c, c->bnd); dev_free(c, c->outc); dev_free(c, c->cnt); dev_free(c, c->status);
    dev_free(c, c->scr_v); dev_free(c, c->scr_n); dev_free(c, c->defer);
    c->defer = nullptr;
    c->scr_v = nullptr;
    c->scr_n = nullptr;
    c->cav = c->outc = nullptr;
    c->bnd = c->cnt = nullptr;
    c->status = nullptr;
    c->list_cap = rmax;
    c->bufC = (size_t)rmax * c->capC;
    c->bufF = (size_t)rmax * c->capF;
    bool ok = true;
    for (int k = 0; k < 4; ++k)
        ok = ok && dev_alloc(c, (void **)&c->lpt[k], rmax * sizeof(uint32_t)) == hipSuccess &&
             dev_alloc(c, (void **)&c->lrank[k], rmax * sizeof(uint32_t)) == hipSuccess;
    // adjacency codes in the cavity and outer lists and the neighbour copies: 4 or 8 bytes
    const size_t cb = c->wide ? sizeof(unsigned long long) : sizeof(uint32_t);
    ok = ok && dev_alloc(c, &c->cav, c->bufC * cb) == hipSuccess &&
         dev_alloc(c, (void **)&c->bnd, c->bufF * sizeof(uint32_t)) == hipSuccess &&
         dev_alloc(c, &c->outc, c->bufF * cb) == hipSuccess &&
         dev_alloc(c, (void **)&c->cnt, 2 * (size_t)rmax * sizeof(uint32_t)) == hipSuccess &&
         dev_alloc(c, (void **)&c->status, rmax) == hipSuccess &&
         dev_alloc(c, (void **)&c->defer, rmax * sizeof(uint32_t)) == hipSuccess &&
         dev_alloc(c, (void **)&c->scr_v, c->bufC * sizeof(uint4)) == hipSuccess &&
         dev_alloc(c, &c->scr_n, c->bufC * 4 * cb) == hipSuccess;
    c->buf_wide = c->wide;
    if (!ok) {
        hipGetLastError();
        c->list_cap = 0;
        return fail(c, DT_E_CAPACITY, "round buffers for %u insertions do not fit", rmax);
    }
    return DT_OK;
}

struct Levels {
    int L = 0;
    std::vector<uint32_t> start, size, bits;  // start: offsets into the level-major order
    std::vector<unsigned long long> rank_base;
    uint64_t total_ranks = 0;
    bool halves = false;  // learned order: level 2k + 1 holds the points of BRIO level k predicted costly
};

// device copies of the level tables live in c->small / c->small64
int upload_levels(dt_ctx *c, const Levels &lv, uint32_t **d_start, uint32_t **d_size, uint32_t **d_bits,
                  unsigned long long **d_rank_base) {
    const int L = lv.L;
    std::vector<uint32_t> packed;
    packed.insert(packed.end(), lv.start.begin(), lv.start.end());  // L + 1
    packed.insert(packed.end(), lv.size.begin(), lv.size.end());    // L
    packed.insert(packed.end(), lv.bits.begin(), lv.bits.end());    // L
    int rc = ensure(c, c->small, packed.size() + 64);
    if (rc) return rc;
    rc = ensure(c, c->small64, (size_t)2 * (L + 1) + 64);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(c->small.p, packed.data(), packed.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                          c->stream));
    HIPCHK(hipMemcpyAsync(c->small64.p, lv.rank_base.data(), (L + 1) * sizeof(unsigned long long),
                          hipMemcpyHostToDevice, c->stream));
    *d_start = c->small.p;
    *d_size = c->small.p + (L + 1);
    *d_bits = c->small.p + (L + 1) + L;
    *d_rank_base = (unsigned long long *)c->small64.p;
    return DT_OK;
}

int grow_tets(dt_ctx *c, uint64_t need);

// launch parameters from the options
void apply_options(dt_ctx *c) {
    c->capC = c->opt.cavity_cap ? c->opt.cavity_cap : DEFAULT_CAVITY_CAP;
    c->lanes = c->opt.lanes_per_insert ? c->opt.lanes_per_insert : DEFAULT_LANES;
    c->lanes_auto = c->opt.lanes_per_insert == 0;
    c->large_lanes = c->opt.large_lanes ? c->opt.large_lanes : DEFAULT_LARGE_LANES;
    c->frac = c->opt.round_fraction > 0 ? c->opt.round_fraction : DEFAULT_ROUND_FRACTION;
    c->frac_auto = !(c->opt.round_fraction > 0);
    c->capF = std::max<uint32_t>(4, (5 * c->capC) / 3);
}

int size_class(uint64_t n) { return n ? 63 - __builtin_clzll(n) : 0; }

// The launch configuration of an insertion of n points: the autotuner's choice for the
// nearest tuned size class (ties to the larger), else the options.
void select_launch(dt_ctx *c, uint64_t n) {
    apply_options(c);
    const int k = size_class(n);
    int best = -1;
    for (int j = 0; j < 64; ++j)
        if (c->tuned[j].set && (best < 0 || std::abs(j - k) < std::abs(best - k) ||
                                (std::abs(j - k) == std::abs(best - k) && j > best)))
            best = j;
    if (best < 0) return;
    const dt_ctx::Tuned &t = c->tuned[best];
    c->lanes = t.lanes ? t.lanes : DEFAULT_LANES;
    c->lanes_auto = t.lanes == 0;
    c->large_lanes = t.large;
    c->capC = t.cap;
    c->frac = t.frac > 0 ? t.frac : DEFAULT_ROUND_FRACTION;
    c->frac_auto = !(t.frac > 0);
    c->capF = std::max<uint32_t>(4, (5 * c->capC) / 3);
}

int check_errors(dt_ctx *c) {
    uint32_t e = c->hctr->error;
    if (e & ERR_POOL) {
        // some insertions found the pool full and will retry: the pool grows before the next
        // round is planned (once no round is in flight)
        HIPCHK(hipMemsetAsync(&c->ctr->error, 0, sizeof(uint32_t), c->stream));
        c->hctr->error &= ~ERR_POOL;
        e &= ~ERR_POOL;
        c->grow_pending = true;
    }
    if (!e) return DT_OK;
    if (e & ERR_CAPACITY) return fail(c, DT_E_CAPACITY, "tetrahedron pool exhausted inside a round");
    if (e & ERR_WALK) return fail(c, DT_E_INTERNAL, "point location or ball construction did not terminate");
    return fail(c, DT_E_INTERNAL, "device error flags 0x%x", e);
}

void accumulate_timing(dt_ctx *c, int slot) {
    if (!c->opt.timing) return;
    const bool ball = c->opt.timing == 1;
    float a = 0.f, b = 0.f;
    if (hipEventSynchronize(c->ev[slot][ball ? 2 : 1]) == hipSuccess &&
        hipEventElapsedTime(&a, c->ev[slot][0], c->ev[slot][1]) == hipSuccess &&
        (!ball || hipEventElapsedTime(&b, c->ev[slot][1], c->ev[slot][2]) == hipSuccess)) {
        c->st.ms_cavity_kernel += a;
        c->st.cavity_launches++;
        if (ball) {
            c->st.ms_ball_kernel += b;
            c->st.ball_launches++;
        }
    } else {
        hipGetLastError();
    }
}

// One round over the candidate list `ci`; losers go to `ni`, overflows to `oi` (slice: the
// candidates are entries off .. off + max_cand of list ci, not the whole list).  The round
// is launched with the copy of its counters into a free snapshot slot (neither the host's
// nor one still in flight); complete_round waits for it.  max_cand bounds the candidates:
// the kernels read the count itself from the device.
int enqueue_round(dt_ctx *c, int ci, int ni, int oi, uint32_t max_cand, uint32_t capC, uint32_t capF,
                  uint64_t base, uint64_t n, int busy, int *slot_out, bool slice = false, uint32_t off = 0,
                  const FillPlan *plan = nullptr, const FillArgs *fa = nullptr) {
    const int host = (int)(c->hctr - c->hring);
    int slot = 0;
    while (slot == host || slot == busy) ++slot;
    Ctr *d = c->ctr;
    RoundArgs a{};
    a.V = c->V.p;
    a.T = c->T;
    a.scr_v = c->scr_v;
    a.scr_n = c->scr_n;
    a.vtet = c->vtet.p;
    a.vlo = (uint32_t)base;
    a.vhi = (uint32_t)(base + n);
    a.anchor = c->anchor.p;
    a.lastt = c->lastt.p;
    a.multi = c->call_clouds > 1 ? 1u : 0u;
    a.walk_cap = c->opt.walk_cap ? c->opt.walk_cap : DEFAULT_WALK_CAP;
    a.clouds = c->clouds.p;
    a.log_att = c->logged ? c->log_att.p : nullptr;
    a.wbucket = c->learned_active ? c->wbucket.p : nullptr;
    a.cand_pt = c->lpt[ci] + off;
    a.cand_rank = c->lrank[ci] + off;
    a.next_pt = c->lpt[ni];
    a.next_rank = c->lrank[ni];
    a.ovf_pt = c->lpt[oi];
    a.ovf_rank = c->lrank[oi];
    a.ncand_ptr = &d->list_count[ci];
    if (slice) {
        c->hctr->chunk = max_cand;
        HIPCHK(hipMemcpyAsync(&d->chunk, &c->hctr->chunk, sizeof(uint32_t), hipMemcpyHostToDevice, c->stream));
        a.ncand_ptr = &d->chunk;
    }
    a.nnext_ptr = &d->list_count[ni];
    a.novf_ptr = &d->list_count[oi];
    a.defer = c->defer;
    a.ndefer_ptr = &d->ndefer;
    a.subd = c->subd;
    a.cav = c->cav;
    a.bnd = c->bnd;
    a.outc = c->outc;
    a.cnt = c->cnt;
    a.status = c->status;
    a.fl_cur = c->fl[c->fl_idx];
    a.fl_next = c->fl[c->fl_idx ^ 1];
    a.flcap = c->flcap;
    a.ctr = d;
    a.stat = c->stat;
    a.stride = std::max<uint32_t>(max_cand, 1);
    a.capC = capC;
    a.capF = capF;
    a.tcap = c->tcap;
    // the global cavity set of the largest cavities: a power of two of entries in the
    // candidate's 16 capC bytes of ball scratch (4-byte entries, or 8-byte with 64-bit codes)
    a.hmg = 1u << (31 - __builtin_clz(std::min<uint32_t>((c->wide ? 2u : 4u) * std::min<uint32_t>(capC, 1u << 24),
                                                         1u << 30)));
    // Claim words are never reset between rounds: later rounds stamp lower.  When the low 32
    // bits of the round counter wrap, every claim left in the pool would outrank the new
    // stamps, so the claim words are reset to the empty value first (the kernels of earlier
    // rounds are ahead of the reset on the same stream).
    if ((c->round_counter & 0xFFFFFFFFull) == 0 && c->round_counter != 0 && c->tcap)
        HIPCHK(launch_reset_claims(c->T, c->wide, c->tcap, c->stream));
    a.round_hi = (0xFFFFFFFFull - (c->round_counter & 0xFFFFFFFFull)) << 32;
    a.clk = nullptr;
    if (c->trace >= 2 && max_cand) {
        if (c->clk_cap[slot] < max_cand) {
            if (c->clk[slot]) hipFree(c->clk[slot]);
            c->clk[slot] = nullptr;
            c->clk_cap[slot] = 0;
            HIPCHK(hipMalloc((void **)&c->clk[slot], 8ull * max_cand * sizeof(unsigned long long)));
            c->clk_cap[slot] = max_cand;
        }
        HIPCHK(hipMemsetAsync(c->clk[slot], 0, 8ull * max_cand * sizeof(unsigned long long), c->stream));
        a.clk = c->clk[slot];
    }
    c->round_counter++;
    // timing 1: events around both kernels in every round; 2: around the cavity kernel in
    // rounds of at least SMALL_ROUND candidates (each event record leaves the GPU idle for a
    // few microseconds, which the short rounds would feel most)
    hipEvent_t evs[3] = {c->ev[slot][0], c->ev[slot][1], c->opt.timing == 1 ? c->ev[slot][2] : nullptr};
    const bool timed = c->opt.timing == 1 || (c->opt.timing == 2 && max_cand >= SMALL_ROUND);
    c->slot_timed[slot] = timed;
    // automatic lanes: a wavefront per insertion in short rounds, which wait on their slowest
    // candidate, c->lanes in the rest
    const uint32_t lanes = c->lanes_auto && max_cand < SMALL_ROUND ? 64u : c->lanes;
    // graph-launched: regular rounds with the snapshot written by the round-end kernel,
    // neither timed nor clocked (their events and clearing stay outside graphs)
    const bool graph = c->opt.graph_rounds && c->ring_direct && !slice && !timed && !a.clk && max_cand &&
                       capC <= DEFAULT_CAVITY_CAP;
    if (graph) {
        const FillPlan none{};
        const FillArgs nofill{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                              nullptr, nullptr, &d->list_count[ci]};
        c->fl_idx ^= 1;
        c->slot_tag[slot] = ++c->tag_counter;
        HIPCHK(launch_round_graph(c->graphs, plan ? *plan : none, fa ? *fa : nofill, a, c->wide, max_cand, lanes,
                                  &c->hring[slot], &c->hseq[slot], c->slot_tag[slot], c->stream));
        c->slot_cand[slot] = max_cand;
        c->slot_capC[slot] = capC;
        c->st.rounds++;
        c->st.graph_rounds++;
        *slot_out = slot;
        return DT_OK;
    }
    if (plan)
        HIPCHK(launch_fill_list(*plan, fa->lvl_start, fa->lvl_size, fa->lvl_bits, fa->rank_base, fa->lord, fa->dup,
                                fa->vtet, fa->cand_pt, fa->cand_rank, fa->ncand, c->stream));
    HIPCHK(launch_round(a, c->wide, max_cand, lanes, c->large_lanes, c->exact_needed, c->stream,
                        timed ? evs : nullptr));
    c->fl_idx ^= 1;
    if (c->ring_direct) {
        c->slot_tag[slot] = ++c->tag_counter;
        HIPCHK(launch_round_end(a, max_cand, c->stream, &c->hring[slot], &c->hseq[slot], c->slot_tag[slot]));
    } else {
        HIPCHK(launch_round_end(a, max_cand, c->stream, nullptr, nullptr, 0));
        HIPCHK(hipMemcpyAsync(&c->hring[slot], c->ctr, sizeof(Ctr), hipMemcpyDeviceToHost, c->stream));
        if (c->evdone[slot]) HIPCHK(hipEventRecord(c->evdone[slot], c->stream));
    }
    c->slot_cand[slot] = max_cand;
    c->slot_capC[slot] = capC;
    c->st.rounds++;
    *slot_out = slot;
    return DT_OK;
}

// Trace mode 2: the filter pass's per-attempt clocks of the round in `slot` (10 ns ticks),
// summarised on stderr as quantiles of the walk, cavity and whole-attempt durations, the
// launch span (first start to last end) and the mean walk and cavity steps.
void trace_clocks(dt_ctx *c, int slot, uint32_t max_cand) {
    std::vector<unsigned long long> &h = c->clk_host;
    h.resize(8ull * max_cand);
    if (hipMemcpy(h.data(), c->clk[slot], h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost) !=
        hipSuccess) {
        hipGetLastError();
        return;
    }
    std::vector<double> walk, cav, att;
    unsigned long long lo = ~0ull, hi = 0;
    double ws = 0, cs = 0;
    std::vector<double> test, copy, build, ball;
    unsigned long long blo = ~0ull, bhi = 0;
    for (uint32_t i = 0; i < max_cand; ++i) {
        const unsigned long long *b = &h[8ull * i + 4];
        if (b[0] && b[1] >= b[0]) {
            test.push_back(0.01 * (double)(b[1] - b[0]));
            blo = std::min(blo, b[0]);
            bhi = std::max(bhi, b[1]);
            if (b[2] >= b[1] && b[3] >= b[2] && b[3]) {
                copy.push_back(0.01 * (double)(b[2] - b[1]));
                build.push_back(0.01 * (double)(b[3] - b[2]));
                ball.push_back(0.01 * (double)(b[3] - b[0]));
                bhi = std::max(bhi, b[3]);
            }
        }
    }
    for (uint32_t i = 0; i < max_cand; ++i) {
        const unsigned long long *r = &h[8ull * i];
        if (r[0] == 0 || r[2] < r[0] || r[1] < r[0]) continue;  // not run (slot of a shorter list)
        walk.push_back(0.01 * (double)(r[1] - r[0]));
        cav.push_back(0.01 * (double)(r[2] - r[1]));
        att.push_back(0.01 * (double)(r[2] - r[0]));
        lo = std::min(lo, r[0]);
        hi = std::max(hi, r[2]);
        ws += (double)(r[3] & 0xFFFFu);
        cs += (double)((r[3] >> 16) & 0xFFFFu);
    }
    if (att.empty()) return;
    auto q = [](std::vector<double> &v, double f) {
        const size_t k = std::min(v.size() - 1, (size_t)(f * (double)(v.size() - 1)));
        std::nth_element(v.begin(), v.begin() + k, v.end());
        return v[k];
    };
    const double n = (double)att.size();
    fprintf(stderr,
            "clocks n=%zu span_us=%.2f walk_us=%.2f/%.2f/%.2f cav_us=%.2f/%.2f/%.2f att_us=%.2f/%.2f/%.2f/%.2f "
            "walk_steps=%.2f cav_steps=%.2f\n",
            att.size(), 0.01 * (double)(hi - lo), q(walk, 0.5), q(walk, 0.9), q(walk, 1.0), q(cav, 0.5), q(cav, 0.9),
            q(cav, 1.0), q(att, 0.5), q(att, 0.9), q(att, 0.99), q(att, 1.0), ws / n, cs / n);
    if (!ball.empty())
        fprintf(stderr,
                "ballclocks n=%zu built=%zu span_us=%.2f test_us=%.2f/%.2f/%.2f copy_us=%.2f/%.2f/%.2f "
                "build_us=%.2f/%.2f/%.2f ball_us=%.2f/%.2f/%.2f/%.2f\n",
                test.size(), ball.size(), 0.01 * (double)(bhi - blo), q(test, 0.5), q(test, 0.9), q(test, 1.0),
                q(copy, 0.5), q(copy, 0.9), q(copy, 1.0), q(build, 0.5), q(build, 0.9), q(build, 1.0), q(ball, 0.5),
                q(ball, 0.9), q(ball, 0.99), q(ball, 1.0));
}

// Waits for the round whose counters go to `slot`; they become the host's snapshot.
int complete_round(dt_ctx *c, int slot) {
    if (c->ring_direct) {
        // the round-end kernel sets the slot's tag after writing its snapshot; the stream is
        // queried now and then so that a failed launch ends the wait
        const volatile unsigned long long *seq = &c->hseq[slot];
        const unsigned long long want = c->slot_tag[slot];
        for (uint64_t spin = 1; *seq != want; ++spin) {
            if ((spin & 4095) == 0) {
                const hipError_t e = hipStreamQuery(c->stream);
                if (e == hipSuccess && *seq != want)
                    return fail(c, DT_E_INTERNAL, "round counters did not arrive (stream idle)");
                if (e != hipSuccess && e != hipErrorNotReady) {
                    hipGetLastError();
                    return fail(c, DT_E_DEVICE, "device error while waiting for a round (%s)", hipGetErrorString(e));
                }
            }
        }
        std::atomic_thread_fence(std::memory_order_acquire);
    } else if (c->evdone[slot]) {
        HIPCHK(hipEventSynchronize(c->evdone[slot]));
    } else {
        // without events (the arena's context) the whole stream is waited for: the round in
        // flight behind this one completes too, which is correct, only not overlapped
        HIPCHK(hipStreamSynchronize(c->stream));
    }
    const uint32_t won_before = c->hctr->won;
    const unsigned long long att_before = c->hctr->attempts;
    c->hctr = &c->hring[slot];
    // from the first attempt the filter handed on, every later round of the call runs the
    // exact pass (the rounds launched before it was seen retry theirs)
    if (c->hctr->deferred != c->deferred_base) c->exact_needed = true;
    const uint32_t max_cand = c->slot_cand[slot], capC = c->slot_capC[slot];
    if (max_cand && c->slot_timed[slot]) {
        accumulate_timing(c, slot);
        c->st.timed_insertions += c->hctr->won - won_before;
        c->st.timed_attempts += c->hctr->attempts - att_before;
    }
    if (c->trace) {
        uint32_t &prev_won = c->trace_prev_won;
        if (prev_won > c->hctr->won) {
            prev_won = c->trace_prev_conf = c->trace_prev_ovf = 0;
            c->trace_prev_att = c->trace_prev_walk = c->trace_prev_cav = c->trace_prev_ins = 0;
            c->trace_rounds = 0;
        }
        float ta = 0.f, tb = 0.f;
        if (c->opt.timing && max_cand) {
            if (c->slot_timed[slot]) hipEventElapsedTime(&ta, c->ev[slot][0], c->ev[slot][1]);
            if (c->opt.timing == 1) hipEventElapsedTime(&tb, c->ev[slot][1], c->ev[slot][2]);
        }
        fprintf(stderr,
                "round %llu cand<=%u won=%u tets=%u free=%u cavity_ms=%.3f ball_ms=%.3f att=%llu walk=%llu "
                "conf=%u ovf=%u capC=%u cavw=%llu insph=%llu\n",
                (unsigned long long)++c->trace_rounds, max_cand, c->hctr->won - prev_won, c->hctr->tet_count, c->hctr->fl_n, ta, tb,
                c->hctr->attempts - c->trace_prev_att, c->hctr->walk_steps - c->trace_prev_walk,
                c->hctr->conflicts - c->trace_prev_conf, c->hctr->overflows - c->trace_prev_ovf, capC,
                c->hctr->cav_tets - c->trace_prev_cav, c->hctr->insphere - c->trace_prev_ins);
        prev_won = c->hctr->won;
        if (c->trace >= 2 && max_cand && c->clk[slot] && c->clk_cap[slot] >= max_cand) trace_clocks(c, slot, max_cand);
        c->trace_prev_att = c->hctr->attempts;
        c->trace_prev_walk = c->hctr->walk_steps;
        c->trace_prev_conf = c->hctr->conflicts;
        c->trace_prev_ovf = c->hctr->overflows;
        c->trace_prev_cav = c->hctr->cav_tets;
        c->trace_prev_ins = c->hctr->insphere;
    }
    return check_errors(c);
}

// grows the pool when a round found it full (no round may be in flight)
int grow_if_pending(dt_ctx *c) {
    if (!c->grow_pending) return DT_OK;
    c->grow_pending = false;
    return grow_tets(c, (uint64_t)c->tcap + c->tcap / 2 + 4096);
}

// one round, waited for
int run_one_round(dt_ctx *c, int ci, int ni, int oi, uint32_t max_cand, uint32_t capC, uint32_t capF,
                  uint64_t base, uint64_t n, bool slice = false, uint32_t off = 0) {
    int slot = -1;
    int rc = enqueue_round(c, ci, ni, oi, max_cand, capC, capF, base, n, -1, &slot, slice, off);
    if (rc) return rc;
    if ((rc = complete_round(c, slot))) return rc;
    return grow_if_pending(c);
}

// Grow the pool ahead of a round when the expected consumption would not fit; an
// insertion that still finds the pool full retries in the next round.
int ensure_capacity_for(dt_ctx *c, uint32_t max_cand, uint32_t capF) {
    const uint64_t per = std::min<uint64_t>(capF, 48);
    uint64_t need = (uint64_t)c->hctr->tet_count + (uint64_t)max_cand * per + 16;
    if (need <= c->tcap) return DT_OK;
    return grow_tets(c, need + need / 8);
}

// Rounds for candidates whose cavities overflowed, in slices of the list in which each
// insertion gets `need` buffer entries (first 1024, the wave-per-insertion kernel with its
// queue in LDS, then the same kernel with queue and set in global memory); `need` grows
// after a pass over the list that inserts nothing or fewer points than overflow.  Large
// cavities of nearby points overlap, so few of them win per round however many are tried:
// a slice holds at most DRAIN_SLICE consecutive entries of the list (taking entries far
// apart on the curve instead measured slower: more of them overflow or conflict).
int drain_overflow(dt_ctx *c, uint64_t base, uint64_t n) {
    size_t need = std::max<size_t>(4 * (size_t)c->capC, 1024);
    while (c->hctr->list_count[2 + c->ovf_idx] > 0) {
        const int ci = 2 + c->ovf_idx, ni = 2 + (c->ovf_idx ^ 1);
        const uint32_t cnt = c->hctr->list_count[ci];
        const uint32_t chunk =
            (uint32_t)std::max<size_t>(1, std::min<size_t>(std::min<size_t>(cnt, DRAIN_SLICE), c->bufC / need));
        const uint32_t capC = (uint32_t)std::min<size_t>(std::min(c->bufC / chunk, need), 1u << 24);
        const uint32_t capF = (uint32_t)std::min<size_t>(std::min(c->bufF / chunk, 2 * need), 1u << 24);
        const uint32_t won0 = c->hctr->won, ovf0 = c->hctr->overflows;
        for (uint32_t off = 0; off < cnt; off += chunk) {
            const uint32_t k = std::min(chunk, cnt - off);
            int rc = ensure_capacity_for(c, k, capF);
            if (rc) return rc;
            const uint32_t w0 = c->hctr->won;
            rc = run_one_round(c, ci, ni, ni, k, capC, capF, base, n, true, off);
            if (rc) return rc;
            c->mesh_vertices += c->hctr->won - w0;
        }
        // list ci is consumed; its losers and overflows are in list ni
        HIPCHK(hipMemsetAsync(&c->ctr->list_count[ci], 0, sizeof(uint32_t), c->stream));
        c->hctr->list_count[ci] = 0;
        c->ovf_idx ^= 1;
        if (c->hctr->won == won0) {
            if (chunk == 1 && need >= c->bufC)  // the whole buffer did not hold one cavity
                return fail(c, DT_E_CAPACITY, "a cavity exceeds the per-insertion buffer (%u tetrahedra)", capC);
            need *= 4;
        } else if (c->hctr->overflows - ovf0 >= c->hctr->won - won0 && need < c->bufC) {
            // more overflows than insertions: retrying them at this size wastes rounds, and
            // their claims block the neighbouring candidates
            need *= 4;
        }
    }
    return DT_OK;
}

// Splits ranks [first, first + W) into at most FILL_BLOCKS aligned power-of-two blocks within
// levels; returns the number of ranks covered (W or fewer).
uint64_t plan_fill(const Levels &lv, uint64_t first, uint64_t W, FillPlan &plan) {
    plan.nblk = 0;
    uint32_t total = 0;
    uint64_t r = first;
    const uint64_t end = first + W;
    while (r < end && plan.nblk < (uint32_t)FILL_BLOCKS) {
        int k = 0;
        while (k + 1 < lv.L && lv.rank_base[k + 1] <= r) ++k;
        const uint64_t lend = std::min<uint64_t>(end, lv.rank_base[k + 1]);
        uint64_t a = r - lv.rank_base[k];
        const uint64_t b = lend - lv.rank_base[k];
        while (a < b && plan.nblk < (uint32_t)FILL_BLOCKS) {
            int w = 31;
            if (a) w = std::min(w, __builtin_ctzll(a));
            while ((1ull << w) > b - a) --w;
            plan.lvl[plan.nblk] = (uint32_t)k;
            plan.a[plan.nblk] = (uint32_t)a;
            plan.w[plan.nblk] = (uint32_t)w;
            plan.off[plan.nblk] = total;
            total += 1u << w;
            a += 1ull << w;
            ++plan.nblk;
        }
        r = lv.rank_base[k] + a;
    }
    plan.off[plan.nblk] = total;
    return r - first;
}

// The rounds of one call.  While new ranks remain, a round is planned and launched while
// the previous one still runs: its size comes from the last completed round's counters,
// with the running round's candidates as the bound on the losers that open the next list
// (the kernels read the exact count on the device), so the GPU does not wait for the host
// between rounds.  Drains, pool growth, the last rounds and anything the bounds cannot
// guarantee run one round at a time.
int run_rounds(dt_ctx *c, const Levels &lv, const uint32_t *d_start, const uint32_t *d_size,
               const uint32_t *d_bits, const unsigned long long *d_rank_base, uint64_t base, uint64_t n) {
    const uint32_t rmax = c->list_cap;
    const double frac = c->frac;
    uint64_t next_rank = 0;
    uint64_t rounds_this_call = 0;
    int fly = -1;            // snapshot slot of the round in flight, or -1
    uint32_t fly_cand = 0;   // its candidates (exact)
    double loss = 0.5;       // share of candidates lost by the last completed round
    uint32_t won_seen = c->hctr->won;
    auto target_size = [&]() {
        double f = frac;
        if (lv.halves && next_rank < lv.total_ranks) {
            // the points predicted costly conflict more: fewer of them per round
            int k = 0;
            while (k + 1 < lv.L && lv.rank_base[k + 1] <= next_rank) ++k;
            if (k & 1) f *= c->costly_scale;
        }
        uint64_t t = (uint64_t)std::llround(f * (double)c->mesh_vertices);
        // automatic fraction: short rounds, which last as long as their slowest insertion
        // whatever their size, take a larger share (up to SMALL_ROUND candidates)
        if (c->frac_auto && t < SMALL_ROUND)
            t = std::min<uint64_t>(SMALL_ROUND, (uint64_t)std::llround(f * SHORT_ROUND_FRACTION_SCALE *
                                                                     (double)c->mesh_vertices));
        if (c->opt.round_size) return std::min<uint64_t>(c->opt.round_size, rmax);
        return std::min<uint64_t>(std::max<uint64_t>(t, ROUND_MIN), rmax);
    };
    // completes the round in flight: mesh size, loss share (a pool growth it asks for waits
    // until no round is in flight)
    auto land = [&]() -> int {
        int rc = complete_round(c, fly);
        if (rc) return rc;
        const uint32_t won = c->hctr->won - won_seen;
        won_seen = c->hctr->won;
        c->mesh_vertices += won;
        if (fly_cand) loss = 1.0 - (double)won / (double)fly_cand;
        fly = -1;
        return DT_OK;
    };
    for (;;) {
        const int ci = c->list_idx, ni = ci ^ 1, oi = 2 + c->ovf_idx;
        if (c->grow_pending) {
            int rc = fly >= 0 ? land() : grow_if_pending(c);
            if (rc) return rc;
            continue;
        }
        if (fly >= 0) {
            // plan the next round while the previous one runs
            const uint64_t est = (uint64_t)std::llround(loss * (double)fly_cand);
            const uint64_t target = target_size();
            uint64_t W = 0;
            if (next_rank < lv.total_ranks && target > est)
                W = std::min<uint64_t>(target - est, lv.total_ranks - next_rank);
            W = std::min<uint64_t>(W, rmax - fly_cand);
            const uint64_t per = std::min<uint64_t>(c->capF, 48);
            const uint64_t bound = fly_cand + W;
            const bool ok = W > 0 && (!c->opt.max_rounds || rounds_this_call < c->opt.max_rounds) &&
                            (uint64_t)c->hctr->list_count[oi] + fly_cand + bound <= rmax &&
                            (uint64_t)c->hctr->tet_count + (fly_cand + bound) * per + 16 <= c->tcap;
            if (ok) {
                FillPlan plan;
                const uint32_t w = (uint32_t)plan_fill(lv, next_rank, W, plan);
                const FillArgs fa{d_start, d_size, d_bits, d_rank_base, c->lord, c->dup.p, c->vtet.p,
                                  c->lpt[ci], c->lrank[ci], &c->ctr->list_count[ci]};
                next_rank += w;
                int slot = -1;
                int rc = enqueue_round(c, ci, ni, oi, fly_cand + w, c->capC, c->capF, base, n, fly, &slot, false, 0,
                                       &plan, &fa);
                if (rc) return rc;
                c->list_idx = ni;
                ++rounds_this_call;
                if ((rc = land())) return rc;  // the previous round; its losers open this one
                fly = slot;
                fly_cand = c->hctr->list_count[ci] + w;
                continue;
            }
            int rc = land();
            if (rc) return rc;
            continue;
        }
        // one round at a time, from exact counts
        const uint32_t nl = c->hctr->list_count[ci];
        const uint64_t target = target_size();
        uint32_t W = 0;
        if (next_rank < lv.total_ranks && target > nl)
            W = (uint32_t)std::min<uint64_t>(target - nl, lv.total_ranks - next_rank);
        if (nl == 0 && W == 0) {
            if (c->hctr->list_count[oi] == 0) break;
            int rc = drain_overflow(c, base, n);
            if (rc) return rc;
            won_seen = c->hctr->won;
            continue;
        }
        // overflowed candidates wait until the regular lists are done (by then their
        // neighbourhoods are filled in and their cavities are smaller), or until their
        // list could not take another round's worth
        if (c->hctr->list_count[oi] + nl + W > rmax) {
            int rc = drain_overflow(c, base, n);
            if (rc) return rc;
            won_seen = c->hctr->won;
            continue;
        }
        if (c->opt.max_rounds && rounds_this_call >= c->opt.max_rounds)
            return fail(c, DT_E_INCOMPLETE, "round limit %u reached", c->opt.max_rounds);
        FillPlan plan;
        W = (uint32_t)plan_fill(lv, next_rank, W, plan);
        const FillArgs fa{d_start, d_size, d_bits, d_rank_base, c->lord, c->dup.p, c->vtet.p,
                          c->lpt[ci], c->lrank[ci], &c->ctr->list_count[ci]};
        next_rank += W;
        const uint32_t max_cand = nl + W;
        int rc = ensure_capacity_for(c, max_cand, c->capF);
        if (rc) return rc;
        rc = enqueue_round(c, ci, ni, oi, max_cand, c->capC, c->capF, base, n, -1, &fly, false, 0, &plan, &fa);
        if (rc) return rc;
        fly_cand = max_cand;
        c->list_idx = ni;
        ++rounds_this_call;
    }
    return DT_OK;
}

void compute_levels(const std::vector<uint32_t> &hist, int L, Levels &lv) {
    lv.L = L;
    lv.start.assign(L + 1, 0);
    lv.size.assign(L, 0);
    lv.bits.assign(L, 0);
    lv.rank_base.assign(L + 1, 0);
    uint64_t acc = 0;
    for (int k = 0; k < L; ++k) {
        lv.start[k] = (uint32_t)acc;
        lv.size[k] = hist[k];
        acc += hist[k];
        uint32_t b = 0;
        while ((1ull << b) < hist[k]) ++b;
        lv.bits[k] = b;
        lv.rank_base[k + 1] = lv.rank_base[k] + (1ull << b);
    }
    lv.start[L] = (uint32_t)acc;
    lv.total_ranks = lv.rank_base[L];
}

// Clouds of one call: cloud k holds input points [off[k], off[k+1]) and vertex records
// [base + off[k], base + off[k+1]).  Uploads the offsets and the chunk table of the box
// reduction; writes the cloud table (all fields when fresh; otherwise only the record range
// and Moore level, so that the cloud's live tetrahedron survives an append).
int prepare_clouds(dt_ctx *c, const std::vector<uint64_t> &off, uint64_t base, bool fresh, int *mmax,
                   uint32_t *nchunks, DevBuf<Cloud> &clouds) {
    const uint32_t C = (uint32_t)(off.size() - 1);
    constexpr uint64_t CHUNK = 65536;
    std::vector<uint64_t> cs, ce;
    std::vector<uint32_t> cch(C + 1, 0);
    std::vector<Cloud> h(C);
    *mmax = 1;
    // adaptive curve: the deepest grid the key holds beside the cloud id, so that points
    // sharing a cell of the fixed level are ordered by the curve's deeper levels too
    int cb = 0;
    while ((1ull << cb) < C) ++cb;
    const uint32_t m_adaptive = (uint32_t)std::min(21, (64 - cb) / 3);
    for (uint32_t k = 0; k < C; ++k) {
        cch[k] = (uint32_t)cs.size();
        for (uint64_t b = off[k]; b < off[k + 1]; b += CHUNK) {
            cs.push_back(b);
            ce.push_back(std::min(off[k + 1], b + CHUNK));
        }
        const uint64_t nk = off[k + 1] - off[k];
        std::memset(&h[k], 0, sizeof(Cloud));
        h[k].lo = (uint32_t)(base + off[k]);
        h[k].hi = (uint32_t)(base + off[k + 1]);
        h[k].m = c->opt.adaptive_curve ? m_adaptive : (uint32_t)moore_level(nk);
        *mmax = std::max(*mmax, (int)h[k].m);
    }
    cch[C] = (uint32_t)cs.size();
    *nchunks = (uint32_t)cs.size();
    int rc;
    if ((rc = ensure(c, clouds, C)) || (rc = ensure(c, c->off, C + 1)) ||
        (rc = ensure(c, c->ch_start, cs.size() + 1)) || (rc = ensure(c, c->ch_end, cs.size() + 1)) ||
        (rc = ensure(c, c->cloud_ch, C + 1)) || (rc = ensure(c, c->partial, 6 * cs.size() + 6)))
        return rc;
    HIPCHK(hipMemcpyAsync(c->off.p, off.data(), (C + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->ch_start.p, cs.data(), cs.size() * sizeof(uint64_t), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->ch_end.p, ce.data(), ce.size() * sizeof(uint64_t), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->cloud_ch.p, cch.data(), (C + 1) * sizeof(uint32_t), hipMemcpyHostToDevice, c->stream));
    if (fresh) {
        HIPCHK(hipMemcpyAsync(clouds.p, h.data(), C * sizeof(Cloud), hipMemcpyHostToDevice, c->stream));
    } else {
        for (uint32_t k = 0; k < C; ++k) {
            HIPCHK(hipMemcpyAsync(&clouds.p[k].lo, &h[k].lo, 2 * sizeof(uint32_t), hipMemcpyHostToDevice, c->stream));
            HIPCHK(hipMemcpyAsync(&clouds.p[k].m, &h[k].m, sizeof(uint32_t), hipMemcpyHostToDevice, c->stream));
        }
    }
    // the host vectors are pageable: finish the copies before they go out of scope
    HIPCHK(hipStreamSynchronize(c->stream));
    return DT_OK;
}

// Validation, per-cloud boxes, (cloud, Moore) keys and their radix sort.  *svals receives,
// for each position of the curve order, the point's index within the call; *skeys the
// sorted keys (cloud << 3 mmax | Moore index).
int sort_points(dt_ctx *c, const double *dxyz, uint64_t n, Cloud *clouds, const uint64_t *d_off, uint32_t C,
                uint32_t nchunks, int mmax, uint32_t **svals, unsigned long long **skeys, bool *bad_input) {
    *bad_input = false;
    int cb = 0;
    while ((1ull << cb) < C) ++cb;
    int rc;
    if ((rc = ensure(c, c->keys, n)) || (rc = ensure(c, c->keys_tmp, n)) || (rc = ensure(c, c->vals, n)) ||
        (rc = ensure(c, c->vals_tmp, n)) || (rc = ensure(c, c->hist, radix_hist_entries(n))) ||
        (rc = ensure(c, c->scan_tmp, scan_tmp_entries(radix_hist_entries(n)) + scan_tmp_entries(n) + 64)) ||
        (rc = ensure(c, c->small64, 256)) || (rc = ensure(c, c->small, 256)))
        return rc;
    HIPCHK(hipMemsetAsync(&c->ctr->error, 0, sizeof(uint32_t), c->stream));
    HIPCHK(launch_cloud_bbox(dxyz, c->ch_start.p, c->ch_end.p, nchunks, c->partial.p, c->cloud_ch.p, C, clouds,
                             &c->ctr->error, c->stream));
    int r = sync_ctr(c);
    if (r) return r;
    if (c->hctr->error & ERR_INPUT) {
        *bad_input = true;
        return DT_OK;
    }
    HIPCHK(launch_keys(dxyz, n, d_off, C, clouds, 3 * mmax, c->keys.p, c->vals.p, c->stream));
    bool swapped = false;
    HIPCHK(radix_sort_pairs(c->keys.p, c->vals.p, c->keys_tmp.p, c->vals_tmp.p, c->hist.p, c->scan_tmp.p, n,
                            cb + 3 * mmax, c->stream, &swapped));
    *svals = swapped ? c->vals_tmp.p : c->vals.p;
    *skeys = swapped ? c->keys_tmp.p : c->keys.p;
    return DT_OK;
}

// BRIO level of every curve-ordered record within its cloud and the stable level-major order
// of the records (base + i) in *lord; the level sizes go to hist_host (asynchronously; the
// caller synchronizes).  svals and the key buffers are consumed.
int level_order(dt_ctx *c, uint32_t *svals, const Vert *V, uint64_t n, uint64_t base, const uint64_t *d_off,
                const Cloud *clouds, int L, uint32_t **lord, uint32_t *hist_host, uint8_t *lev_out) {
    uint32_t *other = (svals == c->vals.p) ? c->vals_tmp.p : c->vals.p;
    const uint64_t salt = host_mix64(c->opt.seed ^ 0x5851F42D4C957F2Dull);
    HIPCHK(launch_levels(svals, V, n, base, d_off, clouds, salt, c->keys.p, other, lev_out, c->stream));
    int lbits = 0;
    while ((1 << lbits) < L) ++lbits;
    bool swapped = false;
    HIPCHK(radix_sort_pairs(c->keys.p, other, c->keys_tmp.p, svals, c->hist.p, c->scan_tmp.p, n, lbits, c->stream,
                            &swapped));
    *lord = swapped ? svals : other;
    HIPCHK(hipMemsetAsync(c->small.p, 0, 64 * sizeof(uint32_t), c->stream));
    HIPCHK(launch_level_hist(c->keys.p, n, 0, c->small.p, c->stream));
    HIPCHK(hipMemcpyAsync(hist_host, c->small.p, 64 * sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
    return DT_OK;
}

// Inserts the n points at xyz, split into clouds by off (C + 1 offsets, off[0] = 0).
// hint (device, optional, one entry per input point of a single cloud): a vertex record
// near the point, where its walk starts (its anchor)
int insert_clouds(dt_ctx *c, const double *xyz, uint64_t n, const std::vector<uint64_t> &off,
                  const uint32_t *hint = nullptr) {
    const uint32_t C = (uint32_t)(off.size() - 1);
    auto t0 = std::chrono::steady_clock::now();
    HIPCHK(hipSetDevice(c->device));
    int rc;
    const double *dxyz = xyz;
    if (!is_device_ptr(xyz)) {
        if ((rc = ensure(c, c->staging, 3 * n))) return rc;
        HIPCHK(hipMemcpyAsync(c->staging.p, xyz, 3 * n * sizeof(double), hipMemcpyHostToDevice, c->stream));
        dxyz = c->staging.p;
    }
    const uint64_t base = c->nv;
    const bool fresh = !c->have_mesh;
    select_launch(c, n);
    if ((rc = ensure(c, c->V, base + n, true)) || (rc = ensure(c, c->vtet, base + n, true)) ||
        (rc = ensure(c, c->dup, base + n, true)) || (rc = ensure(c, c->anchor, n)) || (rc = ensure(c, c->lastt, n)))
        return rc;
    c->out_index = false;
    // 1-2. clouds, validation, boxes, keys, sort
    int mmax = 1;
    uint32_t nchunks = 0;
    if ((rc = prepare_clouds(c, off, base, fresh, &mmax, &nchunks, c->clouds))) return rc;
    int cb = 0;
    while ((1ull << cb) < C) ++cb;
    if (cb + 3 * mmax > 64) return fail(c, DT_E_ARG, "too many clouds for the key width (%u clouds)", C);
    uint32_t *svals = nullptr;
    unsigned long long *skeys = nullptr;
    bool bad = false;
    if ((rc = sort_points(c, dxyz, n, c->clouds.p, c->off.p, C, nchunks, mmax, &svals, &skeys, &bad))) return rc;
    if (bad) return fail(c, DT_E_INPUT, "a coordinate is not finite or outside 0 or [2^-120, 2^120) in magnitude");
    // 3. vertex records in curve order (cloud id in the upper half of idx)
    HIPCHK(launch_permute(dxyz, svals, skeys, 3 * mmax, n, base, c->npoints, c->V.p, c->vtet.p, c->dup.p, c->stream));
    // 4. BRIO levels per cloud: level-major order of the records and level sizes
    int L = 1;
    for (uint32_t k = 0; k < C; ++k) L = std::max(L, (int)brio_cum(off[k + 1] - off[k]).size());
    std::vector<uint32_t> hist(64);
    uint32_t *lord = nullptr;
    if ((rc = ensure(c, c->lev, n))) return rc;
    if ((rc = level_order(c, svals, c->V.p, n, base, c->off.p, c->clouds.p, L, &lord, hist.data(), c->lev.p)))
        return rc;
    // 5. duplicates (within each cloud)
    uint64_t tsize = 1;
    while (tsize < 2 * n) tsize <<= 1;
    if ((rc = ensure(c, c->table, tsize))) return rc;
    HIPCHK(hipMemsetAsync(&c->ctr->dups, 0, sizeof(uint32_t), c->stream));
    HIPCHK(launch_dedupe(c->V.p, base, n, c->table.p, tsize, c->dup.p, &c->ctr->dups, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    Levels lv;
    compute_levels(hist, L, lv);
    // 6. level tables, walk anchors and (learned scheduler) the learned order
    uint32_t *d_start, *d_size, *d_bits;
    unsigned long long *d_rb;
    if ((rc = upload_levels(c, lv, &d_start, &d_size, &d_bits, &d_rb))) return rc;
    HIPCHK(launch_anchor(lord, d_start, L, c->V.p, base, n, c->anchor.p, c->stream));
    if (hint) HIPCHK(launch_hint_anchor(c->V.p, base, n, c->npoints, hint, c->anchor.p, c->stream));
    HIPCHK(hipMemsetAsync(c->lastt.p, 0xFF, n * sizeof(uint32_t), c->stream));
    c->call_clouds = C;
    c->lord = lord;
    c->exact_needed = false;
    c->deferred_base = c->hctr->deferred;
    // without a model the learned scheduler falls back to the plain order (counted in the
    // statistics); the triangulation is the same either way
    const bool learned = c->opt.scheduler == DT_SCHED_LEARNED && c->have_model;
    if (c->opt.scheduler == DT_SCHED_LEARNED && !c->have_model) c->st.sched_fallbacks++;
    c->learned_active = learned;
    if (learned) {
        // learned order: each BRIO level split into the points predicted cheap, then the
        // costly ones; walk-start buckets from the same MLP pass
        if ((rc = ensure(c, c->feat, (size_t)n * NFEAT)) || (rc = ensure(c, c->ypred, (size_t)n * NOUT)) ||
            (rc = ensure(c, c->wbucket, n)))
            return rc;
        HIPCHK(launch_features(c->V.p, base, n, c->clouds.p, c->anchor.p, c->lev.p, L, c->feat.p, c->stream));
        HIPCHK(launch_mlp_infer(c->wbf.p, c->feat.p, n, c->ypred.p, c->stream));
        HIPCHK(launch_learned_keys(c->ypred.p, c->lev.p, n, base, c->thr, c->keys.p, c->vals.p, c->wbucket.p,
                                   c->stream));
        int lbits = 0;
        while ((1 << lbits) < 2 * L) ++lbits;
        bool swapped = false;
        HIPCHK(radix_sort_pairs(c->keys.p, c->vals.p, c->keys_tmp.p, c->vals_tmp.p, c->hist.p, c->scan_tmp.p, n,
                                lbits, c->stream, &swapped));
        c->lord = swapped ? c->vals_tmp.p : c->vals.p;
        HIPCHK(hipMemsetAsync(c->small.p, 0, 64 * sizeof(uint32_t), c->stream));
        HIPCHK(launch_level_hist(swapped ? c->keys_tmp.p : c->keys.p, n, 0, c->small.p, c->stream));
        HIPCHK(hipMemcpyAsync(hist.data(), c->small.p, 64 * sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        L *= 2;
        compute_levels(hist, L, lv);
        lv.halves = true;
        if ((rc = upload_levels(c, lv, &d_start, &d_size, &d_bits, &d_rb))) return rc;
        // anchors stay those of the BRIO levels: a half level is a sparse and, by the cost
        // prediction, uneven subset, and its records make far walk starts
    }
    if (n > BIG_CALL_POINTS) {
        // the keys, the dedupe table, the value buffer not holding the level-major order and
        // the scheduler's features are not needed by the rounds: their memory goes to the
        // pool and round buffers, allocated next
        auto rel = [c](auto &b) { dev_free(c, b.p); b.p = nullptr; b.cap = 0; };
        rel(c->keys);
        rel(c->keys_tmp);
        rel(c->table);
        rel(c->feat);
        rel(c->ypred);
        if (c->lord == c->vals.p) rel(c->vals_tmp);
        else if (c->lord == c->vals_tmp.p) rel(c->vals);
    }
    // 7. initial tetrahedron of each cloud
    if (fresh) {
        // pool layout: 64-bit adjacency codes when asked for, or (automatic) when the pool
        // this call needs passes the 2^30 slots of 32-bit codes
        const uint64_t want = std::max<uint64_t>(
            c->opt.capacity_tets ? c->opt.capacity_tets : (uint64_t)(6.9 * (double)n) + 65536 + 5ull * C, 4096);
        const bool wide = c->opt.index_bits == 64 || (c->opt.index_bits == 0 && want > MAX_TETS);
        if (c->opt.index_bits == 32 && want > MAX_TETS)
            return fail(c, DT_E_CAPACITY, "%llu points need more than %u tetrahedron slots with 32-bit adjacency "
                                          "codes (dt_options.index_bits = 64 or 0 lifts the limit)",
                        (unsigned long long)n, MAX_TETS);
        if (c->tcap == 0 || c->tcap < std::min<uint64_t>(want, 7 * n + 4096 + 5ull * C) || c->wide != wide ||
            (c->opt.subdet_cache != 0) != (c->subd != nullptr)) {
            if (c->tcap) {
                dev_free(c, c->T); dev_free(c, c->fl[0]); dev_free(c, c->fl[1]); dev_free(c, c->subd);
                c->T = nullptr;
                c->subd = nullptr;
                c->tcap = 0;
            }
            c->wide = wide;
            if ((rc = grow_tets(c, want))) return rc;
        }
        HIPCHK(hipMemsetAsync(&c->ctr->error, 0, sizeof(uint32_t), c->stream));
        c->hctr->bad_cloud = NONE;
        c->hctr->tet_count = 5 * C;
        HIPCHK(hipMemcpyAsync(&c->ctr->bad_cloud, &c->hctr->bad_cloud, sizeof(uint32_t), hipMemcpyHostToDevice,
                              c->stream));
        HIPCHK(hipMemcpyAsync(&c->ctr->tet_count, &c->hctr->tet_count, sizeof(uint32_t), hipMemcpyHostToDevice,
                              c->stream));
        HIPCHK(launch_init(c->V.p, c->clouds.p, C, 0, c->dup.p, c->T, c->wide, c->vtet.p, c->ctr, c->subd,
                           c->stream));
        if ((rc = sync_ctr(c))) return rc;
        if (c->hctr->error & ERR_DEGENERATE) {
            if (C == 1) return fail(c, DT_E_DEGENERATE, "fewer than four affinely independent distinct points");
            return fail(c, DT_E_DEGENERATE, "cloud %u has fewer than four affinely independent distinct points",
                        c->hctr->bad_cloud);
        }
        c->mesh_vertices = 4ull * C;
    }
    c->logged = c->opt.log_points != 0;
    if (c->logged) {
        if ((rc = ensure(c, c->log_att, n))) return rc;
        HIPCHK(hipMemsetAsync(c->log_att.p, 0, n * sizeof(uint32_t), c->stream));
        c->log_base = base;
        c->log_n = n;
    }
    if ((rc = sync_ctr(c))) return rc;
    c->st.duplicates += c->hctr->dups;
    auto t1 = std::chrono::steady_clock::now();
    // 8. insertion rounds
    c->have_mesh = true;
    c->nclouds = C;
    c->nv = base + n;
    c->npoints += n;
    c->st.points += n;
    const uint64_t want_r = c->opt.round_size ? std::min<uint64_t>(c->opt.round_size, c->round_cap) : c->round_cap;
    if ((rc = ensure_round_buffers(c, (uint32_t)std::min<uint64_t>(want_r, std::max<uint64_t>(n, ROUND_MIN)))))
        return rc;
    rc = run_rounds(c, lv, d_start, d_size, d_bits, d_rb, base, n);
    auto t2 = std::chrono::steady_clock::now();
    c->st.ms_sort += std::chrono::duration<double, std::milli>(t1 - t0).count();
    c->st.ms_insert += std::chrono::duration<double, std::milli>(t2 - t1).count();
    c->st.ms_total += std::chrono::duration<double, std::milli>(t2 - t0).count();
    return rc;
}

}  // namespace

// ====================================================================== C ABI

extern "C" {

void dt_default_options(dt_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->device = 0;
    o->stream = nullptr;
    o->seed = 0x5EED;
}

int dt_create(dt_ctx **out, const dt_options *opt) {
    if (!out) return DT_E_ARG;
    *out = nullptr;
    dt_ctx *c = new (std::nothrow) dt_ctx();
    if (!c) return DT_E_CAPACITY;
    if (opt) c->opt = *opt;
    else dt_default_options(&c->opt);
    if (c->opt.round_fraction < 0 || c->opt.round_fraction > 64 ||
        (c->opt.lanes_per_insert != 0 && c->opt.lanes_per_insert != 4 && c->opt.lanes_per_insert != 8 &&
         c->opt.lanes_per_insert != 16 && c->opt.lanes_per_insert != 32 && c->opt.lanes_per_insert != 64) ||
        (c->opt.index_bits != 0 && c->opt.index_bits != 32 && c->opt.index_bits != 64) ||
        (c->opt.large_lanes != 0 && c->opt.large_lanes != 64 && c->opt.large_lanes != 256) ||
        (c->opt.graph_rounds != 0 && c->opt.graph_rounds != 1)) {
        delete c;
        return DT_E_ARG;
    }
    c->device = c->opt.device;
    c->trace = getenv("DT_TRACE") ? atoi(getenv("DT_TRACE")) : 0;
    if (hipSetDevice(c->device) != hipSuccess) {
        hipGetLastError();
        delete c;
        return DT_E_DEVICE;
    }
    int rc = DT_OK;
    if (c->opt.stream) {
        c->stream = (hipStream_t)c->opt.stream;
    } else if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) == hipSuccess) {
        c->own_stream = true;
    } else {
        rc = DT_E_DEVICE;
    }
    apply_options(c);
    if (!rc && (hipMalloc((void **)&c->ctr, sizeof(Ctr)) != hipSuccess ||
                hipMalloc((void **)&c->stat, STAT_WORDS * sizeof(unsigned long long)) != hipSuccess ||
                hipHostMalloc((void **)&c->hring, 3 * sizeof(Ctr) + 3 * sizeof(unsigned long long),
                              hipHostMallocDefault) != hipSuccess))
        rc = DT_E_DEVICE;
    if (!rc) {
        c->hctr = c->hring;
        c->hseq = reinterpret_cast<unsigned long long *>(c->hring + 3);
        c->ring_direct = true;
    }
    for (int k = 0; k < 3 && !rc; ++k) {
        for (int j = 0; j < 3 && !rc; ++j)
            if (hipEventCreate(&c->ev[k][j]) != hipSuccess) rc = DT_E_DEVICE;
        if (!rc && hipEventCreateWithFlags(&c->evdone[k], hipEventDisableTiming) != hipSuccess) rc = DT_E_DEVICE;
    }
    if (!rc && (hipMemsetAsync(c->ctr, 0, sizeof(Ctr), c->stream) != hipSuccess ||
                hipMemsetAsync(c->stat, 0, STAT_WORDS * sizeof(unsigned long long), c->stream) != hipSuccess ||
                hipStreamSynchronize(c->stream) != hipSuccess))
        rc = DT_E_DEVICE;
    if (rc) {
        hipGetLastError();
        dt_destroy(c);
        return rc;
    }
    std::memset(c->hring, 0, 3 * sizeof(Ctr) + 3 * sizeof(unsigned long long));
    *out = c;
    return DT_OK;
}

int dt_insert_points(dt_ctx *c, const double *xyz, uint64_t n) {
    if (!c) return DT_E_ARG;
    if (n == 0) return DT_OK;
    if (!xyz) return fail(c, DT_E_ARG, "xyz is NULL");
    if (c->batch) return fail(c, DT_E_ARG, "the context holds a batch of clouds: dt_clear it first");
    if (c->nv + n >= (1ull << 31) || c->npoints + n >= (1ull << 32) - 2 || n >= (1ull << 30))
        return fail(c, DT_E_CAPACITY, "too many points (limits: 2^30 per call, 2^31 in all)");
    c->h_off = {0, n};
    return insert_clouds(c, xyz, n, c->h_off);
}

int dt_insert_batch(dt_ctx *c, const double *xyz, const uint64_t *offsets, uint32_t num_clouds) {
    if (!c) return DT_E_ARG;
    if (!xyz || !offsets || num_clouds == 0) return fail(c, DT_E_ARG, "xyz or offsets is NULL, or no clouds");
    if (c->have_mesh || c->nv) return fail(c, DT_E_ARG, "dt_insert_batch needs an empty context (dt_clear it)");
    std::vector<uint64_t> off(offsets, offsets + num_clouds + 1);
    if (off[0] != 0) return fail(c, DT_E_ARG, "offsets[0] must be 0");
    for (uint32_t k = 0; k < num_clouds; ++k)
        if (off[k + 1] < off[k] + 4) return fail(c, DT_E_ARG, "cloud %u has fewer than 4 points", k);
    const uint64_t n = off[num_clouds];
    if (n >= (1ull << 30)) return fail(c, DT_E_CAPACITY, "too many points (limit 2^30 per call)");
    c->h_off = off;
    int rc = insert_clouds(c, xyz, n, c->h_off);
    c->batch = true;
    return rc;
}

int dt_get_tets(dt_ctx *c, uint32_t *tets, int64_t *nbrs, uint64_t *num_tets) {
    if (!c || !num_tets) return DT_E_ARG;
    HIPCHK(hipSetDevice(c->device));
    if (!c->have_mesh) {
        *num_tets = 0;
        return DT_OK;
    }
    int rc;
    // live finite tetrahedra numbered in slot order: bit set + scan of the per-word counts
    const uint32_t count = c->hctr->tet_count;
    const uint64_t nw = ((uint64_t)count + 63) / 64;
    if ((rc = ensure(c, c->obits, nw + 1)) || (rc = ensure(c, c->owcnt, nw + 1)) ||
        (rc = ensure(c, c->opre, nw + 1)) || (rc = ensure(c, c->scan_tmp, scan_tmp_entries(nw) + 64)))
        return rc;
    HIPCHK(launch_live_bits(c->T, c->wide, count, c->obits.p, c->owcnt.p, c->stream));
    HIPCHK(exclusive_scan_u32(c->owcnt.p, c->opre.p, nw, c->scan_tmp.p, c->opre.p + nw, c->stream));
    uint32_t T = 0;
    HIPCHK(hipMemcpyAsync(&T, c->opre.p + nw, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->st.tets = T;
    if (!tets && !nbrs) {
        *num_tets = T;
        return DT_OK;
    }
    if (*num_tets < T) {
        *num_tets = T;
        return fail(c, DT_E_ARG, "output buffers hold %llu tetrahedra, %u needed", (unsigned long long)*num_tets, T);
    }
    *num_tets = T;
    if ((rc = ensure(c, c->ovid, std::max<uint64_t>(c->nv, 1)))) return rc;
    HIPCHK(launch_out_vid(c->V.p, (uint32_t)c->nv, c->ovid.p, c->stream));
    // The export kernel stores 16-byte vectors: host buffers and device buffers that are not
    // 16-byte aligned are filled through staging buffers, a slot range at a time (chunk
    // boundaries are multiples of 64 slots, so each chunk's first output row is a scan value).
    const bool dev_t = tets && is_device_ptr(tets) && ((uintptr_t)tets & 15u) == 0,
               dev_n = nbrs && is_device_ptr(nbrs) && ((uintptr_t)nbrs & 15u) == 0;
    const bool staged = (tets && !dev_t) || (nbrs && !dev_n);
    const uint32_t chunk = staged ? c->export_chunk : std::max<uint32_t>(count, 64);
    std::vector<uint32_t> obase;
    for (uint64_t t0 = 0; t0 < count; t0 += chunk) obase.push_back(0);
    obase.push_back(T);
    if (staged) {
        if ((tets && !dev_t && (rc = ensure(c, c->otets, 4 * (size_t)chunk))) ||
            (nbrs && !dev_n && (rc = ensure(c, c->onbrs, 4 * (size_t)chunk))))
            return rc;
        for (size_t k = 1; k + 1 < obase.size(); ++k)
            HIPCHK(hipMemcpyAsync(&obase[k], c->opre.p + (k * (uint64_t)chunk) / 64, sizeof(uint32_t),
                                  hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
    }
    for (size_t k = 0; k + 1 < obase.size(); ++k) {
        const uint32_t t0 = (uint32_t)(k * (uint64_t)chunk);
        const uint32_t t1 = (uint32_t)std::min<uint64_t>(count, (uint64_t)t0 + chunk);
        const uint32_t o0 = obase[k], o1 = obase[k + 1];
        uint32_t *ot = tets ? (dev_t ? tets + 4 * (size_t)o0 : c->otets.p) : nullptr;
        int64_t *on = nbrs ? (dev_n ? nbrs + 4 * (size_t)o0 : c->onbrs.p) : nullptr;
        HIPCHK(launch_output(c->T, c->wide, c->ovid.p, c->obits.p, c->opre.p, t0, t1, o0, ot, on, c->stream));
        if (tets && !dev_t && o1 > o0)
            HIPCHK(hipMemcpyAsync(tets + 4 * (size_t)o0, ot, 4 * (size_t)(o1 - o0) * sizeof(uint32_t),
                                  hipMemcpyDefault, c->stream));
        if (nbrs && !dev_n && o1 > o0)
            HIPCHK(hipMemcpyAsync(nbrs + 4 * (size_t)o0, on, 4 * (size_t)(o1 - o0) * sizeof(int64_t),
                                  hipMemcpyDefault, c->stream));
        if (staged) HIPCHK(hipStreamSynchronize(c->stream));  // the staging buffers are reused
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    return DT_OK;
}

// Groups the live finite tetrahedra by cloud (cached until the mesh changes).
static int build_cloud_index(dt_ctx *c) {
    if (c->out_index) return DT_OK;
    const uint32_t count = c->hctr->tet_count, C = c->nclouds;
    int rc;
    if ((rc = ensure(c, c->okeys, 2 * (size_t)count + 2)) || (rc = ensure(c, c->osorted, 2 * (size_t)count + 2)) ||
        (rc = ensure(c, c->omap2, (size_t)count + 1)) || (rc = ensure(c, c->hist, radix_hist_entries(count))) ||
        (rc = ensure(c, c->scan_tmp, scan_tmp_entries(radix_hist_entries(count)) + scan_tmp_entries(count) + 64)) ||
        (rc = ensure(c, c->cloud_ch, (size_t)C + 1)))
        return rc;
    unsigned long long *k0 = c->okeys.p, *k1 = c->okeys.p + count + 1;
    uint32_t *v0 = c->osorted.p, *v1 = c->osorted.p + count + 1;
    HIPCHK(launch_tet_cloud(c->T, c->wide, c->V.p, count, C, k0, v0, c->stream));
    int bits = 0;
    while ((1ull << bits) <= C) ++bits;
    bool swapped = false;
    HIPCHK(radix_sort_pairs(k0, v0, k1, v1, c->hist.p, c->scan_tmp.p, count, bits, c->stream, &swapped));
    unsigned long long *sk = swapped ? k1 : k0;
    uint32_t *sv = swapped ? v1 : v0;
    // toff[C] = first non-finite position (count when every slot is a finite tetrahedron)
    std::vector<uint32_t> toff(C + 1, 0);
    toff[C] = count;
    HIPCHK(hipMemcpyAsync(c->cloud_ch.p, toff.data(), (C + 1) * sizeof(uint32_t), hipMemcpyHostToDevice, c->stream));
    HIPCHK(launch_seg_bounds(sk, count, C, c->cloud_ch.p, c->stream));
    HIPCHK(hipMemcpyAsync(toff.data(), c->cloud_ch.p, (C + 1) * sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(launch_tet_map(sv, toff[C], c->omap2.p, c->stream));
    c->h_toff.assign(toff.begin(), toff.end());
    c->osorted_live = sv;
    c->out_index = true;
    return DT_OK;
}

int dt_get_tets_batch(dt_ctx *c, uint32_t cloud, uint32_t *tets, int64_t *nbrs, uint64_t *num_tets) {
    if (!c || !num_tets) return DT_E_ARG;
    if (!c->have_mesh || cloud >= c->nclouds)
        return fail(c, DT_E_ARG, "no cloud %u in this context (%u clouds)", cloud, c->nclouds);
    HIPCHK(hipSetDevice(c->device));
    int rc;
    if ((rc = build_cloud_index(c))) return rc;
    const uint32_t tb = (uint32_t)c->h_toff[cloud], te = (uint32_t)c->h_toff[cloud + 1];
    const uint64_t T = te - tb;
    if (!tets && !nbrs) {
        *num_tets = T;
        return DT_OK;
    }
    if (*num_tets < T) {
        *num_tets = T;
        return fail(c, DT_E_ARG, "output buffers hold %llu tetrahedra, %llu needed", (unsigned long long)*num_tets,
                    (unsigned long long)T);
    }
    *num_tets = T;
    // the export kernel stores 16-byte vectors: device buffers that are not 16-byte aligned
    // are filled through the staging buffers, like host buffers
    const bool dev_t = tets && is_device_ptr(tets) && ((uintptr_t)tets & 15u) == 0,
               dev_n = nbrs && is_device_ptr(nbrs) && ((uintptr_t)nbrs & 15u) == 0;
    uint32_t *ot = tets;
    int64_t *on = nbrs;
    if (tets && !dev_t) {
        if ((rc = ensure(c, c->otets, 4 * (size_t)T + 4))) return rc;
        ot = c->otets.p;
    }
    if (nbrs && !dev_n) {
        if ((rc = ensure(c, c->onbrs, 4 * (size_t)T + 4))) return rc;
        on = c->onbrs.p;
    }
    HIPCHK(launch_output_cloud(c->T, c->wide, c->V.p, c->osorted_live, c->omap2.p, tb, te, c->h_off[cloud], ot, on,
                               c->stream));
    // the destination is host memory or an unaligned device buffer
    if (tets && !dev_t)
        HIPCHK(hipMemcpyAsync(tets, ot, 4 * T * sizeof(uint32_t), hipMemcpyDefault, c->stream));
    if (nbrs && !dev_n)
        HIPCHK(hipMemcpyAsync(nbrs, on, 4 * T * sizeof(int64_t), hipMemcpyDefault, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return DT_OK;
}

int dt_autotune(dt_ctx *c, const double *xyz, uint64_t n, dt_options *best, double *best_ms) {
    if (!c || !xyz || n < 4) return DT_E_ARG;
    if (c->have_mesh || c->nv) return fail(c, DT_E_ARG, "dt_autotune needs an empty context (dt_clear it)");
    if (n >= (1ull << 30)) return fail(c, DT_E_CAPACITY, "sample too large");
    HIPCHK(hipSetDevice(c->device));
    int rc;
    const double *dxyz = xyz;
    DevBuf<double> sample;
    if (!is_device_ptr(xyz)) {
        if ((rc = ensure(c, sample, 3 * n))) return rc;
        HIPCHK(hipMemcpyAsync(sample.p, xyz, 3 * n * sizeof(double), hipMemcpyHostToDevice, c->stream));
        dxyz = sample.p;
    }
    static const uint32_t lanes[] = {0, 8, 16, 32};  // 0: automatic
    static const double fracs[] = {0.0, 3.0 / 64, 3.0 / 32};  // 0: automatic
    static const uint32_t caps[] = {64, 128};
    static const uint32_t larges[] = {64, 256};
    constexpr int NL = 4, NF = 3, NC = 2, NB = 2;
    const int cls = size_class(n);
    const dt_options saved = c->opt;
    const dt_ctx::Tuned saved_entry = c->tuned[cls];
    dt_options bo = saved;
    double bms = 1e300;
    rc = DT_OK;
    // the configuration under test is the only tuned entry while the loop runs
    dt_ctx::Tuned keep[64];
    std::copy(std::begin(c->tuned), std::end(c->tuned), keep);
    for (auto &t : c->tuned) t.set = false;
    for (int warm = 1, k = 0; k < NL * NF * NC * NB && rc == DT_OK; warm = 0) {
        c->opt.lanes_per_insert = lanes[k / (NF * NC * NB)];
        c->opt.round_fraction = fracs[(k / (NC * NB)) % NF];
        c->opt.cavity_cap = caps[(k / NB) % NC];
        c->opt.large_lanes = larges[k % NB];
        auto t0 = std::chrono::steady_clock::now();
        rc = dt_insert_points(c, dxyz, n);
        if (rc == DT_OK && hipStreamSynchronize(c->stream) != hipSuccess) rc = DT_E_DEVICE;
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        const int rc2 = dt_clear(c);
        if (rc == DT_OK) rc = rc2;
        if (warm) continue;  // the first run only warms up allocations
        if (rc == DT_OK && ms < bms) {
            bms = ms;
            bo = c->opt;
        }
        ++k;
    }
    if (sample.p) {
        hipStreamSynchronize(c->stream);
        hipFree(sample.p);
    }
    std::copy(std::begin(keep), std::end(keep), c->tuned);
    c->opt = saved;
    if (rc != DT_OK) {
        c->tuned[cls] = saved_entry;
        apply_options(c);
        return rc;
    }
    dt_ctx::Tuned &t = c->tuned[cls];
    t.set = true;
    t.lanes = bo.lanes_per_insert;
    t.frac = bo.round_fraction;
    t.cap = bo.cavity_cap;
    t.large = bo.large_lanes;
    t.ms = bms;
    apply_options(c);
    if (best) *best = bo;
    if (best_ms) *best_ms = bms;
    return DT_OK;
}

int dt_autotune_reset(dt_ctx *c) {
    if (!c) return DT_E_ARG;
    for (auto &t : c->tuned) t.set = false;
    apply_options(c);
    return DT_OK;
}

// ------------------------------------------------------------------ learned scheduler

namespace {

constexpr uint32_t MODEL_MAGIC = 0x4C4D5444u;  // "DTML"
// thr: cost above which a point goes to the costly half of its level; costly_scale: round
// size factor for the costly halves
struct ModelHeader {
    uint32_t magic, version, nfeat, nhid, nout, nparam;
    float thr, costly_scale;
};

int model_buffers(dt_ctx *c) {
    int rc;
    if ((rc = ensure(c, c->w32, NPARAM)) || (rc = ensure(c, c->wbf, NPARAM)) || (rc = ensure(c, c->m1, NPARAM)) ||
        (rc = ensure(c, c->m2, NPARAM)) || (rc = ensure(c, c->grad, NPARAM)) || (rc = ensure(c, c->loss, 4)))
        return rc;
    return DT_OK;
}

}  // namespace

int dt_get_point_log(dt_ctx *c, float *features, float *cost, uint8_t *bucket, uint64_t *num_points) {
    if (!c || !num_points) return DT_E_ARG;
    if (!c->logged) return fail(c, DT_E_ARG, "the last insertion did not log points (dt_options.log_points)");
    const uint64_t n = c->log_n;
    if (!features && !cost && !bucket) {
        *num_points = n;
        return DT_OK;
    }
    if (*num_points < n) {
        *num_points = n;
        return fail(c, DT_E_ARG, "buffers hold %llu points, %llu needed", (unsigned long long)*num_points,
                    (unsigned long long)n);
    }
    *num_points = n;
    HIPCHK(hipSetDevice(c->device));
    int rc;
    if ((rc = ensure(c, c->feat, (size_t)n * NFEAT)) || (rc = ensure(c, c->ypred, (size_t)n * NOUT)) ||
        (rc = ensure(c, c->wbucket, n)))
        return rc;
    int L = 1;
    for (size_t k = 0; k + 1 < c->h_off.size(); ++k)
        L = std::max(L, (int)brio_cum(c->h_off[k + 1] - c->h_off[k]).size());
    HIPCHK(launch_features(c->V.p, c->log_base, n, c->clouds.p, c->anchor.p, c->lev.p, L, c->feat.p, c->stream));
    // labels: cost in ypred (stride 1), bucket in wbucket
    HIPCHK(launch_labels(c->V.p, c->log_base, n, c->clouds.p, c->anchor.p, c->lev.p, c->log_att.p, c->ypred.p,
                         c->wbucket.p, c->stream));
    if (features)
        HIPCHK(hipMemcpyAsync(features, c->feat.p, n * NFEAT * sizeof(float), hipMemcpyDefault, c->stream));
    if (cost) HIPCHK(hipMemcpyAsync(cost, c->ypred.p, n * sizeof(float), hipMemcpyDefault, c->stream));
    if (bucket) HIPCHK(hipMemcpyAsync(bucket, c->wbucket.p, n, hipMemcpyDefault, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return DT_OK;
}

int dt_train_model(dt_ctx *c, const float *features, const float *cost, const uint8_t *bucket, uint64_t n,
                   uint32_t epochs, float lr, uint64_t seed, void *model, size_t *model_bytes) {
    if (!c || !features || !cost || !bucket || n == 0 || !model_bytes) return DT_E_ARG;
    const size_t bytes = sizeof(ModelHeader) + NPARAM * sizeof(float);
    if (!model) {
        *model_bytes = bytes;
        return DT_OK;
    }
    if (*model_bytes < bytes) {
        *model_bytes = bytes;
        return fail(c, DT_E_ARG, "model buffer holds %zu bytes, %zu needed", *model_bytes, bytes);
    }
    HIPCHK(hipSetDevice(c->device));
    int rc;
    if ((rc = model_buffers(c))) return rc;
    // samples in a seeded random order (host), on the device
    std::vector<uint64_t> order(n);
    for (uint64_t i = 0; i < n; ++i) order[i] = i;
    uint64_t st = seed;
    for (uint64_t i = n - 1; i > 0; --i) {
        const uint64_t j = host_mix64(st++) % (i + 1);
        std::swap(order[i], order[j]);
    }
    std::vector<float> hf(n * NFEAT), hc(n);
    std::vector<uint8_t> hb(n);
    for (uint64_t i = 0; i < n; ++i) {
        const uint64_t o = order[i];
        std::memcpy(&hf[i * NFEAT], &features[o * NFEAT], NFEAT * sizeof(float));
        hc[i] = cost[o];
        hb[i] = bucket[o];
    }
    DevBuf<float> df, dc;
    DevBuf<uint8_t> db;
    if ((rc = ensure(c, df, n * NFEAT)) || (rc = ensure(c, dc, n)) || (rc = ensure(c, db, n))) return rc;
    HIPCHK(hipMemcpyAsync(df.p, hf.data(), n * NFEAT * sizeof(float), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(dc.p, hc.data(), n * sizeof(float), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(db.p, hb.data(), n, hipMemcpyHostToDevice, c->stream));
    // Glorot-uniform weights, zero biases (seeded)
    std::vector<float> w(NPARAM, 0.0f);
    const int fan[3][2] = {{NFEAT, NHID}, {NHID, NHID}, {NHID, NOUT}};
    int o = 0;
    for (int l = 0; l < 3; ++l) {
        const double a = std::sqrt(6.0 / (fan[l][0] + fan[l][1]));
        for (int k = 0; k < fan[l][0] * fan[l][1]; ++k)
            w[o + k] = (float)(a * (2.0 * ((host_mix64(st++) >> 11) * 0x1p-53) - 1.0));
        o += fan[l][0] * fan[l][1] + fan[l][1];
    }
    HIPCHK(hipMemcpyAsync(c->w32.p, w.data(), NPARAM * sizeof(float), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemsetAsync(c->m1.p, 0, NPARAM * sizeof(float), c->stream));
    HIPCHK(hipMemsetAsync(c->m2.p, 0, NPARAM * sizeof(float), c->stream));
    HIPCHK(hipMemsetAsync(c->grad.p, 0, NPARAM * sizeof(float), c->stream));
    HIPCHK(launch_to_bf16(c->w32.p, c->wbf.p, c->stream));
    constexpr uint32_t BATCH = 4096;
    int t = 0;
    for (uint32_t e = 0; e < epochs; ++e) {
        for (uint64_t b0 = 0; b0 < n; b0 += BATCH) {
            const uint32_t nb = (uint32_t)std::min<uint64_t>(BATCH, n - b0);
            HIPCHK(launch_mlp_grad(c->wbf.p, df.p, dc.p, db.p, b0, nb, c->grad.p, nullptr, c->stream));
            HIPCHK(launch_adam(c->w32.p, c->grad.p, c->m1.p, c->m2.p, c->wbf.p, lr, ++t, c->stream));
        }
    }
    HIPCHK(hipMemcpyAsync(w.data(), c->w32.p, NPARAM * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    hipFree(df.p);
    hipFree(dc.p);
    hipFree(db.p);
    // split threshold of the scheduler: the median cost of the training points.  The rounds
    // over the costly halves shrink only where the costly points are conflict-heavy: their
    // mean cost in training reaches that of COSTLY_ATTEMPTS attempts
    std::vector<float> med(hc);
    std::nth_element(med.begin(), med.begin() + med.size() / 2, med.end());
    const float thr = med[med.size() / 2];
    double sum = 0.0;
    uint64_t cnt = 0;
    for (float v : hc)
        if (v > thr) sum += v, ++cnt;
    const bool heavy = cnt && sum / (double)cnt >= std::log2(1.0 + (double)COSTLY_ATTEMPTS);
    ModelHeader h{MODEL_MAGIC, 2, NFEAT, NHID, NOUT, NPARAM, thr, heavy ? (float)COSTLY_ROUND_SCALE : 1.0f};
    std::memcpy(model, &h, sizeof h);
    std::memcpy((char *)model + sizeof h, w.data(), NPARAM * sizeof(float));
    *model_bytes = bytes;
    c->thr = h.thr;
    c->costly_scale = h.costly_scale;
    c->have_model = true;
    return DT_OK;
}

int dt_load_model(dt_ctx *c, const void *model, size_t bytes) {
    if (!c || !model) return DT_E_ARG;
    ModelHeader h;
    if (bytes < sizeof h) return fail(c, DT_E_ARG, "model too short");
    std::memcpy(&h, model, sizeof h);
    if (h.magic != MODEL_MAGIC || h.version != 2 || h.nfeat != (uint32_t)NFEAT || h.nhid != (uint32_t)NHID ||
        h.nout != (uint32_t)NOUT || h.nparam != (uint32_t)NPARAM || bytes < sizeof h + NPARAM * sizeof(float))
        return fail(c, DT_E_ARG, "not a model of this library (%u-%u-%u)", h.nfeat, h.nhid, h.nout);
    HIPCHK(hipSetDevice(c->device));
    int rc;
    if ((rc = model_buffers(c))) return rc;
    HIPCHK(hipMemcpyAsync(c->w32.p, (const char *)model + sizeof h, NPARAM * sizeof(float), hipMemcpyHostToDevice,
                          c->stream));
    HIPCHK(launch_to_bf16(c->w32.p, c->wbf.p, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->thr = h.thr;
    c->costly_scale = h.costly_scale;
    c->have_model = true;
    return DT_OK;
}

int dt_debug_mlp_grad(dt_ctx *c, const float *features, const float *cost, const uint8_t *bucket, uint32_t n,
                      float *grad, float *loss) {
    if (!c || !features || !cost || !bucket || !grad || n == 0) return DT_E_ARG;
    if (!c->have_model) return fail(c, DT_E_ARG, "no model loaded");
    HIPCHK(hipSetDevice(c->device));
    int rc;
    DevBuf<float> df, dc;
    DevBuf<uint8_t> db;
    if ((rc = model_buffers(c)) || (rc = ensure(c, df, (size_t)n * NFEAT)) || (rc = ensure(c, dc, n)) ||
        (rc = ensure(c, db, n)))
        return rc;
    HIPCHK(hipMemcpyAsync(df.p, features, (size_t)n * NFEAT * sizeof(float), hipMemcpyDefault, c->stream));
    HIPCHK(hipMemcpyAsync(dc.p, cost, n * sizeof(float), hipMemcpyDefault, c->stream));
    HIPCHK(hipMemcpyAsync(db.p, bucket, n, hipMemcpyDefault, c->stream));
    HIPCHK(hipMemsetAsync(c->grad.p, 0, NPARAM * sizeof(float), c->stream));
    HIPCHK(hipMemsetAsync(c->loss.p, 0, sizeof(float), c->stream));
    HIPCHK(launch_mlp_grad(c->wbf.p, df.p, dc.p, db.p, 0, n, c->grad.p, c->loss.p, c->stream));
    HIPCHK(hipMemcpyAsync(grad, c->grad.p, NPARAM * sizeof(float), hipMemcpyDefault, c->stream));
    if (loss) HIPCHK(hipMemcpyAsync(loss, c->loss.p, sizeof(float), hipMemcpyDefault, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemsetAsync(c->grad.p, 0, NPARAM * sizeof(float), c->stream));
    hipFree(df.p);
    hipFree(dc.p);
    hipFree(db.p);
    return DT_OK;
}

int dt_debug_mlp(dt_ctx *c, const float *features, uint64_t n, float *out) {
    if (!c || !features || !out) return DT_E_ARG;
    if (!c->have_model) return fail(c, DT_E_ARG, "no model loaded");
    if (n == 0) return DT_OK;
    HIPCHK(hipSetDevice(c->device));
    int rc;
    if ((rc = ensure(c, c->feat, (size_t)n * NFEAT)) || (rc = ensure(c, c->ypred, (size_t)n * NOUT))) return rc;
    HIPCHK(hipMemcpyAsync(c->feat.p, features, n * NFEAT * sizeof(float), hipMemcpyDefault, c->stream));
    HIPCHK(launch_mlp_infer(c->wbf.p, c->feat.p, n, c->ypred.p, c->stream));
    HIPCHK(hipMemcpyAsync(out, c->ypred.p, n * NOUT * sizeof(float), hipMemcpyDefault, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return DT_OK;
}

int dt_clear(dt_ctx *c) {
    if (!c) return DT_E_ARG;
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipMemsetAsync(c->ctr, 0, sizeof(Ctr), c->stream));
    HIPCHK(hipMemsetAsync(c->stat, 0, STAT_WORDS * sizeof(unsigned long long), c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    std::memset(c->hring, 0, 3 * sizeof(Ctr));
    c->hctr = c->hring;
    c->grow_pending = false;
    c->npoints = c->nv = 0;
    c->have_mesh = false;
    c->mesh_vertices = 0;
    c->fl_idx = c->list_idx = c->ovf_idx = 0;
    c->st = dt_stats{};
    c->batch = false;
    c->nclouds = 0;
    c->out_index = false;
    return DT_OK;
}

int dt_destroy(dt_ctx *c) {
    if (!c) return DT_E_ARG;
    hipSetDevice(c->device);
    if (c->stream) hipStreamSynchronize(c->stream);
    auto f = [](void *p) { if (p) hipFree(p); };
    f(c->V.p); f(c->vtet.p); f(c->anchor.p); f(c->lastt.p); f(c->dup.p);
    f(c->T); f(c->fl[0]); f(c->fl[1]); f(c->subd);
    for (int k = 0; k < 3; ++k) f(c->clk[k]);
    for (int k = 0; k < 4; ++k) { f(c->lpt[k]); f(c->lrank[k]); }
    f(c->cav); f(c->bnd); f(c->outc); f(c->cnt); f(c->status);
    f(c->scr_v); f(c->scr_n); f(c->defer);
    f(c->ctr);
    f(c->stat);
    if (c->hring) hipHostFree(c->hring);
    f(c->staging.p); f(c->keys.p); f(c->keys_tmp.p); f(c->table.p); f(c->vals.p); f(c->vals_tmp.p);
    f(c->hist.p); f(c->scan_tmp.p); f(c->small.p); f(c->small64.p);
    f(c->clouds.p); f(c->off.p); f(c->ch_start.p); f(c->ch_end.p); f(c->cloud_ch.p); f(c->partial.p);
    f(c->okeys.p); f(c->osorted.p); f(c->omap2.p); f(c->dbgV.p); f(c->dbg_cloud.p);
    f(c->lev.p); f(c->wbucket.p); f(c->log_att.p); f(c->feat.p); f(c->ypred.p);
    f(c->w32.p); f(c->m1.p); f(c->m2.p); f(c->grad.p); f(c->loss.p); f(c->wbf.p);
    f(c->obits.p); f(c->owcnt.p); f(c->opre.p); f(c->otets.p); f(c->onbrs.p); f(c->ovid.p);
    f(c->rf_cc.p); f(c->rf_cc2.p); f(c->rf_ccr.p); f(c->rf_pts.p); f(c->rf_partial.p);
    f(c->rf_q.p); f(c->rf_q2.p); f(c->rf_facets.p); f(c->rf_moore.p); f(c->rf_k0.p); f(c->rf_k1.p);
    f(c->rf_v0.p); f(c->rf_v1.p); f(c->rf_ctr.p); f(c->rf_flags.p); f(c->rf_pos.p);
    f(c->rf_src.p); f(c->rf_src2.p); f(c->rf_srcr.p); f(c->rf_hint.p); f(c->rf_rest.p); f(c->rf_near.p);
    f(c->rf_status.p); f(c->rf_flag.p); f(c->rf_pbig.p); f(c->rf_nnear.p); f(c->rf_prev.p); f(c->rf_cloud.p); f(c->rf_off.p);
    for (int k = 0; k < 3; ++k) {
        for (int j = 0; j < 3; ++j)
            if (c->ev[k][j]) hipEventDestroy(c->ev[k][j]);
        if (c->evdone[k]) hipEventDestroy(c->evdone[k]);
    }
    destroy_round_graphs(c->graphs);
    if (c->own_stream && c->stream) hipStreamDestroy(c->stream);
    hipGetLastError();
    delete c;
    return DT_OK;
}

int dt_get_stats(const dt_ctx *c, dt_stats *out) {
    if (!c || !out) return DT_E_ARG;
    *out = c->st;
    const Ctr &h = *c->hctr;
    out->vertices = c->mesh_vertices;
    out->attempts = h.attempts;
    out->inserted = h.won;
    out->conflicts = h.conflicts;
    out->overflows = h.overflows;
    out->walk_steps = h.walk_steps;
    out->cavity_tets = h.cav_tets;
    out->boundary_facets = h.bnd_facets;
    out->orient_calls = h.orient;
    out->orient_exact = h.orient_exact;
    out->insphere_calls = h.insphere;
    out->insphere_exact = h.insphere_exact;
    out->perturbed = h.perturbed;
    out->cavity_units = h.attempts;
    out->ball_units = h.won;
    out->index_bits = c->tcap ? (c->wide ? 64 : 32) : 0;
    out->dropped_slots = h.dropped;
    out->deferred = h.deferred;
    out->walk_caps = h.walk_caps;
    return DT_OK;
}

const char *dt_last_error(const dt_ctx *c) { return c ? c->err.c_str() : "no context"; }

int dt_debug_sort(dt_ctx *c, const double *xyz, uint64_t n, uint64_t *keys, uint32_t *perm, int *moore_m) {
    if (!c || !xyz || n == 0) return DT_E_ARG;
    if (n >= (1ull << 30)) return fail(c, DT_E_CAPACITY, "too many points");
    HIPCHK(hipSetDevice(c->device));
    int rc;
    const double *dxyz = xyz;
    if (!is_device_ptr(xyz)) {
        if ((rc = ensure(c, c->staging, 3 * n))) return rc;
        HIPCHK(hipMemcpyAsync(c->staging.p, xyz, 3 * n * sizeof(double), hipMemcpyHostToDevice, c->stream));
        dxyz = c->staging.p;
    }
    // the same steps as dt_insert_points for one cloud, on scratch records: curve order, then
    // the level-major order of it
    const std::vector<uint64_t> off = {0, n};
    int mmax = 1;
    uint32_t nchunks = 0;
    if ((rc = prepare_clouds(c, off, 0, true, &mmax, &nchunks, c->dbg_cloud))) return rc;
    if ((rc = ensure(c, c->dbgV, n))) return rc;
    uint32_t *sv = nullptr;
    unsigned long long *sk = nullptr;
    bool bad = false;
    if ((rc = sort_points(c, dxyz, n, c->dbg_cloud.p, c->off.p, 1, nchunks, mmax, &sv, &sk, &bad))) return rc;
    if (bad) return fail(c, DT_E_INPUT, "a coordinate is not finite or outside the accepted range");
    std::vector<uint32_t> moore_order(n), lord_h(n), hist(64);
    HIPCHK(hipMemcpyAsync(moore_order.data(), sv, n * sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(launch_permute(dxyz, sv, sk, 3 * mmax, n, 0, 0, c->dbgV.p, nullptr, nullptr, c->stream));
    const int L = (int)brio_cum(n).size();
    uint32_t *lord = nullptr;
    if ((rc = level_order(c, sv, c->dbgV.p, n, 0, c->off.p, c->dbg_cloud.p, L, &lord, hist.data(), nullptr)))
        return rc;
    HIPCHK(hipMemcpyAsync(lord_h.data(), lord, n * sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (keys) {
        // keys in input order: level << 3m | Moore index (the level of the record at
        // level-major position j is the level whose range holds j)
        HIPCHK(launch_keys(dxyz, n, c->off.p, 1, c->dbg_cloud.p, 3 * mmax, c->keys_tmp.p, c->vals_tmp.p, c->stream));
        std::vector<uint64_t> kh(n);
        HIPCHK(hipMemcpyAsync(kh.data(), c->keys_tmp.p, n * sizeof(uint64_t), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        // with the level in front when it fits beside the Moore index
        uint64_t j = 0;
        if (3 * mmax + 8 <= 64)
            for (int k = 0; k < L; ++k)
                for (uint32_t q = 0; q < hist[k]; ++q, ++j)
                    kh[moore_order[lord_h[j]]] |= (uint64_t)k << (3 * mmax);
        HIPCHK(hipMemcpy(keys, kh.data(), n * sizeof(uint64_t), hipMemcpyDefault));
    }
    if (perm) {
        std::vector<uint32_t> ph(n);
        for (uint64_t q = 0; q < n; ++q) ph[q] = moore_order[lord_h[q]];
        HIPCHK(hipMemcpy(perm, ph.data(), n * sizeof(uint32_t), hipMemcpyDefault));
    }
    if (moore_m) *moore_m = mmax;
    return DT_OK;
}

int dt_debug_set_round_counter(dt_ctx *c, uint64_t rounds) {
    if (!c) return DT_E_ARG;
    c->round_counter = rounds;
    return DT_OK;
}

// ---- triangulation without device allocation ----
//
// Every buffer of the call comes from `scratch`, a static device array each GPU holds for the
// life of the process.  Its address on a device is taken once, with that device current, by
// hipGetSymbolAddress; host code then uses that address only (the array's name is a host
// stand-in).  Calls on one device share the array and its context, so calls that overlap on
// one device race.

}  // extern "C"

static __device__ __align__(256) unsigned char scratch[DT_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
constexpr uint32_t NOALLOC_ROUND_CAP = 4096;      // candidates per round
constexpr uint32_t NOALLOC_EXPORT_CHUNK = 1u << 16;

struct NoallocDevice {
    std::once_flag once;
    int status = DT_OK;             // result of the set-up
    unsigned char *ptr = nullptr;   // device address of `scratch` on this device
    dt_ctx *ctx = nullptr;          // host state, rebuilt in place at every call
    Ctr ring[3];                    // host copies of the counters (static: no pinned allocation)
};
NoallocDevice g_noalloc[NOALLOC_MAX_DEVICES];

// once per device, with the device current: the array's device address and the context
void noalloc_setup(int device, NoallocDevice &d) {
    if (hipSetDevice(device) != hipSuccess) {
        hipGetLastError();
        d.status = DT_E_DEVICE;
        return;
    }
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
        hipGetLastError();
        d.status = DT_E_DEVICE;
        return;
    }
    d.ptr = static_cast<unsigned char *>(p);
    d.ctx = new (std::nothrow) dt_ctx();
    d.status = d.ctx ? DT_OK : DT_E_CAPACITY;
}

}  // namespace

extern "C" {

int dt_triangulate_noalloc(int device, void *stream, const double *xyz, uint64_t n, uint32_t *tets, int64_t *nbrs,
                           uint64_t *num_tets) {
    if (device < 0 || device >= NOALLOC_MAX_DEVICES || !num_tets || (n && !xyz)) return DT_E_ARG;
    if (n > DT_NOALLOC_MAX_POINTS) return DT_E_CAPACITY;
    NoallocDevice &d = g_noalloc[device];
    std::call_once(d.once, noalloc_setup, device, std::ref(d));
    if (d.status != DT_OK) return d.status;
    if (hipSetDevice(device) != hipSuccess) {
        hipGetLastError();
        return DT_E_DEVICE;
    }
    // a fresh context over the arena: options at their defaults, no events, static counters
    dt_ctx *c = d.ctx;
    *c = dt_ctx();
    dt_default_options(&c->opt);
    c->opt.device = device;
    c->device = device;
    c->stream = static_cast<hipStream_t>(stream);
    c->arena = d.ptr;
    c->arena_size = DT_NOALLOC_SCRATCH_BYTES;
    c->round_cap = NOALLOC_ROUND_CAP;
    c->export_chunk = NOALLOC_EXPORT_CHUNK;
    c->hring = d.ring;
    c->hctr = d.ring;
    std::memset(d.ring, 0, sizeof d.ring);
    // the pool is sized once for the whole call: besides the tetrahedra of n points it keeps
    // the headroom the rounds check for (48 slots per candidate of a full round), so it never
    // grows (growth in the arena would leave the old pool behind)
    c->opt.capacity_tets = 7 * n + 65536 + 48ull * NOALLOC_ROUND_CAP;
    apply_options(c);
    int rc;
    if ((rc = ensure(c, c->ctrbuf, 1)) || (rc = ensure(c, c->statbuf, STAT_WORDS))) return rc;
    c->ctr = c->ctrbuf.p;
    c->stat = c->statbuf.p;
    HIPCHK(hipMemsetAsync(c->ctr, 0, sizeof(Ctr), c->stream));
    HIPCHK(hipMemsetAsync(c->stat, 0, STAT_WORDS * sizeof(unsigned long long), c->stream));
    if (n == 0) {
        HIPCHK(hipStreamSynchronize(c->stream));
        *num_tets = 0;
        return DT_OK;
    }
    c->h_off = {0, n};
    if ((rc = insert_clouds(c, xyz, n, c->h_off))) return rc;
    if (!tets && !nbrs) {
        // count only
        rc = dt_get_tets(c, nullptr, nullptr, num_tets);
    } else {
        rc = dt_get_tets(c, tets, nbrs, num_tets);
    }
    c->ctr = nullptr;
    c->stat = nullptr;
    return rc;
}

int dt_get_points(dt_ctx *c, double *xyz, uint64_t *num_points) {
    if (!c || !num_points) return DT_E_ARG;
    if (c->batch) return fail(c, DT_E_ARG, "the context holds a batch of clouds");
    const uint64_t n = c->have_mesh ? c->nv : 0;
    if (!xyz) {
        *num_points = n;
        return DT_OK;
    }
    if (*num_points < n) {
        *num_points = n;
        return fail(c, DT_E_ARG, "the buffer holds %llu points, %llu needed", (unsigned long long)*num_points,
                    (unsigned long long)n);
    }
    *num_points = n;
    if (n == 0) return DT_OK;
    HIPCHK(hipSetDevice(c->device));
    double *out = xyz;
    const bool dev = is_device_ptr(xyz);
    int rc;
    if (!dev) {
        if ((rc = ensure(c, c->staging, 3 * n))) return rc;
        out = c->staging.p;
    }
    HIPCHK(launch_points_out(c->V.p, (uint32_t)n, out, c->stream));
    if (!dev) HIPCHK(hipMemcpyAsync(xyz, out, 3 * n * sizeof(double), hipMemcpyDefault, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return DT_OK;
}

namespace {

// stable radix sort of (keys, vals) by the low `bits` bits; the sorted pair lands in
// (k0, v0) or (k1, v1): returns the values' buffer, *ko the keys'
uint32_t *sort_into(dt_ctx *c, unsigned long long *k0, uint32_t *v0, unsigned long long *k1, uint32_t *v1,
                    uint32_t n, int bits, unsigned long long **ko, hipError_t *err) {
    bool swapped = false;
    *err = radix_sort_pairs_any(k0, v0, k1, v1, c->hist.p, c->scan_tmp.p, n, bits, c->stream, &swapped);
    if (ko) *ko = swapped ? k1 : k0;
    return swapped ? v1 : v0;
}

int bits_for(uint64_t x) {
    int b = 1;
    while (b < 64 && (1ull << b) <= x) ++b;
    return b;
}

}  // namespace

// The inner box of the hull test: the points' box [lo, hi] shrunk on every side by a fraction
// of its extent, the largest of a few candidates whose eight corners the hull test (exact)
// finds strictly inside.  None (lo > hi) when no candidate passes.
static int find_inner_box(dt_ctx *c, uint32_t nf, const double lo[3], const double hi[3], InnerBox *out) {
    *out = InnerBox{{1.0, 1.0, 1.0}, {0.0, 0.0, 0.0}};
    if (nf == 0) return DT_OK;
    constexpr int NBOX = 7;
    constexpr uint32_t NP = 8 * NBOX;
    const double shrink[NBOX] = {0x1p-10, 0x1p-8, 0x1p-6, 0x1p-5, 0x1p-4, 0x1p-3, 0x1p-2};
    InnerBox boxes[NBOX];
    double pts[3 * NP];
    uint4 ids[NP];
    for (int b = 0; b < NBOX; ++b) {
        for (int k = 0; k < 3; ++k) {
            const double e = hi[k] - lo[k];
            boxes[b].lo[k] = lo[k] + shrink[b] * e;
            boxes[b].hi[k] = hi[k] - shrink[b] * e;
        }
        for (uint32_t q = 0; q < 8; ++q) {
            const uint32_t j = 8 * b + q;
            for (int k = 0; k < 3; ++k) pts[3 * j + k] = (q >> k) & 1u ? boxes[b].hi[k] : boxes[b].lo[k];
            ids[j] = make_uint4(j, 0, 0, 0);
        }
    }
    int rc;
    if ((rc = ensure(c, c->rf_cc, 3 * (size_t)NP)) || (rc = ensure(c, c->rf_q, NP)) ||
        (rc = ensure(c, c->rf_src, NP)) || (rc = ensure(c, c->rf_flag, NP)) ||
        (rc = ensure(c, c->rf_cc2, 3 * (size_t)NP)) || (rc = ensure(c, c->rf_q2, NP)) ||
        (rc = ensure(c, c->rf_src2, NP)) || (rc = ensure(c, c->rf_rest, NP)))
        return rc;
    HIPCHK(hipMemcpyAsync(c->rf_cc.p, pts, sizeof pts, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->rf_q.p, ids, sizeof ids, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemsetAsync(c->rf_src.p, 0, NP * sizeof(uint32_t), c->stream));
    HIPCHK(hipMemsetAsync(c->rf_ctr.p + 1, 0, 2 * sizeof(uint32_t), c->stream));
    HIPCHK(launch_inside(c->V.p, c->rf_facets.p, nf, c->rf_cc.p, c->rf_q.p, c->rf_src.p, NP, *out, c->rf_rest.p,
                         c->rf_ctr.p + 2, c->rf_flag.p, c->rf_cc2.p, c->rf_q2.p, c->rf_src2.p, c->rf_ctr.p + 1,
                         c->stream));
    uint32_t nin = 0;
    uint4 got[NP];
    HIPCHK(hipMemcpyAsync(&nin, c->rf_ctr.p + 1, sizeof nin, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (nin > NP) return fail(c, DT_E_INTERNAL, "inner box test returned %u of %u corners", nin, NP);
    if (nin) {
        HIPCHK(hipMemcpyAsync(got, c->rf_q2.p, nin * sizeof(uint4), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
    }
    bool inside[NP] = {};
    for (uint32_t j = 0; j < nin; ++j)
        if (got[j].x < NP) inside[got[j].x] = true;
    for (int b = 0; b < NBOX; ++b) {
        bool ok = true;
        for (uint32_t q = 0; q < 8; ++q) ok = ok && inside[8 * b + q];
        for (int k = 0; k < 3; ++k) ok = ok && boxes[b].lo[k] <= boxes[b].hi[k];
        if (ok) {
            *out = boxes[b];
            break;
        }
    }
    return DT_OK;
}

int dt_refine(dt_ctx *c, double h, uint32_t max_steps, uint32_t *step_counts, uint32_t *num_steps,
              uint64_t *inserted) {
    if (!c || !(h > 0.0) || !std::isfinite(h)) return DT_E_ARG;
    if (num_steps) *num_steps = 0;
    if (inserted) *inserted = 0;
    if (!c->have_mesh || c->batch || c->nclouds != 1)
        return fail(c, DT_E_ARG, "dt_refine needs the triangulation of dt_insert_points calls");
    HIPCHK(hipSetDevice(c->device));
    int rc;
    hipError_t he;
    // the input's grid for the candidates' Moore keys: the box of the points present now and
    // the Moore level of their number
    const uint64_t n0 = c->nv;
    const uint32_t m = (uint32_t)moore_level(n0);
    constexpr uint32_t BOX_BLOCKS = 256;
    if ((rc = ensure(c, c->rf_cloud, 1)) || (rc = ensure(c, c->rf_partial, 6 * BOX_BLOCKS)) ||
        (rc = ensure(c, c->rf_off, 2)) || (rc = ensure(c, c->rf_ctr, 4)))
        return rc;
    HIPCHK(launch_vert_box(c->V.p, (uint32_t)n0, m, c->rf_partial.p, BOX_BLOCKS, c->rf_cloud.p, c->stream));
    Cloud box{};
    std::vector<double> part(6 * BOX_BLOCKS);
    HIPCHK(hipMemcpyAsync(&box, c->rf_cloud.p, sizeof box, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(part.data(), c->rf_partial.p, part.size() * sizeof(double), hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    // the points' box per axis, from the per-block partial boxes
    double plo[3] = {INFINITY, INFINITY, INFINITY}, phi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (uint32_t b = 0; b < BOX_BLOCKS; ++b)
        for (int k = 0; k < 3; ++k) {
            plo[k] = std::fmin(plo[k], part[6 * b + k]);
            phi[k] = std::fmax(phi[k], part[6 * b + 3 + k]);
        }
    const double ext = box.box[3] > 0 ? std::ldexp(1.0, (int)m) / box.box[3] : 0.0;
    // thresholds as (1.4 h)^2 and (0.7 h)^2 in fp64; grid cells a little wider than 0.7 h so
    // that points closer than it always lie in neighbouring cells
    const double g1 = 1.4 * h, f1 = 0.7 * h;
    const double grow = g1 * g1, lim = f1 * f1;
    const double cell = f1 * (1.0 + 0x1p-20);
    const double cells = std::floor(ext / cell) + 3.0;
    if (cells > (double)(1u << 20))
        return fail(c, DT_E_ARG, "h = %g is too small for the point set's extent %g", h, ext);
    const uint64_t G = (uint64_t)cells;
    const int gbits = bits_for(G * G * G);
    const double lo[3] = {box.box[0], box.box[1], box.box[2]};
    // hull facets: the ghosts' facets; points strictly inside never change them
    uint32_t count = c->hctr->tet_count;
    if ((rc = ensure(c, c->rf_facets, std::max<uint32_t>(count, 1)))) return rc;
    HIPCHK(hipMemsetAsync(c->rf_ctr.p, 0, 4 * sizeof(uint32_t), c->stream));
    HIPCHK(launch_hull_facets(c->T, c->wide, count, c->rf_facets.p, c->rf_ctr.p, c->stream));
    uint32_t nf = 0;
    HIPCHK(hipMemcpyAsync(&nf, c->rf_ctr.p, sizeof nf, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    InnerBox ibox;
    if ((rc = find_inner_box(c, nf, plo, phi, &ibox))) return rc;
    uint64_t total = 0;
    uint32_t known = 0;  // slots whose last-pass vertices and size flag rf_prev / rf_pbig hold
    for (uint32_t step = 0; step < max_steps; ++step) {
        count = c->hctr->tet_count;
        const uint64_t nv = c->nv;
        // 1. candidates: circumcentres of the tetrahedra larger than 1.4 h, strictly inside
        if ((rc = ensure(c, c->rf_cc, 3 * (size_t)count)) || (rc = ensure(c, c->rf_q, count)) ||
            (rc = ensure(c, c->rf_cc2, 3 * (size_t)count)) || (rc = ensure(c, c->rf_q2, count)) ||
            (rc = ensure(c, c->rf_src, count)) || (rc = ensure(c, c->rf_src2, count)) ||
            (rc = ensure(c, c->rf_rest, count)) ||
            (rc = ensure(c, c->rf_flag, count)) || (rc = ensure(c, c->rf_prev, count, true)) ||
            (rc = ensure(c, c->rf_pbig, count, true)))
            return rc;
        HIPCHK(hipMemsetAsync(c->rf_ctr.p, 0, 4 * sizeof(uint32_t), c->stream));
        HIPCHK(launch_circum(c->T, c->wide, c->V.p, count, grow, c->rf_prev.p, c->rf_pbig.p, known, c->rf_cc.p,
                             c->rf_q.p, c->rf_src.p, count, c->rf_ctr.p, c->stream));
        known = count;
        uint32_t k0 = 0;
        HIPCHK(hipMemcpyAsync(&k0, c->rf_ctr.p, sizeof k0, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        // rf_ctr[2] counts the candidates outside the inner box here (the filter rounds below
        // clear it before they use it)
        HIPCHK(launch_inside(c->V.p, c->rf_facets.p, nf, c->rf_cc.p, c->rf_q.p, c->rf_src.p, k0, ibox,
                             c->rf_rest.p, c->rf_ctr.p + 2, c->rf_flag.p, c->rf_cc2.p, c->rf_q2.p, c->rf_src2.p,
                             c->rf_ctr.p + 1, c->stream));
        uint32_t K = 0;
        HIPCHK(hipMemcpyAsync(&K, c->rf_ctr.p + 1, sizeof K, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        if (K == 0) {
            if (step_counts) step_counts[2 * step] = step_counts[2 * step + 1] = 0;
            if (num_steps) *num_steps = step + 1;
            break;
        }
        // 2. filter order: Moore key in the input's grid, then the sorted vertex indices
        const size_t sortn = std::max<size_t>(K, nv);
        if ((rc = ensure(c, c->rf_moore, K)) || (rc = ensure(c, c->rf_k0, sortn)) || (rc = ensure(c, c->rf_k1, sortn)) ||
            (rc = ensure(c, c->rf_v0, sortn)) || (rc = ensure(c, c->rf_v1, sortn)) ||
            (rc = ensure(c, c->hist, radix_hist_entries(sortn))) ||
            (rc = ensure(c, c->scan_tmp, scan_tmp_entries(radix_hist_entries(sortn)) + scan_tmp_entries(sortn) + 64)) ||
            (rc = ensure(c, c->rf_ccr, 3 * (size_t)K)) || (rc = ensure(c, c->rf_status, K)) ||
            (rc = ensure(c, c->rf_near, FILTER_NEAR_MAX * (size_t)K)) || (rc = ensure(c, c->rf_nnear, K)) ||
            (rc = ensure(c, c->rf_srcr, K)) ||
            (rc = ensure(c, c->rf_flags, (size_t)K + 1)) || (rc = ensure(c, c->rf_pos, (size_t)K + 1)))
            return rc;
        const uint64_t off[2] = {0, K};
        HIPCHK(hipMemcpyAsync(c->rf_off.p, off, sizeof off, hipMemcpyHostToDevice, c->stream));
        HIPCHK(launch_keys(c->rf_cc2.p, K, c->rf_off.p, 1, c->rf_cloud.p, 0, c->rf_moore.p, c->rf_v1.p, c->stream));
        const int ib = bits_for(nv);  // bits of an input index
        unsigned long long *ks = nullptr;
        HIPCHK(launch_order_keys(c->rf_q2.p, nullptr, nullptr, K, 0, ib, c->rf_k0.p, c->rf_v0.p, c->stream));
        uint32_t *perm = sort_into(c, c->rf_k0.p, c->rf_v0.p, c->rf_k1.p, c->rf_v1.p, K, 2 * ib, &ks, &he);
        HIPCHK(he);
        uint32_t *vb = perm == c->rf_v0.p ? c->rf_v1.p : c->rf_v0.p;
        HIPCHK(launch_order_keys(c->rf_q2.p, nullptr, perm, K, 1, ib, c->rf_k0.p, vb, c->stream));
        perm = sort_into(c, c->rf_k0.p, vb, c->rf_k1.p, perm, K, 2 * ib, &ks, &he);
        HIPCHK(he);
        vb = perm == c->rf_v0.p ? c->rf_v1.p : c->rf_v0.p;
        HIPCHK(launch_order_keys(c->rf_q2.p, c->rf_moore.p, perm, K, 2, 0, c->rf_k0.p, vb, c->stream));
        perm = sort_into(c, c->rf_k0.p, vb, c->rf_k1.p, perm, K, 3 * (int)m, &ks, &he);
        HIPCHK(he);
        // perm[r] = the candidate of rank r; keep it in rf_pos until the grids are built
        HIPCHK(hipMemcpyAsync(c->rf_pos.p, perm, (size_t)K * sizeof(uint32_t), hipMemcpyDeviceToDevice, c->stream));
        // 3. no vertex closer than 0.7 h: vertex grid, sorted cell keys
        HIPCHK(launch_cell_keys(lo, cell, G, nullptr, c->V.p, (uint32_t)nv, c->rf_k0.p, c->rf_v0.p, c->stream));
        unsigned long long *vkeys = nullptr;
        uint32_t *vidx = sort_into(c, c->rf_k0.p, c->rf_v0.p, c->rf_k1.p, c->rf_v1.p, (uint32_t)nv, gbits, &vkeys, &he);
        HIPCHK(he);
        HIPCHK(launch_near_vertex(lo, cell, G, c->V.p, vkeys, vidx, (uint32_t)nv, c->rf_cc2.p, c->rf_src2.p,
                                  c->rf_pos.p, K, lim, c->rf_ccr.p, c->rf_srcr.p, c->rf_status.p, c->stream));
        // 4. the greedy filter among the candidates, in rounds over the candidate grid
        HIPCHK(launch_cell_keys(lo, cell, G, c->rf_ccr.p, nullptr, K, c->rf_k0.p, c->rf_v0.p, c->stream));
        unsigned long long *ckeys = nullptr;
        uint32_t *crank = sort_into(c, c->rf_k0.p, c->rf_v0.p, c->rf_k1.p, c->rf_v1.p, K, gbits, &ckeys, &he);
        HIPCHK(he);
        // the close earlier candidates of each, listed once for all the rounds
        HIPCHK(launch_filter_near(lo, cell, G, ckeys, crank, K, c->rf_ccr.p, lim, c->rf_status.p, c->rf_near.p,
                                  c->rf_nnear.p, c->stream));
        // two rounds per look at the flags: a round after the last deciding one is a pass that
        // changes nothing, cheaper than a wait for the host
        for (uint32_t round = 0;; round += 2) {
            if (round > K) return fail(c, DT_E_INTERNAL, "refinement filter did not settle");
            HIPCHK(hipMemsetAsync(c->rf_ctr.p + 2, 0, 2 * sizeof(uint32_t), c->stream));
            for (int r2 = 0; r2 < 2; ++r2)
                HIPCHK(launch_filter_round(lo, cell, G, ckeys, crank, K, c->rf_ccr.p, lim, c->rf_near.p,
                                           c->rf_nnear.p, c->rf_status.p, c->rf_ctr.p + 2 + r2, c->stream));
            uint32_t und = 0;
            HIPCHK(hipMemcpyAsync(&und, c->rf_ctr.p + 3, sizeof und, hipMemcpyDeviceToHost, c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
            if (und == 0) break;
        }
        // 5. the kept points in filter order, appended
        HIPCHK(launch_kept(c->rf_status.p, K, c->rf_flags.p, nullptr, nullptr, nullptr, nullptr, nullptr, 0,
                           c->stream));
        HIPCHK(exclusive_scan_u32(c->rf_flags.p, c->rf_pos.p, K, c->scan_tmp.p, c->rf_pos.p + K, c->stream));
        uint32_t nk = 0;
        HIPCHK(hipMemcpyAsync(&nk, c->rf_pos.p + K, sizeof nk, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        if (step_counts) {
            step_counts[2 * step] = K;
            step_counts[2 * step + 1] = nk;
        }
        if (num_steps) *num_steps = step + 1;
        if (nk == 0) break;
        if ((rc = ensure(c, c->rf_pts, 3 * (size_t)nk)) || (rc = ensure(c, c->rf_hint, nk))) return rc;
        HIPCHK(launch_kept(c->rf_status.p, K, nullptr, c->rf_pos.p, c->rf_ccr.p, c->rf_srcr.p, c->rf_pts.p,
                           c->rf_hint.p, 1, c->stream));
        // inserted as one call's cloud; each point's walk starts at a vertex of the tetrahedron
        // whose circumcentre it is (the mesher inserts a circumcentre from its tetrahedron)
        if (c->nv + nk >= (1ull << 31) || c->npoints + nk >= (1ull << 32) - 2 || nk >= (1ull << 30))
            return fail(c, DT_E_CAPACITY, "too many points (limits: 2^30 per call, 2^31 in all)");
        c->h_off = {0, nk};
        if ((rc = insert_clouds(c, c->rf_pts.p, nk, c->h_off, c->rf_hint.p))) return rc;
        total += nk;
        if (inserted) *inserted = total;
    }
    return DT_OK;
}

int dt_debug_widen_at(dt_ctx *c, uint64_t slots) {
    if (!c || slots < 4096 || slots > MAX_TETS) return DT_E_ARG;
    c->narrow_max = slots;
    return DT_OK;
}

int dt_debug_predicates(dt_ctx *c, int kind, const double *pts, const int64_t *idx, uint64_t k, int8_t *out) {
    if (!c || !pts || !out || kind < 0 || kind > 2 || (kind == 2 && !idx)) return DT_E_ARG;
    if (k == 0) return DT_OK;
    HIPCHK(hipSetDevice(c->device));
    const int np = kind == 0 ? 4 : 5;
    double *dp = nullptr;
    int64_t *di = nullptr;
    int8_t *dout = nullptr;
    HIPCHK(hipMalloc((void **)&dp, k * np * 3 * sizeof(double)));
    HIPCHK(hipMalloc((void **)&dout, k));
    if (kind == 2) HIPCHK(hipMalloc((void **)&di, k * 5 * sizeof(int64_t)));
    HIPCHK(hipMemcpyAsync(dp, pts, k * np * 3 * sizeof(double), hipMemcpyDefault, c->stream));
    if (kind == 2) HIPCHK(hipMemcpyAsync(di, idx, k * 5 * sizeof(int64_t), hipMemcpyDefault, c->stream));
    HIPCHK(launch_predicates(kind, dp, di, k, dout, c->stream));
    HIPCHK(hipMemcpyAsync(out, dout, k, hipMemcpyDefault, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    hipFree(dp);
    hipFree(dout);
    if (di) hipFree(di);
    return DT_OK;
}

}  // extern "C"
