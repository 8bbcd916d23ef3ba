// Host engine and C interface (include/ppsp.h) of the point-to-point
// shortest-path library.
//
// A call goes through four steps:
//   1. plan: turn the queries into searches (frontier copies) and query slots
//      (mu values), following Table 2 for single queries and Section 4 for
//      batches (Plain: one query at a time; Plain*: all queries at once with
//      their own searches; Multi-BiDS: one search per query-graph vertex);
//   2. split the searches into memory waves (whole queries, or whole
//      query-graph components for Multi-BiDS) that fit the state budget;
//   3. per wave: clear the state slabs, Init(), then rounds of k_round +
//      k_control until every frontier is empty, checking termination on the
//      host every `rounds_per_sync` rounds (the rounds in between are queued
//      back to back, optionally as one captured hipGraph);
//   4. read the mu slots (distance + meeting vertex) and, on request, walk
//      the parent words into s->t paths.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <deque>
#include <mutex>
#include <thread>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/ppsp.h"
#include "mlp_dev.h"
#include "ppsp_dev.h"

namespace ppsp {
hipError_t launch_init(const RoundArgs &A, hipStream_t st);
hipError_t launch_round(const RoundArgs &A, uint32_t grid, hipStream_t st, hipEvent_t e0 = nullptr,
                        hipEvent_t e1 = nullptr);
hipError_t launch_control(const RoundArgs &A, hipStream_t st);
hipError_t launch_heavy(const RoundArgs &A, uint32_t grid, hipStream_t st, hipEvent_t e0 = nullptr,
                        hipEvent_t e1 = nullptr);
hipError_t launch_admit(const RoundArgs &A, const uint32_t *ids, uint32_t k, hipStream_t st);
hipError_t launch_idle(const RoundArgs &A, hipStream_t st);
hipError_t launch_mlp_forward(const float *P, const float *X, uint32_t n, float *logits, hipStream_t st);
hipError_t launch_mlp_grad(const float *P, const float *X, const uint32_t *Y, const uint32_t *idx, uint32_t beg,
                           uint32_t end, uint32_t per, uint32_t nw, float scale, float *partial, double *loss,
                           hipStream_t st);
hipError_t launch_mlp_reduce(const float *partial, uint32_t nw, float *grad, hipStream_t st);
hipError_t launch_mlp_adam(float *P, float *m, float *v, const float *partial, uint32_t nw, float lr, uint32_t t,
                           hipStream_t st);
hipError_t launch_gather(const RoundArgs &A, const PairDesc *pd, hipStream_t st);
hipError_t launch_path_len(const RoundArgs &A, const PairDesc *pd, uint32_t *len, hipStream_t st);
hipError_t launch_path_write(const RoundArgs &A, const PairDesc *pd, const uint32_t *len, const uint64_t *off,
                             uint32_t *out, hipStream_t st);
}  // namespace ppsp

using namespace ppsp;

namespace {

extern thread_local std::string g_last_error;

// Device allocation owned by its holder (freed with it, movable, not
// copyable), or a borrowed view into the no-allocation scratch (never freed).
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    bool borrowed = false;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes), borrowed(o.borrowed) {
        o.p = nullptr;
        o.bytes = 0;
        o.borrowed = false;
    }
    DevBuf &operator=(DevBuf &&o) noexcept {
        std::swap(p, o.p);
        std::swap(bytes, o.bytes);
        std::swap(borrowed, o.borrowed);
        return *this;
    }
    ~DevBuf() { if (p && !borrowed) (void)hipFree(p); }
    template <class T> T *as() const { return (T *)p; }
};

extern thread_local std::string g_last_error;

// The no-allocation entry point (ppsp_batch_query_noalloc) serves every
// workspace buffer of its call from one fixed device region: while t_arena is
// set on the calling thread, ensure() carves 256-byte-aligned views from it
// (bump allocation) and never calls hipMalloc.
struct Arena {
    char *base = nullptr;
    uint64_t size = 0;
    uint64_t off = 0;
    uint64_t state_budget = 0;   // bytes of search state a wave may take
};
thread_local Arena *t_arena = nullptr;
// run_wave asks its caller to retry with fewer queries per wave: a frontier
// buffer overflowed and cannot grow inside the arena (internal, never returned)
constexpr int E_ARENA_RETRY = -1000;
// PPSP_REORDER without coordinates numbers the vertices above this degree
// first (the default "list_deg": the vertices whose arcs the hub-list kernel
// relaxes)
constexpr uint64_t REORDER_HUB_DEG = 128;

int ensure(DevBuf &b, size_t bytes) {
    if (bytes == 0) bytes = 8;
    if (b.bytes >= bytes) return PPSP_OK;
    if (t_arena) {
        const uint64_t o = (t_arena->off + 255) & ~255ull;
        if (o + bytes > t_arena->size) {
            // the caller retries with fewer queries per wave (or reports PPSP_E_OOM for one)
            g_last_error = "no-allocation call: " + std::to_string(bytes) + " more bytes do not fit the " +
                           std::to_string(t_arena->size) + "-byte scratch";
            return E_ARENA_RETRY;
        }
        if (b.p && !b.borrowed) (void)hipFree(b.p);
        b.p = t_arena->base + o;
        b.bytes = bytes;
        b.borrowed = true;
        t_arena->off = o + bytes;
        return PPSP_OK;
    }
    if (b.p && !b.borrowed) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
    b.borrowed = false;
    if (hipMalloc(&b.p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        g_last_error = "hipMalloc of " + std::to_string(bytes) + " bytes failed";
        return PPSP_E_OOM;
    }
    b.bytes = bytes;
    return PPSP_OK;
}

void release(DevBuf &b) {
    if (b.p && !b.borrowed) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
    b.borrowed = false;
}

thread_local std::string g_last_error;

int device_error(const char *what, hipError_t e) {
    g_last_error = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
    (void)hipGetLastError();
    return PPSP_E_DEVICE;
}

#define HIPCHK(x)                                                 \
    do {                                                          \
        hipError_t _e = (x);                                      \
        if (_e != hipSuccess) return device_error(#x, _e);        \
    } while (0)
#define CHK(x)                            \
    do {                                  \
        int _rc = (x);                    \
        if (_rc != PPSP_OK) return _rc;   \
    } while (0)

// A query slot of one wave: which searches meet in it and where the answer goes.
struct Plan {
    uint32_t G = 1;                 // searches per interleaved state group
    bool pair2 = false;             // searches 2q, 2q + 1 are query q's forward and backward copies
    std::vector<SearchDesc> sd;
    std::vector<Partner> partners;
    std::vector<PairDesc> pairs;
    std::vector<uint64_t> delta;    // per search, key units
    bool gather = false;            // read each query's distance off its root's search after the rounds
    std::vector<uint8_t> bin;       // per search: Delta-multiplier bin (learned / traced schedule)
    std::vector<uint8_t> bin_after; // per search (traced switch, empty: none): bin from sw_round on
    std::vector<uint32_t> sw_round; // per search: the round whose step first uses bin_after
    std::vector<uint32_t> qid;      // per search: index of its query among the call's distinct queries
    std::vector<uint8_t> side;      // per search: its position among its query's searches (0 forward, 1 backward)
};

// Learned or traced step schedule of the current call.
struct MlCtx {
    int mode = 0;                        // 0 off, 1 trace with fixed bins, 2 learned, 3 rho rule
    const std::vector<uint8_t> *qbin = nullptr;  // trace: bin per distinct query
    const std::vector<uint8_t> *qbin_after = nullptr;   // trace with a switch: bin from qsw on
    const std::vector<uint32_t> *qsw = nullptr;         // per distinct query: switch round
    bool nodedup = false;                // every input pair is its own query (no merging of equal pairs)
    bool dense = false;                  // dense frontiers available (switched by traced bins >= 8 or the network)
    bool rows = false;                   // trace: record feature rows
    bool collect = false;                // collect per-query rounds, arcs, entries (and rows)
    uint64_t cap = 0;                    // row capacity
    // outputs per distinct query / per row (trace)
    std::vector<uint32_t> q_rounds;
    std::vector<uint64_t> q_arcs;
    std::vector<uint64_t> q_ent;
    std::vector<float> feat;
    std::vector<uint32_t> row_q;
    std::vector<uint32_t> row_r;
    std::vector<uint8_t> row_b;
    std::vector<uint8_t> row_side;
    uint64_t rows_total = 0;             // rows produced (may exceed cap)
};

}  // namespace

struct ppsp_graph_s {
    int device = 0;
    uint32_t n = 0;
    uint64_t m = 0;
    bool symmetric = false, has_xy = false, xy_ok = false;
    uint32_t wmin = 0, wmax = 0, fb = 0, w_scale = 0;
    uint64_t ws2 = 0;
    std::vector<int32_t> h_xy;      // host copy of coordinates (device numbering, for descriptors)
    std::vector<uint32_t> perm;     // PPSP_REORDER: device id of each caller id (empty: identity)
    std::vector<uint32_t> iperm;    // caller id of each device id
    DevBuf row_ptr, arcs, xy, in_row_ptr, in_arcs;   // transpose only for a directed graph
    DevBuf hub_id, hub_vert;        // symmetric graphs with hubs: index of each vertex among them, their vertices
    uint32_t nhub = 0;
    DevBuf hmask, hrec, hgcount;    // the hub list grouped by vertex (workspace)
    // workspace (grow only)
    DevBuf tsum;                    // local-chunk time limit: 4 sums, then 2 limits
    DevBuf S, q0, q1, sd, partners, pairdesc, ctl, delta, done, exh, alive, minkey, mu, qcount, cpre, round, err,
        stats, wstats, pathlen, pathoff, pathbuf, heavy, hcount, hlim, memo;
    uint32_t maxdeg = 0;
    uint64_t hchunks = 0;           // heavy-list chunks of all vertices of degree > HEAVY_DEG
    uint64_t hchunks_at[6] = {};    // the same for degree > 16 << k (k = 0..5), for the "list_deg" option
    uint32_t hcap = 0;              // heavy list capacity (0 while no vertex exceeds HEAVY_DEG)
    hipStream_t st = nullptr;
    uint32_t *h_poll = nullptr;     // pinned
    std::vector<hipEvent_t> ev;
    ppsp_stats last{};
    int cu = 256;
    // options
    int64_t opt_profile = 0, opt_rounds_per_sync = 16, opt_grid_blocks = 0, opt_mem_budget_mb = 0,
            opt_default_delta = 0, opt_use_graph = 0, opt_timeout_ms = 600000, opt_theta_mode = 2, opt_queue_cap = 0,
            opt_ml_every = 4, opt_heavy_window = 64, opt_multi_group = 32, opt_rho = 4096, opt_local = 16, opt_local_plain = 0, opt_local_fill = 0,
            opt_min_chunk = 16, opt_local_small = 4, opt_local_pct = 90, opt_defer_pct = 105,
            opt_server_round_base = 0, opt_dense_min = 0, opt_dense_force = 0, opt_dense_ring = 16,
            opt_dense_learned = 0, opt_plain_group = 2, opt_heavy_grouped = 1, opt_heavy_claim = 4, opt_list_deg = 128, opt_heavy_waves = 24;
    uint64_t wmean = 1;             // mean arc weight (rounded up)
    uint64_t fingerprint = 0;       // hash of the CSR, keys the tuning cache
    struct Tuned {
        bool valid = false;
        uint64_t delta = 0;
        int64_t theta_mode = 2, grid = 0, hwin = 64, local = 16, dense_min = 0, dense_ring = 16;
        double ms = 0;
    } tuned[5][6];                  // per (algo, batch strategy)
    uint64_t qcap = 0;
    bool served = false;            // attached to a server, which owns the workspace
    uint32_t memo_epoch = 0;        // epoch of the last wave that used the heuristic memo
    bool memo_call = false;         // the current call memoises the heuristic (PPSP_MEMO_H)
    bool pull_call = false;         // the current call pulls before pushing (PPSP_PULL)
    // learned schedule
    DevBuf sc, bin, bin_after, sw_round, done_round, tot_arcs, tot_ent, trace, trace_s, trace_r, trace_b, trace_n, mlpw;
    // dense frontiers (options "dense_min" / "dense_force")
    DevBuf dbits, dmode, dbase, dW, dread, docc, dlist, dcount;
    bool mlp_loaded = false;
    bool ml_plain = false;          // the fit's referee preferred the plain fixed path: LEARNED runs it
    MlCtx *ml = nullptr;            // set for the duration of a learned or traced call
};

namespace {

int set_device(ppsp_graph g) {
    HIPCHK(hipSetDevice(g->device));
    return PPSP_OK;
}

// The workspace buffers of a batch (everything run_wave sizes per wave);
// a no-allocation call swaps them out for views into the scratch.
std::vector<DevBuf *> wave_buffers(ppsp_graph g) {
    return {&g->S, &g->q0, &g->q1, &g->sd, &g->partners, &g->pairdesc, &g->ctl, &g->delta, &g->done, &g->exh,
            &g->alive, &g->minkey, &g->mu, &g->qcount, &g->cpre, &g->round, &g->err, &g->stats, &g->wstats,
            &g->heavy, &g->hcount, &g->hlim, &g->tsum};
}

// Inside a no-allocation call: drop every view and start carving again.
void arena_reset(ppsp_graph g) {
    for (DevBuf *b : wave_buffers(g)) release(*b);
    t_arena->off = 0;
}

// Workgroups of the round kernel: the "grid_blocks" option, else 20 per
// compute unit, the most that are resident at once (5 waves per SIMD by
// registers, 7.4 KB of LDS each). On the 2048^2 lattice batch 16, 18 and 20
// per unit gave 5,240, 5,320 and 5,360 queries/s.
uint32_t round_grid(ppsp_graph g) {
    return g->opt_grid_blocks > 0 ? (uint32_t)g->opt_grid_blocks : (uint32_t)(20 * g->cu);
}

// The hub-list kernel takes its records from a counter, so its grid is free
// of the round kernel's (option "heavy_waves": single-wave workgroups per CU).
uint32_t heavy_grid(ppsp_graph g) {
    return g->opt_heavy_waves > 0 ? (uint32_t)(g->opt_heavy_waves * g->cu) : round_grid(g);
}

uint64_t key_delta(uint32_t kind, uint64_t d) {
    return (kind == K_2DIST || kind == K_BIDA_F || kind == K_BIDA_B) ? 2 * d : d;
}

uint64_t graph_default_delta(ppsp_graph g) {
    if (g->opt_default_delta > 0) return (uint64_t)g->opt_default_delta;
    return std::max<uint64_t>(1, 2 * g->wmean);
}

bool dense_on(ppsp_graph g) { return g->opt_dense_min > 0 || g->opt_dense_force != 0; }

// Step buckets of a dense frontier's ring ahead of its current one.
uint32_t dense_ring(ppsp_graph g) { return (uint32_t)g->opt_dense_ring; }

// 32-bit words of one dense bitmap.
uint64_t dense_words(ppsp_graph g) { return ((uint64_t)g->n + 31) / 32; }

// Hub-list chunks of the vertices that go to the list (degree above
// "list_deg", rounded down to 16 << k: never fewer than the list can hold).
uint64_t list_chunks(ppsp_graph g) {
    int k = 0;
    while (k < 5 && (16ll << (k + 1)) <= g->opt_list_deg) k++;
    return g->hchunks_at[k];
}

// Bytes of search state per search (where dense frontiers may be used: by
// size, by the learned schedule's mode output or by traced switches, plus
// its bitmaps).
uint64_t state_bytes_per_search(ppsp_graph g) {
    const bool dense = dense_on(g) || g->opt_dense_learned || (g->ml && g->ml->dense);
    return (uint64_t)g->n * 8 + (dense ? (uint64_t)(dense_ring(g) + 1) * dense_words(g) * 4 : 0);
}

uint64_t state_budget(ppsp_graph g) {
    if (t_arena) return t_arena->state_budget;
    if (g->opt_mem_budget_mb > 0) return (uint64_t)g->opt_mem_budget_mb << 20;
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) { (void)hipGetLastError(); return 1ull << 30; }
    uint64_t have = fr + g->S.bytes + g->dbits.bytes;   // reusable
    // queues (at their largest default size), the hub list, trace buffers and small buffers
    uint64_t reserve = (2ull << 30) + 2 * std::max<uint64_t>(g->qcap, 1ull << 28) * 16 +
                       (g->maxdeg > HEAVY_DEG ? (1ull << 26) * 32 : 0) + (1ull << 30);
    return have > reserve ? (uint64_t)((have - reserve) * 0.9) : (1ull << 28);
}

// Searches per wave: what the state budget holds, below 2^30 (frontier
// entries flag carried entries in bit 31 of the search index).
uint64_t search_limit(ppsp_graph g) {
    uint64_t per = state_bytes_per_search(g);
    uint64_t lim = state_budget(g) / per;
    return std::min<uint64_t>(std::max<uint64_t>(lim, 1), 1ull << 30);
}

void set_args(ppsp_graph g, RoundArgs &A, uint32_t nsearch, uint32_t npair, uint32_t G, bool pair2) {
    memset(&A, 0, sizeof(A));
    A.row_ptr = g->row_ptr.as<uint32_t>();
    A.arcs = g->arcs.as<uint2>();
    A.in_row_ptr = g->symmetric ? A.row_ptr : g->in_row_ptr.as<uint32_t>();
    A.in_arcs = g->symmetric ? A.arcs : g->in_arcs.as<uint2>();
    A.xy = g->has_xy ? g->xy.as<int2>() : nullptr;
    A.ws2 = g->ws2;
    A.fb = g->fb;
    A.n = g->n;
    A.sd = g->sd.as<SearchDesc>();
    A.partners = g->partners.as<Partner>();
    A.nsearch = nsearch;
    A.npair = npair;
    A.G = G;
    A.pair2 = pair2 ? 1u : 0u;
    A.S = g->S.as<uint64_t>();
    A.ctl = g->ctl.as<ulonglong2>();
    A.delta = g->delta.as<uint64_t>();
    A.done = g->done.as<uint32_t>();
    A.exh = g->exh.as<uint32_t>();
    A.alive = g->alive.as<uint32_t>();
    A.minkey = g->minkey.as<uint64_t>();
    A.mu = g->mu.as<uint64_t>();
    A.q0 = g->q0.as<uint4>();
    A.q1 = g->q1.as<uint4>();
    A.qcount = g->qcount.as<uint32_t>();
    A.cpre = g->cpre.as<uint32_t>();
    A.qseg = g->qcap / NSEG;
    A.round = g->round.as<uint32_t>();
    A.err = g->err.as<uint32_t>();
    A.stats = g->stats.as<unsigned long long>();
    A.wstats = g->wstats.as<unsigned long long>();
    A.heavy = g->heavy.as<uint4>();
    A.hcount = g->hcount.as<unsigned long long>();
    A.hcap = g->maxdeg > HEAVY_DEG ? g->hcap : 0;
    A.hclaim = (uint32_t)g->opt_heavy_claim;
    A.list_deg = t_arena ? HEAVY_DEG : (uint32_t)g->opt_list_deg;
    A.hlim = g->hlim.as<uint64_t>();
    A.hwin = (uint32_t)g->opt_heavy_window;
    A.local = (uint32_t)g->opt_local;
    A.local_plain = (uint32_t)g->opt_local_plain;
    A.local_fill = (uint32_t)g->opt_local_fill;
    A.min_chunk = (uint32_t)g->opt_min_chunk;
    A.local_small = (uint32_t)g->opt_local_small;
    if ((g->opt_local_pct > 0 && (g->opt_local > 0 || g->opt_local_plain > 0)) || g->opt_defer_pct > 0) {
        A.tsum = g->tsum.as<unsigned long long>();
        A.lcap = g->tsum.as<uint32_t>() + 8;             // after the 4 sums
        A.local_pct = (uint32_t)g->opt_local_pct;
        A.defer_pct = (uint32_t)g->opt_defer_pct;
    }
    A.pull = g->pull_call && g->symmetric ? 1u : 0u;
    if (g->memo_call && g->has_xy && (pair2 || G == 1)) {
        A.memo = g->memo.as<uint64_t>();
        A.epoch = g->memo_epoch;
    }
    A.theta_mode = (uint32_t)g->opt_theta_mode;
    if (g->ml && g->ml->mode) {
        A.sc = g->sc.as<unsigned long long>();
        A.ml_mode = (uint32_t)g->ml->mode;
        A.mlp = g->ml->mode == 2 ? g->mlpw.as<uint16_t>() : nullptr;
        A.bin = g->bin.as<uint8_t>();
        A.done_round = g->done_round.as<uint32_t>();
        A.tot_arcs = g->tot_arcs.as<unsigned long long>();
        A.tot_ent = g->tot_ent.as<unsigned long long>();
        if (g->ml->rows && g->ml->cap) {
            A.trace = g->trace.as<float>();
            A.trace_s = g->trace_s.as<uint32_t>();
            A.trace_r = g->trace_r.as<uint32_t>();
            A.trace_b = g->trace_b.as<uint8_t>();
            A.trace_cap = g->ml->cap;
        }
        A.trace_n = g->trace_n.as<unsigned long long>();
        A.deg_feat = g->n ? (float)(std::log2(std::max(1.0, (double)g->m / g->n)) / 4.0) : 0.f;
        A.ml_every = (uint32_t)std::max<int64_t>(1, g->opt_ml_every);
        A.rho = (uint32_t)g->opt_rho;
    }
    A.grid = round_grid(g);
}

int ensure_events(ppsp_graph g, size_t k) {
    while (g->ev.size() < k) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        g->ev.push_back(e);
    }
    return PPSP_OK;
}

struct WaveOut {
    std::vector<uint64_t> mu;       // per pair slot
    std::vector<uint32_t> path;     // concatenated paths (if requested)
    std::vector<uint64_t> path_off; // npair + 1
    unsigned long long stats[ST_N] = {0};
    double relax_ms = 0, heavy_ms = 0;  // summed durations of the timed round / hub-list launches
    uint64_t launches = 0, timed = 0;   // round-kernel launches, and those timed
    // learned / traced schedule: per search
    std::vector<uint32_t> done_round;
    std::vector<unsigned long long> tot_arcs, tot_ent;
    std::vector<float> feat;        // trace rows
    std::vector<uint32_t> row_s, row_r;
    std::vector<uint8_t> row_b;
    uint64_t rows_total = 0;
};

// Runs one wave of searches to completion.
int run_wave(ppsp_graph g, const Plan &P, bool want_path, WaveOut &out) {
    const uint32_t ns = (uint32_t)P.sd.size(), npair = (uint32_t)P.pairs.size();
    const uint64_t n = g->n;
    const uint64_t ns_words = ((uint64_t)ns + P.G - 1) / P.G * P.G;   // whole groups of G searches
    hipStream_t st = g->st;
    const uint64_t sbytes = ns_words * n * 8;
    CHK(ensure(g->S, sbytes));
    CHK(ensure(g->round, 16));
    CHK(ensure(g->hcount, 16));
    if (g->maxdeg > HEAVY_DEG) {
        // a round can extract each hub once per search; a quarter of that at once is ample
        // (inside the no-allocation scratch: a quarter of the hub chunks, at least 4,096)
        const uint64_t chunks = t_arena ? g->hchunks : list_chunks(g);
        const uint64_t want = t_arena ? std::max<uint64_t>(4096, (uint64_t)ns * chunks / 4)
                                      : std::min<uint64_t>(1u << 26, std::max<uint64_t>(1u << 20, (uint64_t)ns * chunks / 4));
        if (g->hcap < want || t_arena) g->hcap = (uint32_t)std::min<uint64_t>(want, 1u << 28);
        CHK(ensure(g->heavy, (uint64_t)g->hcap * 32));
    }
    // the hub list grouped by vertex: symmetric graphs with hubs, state groups of 4 or more searches
    const bool hgrouped = g->nhub && g->opt_heavy_grouped && P.G >= 4 && !t_arena;
    const uint64_t ngroups = ns_words / P.G;
    if (hgrouped) {
        CHK(ensure(g->hmask, 2ull * g->nhub * ngroups * 8));
        CHK(ensure(g->hrec, 2ull * g->hcap * 16));
        CHK(ensure(g->hgcount, 16));
    }
    CHK(ensure(g->sd, ns * sizeof(SearchDesc)));
    CHK(ensure(g->partners, P.partners.size() * sizeof(Partner)));
    CHK(ensure(g->pairdesc, npair * sizeof(PairDesc)));
    CHK(ensure(g->ctl, ns * 16));
    CHK(ensure(g->hlim, ns * 8));
    CHK(ensure(g->delta, ns * 8));
    CHK(ensure(g->done, ns * 4));
    CHK(ensure(g->exh, ns * 4));
    CHK(ensure(g->alive, 2 * ns * 4));
    CHK(ensure(g->minkey, 2 * ns * 8));
    CHK(ensure(g->mu, npair * 8));
    CHK(ensure(g->qcount, 2 * NSEG * 4));
    CHK(ensure(g->cpre, 2 * (NSEG + 1) * 4));
    CHK(ensure(g->tsum, 48));
    CHK(ensure(g->err, 16));
    CHK(ensure(g->stats, ST_N * 8));
    {
        // one frontier holds at most one entry per (search, vertex) plus rare duplicates
        const uint64_t want = std::min<uint64_t>(std::max<uint64_t>(std::min<uint64_t>(16384ull * ns, ns * n + 1024),
                                                                    1ull << 16), 1ull << 28);
        if (g->qcap < want && g->opt_queue_cap == 0) g->qcap = want;
    }
    const uint32_t grid = round_grid(g);
    // per-workgroup counters of both relaxing kernels (the hub-list kernel's grid may be larger)
    const uint32_t wgrid = std::max(grid, heavy_grid(g));
    CHK(ensure(g->wstats, (uint64_t)wgrid * ST_N * 8));
    if (t_arena) {
        // the two frontier queues take what the scratch has left (up to the usual size)
        const uint64_t used = ((t_arena->off + 255) & ~255ull) + 512;
        const uint64_t left = t_arena->size > used ? t_arena->size - used : 0;
        const uint64_t fit = (left / 32) / NSEG * NSEG;
        if (fit < 4096) {
            g_last_error = "no-allocation call: no room left in the scratch for the frontier queues";
            return E_ARENA_RETRY;
        }
        g->qcap = std::min<uint64_t>(g->qcap, fit);
    }
    for (;;) {
        CHK(ensure(g->q0, g->qcap * 16));
        CHK(ensure(g->q1, g->qcap * 16));
        HIPCHK(hipMemsetAsync(g->S.p, 0xFF, sbytes, st));
        if (hgrouped) {
            HIPCHK(hipMemsetAsync(g->hmask.p, 0, 2ull * g->nhub * ngroups * 8, st));
            HIPCHK(hipMemsetAsync(g->hgcount.p, 0, 16, st));
        }
        HIPCHK(hipMemcpyAsync(g->sd.p, P.sd.data(), ns * sizeof(SearchDesc), hipMemcpyHostToDevice, st));
        if (!P.partners.empty())
            HIPCHK(hipMemcpyAsync(g->partners.p, P.partners.data(), P.partners.size() * sizeof(Partner),
                                  hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(g->pairdesc.p, P.pairs.data(), npair * sizeof(PairDesc), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(g->delta.p, P.delta.data(), ns * 8, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemsetAsync(g->mu.p, 0xFF, npair * 8, st));
        HIPCHK(hipMemsetAsync(g->qcount.p, 0, 2 * NSEG * 4, st));
        HIPCHK(hipMemsetAsync(g->tsum.p, 0, 48, st));
        HIPCHK(hipMemsetAsync(g->wstats.p, 0, (uint64_t)wgrid * ST_N * 8, st));
        HIPCHK(hipMemsetAsync(g->round.p, 0, 16, st));
        HIPCHK(hipMemsetAsync(g->hcount.p, 0, 16, st));
        HIPCHK(hipMemsetAsync(g->err.p, 0, 16, st));
        HIPCHK(hipMemsetAsync(g->stats.p, 0, ST_N * 8, st));
        // dense frontiers: by size (options), or by the learned schedule's mode
        // output ("dense_learned"), or by traced switches
        const bool dense = (dense_on(g) || (g->ml && (g->ml->dense || (g->ml->mode == 2 && g->opt_dense_learned)))) &&
                           !g->pull_call;
        if ((g->ml && g->ml->mode) || dense) {
            // per-search counters (the learned / traced schedules, and the dense-mode switch)
            CHK(ensure(g->sc, 2ull * ns * 16));
            CHK(ensure(g->bin, ns));
            CHK(ensure(g->done_round, (uint64_t)ns * 4));
            CHK(ensure(g->tot_arcs, (uint64_t)ns * 8));
            CHK(ensure(g->tot_ent, (uint64_t)ns * 8));
            CHK(ensure(g->trace_n, 8));
            if (g->ml && g->ml->rows && g->ml->cap) {
                CHK(ensure(g->trace, g->ml->cap * MLP_F * 4));
                CHK(ensure(g->trace_s, g->ml->cap * 4));
                CHK(ensure(g->trace_r, g->ml->cap * 4));
                CHK(ensure(g->trace_b, g->ml->cap));
            }
            if (!P.sw_round.empty()) {
                CHK(ensure(g->bin_after, ns));
                CHK(ensure(g->sw_round, (uint64_t)ns * 4));
                HIPCHK(hipMemcpyAsync(g->bin_after.p, P.bin_after.data(), ns, hipMemcpyHostToDevice, st));
                HIPCHK(hipMemcpyAsync(g->sw_round.p, P.sw_round.data(), (uint64_t)ns * 4, hipMemcpyHostToDevice, st));
            }
            HIPCHK(hipMemsetAsync(g->sc.p, 0, 2ull * ns * 16, st));
            if (P.bin.size() == ns) HIPCHK(hipMemcpyAsync(g->bin.p, P.bin.data(), ns, hipMemcpyHostToDevice, st));
            else HIPCHK(hipMemsetAsync(g->bin.p, MLP_K / 2, ns, st));
            HIPCHK(hipMemsetAsync(g->done_round.p, 0, (uint64_t)ns * 4, st));
            HIPCHK(hipMemsetAsync(g->tot_arcs.p, 0, (uint64_t)ns * 8, st));
            HIPCHK(hipMemsetAsync(g->tot_ent.p, 0, (uint64_t)ns * 8, st));
            HIPCHK(hipMemsetAsync(g->trace_n.p, 0, 8, st));
        }
        if (g->memo_call) {
            // one word per query slot and vertex; a new epoch per wave invalidates the old words
            const uint64_t slots = P.pair2 ? (ns + 1) / 2 : ns;
            if (g->memo.bytes < slots * n * 8) {
                CHK(ensure(g->memo, slots * n * 8));
                HIPCHK(hipMemsetAsync(g->memo.p, 0, g->memo.bytes, st));
                g->memo_epoch = 0;
            }
            if (++g->memo_epoch == 0) {
                HIPCHK(hipMemsetAsync(g->memo.p, 0, g->memo.bytes, st));
                g->memo_epoch = 1;
            }
        }
        if (dense) {
            const uint64_t dw = dense_words(g);
            CHK(ensure(g->dbits, (uint64_t)ns * (dense_ring(g) + 1) * dw * 4));
            CHK(ensure(g->dmode, ns));
            CHK(ensure(g->dbase, (uint64_t)ns * 8));
            CHK(ensure(g->dW, (uint64_t)ns * 8));
            CHK(ensure(g->dread, ns));
            CHK(ensure(g->docc, (uint64_t)ns * (dense_ring(g) + 1) * 4));
            CHK(ensure(g->dlist, 2ull * ns * 4));
            CHK(ensure(g->dcount, 16));
            HIPCHK(hipMemsetAsync(g->dbits.p, 0, (uint64_t)ns * (dense_ring(g) + 1) * dw * 4, st));
            HIPCHK(hipMemsetAsync(g->docc.p, 0, (uint64_t)ns * (dense_ring(g) + 1) * 4, st));
            HIPCHK(hipMemsetAsync(g->dcount.p, 0, 16, st));
        }
        RoundArgs A;
        set_args(g, A, ns, npair, P.G, P.pair2);
        if (hgrouped) {
            A.hgrouped = 1;
            A.list_deg = HEAVY_DEG;              // grouped records index the hubs
            A.hub_id = g->hub_id.as<uint32_t>();
            A.hub_vert = g->hub_vert.as<uint32_t>();
            A.hmask = g->hmask.as<unsigned long long>();
            A.hrec = g->hrec.as<uint4>();
            A.hgcount = g->hgcount.as<unsigned long long>();
            A.nhub = g->nhub;
            A.ngroups = (uint32_t)ngroups;
        }
        if (dense) {
            if (!A.sc) {
                // counters without a learned or traced schedule (ml_mode 0: the base step)
                A.sc = g->sc.as<unsigned long long>();
                A.ml_mode = 0;
                A.bin = g->bin.as<uint8_t>();
                A.done_round = g->done_round.as<uint32_t>();
                A.tot_arcs = g->tot_arcs.as<unsigned long long>();
                A.tot_ent = g->tot_ent.as<unsigned long long>();
                A.trace_n = g->trace_n.as<unsigned long long>();
                A.ml_every = 1;
            }
            A.dbits = g->dbits.as<uint32_t>();
            A.dwords = dense_words(g);
            A.dmode = g->dmode.as<uint8_t>();
            A.dbase = g->dbase.as<uint64_t>();
            A.dW = g->dW.as<uint64_t>();
            A.dread = g->dread.as<uint8_t>();
            A.docc = g->docc.as<uint32_t>();
            A.dlist = g->dlist.as<uint32_t>();
            A.dcount = g->dcount.as<uint32_t>();
            A.dense_min = g->opt_dense_min > 0 ? (uint64_t)g->opt_dense_min : ~0ull;
            A.dring = dense_ring(g);
            A.dense_force = g->opt_dense_force ? 1u : 0u;
        }
        if (A.sc && A.ml_mode == 1 && !P.sw_round.empty()) {
            A.bin_after = g->bin_after.as<uint8_t>();
            A.sw_round = g->sw_round.as<uint32_t>();
        }
        // The time limits serve waves with local chunks: without heuristic
        // searches (and without "local_chunks_plain") they only cost (Multi-BiDS
        // on the hub lattice: 534 -> 508 queries/s), so they are off.
        {
            bool heur = false;
            for (const SearchDesc &d : P.sd) heur = heur || d.kind == K_ASTAR || d.kind == K_BIDA_F || d.kind == K_BIDA_B;
            if (!heur && g->opt_local_plain == 0) {
                A.tsum = nullptr;
                A.lcap = nullptr;
            }
        }
        HIPCHK(launch_init(A, st));
        const int K = std::max<int64_t>(1, g->opt_rounds_per_sync);
        const bool prof = g->opt_profile != 0;
        const uint64_t every = prof ? (uint64_t)g->opt_profile : 0;   // time every `every`-th launch
        if (prof) CHK(ensure_events(g, 4 * (size_t)K));
        uint64_t r = 0;
        double relax_ms = 0, heavy_ms = 0;
        uint64_t launches = 0, timed = 0;
        const auto t_start = std::chrono::steady_clock::now();
        bool timed_out = false;
        // the captured round chunk of this wave, released on every way out
        struct GraphHold {
            hipGraphExec_t exec = nullptr;
            hipGraph_t graph = nullptr;
            ~GraphHold() {
                if (exec) (void)hipGraphExecDestroy(exec);
                if (graph) (void)hipGraphDestroy(graph);
            }
        } gh;
        hipGraphExec_t &gexec = gh.exec;
        hipGraph_t &graph = gh.graph;
        if (g->opt_use_graph && !prof) {
            // Capture K rounds (K even keeps the parity pattern) once per wave.
            const int Kg = K + (K & 1);
            HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            hipError_t le = hipSuccess;
            for (int k = 0; k < Kg && le == hipSuccess; k++) {
                le = launch_round(A, grid, st);
                if (le == hipSuccess && A.hcap) le = launch_heavy(A, heavy_grid(g), st);
                if (le == hipSuccess) le = launch_control(A, st);
            }
            const hipError_t ee = hipStreamEndCapture(st, &graph);
            if (le != hipSuccess || ee != hipSuccess) {
                // a launch that failed inside the capture: end it, report that launch's error
                return device_error(le != hipSuccess ? "round launch during hipGraph capture" : "hipStreamEndCapture",
                                    le != hipSuccess ? le : ee);
            }
            if (const hipError_t ie = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0); ie != hipSuccess) {
                gexec = nullptr;
                return device_error("hipGraphInstantiate", ie);
            }
        }
        for (;;) {
            int kk, nt = 0;
            if (gexec) {
                if (const hipError_t ge = hipGraphLaunch(gexec, st); ge != hipSuccess)
                    return device_error("hipGraphLaunch", ge);
                kk = K + (K & 1);
                r += kk;
            } else {
                for (kk = 0; kk < K; kk++, r++) {
                    if (prof && r % every == 0) {
                        // the round and hub-list kernels of this round carry their own events
                        HIPCHK(launch_round(A, grid, st, g->ev[4 * nt], g->ev[4 * nt + 1]));
                        if (A.hcap) HIPCHK(launch_heavy(A, heavy_grid(g), st, g->ev[4 * nt + 2], g->ev[4 * nt + 3]));
                        nt++;
                    } else {
                        HIPCHK(launch_round(A, grid, st));
                        if (A.hcap) HIPCHK(launch_heavy(A, heavy_grid(g), st));
                    }
                    HIPCHK(launch_control(A, st));
                }
            }
            launches += kk;
            HIPCHK(hipMemcpyAsync(g->h_poll, g->qcount.p, 2 * NSEG * 4, hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(g->h_poll + 2 * NSEG, g->err.p, 4, hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(g->h_poll + 2 * NSEG + 1, g->round.p, 4, hipMemcpyDeviceToHost, st));
            g->h_poll[2 * NSEG + 2] = 0;
            if (A.dbits) HIPCHK(hipMemcpyAsync(g->h_poll + 2 * NSEG + 2, A.dcount + 2, 4, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            for (int k = 0; k < nt; k++) {
                float ms = 0;
                HIPCHK(hipEventElapsedTime(&ms, g->ev[4 * k], g->ev[4 * k + 1]));
                relax_ms += ms;
                if (A.hcap) {
                    HIPCHK(hipEventElapsedTime(&ms, g->ev[4 * k + 2], g->ev[4 * k + 3]));
                    heavy_ms += ms;
                }
            }
            timed += nt;
            uint64_t pending = g->h_poll[2 * NSEG + 2];        // dense searches still running
            const uint32_t next = g->h_poll[2 * NSEG + 1];   // round to run next
            for (uint32_t x = 0; x < (uint32_t)NSEG; x++) pending += g->h_poll[(next & 1) * NSEG + x];
            if (pending == 0 || g->h_poll[2 * NSEG] != 0) break;
            const double el = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
            if (g->opt_timeout_ms > 0 && el > (double)g->opt_timeout_ms) { timed_out = true; break; }
        }
        if (timed_out) return PPSP_E_TIMEOUT;
        const uint32_t errbits = g->h_poll[2 * NSEG];
        if (errbits & ERR_OVERFLOW) return PPSP_E_OVERFLOW;
        if ((errbits & (ERR_QUEUE | ERR_HEAVY)) && t_arena) {
            // the buffers cannot grow inside the scratch: fewer queries per wave
            g->last.retries++;
            return E_ARENA_RETRY;
        }
        if (errbits & (ERR_QUEUE | ERR_HEAVY)) {
            g->last.retries++;
            // Grow the frontier queues (or the heavy list) and rerun the wave from scratch.
            if (errbits & ERR_QUEUE) {
                uint64_t want = g->qcap * 4;
                if (want > (1ull << 31)) return PPSP_E_OOM;
                g->qcap = want;
            }
            if (errbits & ERR_HEAVY) {
                if (g->hcap >= (1u << 28)) return PPSP_E_OOM;
                g->hcap *= 4;
                CHK(ensure(g->heavy, (uint64_t)g->hcap * 32));
                if (hgrouped) CHK(ensure(g->hrec, 2ull * g->hcap * 16));
            }
            continue;
        }
        if (P.gather) HIPCHK(launch_gather(A, g->pairdesc.as<PairDesc>(), st));
        out.mu.resize(npair);
        HIPCHK(hipMemcpyAsync(out.mu.data(), g->mu.p, npair * 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(out.stats, g->stats.p, ST_N * 8, hipMemcpyDeviceToHost, st));
        std::vector<unsigned long long> ws((uint64_t)wgrid * ST_N);
        HIPCHK(hipMemcpyAsync(ws.data(), g->wstats.p, ws.size() * 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (uint64_t b = 0; b < wgrid; b++)
            for (int k = 1; k < ST_N; k++) out.stats[k] += ws[b * ST_N + k];
        if (g->ml && g->ml->collect) {
            out.done_round.resize(ns);
            out.tot_arcs.resize(ns);
            out.tot_ent.resize(ns);
            HIPCHK(hipMemcpyAsync(out.done_round.data(), g->done_round.p, (uint64_t)ns * 4, hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(out.tot_arcs.data(), g->tot_arcs.p, (uint64_t)ns * 8, hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(out.tot_ent.data(), g->tot_ent.p, (uint64_t)ns * 8, hipMemcpyDeviceToHost, st));
            unsigned long long nrow = 0;
            HIPCHK(hipMemcpyAsync(&nrow, g->trace_n.p, 8, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            out.rows_total = nrow;
            if (g->ml->rows && g->ml->cap) {
                const uint64_t keep = std::min<uint64_t>(nrow, g->ml->cap);
                out.feat.resize(keep * MLP_F);
                out.row_s.resize(keep);
                out.row_r.resize(keep);
                out.row_b.resize(keep);
                if (keep) {
                    HIPCHK(hipMemcpyAsync(out.feat.data(), g->trace.p, keep * MLP_F * 4, hipMemcpyDeviceToHost, st));
                    HIPCHK(hipMemcpyAsync(out.row_s.data(), g->trace_s.p, keep * 4, hipMemcpyDeviceToHost, st));
                    HIPCHK(hipMemcpyAsync(out.row_r.data(), g->trace_r.p, keep * 4, hipMemcpyDeviceToHost, st));
                    HIPCHK(hipMemcpyAsync(out.row_b.data(), g->trace_b.p, keep, hipMemcpyDeviceToHost, st));
                    HIPCHK(hipStreamSynchronize(st));
                }
            }
        }
        out.relax_ms = relax_ms;
        out.heavy_ms = heavy_ms;
        out.launches = launches;
        out.timed = timed;
        if (want_path) {
            CHK(ensure(g->pathlen, npair * 4));
            CHK(ensure(g->pathoff, (npair + 1) * 8));
            HIPCHK(launch_path_len(A, g->pairdesc.as<PairDesc>(), g->pathlen.as<uint32_t>(), st));
            std::vector<uint32_t> len(npair);
            HIPCHK(hipMemcpyAsync(len.data(), g->pathlen.p, npair * 4, hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(g->h_poll + 2 * NSEG, g->err.p, 4, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            if (g->h_poll[2 * NSEG] & ERR_PATH) return PPSP_E_NOPATH;
            out.path_off.assign(npair + 1, 0);
            for (uint32_t p = 0; p < npair; p++) out.path_off[p + 1] = out.path_off[p] + len[p];
            const uint64_t tot = out.path_off[npair];
            CHK(ensure(g->pathbuf, tot * 4));
            HIPCHK(hipMemcpyAsync(g->pathoff.p, out.path_off.data(), (npair + 1) * 8, hipMemcpyHostToDevice, st));
            HIPCHK(launch_path_write(A, g->pairdesc.as<PairDesc>(), g->pathlen.as<uint32_t>(),
                                     g->pathoff.as<uint64_t>(), g->pathbuf.as<uint32_t>(), st));
            out.path.resize(tot);
            if (tot) HIPCHK(hipMemcpyAsync(out.path.data(), g->pathbuf.p, tot * 4, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
        }
        return PPSP_OK;
    }
}

// ---- planning ---------------------------------------------------------------

bool is_bidir(uint32_t algo) { return algo == PPSP_BIDS || algo == PPSP_BIDASTAR; }
bool is_astar(uint32_t algo) { return algo == PPSP_ASTAR || algo == PPSP_BIDASTAR; }

SearchDesc make_sd(ppsp_graph g, uint32_t src, uint32_t kind, uint32_t s, uint32_t t) {
    SearchDesc d;
    memset(&d, 0, sizeof(d));
    d.src = src;
    d.kind = kind;
    if (g->has_xy) {
        d.tx = g->h_xy[2 * (uint64_t)t];
        d.ty = g->h_xy[2 * (uint64_t)t + 1];
        d.sx = g->h_xy[2 * (uint64_t)s];
        d.sy = g->h_xy[2 * (uint64_t)s + 1];
    }
    return d;
}

// Adds the searches of one query (s, t) for a single-query algorithm.
void plan_single(ppsp_graph g, Plan &P, uint32_t s, uint32_t t, uint32_t algo, uint64_t delta) {
    const uint32_t pair = (uint32_t)P.pairs.size();
    const uint32_t a = (uint32_t)P.sd.size();
    if (is_bidir(algo)) {
        const uint32_t kf = algo == PPSP_BIDS ? K_2DIST : K_BIDA_F;
        const uint32_t kb = algo == PPSP_BIDS ? K_2DIST : K_BIDA_B;
        SearchDesc f = make_sd(g, s, kf, s, t), b = make_sd(g, t, kb, s, t);
        b.rev = g->symmetric ? 0u : 1u;      // on a directed graph the backward search walks the transpose
        f.pbeg = (uint32_t)P.partners.size();
        P.partners.push_back({a + 1, pair});
        f.pend = (uint32_t)P.partners.size();
        b.pbeg = (uint32_t)P.partners.size();
        P.partners.push_back({a, pair});
        b.pend = (uint32_t)P.partners.size();
        P.sd.push_back(f);
        P.sd.push_back(b);
        P.delta.push_back(key_delta(kf, delta));
        P.delta.push_back(key_delta(kb, delta));
        P.pairs.push_back({a, a + 1});
    } else {
        const uint32_t k = algo == PPSP_ASTAR ? K_ASTAR : K_DIST;
        SearchDesc f = make_sd(g, s, k, s, t);
        f.noprune = algo == PPSP_SSSP;
        f.pbeg = (uint32_t)P.partners.size();
        P.partners.push_back({TARGET_BIT | t, pair});
        f.pend = (uint32_t)P.partners.size();
        P.sd.push_back(f);
        P.delta.push_back(key_delta(k, delta));
        P.pairs.push_back({a, TARGET_BIT | t});
    }
}

int check_opts(ppsp_graph g, const ppsp_opts *o) {
    if (!o) return PPSP_E_INVALID;
    if (o->algo > PPSP_BIDASTAR || o->batch > PPSP_BATCH_AUTO || o->sched > PPSP_SCHED_RHO) return PPSP_E_INVALID;
    if (is_astar(o->algo) && !g->xy_ok) return PPSP_E_NOCOORD;
    // directed graphs: backward searches run on the transpose, and the query
    // graph of the shared-search strategies is bipartite (sources, targets)
    if ((o->batch == PPSP_BATCH_MULTI || o->batch == PPSP_BATCH_AUTO) && o->algo != PPSP_BIDS) return PPSP_E_INVALID;
    if ((o->batch == PPSP_BATCH_SSSP || o->batch == PPSP_BATCH_VC) && o->algo != PPSP_SSSP) return PPSP_E_INVALID;
    if ((o->flags & PPSP_WANT_PATH) && g->wmin == 0 && g->m > 0) return PPSP_E_NOPATH;
    if (o->sched == PPSP_SCHED_LEARNED && !g->mlp_loaded) return PPSP_E_INVALID;
    return PPSP_OK;
}

struct Query {
    uint32_t s, t;
};

// Answers for distinct canonical queries, then scattered to the input order.
struct Answer {
    uint64_t dist = PPSP_INF;
    std::vector<uint32_t> path;
};

void accumulate(ppsp_graph g, const WaveOut &w) {
    g->last.rounds += w.stats[ST_ROUNDS];
    g->last.entries += w.stats[ST_ENTRIES];
    g->last.scanned_vertices += w.stats[ST_SCANV];
    g->last.scanned_arcs += w.stats[ST_SCANE];
    g->last.relax_success += w.stats[ST_SUCC] + w.stats[ST_HSUCC];
    g->last.heavy_success += w.stats[ST_HSUCC];
    g->last.carried += w.stats[ST_CARRY];
    g->last.relax_kernel_ms += w.relax_ms;
    g->last.relax_launches += w.launches;
    g->last.relax_timed += w.timed;
    g->last.heavy_kernel_ms += w.heavy_ms;
    g->last.heavy_arcs += w.stats[ST_HEAVYE];
    g->last.heavy_chunks += w.stats[ST_HCHUNK];
    g->last.dense_searches += w.stats[ST_DENSE];
    g->last.waves += 1;
}

// Copies wave results for pair slots [0, npair) into answers idx[...].
void collect(const WaveOut &w, const std::vector<uint32_t> &ans_of_pair, std::vector<Answer> &ans, bool want_path) {
    for (size_t p = 0; p < ans_of_pair.size(); p++) {
        Answer &a = ans[ans_of_pair[p]];
        const uint32_t d32 = (uint32_t)(w.mu[p] >> 32);
        a.dist = d32 == INF32 ? PPSP_INF : d32;
        if (want_path && d32 != INF32)
            a.path.assign(w.path.begin() + w.path_off[p], w.path.begin() + w.path_off[p + 1]);
    }
}

// Runs distinct queries with Plain / Plain* (each query owns its searches).
int run_independent(ppsp_graph g, const std::vector<Query> &qs, const ppsp_opts *o, uint64_t delta,
                    std::vector<Answer> &ans) {
    const bool want_path = o->flags & PPSP_WANT_PATH;
    const uint32_t per = is_bidir(o->algo) ? 2 : 1;
    // queries per wave; the heuristic memo adds one 8-byte word per query and vertex (one search's worth)
    uint64_t lim = o->batch == PPSP_BATCH_PLAIN ? 1
                   : std::max<uint64_t>(1, search_limit(g) / (per + (g->memo_call ? 1 : 0)));
    // bidirectional: G / 2 queries per state group (option "plain_group"); a
    // wave holds whole groups, and one too small for a group uses groups of one query
    uint32_t grp = 2;
    if (per == 2 && o->batch != PPSP_BATCH_PLAIN) {
        const uint64_t qpg = (uint64_t)g->opt_plain_group / 2;
        if (lim >= qpg) {
            grp = (uint32_t)g->opt_plain_group;
            lim = lim / qpg * qpg;
        }
    }
    for (size_t q0 = 0; q0 < qs.size(); q0 += lim) {
        const size_t q1 = std::min<size_t>(qs.size(), q0 + lim);
        if (t_arena) arena_reset(g);
        Plan P;
        P.G = per == 2 ? grp : 1;
        P.pair2 = per == 2;
        std::vector<uint32_t> ans_of_pair;
        for (size_t q = q0; q < q1; q++) {
            const size_t a = P.sd.size();
            plan_single(g, P, qs[q].s, qs[q].t, o->algo, delta);
            ans_of_pair.push_back((uint32_t)q);
            const bool traced = g->ml && g->ml->mode == 1;
            const uint8_t b = traced ? (*g->ml->qbin)[q] : (uint8_t)(MLP_K / 2);
            for (size_t i = a; i < P.sd.size(); i++) {
                P.bin.push_back(b);
                P.qid.push_back((uint32_t)q);
                P.side.push_back((uint8_t)(i - a));
                if (traced && g->ml->qsw) {
                    P.bin_after.push_back((*g->ml->qbin_after)[q]);
                    P.sw_round.push_back((*g->ml->qsw)[q]);
                }
            }
        }
        g->last.searches += P.sd.size();
        WaveOut w;
        const int rc = run_wave(g, P, want_path, w);
        if (rc == E_ARENA_RETRY) {
            // inside the no-allocation scratch: the same queries again in smaller waves
            if (q1 - q0 == 1) {
                g_last_error = "no-allocation call: one query's frontier does not fit the scratch";
                return PPSP_E_OOM;
            }
            g->last.searches -= P.sd.size();
            lim = std::max<uint64_t>(1, (q1 - q0) / 2);
            q0 -= lim;          // the loop adds lim back: the same first query
            continue;
        }
        CHK(rc);
        accumulate(g, w);
        collect(w, ans_of_pair, ans, want_path);
        if (g->ml && g->ml->collect) {
            MlCtx &c = *g->ml;
            for (size_t i = 0; i < P.sd.size(); i++) {
                const uint32_t q = P.qid[i];
                c.q_rounds[q] = std::max(c.q_rounds[q], w.done_round[i]);
                c.q_arcs[q] += w.tot_arcs[i];
                c.q_ent[q] += w.tot_ent[i];
            }
            c.rows_total += w.rows_total;
            for (size_t r = 0; r < w.row_s.size() && c.row_q.size() < c.cap; r++) {
                c.row_q.push_back(P.qid[w.row_s[r]]);
                c.row_r.push_back(w.row_r[r]);
                c.row_b.push_back(w.row_b[r]);
                c.row_side.push_back(P.side[w.row_s[r]]);
                c.feat.insert(c.feat.end(), w.feat.begin() + r * MLP_F, w.feat.begin() + (r + 1) * MLP_F);
            }
        }
    }
    return PPSP_OK;
}

// Multi-BiDS (Section 4.2): searches are the query-graph vertices, waves are
// unions of whole query-graph components. On a directed graph the query
// graph is bipartite (Appendix on directed graphs): a source gets a forward
// search, a target a backward search on the transpose, and a vertex that is
// both gets both.
int run_multi(ppsp_graph g, const std::vector<Query> &qs, const ppsp_opts *o, uint64_t delta,
              std::vector<Answer> &ans) {
    const bool want_path = o->flags & PPSP_WANT_PATH;
    // query graph G_q: vertex ids and adjacency (Section 4.1); a vertex id
    // carries its direction (always forward on a symmetric graph)
    std::unordered_map<uint64_t, uint32_t> vid;
    std::vector<uint32_t> verts;
    std::vector<uint8_t> vrev;
    auto id_of = [&](uint32_t v, uint8_t rev) {
        const uint64_t key = ((uint64_t)rev << 32) | v;
        auto it = vid.find(key);
        if (it != vid.end()) return it->second;
        uint32_t k = (uint32_t)verts.size();
        vid.emplace(key, k);
        verts.push_back(v);
        vrev.push_back(rev);
        return k;
    };
    const uint8_t trev = g->symmetric ? 0 : 1;
    std::vector<std::pair<uint32_t, uint32_t>> qe(qs.size());
    for (size_t q = 0; q < qs.size(); q++) qe[q] = {id_of(qs[q].s, 0), id_of(qs[q].t, trev)};
    const uint32_t nv = (uint32_t)verts.size();
    // components (union-find)
    std::vector<uint32_t> par(nv);
    std::iota(par.begin(), par.end(), 0u);
    auto find = [&](uint32_t x) {
        while (par[x] != x) { par[x] = par[par[x]]; x = par[x]; }
        return x;
    };
    for (auto &e : qe) {
        uint32_t a = find(e.first), b = find(e.second);
        if (a != b) par[std::max(a, b)] = std::min(a, b);
    }
    std::map<uint32_t, std::vector<uint32_t>> comp_verts, comp_queries;
    for (uint32_t v = 0; v < nv; v++) comp_verts[find(v)].push_back(v);
    for (size_t q = 0; q < qe.size(); q++) comp_queries[find(qe[q].first)].push_back((uint32_t)q);
    const uint64_t lim = search_limit(g);
    std::vector<uint32_t> wave_comps;
    uint64_t wave_size = 0;
    auto flush = [&]() -> int {
        if (wave_comps.empty()) return PPSP_OK;
        Plan P;
        P.G = (uint32_t)g->opt_multi_group;
        std::vector<uint32_t> local(nv, UINT32_MAX);
        for (uint32_t c : wave_comps)
            for (uint32_t v : comp_verts[c]) {
                local[v] = (uint32_t)P.sd.size();
                P.sd.push_back(make_sd(g, verts[v], K_2DIST, verts[v], verts[v]));
                P.sd.back().rev = vrev[v];
                P.delta.push_back(key_delta(K_2DIST, delta));
                P.bin.push_back((uint8_t)(MLP_K / 2));
            }
        // adjacency with pair slots
        std::vector<std::vector<Partner>> adj(P.sd.size());
        std::vector<uint32_t> ans_of_pair;
        for (uint32_t c : wave_comps)
            for (uint32_t q : comp_queries[c]) {
                const uint32_t a = local[qe[q].first], b = local[qe[q].second];
                const uint32_t slot = (uint32_t)P.pairs.size();
                P.pairs.push_back({a, b});
                adj[a].push_back({b, slot});
                adj[b].push_back({a, slot});
                ans_of_pair.push_back(q);
            }
        for (size_t i = 0; i < P.sd.size(); i++) {
            P.sd[i].pbeg = (uint32_t)P.partners.size();
            P.partners.insert(P.partners.end(), adj[i].begin(), adj[i].end());
            P.sd[i].pend = (uint32_t)P.partners.size();
        }
        g->last.searches += P.sd.size();
        WaveOut w;
        CHK(run_wave(g, P, want_path, w));
        accumulate(g, w);
        collect(w, ans_of_pair, ans, want_path);
        wave_comps.clear();
        wave_size = 0;
        return PPSP_OK;
    };
    for (auto &kv : comp_verts) {
        const uint64_t sz = kv.second.size();
        if (sz > lim) {
            // a component larger than the budget: answer its queries with Plain*
            CHK(flush());
            std::vector<Query> sub;
            std::vector<uint32_t> ids;
            for (uint32_t q : comp_queries[kv.first]) { sub.push_back(qs[q]); ids.push_back(q); }
            std::vector<Answer> sa(sub.size());
            ppsp_opts o2 = *o;
            o2.batch = PPSP_BATCH_PLAINSTAR;
            CHK(run_independent(g, sub, &o2, delta, sa));
            for (size_t j = 0; j < ids.size(); j++) ans[ids[j]] = sa[j];
            continue;
        }
        if (wave_size + sz > lim) CHK(flush());
        wave_comps.push_back(kv.first);
        wave_size += sz;
    }
    return flush();
}

// Minimum vertex cover of a bipartite graph (left: nl sources, right: nr
// targets, one edge per query) by Koenig's theorem: a maximum matching
// (Hopcroft-Karp: BFS layers from the free left vertices, then vertex-
// disjoint shortest augmenting paths by DFS, repeated until none is left),
// then Z = the vertices reachable from free left vertices by alternating
// paths; the cover is (left \ Z) + (right in Z). Returns, per edge, 1 if its
// left endpoint covers it (else its right endpoint does).
std::vector<uint8_t> bipartite_cover(uint32_t nl, uint32_t nr, const std::vector<std::pair<uint32_t, uint32_t>> &e) {
    const uint32_t NIL = UINT32_MAX, FAR = UINT32_MAX;
    std::vector<std::vector<uint32_t>> adj(nl);
    for (const auto &x : e) adj[x.first].push_back(x.second);
    std::vector<uint32_t> ml(nl, NIL), mr(nr, NIL), lay(nl, FAR);
    auto layers = [&]() {
        std::deque<uint32_t> Q;
        bool free_right = false;
        for (uint32_t u = 0; u < nl; u++) {
            lay[u] = ml[u] == NIL ? 0 : FAR;
            if (ml[u] == NIL) Q.push_back(u);
        }
        while (!Q.empty()) {
            const uint32_t u = Q.front();
            Q.pop_front();
            for (uint32_t v : adj[u]) {
                const uint32_t w = mr[v];
                if (w == NIL) free_right = true;
                else if (lay[w] == FAR) { lay[w] = lay[u] + 1; Q.push_back(w); }
            }
        }
        return free_right;
    };
    // One augmenting path from free left vertex r along the layers (iterative
    // DFS: st holds (left vertex, next arc), via the right vertices taken).
    auto augment = [&](uint32_t r) {
        std::vector<std::pair<uint32_t, size_t>> st{{r, 0}};
        std::vector<uint32_t> via;
        while (!st.empty()) {
            const uint32_t u = st.back().first;
            const size_t k = st.back().second;
            if (k == adj[u].size()) {
                lay[u] = FAR;                  // dead end for this phase
                st.pop_back();
                if (!via.empty()) via.pop_back();
                continue;
            }
            st.back().second = k + 1;
            const uint32_t v = adj[u][k], w = mr[v];
            if (w == NIL) {
                via.push_back(v);
                for (size_t j = 0; j < st.size(); j++) {
                    ml[st[j].first] = via[j];
                    mr[via[j]] = st[j].first;
                }
                return true;
            }
            if (lay[w] != FAR && lay[w] == lay[u] + 1) {
                via.push_back(v);
                st.push_back({w, 0});
            }
        }
        return false;
    };
    while (layers())
        for (uint32_t u = 0; u < nl; u++)
            if (ml[u] == NIL) augment(u);
    std::vector<uint8_t> zl(nl, 0), zr(nr, 0);
    std::deque<uint32_t> Q;
    for (uint32_t u = 0; u < nl; u++)
        if (ml[u] == NIL) { zl[u] = 1; Q.push_back(u); }
    while (!Q.empty()) {
        const uint32_t u = Q.front();
        Q.pop_front();
        for (uint32_t v : adj[u]) {
            if (ml[u] == v || zr[v]) continue;
            zr[v] = 1;
            const uint32_t w = mr[v];
            if (w != NIL && !zl[w]) { zl[w] = 1; Q.push_back(w); }
        }
    }
    std::vector<uint8_t> by_left(e.size());
    for (size_t q = 0; q < e.size(); q++) by_left[q] = zl[e[q].first] ? 0 : 1;
    return by_left;
}

// A vertex cover of the query graph (edges = queries). Undirected: exact
// minimum per connected component of at most 16 vertices (smallest mask
// among the minimum ones), greedy by uncovered degree otherwise. Directed:
// the query graph is bipartite (sources, targets) and its minimum cover is
// exact (bipartite_cover). Returns, per query, the cover endpoint that
// answers it; rev[q] = 1 when that endpoint is the target of a directed
// query (a backward search on the transpose).
std::vector<uint32_t> query_cover(const std::vector<Query> &qs, bool directed, std::vector<uint8_t> &rev) {
    rev.assign(qs.size(), 0);
    if (directed) {
        std::unordered_map<uint32_t, uint32_t> lid, rid;
        std::vector<std::pair<uint32_t, uint32_t>> e(qs.size());
        for (size_t q = 0; q < qs.size(); q++) {
            const uint32_t a = lid.emplace(qs[q].s, (uint32_t)lid.size()).first->second;
            const uint32_t b = rid.emplace(qs[q].t, (uint32_t)rid.size()).first->second;
            e[q] = {a, b};
        }
        const std::vector<uint8_t> by_left = bipartite_cover((uint32_t)lid.size(), (uint32_t)rid.size(), e);
        std::vector<uint32_t> by(qs.size());
        for (size_t q = 0; q < qs.size(); q++) {
            by[q] = by_left[q] ? qs[q].s : qs[q].t;
            rev[q] = by_left[q] ? 0 : 1;
        }
        return by;
    }
    std::unordered_map<uint32_t, uint32_t> vid;
    std::vector<uint32_t> verts;
    auto id_of = [&](uint32_t v) {
        auto it = vid.find(v);
        if (it != vid.end()) return it->second;
        vid.emplace(v, (uint32_t)verts.size());
        verts.push_back(v);
        return (uint32_t)verts.size() - 1;
    };
    const size_t nq = qs.size();
    std::vector<std::pair<uint32_t, uint32_t>> e(nq);
    for (size_t q = 0; q < nq; q++) e[q] = {id_of(qs[q].s), id_of(qs[q].t)};
    const uint32_t nv = (uint32_t)verts.size();
    std::vector<std::vector<uint32_t>> adj(nv);
    for (size_t q = 0; q < nq; q++) {
        adj[e[q].first].push_back((uint32_t)q);
        adj[e[q].second].push_back((uint32_t)q);
    }
    std::vector<uint32_t> by(nq, UINT32_MAX);
    std::vector<int> comp(nv, -1);
    for (uint32_t r = 0; r < nv; r++) {
        if (comp[r] >= 0) continue;
        std::vector<uint32_t> cv{r}, cq;
        comp[r] = (int)r;
        for (size_t h = 0; h < cv.size(); h++)
            for (uint32_t q : adj[cv[h]]) {
                const uint32_t o = e[q].first == cv[h] ? e[q].second : e[q].first;
                if (comp[o] < 0) { comp[o] = (int)r; cv.push_back(o); }
            }
        for (uint32_t v : cv)
            for (uint32_t q : adj[v])
                if (e[q].first == v) cq.push_back(q);
        if (cv.size() <= 16) {
            std::unordered_map<uint32_t, uint32_t> loc;
            for (uint32_t j = 0; j < cv.size(); j++) loc[cv[j]] = j;
            uint32_t best = 0, bestc = 99;
            for (uint32_t m = 0; m < (1u << cv.size()); m++) {
                const uint32_t c = (uint32_t)__builtin_popcount(m);
                if (c >= bestc) continue;
                bool ok = true;
                for (uint32_t q : cq)
                    if (!((m >> loc[e[q].first]) & 1) && !((m >> loc[e[q].second]) & 1)) { ok = false; break; }
                if (ok) { best = m; bestc = c; }
            }
            for (uint32_t q : cq)
                by[q] = ((best >> loc[e[q].first]) & 1) ? verts[e[q].first] : verts[e[q].second];
        } else {
            std::map<std::pair<uint32_t, uint32_t>, uint32_t> heap;   // (-degree, vertex)
            std::unordered_map<uint32_t, uint32_t> deg;
            for (uint32_t v : cv) {
                deg[v] = (uint32_t)adj[v].size();
                heap[{UINT32_MAX - deg[v], v}] = v;
            }
            while (!heap.empty()) {
                const uint32_t v = heap.begin()->second;
                heap.erase(heap.begin());
                if (deg[v] == 0) continue;
                for (uint32_t q : adj[v]) {
                    if (by[q] != UINT32_MAX) continue;
                    by[q] = verts[v];
                    const uint32_t o = e[q].first == v ? e[q].second : e[q].first;
                    heap.erase({UINT32_MAX - deg[o], o});
                    deg[o]--;
                    heap[{UINT32_MAX - deg[o], o}] = o;
                }
                deg[v] = 0;
            }
        }
    }
    return by;
}

// Plain-SSSP and VC-SSSP (Section 4.3): one search without pruning per root,
// each query read off its root's search (a gather after the rounds).
int run_cover(ppsp_graph g, const std::vector<Query> &qs, const ppsp_opts *o, uint64_t delta,
              std::vector<Answer> &ans, const std::vector<uint32_t> &root_of, const std::vector<uint8_t> &root_rev) {
    const bool want_path = o->flags & PPSP_WANT_PATH;
    // roots keyed by (direction, vertex): a backward root walks the transpose
    std::map<uint64_t, std::vector<uint32_t>> by_root;
    for (size_t q = 0; q < qs.size(); q++)
        by_root[((uint64_t)root_rev[q] << 32) | root_of[q]].push_back((uint32_t)q);
    std::vector<uint64_t> roots;
    for (auto &kv : by_root) roots.push_back(kv.first);
    const uint64_t lim = std::max<uint64_t>(1, search_limit(g));
    for (size_t r0 = 0; r0 < roots.size(); r0 += lim) {
        const size_t r1 = std::min<size_t>(roots.size(), r0 + lim);
        Plan P;
        P.G = 1;
        P.gather = true;
        std::vector<uint32_t> ans_of_pair;
        for (size_t r = r0; r < r1; r++) {
            const uint32_t root = (uint32_t)roots[r];
            const uint32_t a = (uint32_t)P.sd.size();
            SearchDesc sd = make_sd(g, root, K_DIST, root, root);
            sd.rev = (uint32_t)(roots[r] >> 32);
            sd.noprune = 1;
            sd.pbeg = sd.pend = 0;
            P.sd.push_back(sd);
            P.delta.push_back(key_delta(K_DIST, delta));
            P.bin.push_back((uint8_t)(MLP_K / 2));
            for (uint32_t q : by_root[roots[r]]) {
                const uint32_t other = qs[q].s == root ? qs[q].t : qs[q].s;
                P.pairs.push_back({a, TARGET_BIT | other});
                ans_of_pair.push_back(q);
            }
        }
        g->last.searches += P.sd.size();
        WaveOut w;
        CHK(run_wave(g, P, want_path, w));
        accumulate(g, w);
        collect(w, ans_of_pair, ans, want_path);
        if (want_path)
            for (uint32_t q : ans_of_pair)
                if (root_of[q] != qs[q].s) std::reverse(ans[q].path.begin(), ans[q].path.end());
    }
    return PPSP_OK;
}

int batch_impl(ppsp_graph g, const uint32_t *pairs, uint32_t k, const ppsp_opts *o, void *hip_stream,
               uint64_t *dist, uint64_t *path_off, uint32_t *path_vtx, uint64_t path_cap, uint32_t *need_out) {
    auto t0 = std::chrono::steady_clock::now();
    if (!g || (!pairs && k) || (!dist && k)) return PPSP_E_INVALID;
    if (g->served) return PPSP_E_BUSY;
    CHK(check_opts(g, o));
    const bool want_path = o->flags & PPSP_WANT_PATH;
    if (want_path && (!path_off || (!path_vtx && path_cap))) return PPSP_E_INVALID;
    for (uint64_t i = 0; i < 2ull * k; i++)
        if (pairs[i] >= g->n) return PPSP_E_RANGE;
    // PPSP_REORDER: caller ids -> device ids (paths are translated back below)
    std::vector<uint32_t> mapped;
    const uint32_t *caller_pairs = pairs;
    if (!g->perm.empty()) {
        mapped.resize(2ull * k);
        for (uint64_t i = 0; i < 2ull * k; i++) mapped[i] = g->perm[pairs[i]];
        pairs = mapped.data();
    }
    CHK(set_device(g));
    g->last = ppsp_stats{};
    // order the library stream after the caller's stream (a no-allocation
    // call runs on the caller's stream itself)
    if (!t_arena) {
        hipEvent_t ev;
        HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        HIPCHK(hipEventRecord(ev, (hipStream_t)hip_stream));
        HIPCHK(hipStreamWaitEvent(g->st, ev, 0));
        (void)hipEventDestroy(ev);
    }
    uint64_t delta = o->delta ? o->delta : graph_default_delta(g);
    // PPSP_SCHED_AUTOTUNED: the threshold rule, Delta and launch shape that
    // ppsp_tune chose for this algorithm and batch strategy.
    struct Restore {
        ppsp_graph g;
        int64_t mode, grid, hwin, local, dmin, dring;
        ~Restore() {
            g->opt_theta_mode = mode;
            g->opt_grid_blocks = grid;
            g->opt_heavy_window = hwin;
            g->opt_local = local;
            g->opt_dense_min = dmin;
            g->opt_dense_ring = dring;
        }
    } restore{g, g->opt_theta_mode, g->opt_grid_blocks, g->opt_heavy_window, g->opt_local, g->opt_dense_min,
              g->opt_dense_ring};
    if (o->sched == PPSP_SCHED_AUTOTUNED && g->tuned[o->algo][o->batch].valid) {
        const auto &t = g->tuned[o->algo][o->batch];
        delta = t.delta;
        g->opt_theta_mode = t.theta_mode;
        g->opt_grid_blocks = t.grid;
        g->opt_heavy_window = t.hwin;
        g->opt_local = t.local;
        g->opt_dense_min = t.dense_min;
        g->opt_dense_ring = t.dense_ring;
    }
    struct MemoRestore {
        ppsp_graph g;
        ~MemoRestore() { g->memo_call = false; g->pull_call = false; }
    } memorestore{g};
    g->pull_call = (o->flags & PPSP_PULL) != 0;
    g->memo_call = (o->flags & PPSP_MEMO_H) && is_astar(o->algo) &&
                   (o->batch == PPSP_BATCH_PLAIN || o->batch == PPSP_BATCH_PLAINSTAR);
    // PPSP_SCHED_LEARNED: the loaded network picks each search's step
    // (a trace call has set its own context already).
    MlCtx learned;
    struct MlRestore {
        ppsp_graph g;
        bool set;
        ~MlRestore() { if (set) g->ml = nullptr; }
    } mlrestore{g, false};
    if ((o->sched == PPSP_SCHED_RHO || (o->sched == PPSP_SCHED_LEARNED && !g->ml_plain)) && !g->ml) {
        learned.mode = o->sched == PPSP_SCHED_LEARNED ? 2 : 3;
        g->ml = &learned;
        mlrestore.set = true;
    }
    // distinct queries; on symmetric graphs (t,s) is the same query as (s,t)
    std::vector<Query> qs;
    std::vector<uint32_t> qidx(k);
    std::vector<uint8_t> flip(k, 0), self(k, 0);
    {
        std::unordered_map<uint64_t, uint32_t> seen;
        for (uint32_t i = 0; i < k; i++) {
            uint32_t s = pairs[2 * i], t = pairs[2 * i + 1];
            if (s == t) { self[i] = 1; continue; }
            if (g->symmetric && s > t && o->algo != PPSP_SSSP) { std::swap(s, t); flip[i] = 1; }
            if (g->ml && g->ml->nodedup) {            // every pair its own query (traced variants)
                qidx[i] = (uint32_t)qs.size();
                qs.push_back({s, t});
                continue;
            }
            const uint64_t key = ((uint64_t)s << 32) | t;
            auto it = seen.find(key);
            if (it == seen.end()) {
                it = seen.emplace(key, (uint32_t)qs.size()).first;
                qs.push_back({s, t});
            }
            qidx[i] = it->second;
        }
    }
    std::vector<Answer> ans(qs.size());
    if (!qs.empty()) {
        if (o->batch == PPSP_BATCH_SSSP) {
            std::vector<uint32_t> root_of(qs.size());
            for (size_t q = 0; q < qs.size(); q++) root_of[q] = qs[q].s;
            CHK(run_cover(g, qs, o, delta, ans, root_of, std::vector<uint8_t>(qs.size(), 0)));
        } else if (o->batch == PPSP_BATCH_VC || o->batch == PPSP_BATCH_AUTO) {
            std::vector<uint8_t> root_rev;
            const std::vector<uint32_t> root_of = query_cover(qs, !g->symmetric, root_rev);
            // query-graph vertices and cover vertices, with their direction on a directed graph
            const uint64_t tdir = g->symmetric ? 0 : 1ull << 32;
            std::unordered_map<uint64_t, char> cover, vq;
            for (size_t q = 0; q < qs.size(); q++) {
                cover[((uint64_t)root_rev[q] << 32) | root_of[q]] = 1;
                vq[qs[q].s] = 1;
                vq[tdir | qs[q].t] = 1;
            }
            if (o->batch == PPSP_BATCH_VC || 4 * cover.size() <= vq.size()) {
                ppsp_opts oo = *o;
                oo.algo = PPSP_SSSP;
                CHK(run_cover(g, qs, &oo, delta, ans, root_of, root_rev));
            } else {
                ppsp_opts oo = *o;
                oo.batch = PPSP_BATCH_MULTI;
                CHK(run_multi(g, qs, &oo, delta, ans));
            }
        } else if (o->batch == PPSP_BATCH_MULTI) {
            CHK(run_multi(g, qs, o, delta, ans));
        } else {
            CHK(run_independent(g, qs, o, delta, ans));
        }
    }
    // scatter
    uint64_t need = 0;
    for (uint32_t i = 0; i < k; i++) {
        if (self[i]) need += 1;
        else need += ans[qidx[i]].path.size();
    }
    if (want_path && need > path_cap) {
        if (need_out) *need_out = (uint32_t)std::min<uint64_t>(need, UINT32_MAX);
        return PPSP_E_PATHCAP;
    }
    uint64_t off = 0;
    const bool re = !g->iperm.empty();
    for (uint32_t i = 0; i < k; i++) {
        if (self[i]) {
            dist[i] = 0;
            if (want_path) { path_off[i] = off; path_vtx[off++] = caller_pairs[2 * i]; }
            continue;
        }
        const Answer &a = ans[qidx[i]];
        dist[i] = a.dist;
        if (want_path) {
            path_off[i] = off;
            if (flip[i]) for (size_t j = a.path.size(); j-- > 0;) path_vtx[off++] = re ? g->iperm[a.path[j]] : a.path[j];
            else for (uint32_t v : a.path) path_vtx[off++] = re ? g->iperm[v] : v;
        }
    }
    if (want_path) path_off[k] = off;
    g->last.wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return PPSP_OK;
}

}  // namespace

// ---- learned schedule: tracing, training, fitting ------------------------------

// What a traced batch records (host arrays sized by the caller).
struct TraceReq {
    const uint8_t *bins = nullptr;         // per pair: bin (NULL: 4)
    const uint8_t *bins_after = nullptr;   // per pair: bin from switch_round on
    const uint32_t *switch_round = nullptr;
    bool network = false;                  // the loaded network picks the bins
    bool distinct = false;                 // every pair its own query
    bool rows = false;
    uint64_t cap = 0;
};
struct TraceOut {
    std::vector<uint32_t> row_pair, row_round;
    std::vector<uint8_t> row_bin, row_side;
    std::vector<float> feat;
    uint64_t rows_total = 0;
    std::vector<uint32_t> pair_rounds;
    std::vector<uint64_t> pair_arcs, pair_ent, dist;
};

// Runs a Plain / Plain* batch with the multiplier bin of every pair fixed
// (ml mode 1; optionally switching to another bin from a given round on), or
// chosen by the loaded network (ml mode 2), and collects per pair the rounds
// its searches ran, the arcs they scanned and the entries they put in their
// next frontiers, and optionally the feature rows of their step decisions.
int trace_run(ppsp_graph g, const uint32_t *pairs, uint32_t k, const ppsp_opts *o, const TraceReq &rq, TraceOut &out) {
    if (o->batch != PPSP_BATCH_PLAIN && o->batch != PPSP_BATCH_PLAINSTAR) return PPSP_E_INVALID;
    if (rq.network && !g->mlp_loaded) return PPSP_E_INVALID;
    for (uint32_t i = 0; i < k; i++)
        if ((rq.bins && rq.bins[i] >= MLP_K) || (rq.switch_round && (!rq.bins_after || rq.bins_after[i] >= 2 * MLP_K)))
            return PPSP_E_INVALID;
    // distinct queries in first-occurrence order, as batch_impl forms them
    std::unordered_map<uint64_t, uint32_t> seen;
    std::vector<uint32_t> first, qof(k, UINT32_MAX);
    std::vector<uint8_t> qbin, qbin_after;
    std::vector<uint32_t> qsw;
    for (uint32_t i = 0; i < k; i++) {
        uint32_t s = pairs[2 * i], t = pairs[2 * i + 1];
        if (s >= g->n || t >= g->n) return PPSP_E_RANGE;
        if (s == t) continue;
        if (g->symmetric && s > t && o->algo != PPSP_SSSP) std::swap(s, t);
        const uint64_t key = rq.distinct ? (uint64_t)i : (((uint64_t)s << 32) | t);
        auto it = seen.find(key);
        if (it == seen.end()) {
            it = seen.emplace(key, (uint32_t)first.size()).first;
            first.push_back(i);
            qbin.push_back(rq.bins ? rq.bins[i] : (uint8_t)(MLP_K / 2));
            if (rq.switch_round) {
                qbin_after.push_back(rq.bins_after[i]);
                qsw.push_back(rq.switch_round[i]);
            }
        }
        qof[i] = it->second;
    }
    MlCtx c;
    c.mode = rq.network ? 2 : 1;
    c.qbin = &qbin;
    if (rq.switch_round) {
        c.qbin_after = &qbin_after;
        c.qsw = &qsw;
    }
    c.nodedup = rq.distinct;
    c.collect = true;
    for (uint32_t i = 0; i < k && rq.switch_round; i++) c.dense = c.dense || rq.bins_after[i] >= MLP_K;
    c.rows = rq.rows;
    c.cap = rq.rows ? rq.cap : 0;
    c.q_rounds.assign(first.size(), 0);
    c.q_arcs.assign(first.size(), 0);
    c.q_ent.assign(first.size(), 0);
    g->ml = &c;
    out.dist.assign(k, 0);
    ppsp_opts oo = *o;
    oo.sched = PPSP_SCHED_FIXED;
    oo.flags &= ~(uint32_t)(PPSP_WANT_PATH | PPSP_DEVICE_IO);
    const int rc = batch_impl(g, pairs, k, &oo, nullptr, out.dist.data(), nullptr, nullptr, 0, nullptr);
    g->ml = nullptr;
    CHK(rc);
    out.row_pair.resize(c.row_q.size());
    for (size_t r = 0; r < c.row_q.size(); r++) out.row_pair[r] = first[c.row_q[r]];
    out.row_round = std::move(c.row_r);
    out.row_bin = std::move(c.row_b);
    out.row_side = std::move(c.row_side);
    out.feat = std::move(c.feat);
    out.rows_total = c.rows_total;
    out.pair_rounds.assign(k, 0);
    out.pair_arcs.assign(k, 0);
    out.pair_ent.assign(k, 0);
    for (uint32_t i = 0; i < k; i++)
        if (qof[i] != UINT32_MAX) {
            out.pair_rounds[i] = c.q_rounds[qof[i]];
            out.pair_arcs[i] = c.q_arcs[qof[i]];
            out.pair_ent[i] = c.q_ent[qof[i]];
        }
    return PPSP_OK;
}

// The earlier interface: fixed bins (NULL: 4), rows, per-pair rounds and arcs.
int trace_impl(ppsp_graph g, const uint32_t *pairs, uint32_t k, const ppsp_opts *o, const uint8_t *bins,
               bool rows, uint64_t cap, MlCtx &c, std::vector<uint32_t> &row_pair, std::vector<uint32_t> &pair_rounds,
               std::vector<uint64_t> &pair_arcs) {
    TraceReq rq;
    rq.bins = bins;
    rq.rows = rows;
    rq.cap = cap;
    TraceOut out;
    CHK(trace_run(g, pairs, k, o, rq, out));
    c = MlCtx{};
    c.feat = std::move(out.feat);
    c.rows_total = out.rows_total;
    row_pair = std::move(out.row_pair);
    pair_rounds = std::move(out.pair_rounds);
    pair_arcs = std::move(out.pair_arcs);
    return PPSP_OK;
}

uint64_t splitmix64(uint64_t &x) {
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Device buffers of one training or evaluation call.
struct MlpDev {
    DevBuf P, X, Y, idx, partial, loss, m, v, grad, logits;
    hipStream_t st = nullptr;
    ~MlpDev() {
        if (st) (void)hipStreamDestroy(st);
    }
};

int mlp_setup(int device, MlpDev &d, const float *params, const float *x, const uint32_t *y, uint32_t n) {
    HIPCHK(hipSetDevice(device));
    HIPCHK(hipStreamCreateWithFlags(&d.st, hipStreamNonBlocking));
    CHK(ensure(d.P, MLP_NPARAM * 4));
    HIPCHK(hipMemcpyAsync(d.P.p, params, MLP_NPARAM * 4, hipMemcpyHostToDevice, d.st));
    if (n) {
        CHK(ensure(d.X, (uint64_t)n * MLP_F * 4));
        HIPCHK(hipMemcpyAsync(d.X.p, x, (uint64_t)n * MLP_F * 4, hipMemcpyHostToDevice, d.st));
        if (y) {
            CHK(ensure(d.Y, (uint64_t)n * 4));
            HIPCHK(hipMemcpyAsync(d.Y.p, y, (uint64_t)n * 4, hipMemcpyHostToDevice, d.st));
        }
    }
    return PPSP_OK;
}

// Full-batch gradient (mean cross-entropy) and loss of the parameters in d.P.
int mlp_full_grad(MlpDev &d, uint32_t n, float *grad, double *loss) {
    const uint32_t nw = std::max<uint32_t>(1, std::min<uint32_t>(1024, (n + 15) / 16));
    const uint32_t per = (n + nw - 1) / nw;
    CHK(ensure(d.partial, (uint64_t)nw * MLP_NPARAM * 4));
    CHK(ensure(d.loss, (uint64_t)nw * 8));
    CHK(ensure(d.grad, MLP_NPARAM * 4));
    HIPCHK(launch_mlp_grad(d.P.as<float>(), d.X.as<float>(), d.Y.as<uint32_t>(), nullptr, 0, n, per, nw,
                           1.f / (float)std::max<uint32_t>(n, 1), d.partial.as<float>(), d.loss.as<double>(), d.st));
    HIPCHK(launch_mlp_reduce(d.partial.as<float>(), nw, d.grad.as<float>(), d.st));
    std::vector<double> l(nw);
    HIPCHK(hipMemcpyAsync(l.data(), d.loss.p, (uint64_t)nw * 8, hipMemcpyDeviceToHost, d.st));
    if (grad) HIPCHK(hipMemcpyAsync(grad, d.grad.p, MLP_NPARAM * 4, hipMemcpyDeviceToHost, d.st));
    HIPCHK(hipStreamSynchronize(d.st));
    double s = 0;
    for (double v : l) s += v;
    if (loss) *loss = n ? s / n : 0.0;
    return PPSP_OK;
}

int mlp_train_impl(int device, float *params, const float *x, const uint32_t *y, uint32_t n, uint32_t epochs,
                   uint32_t batch, float lr, uint64_t seed, double *loss_first, double *loss_last) {
    if (!params || (n && (!x || !y)) || batch == 0 || !(lr > 0.f)) return PPSP_E_INVALID;
    for (uint32_t i = 0; i < n; i++)
        if (y[i] >= (uint32_t)MLP_Y) return PPSP_E_INVALID;
    MlpDev d;
    CHK(mlp_setup(device, d, params, x, y, n));
    if (loss_first) CHK(mlp_full_grad(d, n, nullptr, loss_first));
    const uint32_t per = 16;
    const uint32_t nwmax = (batch + per - 1) / per;
    CHK(ensure(d.partial, (uint64_t)nwmax * MLP_NPARAM * 4));
    CHK(ensure(d.loss, (uint64_t)std::max<uint32_t>(nwmax, 1024) * 8));
    CHK(ensure(d.m, MLP_NPARAM * 4));
    CHK(ensure(d.v, MLP_NPARAM * 4));
    CHK(ensure(d.idx, (uint64_t)std::max<uint32_t>(n, 1) * 4));
    HIPCHK(hipMemsetAsync(d.m.p, 0, MLP_NPARAM * 4, d.st));
    HIPCHK(hipMemsetAsync(d.v.p, 0, MLP_NPARAM * 4, d.st));
    std::vector<uint32_t> perm(n);
    std::iota(perm.begin(), perm.end(), 0u);
    uint64_t rs = seed;
    uint32_t t = 0;
    for (uint32_t e = 0; e < epochs && n; e++) {
        for (uint32_t i = n - 1; i > 0; i--) std::swap(perm[i], perm[splitmix64(rs) % (i + 1)]);
        HIPCHK(hipMemcpyAsync(d.idx.p, perm.data(), (uint64_t)n * 4, hipMemcpyHostToDevice, d.st));
        HIPCHK(hipStreamSynchronize(d.st));    // perm is rewritten next epoch
        for (uint32_t b = 0; b < n; b += batch) {
            const uint32_t end = std::min<uint32_t>(n, b + batch);
            const uint32_t nw = (end - b + per - 1) / per;
            HIPCHK(launch_mlp_grad(d.P.as<float>(), d.X.as<float>(), d.Y.as<uint32_t>(), d.idx.as<uint32_t>(), b, end,
                                   per, nw, 1.f / (float)(end - b), d.partial.as<float>(), d.loss.as<double>(), d.st));
            HIPCHK(launch_mlp_adam(d.P.as<float>(), d.m.as<float>(), d.v.as<float>(), d.partial.as<float>(), nw, lr,
                                   ++t, d.st));
        }
    }
    if (loss_last) CHK(mlp_full_grad(d, n, nullptr, loss_last));
    HIPCHK(hipMemcpyAsync(params, d.P.p, MLP_NPARAM * 4, hipMemcpyDeviceToHost, d.st));
    HIPCHK(hipStreamSynchronize(d.st));
    return PPSP_OK;
}

int mlp_forward_impl(int device, const float *params, const float *x, uint32_t n, float *logits) {
    if (!params || (n && (!x || !logits))) return PPSP_E_INVALID;
    MlpDev d;
    CHK(mlp_setup(device, d, params, x, nullptr, n));
    if (n == 0) return PPSP_OK;
    CHK(ensure(d.logits, (uint64_t)n * MLP_O * 4));
    HIPCHK(launch_mlp_forward(d.P.as<float>(), d.X.as<float>(), n, d.logits.as<float>(), d.st));
    HIPCHK(hipMemcpyAsync(logits, d.logits.p, (uint64_t)n * MLP_O * 4, hipMemcpyDeviceToHost, d.st));
    HIPCHK(hipStreamSynchronize(d.st));
    return PPSP_OK;
}

uint16_t f32_to_bf16(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return (uint16_t)((u >> 16) | 0x40);  // NaN stays NaN
    u += 0x7FFFu + ((u >> 16) & 1u);                                                                 // nearest even
    return (uint16_t)(u >> 16);
}

int mlp_load_impl(ppsp_graph g, const float *params) {
    if (!g || !params) return PPSP_E_INVALID;
    for (int i = 0; i < MLP_NPARAM; i++)
        if (!std::isfinite(params[i])) return PPSP_E_INVALID;
    CHK(set_device(g));
    std::vector<uint16_t> h(MLP_NPARAM);
    for (int i = 0; i < MLP_NPARAM; i++) h[i] = f32_to_bf16(params[i]);
    CHK(ensure(g->mlpw, MLP_NPARAM * 2));
    HIPCHK(hipMemcpyAsync(g->mlpw.p, h.data(), MLP_NPARAM * 2, hipMemcpyHostToDevice, g->st));
    HIPCHK(hipStreamSynchronize(g->st));
    g->mlp_loaded = true;
    g->ml_plain = false;
    return PPSP_OK;
}

// ---- serving: continuous batching --------------------------------------------
//
// Each resident graph has a fixed pool of query slots (a forward and a
// backward search in one interleaved state group each), sized by the memory
// budget. A worker thread drives the device round loop without ever
// resetting it. Between chunks of rounds it
//   - admits waiting queries into free slots (clears their state slabs,
//     k_admit seeds their roots into the frontier the next round reads),
//   - reads the per-search done flags and the mu slots, and retires finished
//     queries (a slot is reused only one chunk after its query finished, so
//     no frontier entry of the old query is still queued),
// so requests that arrive while others run join them on the device.

namespace {

struct SrvRequest {
    uint32_t graph = 0;
    std::vector<uint32_t> pairs;
    std::vector<uint64_t> dist;
    uint32_t next = 0;              // next query to admit
    uint32_t remaining = 0;         // queries not finished
    std::chrono::steady_clock::time_point t_submit, t_done;
    bool done = false;
};

struct SrvGraph {
    ppsp_graph g = nullptr;
    uint32_t C = 0;                 // query slots
    std::vector<SearchDesc> sd;
    std::vector<Partner> partners;
    std::vector<PairDesc> pairs;
    std::vector<uint64_t> delta;
    std::vector<int> state;         // 0 free, 1 running, 2 finished (reusable next chunk)
    std::vector<uint64_t> slot_req;
    std::vector<uint32_t> slot_q;
    RoundArgs A;
    uint32_t grid = 0;
    uint32_t *h_done = nullptr;     // pinned: 2C done flags, then err
    uint64_t *h_mu = nullptr;       // pinned: C mu slots
    DevBuf ids;
    std::vector<uint32_t> h_ids;    // admitted search ids (kept until the chunk's sync)
    uint32_t running = 0;           // slots in state 1
    uint32_t draining = 0;          // slots in state 2
    uint64_t round = 0;             // the device round counter, mirrored on the host
    bool learned = false;           // the graph's loaded network picks every search's step
    std::deque<std::pair<uint64_t, uint32_t>> redo;   // (request, query) to admit first, after an overflow
};

}  // namespace

struct ppsp_server_s {
    std::vector<SrvGraph> gs;
    std::vector<ppsp_opts> opts;    // per graph
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> pending;
    std::unordered_map<uint64_t, SrvRequest> reqs;
    uint64_t next_id = 1;
    std::thread worker;
    bool stop = false;
    int err = PPSP_OK;
    uint64_t admitted = 0, completed = 0, chunks = 0, rounds = 0, restarts = 0, renumbers = 0;
    uint32_t rounds_per_chunk = 16;
};

namespace {

// The learned schedule in a server's round loop: per-search counters and
// bins (reset for each admitted search by k_admit) and the loaded network.
void srv_learned_args(const SrvGraph &G, RoundArgs &A) {
    if (!G.learned) return;
    ppsp_graph g = G.g;
    A.sc = g->sc.as<unsigned long long>();
    A.ml_mode = 2;
    A.mlp = g->mlpw.as<uint16_t>();
    A.bin = g->bin.as<uint8_t>();
    A.done_round = g->done_round.as<uint32_t>();
    A.tot_arcs = g->tot_arcs.as<unsigned long long>();
    A.tot_ent = g->tot_ent.as<unsigned long long>();
    A.trace_n = g->trace_n.as<unsigned long long>();
    A.deg_feat = g->n ? (float)(std::log2(std::max(1.0, (double)g->m / g->n)) / 4.0) : 0.f;
    A.ml_every = (uint32_t)std::max<int64_t>(1, g->opt_ml_every);
}

int srv_setup_graph(ppsp_server srv, SrvGraph &G, const ppsp_opts &o, uint64_t budget) {
    ppsp_graph g = G.g;
    G.learned = o.sched == PPSP_SCHED_LEARNED && g->mlp_loaded && !g->ml_plain;
    const uint64_t n = g->n;
    const uint64_t per_query = 2 * n * 8;
    // two thirds of the budget for search state, one third for the two frontier queues
    G.C = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(budget / 3 * 2 / per_query, 1), 1u << 20);
    const uint32_t ns = 2 * G.C, npair = G.C;
    const uint32_t algo = o.algo;
    const uint32_t kf = algo == PPSP_BIDS ? K_2DIST : K_BIDA_F, kb = algo == PPSP_BIDS ? K_2DIST : K_BIDA_B;
    const uint64_t delta = o.delta ? o.delta : graph_default_delta(g);
    G.sd.assign(ns, SearchDesc{});
    G.partners.resize(ns);
    G.pairs.resize(npair);
    G.delta.resize(ns);
    for (uint32_t q = 0; q < G.C; q++) {
        G.sd[2 * q].kind = kf;
        G.sd[2 * q + 1].kind = kb;
        G.sd[2 * q].pbeg = 2 * q;
        G.sd[2 * q].pend = 2 * q + 1;
        G.sd[2 * q + 1].pbeg = 2 * q + 1;
        G.sd[2 * q + 1].pend = 2 * q + 2;
        G.partners[2 * q] = {2 * q + 1, q};
        G.partners[2 * q + 1] = {2 * q, q};
        G.pairs[q] = {2 * q, 2 * q + 1};
        G.delta[2 * q] = key_delta(kf, delta);
        G.delta[2 * q + 1] = key_delta(kb, delta);
    }
    G.state.assign(G.C, 0);
    G.slot_req.assign(G.C, 0);
    G.slot_q.assign(G.C, 0);
    hipStream_t st = g->st;
    CHK(set_device(g));
    CHK(ensure(g->S, (uint64_t)ns * n * 8));
    CHK(ensure(g->round, 16));
    CHK(ensure(g->hcount, 16));
    if (g->maxdeg > HEAVY_DEG) {
        const uint64_t want = std::min<uint64_t>(1u << 26, std::max<uint64_t>(1u << 20, (uint64_t)ns * list_chunks(g) / 4));
        if (g->hcap < want) g->hcap = (uint32_t)want;
        CHK(ensure(g->heavy, (uint64_t)g->hcap * 32));
    }
    CHK(ensure(g->sd, ns * sizeof(SearchDesc)));
    CHK(ensure(g->partners, ns * sizeof(Partner)));
    CHK(ensure(g->pairdesc, npair * sizeof(PairDesc)));
    CHK(ensure(g->ctl, (uint64_t)ns * 16));
    CHK(ensure(g->hlim, (uint64_t)ns * 8));
    CHK(ensure(g->delta, (uint64_t)ns * 8));
    CHK(ensure(g->done, (uint64_t)ns * 4));
    CHK(ensure(g->exh, (uint64_t)ns * 4));
    CHK(ensure(g->alive, 2ull * ns * 4));
    CHK(ensure(g->minkey, 2ull * ns * 8));
    CHK(ensure(g->mu, (uint64_t)npair * 8));
    CHK(ensure(g->qcount, 2 * NSEG * 4));
    CHK(ensure(g->cpre, 2 * (NSEG + 1) * 4));
    CHK(ensure(g->tsum, 48));
    CHK(ensure(g->err, 16));
    CHK(ensure(g->stats, ST_N * 8));
    G.grid = round_grid(g);
    CHK(ensure(g->wstats, (uint64_t)G.grid * ST_N * 8));
    if (g->opt_queue_cap == 0)   // an explicit "queue_cap" stands (and grows on overflow)
        g->qcap = std::max<uint64_t>(g->qcap, std::min<uint64_t>(std::max<uint64_t>(budget / 3 / 32, 1ull << 22), 1ull << 31));
    CHK(ensure(g->q0, g->qcap * 16));
    CHK(ensure(g->q1, g->qcap * 16));
    CHK(ensure(G.ids, (uint64_t)ns * 4));
    HIPCHK(hipHostMalloc((void **)&G.h_done, ((uint64_t)ns + 4) * 4, hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&G.h_mu, (uint64_t)npair * 8, hipHostMallocDefault));
    HIPCHK(hipMemcpyAsync(g->sd.p, G.sd.data(), ns * sizeof(SearchDesc), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(g->partners.p, G.partners.data(), ns * sizeof(Partner), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(g->pairdesc.p, G.pairs.data(), npair * sizeof(PairDesc), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(g->delta.p, G.delta.data(), (uint64_t)ns * 8, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemsetAsync(g->qcount.p, 0, 2 * NSEG * 4, st));
    HIPCHK(hipMemsetAsync(g->cpre.p, 0, 2 * (NSEG + 1) * 4, st));
    HIPCHK(hipMemsetAsync(g->tsum.p, 0, 48, st));
    HIPCHK(hipMemsetAsync(g->round.p, 0, 16, st));
    if (g->opt_server_round_base > 0) {
        // the round loop starts at this round (a test of the renumbering below)
        const uint32_t rb[2] = {(uint32_t)g->opt_server_round_base, (uint32_t)g->opt_server_round_base};
        HIPCHK(hipMemcpyAsync(g->round.p, rb, 8, hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    G.round = (uint64_t)g->opt_server_round_base;
    HIPCHK(hipMemsetAsync(g->hcount.p, 0, 16, st));
    HIPCHK(hipMemsetAsync(g->err.p, 0, 16, st));
    HIPCHK(hipMemsetAsync(g->stats.p, 0, ST_N * 8, st));
    HIPCHK(hipMemsetAsync(g->wstats.p, 0, (uint64_t)G.grid * ST_N * 8, st));
    HIPCHK(hipMemsetAsync(g->mu.p, 0xFF, (uint64_t)npair * 8, st));
    if (G.learned) {
        CHK(ensure(g->sc, 2ull * ns * 16));
        CHK(ensure(g->bin, ns));
        CHK(ensure(g->done_round, (uint64_t)ns * 4));
        CHK(ensure(g->tot_arcs, (uint64_t)ns * 8));
        CHK(ensure(g->tot_ent, (uint64_t)ns * 8));
        CHK(ensure(g->trace_n, 8));
        HIPCHK(hipMemsetAsync(g->sc.p, 0, 2ull * ns * 16, st));
        HIPCHK(hipMemsetAsync(g->bin.p, MLP_K / 2, ns, st));
        HIPCHK(hipMemsetAsync(g->done_round.p, 0, (uint64_t)ns * 4, st));
        HIPCHK(hipMemsetAsync(g->tot_arcs.p, 0, (uint64_t)ns * 8, st));
        HIPCHK(hipMemsetAsync(g->tot_ent.p, 0, (uint64_t)ns * 8, st));
        HIPCHK(hipMemsetAsync(g->trace_n.p, 0, 8, st));
    }
    set_args(g, G.A, ns, npair, 2, true);
    srv_learned_args(G, G.A);
    HIPCHK(launch_idle(G.A, st));
    HIPCHK(hipStreamSynchronize(st));
    return PPSP_OK;
}

// A round's stamp (1 + its number, see ppsp_dev.h) must stay below the
// reserved stamp values (0xFFFFFFFE marks a check-only entry, 0xFFFFFFFF a
// cleared word), so a server renumbers its round loop from 0 before its
// round counter reaches SRV_ROUND_LIMIT.
constexpr uint64_t SRV_ROUND_LIMIT = 0xFFFFFF00ull;

// Grows the buffer that overflowed (errbits), or with renumber resets the
// round counter to 0; in both cases resets the graph's round loop to idle and
// puts every running query back in front of the admission order (each
// admitted query clears its own state slab, so no stamp of an earlier round
// number survives). Called with the lock held, after the stream is idle.
int srv_restart(ppsp_server srv, SrvGraph &G, uint32_t errbits, bool renumber = false) {
    ppsp_graph g = G.g;
    hipStream_t st = g->st;
    if (errbits & ERR_QUEUE) {
        if (g->qcap >= (1ull << 31)) return PPSP_E_OOM;
        g->qcap *= 2;
        CHK(ensure(g->q0, g->qcap * 16));
        CHK(ensure(g->q1, g->qcap * 16));
    }
    if (errbits & ERR_HEAVY) {
        if (g->hcap >= (1u << 28)) return PPSP_E_OOM;
        g->hcap *= 4;
        CHK(ensure(g->heavy, (uint64_t)g->hcap * 32));
    }
    for (uint32_t q = G.C; q-- > 0;) {
        if (G.state[q] == 1) {
            G.redo.emplace_front(G.slot_req[q], G.slot_q[q]);
            G.running--;
        } else if (G.state[q] == 2) {
            G.draining--;
        }
        G.state[q] = 0;
    }
    const uint32_t ns = 2 * G.C;
    HIPCHK(hipMemsetAsync(g->qcount.p, 0, 2 * NSEG * 4, st));
    HIPCHK(hipMemsetAsync(g->cpre.p, 0, 2 * (NSEG + 1) * 4, st));
    HIPCHK(hipMemsetAsync(g->tsum.p, 0, 48, st));
    HIPCHK(hipMemsetAsync(g->hcount.p, 0, 16, st));
    HIPCHK(hipMemsetAsync(g->err.p, 0, 16, st));
    if (renumber) {
        HIPCHK(hipMemsetAsync(g->round.p, 0, 16, st));
        G.round = 0;
    }
    set_args(g, G.A, ns, G.C, 2, true);
    srv_learned_args(G, G.A);
    HIPCHK(launch_idle(G.A, st));
    HIPCHK(hipStreamSynchronize(st));
    if (renumber) srv->renumbers++; else srv->restarts++;
    return PPSP_OK;
}

// One chunk of the worker: admit, run rounds, collect. Called without the lock.
int srv_chunk(ppsp_server srv, bool &any_running) {
    std::vector<std::vector<uint32_t>> admit(srv->gs.size());
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        for (size_t gi = 0; gi < srv->gs.size(); gi++) {
            SrvGraph &G = srv->gs[gi];
            uint32_t slot = 0;
            // puts query q of request id into the next free slot; false when none is free
            auto place = [&](uint64_t id, uint32_t q) -> bool {
                while (slot < G.C && G.state[slot] != 0) slot++;
                if (slot == G.C) return false;
                SrvRequest &rq = srv->reqs[id];
                const uint32_t s0 = rq.pairs[2 * q], t0 = rq.pairs[2 * q + 1];
                G.state[slot] = 1;
                G.slot_req[slot] = id;
                G.slot_q[slot] = q;
                SearchDesc f = make_sd(G.g, s0, G.sd[2 * slot].kind, s0, t0);
                SearchDesc b = make_sd(G.g, t0, G.sd[2 * slot + 1].kind, s0, t0);
                f.pbeg = G.sd[2 * slot].pbeg; f.pend = G.sd[2 * slot].pend;
                b.pbeg = G.sd[2 * slot + 1].pbeg; b.pend = G.sd[2 * slot + 1].pend;
                b.rev = G.g->symmetric ? 0u : 1u;    // directed: the backward half walks the transpose
                G.sd[2 * slot] = f;
                G.sd[2 * slot + 1] = b;
                admit[gi].push_back(slot);
                srv->admitted++;
                return true;
            };
            while (!G.redo.empty() && place(G.redo.front().first, G.redo.front().second)) G.redo.pop_front();
            if (!G.redo.empty()) continue;
            for (auto it = srv->pending.begin(); it != srv->pending.end();) {
                SrvRequest &rq = srv->reqs[*it];
                if (rq.graph != gi) { ++it; continue; }
                const uint32_t k = (uint32_t)(rq.pairs.size() / 2);
                bool full = false;
                while (rq.next < k) {
                    const uint32_t s0 = rq.pairs[2 * rq.next], t0 = rq.pairs[2 * rq.next + 1];
                    if (s0 == t0) {                              // d(s,s) = 0 needs no search
                        rq.dist[rq.next++] = 0;
                        if (--rq.remaining == 0) { rq.done = true; rq.t_done = std::chrono::steady_clock::now(); srv->completed++; }
                        continue;
                    }
                    if (!place(*it, rq.next)) { full = true; break; }
                    rq.next++;
                }
                if (rq.done) srv->cv_done.notify_all();
                if (rq.next == k) it = srv->pending.erase(it); else ++it;
                if (full) break;
            }
        }
    }
    any_running = false;
    for (size_t gi = 0; gi < srv->gs.size(); gi++) {
        SrvGraph &G = srv->gs[gi];
        ppsp_graph g = G.g;
        hipStream_t st = g->st;
        if (!admit[gi].empty()) {
            std::vector<uint32_t> &ids = G.h_ids;
            ids.clear();
            for (uint32_t q : admit[gi]) {
                ids.push_back(2 * q);
                ids.push_back(2 * q + 1);
                HIPCHK(hipMemsetAsync(g->S.as<uint64_t>() + (uint64_t)q * g->n * 2, 0xFF, (uint64_t)g->n * 16, st));
            }
            HIPCHK(hipMemcpyAsync(g->sd.p, G.sd.data(), G.sd.size() * sizeof(SearchDesc), hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(G.ids.p, ids.data(), ids.size() * 4, hipMemcpyHostToDevice, st));
            HIPCHK(launch_admit(G.A, G.ids.as<uint32_t>(), (uint32_t)ids.size(), st));
            G.running += (uint32_t)admit[gi].size();
        }
        // Rounds also run while slots drain: a finished search's last frontier
        // entries are dropped by the round after the one that finished it.
        if (G.running == 0 && G.draining == 0) continue;
        any_running = true;
        for (uint32_t k = 0; k < srv->rounds_per_chunk; k++) {
            HIPCHK(launch_round(G.A, G.grid, st));
            if (G.A.hcap) HIPCHK(launch_heavy(G.A, G.grid, st));
            HIPCHK(launch_control(G.A, st));
        }
        HIPCHK(hipMemcpyAsync(G.h_done, g->done.p, (uint64_t)2 * G.C * 4, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(G.h_done + 2 * G.C, g->err.p, 4, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(G.h_mu, g->mu.p, (uint64_t)G.C * 8, hipMemcpyDeviceToHost, st));
    }
    for (auto &G : srv->gs) HIPCHK(hipStreamSynchronize(G.g->st));
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->chunks++;
    for (auto &G : srv->gs) {
        if (G.running == 0 && G.draining == 0) continue;
        srv->rounds += srv->rounds_per_chunk;
        G.round += srv->rounds_per_chunk;
        if (G.h_done[2 * G.C] & ERR_OVERFLOW) return PPSP_E_OVERFLOW;
        if (G.h_done[2 * G.C] & (ERR_QUEUE | ERR_HEAVY)) {
            // A queue or the heavy list overflowed in this chunk: frontier
            // entries were lost, so every query on the device starts again
            // with larger buffers (results of earlier chunks stand).
            CHK(srv_restart(srv, G, G.h_done[2 * G.C]));
            continue;
        }
        for (uint32_t q = 0; q < G.C; q++) {
            if (G.state[q] == 2) { G.state[q] = 0; G.draining--; continue; }
            if (G.state[q] != 1 || !G.h_done[2 * q] || !G.h_done[2 * q + 1]) continue;
            SrvRequest &rq = srv->reqs[G.slot_req[q]];
            const uint32_t d32 = (uint32_t)(G.h_mu[q] >> 32);
            rq.dist[G.slot_q[q]] = d32 == INF32 ? PPSP_INF : d32;
            G.state[q] = 2;
            G.draining++;
            G.running--;
            if (--rq.remaining == 0) {
                rq.done = true;
                rq.t_done = std::chrono::steady_clock::now();
                srv->completed++;
            }
        }
        // the next chunk would run rounds with stamps too close to the reserved ones
        if (G.round + srv->rounds_per_chunk >= SRV_ROUND_LIMIT) CHK(srv_restart(srv, G, 0, true));
    }
    srv->cv_done.notify_all();
    return PPSP_OK;
}

void srv_worker(ppsp_server srv) {
    (void)hipSetDevice(srv->gs[0].g->device);
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            bool idle = srv->pending.empty();
            for (auto &G : srv->gs) idle = idle && G.running == 0 && G.draining == 0;
            if (idle && !srv->stop)
                srv->cv_work.wait_for(lk, std::chrono::milliseconds(20));
            if (srv->stop) return;
        }
        bool any = false;
        const int rc = srv_chunk(srv, any);
        if (rc != PPSP_OK) {
            std::lock_guard<std::mutex> lk(srv->mu);
            srv->err = rc;
            srv->cv_done.notify_all();
            return;
        }
    }
}

}  // namespace

// ---- C interface --------------------------------------------------------------

extern "C" {

const char *ppsp_version(void) { return "0.1.0"; }

const char *ppsp_last_error(void) { return g_last_error.c_str(); }

const char *ppsp_status_str(int s) {
    switch (s) {
        case PPSP_OK: return "ok";
        case PPSP_E_INVALID: return "invalid argument";
        case PPSP_E_RANGE: return "value out of range";
        case PPSP_E_OOM: return "out of device memory";
        case PPSP_E_OVERFLOW: return "distance overflow (>= 2^32-1)";
        case PPSP_E_NOCOORD: return "A* needs consistent coordinates";
        case PPSP_E_NOTSYM: return "mode needs a symmetric graph";
        case PPSP_E_DEVICE: return "HIP runtime error";
        case PPSP_E_BUSY: return "request not finished";
        case PPSP_E_PATHCAP: return "path buffer too small";
        case PPSP_E_NOPATH: return "paths need positive weights";
        case PPSP_E_TIMEOUT: return "round loop exceeded its time limit";
        default: return "unknown status";
    }
}

int ppsp_query_cover(const uint32_t *pairs, uint32_t k, uint32_t directed, uint32_t *root, uint8_t *from_target,
                     uint32_t *cover_size) {
    if ((k && (!pairs || !root || !from_target)) || !cover_size) return PPSP_E_INVALID;
    std::vector<Query> qs;
    std::vector<uint32_t> qidx(k, UINT32_MAX);
    std::vector<uint8_t> flip(k, 0);
    std::unordered_map<uint64_t, uint32_t> seen;
    for (uint32_t i = 0; i < k; i++) {
        uint32_t s = pairs[2 * i], t = pairs[2 * i + 1];
        if (s == t) continue;
        if (!directed && s > t) { std::swap(s, t); flip[i] = 1; }
        const uint64_t key = ((uint64_t)s << 32) | t;
        auto it = seen.emplace(key, (uint32_t)qs.size()).first;
        if (it->second == qs.size()) qs.push_back({s, t});
        qidx[i] = it->second;
    }
    std::vector<uint8_t> rev;
    const std::vector<uint32_t> by = query_cover(qs, directed != 0, rev);
    std::unordered_map<uint64_t, char> roots;
    for (size_t q = 0; q < qs.size(); q++) roots[((uint64_t)rev[q] << 32) | by[q]] = 1;
    for (uint32_t i = 0; i < k; i++) {
        if (qidx[i] == UINT32_MAX) {                       // s = t: no search
            root[i] = pairs[2 * i];
            from_target[i] = 0;
            continue;
        }
        root[i] = by[qidx[i]];
        from_target[i] = root[i] == pairs[2 * i + 1] ? 1 : 0;
    }
    *cover_size = (uint32_t)roots.size();
    return PPSP_OK;
}

uint64_t ppsp_heuristic_fx(int32_t x0, int32_t y0, int32_t x1, int32_t y1, uint32_t w_scale, uint32_t frac_bits) {
    const __int128 dx = (__int128)x1 - x0, dy = (__int128)y1 - y0;
    const unsigned __int128 d2 = (unsigned __int128)(dx * dx) + (unsigned __int128)(dy * dy);
    const unsigned __int128 q = d2 * ((unsigned __int128)w_scale * w_scale);
    if (q >> 63) return UINT64_MAX;
    return heur(x0, y0, x1, y1, (uint64_t)w_scale * w_scale, frac_bits);
}

int ppsp_graph_create(int device, uint32_t n, uint64_t m, const uint64_t *row_ptr, const uint32_t *col,
                      const uint32_t *w, const int32_t *coord_fx, uint32_t coord_frac_bits, uint32_t w_scale,
                      uint32_t flags, void *hip_stream, ppsp_graph *out) {
    g_last_error.clear();
    if (!out || !row_ptr || (m && (!col || !w)) || n == 0) return PPSP_E_INVALID;
    if (n >= TARGET_BIT || m >= (1ull << 32)) return PPSP_E_RANGE;
    if (row_ptr[0] != 0 || row_ptr[n] != m) return PPSP_E_INVALID;
    for (uint32_t v = 0; v < n; v++)
        if (row_ptr[v + 1] < row_ptr[v]) return PPSP_E_INVALID;
    uint32_t wmin = UINT32_MAX, wmax = 0;
    uint64_t wsum = 0;
    for (uint64_t e = 0; e < m; e++) {
        if (col[e] >= n) return PPSP_E_RANGE;
        wmin = std::min(wmin, w[e]);
        wmax = std::max(wmax, w[e]);
        wsum += w[e];
    }
    if (m == 0) wmin = wmax = 1;
    uint32_t maxdeg = 0;
    uint64_t hchunks = 0, hchunks_at[6] = {};
    for (uint32_t v = 0; v < n; v++) {
        const uint64_t d = row_ptr[v + 1] - row_ptr[v];
        maxdeg = std::max<uint32_t>(maxdeg, (uint32_t)d);
        if (d > HEAVY_DEG) hchunks += (d + HEAVY_CHUNK - 1) / HEAVY_CHUNK;
        for (int k = 0; k < 6; k++)
            if (d > (16ull << k)) hchunks_at[k] += (d + HEAVY_CHUNK - 1) / HEAVY_CHUNK;
    }
    if (coord_fx && coord_frac_bits > 30) return PPSP_E_RANGE;
    ppsp_graph g = new ppsp_graph_s();
    g->device = device;
    g->n = n;
    g->m = m;
    g->symmetric = flags & PPSP_SYMMETRIC;
    g->wmin = wmin;
    g->wmax = wmax;
    g->wmean = m ? std::max<uint64_t>(1, (wsum + m - 1) / m) : 1;
    {
        // FNV-1a over n, m and a stride sample of the arcs
        uint64_t h = 1469598103934665603ull;
        auto mix = [&](uint64_t x) { h = (h ^ x) * 1099511628211ull; };
        mix(n);
        mix(m);
        const uint64_t step = std::max<uint64_t>(1, m / 4096);
        for (uint64_t e = 0; e < m; e += step) { mix(col[e]); mix(w[e]); }
        for (uint64_t v = 0; v <= n; v += std::max<uint64_t>(1, n / 1024)) mix(row_ptr[v]);
        g->fingerprint = h;
    }
    g->maxdeg = maxdeg;
    g->hchunks = hchunks;
    for (int k = 0; k < 6; k++) g->hchunks_at[k] = hchunks_at[k];
    auto fail = [&](int rc) {
        ppsp_graph_destroy(g);
        return rc;
    };
    // PPSP_REORDER: a locality order of the vertices, and the CSR (and
    // coordinates) renumbered into it; everything below uses the renumbered
    // arrays, the interface translates ids.
    std::vector<uint64_t> rp_re;
    std::vector<uint32_t> col_re, w_re;
    std::vector<int32_t> xy_re;
    if ((flags & PPSP_REORDER) && n > 1) {
        std::vector<uint32_t> order(n);
        if (coord_fx) {
            // Morton (Z-order) key of the coordinates shifted to non-negative
            int64_t x0 = INT64_MAX, y0 = INT64_MAX;
            for (uint32_t v = 0; v < n; v++) {
                x0 = std::min<int64_t>(x0, coord_fx[2 * (uint64_t)v]);
                y0 = std::min<int64_t>(y0, coord_fx[2 * (uint64_t)v + 1]);
            }
            auto spread = [](uint64_t x) {   // the 32 bits of x to the even bit positions
                x &= 0xFFFFFFFFull;
                x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
                x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
                x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
                x = (x | (x << 2)) & 0x3333333333333333ull;
                x = (x | (x << 1)) & 0x5555555555555555ull;
                return x;
            };
            std::vector<uint64_t> key(n);
            for (uint32_t v = 0; v < n; v++)
                key[v] = spread((uint64_t)(coord_fx[2 * (uint64_t)v] - x0)) |
                         (spread((uint64_t)(coord_fx[2 * (uint64_t)v + 1] - y0)) << 1);
            std::iota(order.begin(), order.end(), 0u);
            std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return key[a] < key[b]; });
        } else {
            // Breadth-first order from the highest-degree vertex, then from
            // each unvisited vertex; afterwards the vertices the hub-list
            // kernel relaxes at the default "list_deg" (degree above
            // REORDER_HUB_DEG) are moved to the front in descending degree
            // (ties keep their breadth-first order). On power-law graphs the
            // heads of most arcs are such vertices, so their state words of a
            // search then sit in a few contiguous megabytes per search group
            // that stay in the caches, instead of being spread over all n.
            // Inside that front block, runs of 8 vertices (one 128-byte line
            // of a two-search group's state) are interleaved by quarter of the
            // degree ranking: line j of quarter q goes to slot 4j + q, so the
            // hottest lines are 512 bytes apart rather than packed together
            // (packed, the few hottest kilobytes of each group slow the round
            // kernel by a fifth).
            std::vector<uint8_t> seen(n, 0);
            uint32_t head = 0, tail = 0, root = 0;
            for (uint32_t v = 1; v < n; v++)
                if (row_ptr[v + 1] - row_ptr[v] > row_ptr[root + 1] - row_ptr[root]) root = v;
            uint32_t next_root = 0;
            while (tail < n) {
                if (head == tail) {
                    while (seen[root]) root = next_root++;
                    seen[root] = 1;
                    order[tail++] = root;
                }
                const uint32_t u = order[head++];
                for (uint64_t e = row_ptr[u]; e < row_ptr[u + 1]; e++)
                    if (!seen[col[e]]) { seen[col[e]] = 1; order[tail++] = col[e]; }
            }
            auto deg = [&](uint32_t v) { return row_ptr[v + 1] - row_ptr[v]; };
            std::stable_partition(order.begin(), order.end(), [&](uint32_t v) { return deg(v) > REORDER_HUB_DEG; });
            const auto nh = std::count_if(order.begin(), order.end(), [&](uint32_t v) { return deg(v) > REORDER_HUB_DEG; });
            std::stable_sort(order.begin(), order.begin() + nh, [&](uint32_t a, uint32_t b) { return deg(a) > deg(b); });
            {
                const uint64_t nl = ((uint64_t)nh + 7) / 8;              // lines of 8 ranked hubs
                const uint64_t q = (nl + 3) / 4;                         // lines per quarter
                std::vector<uint64_t> slot(nl);                           // line -> its new slot key
                for (uint64_t L = 0; L < nl; L++) slot[L] = 4 * (L % q) + L / q;
                std::vector<uint64_t> lines(nl);
                std::iota(lines.begin(), lines.end(), 0ull);
                std::sort(lines.begin(), lines.end(), [&](uint64_t a, uint64_t b) { return slot[a] < slot[b]; });
                const std::vector<uint32_t> ranked(order.begin(), order.begin() + nh);
                uint64_t k = 0;
                for (uint64_t L : lines)
                    for (uint64_t j = 8 * L; j < std::min<uint64_t>(8 * L + 8, (uint64_t)nh); j++) order[k++] = ranked[j];
            }
        }
        g->iperm = order;
        g->perm.assign(n, 0);
        for (uint32_t k = 0; k < n; k++) g->perm[order[k]] = k;
        rp_re.assign(n + 1, 0);
        col_re.resize(m);
        w_re.resize(m);
        for (uint32_t k = 0; k < n; k++) {
            const uint32_t u = order[k];
            uint64_t o = rp_re[k];
            for (uint64_t e = row_ptr[u]; e < row_ptr[u + 1]; e++, o++) {
                col_re[o] = g->perm[col[e]];
                w_re[o] = w[e];
            }
            rp_re[k + 1] = o;
        }
        // Each row's arcs by new head id: the heads a wave relaxes in one step
        // then share state lines wherever the new order put a vertex's
        // neighbours near each other (the breadth-first order numbers the
        // unvisited neighbours of a vertex consecutively). Rows in parallel.
        {
            const uint32_t nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
            std::vector<std::thread> th;
            for (uint32_t t = 0; t < nt; t++)
                th.emplace_back([&, t]() {
                    std::vector<std::pair<uint32_t, uint32_t>> tmp;
                    for (uint64_t k = t; k < n; k += nt) {
                        const uint64_t a = rp_re[k], b = rp_re[k + 1];
                        if (b - a < 2) continue;
                        tmp.resize(b - a);
                        for (uint64_t e = a; e < b; e++) tmp[e - a] = {col_re[e], w_re[e]};
                        std::sort(tmp.begin(), tmp.end());
                        for (uint64_t e = a; e < b; e++) {
                            col_re[e] = tmp[e - a].first;
                            w_re[e] = tmp[e - a].second;
                        }
                    }
                });
            for (auto &x : th) x.join();
        }
        if (coord_fx) {
            xy_re.resize(2 * (uint64_t)n);
            for (uint32_t k = 0; k < n; k++) {
                xy_re[2 * (uint64_t)k] = coord_fx[2 * (uint64_t)order[k]];
                xy_re[2 * (uint64_t)k + 1] = coord_fx[2 * (uint64_t)order[k] + 1];
            }
            coord_fx = xy_re.data();
        }
        row_ptr = rp_re.data();
        col = col_re.data();
        w = w_re.data();
    }
    if (coord_fx) {
        // exact 64-bit heuristic arithmetic needs w_scale^2 * (span_x^2 + span_y^2) < 2^63
        int64_t x0 = INT64_MAX, x1 = INT64_MIN, y0 = INT64_MAX, y1 = INT64_MIN;
        for (uint32_t v = 0; v < n; v++) {
            x0 = std::min<int64_t>(x0, coord_fx[2 * (uint64_t)v]);
            x1 = std::max<int64_t>(x1, coord_fx[2 * (uint64_t)v]);
            y0 = std::min<int64_t>(y0, coord_fx[2 * (uint64_t)v + 1]);
            y1 = std::max<int64_t>(y1, coord_fx[2 * (uint64_t)v + 1]);
        }
        const __int128 sx = (__int128)x1 - x0, sy = (__int128)y1 - y0;
        const unsigned __int128 span = (unsigned __int128)(sx * sx) + (unsigned __int128)(sy * sy);
        if ((span * ((unsigned __int128)w_scale * w_scale)) >> 63) return fail(PPSP_E_RANGE);
        // The kernels carry a vertex's heuristic term (h_t, or h_t - h_s) as a
        // signed 32-bit value: every heuristic value is at most the one across
        // the bounding box's diagonal, which must stay below 2^31.
        if ((isqrt_floor((uint64_t)(span * ((unsigned __int128)w_scale * w_scale))) >> coord_frac_bits) >= (1ull << 31))
            return fail(PPSP_E_RANGE);
        g->has_xy = true;
        g->fb = coord_frac_bits;
        g->w_scale = w_scale;
        g->ws2 = (uint64_t)w_scale * w_scale;
        g->h_xy.assign(coord_fx, coord_fx + 2 * (uint64_t)n);
        // Consistency of h (Section 3.3): h(u) <= w(u,v) + h(v) holds for the
        // floor heuristic whenever w >= w_scale * |p_u - p_v|, i.e.
        // (w * 2^fb)^2 >= w_scale^2 * |p_u - p_v|^2 in exact integers.
        bool ok = true;
        for (uint32_t u = 0; u < n && ok; u++)
            for (uint64_t e = row_ptr[u]; e < row_ptr[u + 1]; e++) {
                const uint32_t v = col[e];
                const __int128 dx = (__int128)coord_fx[2 * (uint64_t)v] - coord_fx[2 * (uint64_t)u];
                const __int128 dy = (__int128)coord_fx[2 * (uint64_t)v + 1] - coord_fx[2 * (uint64_t)u + 1];
                const unsigned __int128 lhs = (unsigned __int128)((uint64_t)w[e] << coord_frac_bits) * ((uint64_t)w[e] << coord_frac_bits);
                const unsigned __int128 rhs = (unsigned __int128)g->ws2 * (unsigned __int128)(dx * dx + dy * dy);
                if (lhs < rhs) { ok = false; break; }
            }
        g->xy_ok = ok;
    }
    hipError_t he;
    if ((he = hipSetDevice(device)) != hipSuccess) return fail(device_error("hipSetDevice", he));
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) g->cu = prop.multiProcessorCount;
    if ((he = hipStreamCreateWithFlags(&g->st, hipStreamNonBlocking)) != hipSuccess) {
        g->st = nullptr;
        return fail(device_error("hipStreamCreateWithFlags", he));
    }
    if ((he = hipHostMalloc((void **)&g->h_poll, 4096, hipHostMallocDefault)) != hipSuccess) {
        g->h_poll = nullptr;
        return fail(device_error("hipHostMalloc", he));
    }
    // device CSR: row_ptr as uint32 (m < 2^32), arcs interleaved (neighbour, weight)
    std::vector<uint32_t> rp32(n + 1);
    for (uint64_t v = 0; v <= n; v++) rp32[v] = (uint32_t)row_ptr[v];
    std::vector<uint2> arcs(m);
    for (uint64_t e = 0; e < m; e++) arcs[e] = make_uint2(col[e], w[e]);
    int rc;
    if ((rc = ensure(g->row_ptr, (n + 1) * 4ull)) != PPSP_OK) return fail(rc);
    if ((rc = ensure(g->arcs, std::max<uint64_t>(m, 1) * 8)) != PPSP_OK) return fail(rc);
    hipStream_t st = g->st;
    hipEvent_t ev;
    if ((he = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess)
        return fail(device_error("hipEventCreateWithFlags", he));
    if ((he = hipEventRecord(ev, (hipStream_t)hip_stream)) != hipSuccess) {
        (void)hipEventDestroy(ev);
        return fail(device_error("hipEventRecord on the caller's stream", he));
    }
    (void)hipStreamWaitEvent(st, ev, 0);
    (void)hipEventDestroy(ev);
    if ((he = hipMemcpyAsync(g->row_ptr.p, rp32.data(), (n + 1) * 4ull, hipMemcpyHostToDevice, st)) != hipSuccess)
        return fail(device_error("upload row_ptr", he));
    if (m && (he = hipMemcpyAsync(g->arcs.p, arcs.data(), m * 8, hipMemcpyHostToDevice, st)) != hipSuccess)
        return fail(device_error("upload arcs", he));
    // hubs of a symmetric graph, for the hub list grouped by vertex
    std::vector<uint32_t> hid, hvert;
    if (g->symmetric && maxdeg > HEAVY_DEG) {
        hid.assign(n, INF32);
        for (uint32_t v = 0; v < n; v++)
            if (row_ptr[v + 1] - row_ptr[v] > HEAVY_DEG) {
                hid[v] = (uint32_t)hvert.size();
                hvert.push_back(v);
            }
        g->nhub = (uint32_t)hvert.size();
        if ((rc = ensure(g->hub_id, n * 4ull)) != PPSP_OK) return fail(rc);
        if ((rc = ensure(g->hub_vert, hvert.size() * 4ull)) != PPSP_OK) return fail(rc);
        if ((he = hipMemcpyAsync(g->hub_id.p, hid.data(), n * 4ull, hipMemcpyHostToDevice, st)) != hipSuccess)
            return fail(device_error("upload hub index", he));
        if ((he = hipMemcpyAsync(g->hub_vert.p, hvert.data(), hvert.size() * 4ull, hipMemcpyHostToDevice, st)) !=
            hipSuccess)
            return fail(device_error("upload hub index", he));
    }
    std::vector<uint32_t> trp;
    std::vector<uint2> tarcs;
    if (!g->symmetric) {
        // transpose (in-arcs) for the tight-arc path walk
        trp.assign(n + 1, 0);
        for (uint64_t e = 0; e < m; e++) trp[col[e] + 1]++;
        for (uint32_t v = 0; v < n; v++) trp[v + 1] += trp[v];
        std::vector<uint32_t> pos(trp.begin(), trp.end() - 1);
        tarcs.resize(m);
        for (uint32_t u = 0; u < n; u++)
            for (uint64_t e = row_ptr[u]; e < row_ptr[u + 1]; e++) tarcs[pos[col[e]]++] = make_uint2(u, w[e]);
        if ((rc = ensure(g->in_row_ptr, (n + 1) * 4ull)) != PPSP_OK) return fail(rc);
        if ((rc = ensure(g->in_arcs, std::max<uint64_t>(m, 1) * 8)) != PPSP_OK) return fail(rc);
        if ((he = hipMemcpyAsync(g->in_row_ptr.p, trp.data(), (n + 1) * 4ull, hipMemcpyHostToDevice, st)) != hipSuccess)
            return fail(device_error("upload transpose", he));
        if (m && (he = hipMemcpyAsync(g->in_arcs.p, tarcs.data(), m * 8, hipMemcpyHostToDevice, st)) != hipSuccess)
            return fail(device_error("upload transpose", he));
    }
    if (g->has_xy) {
        if ((rc = ensure(g->xy, n * 8ull)) != PPSP_OK) return fail(rc);
        if ((he = hipMemcpyAsync(g->xy.p, coord_fx, n * 8ull, hipMemcpyHostToDevice, st)) != hipSuccess)
            return fail(device_error("upload coordinates", he));
    }
    if ((he = hipStreamSynchronize(st)) != hipSuccess) return fail(device_error("graph upload sync", he));
    *out = g;
    return PPSP_OK;
}

int ppsp_graph_destroy(ppsp_graph g) {
    if (!g) return PPSP_OK;
    if (g->served) return PPSP_E_BUSY;   // the server's worker still uses it
    (void)hipSetDevice(g->device);
    if (g->st) (void)hipStreamSynchronize(g->st);
    DevBuf *bufs[] = {&g->row_ptr, &g->arcs, &g->xy, &g->in_row_ptr, &g->in_arcs, &g->S, &g->q0, &g->q1,
                      &g->sd, &g->partners, &g->pairdesc, &g->ctl, &g->delta, &g->done, &g->exh, &g->alive,
                      &g->minkey, &g->mu, &g->qcount, &g->cpre, &g->round, &g->err, &g->stats, &g->wstats, &g->heavy, &g->hcount, &g->pathlen, &g->pathoff,
                      &g->pathbuf};
    for (DevBuf *b : bufs) release(*b);
    for (hipEvent_t e : g->ev) (void)hipEventDestroy(e);
    if (g->h_poll) (void)hipHostFree(g->h_poll);
    if (g->st) (void)hipStreamDestroy(g->st);
    delete g;                          // frees every remaining buffer
    return PPSP_OK;
}

int ppsp_batch_query(ppsp_graph g, const uint32_t *pairs, uint32_t k, const ppsp_opts *opts, void *hip_stream,
                     uint64_t *dist, uint64_t *path_off, uint32_t *path_vtx, uint64_t path_cap) {
    if (opts && (opts->flags & PPSP_DEVICE_IO)) {
        // device-resident pairs and distances: staged through the host, where
        // the batch is planned, in order on the caller's stream
        if (!g || (!pairs && k) || (!dist && k)) return PPSP_E_INVALID;
        CHK(set_device(g));
        hipStream_t cs = (hipStream_t)hip_stream;
        std::vector<uint32_t> hp(2ull * k);
        std::vector<uint64_t> hd(k);
        if (k) {
            HIPCHK(hipMemcpyAsync(hp.data(), pairs, 8ull * k, hipMemcpyDeviceToHost, cs));
            HIPCHK(hipStreamSynchronize(cs));
        }
        ppsp_opts o = *opts;
        o.flags &= ~PPSP_DEVICE_IO;
        CHK(batch_impl(g, hp.data(), k, &o, hip_stream, hd.data(), path_off, path_vtx, path_cap, nullptr));
        if (k) {
            HIPCHK(hipMemcpyAsync(dist, hd.data(), 8ull * k, hipMemcpyHostToDevice, cs));
            HIPCHK(hipStreamSynchronize(cs));
        }
        return PPSP_OK;
    }
    return batch_impl(g, pairs, k, opts, hip_stream, dist, path_off, path_vtx, path_cap, nullptr);
}

}  // extern "C"

// ---- the no-allocation entry point ---------------------------------------------
//
// ppsp_batch_query_noalloc runs Plain / Plain* batches with every workspace
// buffer (search state, frontier queues, heavy list, control words) carved
// from `scratch`, a fixed device array that each GPU holds from the first
// call until the process ends. Its device address comes from
// hipGetSymbolAddress, once per device with that device current; host code
// never uses the array's name as an address. Calls on one GPU share it, so
// calls that overlap on one GPU race; every call clears what it reads
// before use (state words, queue counters, control words).

namespace {

constexpr uint64_t NOALLOC_SCRATCH_BYTES = 128ull << 20;
static __device__ __align__(256) uint8_t scratch[NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {nullptr};

// The device address of `scratch` on `device` (the current device).
int scratch_ptr(int device, char **out) {
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return PPSP_E_INVALID;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return device_error("hipGetSymbolAddress(scratch)", e);
        g_scratch_ptr[device] = p;
    }
    *out = (char *)g_scratch_ptr[device];
    return PPSP_OK;
}

}  // namespace

extern "C" {

int ppsp_batch_query_noalloc(ppsp_graph g, const uint32_t *pairs, uint32_t k, const ppsp_opts *opts,
                             void *hip_stream, uint64_t *dist) {
    if (!g || !opts || (k && (!pairs || !dist))) return PPSP_E_INVALID;
    if (opts->batch != PPSP_BATCH_PLAIN && opts->batch != PPSP_BATCH_PLAINSTAR) return PPSP_E_INVALID;
    if (opts->sched != PPSP_SCHED_FIXED && opts->sched != PPSP_SCHED_AUTOTUNED) return PPSP_E_INVALID;
    if (opts->flags & (PPSP_WANT_PATH | PPSP_MEMO_H)) return PPSP_E_INVALID;
    if (g->served) return PPSP_E_BUSY;
    CHK(set_device(g));
    // the smallest wave: one query's two searches, the queues and the per-workgroup counters
    const uint64_t need = 2 * (uint64_t)g->n * 8 + 2 * 4096ull * 16 + (uint64_t)round_grid(g) * ST_N * 8 +
                          (g->maxdeg > HEAVY_DEG ? 4096ull * 32 : 0) + (1ull << 20);
    if (need > NOALLOC_SCRATCH_BYTES) {
        g_last_error = "no-allocation call: one query on this graph needs " + std::to_string(need) +
                       " bytes, the scratch holds " + std::to_string(NOALLOC_SCRATCH_BYTES);
        return PPSP_E_OOM;
    }
    char *base = nullptr;
    CHK(scratch_ptr(g->device, &base));
    // the graph's own workspace is set aside (and kept) for the duration of the call
    struct Swap {
        ppsp_graph g;
        std::vector<DevBuf> saved;
        hipStream_t st;
        uint64_t qcap;
        uint32_t hcap;
        int64_t profile, use_graph, dense_min, dense_force, heavy_waves;
        Arena arena;
        Swap(ppsp_graph g_, hipStream_t cs) : g(g_), st(g_->st), qcap(g_->qcap), hcap(g_->hcap),
                                             profile(g_->opt_profile), use_graph(g_->opt_use_graph),
                                             dense_min(g_->opt_dense_min), dense_force(g_->opt_dense_force),
                                             heavy_waves(g_->opt_heavy_waves) {
            for (DevBuf *b : wave_buffers(g)) saved.push_back(std::move(*b));
            g->st = cs;               // work is ordered on the caller's stream
            g->opt_profile = 0;       // no events
            g->opt_use_graph = 0;     // no captured graphs
            g->opt_dense_min = 0;     // sparse frontiers only (the dense bitmaps are not in the scratch)
            g->opt_dense_force = 0;
            g->opt_heavy_waves = 0;   // the per-workgroup counters in the scratch are sized for the round grid
            if (g->opt_queue_cap == 0) g->qcap = 0;
            g->hcap = 0;
        }
        ~Swap() {
            t_arena = nullptr;
            auto bufs = wave_buffers(g);
            for (size_t i = 0; i < bufs.size(); i++) {
                release(*bufs[i]);
                *bufs[i] = std::move(saved[i]);
            }
            g->st = st;
            g->qcap = qcap;
            g->hcap = hcap;
            g->opt_profile = profile;
            g->opt_use_graph = use_graph;
            g->opt_dense_min = dense_min;
            g->opt_dense_force = dense_force;
            g->opt_heavy_waves = heavy_waves;
        }
    } swap(g, (hipStream_t)hip_stream);
    swap.arena.base = base;
    swap.arena.size = NOALLOC_SCRATCH_BYTES;
    // search state takes at most five eighths of the scratch; queues and the rest share what is left
    swap.arena.state_budget = NOALLOC_SCRATCH_BYTES / 8 * 5;
    t_arena = &swap.arena;
    ppsp_opts o = *opts;
    if (o.flags & PPSP_DEVICE_IO) {
        // device-resident pairs and distances, staged through the host on the caller's stream
        o.flags &= ~PPSP_DEVICE_IO;
        hipStream_t cs = (hipStream_t)hip_stream;
        std::vector<uint32_t> hp(2ull * k);
        std::vector<uint64_t> hd(k);
        if (k) {
            HIPCHK(hipMemcpyAsync(hp.data(), pairs, 8ull * k, hipMemcpyDeviceToHost, cs));
            HIPCHK(hipStreamSynchronize(cs));
        }
        CHK(batch_impl(g, hp.data(), k, &o, hip_stream, hd.data(), nullptr, nullptr, 0, nullptr));
        if (k) {
            HIPCHK(hipMemcpyAsync(dist, hd.data(), 8ull * k, hipMemcpyHostToDevice, cs));
            HIPCHK(hipStreamSynchronize(cs));
        }
        return PPSP_OK;
    }
    return batch_impl(g, pairs, k, &o, hip_stream, dist, nullptr, nullptr, 0, nullptr);
}

int ppsp_query(ppsp_graph g, uint32_t s, uint32_t t, const ppsp_opts *opts, void *hip_stream, uint64_t *dist,
               uint32_t *path, uint32_t path_cap, uint32_t *path_len) {
    if (!g || !opts || !dist) return PPSP_E_INVALID;
    const bool want_path = opts->flags & PPSP_WANT_PATH;
    if (want_path && !path_len) return PPSP_E_INVALID;
    ppsp_opts o = *opts;
    o.batch = PPSP_BATCH_PLAIN;
    uint32_t pr[2] = {s, t};
    uint64_t off[2] = {0, 0};
    uint32_t need = 0;
    uint64_t d = 0;
    int rc = batch_impl(g, pr, 1, &o, hip_stream, &d, want_path ? off : nullptr, path, path ? path_cap : 0, &need);
    if (rc == PPSP_E_PATHCAP) { *path_len = need; return rc; }
    if (rc != PPSP_OK) return rc;
    *dist = d;
    if (want_path) *path_len = (uint32_t)(off[1] - off[0]);
    return PPSP_OK;
}

int ppsp_sssp(ppsp_graph g, uint32_t s, const ppsp_opts *opts, void *hip_stream, uint64_t *dist) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!g || !opts || !dist) return PPSP_E_INVALID;
    if (g->served) return PPSP_E_BUSY;
    if (s >= g->n) return PPSP_E_RANGE;
    if (opts->sched == PPSP_SCHED_LEARNED || opts->sched > PPSP_SCHED_RHO) return PPSP_E_INVALID;
    CHK(set_device(g));
    g->last = ppsp_stats{};
    hipEvent_t ev;
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIPCHK(hipEventRecord(ev, (hipStream_t)hip_stream));
    HIPCHK(hipStreamWaitEvent(g->st, ev, 0));
    (void)hipEventDestroy(ev);
    const uint32_t root = g->perm.empty() ? s : g->perm[s];
    const uint64_t delta = opts->delta ? opts->delta : graph_default_delta(g);
    // one search without pruning and without queries: it runs until its frontier is empty
    Plan P;
    P.G = 1;
    SearchDesc sd = make_sd(g, root, K_DIST, root, root);
    sd.noprune = 1;
    P.sd.push_back(sd);
    P.delta.push_back(key_delta(K_DIST, delta));
    P.bin.push_back((uint8_t)(MLP_K / 2));
    g->last.searches = 1;
    WaveOut w;
    CHK(run_wave(g, P, false, w));
    accumulate(g, w);
    std::vector<uint64_t> words(g->n);
    HIPCHK(hipMemcpyAsync(words.data(), g->S.p, (uint64_t)g->n * 8, hipMemcpyDeviceToHost, g->st));
    HIPCHK(hipStreamSynchronize(g->st));
    const bool re = !g->iperm.empty();
    for (uint32_t v = 0; v < g->n; v++) {
        const uint32_t d32 = (uint32_t)(words[v] >> 32);
        dist[re ? g->iperm[v] : v] = d32 == INF32 ? PPSP_INF : d32;
    }
    g->last.wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return PPSP_OK;
}

int ppsp_tune(ppsp_graph g, const uint32_t *pairs, uint32_t k, const ppsp_opts *opts, const char *cache_path,
              ppsp_tune_result *out) {
    if (!g || !pairs || k == 0 || !opts || !out) return PPSP_E_INVALID;
    CHK(check_opts(g, opts));
    auto &slot = g->tuned[opts->algo][opts->batch];
    char key[128];
    snprintf(key, sizeof key, "ppsp-tune-v5 %016llx %u %u", (unsigned long long)g->fingerprint, opts->algo, opts->batch);
    if (cache_path) {
        if (FILE *f = fopen(cache_path, "r")) {
            char line[256];
            while (fgets(line, sizeof line, f)) {
                unsigned long long d;
                long long mode, grid, hw, lc, dm, dr;
                double ms;
                if (strncmp(line, key, strlen(key)) == 0 &&
                    sscanf(line + strlen(key), " %llu %lld %lld %lld %lld %lld %lld %lf", &d, &mode, &grid, &hw, &lc, &dm,
                           &dr, &ms) == 8) {
                    slot.valid = true;
                    slot.delta = d;
                    slot.theta_mode = mode;
                    slot.grid = grid;
                    slot.hwin = hw;
                    slot.local = lc;
                    slot.dense_min = dm;
                    slot.dense_ring = dr;
                    slot.ms = ms;
                }
            }
            fclose(f);
            if (slot.valid) {
                *out = ppsp_tune_result{slot.delta, (uint32_t)slot.theta_mode, (uint32_t)slot.grid, slot.ms, 0, 0, 1,
                                        (uint32_t)slot.hwin, (uint32_t)slot.local, (uint64_t)slot.dense_min,
                                        (uint32_t)slot.dense_ring};
                return PPSP_OK;
            }
        }
    }
    std::vector<uint64_t> dist(k);
    ppsp_opts o = *opts;
    o.sched = PPSP_SCHED_FIXED;
    o.flags &= ~PPSP_WANT_PATH;
    const int64_t mode0 = g->opt_theta_mode, grid0 = g->opt_grid_blocks, hwin0 = g->opt_heavy_window,
                  local0 = g->opt_local, dmin0 = g->opt_dense_min, dring0 = g->opt_dense_ring;
    uint32_t trials = 0;
    int64_t best_hw = hwin0, best_local = local0, best_dmin = 0, best_dring = dring0;
    // wall time of one configuration (best of two runs; the first may allocate)
    auto trial = [&](uint64_t delta, int64_t mode, int64_t grid) -> double {
        g->opt_theta_mode = mode;
        g->opt_grid_blocks = grid;
        g->opt_heavy_window = best_hw;
        g->opt_local = best_local;
        g->opt_dense_min = best_dmin;
        g->opt_dense_ring = best_dring;
        o.delta = delta;
        double best = 1e300;
        for (int rep = 0; rep < 2; rep++) {
            if (batch_impl(g, pairs, k, &o, nullptr, dist.data(), nullptr, nullptr, 0, nullptr) != PPSP_OK) return 1e300;
            best = std::min(best, g->last.wall_ms);
        }
        trials++;
        return best;
    };
    const double default_ms = trial(graph_default_delta(g), 2, 0);
    // 1. Delta by doubling (Section 6.1: start small, double while the time improves).
    uint64_t d = std::max<uint64_t>(g->wmin ? g->wmin : 1, g->wmean / 16);
    uint64_t best_d = d;
    double best_ms = trial(d, 2, 0);
    int worse = 0;
    while (worse < 2 && d < 64 * g->wmean) {
        d *= 2;
        const double ms = trial(d, 2, 0);
        if (ms < best_ms) { best_ms = ms; best_d = d; worse = 0; } else worse++;
    }
    int64_t best_mode = 2, best_grid = 0;
    // 2. Refinement: the hub window (graphs with hubs), threshold rule,
    //    Delta between the doublings, launch shape.
    if (g->maxdeg > HEAVY_DEG) {
        const int64_t hw_start = best_hw;
        for (int64_t hw : {8, 64, 512}) {
            if (hw == hw_start) continue;
            const int64_t keep = best_hw;
            best_hw = hw;
            const double ms = trial(best_d, 2, 0);
            if (ms < best_ms) best_ms = ms; else best_hw = keep;
        }
    }
    for (int64_t mode : {0, 1}) {
        const double ms = trial(best_d, mode, 0);
        if (ms < best_ms) { best_ms = ms; best_mode = mode; }
    }
    const uint64_t base_d = best_d;
    for (double f : {0.7, 1.4}) {
        const uint64_t dd = std::max<uint64_t>(1, (uint64_t)(base_d * f));
        const double ms = trial(dd, best_mode, 0);
        if (ms < best_ms) { best_ms = ms; best_d = dd; }
    }
    for (int64_t per_cu : {12, 16}) {
        const double ms = trial(best_d, best_mode, per_cu * g->cu);
        if (ms < best_ms) { best_ms = ms; best_grid = per_cu * g->cu; }
    }
    // 3. Dense frontiers (Appendix B): the switch size, then the ring and a
    //    half-width step, which dense frontiers make cheaper (entries waiting
    //    for later buckets cost nothing per round)
    if (!(opts->flags & PPSP_PULL)) {
        for (int64_t dm : {1ll << 16, 1ll << 18}) {
            const int64_t keep = best_dmin;
            best_dmin = dm;
            const double ms = trial(best_d, best_mode, best_grid);
            if (ms < best_ms) best_ms = ms; else best_dmin = keep;
        }
        if (best_dmin) {
            // ring and step width together: a narrower step needs more buckets ahead
            const uint64_t d_dense = best_d;
            const int64_t ring0 = best_dring;
            const struct { int64_t ring; uint64_t div; } combo[] = {{ring0, 2}, {32, 1}, {32, 2}, {64, 2}, {64, 4}};
            int64_t win_ring = ring0;
            for (const auto &c : combo) {
                if (c.ring == ring0 && c.div == 1) continue;
                const uint64_t dd = std::max<uint64_t>(1, d_dense / c.div);
                best_dring = c.ring;
                const double ms = trial(dd, best_mode, best_grid);
                if (ms < best_ms) { best_ms = ms; best_d = dd; win_ring = c.ring; }
            }
            best_dring = win_ring;
        }
    }
    // 4. The local-chunk budget of heuristic searches (the only ones that use it by default).
    if (is_astar(opts->algo)) {
        const int64_t start = best_local;
        for (int64_t lc : {8, 32}) {
            if (lc == start) continue;
            const int64_t keep = best_local;
            best_local = lc;
            const double ms = trial(best_d, best_mode, best_grid);
            if (ms < best_ms) best_ms = ms; else best_local = keep;
        }
    }
    g->opt_theta_mode = mode0;
    g->opt_grid_blocks = grid0;
    g->opt_heavy_window = hwin0;
    g->opt_local = local0;
    g->opt_dense_min = dmin0;
    g->opt_dense_ring = dring0;
    if (best_ms >= 1e300) return PPSP_E_DEVICE;
    slot.valid = true;
    slot.delta = best_d;
    slot.theta_mode = best_mode;
    slot.grid = best_grid;
    slot.hwin = best_hw;
    slot.local = best_local;
    slot.dense_min = best_dmin;
    slot.dense_ring = best_dring;
    slot.ms = best_ms;
    if (cache_path) {
        if (FILE *f = fopen(cache_path, "a")) {
            fprintf(f, "%s %llu %lld %lld %lld %lld %lld %lld %.3f\n", key, (unsigned long long)best_d,
                    (long long)best_mode, (long long)best_grid, (long long)best_hw, (long long)best_local,
                    (long long)best_dmin, (long long)best_dring, best_ms);
            fclose(f);
        }
    }
    *out = ppsp_tune_result{best_d, (uint32_t)best_mode, (uint32_t)best_grid, best_ms, default_ms, trials, 0,
                            (uint32_t)best_hw, (uint32_t)best_local, (uint64_t)best_dmin, (uint32_t)best_dring};
    return PPSP_OK;
}

int ppsp_last_stats(ppsp_graph g, ppsp_stats *s) {
    if (!g || !s) return PPSP_E_INVALID;
    *s = g->last;
    return PPSP_OK;
}

int ppsp_set_option(ppsp_graph g, const char *name, int64_t v) {
    if (!g || !name) return PPSP_E_INVALID;
    if (g->served) return PPSP_E_BUSY;   // the server's worker reads the options
    std::string k(name);
    if (k == "profile") g->opt_profile = v;
    else if (k == "rounds_per_sync") { if (v < 1) return PPSP_E_INVALID; g->opt_rounds_per_sync = v; }
    else if (k == "grid_blocks") { if (v < 0) return PPSP_E_INVALID; g->opt_grid_blocks = v; }
    else if (k == "mem_budget_mb") { if (v < 0) return PPSP_E_INVALID; g->opt_mem_budget_mb = v; }
    else if (k == "default_delta") { if (v < 0) return PPSP_E_INVALID; g->opt_default_delta = v; }
    else if (k == "use_graph") g->opt_use_graph = v;
    else if (k == "timeout_ms") { if (v < 0) return PPSP_E_INVALID; g->opt_timeout_ms = v; }
    else if (k == "theta_mode") { if (v < 0 || v > 3) return PPSP_E_INVALID; g->opt_theta_mode = v; }
    else if (k == "queue_cap") { if (v < (int64_t)NSEG || v > (1ll << 31)) return PPSP_E_INVALID; g->qcap = (uint64_t)v; g->opt_queue_cap = v; }
    else if (k == "heavy_cap") { if (v < 1 || v > (1ll << 28)) return PPSP_E_INVALID; g->hcap = (uint32_t)v; }
    else if (k == "ml_every") { if (v < 1 || v > 1024) return PPSP_E_INVALID; g->opt_ml_every = v; }
    else if (k == "heavy_window") { if (v < 1 || v > 4096) return PPSP_E_INVALID; g->opt_heavy_window = v; }
    else if (k == "rho") { if (v < 1 || v > (1ll << 31)) return PPSP_E_INVALID; g->opt_rho = v; }
    else if (k == "local_chunks") { if (v < 0 || v > 1024) return PPSP_E_INVALID; g->opt_local = v; }
    else if (k == "local_chunks_plain") { if (v < 0 || v > 1024) return PPSP_E_INVALID; g->opt_local_plain = v; }
    else if (k == "local_fill") { if (v < 0 || v > (1ll << 31)) return PPSP_E_INVALID; g->opt_local_fill = v; }
    else if (k == "local_chunks_small") { if (v < 0 || v > 1024) return PPSP_E_INVALID; g->opt_local_small = v; }
    else if (k == "local_time_pct") { if (v < 0 || v > 100000) return PPSP_E_INVALID; g->opt_local_pct = v; }
    else if (k == "defer_time_pct") {
        // below 100 % a wave would defer before the average wave is done
        if (v < 0 || (v > 0 && v < 100) || v > 100000) return PPSP_E_INVALID;
        g->opt_defer_pct = v;
    }
    else if (k == "min_chunk") {
        if (v < 1 || v > (int64_t)WAVE || (v & (v - 1))) return PPSP_E_INVALID;
        g->opt_min_chunk = v;
    }
    else if (k == "multi_group") {
        if (v < 1 || v > 64 || (v & (v - 1))) return PPSP_E_INVALID;
        g->opt_multi_group = v;
    }
    else if (k == "plain_group") {
        if (v < 2 || v > 64 || (v & (v - 1))) return PPSP_E_INVALID;
        g->opt_plain_group = v;
    }
    else if (k == "heavy_grouped") {
        if (v < 0 || v > 1) return PPSP_E_INVALID;
        g->opt_heavy_grouped = v;
    }
    else if (k == "heavy_claim") {
        if (v < 1 || v > 64) return PPSP_E_INVALID;
        g->opt_heavy_claim = v;
    }
    else if (k == "list_deg") {
        if (v < 16 || v > (int64_t)HEAVY_DEG) return PPSP_E_INVALID;
        g->opt_list_deg = v;
    }
    else if (k == "heavy_waves") {
        if (v < 0 || v > 32) return PPSP_E_INVALID;
        g->opt_heavy_waves = v;
    }

    else if (k == "server_round_base") {
        if (v < 0 || v >= (int64_t)SRV_ROUND_LIMIT) return PPSP_E_INVALID;
        g->opt_server_round_base = v;
    }
    else if (k == "dense_min") { if (v < 0) return PPSP_E_INVALID; g->opt_dense_min = v; }
    else if (k == "dense_force") { if (v < 0 || v > 1) return PPSP_E_INVALID; g->opt_dense_force = v; }
    else if (k == "dense_learned") { if (v < 0 || v > 1) return PPSP_E_INVALID; g->opt_dense_learned = v; }
    else if (k == "dense_ring") {
        if (v < 2 || v > 64 || (v & (v - 1))) return PPSP_E_INVALID;   // a power of two
        g->opt_dense_ring = v;
    }

    else return PPSP_E_INVALID;
    return PPSP_OK;
}

int ppsp_get_option(ppsp_graph g, const char *name, int64_t *v) {
    if (!g || !name || !v) return PPSP_E_INVALID;
    std::string k(name);
    if (k == "profile") *v = g->opt_profile;
    else if (k == "rounds_per_sync") *v = g->opt_rounds_per_sync;
    else if (k == "grid_blocks") *v = g->opt_grid_blocks;
    else if (k == "mem_budget_mb") *v = g->opt_mem_budget_mb;
    else if (k == "default_delta") *v = (int64_t)graph_default_delta(g);
    else if (k == "use_graph") *v = g->opt_use_graph;
    else if (k == "timeout_ms") *v = g->opt_timeout_ms;
    else if (k == "theta_mode") *v = g->opt_theta_mode;
    else if (k == "queue_cap") *v = (int64_t)g->qcap;
    else if (k == "heavy_cap") *v = g->hcap;
    else if (k == "ml_every") *v = g->opt_ml_every;
    else if (k == "heavy_window") *v = g->opt_heavy_window;
    else if (k == "multi_group") *v = g->opt_multi_group;
    else if (k == "plain_group") *v = g->opt_plain_group;
    else if (k == "heavy_grouped") *v = g->opt_heavy_grouped;
    else if (k == "heavy_claim") *v = g->opt_heavy_claim;
    else if (k == "list_deg") *v = g->opt_list_deg;
    else if (k == "heavy_waves") *v = g->opt_heavy_waves;

    else if (k == "rho") *v = g->opt_rho;
    else if (k == "local_chunks") *v = g->opt_local;
    else if (k == "local_chunks_plain") *v = g->opt_local_plain;
    else if (k == "local_fill") *v = g->opt_local_fill;
    else if (k == "min_chunk") *v = g->opt_min_chunk;
    else if (k == "local_chunks_small") *v = g->opt_local_small;
    else if (k == "local_time_pct") *v = g->opt_local_pct;
    else if (k == "defer_time_pct") *v = g->opt_defer_pct;
    else if (k == "server_round_base") *v = g->opt_server_round_base;
    else if (k == "dense_min") *v = g->opt_dense_min;
    else if (k == "dense_force") *v = g->opt_dense_force;
    else if (k == "dense_learned") *v = g->opt_dense_learned;
    else if (k == "dense_ring") *v = g->opt_dense_ring;

    else return PPSP_E_INVALID;
    return PPSP_OK;
}


int ppsp_server_create(const ppsp_graph *graphs, uint32_t ngraphs, const ppsp_opts *opts, uint64_t state_budget,
                       ppsp_server *out) {
    if (!graphs || ngraphs == 0 || !opts || !out) return PPSP_E_INVALID;
    for (uint32_t i = 0; i < ngraphs; i++) {
        if (opts[i].algo != PPSP_BIDS && opts[i].algo != PPSP_BIDASTAR) return PPSP_E_INVALID;
        if (!graphs[i] || graphs[i]->served) return PPSP_E_INVALID;
        for (uint32_t j = 0; j < i; j++)
            if (graphs[j] == graphs[i]) return PPSP_E_INVALID;
        if (opts[i].algo == PPSP_BIDASTAR && !graphs[i]->xy_ok) return PPSP_E_NOCOORD;
        if (opts[i].sched != PPSP_SCHED_FIXED && opts[i].sched != PPSP_SCHED_LEARNED) return PPSP_E_INVALID;
        if (opts[i].sched == PPSP_SCHED_LEARNED && !graphs[i]->mlp_loaded) return PPSP_E_INVALID;
        if (graphs[i]->device != graphs[0]->device) return PPSP_E_INVALID;
    }
    ppsp_server srv = new ppsp_server_s();
    srv->opts.assign(opts, opts + ngraphs);
    // rounds between admission points: the first graph's rounds_per_sync, at least 2
    // (a finished slot must see one more round before it is reused)
    srv->rounds_per_chunk = (uint32_t)std::min<int64_t>(std::max<int64_t>(graphs[0]->opt_rounds_per_sync, 2), 1024);
    srv->gs.resize(ngraphs);
    uint64_t total_n = 0;
    for (uint32_t i = 0; i < ngraphs; i++) total_n += graphs[i]->n;
    for (uint32_t i = 0; i < ngraphs; i++) {
        srv->gs[i].g = graphs[i];
        // the budget is shared in proportion to the graphs' sizes: equal slots per vertex
        const uint64_t b = (uint64_t)((double)state_budget * graphs[i]->n / total_n);
        int rc = srv_setup_graph(srv, srv->gs[i], srv->opts[i], b);
        if (rc != PPSP_OK) {
            for (uint32_t j = 0; j <= i; j++) {
                if (srv->gs[j].h_done) (void)hipHostFree(srv->gs[j].h_done);
                if (srv->gs[j].h_mu) (void)hipHostFree(srv->gs[j].h_mu);
                release(srv->gs[j].ids);
            }
            delete srv;
            return rc;
        }
        graphs[i]->served = true;
    }
    srv->worker = std::thread(srv_worker, srv);
    *out = srv;
    return PPSP_OK;
}

int ppsp_server_submit(ppsp_server srv, uint32_t graph_id, const uint32_t *pairs, uint32_t k, uint64_t *req_id) {
    if (!srv || !req_id || (k && !pairs) || graph_id >= srv->gs.size()) return PPSP_E_INVALID;
    const uint32_t n = srv->gs[graph_id].g->n;
    for (uint64_t i = 0; i < 2ull * k; i++)
        if (pairs[i] >= n) return PPSP_E_RANGE;
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->err != PPSP_OK) return srv->err;
    const uint64_t id = srv->next_id++;
    SrvRequest &rq = srv->reqs[id];
    rq.graph = graph_id;
    rq.pairs.assign(pairs, pairs + 2ull * k);
    const std::vector<uint32_t> &perm = srv->gs[graph_id].g->perm;   // PPSP_REORDER: device ids
    if (!perm.empty())
        for (auto &v : rq.pairs) v = perm[v];
    rq.dist.assign(k, PPSP_INF);
    rq.remaining = k;
    rq.t_submit = std::chrono::steady_clock::now();
    if (k == 0) { rq.done = true; rq.t_done = rq.t_submit; srv->completed++; }
    else srv->pending.push_back(id);
    *req_id = id;
    srv->cv_work.notify_all();
    return PPSP_OK;
}

static int server_take(ppsp_server srv, uint64_t req_id, uint64_t *dist, double *latency_ms) {
    auto it = srv->reqs.find(req_id);
    if (it == srv->reqs.end()) return PPSP_E_INVALID;
    if (!it->second.done) return srv->err != PPSP_OK ? srv->err : PPSP_E_BUSY;
    if (dist) std::copy(it->second.dist.begin(), it->second.dist.end(), dist);
    if (latency_ms)
        *latency_ms = std::chrono::duration<double, std::milli>(it->second.t_done - it->second.t_submit).count();
    srv->reqs.erase(it);
    return PPSP_OK;
}

int ppsp_server_poll(ppsp_server srv, uint64_t req_id, uint64_t *dist, double *latency_ms) {
    if (!srv) return PPSP_E_INVALID;
    std::lock_guard<std::mutex> lk(srv->mu);
    return server_take(srv, req_id, dist, latency_ms);
}

int ppsp_server_wait(ppsp_server srv, uint64_t req_id, uint64_t *dist, double *latency_ms, uint32_t timeout_ms) {
    if (!srv) return PPSP_E_INVALID;
    std::unique_lock<std::mutex> lk(srv->mu);
    const auto until = std::chrono::steady_clock::now() + std::chrono::milliseconds(timeout_ms);
    for (;;) {
        const int rc = server_take(srv, req_id, dist, latency_ms);
        if (rc != PPSP_E_BUSY) return rc;
        if (srv->cv_done.wait_until(lk, until) == std::cv_status::timeout) return server_take(srv, req_id, dist, latency_ms);
    }
}

int ppsp_server_stats(ppsp_server srv, ppsp_server_counters *out) {
    if (!srv || !out) return PPSP_E_INVALID;
    std::lock_guard<std::mutex> lk(srv->mu);
    *out = ppsp_server_counters{};
    out->admitted = srv->admitted;
    out->completed = srv->completed;
    out->chunks = srv->chunks;
    out->rounds = srv->rounds;
    for (auto &G : srv->gs) { out->running += G.running; out->slots += G.C; }
    out->pending = srv->pending.size();
    out->restarts = srv->restarts;
    out->renumbers = srv->renumbers;
    return PPSP_OK;
}

int ppsp_server_destroy(ppsp_server srv) {
    if (!srv) return PPSP_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        srv->cv_work.notify_all();
    }
    if (srv->worker.joinable()) srv->worker.join();
    for (auto &G : srv->gs) {
        (void)hipStreamSynchronize(G.g->st);
        if (G.h_done) (void)hipHostFree(G.h_done);
        if (G.h_mu) (void)hipHostFree(G.h_mu);
        release(G.ids);
        G.g->served = false;
    }
    delete srv;
    return PPSP_OK;
}


int ppsp_mlp_forward(int device, const float *params, const float *x, uint32_t n, float *logits) {
    return mlp_forward_impl(device, params, x, n, logits);
}

int ppsp_mlp_grad(int device, const float *params, const float *x, const uint32_t *y, uint32_t n, float *grad,
                  double *loss) {
    if (!params || (n && (!x || !y)) || !grad) return PPSP_E_INVALID;
    for (uint32_t i = 0; i < n; i++)
        if (y[i] >= (uint32_t)MLP_Y) return PPSP_E_INVALID;
    MlpDev d;
    CHK(mlp_setup(device, d, params, x, y, n));
    return mlp_full_grad(d, n, grad, loss);
}

int ppsp_mlp_train(int device, float *params, const float *x, const uint32_t *y, uint32_t n, uint32_t epochs,
                   uint32_t batch, float lr, uint64_t seed, double *loss_first, double *loss_last) {
    return mlp_train_impl(device, params, x, y, n, epochs, batch, lr, seed, loss_first, loss_last);
}

int ppsp_mlp_load(ppsp_graph g, const float *params) { return mlp_load_impl(g, params); }

int ppsp_sched_trace(ppsp_graph g, const uint32_t *pairs, uint32_t k, const ppsp_opts *opts, const uint8_t *bins,
                     float *feat, uint32_t *row_pair, uint64_t cap, uint64_t *nrows, uint32_t *pair_rounds,
                     uint64_t *pair_arcs) {
    if (!g || !opts || (k && !pairs) || (cap && (!feat || !row_pair))) return PPSP_E_INVALID;
    if (g->served) return PPSP_E_BUSY;
    MlCtx c;
    std::vector<uint32_t> rp, pr;
    std::vector<uint64_t> pa;
    CHK(trace_impl(g, pairs, k, opts, bins, cap > 0, cap, c, rp, pr, pa));
    if (cap) {
        memcpy(feat, c.feat.data(), c.feat.size() * 4);
        memcpy(row_pair, rp.data(), rp.size() * 4);
    }
    if (nrows) *nrows = c.rows_total;
    if (pair_rounds) memcpy(pair_rounds, pr.data(), (uint64_t)k * 4);
    if (pair_arcs) memcpy(pair_arcs, pa.data(), (uint64_t)k * 8);
    return PPSP_OK;
}

int ppsp_sched_trace_ex(ppsp_graph g, const uint32_t *pairs, uint32_t k, const ppsp_opts *opts,
                        ppsp_trace_spec *spec) {
    if (!g || !opts || !spec || (k && !pairs)) return PPSP_E_INVALID;
    if (spec->cap && (!spec->feat || !spec->row_pair)) return PPSP_E_INVALID;
    if ((spec->switch_round != nullptr) != (spec->bins_after != nullptr)) return PPSP_E_INVALID;
    if (g->served) return PPSP_E_BUSY;
    CHK(check_opts(g, opts));
    TraceReq rq;
    rq.bins = spec->bins;
    rq.bins_after = spec->bins_after;
    rq.switch_round = spec->switch_round;
    rq.network = spec->network != 0;
    rq.distinct = spec->distinct != 0;
    rq.rows = spec->cap > 0;
    rq.cap = spec->cap;
    TraceOut out;
    CHK(trace_run(g, pairs, k, opts, rq, out));
    const uint64_t kept = out.row_pair.size();
    if (spec->cap) {
        memcpy(spec->feat, out.feat.data(), kept * MLP_F * 4);
        memcpy(spec->row_pair, out.row_pair.data(), kept * 4);
        if (spec->row_round) memcpy(spec->row_round, out.row_round.data(), kept * 4);
        if (spec->row_side) memcpy(spec->row_side, out.row_side.data(), kept);
        if (spec->row_bin) memcpy(spec->row_bin, out.row_bin.data(), kept);
    }
    spec->nrows = out.rows_total;
    if (spec->pair_rounds) memcpy(spec->pair_rounds, out.pair_rounds.data(), (uint64_t)k * 4);
    if (spec->pair_arcs) memcpy(spec->pair_arcs, out.pair_arcs.data(), (uint64_t)k * 8);
    if (spec->pair_entries) memcpy(spec->pair_entries, out.pair_ent.data(), (uint64_t)k * 8);
    if (spec->dist) memcpy(spec->dist, out.dist.data(), (uint64_t)k * 8);
    return PPSP_OK;
}

// Batch-aware labels: the sample batch under each fixed multiplier gives its
// wall time and, per pair, rounds and arcs. Batch time is fitted as
// c0 + c_round * rounds + c_arc * arcs; a pair's label is the bin that
// minimises c_arc * its arcs + c_round * its rounds beyond those of the best
// fixed batch (rounds that end before the batch does cost nothing).
int batch_labels(ppsp_graph g, const uint32_t *pairs, uint32_t k, const ppsp_opts *opts, std::vector<uint8_t> &y,
                 ppsp_fit_report &R) {
    std::vector<std::vector<uint32_t>> pr(MLP_K);
    std::vector<std::vector<uint64_t>> pa(MLP_K);
    double T[MLP_K], Rb[MLP_K], Ab[MLP_K];
    for (uint8_t b = 0; b < MLP_K; b++) {
        const std::vector<uint8_t> bins(k, b);
        double best = 1e300;
        for (int rep = 0; rep < 2; rep++) {
            MlCtx c;
            std::vector<uint32_t> rp;
            const auto a = std::chrono::steady_clock::now();
            CHK(trace_impl(g, pairs, k, opts, bins.data(), false, 0, c, rp, pr[b], pa[b]));
            best = std::min(best, std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - a).count());
        }
        T[b] = best;
        Rb[b] = *std::max_element(pr[b].begin(), pr[b].end());
        Ab[b] = 0;
        for (uint64_t v : pa[b]) Ab[b] += (double)v;
    }
    // least squares T = c0 + c1 R + c2 A (normal equations, 3 x 3), coefficients kept >= 0
    auto fit = [&](bool use_r, bool use_a, double &c0, double &c1, double &c2) {
        double M[3][4] = {{0}};
        for (int b = 0; b < MLP_K; b++) {
            const double x[3] = {1.0, use_r ? Rb[b] : 0.0, use_a ? Ab[b] : 0.0};
            for (int r = 0; r < 3; r++) {
                for (int c = 0; c < 3; c++) M[r][c] += x[r] * x[c];
                M[r][3] += x[r] * T[b];
            }
        }
        if (!use_r) { M[1][1] = 1; M[1][3] = 0; }
        if (!use_a) { M[2][2] = 1; M[2][3] = 0; }
        for (int c = 0; c < 3; c++) {
            int piv = c;
            for (int r = c + 1; r < 3; r++) if (std::fabs(M[r][c]) > std::fabs(M[piv][c])) piv = r;
            for (int j = 0; j < 4; j++) std::swap(M[c][j], M[piv][j]);
            if (std::fabs(M[c][c]) < 1e-30) continue;
            for (int r = 0; r < 3; r++) {
                if (r == c) continue;
                const double f = M[r][c] / M[c][c];
                for (int j = 0; j < 4; j++) M[r][j] -= f * M[c][j];
            }
        }
        c0 = M[0][3] / M[0][0];
        c1 = use_r ? M[1][3] / M[1][1] : 0.0;
        c2 = use_a ? M[2][3] / M[2][2] : 0.0;
    };
    double c0, cr, ca;
    fit(true, true, c0, cr, ca);
    if (cr < 0) fit(false, true, c0, cr, ca);
    if (ca < 0) fit(cr > 0, false, c0, cr, ca);
    uint32_t bbest = 0;
    for (uint32_t b = 1; b < (uint32_t)MLP_K; b++) if (T[b] < T[bbest]) bbest = b;
    const double Rstar = Rb[bbest];
    for (uint32_t i = 0; i < k; i++) {
        double best = 1e300;
        y[i] = (uint8_t)bbest;
        for (uint32_t b = 0; b < (uint32_t)MLP_K; b++) {
            const double cost = ca * (double)pa[b][i] + cr * std::max(0.0, (double)pr[b][i] - Rstar);
            if (cost < best - 1e-12) { best = cost; y[i] = (uint8_t)b; }
        }
    }
    R.c_round_ms = cr;
    R.c_arc_ns = ca * 1e6;
    R.best_fixed_bin = bbest;
    return PPSP_OK;
}

}  // extern "C"

namespace {

// Batch time T = c0 + c_r R + c_a A + c_e E by least squares over the fixed
// bins, with every coefficient non-negative: the best fit among the subsets of
// (R, A, E) whose own least-squares coefficients are all non-negative, taken
// among the subsets with the rounds term whenever one of those qualifies
// (every round has a cost; rounds and entries both fall as the step grows,
// and a fit that credits the entries alone labels steps that add rounds).
void fit_cost4(int nb, const double *T, const double *Rb, const double *Ab, const double *Eb, double &c0, double &cr,
               double &ca, double &ce) {
    double best_err = 1e300;
    c0 = T[0];
    cr = ca = ce = 0;
    for (int pass = 0; pass < 2 && best_err == 1e300; pass++)
    for (int mask = 0; mask < 8; mask++) {
        if (pass == 0 && !(mask & 1)) continue;     // first the subsets with the rounds term
        const double *col[3] = {Rb, Ab, Eb};
        int idx[3], m = 0;
        for (int j = 0; j < 3; j++)
            if (mask >> j & 1) idx[m++] = j;
        // normal equations of [1, cols] (up to 4 x 4), Gauss-Jordan with pivoting
        double M[4][5] = {{0}};
        for (int b = 0; b < nb; b++) {
            double x[4] = {1.0, 0, 0, 0};
            for (int j = 0; j < m; j++) x[j + 1] = col[idx[j]][b];
            for (int r = 0; r <= m; r++) {
                for (int c = 0; c <= m; c++) M[r][c] += x[r] * x[c];
                M[r][4] += x[r] * T[b];
            }
        }
        bool ok = true;
        for (int c = 0; c <= m && ok; c++) {
            int piv = c;
            for (int r = c + 1; r <= m; r++) if (std::fabs(M[r][c]) > std::fabs(M[piv][c])) piv = r;
            for (int j = 0; j < 5; j++) std::swap(M[c][j], M[piv][j]);
            if (std::fabs(M[c][c]) < 1e-300) { ok = false; break; }
            for (int r = 0; r <= m; r++) {
                if (r == c) continue;
                const double f = M[r][c] / M[c][c];
                for (int j = 0; j < 5; j++) M[r][j] -= f * M[c][j];
            }
        }
        if (!ok) continue;
        double coef[4];
        for (int j = 0; j <= m; j++) coef[j] = M[j][4] / M[j][j];
        bool nonneg = true;
        for (int j = 1; j <= m; j++) nonneg = nonneg && coef[j] >= 0;
        if (!nonneg) continue;
        double err = 0;
        for (int b = 0; b < nb; b++) {
            double p = coef[0];
            for (int j = 0; j < m; j++) p += coef[j + 1] * col[idx[j]][b];
            err += (p - T[b]) * (p - T[b]);
        }
        if (err < best_err) {
            best_err = err;
            c0 = coef[0];
            cr = ca = ce = 0;
            for (int j = 0; j < m; j++) (idx[j] == 0 ? cr : idx[j] == 1 ? ca : ce) = coef[j + 1];
        }
    }
}

double wall_ms_since(std::chrono::steady_clock::time_point a) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - a).count();
}

// label_mode 2 of ppsp_mlp_fit (see include/ppsp.h).
int fit_counterfactual(ppsp_graph g, const uint32_t *pairs, uint32_t k, const ppsp_opts *opts, const float *init,
                       uint32_t epochs, uint64_t seed, float *params_out, ppsp_fit_report &R) {
    const auto t0 = std::chrono::steady_clock::now();
    const uint32_t kt = k >= 8 ? (3 * k + 3) / 4 : k;             // training pairs
    const uint32_t *hp = k >= 8 ? pairs + 2ull * kt : pairs;       // held-out pairs of the referee
    const uint32_t hk = k >= 8 ? k - kt : k;
    ppsp_opts o = *opts;
    o.sched = PPSP_SCHED_FIXED;
    o.flags &= ~(uint32_t)(PPSP_WANT_PATH | PPSP_DEVICE_IO);
    const uint32_t every = (uint32_t)std::max<int64_t>(1, g->opt_ml_every);
    // 1. Every fixed bin on the training pairs: batch time, and per pair rounds, arcs, entries.
    double T[MLP_K], Rb[MLP_K], Ab[MLP_K], Eb[MLP_K];
    {
        TraceReq warm;
        TraceOut w;
        CHK(trace_run(g, pairs, kt, &o, warm, w));                 // buffers grown once, untimed
    }
    for (uint32_t b = 0; b < (uint32_t)MLP_K; b++) {
        const std::vector<uint8_t> bins(kt, (uint8_t)b);
        TraceReq rq;
        rq.bins = bins.data();
        TraceOut out;
        const auto a = std::chrono::steady_clock::now();
        CHK(trace_run(g, pairs, kt, &o, rq, out));
        T[b] = wall_ms_since(a);
        Rb[b] = *std::max_element(out.pair_rounds.begin(), out.pair_rounds.end());
        Ab[b] = Eb[b] = 0;
        for (uint32_t i = 0; i < kt; i++) { Ab[b] += (double)out.pair_arcs[i]; Eb[b] += (double)out.pair_ent[i]; }
    }
    double c0, cr, ca, ce;
    fit_cost4(MLP_K, T, Rb, Ab, Eb, c0, cr, ca, ce);
    uint32_t bbest = 0;
    for (uint32_t b = 1; b < (uint32_t)MLP_K; b++) if (T[b] < T[bbest]) bbest = b;
    const double Rstar = Rb[bbest];
    R.c_round_ms = cr;
    R.c_arc_ns = ca * 1e6;
    R.c_entry_ns = ce * 1e6;
    R.best_fixed_bin = bbest;
    // 2. The base trajectory (bin 4) with its feature rows.
    TraceReq dq;
    dq.rows = true;
    dq.cap = 1ull << 22;
    TraceOut base;
    CHK(trace_run(g, pairs, kt, &o, dq, base));
    // 3. Replays: the base bin until a decision round, then each bin to the
    //    end, with a sparse frontier and (bins 8..15) switched to dense there.
    constexpr int NPOINT = 6;
    constexpr uint32_t NVAR = 2 * MLP_K;
    std::vector<uint32_t> vp, vsw, vq, vr;
    std::vector<uint8_t> vb, v4;
    std::vector<std::vector<uint32_t>> points(kt);
    for (uint32_t q = 0; q < kt; q++) {
        if (pairs[2 * q] == pairs[2 * q + 1] || base.pair_rounds[q] == 0) continue;
        const uint32_t Rq = base.pair_rounds[q];
        for (int j = 0; j < NPOINT; j++) {
            const uint32_t r = (uint32_t)((uint64_t)j * Rq / NPOINT) / every * every;   // a decision round
            if (r >= Rq || (!points[q].empty() && points[q].back() == r)) continue;
            points[q].push_back(r);
            for (uint32_t b = 0; b < NVAR; b++) {
                vp.push_back(pairs[2 * q]);
                vp.push_back(pairs[2 * q + 1]);
                vsw.push_back(r + 1);            // the step chosen after round r runs bin b
                vb.push_back((uint8_t)b);
                v4.push_back((uint8_t)(MLP_K / 2));
                vq.push_back(q);
                vr.push_back(r);
            }
        }
    }
    const uint32_t nv = (uint32_t)vq.size();
    R.variants = nv;
    // in batches of at most 256 replays, the size of batch whose frontier
    // queues and hub list are known to fit (all replays at once can hold
    // several times the frontier entries)
    TraceOut rep;
    constexpr uint32_t VCHUNK = 256;
    for (uint32_t v0 = 0; v0 < nv; v0 += VCHUNK) {
        const uint32_t nc = std::min(VCHUNK, nv - v0);
        TraceReq vq_;
        vq_.bins = v4.data() + v0;
        vq_.bins_after = vb.data() + v0;
        vq_.switch_round = vsw.data() + v0;
        vq_.distinct = true;
        TraceOut part;
        CHK(trace_run(g, vp.data() + 2ull * v0, nc, &o, vq_, part));
        rep.pair_rounds.insert(rep.pair_rounds.end(), part.pair_rounds.begin(), part.pair_rounds.end());
        rep.pair_arcs.insert(rep.pair_arcs.end(), part.pair_arcs.begin(), part.pair_arcs.end());
        rep.pair_ent.insert(rep.pair_ent.end(), part.pair_ent.begin(), part.pair_ent.end());
    }
    // 4. Labels per (pair, switch point): the bin and frontier mode of lowest
    //    fitted remaining cost (the base, sparse bin 4, unless another is at
    //    least 1% cheaper), as y = bin + 8 * (1 sparse | 2 dense).
    std::map<std::pair<uint32_t, uint32_t>, uint8_t> label;
    uint32_t dense_labels = 0;
    for (uint32_t v0 = 0; v0 < nv; v0 += NVAR) {
        double cost[NVAR];
        for (uint32_t b = 0; b < NVAR; b++) {
            const uint32_t v = v0 + b;
            cost[b] = ca * (double)rep.pair_arcs[v] + ce * (double)rep.pair_ent[v] +
                      cr * std::max(0.0, (double)rep.pair_rounds[v] - Rstar);
            // a dense frontier reads its search's bitmap of n bits every round
            // from the switch on (two searches), priced at 4 TB/s: a cost the
            // fixed-bin fit cannot see
            if (b >= (uint32_t)MLP_K)
                cost[b] += 2.0 * ((double)g->n / 8.0) / 4e9 * std::max(0.0, (double)rep.pair_rounds[v] - vr[v]);
        }
        uint32_t lb = MLP_K / 2;
        for (uint32_t b = 0; b < NVAR; b++)
            if (cost[b] < cost[lb] && cost[b] < cost[MLP_K / 2] * 0.99) lb = b;
        const bool dn = lb >= (uint32_t)MLP_K;
        label[{vq[v0], vr[v0]}] = (uint8_t)((lb & (MLP_K - 1)) + MLP_K * (dn ? 2 : 1));
        R.label_hist[lb & (MLP_K - 1)]++;
        dense_labels += dn;
    }
    R.dense_labels = dense_labels;
    // rows: the base trajectory's decision rounds, each labelled by the switch
    // point at or before it
    std::vector<float> X;
    std::vector<uint32_t> Y;
    for (size_t r = 0; r < base.row_pair.size(); r++) {
        const uint32_t q = base.row_pair[r], rr = base.row_round[r];
        if (q >= kt || rr % every != 0 || points[q].empty()) continue;
        uint32_t pt = points[q][0];
        for (uint32_t p : points[q]) if (p <= rr) pt = p;
        if (pt > rr) continue;
        X.insert(X.end(), base.feat.begin() + r * MLP_F, base.feat.begin() + (r + 1) * MLP_F);
        Y.push_back(label[{q, pt}]);
    }
    R.rows = Y.size();
    R.label_ms = wall_ms_since(t0);
    // 5. Training on the GPU.
    auto t1 = std::chrono::steady_clock::now();
    memcpy(params_out, init, MLP_NPARAM * 4);
    if (!Y.empty())
        CHK(mlp_train_impl(g->device, params_out, X.data(), Y.data(), (uint32_t)Y.size(), epochs,
                           std::min<uint32_t>(256, (uint32_t)Y.size()), 2e-3f, seed, &R.loss_first, &R.loss_last));
    R.train_ms = wall_ms_since(t1);
    if (!Y.empty()) {
        // a row is right when its bin and (where labelled) its mode are
        std::vector<float> lg((uint64_t)Y.size() * MLP_O);
        CHK(mlp_forward_impl(g->device, params_out, X.data(), (uint32_t)Y.size(), lg.data()));
        uint64_t hit = 0;
        for (size_t r = 0; r < Y.size(); r++) {
            uint32_t bb = 0;
            for (uint32_t b = 1; b < (uint32_t)MLP_K; b++) if (lg[r * MLP_O + b] > lg[r * MLP_O + bb]) bb = b;
            const uint32_t m = Y[r] / MLP_K;
            const bool mode_ok = m == 0 || ((lg[r * MLP_O + MLP_K] > 0.f) == (m == 2));
            hit += bb == Y[r] % MLP_K && mode_ok;
        }
        R.train_acc = (double)hit / Y.size();
    }
    // 6. The referee, on held-out pairs: the trained network against the plain
    //    fixed-Delta path (base Delta, the graph's threshold rule). The
    //    network's mode output is used when some label asked for a dense frontier.
    CHK(mlp_load_impl(g, params_out));
    g->opt_dense_learned = dense_labels > 0 ? 1 : 0;
    R.heldout = hk;
    std::vector<uint64_t> dd(hk);
    ppsp_opts lo = o;
    lo.sched = PPSP_SCHED_LEARNED;
    R.heldout_learned_ms = R.heldout_fixed_ms = 1e300;
    for (int rep2 = 0; rep2 < 2; rep2++) {
        auto a = std::chrono::steady_clock::now();
        CHK(batch_impl(g, hp, hk, &lo, nullptr, dd.data(), nullptr, nullptr, 0, nullptr));
        R.heldout_learned_ms = std::min(R.heldout_learned_ms, wall_ms_since(a));
        a = std::chrono::steady_clock::now();
        CHK(batch_impl(g, hp, hk, &o, nullptr, dd.data(), nullptr, nullptr, 0, nullptr));
        R.heldout_fixed_ms = std::min(R.heldout_fixed_ms, wall_ms_since(a));
    }
    // fitted costs of the two held-out runs (traced: same schedules, counters kept)
    {
        TraceReq nq;
        nq.network = true;
        TraceOut nl, nf;
        CHK(trace_run(g, hp, hk, &o, nq, nl));
        TraceReq fq;
        CHK(trace_run(g, hp, hk, &o, fq, nf));
        auto cost = [&](const TraceOut &t) {
            double a = 0, e = 0, rmax = 0;
            for (uint32_t i = 0; i < hk; i++) {
                a += (double)t.pair_arcs[i];
                e += (double)t.pair_ent[i];
                rmax = std::max(rmax, (double)t.pair_rounds[i]);
            }
            return c0 + cr * rmax + ca * a + ce * e;
        };
        R.heldout_learned_cost = cost(nl);
        R.heldout_fixed_cost = cost(nf);
    }
    R.fallback_bin = MLP_K;
    R.learned_ms = R.heldout_learned_ms;
    R.fixed_ms = R.heldout_fixed_ms;
    if (R.heldout_fixed_ms < R.heldout_learned_ms) {
        g->ml_plain = true;            // LEARNED runs the plain fixed path on this graph
        R.plain_fallback = 1;
    }
    return PPSP_OK;
}

}  // namespace

extern "C" {

int ppsp_mlp_fit(ppsp_graph g, const uint32_t *pairs, uint32_t k, const ppsp_opts *opts, const float *init,
                 uint32_t epochs, uint64_t seed, uint32_t label_mode, float *params_out, ppsp_fit_report *rep) {
    if (!g || !opts || !pairs || k == 0 || !init || !params_out || label_mode > 2) return PPSP_E_INVALID;
    if (g->served) return PPSP_E_BUSY;
    if (opts->batch != PPSP_BATCH_PLAIN && opts->batch != PPSP_BATCH_PLAINSTAR) return PPSP_E_INVALID;
    CHK(check_opts(g, opts));
    for (uint64_t i = 0; i < 2ull * k; i++)
        if (pairs[i] >= g->n) return PPSP_E_RANGE;
    if (label_mode == 2) {
        ppsp_fit_report R{};
        CHK(fit_counterfactual(g, pairs, k, opts, init, epochs, seed, params_out, R));
        if (rep) *rep = R;
        return PPSP_OK;
    }
    ppsp_fit_report R{};
    auto t0 = std::chrono::steady_clock::now();
    std::vector<uint8_t> y(k, (uint8_t)(MLP_K / 2));
    ppsp_opts one = *opts;
    one.batch = PPSP_BATCH_PLAIN;
    // 1. Labels. Mode 1: batch-aware (batch_labels). Mode 0: each pair alone
    //    under every fixed multiplier; the label is the bin that finished it
    //    fastest (best of two runs).
    if (label_mode == 1) CHK(batch_labels(g, pairs, k, opts, y, R));
    for (uint32_t i = 0; i < k && label_mode == 0; i++) {
        if (pairs[2 * i] == pairs[2 * i + 1]) continue;
        double best = 1e300;
        for (uint8_t b = 0; b < MLP_K; b++) {
            double tb = 1e300;
            for (int rep2 = 0; rep2 < 2; rep2++) {
                MlCtx c;
                std::vector<uint32_t> rp, pr;
                std::vector<uint64_t> pa;
                const auto a = std::chrono::steady_clock::now();
                CHK(trace_impl(g, pairs + 2ull * i, 1, &one, &b, false, 0, c, rp, pr, pa));
                tb = std::min(tb, std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - a).count());
            }
            if (tb < best) { best = tb; y[i] = b; }
        }
    }
    for (uint32_t i = 0; i < k; i++) R.label_hist[y[i]]++;
    R.label_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    // 2. Feature rows along the labelled trajectories and the default one.
    std::vector<float> X;
    std::vector<uint32_t> Y;
    const uint64_t cap = 1ull << 21;
    for (int pass = 0; pass < 2; pass++) {
        std::vector<uint8_t> bins(k, (uint8_t)(MLP_K / 2));
        if (pass == 0) bins = y;
        MlCtx c;
        std::vector<uint32_t> rp, pr;
        std::vector<uint64_t> pa;
        CHK(trace_impl(g, pairs, k, opts, bins.data(), true, cap, c, rp, pr, pa));
        X.insert(X.end(), c.feat.begin(), c.feat.end());
        for (uint32_t q : rp) Y.push_back(y[q]);
    }
    R.rows = Y.size();
    // 3. Training on the GPU.
    t0 = std::chrono::steady_clock::now();
    memcpy(params_out, init, MLP_NPARAM * 4);
    CHK(mlp_train_impl(g->device, params_out, X.data(), Y.data(), (uint32_t)Y.size(), epochs, 512, 2e-3f, seed,
                       &R.loss_first, &R.loss_last));
    R.train_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    // 4. Training accuracy and loading.
    std::vector<float> lg((uint64_t)Y.size() * MLP_O);
    CHK(mlp_forward_impl(g->device, params_out, X.data(), (uint32_t)Y.size(), lg.data()));
    uint64_t hit = 0;
    for (size_t r = 0; r < Y.size(); r++) {
        uint32_t best = 0;
        for (uint32_t b = 1; b < (uint32_t)MLP_K; b++)
            if (lg[r * MLP_O + b] > lg[r * MLP_O + best]) best = b;
        hit += best == Y[r];
    }
    R.train_acc = Y.empty() ? 0.0 : (double)hit / Y.size();
    // 5. Fixed-Delta stepping referees the network. The sample batch runs under
    //    the trained network and under constant networks that always pick the
    //    base multiplier (bin 4) or, with batch labels, the fastest fixed one;
    //    all through the same learned-schedule path. If a constant network is
    //    faster, it is the one installed (and returned).
    const std::vector<float> trained(params_out, params_out + MLP_NPARAM);
    auto constant_net = [](uint32_t b) {
        std::vector<float> p(MLP_NPARAM, 0.f);
        p[MLP_B3 + b] = 1.f;   // output bias: the logits are constant, argmax b (mode logit 0: sparse)
        return p;
    };
    ppsp_opts lo = *opts;
    lo.sched = PPSP_SCHED_LEARNED;
    lo.flags &= ~(uint32_t)PPSP_WANT_PATH;
    std::vector<uint64_t> jd(k);
    auto time_net = [&](const float *p, double &ms) -> int {
        CHK(mlp_load_impl(g, p));
        ms = 1e300;
        for (int r = 0; r < 2; r++) {   // best of two (the first run may grow buffers)
            const auto a = std::chrono::steady_clock::now();
            CHK(batch_impl(g, pairs, k, &lo, nullptr, jd.data(), nullptr, nullptr, 0, nullptr));
            ms = std::min(ms, std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - a).count());
        }
        return PPSP_OK;
    };
    CHK(time_net(trained.data(), R.learned_ms));
    std::vector<uint32_t> cand{(uint32_t)(MLP_K / 2)};
    if (label_mode == 1 && R.best_fixed_bin != (uint32_t)(MLP_K / 2)) cand.push_back(R.best_fixed_bin);
    uint32_t fb = cand[0];
    R.fixed_ms = 1e300;
    for (uint32_t b : cand) {
        double ms = 0;
        CHK(time_net(constant_net(b).data(), ms));
        if (ms < R.fixed_ms) { R.fixed_ms = ms; fb = b; }
    }
    R.fallback_bin = MLP_K;
    if (R.fixed_ms < R.learned_ms) {
        const std::vector<float> p = constant_net(fb);
        memcpy(params_out, p.data(), MLP_NPARAM * 4);
        R.fallback_bin = fb;
    }
    CHK(mlp_load_impl(g, params_out));
    if (rep) *rep = R;
    return PPSP_OK;
}

}  // extern "C"
