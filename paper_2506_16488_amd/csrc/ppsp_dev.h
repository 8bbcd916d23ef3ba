// Device-side data layout and helpers of the gfx950 point-to-point
// shortest-path engine.
//
// Search state. Every search (one frontier copy v^(i) in the notation of
// Section 3.1: the forward or backward copy of a bidirectional query, or the
// copy rooted at query-graph vertex q_i in Multi-BiDS, Section 4.2) owns n
// 64-bit words:
//     bits 63..32  tentative distance delta[v^(i)] (0xFFFFFFFF = +infinity)
//     bits 31..0   stamp: 1 + the round in which the word last changed
// so WriteMin of Section 2 (write if smaller, report success) is one 64-bit
// atomicMin of (candidate << 32 | stamp); success is a strict decrease of the
// distance field, and the returned old word tells whether the vertex was
// already lowered, and so already added to the next frontier, in this round.
// Add (Algorithm 1: add v unless already present) therefore needs no extra
// memory. Every frontier entry records the stamp of the round that added it;
// an entry whose vertex has been lowered in a later round (word stamp newer
// than the entry's) is stale, because that later lowering added a fresh
// entry (or pruned the vertex), and is dropped. So an entry kept for a later
// round is simply added again, with no atomic and no duplicate work.
// Stamp 0 also marks a word whose vertex a wave has taken from its own list
// in the round that added it (local chunks, see the round kernel): a later
// lowering in that round then adds the vertex again.
// Parents are not stored: every vertex of an exact
// path has a tight in-arc (delta[p] + w(p,v) = delta[v]) to an exact vertex,
// so paths are recovered by walking tight arcs back to the root.
// Words are grouped G searches at a time, vertex-major inside a group:
//     S[((i / G) * n + v) * G + i % G]
// Bidirectional Plain and Plain* batches ("pair2") number a query's forward
// and backward copies 2q and 2q + 1, so with any even G they sit side by side
// and one 16-byte load returns both delta[v+] and delta[v-] (the two terms of
// UpdateDistance). G = 2 is one query per group; a larger G also puts the
// words of G / 2 queries for one vertex in the same lines (option
// "plain_group"). G = 1 is plain search-major. Multi-BiDS groups
// G consecutive query-graph vertices (by default 32: the copies of v for the
// searches of one component share a few cache lines, the vertex-major layout
// of Section 4.2), so its UpdateDistance over the neighbours in the query
// graph reads few lines.
//
// Frontier. Queues of 16-byte entries (search, vertex, stamp when added,
// heuristic term) per round parity. An entry kept for a later round holds
// its key instead of the heuristic term (CARRY_BIT in the search field). A queue is NSEG segments; a wave appends
// to segment (workgroup id mod NSEG), which spreads the append counters over
// NSEG addresses, and the next round walks the segments as one list of
// WAVE-entry chunks through a prefix sum of their chunk counts.
//
// Keys. Extraction and pruning compare integer keys (Table 2), doubled where
// the paper halves mu so that everything stays exact:
//     K_DIST    key = delta                      (early termination, SSSP)
//     K_ASTAR   key = delta + h_t(v)             (A*)
//     K_2DIST   key = 2 delta                    (BiDS, Multi-BiDS: delta >= mu/2)
//     K_BIDA_F  key = 2 delta + h_t(v) - h_s(v)  (BiD-A* forward:  delta + h_F >= mu/2)
//     K_BIDA_B  key = 2 delta - h_t(v) + h_s(v)  (BiD-A* backward: delta + h_B >= mu/2)
// with h_F = (h_t - h_s)/2 = -h_B (Section 3.5). The vertex-only term
// (0, h_t, h_t - h_s or h_s - h_t) is the entry's heuristic term hk, so a key
// is scale * delta + hk with scale 1 or 2. A search prunes a vertex when
// key >= bound, bound being mu of its query (or mumax[i] of Table 2's
// Multi-PPSP row); bound = 0 marks a finished search.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ppsp {

constexpr uint32_t INF32 = 0xFFFFFFFFu;
constexpr uint64_t INF64 = ~0ull;
constexpr uint32_t TARGET_BIT = 0x80000000u;  // Partner.other: a target vertex, not a search
constexpr uint32_t CARRY_BIT = 0x80000000u;   // frontier entry .x: carried entry, .w holds its key
constexpr uint32_t DENSE_BIT = 0x40000000u;   // entry .x inside the round kernel: taken from a dense bitmap
constexpr uint32_t KEY_UNKNOWN = 0xFFFFFFFFu; // carried key too large for 32 bits
constexpr int BLOCK = 256;                     // threads per block (four wave64s)
constexpr int WAVE = 64;
constexpr int WSTAGE = 256;                    // LDS staging slots per wave (round kernel)
constexpr uint32_t HEAVY_DEG = 512;            // extracted vertices above this go to the heavy list
constexpr uint32_t HEAVY_CHUNK = 2048;         // arcs per heavy-list chunk
constexpr int NSEG = 64;                       // append segments of a frontier queue

constexpr uint32_t ERR_OVERFLOW = 1u;          // a distance reached 2^32-1
constexpr uint32_t ERR_QUEUE = 2u;             // the frontier queue overflowed
constexpr uint32_t ERR_PATH = 4u;              // a tight-arc walk did not reach its root
constexpr uint32_t ERR_HEAVY = 8u;             // the heavy list overflowed

enum KeyKind : uint32_t { K_DIST = 0, K_ASTAR = 1, K_2DIST = 2, K_BIDA_F = 3, K_BIDA_B = 4 };

// Per-search constant description (uploaded once per wave).
struct SearchDesc {
    uint32_t src;       // root vertex of this search
    uint32_t kind;      // KeyKind
    uint32_t pbeg;      // partner list [pbeg, pend) in the partner array
    uint32_t pend;
    int32_t tx, ty;     // coordinates of the target t (h_t), A* kinds only
    int32_t sx, sy;     // coordinates of the source s (h_s), bidirectional A* only
    uint32_t noprune;   // 1: never prune (plain single-source search)
    uint32_t rev;       // 1: the search walks arcs backwards (the transpose), as the backward
                        //    search of a bidirectional query on a directed graph does
};

// One query the search takes part in: the other endpoint (a search index, or
// TARGET_BIT | t for a one-sided search towards t) and the query's mu slot.
struct Partner {
    uint32_t other;
    uint32_t pair;
};

// For path extraction: the two roots of a query's mu slot.
struct PairDesc {
    uint32_t a;         // search rooted at the query's first endpoint
    uint32_t b;         // search rooted at the second endpoint, or TARGET_BIT | t
};

// floor(sqrt(q)) for q < 2^63, exact: a double-precision estimate corrected
// by exact integer steps.
__host__ __device__ inline uint64_t isqrt_floor(uint64_t q) {
    uint64_t x = (uint64_t)sqrt((double)q);
    while (x * x > q) x--;
    while ((x + 1) * (x + 1) <= q) x++;
    return x;
}

// Euclidean heuristic on fixed-point coordinates:
// floor(w_scale * |p - p'| / 2^fb) = floor(isqrt(w_scale^2 * d2) / 2^fb).
__host__ __device__ inline uint64_t heur(int32_t x0, int32_t y0, int32_t x1, int32_t y1,
                                         uint64_t ws2, uint32_t fb) {
    int64_t dx = (int64_t)x1 - x0, dy = (int64_t)y1 - y0;
    uint64_t d2 = (uint64_t)(dx * dx) + (uint64_t)(dy * dy);
    return isqrt_floor(ws2 * d2) >> fb;
}

// Everything a round needs, passed by value to each kernel.
struct RoundArgs {
    // graph
    const uint32_t *row_ptr;   // n+1
    const uint2 *arcs;         // m: (neighbour, weight)
    const uint32_t *in_row_ptr;  // transpose (same arrays on a symmetric graph), for path walks
    const uint2 *in_arcs;
    const int2 *xy;            // n fixed-point coordinates or null
    uint64_t ws2;              // w_scale^2
    uint32_t fb;               // coordinate fractional bits
    uint32_t n;
    // searches
    const SearchDesc *sd;
    const Partner *partners;
    uint32_t nsearch;
    uint32_t npair;
    uint32_t G;                // searches per interleaved group (a power of two)
    uint32_t pair2;            // 1: searches 2q and 2q + 1 are one query's forward and backward copies
    uint64_t *S;               // packed (distance, stamp) words, layout above
    ulonglong2 *ctl;           // [nsearch] (theta, bound) in key units; bound 0 = finished
    const uint64_t *delta;     // [nsearch] threshold increment (key units)
    uint32_t *done;            // [nsearch]
    uint32_t *exh;             // [nsearch] frontier ran dry while the bound was infinite
    uint32_t *alive;           // [2][nsearch] 1 if the search added anything to that frontier
    uint64_t *minkey;          // [2][nsearch] smallest key added to the next frontier
    uint64_t *mu;              // [npair] packed (distance, meeting vertex)
    uint4 *q0, *q1;            // frontier queues by round parity, NSEG segments of qseg entries
    uint32_t *qcount;          // [2][NSEG] segment lengths
    uint32_t *cpre;            // [2][NSEG + 1]: [0] entries per chunk, [k + 1] prefix sums of the
                               // chunk counts of segments 0..k
    uint64_t qseg;             // capacity of one segment (entries)
    uint32_t *round;           // [0] round to run next (read by k_round), [1] round just run (k_control)
    uint4 *heavy;              // [hcap][2] arc chunks of this round's extracted high-degree vertices:
                               //   (search, vertex, distance, first arc), (end arc, 0, 0, 0)
    unsigned long long *hcount;  // [0] chunks written this round, [1] claim counter of the hub-list kernel
    uint32_t hclaim;           // hub-list records a wave claims at a time
    uint32_t list_deg;         // extracted vertices of higher degree go to the hub list (at most HEAVY_DEG)
    uint32_t hcap;             // heavy list capacity (chunks); 0 = no heavy path
    // The hub list grouped by vertex (hgrouped = 1: a symmetric graph with
    // state groups of G >= 4 searches). The searches of one group that
    // extract hub h in a round set their bits in hmask[round parity][index of
    // h][group]; the first of them lists h's chunks once for the group in
    // hrec[round parity], and the hub-list kernel relaxes each listed chunk
    // for all of the group's searches with bits set, reading the arcs once
    // and their heads' words for the group from the same lines.
    const uint32_t *hub_id;    // [n] index of each vertex among the hubs (degree > HEAVY_DEG), else INF32
    const uint32_t *hub_vert;  // [nhub] vertex of each hub
    unsigned long long *hmask; // [2][nhub][ngroups] bits of the searches of a group that extracted the hub
    uint4 *hrec;               // [2][hcap] (hub index, group, first arc, end arc)
    unsigned long long *hgcount;  // [2] records listed per round parity
    uint32_t nhub, ngroups, hgrouped;
    uint32_t *err;             // ERR_* bits
    unsigned long long *stats; // [ST_ROUNDS] rounds run
    unsigned long long *wstats; // [grid][ST_N] per-workgroup counters of the round kernel
    uint32_t theta_mode;       // 0: theta += Delta; 1: end of the smallest key's Delta bucket; 2: smallest key + Delta
    // Learned or traced step schedule (sc = null: off). Delta of search i in
    // a round is its base Delta times 2^(bin[i] - 4).
    unsigned long long *sc;    // [2][nsearch][2] per-search counters of a round, by round parity:
                               //   (arcs of extracted vertices << 32) + extracted vertices; entries for the next frontier
    uint32_t ml_mode;          // 1: bins fixed per search (tracing), 2: the network picks them,
                               // 3: a rule steers each search's next frontier towards rho entries
    // Tracing (ml_mode 1) with a switch: search i runs bin[i] until its step
    // for round sw_round[i], and bin_after[i] from then on (null: no switch).
    const uint8_t *bin_after;
    const uint32_t *sw_round;
    uint32_t rho;
    const uint16_t *mlp;       // network parameters in bf16 (layout in mlp_dev.h)
    uint8_t *bin;              // [nsearch] multiplier bin of the search's next round
    uint32_t *done_round;      // [nsearch] rounds the search ran
    unsigned long long *tot_arcs;  // [nsearch] arcs it scanned
    unsigned long long *tot_ent;   // [nsearch] entries it put in its next frontiers (carried ones included)
    float *trace;              // [trace_cap][12] feature rows, or null
    uint32_t *trace_s;         // [trace_cap] search of each row
    uint32_t *trace_r;         // [trace_cap] the round after which the row's step was chosen
    uint8_t *trace_b;          // [trace_cap] the bin chosen (the network's, or the fixed one)
    unsigned long long *trace_n;
    uint64_t trace_cap;
    float deg_feat;            // log2(m / n) / 4
    uint32_t grid;             // workgroups of the round kernel
    uint32_t ml_every;         // the network runs every ml_every rounds (bins are kept in between)
    // Degree-aware extraction: a vertex of degree > HEAVY_DEG is extracted
    // only while its key <= hlim[i] = smallest key + max(1, Delta / hwin) - 1,
    // i.e. from the low end of the window, where its distance is close to
    // final, so its long arc list is pushed fewer times. The smallest key
    // always qualifies, so every round makes progress.
    uint64_t *hlim;            // [nsearch]
    uint32_t hwin;             // window divisor for heavy vertices (1 = the whole window)
    // Memoised heuristic (Section 5): per query slot, per vertex, the word
    // (epoch << 32 | forward term h_t - h_s, or h_t for one-sided A*); a word
    // from another epoch is a miss. Null: computed on every use.
    uint64_t *memo;
    uint32_t epoch;
    uint32_t pull;             // 1: pull relaxation before pushing (Appendix B)
    // Local chunks of the round kernel: up to max(local, local_plain) chunks
    // per wave per round taken from the wave's own additions: entries of
    // heuristic searches (A*, BiD-A*) when local > 0, of the others when
    // local_plain > 0; in rounds whose frontier holds fewer than local_fill
    // entries (0: every round).
    uint32_t local;
    uint32_t local_plain;
    uint32_t local_fill;
    uint32_t local_small;      // the budget in rounds whose chunks are below WAVE entries
    uint32_t min_chunk;        // smallest chunk of a small queue (a power of two <= WAVE; WAVE or 0: fixed)
    // In rounds of full chunks, local chunks stop in a wave once it has run
    // local_pct % of the previous round's mean wave time (null tsum: no
    // limit), its listed entries going to the next round; past defer_pct %
    // (0: never) its remaining queue chunks go there too. tsum[2][2]: sampled
    // wave-time sums and counts by round parity; lcap[2]: the mean wave time
    // (wall-clock ticks) of the round before the round of each parity.
    unsigned long long *tsum;
    uint32_t *lcap;
    uint32_t local_pct;
    uint32_t defer_pct;
    // Dense frontiers (the dense mode of Appendix B; dbits null: off). Once a
    // search's next frontier reaches dense_min entries (sampled counts; or
    // from its first step with dense_force), its frontier is kept as bitmaps
    // of n bits, one per step bucket of width dW (key / dW): the current
    // bucket dbase is read from bitmap dread, its refills go to the other of
    // {dbase mod dring, dring}, and bucket b < dbase + dring lives in bitmap
    // b mod dring (dring a power of two). Entries beyond the ring stay in the queue. A search stays
    // dense until it finishes; its threshold is the end of its current bucket.
    uint32_t *dbits;           // [nsearch][dring + 1][dwords]
    uint32_t dring;            // step buckets of the ring ahead of the current one
    uint64_t dwords;           // 32-bit words per bitmap
    uint8_t *dmode;            // [nsearch] 1: dense
    uint64_t *dbase;           // [nsearch] current bucket (absolute index)
    uint64_t *dW;              // [nsearch] bucket width (key units)
    uint8_t *dread;            // [nsearch] the bitmap read this round
    uint32_t *docc;            // [nsearch][dring + 1] 1: the bitmap may have bits set
    uint32_t *dlist;           // [2][nsearch] by round parity: dense searches whose read bitmap the round scans
    uint32_t *dcount;          // [0], [1] entries of dlist by parity; [2] dense searches still running (host poll)
    uint64_t dense_min;
    uint32_t dense_force;
};

// Only the first ML_SAMPLE workgroups of the round kernels update the
// per-search counters; the control kernel scales their counts by the share
// of chunks those workgroups processed (all of them when a round has at most
// ML_SAMPLE chunks). Counter atomics on one search's address stay few.
constexpr uint32_t ML_SAMPLE = 64;

// G is a power of two: searches i and i^1.. of one group of G keep their
// words of vertex v side by side (G = 1: search-major).
__host__ __device__ inline uint64_t state_index(uint32_t G, uint32_t n, uint32_t i, uint32_t v) {
    const uint32_t s = (uint32_t)__builtin_ctz(G);
    return ((((uint64_t)(i >> s) * n) + v) << s) | (i & (G - 1u));
}

// ST_HEAVYE / ST_HCHUNK: arcs and chunk records the round kernel handed to the
// heavy list (relaxed by k_heavy; ST_SCANE counts every scanned arc);
// ST_HSUCC: successful relaxations in k_heavy (ST_SUCC: in k_round);
// ST_DENSE: searches switched to dense frontiers (counted by the control step).
enum StatIdx { ST_ROUNDS = 0, ST_ENTRIES = 1, ST_SCANV = 2, ST_SCANE = 3, ST_SUCC = 4, ST_CARRY = 5, ST_HEAVYE = 6,
               ST_HCHUNK = 7, ST_HSUCC = 8, ST_DENSE = 9, ST_N = 16 };

}  // namespace ppsp
