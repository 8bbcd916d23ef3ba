// Device-side data layout and helpers of the gfx950 point-to-point
// shortest-path engine.
//
// Search state. Every search (one frontier copy v^(i) in the notation of
// Section 3.1: the forward or backward copy of a bidirectional query, or the
// copy rooted at query-graph vertex q_i in Multi-BiDS, Section 4.2) owns a
// slab of n 64-bit words laid out search-major, S[i*n + v]:
//     bits 63..32  tentative distance delta[v^(i)] (0xFFFFFFFF = +infinity)
//     bits 31..0   the vertex whose relaxation last lowered it (parent)
// so WriteMin of Section 2 (write if smaller, report success) is one 64-bit
// atomicMin; success is a strict decrease of the distance field.
//
// Frontier. A flat queue of 64-bit entries (search << 32 | vertex) per round
// parity; membership of (i, v) in the next frontier is one bit in a per-parity
// bitmap, so Add (Algorithm 1: add v unless already present) is one atomicOr.
//
// Keys. Extraction and pruning compare integer keys (Table 2), doubled where
// the paper halves mu so that everything stays exact:
//     K_DIST    key = delta                      (early termination, SSSP)
//     K_ASTAR   key = delta + h_t(v)             (A*)
//     K_2DIST   key = 2 delta                    (BiDS, Multi-BiDS: delta >= mu/2)
//     K_BIDA_F  key = 2 delta + h_t(v) - h_s(v)  (BiD-A* forward:  delta + h_F >= mu/2)
//     K_BIDA_B  key = 2 delta - h_t(v) + h_s(v)  (BiD-A* backward: delta + h_B >= mu/2)
// with h_F = (h_t - h_s)/2 = -h_B (Section 3.5). A search prunes a vertex when
// key >= bound, bound being mu of its query (or mumax[i] of Table 2's
// Multi-PPSP row).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ppsp {

constexpr uint32_t INF32 = 0xFFFFFFFFu;
constexpr uint64_t INF64 = ~0ull;
constexpr uint32_t TARGET_BIT = 0x80000000u;  // Partner.other: a target vertex, not a search
constexpr int BLOCK = 256;                     // threads per block (four wave64s)
constexpr int WAVE = 64;
constexpr int STAGE_CAP = 2048;                // LDS staging slots per block
constexpr uint32_t HEAVY_DEG = 32;             // above this a whole wave relaxes the arc list

constexpr uint32_t ERR_OVERFLOW = 1u;          // a distance reached 2^32-1
constexpr uint32_t ERR_QUEUE = 2u;             // the frontier queue overflowed
constexpr uint32_t ERR_PATH = 4u;              // a parent walk did not reach its root

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
    uint32_t pad;
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
    const int2 *xy;            // n fixed-point coordinates or null
    uint64_t ws2;              // w_scale^2
    uint32_t fb;               // coordinate fractional bits
    uint32_t n;
    // searches
    const SearchDesc *sd;
    const Partner *partners;
    uint32_t nsearch;
    uint32_t npair;
    uint64_t *S;               // [nsearch][n] packed (dist, parent)
    uint32_t *flags;           // [2][nsearch][fw] frontier membership bits
    uint64_t fw;               // 32-bit words per search per parity
    uint64_t *theta;           // [nsearch] current threshold (key units)
    const uint64_t *delta;     // [nsearch] threshold increment (key units)
    uint64_t *bound;           // [nsearch] prune bound (key units), INF64 = none
    uint32_t *done;            // [nsearch]
    uint32_t *exh;             // [nsearch] frontier ran dry while the bound was infinite
    uint32_t *cnt;             // [2][nsearch] entries added to the next frontier
    uint64_t *minkey;          // [2][nsearch] smallest key added to the next frontier
    uint64_t *mu;              // [npair] packed (distance, meeting vertex)
    uint64_t *q0, *q1;         // frontier queues by round parity
    uint32_t *qcount;          // [2] queue lengths
    uint64_t qcap;             // queue capacity (entries)
    uint32_t *err;             // ERR_* bits
    unsigned long long *stats; // counters, see StatIdx
};

enum StatIdx { ST_ROUNDS = 0, ST_ENTRIES = 1, ST_SCANV = 2, ST_SCANE = 3, ST_SUCC = 4, ST_N = 8 };

}  // namespace ppsp
