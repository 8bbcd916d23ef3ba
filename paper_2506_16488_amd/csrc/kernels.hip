// gfx950 kernels of the point-to-point shortest-path engine.
//
// One stepping round (the loop body of Algorithm 2) is one launch of
// k_round followed by one launch of k_control:
//
//   k_round     for every frontier entry u^(i):
//                 - read delta[u^(i)] (and, for an interleaved bidirectional
//                   pair, delta of the other copy in the same 16-byte load);
//                   the key is scale * delta + the entry's stored heuristic
//                   term, so no coordinates are read here;
//                 - Extract(theta): key above theta -> keep for a later round;
//                 - otherwise run UpdateDistance for u (the deferred meeting
//                   check, see below) and Prune(u^(i)): key >= bound;
//                 - relax every arc (u, v, w) with a 64-bit atomicMin on the
//                   packed (distance, stamp) word; on a strict decrease run
//                   UpdateDistance for v^(i) at once, then Prune(v^(i)) and
//                   Add(v^(i)) to the next frontier.
//   k_control   per search: the next threshold (Delta*-stepping of Section 2:
//               theta grows by Delta per round, raised to the smallest key of
//               the next frontier when a step would be empty; or, in the
//               bucketed variant, the end of the Delta bucket holding that
//               key); the mumax bound over the search's queries (Table 2);
//               termination when the frontier is empty; the disconnected-
//               query rule of Appendix B.
//
// Meeting checks. UpdateDistance(v) needs delta of the other copies of v.
// A value written by another wave in the same launch may not be visible
// (per-XCD L2s are only coherent at kernel boundaries), so the check runs
// twice: immediately after a successful relaxation (sees every earlier
// round) and again when the entry is extracted in a later round (sees the
// whole previous round). For the meeting vertex of the correctness proofs
// (Theorems bids-correctness and bdastar-correctness) one of its two copies
// is unpruned when it becomes exact, so that copy is added to the frontier
// and the later check covers the case where both copies became exact in the
// same round. A copy that its own wave extracts in the launch that added it
// (local chunks, below) leaves a check-only entry, so the later check still
// runs in a later launch.
//
// Work distribution. The queue is walked in chunks of 64 entries (16 or 32
// while the whole queue is too small to give every workgroup a full chunk)
// with a static stride over the workgroups. A wave also keeps its own
// additions whose key is within the round's threshold in an LDS list and
// extracts them as local chunks in the same launch, up to a budget, so a
// frontier advances several hops per round. In rounds of full chunks, a wave
// that has run a set share of the previous round's mean wave time hands its
// listed entries, and later its remaining queue chunks, to the next round,
// so that no single wave holds the round open.
//
// Frontier building. The round kernel runs one wave per workgroup and the
// waves never wait for each other. A wave appends with a ballot + mbcnt
// prefix into its own LDS buffer and flushes it to its queue segment with
// one global atomic and coalesced 16-byte stores. Atomics on shared counters
// are kept rare, because atomics on one address serialise at the memory
// side: appends spread over NSEG segment counters, the per-search liveness
// flag is a plain store, the per-search minimum key is only atomically
// lowered when a plain read shows it would change, and the round kernel's
// counters go to per-workgroup slots. Duplicate Adds are avoided with the
// round stamp in the low half of each state word (see ppsp_dev.h). Per-search
// counts and minimum keys are reduced across the wave before their atomics.
// The arcs of the vertices extracted from a chunk are relaxed arc-parallel:
// a wave scan of their degrees turns them into one list that all lanes walk,
// so there is no per-vertex loop and no idle lane behind a vertex that was
// only kept for a later round.
//
// The round number lives in device memory (written by the kernel that does
// not read it in the same launch), so a fixed sequence of launches can be
// captured once in a hipGraph and replayed.
#include <hip/hip_ext.h>

#include "mlp_dev.h"
#include "ppsp_dev.h"

namespace ppsp {

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t mbcnt64(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t x) {
    for (int o = 32; o > 0; o >>= 1) {
        uint64_t y = __shfl_xor(x, o);
        x = y < x ? y : x;
    }
    return x;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

__device__ __forceinline__ uint32_t key_scale(uint32_t kind) { return kind >= K_2DIST ? 2u : 1u; }

// key = scale * delta + hk (see ppsp_dev.h); never negative for a consistent heuristic.
__device__ __forceinline__ uint64_t key_of(uint32_t kind, uint64_t d, int32_t hk) {
    const int64_t k = (int64_t)((kind >= K_2DIST ? 2 : 1) * d) + hk;
    return k < 0 ? 0 : (uint64_t)k;
}

// Heuristic term of vertex v for a search: 0, h_t(v), h_t(v) - h_s(v) or h_s(v) - h_t(v).
__device__ __forceinline__ int32_t hterm(const RoundArgs &A, const SearchDesc &sd, uint32_t v) {
    if (sd.kind == K_DIST || sd.kind == K_2DIST) return 0;
    const int2 p = A.xy[v];
    const int64_t ht = (int64_t)heur(p.x, p.y, sd.tx, sd.ty, A.ws2, A.fb);
    if (sd.kind == K_ASTAR) return (int32_t)ht;
    const int64_t hs = (int64_t)heur(p.x, p.y, sd.sx, sd.sy, A.ws2, A.fb);
    return (int32_t)(sd.kind == K_BIDA_F ? ht - hs : hs - ht);
}

// hterm through the memo: the query's forward term is read when this wave's
// epoch wrote it, else computed from the coordinates and stored. The two
// searches of a query share the word (the backward term is its negation);
// a racing write stores the same value, and a write not yet visible is a miss.
__device__ __forceinline__ int32_t hterm_memo(const RoundArgs &A, const SearchDesc &sd, uint32_t i, uint32_t v) {
    if (sd.kind == K_DIST || sd.kind == K_2DIST) return 0;
    if (!A.memo) return hterm(A, sd, v);
    uint64_t *m = A.memo + (uint64_t)(A.pair2 ? (i >> 1) : i) * A.n + v;
    const uint64_t w = *m;
    int32_t h;
    if ((uint32_t)(w >> 32) == A.epoch) {
        h = (int32_t)(uint32_t)w;
    } else {
        const int2 p = A.xy[v];
        const int64_t ht = (int64_t)heur(p.x, p.y, sd.tx, sd.ty, A.ws2, A.fb);
        h = sd.kind == K_ASTAR ? (int32_t)ht : (int32_t)(ht - (int64_t)heur(p.x, p.y, sd.sx, sd.sy, A.ws2, A.fb));
        *m = ((uint64_t)A.epoch << 32) | (uint32_t)h;
    }
    return sd.kind == K_BIDA_B ? -h : h;
}

__device__ __forceinline__ void mu_update(const RoundArgs &A, uint32_t pair, uint64_t sum, uint32_t v) {
    if (sum >= INF32) { atomicOr(A.err, ERR_OVERFLOW); return; }
    unsigned long long *mp = (unsigned long long *)(A.mu + pair);
    if (sum < (*mp >> 32)) atomicMin(mp, (sum << 32) | v);
}

// UpdateDistance (Table 2) of copy v^(i) at distance d against every query
// of the search (one-sided searches meet their target, others the copies
// of their query-graph neighbours).
__device__ __forceinline__ void meet_list(const RoundArgs &A, const SearchDesc &sd, uint32_t d, uint32_t v) {
    for (uint32_t p = sd.pbeg; p < sd.pend; p++) {
        const Partner pt = A.partners[p];
        if (pt.other & TARGET_BIT) {
            if (v == (pt.other & ~TARGET_BIT)) mu_update(A, pt.pair, d, v);
        } else {
            const uint32_t dj = (uint32_t)(A.S[state_index(A.G, A.n, pt.other, v)] >> 32);
            if (dj != INF32) mu_update(A, pt.pair, (uint64_t)d + dj, v);
        }
    }
}

// Per-search frontier statistics of this wave: whether the search added
// anything (a plain store of 1) and the smallest key seen (an atomicMin only
// when a plain read shows it would lower the value). The lanes of a wave
// usually share one search, so the reduction is per wave.
__device__ __forceinline__ void search_stats(const RoundArgs &A, uint32_t np, uint32_t i, uint32_t cnt,
                                             uint64_t mink, bool count) {
    const bool has = cnt > 0 || mink != INF64;
    const uint64_t mask = __ballot(has);
    if (mask == 0) return;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    const uint32_t i0 = __shfl(i, leader);
    if (__all(!has || i == i0)) {
        const uint32_t tot = wave_sum_u32(has ? cnt : 0u);
        const uint64_t mn = wave_min_u64(has ? mink : INF64);
        if ((int)lane_id() == leader) {
            uint32_t *al = &A.alive[(uint64_t)np * A.nsearch + i0];
            if (tot && *al == 0) *al = 1;
            unsigned long long *mp = (unsigned long long *)&A.minkey[(uint64_t)np * A.nsearch + i0];
            if (mn < *mp) atomicMin(mp, mn);
            if (count && tot) atomicAdd(&A.sc[((uint64_t)(np ^ 1) * A.nsearch + i0) * 2 + 1], (unsigned long long)tot);
        }
    } else if (has) {
        uint32_t *al = &A.alive[(uint64_t)np * A.nsearch + i];
        if (cnt && *al == 0) *al = 1;
        unsigned long long *mp = (unsigned long long *)&A.minkey[(uint64_t)np * A.nsearch + i];
        if (mink < *mp) atomicMin(mp, mink);
        if (count && cnt) atomicAdd(&A.sc[((uint64_t)(np ^ 1) * A.nsearch + i) * 2 + 1], (unsigned long long)cnt);
    }
}

// ctr[2 * key + field] += val for every active lane: one atomic per distinct
// key for the first few keys of the wave, then one per lane.
__device__ __forceinline__ void wave_add_keyed(unsigned long long *ctr, uint32_t key, uint32_t field,
                                               unsigned long long val, bool active) {
    for (int it = 0; it < 4; it++) {
        const uint64_t m = __ballot(active);
        if (m == 0) return;
        const int leader = __ffsll((unsigned long long)m) - 1;
        const uint32_t k0 = __shfl(key, leader);
        const bool mine = active && key == k0;
        const unsigned long long s = wave_sum_u64(mine ? val : 0ull);
        if ((int)lane_id() == leader) atomicAdd(&ctr[(uint64_t)k0 * 2 + field], s);
        active = active && !mine;
    }
    if (active) atomicAdd(&ctr[(uint64_t)key * 2 + field], val);
}

// The part of a relaxation after its WriteMin returned `old`: on a strict
// decrease the meeting check (with the partner copy `other` read before the
// atomic), then Prune(v) and Add(v). Returns true if v^(i) must be added to
// the next frontier; *out is that entry. *lmin takes the key of every
// unpruned decrease (added now or by an earlier decrease of this round).
template <bool MEMO>
__device__ __forceinline__ bool relax_commit(const RoundArgs &A, const SearchDesc &sd, uint32_t i, uint32_t v,
                                             uint64_t cand, uint64_t other, uint64_t old, uint64_t bnd,
                                             uint32_t stamp, uint4 *out, uint64_t *lmin, unsigned long long *succ,
                                             uint64_t *kout, bool dense = false) {
    if (cand >= (old >> 32)) return false;
    (*succ)++;
    if (A.pair2) {
        const uint32_t dp = (uint32_t)(other >> 32);
        if (dp != INF32) mu_update(A, A.partners[sd.pbeg].pair, cand + dp, v);
    } else {
        meet_list(A, sd, (uint32_t)cand, v);
    }
    const int32_t hk = MEMO ? hterm_memo(A, sd, i, v) : hterm(A, sd, v);
    const uint64_t kv = key_of(sd.kind, cand, hk);
    if (kv >= bnd) return false;        // Prune(v) before Add(v)
    if (kv < *lmin) *lmin = kv;
    // Lowered before in this round: that lowering added v unless it was pruned
    // (a dense search adds every lowering: its bucket may have changed).
    if (!dense && (uint32_t)old == stamp && key_of(sd.kind, old >> 32, hk) < bnd) return false;
    *out = make_uint4(i, v, stamp, (uint32_t)hk);
    *kout = kv;
    return true;
}

// Relaxation of arc e out of u^(i) (Algorithm 2, inner loop) in the round
// whose stamp is `stamp`. Returns true if v^(i) must be added to the next
// frontier; *out is that entry. *lmin takes the key of every unpruned
// decrease (added now or by an earlier decrease of this round).
template <bool MEMO>
__device__ __forceinline__ bool relax_to(const RoundArgs &A, const SearchDesc &sd, uint32_t i, uint2 a, uint32_t du,
                                         uint64_t bnd, uint32_t stamp, uint4 *out, uint64_t *lmin,
                                         unsigned long long *succ, uint64_t *kout, bool dense) {
    const uint32_t v = a.x;
    const uint64_t cand = (uint64_t)du + a.y;
    if (cand >= INF32) { atomicOr(A.err, ERR_OVERFLOW); return false; }
    unsigned long long *p;
    uint64_t own, other = INF64;
    if (A.pair2) {
        const uint64_t base = state_index(A.G, A.n, i & ~1u, v);
        const ulonglong2 w = *(const ulonglong2 *)(A.S + base);   // possibly stale: never below the truth
        own = (i & 1) ? w.y : w.x;
        other = (i & 1) ? w.x : w.y;
        p = (unsigned long long *)(A.S + base + (i & 1));
    } else {
        p = (unsigned long long *)(A.S + state_index(A.G, A.n, i, v));
        own = *p;
    }
    if (cand >= (own >> 32)) return false;
    const uint64_t old = atomicMin(p, (cand << 32) | stamp);
    return relax_commit<MEMO>(A, sd, i, v, cand, other, old, bnd, stamp, out, lmin, succ, kout, dense);
}

// The same for arc e of the search's CSR (the transpose for a backward
// search on a directed graph).
template <bool MEMO, bool REV>
__device__ __forceinline__ bool relax_arc(const RoundArgs &A, const SearchDesc &sd, uint32_t i, uint32_t u,
                                          uint32_t du, uint64_t bnd, uint32_t e, uint32_t stamp, uint4 *out,
                                          uint64_t *lmin, unsigned long long *succ, uint64_t *kout, bool dense) {
    (void)u;
    const uint2 a = ((REV && sd.rev) ? A.in_arcs : A.arcs)[e];
    return relax_to<MEMO>(A, sd, i, a, du, bnd, stamp, out, lmin, succ, kout, dense);
}

// Dense frontiers (RoundArgs::dbits): sets v^(i)'s bit in the bitmap of the
// step bucket of key k. Returns false when that bucket lies beyond the ring;
// the caller then queues the entry.
__device__ __forceinline__ bool dense_add(const RoundArgs &A, uint32_t i, uint32_t v, uint64_t k) {
    const uint64_t W = A.dW[i], base = A.dbase[i];
    uint64_t b = k / W;
    if (b < base) b = base;
    uint32_t id;
    if (b == base) id = A.dread[i] == A.dring ? (uint32_t)(base & (A.dring - 1)) : A.dring;   // a refill of the current bucket
    else if (b - base < A.dring) id = (uint32_t)(b & (A.dring - 1));
    else return false;
    const uint64_t slot = (uint64_t)i * (A.dring + 1) + id;
    uint32_t *w = A.dbits + slot * A.dwords + (v >> 5);
    const uint32_t bit = 1u << (v & 31);
    if (!(*w & bit)) atomicOr(w, bit);
    if (A.docc[slot] == 0) A.docc[slot] = 1;
    return true;
}

// LDS staging of one wave's frontier adds. The wave appends with a ballot
// + mbcnt prefix (no atomics: the count is wave-uniform) and flushes to the
// global queue with one atomic and coalesced 16-byte stores.
struct WaveStage {
    uint4 buf[WSTAGE];
};

__device__ __forceinline__ void wstage_flush(WaveStage &st, uint32_t &cnt, uint4 *qout, uint32_t *qcout,
                                             uint64_t qseg, uint32_t *err) {
    if (cnt == 0) return;
    __syncthreads();                       // one wave per block: orders the LDS writes before the reads
    uint32_t base = 0;
    if (lane_id() == 0) base = atomicAdd(qcout, cnt);
    base = __shfl(base, 0);
    for (uint32_t j = lane_id(); j < cnt; j += WAVE) {
        if ((uint64_t)base + j < qseg) qout[(uint64_t)base + j] = st.buf[j]; else atomicOr(err, ERR_QUEUE);
    }
    __syncthreads();
    cnt = 0;
}

// Appends the entries of the lanes with pred set; flushes first if the
// buffer could overflow. Every lane of the wave calls it.
__device__ __forceinline__ void wstage_push(WaveStage &st, uint32_t &cnt, bool pred, uint4 entry, uint4 *qout,
                                            uint32_t *qcout, uint64_t qseg, uint32_t *err) {
    const uint64_t mask = __ballot(pred);
    if (mask == 0) return;
    if (cnt + WAVE > (uint32_t)WSTAGE) wstage_flush(st, cnt, qout, qcout, qseg, err);
    if (pred) st.buf[cnt + mbcnt64(mask)] = entry;
    cnt += __popcll(mask);
}

// Wave-wide exclusive prefix sum; *total receives the sum.
__device__ __forceinline__ uint32_t wave_exscan(uint32_t v, uint32_t *total) {
    const uint32_t lane = lane_id();
    uint32_t x = v;
    for (int o = 1; o < WAVE; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= (uint32_t)o) x += y;
    }
    *total = __shfl(x, WAVE - 1);
    return x - v;
}

#ifndef CARRY_CHECK
#define CARRY_CHECK 2   // rounds between state checks of a carried entry (a power of two; 1 = every round)
#endif

#ifndef RELAX_WAYS
#define RELAX_WAYS 1   // arcs per lane in flight in the round kernel's relaxation loop (1, 2 and 3 measured equal)
#endif

// Extracted vertices of one wave chunk, for the arc-parallel relaxation.
struct Advance {
    uint32_t off[WAVE + 1];   // exclusive prefix of the extracted degrees (0 for other lanes)
    uint32_t i[WAVE], u[WAVE], du[WAVE], rb[WAVE];
    uint64_t bnd[WAVE], th[WAVE];
    uint8_t dm[WAVE];         // the lane's search keeps a dense frontier
};

// Local chunks (RoundArgs::local): entries a wave adds whose key is within
// the round's threshold are kept in its LDS list and extracted by the same
// wave in the same round, so a frontier advances several hops per launch.
// A local entry carries the current round's stamp in .z; extracting it
// first clears the stamp of its state word to 0 with a compare-and-swap
// (the distance unchanged), so a later lowering in the round adds the
// vertex again. A wave only lists entries it has reserved local chunks for,
// so every listed entry is extracted before the launch ends.
constexpr uint32_t LCAP = 64;                  // LDS list slots per wave
// Check-only entry (.z): the meeting check of a vertex that was extracted
// locally in a search with partner copies, repeated in the next round.
// Within one launch another XCD's write of a partner copy may not be
// visible; the next launch sees it (the deferred check described above).
constexpr uint32_t RECHECK_Z = 0xFFFFFFFEu;

// One round. Workgroups are single waves that work independently (no
// barriers between waves): each takes WAVE-entry chunks of its sub-queue.
// Held to 96 registers, i.e. 5 waves per SIMD: the default grid of 20
// single-wave workgroups per CU is then resident at once (at 4 waves per
// SIMD a fifth of the workgroups would start only when others finish, and
// the static chunk stride would leave them a tail: 1.5x the launch time on
// the 2048^2 lattice).
template <bool PULL, bool MEMO, bool REV, bool DENSE>
__global__ __launch_bounds__(WAVE, 5) void k_round(RoundArgs A) {
    __shared__ WaveStage st;
    __shared__ Advance adv;
    uint32_t scnt = 0;
    const uint32_t r = A.round[0];
    const uint32_t par = r & 1, np = par ^ 1, stamp = r + 1;
    // Dense frontiers: after its queue chunks a wave takes tiles of 64 words
    // (2,048 vertices) of the read bitmaps of the searches in this round's
    // dense list, one word per lane, and extracts their set bits 64 at a time.
    const uint32_t ndense = DENSE ? A.dcount[par] : 0u;
    const uint64_t tiles_per = DENSE ? (A.dwords + WAVE - 1) / WAVE : 1ull;
    const uint64_t dtiles = (uint64_t)ndense * tiles_per;
    uint64_t dt = blockIdx.x, dwidx = 0;
    uint32_t dword = 0, dsi = 0;
    if (DENSE && blockIdx.x == 0 && lane_id() == 0) {
        A.dcount[np] = 0;                                  // the list the control step builds next
        A.dcount[2] = 0;                                   // dense searches still running, counted by it
    }
    const uint32_t sego = blockIdx.x % NSEG;                // segment this wave appends to
    const uint4 *qin = par ? A.q1 : A.q0;
    uint4 *qout = (par ? A.q0 : A.q1) + (uint64_t)sego * A.qseg;
    uint32_t *qcout = &A.qcount[np * NSEG + sego];
    // The chunk layout of the queue in registers: lane k holds the prefix of
    // segments 0..k and the length of segment k, so a chunk's segment is a
    // ballot and a popcount (the prefix is non-decreasing), with no memory
    // access on the chunk's critical path.
    static_assert(NSEG == WAVE, "one segment per lane");
    const uint32_t my_cpre = A.cpre[par * (NSEG + 1) + lane_id() + 1];
    const uint32_t my_qc = (uint32_t)min((uint64_t)A.qcount[par * NSEG + lane_id()], A.qseg);
    const uint32_t nchunks = __shfl(my_cpre, NSEG - 1);
    const uint32_t csize = A.cpre[par * (NSEG + 1)];         // entries per chunk this round
    if (blockIdx.x == 0 && lane_id() == 0) {
        A.round[1] = r;                                    // for k_control
        if (nchunks || ndense) atomicAdd(&A.stats[ST_ROUNDS], 1ull);
    }
    unsigned long long c_ent = 0, c_sv = 0, c_se = 0, c_succ = 0, c_keep = 0, c_he = 0, c_hc = 0;
    const bool count = A.sc && blockIdx.x < ML_SAMPLE;

    __shared__ uint4 lq[LCAP];
    uint32_t lpend = 0;                                    // listed local entries not yet taken
    // budget: local_small in rounds of small chunks (a small frontier: short
    // rounds matter), local / local_plain in rounds of full chunks
    const uint32_t lmain = A.local > A.local_plain ? A.local : A.local_plain;
    const uint32_t lmax = (csize < (uint32_t)WAVE && lmain) ? A.local_small : lmain;
    uint32_t lbud = (!PULL && lmax && (A.local_fill == 0 || (uint64_t)nchunks * csize < A.local_fill)) ? lmax : 0u;
    uint32_t ch = blockIdx.x;
    // Time limit for local chunks in rounds of full chunks: a percentage of
    // the previous round's mean wave time (set with the chunk prefix; 0:
    // none), so a wave with a long chain of local chunks does not hold a
    // loaded round open for all others. Small rounds (a small frontier: the
    // chain is the point) have none.
    const unsigned long long tmean = (A.lcap && csize == (uint32_t)WAVE) ? A.lcap[par] : 0ull;
    const unsigned long long lcap = tmean * A.local_pct / 100;
    // Past defer_pct % of that mean, a wave hands its remaining queue chunks to
    // the next round unprocessed (0: never). Its first chunk is always
    // processed, so every round makes progress whatever the setting.
    const unsigned long long dcap = tmean * A.defer_pct / 100;
    bool first_global = true;
    const unsigned long long t_begin = wall_clock64();
    for (;;) {
        // The next chunk: this wave's own listed entries first, then the queue.
        uint4 ent = make_uint4(0, 0, 0, 0);
        bool valid;
        if (lpend && lcap && wall_clock64() - t_begin > lcap) {
            // Out of time for local chunks: the listed entries go to the next
            // round's queue (live, with no key: that only widens the next
            // threshold), and this wave lists no more.
            for (uint32_t j = 0; j < lpend; j += WAVE) {
                const bool v = j + lane_id() < lpend;
                const uint4 e = v ? lq[j + lane_id()] : make_uint4(0, 0, 0, 0);
                wstage_push(st, scnt, v, e, qout, qcout, A.qseg, A.err);
                search_stats(A, np, e.x, v ? 1u : 0u, INF64, false);
            }
            __syncthreads();
            lpend = 0;
            lbud = 0;
        }
        if (lpend) {
            const uint32_t take = lpend < (uint32_t)WAVE ? lpend : (uint32_t)WAVE;
            valid = lane_id() < take;
            if (valid) ent = lq[lpend - take + lane_id()];
            lpend -= take;
            lbud--;
            __syncthreads();                                // read before this chunk lists more
        } else if (ch < nchunks) {
            const uint32_t lo = (uint32_t)__popcll(__ballot(my_cpre <= ch));   // cpre[lo] <= ch < cpre[lo + 1]
            const uint32_t c0 = lo ? __shfl(my_cpre, lo - 1) : 0u;
            const uint64_t nseg = __shfl(my_qc, lo);
            const uint64_t pos = (uint64_t)(ch - c0) * csize + lane_id();
            valid = lane_id() < csize && pos < nseg;
            if (valid) ent = qin[(uint64_t)lo * A.qseg + pos];
            ch += gridDim.x;
            const bool defer = !first_global && dcap && wall_clock64() - t_begin > dcap;
            first_global = false;
            if (defer) {
                // deferred as it is: live in the next round; a carried entry
                // keeps its key, any other counts with none
                const bool carried = (ent.x & CARRY_BIT) != 0;
                const uint64_t k = (valid && carried && ent.w != KEY_UNKNOWN) ? (uint64_t)ent.w : INF64;
                wstage_push(st, scnt, valid, ent, qout, qcout, A.qseg, A.err);
                search_stats(A, np, ent.x & ~CARRY_BIT, valid ? 1u : 0u, k, false);
                continue;
            }
        } else if (DENSE && (__any(dword != 0) || dt < dtiles)) {
            if (!__any(dword != 0)) {
                // the next tile; its words are cleared as they are read (no adds
                // go to a read bitmap: refills of the current bucket use the other one)
                dsi = A.dlist[(uint64_t)par * A.nsearch + dt / tiles_per];
                dwidx = (dt % tiles_per) * WAVE + lane_id();
                dt += gridDim.x;
                dword = 0;
                if (dwidx < A.dwords) {
                    uint32_t *wp = A.dbits + ((uint64_t)dsi * (A.dring + 1) + A.dread[dsi]) * A.dwords + dwidx;
                    dword = *wp;
                    if (dword) *wp = 0;
                }
                if (!__any(dword != 0)) continue;
            }
            valid = dword != 0;
            if (valid) {
                const uint32_t b = (uint32_t)__builtin_ctz(dword);
                dword &= dword - 1;
                ent = make_uint4(dsi | DENSE_BIT, (uint32_t)(dwidx * 32 + b), 0u, 0u);
            }
        } else {
            break;
        }

        // 1. One entry per lane: stale, kept for later, pruned or extracted.
        // A carried entry stores its exact key (CARRY_BIT set in .x, the key in
        // .w instead of the heuristic term): while that key lies between the
        // threshold and the bound it is carried again without reading the
        // state, except every CARRY_CHECK-th round (staggered by vertex),
        // which drops it if the vertex was lowered since (then a fresher
        // entry exists).
        uint32_t si = 0, du = 0, rb = 0, re = 0;
        uint64_t key = 0, bnd = 0, th = 0;
        int action = 0;  // 0 nothing, 1 keep for a later round, 2 relax
        bool recheck = false;   // push a check-only entry for the next round
        bool dent = false;
        if (valid) {
            const bool carried = (ent.x & CARRY_BIT) != 0;
            dent = DENSE && (ent.x & DENSE_BIT) != 0;     // from a dense bitmap: no stamp, no stored term
            si = ent.x & ~(CARRY_BIT | DENSE_BIT);
            const uint32_t i = si, u = ent.y;
            c_ent++;
            const ulonglong2 c = A.ctl[i];
            bnd = c.y;
            th = c.x;
            if (bnd != 0 && ent.z == RECHECK_Z) {
                // the deferred meeting check of a vertex extracted locally last round
                const SearchDesc sd = A.sd[i];
                if (A.pair2) {
                    const ulonglong2 w = *(const ulonglong2 *)(A.S + state_index(A.G, A.n, i & ~1u, u));
                    const uint32_t d0 = (uint32_t)(((i & 1) ? w.y : w.x) >> 32);
                    const uint32_t d1 = (uint32_t)(((i & 1) ? w.x : w.y) >> 32);
                    if (d0 != INF32 && d1 != INF32) mu_update(A, A.partners[sd.pbeg].pair, (uint64_t)d0 + d1, u);
                } else {
                    const uint32_t d0 = (uint32_t)(A.S[state_index(A.G, A.n, i, u)] >> 32);
                    if (d0 != INF32) meet_list(A, sd, d0, u);
                }
            } else if (bnd != 0 && carried && ent.w != KEY_UNKNOWN && ent.w > c.x && ent.w < bnd &&
                ((r + u) & (CARRY_CHECK - 1)) != 0) {
                key = ent.w;
                action = 1;
            } else if (bnd != 0) {
                const SearchDesc sd = A.sd[i];
                uint64_t word;
                uint32_t dp = INF32;
                unsigned long long *wp;
                if (A.pair2) {
                    const uint64_t base = state_index(A.G, A.n, i & ~1u, u);
                    const ulonglong2 w = *(const ulonglong2 *)(A.S + base);
                    word = (i & 1) ? w.y : w.x;
                    dp = (uint32_t)(((i & 1) ? w.x : w.y) >> 32);
                    wp = (unsigned long long *)(A.S + base + (i & 1));
                } else {
                    wp = (unsigned long long *)(A.S + state_index(A.G, A.n, i, u));
                    word = *wp;
                }
                bool local = false;
                if (ent.z == stamp && (uint32_t)word == stamp) {
                    // A local entry: take it by clearing the stamp (a lowering
                    // since it was listed keeps the stamp; retry with that).
                    for (;;) {
                        const uint64_t prev = atomicCAS(wp, (unsigned long long)word, word & ~0xFFFFFFFFull);
                        if (prev == word || (uint32_t)prev != stamp) {
                            local = prev == word;
                            word = prev == word ? (word & ~0xFFFFFFFFull) : prev;
                            break;
                        }
                        word = prev;
                    }
                    if (local) ent.z = 0;       // what the state word now holds
                }
                du = (uint32_t)(word >> 32);
                if (!dent && (uint32_t)word != ent.z && (uint32_t)word != INF32) {
                    // lowered after this entry was added: a fresher entry exists
                } else {
                    // the heuristic term: stored, or (unchanged distance) the stored key minus scale * delta
                    int32_t hk;
                    if (dent) hk = MEMO ? hterm_memo(A, sd, i, u) : hterm(A, sd, u);
                    else if (!carried) hk = (int32_t)ent.w;
                    else if (ent.w != KEY_UNKNOWN) hk = (int32_t)((int64_t)ent.w - (int64_t)key_scale(sd.kind) * du);
                    else hk = hterm(A, sd, u);
                    key = key_of(sd.kind, du, hk);
                    if (dent && key / A.dW[i] < A.dbase[i]) {
                        // a stale bit: the vertex was lowered into an earlier bucket,
                        // whose bitmap got its bit and has been read
                    } else if (key > c.x && key < bnd) {
                        action = 1;                     // above the threshold: later round
                    } else {
                        bool wait = false;
                        const uint32_t *rp = (REV && sd.rev) ? A.in_row_ptr : A.row_ptr;
                        if (A.hcap && key < bnd && key > A.hlim[i]) {
                            rb = rp[u];
                            re = rp[u + 1];
                            wait = re - rb > HEAVY_DEG;   // a hub above the low end of the window
                        }
                        if (wait) {
                            action = 1;
                        } else {
                            if (A.pair2) {
                                if (dp != INF32) mu_update(A, A.partners[sd.pbeg].pair, (uint64_t)du + dp, u);
                            } else {
                                meet_list(A, sd, du, u);
                            }
                            if (key < bnd) {
                                action = 2;
                                rb = rp[u];
                                re = rp[u + 1];
                                c_sv++;
                                c_se += re - rb;
                                recheck = local && (A.pair2 || sd.pend > sd.pbeg + 1 ||
                                                    (sd.pend > sd.pbeg && !(A.partners[sd.pbeg].other & TARGET_BIT)));
                            }
                        }
                    }
                    if (action == 1)
                        ent = make_uint4(i | CARRY_BIT, u, dent ? (uint32_t)word : ent.z,
                                         key < KEY_UNKNOWN ? (uint32_t)key : KEY_UNKNOWN);
                }
            }
        }
        if (count)
            wave_add_keyed(A.sc + (uint64_t)par * A.nsearch * 2, si, 0,
                           ((unsigned long long)(re - rb) << 32) + 1ull, action == 2);
        // Entries above the threshold stay in the frontier (a lowering of the
        // vertex in this round adds a fresher entry, which makes this one
        // stale); a dense search keeps them in the bitmap of their bucket.
        const bool keep = action == 1;
        const bool kq = keep && !(DENSE && A.dmode[si] && dense_add(A, si, ent.y, key));
        c_keep += keep;
        wstage_push(st, scnt, kq || recheck, kq ? ent : make_uint4(si, ent.y, RECHECK_Z, 0u), qout, qcout, A.qseg,
                    A.err);
        // a check-only entry keeps its search alive for one more round, at no key
        search_stats(A, np, si, (kq || recheck) ? 1u : 0u, keep ? key : INF64, count);

        // High-degree vertices go to the heavy list as chunks of at most
        // HEAVY_CHUNK arcs, which all waves of k_heavy share; one atomic per
        // wave reserves the wave's chunks.
        const bool heavy = action == 2 && A.hcap && re - rb > A.list_deg;
        if (__ballot(heavy)) {
            uint32_t nck = heavy ? (re - rb + HEAVY_CHUNK - 1) / HEAVY_CHUNK : 0u;
            if (heavy) {
                c_he += re - rb;
                c_hc += nck;
            }
            uint32_t hid = 0, grp = 0;
            if (A.hgrouped && heavy) {
                // grouped by vertex: only the group's first search to extract the hub lists its chunks
                hid = A.hub_id[ent.y];
                grp = si / A.G;
                const unsigned long long old =
                    atomicOr(A.hmask + ((uint64_t)par * A.nhub + hid) * A.ngroups + grp, 1ull << (si & (A.G - 1)));
                if (old != 0) nck = 0;
            }
            uint32_t tot;
            const uint32_t pre = wave_exscan(nck, &tot);
            unsigned long long b0 = 0;
            if (lane_id() == 0 && tot) b0 = atomicAdd(A.hgrouped ? A.hgcount + par : A.hcount, (unsigned long long)tot);
            b0 = __shfl(b0, 0);
            for (uint32_t k = 0; k < nck; k++) {
                const uint64_t slot = b0 + pre + k;
                const uint32_t eb = rb + k * HEAVY_CHUNK;
                const uint32_t ee = min(re, eb + HEAVY_CHUNK);
                if (slot >= A.hcap) {
                    atomicOr(A.err, ERR_HEAVY);
                } else if (A.hgrouped) {
                    A.hrec[(uint64_t)par * A.hcap + slot] = make_uint4(hid, grp, eb, ee);
                } else {
                    A.heavy[2 * slot] = make_uint4(si, ent.y, du, eb);
                    A.heavy[2 * slot + 1] = make_uint4(ee, 0u, 0u, 0u);
                }
            }
        }

        // 2. Arc-parallel relaxation of the extracted vertices: a wave scan of
        // their degrees lays their arcs out as one list, and each lane takes
        // one arc per step (its vertex found by binary search).
        const uint32_t deg = (action == 2 && !heavy) ? re - rb : 0u;
        uint32_t T;
        const uint32_t pre = wave_exscan(deg, &T);
        if (T == 0) continue;
        adv.off[lane_id()] = pre;
        if (lane_id() == WAVE - 1) adv.off[WAVE] = pre + deg;
        adv.i[lane_id()] = si;
        adv.u[lane_id()] = ent.y;
        adv.du[lane_id()] = du;
        adv.rb[lane_id()] = rb;
        adv.bnd[lane_id()] = bnd;
        adv.th[lane_id()] = th;
        adv.dm[lane_id()] = DENSE && deg && A.dmode[si];
        __syncthreads();
        if (PULL) {
            // Pull (Appendix B, undirected graphs): delta[u] <- min over the
            // arcs (v, u) of delta[v] + w before u pushes, as an LDS minimum
            // per extracted vertex; a lower value is written back (WriteMin)
            // and met against the partner copies, then pushed.
            for (uint32_t a0 = 0; a0 < T; a0 += WAVE) {
                const uint32_t a = a0 + lane_id();
                if (a < T) {
                    uint32_t lo = 0, hi = WAVE;
                    while (hi - lo > 1) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (adv.off[mid] <= a) lo = mid; else hi = mid;
                    }
                    const uint2 e = A.arcs[adv.rb[lo] + (a - adv.off[lo])];
                    const uint32_t dv = (uint32_t)(A.S[state_index(A.G, A.n, adv.i[lo], e.x)] >> 32);
                    if (dv != INF32 && (uint64_t)dv + e.y < adv.du[lo]) atomicMin(&adv.du[lo], dv + e.y);
                }
            }
            __syncthreads();
            const uint32_t k = lane_id();
            if (deg && adv.du[k] < du) {
                // Written with the entry's own stamp, not this round's: the
                // round stamp would tell a later lowering of u in this round
                // that u is already in the next frontier, and it is not (it is
                // being pushed now), so that lowering must add it.
                const uint32_t nd = adv.du[k];
                const uint64_t old = atomicMin((unsigned long long *)(A.S + state_index(A.G, A.n, si, ent.y)),
                                               ((uint64_t)nd << 32) | ent.z);
                if (nd < (uint32_t)(old >> 32)) {
                    const SearchDesc sd = A.sd[si];
                    if (A.pair2) {
                        const uint32_t dp = (uint32_t)(A.S[state_index(A.G, A.n, si ^ 1u, ent.y)] >> 32);
                        if (dp != INF32) mu_update(A, A.partners[sd.pbeg].pair, (uint64_t)nd + dp, ent.y);
                    } else {
                        meet_list(A, sd, nd, ent.y);
                    }
                } else {
                    adv.du[k] = (uint32_t)(old >> 32) < du ? (uint32_t)(old >> 32) : du;
                }
            }
            __syncthreads();
        }
        // RELAX_WAYS arcs per lane per step: their arc loads, then their state
        // loads, then their WriteMins are all in flight before any result is
        // used (the relaxation is a chain of dependent memory accesses).
        for (uint32_t a0 = 0; a0 < T; a0 += RELAX_WAYS * WAVE) {
            uint32_t lo[RELAX_WAYS], ai[RELAX_WAYS], v[RELAX_WAYS];
            bool want[RELAX_WAYS];
            uint2 arc[RELAX_WAYS];
            uint64_t cand[RELAX_WAYS], own[RELAX_WAYS], other[RELAX_WAYS], old[RELAX_WAYS];
            unsigned long long *wp[RELAX_WAYS];
#pragma unroll
            for (int h = 0; h < RELAX_WAYS; h++) {
                const uint32_t a = a0 + h * WAVE + lane_id();
                lo[h] = 0;
                ai[h] = 0;
                arc[h] = make_uint2(0, 0);
                want[h] = a < T;
                if (want[h]) {
                    uint32_t l = 0, r = WAVE;               // off[l] <= a < off[r]
                    while (r - l > 1) {
                        const uint32_t mid = (l + r) >> 1;
                        if (adv.off[mid] <= a) l = mid; else r = mid;
                    }
                    lo[h] = l;
                    ai[h] = adv.i[l];
                    const uint32_t e = adv.rb[l] + (a - adv.off[l]);
                    arc[h] = REV ? ((A.sd[ai[h]].rev ? A.in_arcs : A.arcs)[e]) : A.arcs[e];
                }
            }
#pragma unroll
            for (int h = 0; h < RELAX_WAYS; h++) {
                v[h] = arc[h].x;
                own[h] = 0;
                other[h] = INF64;
                wp[h] = nullptr;
                if (want[h]) {
                    if (A.pair2) {
                        const uint64_t base = state_index(A.G, A.n, ai[h] & ~1u, v[h]);
                        const ulonglong2 w = *(const ulonglong2 *)(A.S + base);   // possibly stale: never below the truth
                        own[h] = (ai[h] & 1) ? w.y : w.x;
                        other[h] = (ai[h] & 1) ? w.x : w.y;
                        wp[h] = (unsigned long long *)(A.S + base + (ai[h] & 1));
                    } else {
                        wp[h] = (unsigned long long *)(A.S + state_index(A.G, A.n, ai[h], v[h]));
                        own[h] = *wp[h];
                    }
                }
            }
#pragma unroll
            for (int h = 0; h < RELAX_WAYS; h++) {
                cand[h] = want[h] ? (uint64_t)adv.du[lo[h]] + arc[h].y : 0;
                if (want[h] && cand[h] >= INF32) { atomicOr(A.err, ERR_OVERFLOW); want[h] = false; }
                want[h] = want[h] && cand[h] < (own[h] >> 32);
                old[h] = want[h] ? atomicMin(wp[h], (cand[h] << 32) | stamp) : 0ull;
            }
#pragma unroll
            for (int h = 0; h < RELAX_WAYS; h++) {
                bool app = false;
                uint4 ne = make_uint4(0, 0, 0, 0);
                uint64_t lmin = INF64, kv = INF64;
                bool heur = false;
                const bool dm = DENSE && want[h] && adv.dm[lo[h]];
                if (want[h]) {
                    const SearchDesc sd = A.sd[ai[h]];
                    heur = sd.kind == K_ASTAR || sd.kind == K_BIDA_F || sd.kind == K_BIDA_B;
                    app = relax_commit<MEMO>(A, sd, ai[h], v[h], cand[h], other[h], old[h], adv.bnd[lo[h]], stamp,
                                             &ne, &lmin, &c_succ, &kv, dm);
                }
                // a dense search's addition goes to the bitmap of its bucket
                if (DENSE && app && dm && dense_add(A, ai[h], v[h], kv)) app = false;
                // Within the threshold: list it for this wave's next local
                // chunk if its chunks fit the budget, else the next round.
                bool loc = false;
                if (lbud) {
                    loc = app && !dm && kv <= adv.th[lo[h]] && (heur ? A.local : A.local_plain) != 0;
                    const uint64_t lm = __ballot(loc);
                    const uint32_t nl = (uint32_t)__popcll(lm);
                    if (nl && lpend + nl <= LCAP && (lpend + nl + WAVE - 1) / WAVE <= lbud) {
                        if (loc) lq[lpend + mbcnt64(lm)] = ne;
                        lpend += nl;
                    } else {
                        loc = false;
                    }
                }
                wstage_push(st, scnt, app && !loc, ne, qout, qcout, A.qseg, A.err);
                search_stats(A, np, ai[h], (app && !loc) ? 1u : 0u, loc ? INF64 : lmin, count);
            }
        }
        __syncthreads();                          // adv is rewritten by the next chunk
    }
    wstage_flush(st, scnt, qout, qcout, A.qseg, A.err);
    c_ent = wave_sum_u64(c_ent);
    c_sv = wave_sum_u64(c_sv);
    c_se = wave_sum_u64(c_se);
    c_succ = wave_sum_u64(c_succ);
    c_keep = wave_sum_u64(c_keep);
    c_he = wave_sum_u64(c_he);
    c_hc = wave_sum_u64(c_hc);
    if (lane_id() == 0 && c_ent) {
        // this workgroup's own slot: no atomics, summed by the host
        unsigned long long *ws = A.wstats + (uint64_t)blockIdx.x * ST_N;
        ws[ST_CARRY] += c_keep;
        ws[ST_HEAVYE] += c_he;
        ws[ST_HCHUNK] += c_hc;
        ws[ST_ENTRIES] += c_ent;
        ws[ST_SCANV] += c_sv;
        ws[ST_SCANE] += c_se;
        ws[ST_SUCC] += c_succ;
    }
    if (A.tsum && blockIdx.x < ML_SAMPLE && lane_id() == 0) {
        // sampled wave times of this round, for the next round's limit
        atomicAdd(&A.tsum[par * 2], (unsigned long long)(wall_clock64() - t_begin));
        atomicAdd(&A.tsum[par * 2 + 1], 1ull);
    }
}


// The heavy list, relaxed by every wave of the grid: each wave takes whole
// chunks (at most HEAVY_CHUNK arcs of one vertex), 64 arcs per step. Runs
// after k_round in the same round, on the same grid, so it too must keep 5
// waves per SIMD resident.
template <bool MEMO, bool REV>
__global__ __launch_bounds__(WAVE, 5) void k_heavy(RoundArgs A) {
    __shared__ WaveStage st;
    uint32_t scnt = 0;
    const uint32_t r = A.round[1];                          // set by this round's k_round
    const uint32_t np = (r & 1) ^ 1, stamp = r + 1;
    const uint64_t nh = min((uint64_t)*A.hcount, (uint64_t)A.hcap);
    if (nh == 0) return;
    const bool count = A.sc && blockIdx.x < ML_SAMPLE;   // scaled like the round kernel's counts
    const uint32_t sego = blockIdx.x % NSEG;
    uint4 *qout = ((r & 1) ? A.q0 : A.q1) + (uint64_t)sego * A.qseg;
    uint32_t *qcout = &A.qcount[np * NSEG + sego];
    unsigned long long c_succ = 0;
    // Records are claimed hclaim at a time from a counter (hcount[1], cleared
    // with the list by the control step), so a wave that drew short records
    // takes more; every wave leaves once the counter has passed the list.
    for (;;) {
        unsigned long long got = 0;
        if (lane_id() == 0) got = atomicAdd(A.hcount + 1, (unsigned long long)A.hclaim);
        // wave-uniform in a scalar register, so the records load through the scalar cache
        const uint32_t base = __builtin_amdgcn_readfirstlane((uint32_t)min(got, (unsigned long long)nh));
        if (base >= nh) break;
        const uint32_t end = (uint32_t)min((uint64_t)base + A.hclaim, nh);
        for (uint32_t slot = base; slot < end; slot++) {
            const uint4 h1 = A.heavy[2 * slot];
            const uint32_t ee = A.heavy[2 * slot + 1].x;
            const uint32_t ai = h1.x;
            const SearchDesc sd = A.sd[ai];
            const uint64_t bnd = A.ctl[ai].y;
            const bool dm = A.dbits && A.dmode[ai];
            for (uint32_t e0 = h1.w; e0 < ee; e0 += WAVE) {
                const uint32_t e = e0 + lane_id();
                bool app = false;
                uint4 ne = make_uint4(0, 0, 0, 0);
                uint64_t lmin = INF64, kv = INF64;
                if (e < ee) app = relax_arc<MEMO, REV>(A, sd, ai, h1.y, h1.z, bnd, e, stamp, &ne, &lmin, &c_succ, &kv, dm);
                if (app && dm && dense_add(A, ai, ne.y, kv)) app = false;
                wstage_push(st, scnt, app, ne, qout, qcout, A.qseg, A.err);
                search_stats(A, np, ai, app ? 1u : 0u, lmin, count);
            }
        }
    }
    wstage_flush(st, scnt, qout, qcout, A.qseg, A.err);
    c_succ = wave_sum_u64(c_succ);
    if (lane_id() == 0 && c_succ) A.wstats[(uint64_t)blockIdx.x * ST_N + ST_HSUCC] += c_succ;
}

// The hub list grouped by vertex (RoundArgs::hgrouped; symmetric graphs): a
// wave takes one listed chunk of hub u and relaxes its arcs, 64 at a time,
// for every search of the group whose bit is set, one search after the
// other, so each arc is read once and the group's words of its head are in
// the lines the first search brought in. The relaxation starts from each
// search's current distance of u (never above the one it extracted: an exact
// upper bound either way). First it clears the bits of the previous round's
// list, which that round's kernel has finished reading.
template <bool MEMO>
__global__ __launch_bounds__(WAVE) void k_heavy_grouped(RoundArgs A) {
    __shared__ WaveStage st;
    __shared__ uint32_t s_du[WAVE];
    __shared__ uint64_t s_bnd[WAVE];
    uint32_t scnt = 0;
    const uint32_t r = A.round[1];                          // set by this round's k_round
    const uint32_t par = r & 1, np = par ^ 1, stamp = r + 1;
    {
        const uint64_t nprev = min((uint64_t)A.hgcount[np], (uint64_t)A.hcap);
        for (uint64_t s = (uint64_t)blockIdx.x * WAVE + lane_id(); s < nprev; s += (uint64_t)gridDim.x * WAVE) {
            const uint4 rc = A.hrec[(uint64_t)np * A.hcap + s];
            A.hmask[((uint64_t)np * A.nhub + rc.x) * A.ngroups + rc.y] = 0;
        }
    }
    const uint64_t nh = min((uint64_t)A.hgcount[par], (uint64_t)A.hcap);
    if (nh == 0) return;
    const bool count = A.sc && blockIdx.x < ML_SAMPLE;
    const uint32_t sego = blockIdx.x % NSEG;
    uint4 *qout = (par ? A.q0 : A.q1) + (uint64_t)sego * A.qseg;
    uint32_t *qcout = &A.qcount[np * NSEG + sego];
    unsigned long long c_succ = 0;
    for (uint64_t slot = blockIdx.x; slot < nh; slot += gridDim.x) {
        const uint4 rc = A.hrec[(uint64_t)par * A.hcap + slot];
        const uint32_t u = A.hub_vert[rc.x], grp = rc.y;
        const unsigned long long M = A.hmask[((uint64_t)par * A.nhub + rc.x) * A.ngroups + grp];
        const uint32_t j = lane_id();
        __syncthreads();                                    // the previous chunk's reads of s_du / s_bnd are done
        if (j < A.G && ((M >> j) & 1ull)) {
            const uint32_t si = grp * A.G + j;
            s_du[j] = (uint32_t)(A.S[state_index(A.G, A.n, si, u)] >> 32);
            s_bnd[j] = A.ctl[si].y;
        }
        __syncthreads();
        for (uint32_t e0 = rc.z; e0 < rc.w; e0 += WAVE) {
            const uint32_t e = e0 + lane_id();
            const uint2 a = e < rc.w ? A.arcs[e] : make_uint2(0u, 0u);
            for (unsigned long long mm = M; mm; mm &= mm - 1) {
                const uint32_t jj = (uint32_t)__builtin_ctzll(mm);
                const uint32_t ai = grp * A.G + jj;
                const SearchDesc sd = A.sd[ai];
                const bool dm = A.dbits && A.dmode[ai];
                bool app = false;
                uint4 ne = make_uint4(0, 0, 0, 0);
                uint64_t lmin = INF64, kv = INF64;
                if (e < rc.w) app = relax_to<MEMO>(A, sd, ai, a, s_du[jj], s_bnd[jj], stamp, &ne, &lmin, &c_succ, &kv, dm);
                if (app && dm && dense_add(A, ai, ne.y, kv)) app = false;
                wstage_push(st, scnt, app, ne, qout, qcout, A.qseg, A.err);
                search_stats(A, np, ai, app ? 1u : 0u, lmin, count);
            }
        }
    }
    wstage_flush(st, scnt, qout, qcout, A.qseg, A.err);
    c_succ = wave_sum_u64(c_succ);
    if (lane_id() == 0 && c_succ) A.wstats[(uint64_t)blockIdx.x * ST_N + ST_HSUCC] += c_succ;
}

// Prefix sum of the chunk counts of the NSEG segments of queue `q` (one
// wave of 64 = NSEG lanes). A chunk is WAVE entries, or fewer while the
// whole queue is too small to give every workgroup of the round kernel a
// full chunk: then min_chunk, 2 min_chunk, ... entries (the fewest that
// still cover the queue in one chunk per workgroup), so a small frontier is
// spread over more waves, each with a shorter chain of dependent accesses.
// The chunk size is stored in cpre[q][0].
__device__ __forceinline__ void chunk_prefix(const RoundArgs &A, uint32_t q) {
    const uint32_t k = lane_id();
    const uint32_t n = (uint32_t)min((uint64_t)A.qcount[q * NSEG + k], A.qseg);
    const unsigned long long tot = wave_sum_u64(n);
    uint32_t ch = WAVE;
    if (A.min_chunk && A.min_chunk < (uint32_t)WAVE) {
        ch = A.min_chunk;
        while (ch < (uint32_t)WAVE && tot > (unsigned long long)ch * A.grid) ch <<= 1;
    }
    const uint32_t c = (n + ch - 1) / ch;
    uint32_t x = c;
    for (int o = 1; o < WAVE; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (k >= (uint32_t)o) x += y;
    }
    A.cpre[q * (NSEG + 1) + k + 1] = x;
    if (k == 0) A.cpre[q * (NSEG + 1)] = ch;
    if (k == 0 && A.tsum) {
        // the local-chunk time limit of the round that reads queue q, from
        // the sampled wave times of the round before; its own sums start at 0
        const unsigned long long sum = A.tsum[(q ^ 1) * 2], cnt = A.tsum[(q ^ 1) * 2 + 1];
        A.lcap[q] = (uint32_t)min(cnt ? sum / cnt : 0ull, 0xFFFFFFFFull);   // mean wave time, in ticks
        A.tsum[q * 2] = 0;
        A.tsum[q * 2 + 1] = 0;
    }
}

__global__ __launch_bounds__(WAVE) void k_seed_prefix(RoundArgs A) { chunk_prefix(A, 0); }

// Liveness, termination and the bound of search i after round r: the part
// of the step control that does not depend on the step rule. Returns 0 if
// the search had already finished, 1 if it finished now, 2 if it goes on;
// then *mk is the smallest key of its next frontier and *nb its new bound.
// Only the writer lane stores.
__device__ __forceinline__ int control_search(const RoundArgs &A, uint32_t i, uint32_t par, uint32_t np, bool writer,
                                              uint64_t *mk_out, uint64_t *nb_out) {
    uint32_t c = A.alive[(uint64_t)np * A.nsearch + i];
    if (A.dbits && A.dmode[i] && !c) {
        // a dense search lives on while a bitmap other than the one just read holds bits
        const uint32_t rd = A.dread[i];
        for (uint32_t j = 0; j <= A.dring; j++)
            if (j != rd && A.docc[(uint64_t)i * (A.dring + 1) + j]) c = 1;
    }
    const uint64_t mk = A.minkey[(uint64_t)np * A.nsearch + i];
    if (writer) {
        A.alive[(uint64_t)par * A.nsearch + i] = 0;
        A.minkey[(uint64_t)par * A.nsearch + i] = INF64;
    }
    if (A.done[i]) return 0;
    const SearchDesc sd = A.sd[i];
    const ulonglong2 c0 = A.ctl[i];
    // A frontier that ran dry while nothing could be pruned has covered the
    // whole component of its root (Appendix B, disconnected queries).
    uint32_t ex = A.exh[i];
    if (c == 0 && c0.y == INF64 && !ex) {
        ex = 1;
        if (writer) A.exh[i] = 1;
    }
    uint64_t mx = 0;
    bool open = sd.noprune != 0;     // a search without pruning runs until its frontier is empty
    for (uint32_t p = sd.pbeg; p < sd.pend; p++) {
        const Partner pt = A.partners[p];
        const uint32_t m32 = (uint32_t)(A.mu[pt.pair] >> 32);
        if (m32 == INF32) {
            const bool other_ex = (pt.other & TARGET_BIT) ? false : (A.exh[pt.other] != 0);
            if (ex || other_ex) continue;    // settled: unreachable
            mx = INF64;
        } else if (mx != INF64 && m32 > mx) {
            mx = m32;
        }
        open = true;
    }
    const uint64_t nb = sd.noprune ? INF64 : (open ? mx : 0);
    if (c == 0 || !open) {
        if (writer) {
            A.done[i] = 1;
            A.ctl[i] = make_ulonglong2(c0.x, 0);
        }
        return 1;
    }
    *mk_out = mk;
    *nb_out = nb;
    return 2;
}

// The next threshold from the current one, the smallest key of the next
// frontier and the step Delta d (key units).
__device__ __forceinline__ uint64_t step_threshold(uint32_t mode, uint64_t th0, uint64_t mk, uint64_t d) {
    uint64_t th;
    if (mode == 3) return INF64;     // Bellman-Ford: extract everything every round
    if (mode == 0 || mk == INF64) {
        // Delta*-stepping: the i-th threshold is i * Delta; steps that would
        // extract nothing are skipped by raising it to the smallest key.
        th = th0 + d;
        if (th < th0) th = INF64;
        if (mk != INF64 && mk > th) th = mk;
    } else if (mode == 1) {
        // Bucketed variant: extract the Delta-wide bucket that holds the
        // smallest key; the threshold stays while that bucket refills.
        const uint64_t b = mk / d;
        th = (b + 1 > INF64 / d) ? INF64 : (b + 1) * d - 1;
        if (th < th0) th = th0;
    } else {
        // Sliding window: everything within Delta of the smallest key.
        th = mk + d - 1;
        if (th < mk) th = INF64;
        if (th < th0) th = th0;
    }
    return th;
}

// Upper end of the extraction window of heavy vertices (see RoundArgs::hlim).
__device__ __forceinline__ uint64_t heavy_limit(uint64_t mk, uint64_t d, uint32_t hwin) {
    if (mk == INF64) return INF64;
    uint64_t w = d / (hwin ? hwin : 1u);
    if (w == 0) w = 1;
    const uint64_t h = mk + w - 1;
    return h < mk ? INF64 : h;
}

// Per-search step control after a round (see the file comment).
__global__ __launch_bounds__(BLOCK) void k_control(RoundArgs A) {
    const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
    const uint32_t r = A.round[1];
    const uint32_t par = r & 1, np = par ^ 1;
    if (blockIdx.x == 0 && threadIdx.x < WAVE) {
        chunk_prefix(A, np);                      // chunk layout of the queue the next round reads
        A.qcount[par * NSEG + threadIdx.x] = 0;   // the queue just consumed becomes the next output
    }
    if (i == 0) {
        A.round[0] = r + 1;
        A.hcount[0] = 0;
        A.hcount[1] = 0;
        if (A.hgrouped) A.hgcount[np] = 0;       // the list whose bits the hub-list kernel just cleared
    }
    if (i >= A.nsearch) return;
    uint64_t mk = 0, nb = 0;
    if (control_search(A, i, par, np, true, &mk, &nb) != 2) return;
    const uint64_t th = step_threshold(A.theta_mode, A.ctl[i].x, mk, A.delta[i]);
    A.ctl[i] = make_ulonglong2(th, nb);
    if (A.hcap) A.hlim[i] = heavy_limit(mk, A.delta[i], A.hwin);
}

__device__ __forceinline__ float lg2p(double x) { return log2f((float)(1.0 + x)); }

// Features of search i for the step after round r (all roughly in [-2, 2]):
//   0  log2(1 + vertices extracted in the round) / 16
//   1  log2(1 + arcs scanned in the round) / 16
//   2  log2(1 + entries of the next frontier) / 16
//   3  (log2(1 + next frontier) - log2(1 + the partner search's)) / 8; 0 without a partner search
//   4  log2(1 + (bound - smallest key) / Delta) / 16; 0 while the bound is infinite
//   5  1 while the bound is infinite, else 0
//   6  log2(1 + (smallest key - threshold) / Delta) / 8
//   7  log2(1 + (threshold - root key) / Delta) / 16   (progress)
//   8  log2(1 + heuristic distance of the query / Delta) / 16; 0 without coordinates
//   9  log2(1 + round) / 16
//  10  progress towards the bound: (threshold - root key) / (bound - root key),
//      clipped to [0, 1]; 0 while the bound is infinite
//  11  log2(m / n) / 4
// Delta is the search's base Delta in key units. No feature holds the bin the
// search ran with, so the choice is a function of the search's state alone.
__device__ __forceinline__ void ml_features(const RoundArgs &A, uint32_t i, const SearchDesc &sd, uint32_t r,
                                            uint32_t par, unsigned long long c0, unsigned long long nxt, double scale,
                                            uint64_t th0, uint64_t mk, uint64_t nb, uint64_t db, uint32_t bin,
                                            float *f) {
    const double d = (double)db;
    const double near = scale * (double)(c0 & 0xFFFFFFFFull), arcs = scale * (double)(c0 >> 32);
    f[0] = lg2p(near) / 16.f;
    f[1] = lg2p(arcs) / 16.f;
    f[2] = lg2p(scale * (double)nxt) / 16.f;
    uint32_t pj = INF32;
    if (A.pair2) {
        pj = i ^ 1u;
    } else if (sd.pend > sd.pbeg) {
        const uint32_t o = A.partners[sd.pbeg].other;
        if (!(o & TARGET_BIT)) pj = o;
    }
    f[3] = 0.f;
    if (pj != INF32 && pj < A.nsearch)
        f[3] = (lg2p(scale * (double)nxt) - lg2p(scale * (double)A.sc[((uint64_t)par * A.nsearch + pj) * 2 + 1])) / 8.f;
    f[4] = nb == INF64 ? 0.f : lg2p((double)(nb > mk ? nb - mk : 0) / d) / 16.f;
    f[5] = nb == INF64 ? 1.f : 0.f;
    f[6] = mk == INF64 ? 1.f : lg2p((double)(mk > th0 ? mk - th0 : 0) / d) / 8.f;
    const uint64_t key0 = key_of(sd.kind, 0, hterm(A, sd, sd.src));
    f[7] = lg2p((double)(th0 > key0 ? th0 - key0 : 0) / d) / 16.f;
    double est = 0.0;
    if (A.xy && sd.kind != K_DIST && sd.kind != K_2DIST) {
        const int2 p = A.xy[sd.src];
        const bool to_s = sd.kind == K_BIDA_B;
        const uint64_t h = heur(p.x, p.y, to_s ? sd.sx : sd.tx, to_s ? sd.sy : sd.ty, A.ws2, A.fb);
        est = (double)h * (sd.kind == K_ASTAR ? 1.0 : 2.0);
    }
    f[8] = lg2p(est / d) / 16.f;
    f[9] = lg2p((double)r) / 16.f;
    f[10] = 0.f;
    if (nb != INF64 && nb > key0) f[10] = (float)fmin(1.0, (double)(th0 > key0 ? th0 - key0 : 0) / (double)(nb - key0));
    f[11] = A.deg_feat;
    (void)bin;
}

// Step control of the learned or traced schedule: one wave per search (the
// waves of the grid stride over the searches). Termination and bounds as in
// k_control; the step Delta is the base Delta times 2^(bin - 4), the bin
// chosen by the network (ml_mode 2) or fixed per search (ml_mode 1). With a
// trace buffer every step decision appends its feature row.
__global__ __launch_bounds__(WAVE) void k_control_ml(RoundArgs A) {
    const uint32_t r = A.round[1];
    const uint32_t par = r & 1, np = par ^ 1;
    const uint32_t lane = lane_id();
    const bool w = lane == 0;
    if (blockIdx.x == 0) {
        chunk_prefix(A, np);
        A.qcount[par * NSEG + lane] = 0;
        if (w) {
            A.round[0] = r + 1;
            A.hcount[0] = 0;
            A.hcount[1] = 0;
            if (A.hgrouped) A.hgcount[np] = 0;   // the list whose bits the hub-list kernel just cleared
        }
    }
    // share of this round's chunks that the counting workgroups processed
    const uint32_t nch = A.cpre[par * (NSEG + 1) + NSEG];
    const uint32_t q = nch / A.grid, rem = nch % A.grid;
    const uint32_t sampled = A.grid <= ML_SAMPLE ? nch : q * ML_SAMPLE + min(rem, ML_SAMPLE);
    const double scale = sampled ? (double)nch / sampled : 1.0;
    const bool net = A.ml_mode == 2 && r % A.ml_every == 0;
    MlpLane L;
    if (net) mlp_load_lane(A.mlp, L);
    for (uint32_t i = blockIdx.x; i < A.nsearch; i += gridDim.x) {
        const unsigned long long *sc = A.sc + ((uint64_t)par * A.nsearch + i) * 2;
        const unsigned long long c0 = sc[0], nxt = sc[1];
        uint64_t mk = 0, nb = 0;
        const int st = control_search(A, i, par, np, w, &mk, &nb);
        if (w) {
            unsigned long long *sn = A.sc + ((uint64_t)np * A.nsearch + i) * 2;   // next round's counters
            sn[0] = 0;
            sn[1] = 0;
        }
        if (st == 0) continue;
        if (w) {
            A.tot_arcs[i] += (unsigned long long)(scale * (double)(c0 >> 32) + 0.5);
            A.tot_ent[i] += (unsigned long long)(scale * (double)nxt + 0.5);
        }
        if (st == 1) {
            if (w) A.done_round[i] = r + 1;
            continue;
        }
        const uint64_t th0 = A.ctl[i].x;
        const uint64_t db = A.delta[i];
        uint32_t bin = A.bin[i];
        float f[MLP_F];
        if (net || A.trace) {
            const SearchDesc sd = A.sd[i];
            ml_features(A, i, sd, r, par, c0, nxt, scale, th0, mk, nb, db, bin, f);
        }
        bool want_dense = false;
        if (net) {
            float z1, h1, z2, h2, lg[MLP_O];
            mlp_forward(L, f, z1, h1, z2, h2, lg);
            bin = mlp_argmax(lg);
            want_dense = lg[MLP_K] > 0.f;        // the mode output: make this search's frontier dense
        } else if (A.ml_mode == 3) {
            // rho-stepping style: steer the next frontier towards rho entries
            const double nx = scale * (double)nxt;
            if (nx > 2.0 * A.rho && bin > 0) bin--;
            else if (nx < 0.5 * A.rho && bin < (uint32_t)MLP_K - 1) bin++;
        } else if (A.ml_mode == 1 && A.sw_round && r + 1 >= A.sw_round[i]) {
            // a traced switch: this step and all later ones; bins 8..15 also make the frontier dense
            bin = A.bin_after[i] & (MLP_K - 1);
            want_dense = A.bin_after[i] >= MLP_K;
        }
        if (A.dbits && !A.dmode[i] && (A.dense_force || want_dense || scale * (double)nxt >= (double)A.dense_min)) {
            // sparse -> dense (for good): buckets of this step's width, the
            // current one holding the smallest key of the next frontier
            uint64_t W = (db << bin) >> 4;
            if (W == 0) W = 1;
            if (w) {
                // the frontier of the next round is still the queue's: its
                // entries above the current bucket move into the ring then
                const uint64_t base = mk == INF64 ? 0 : mk / W;
                A.dmode[i] = 1;
                A.dW[i] = W;
                A.dbase[i] = base;
                A.dread[i] = (uint8_t)(base & (A.dring - 1));
                for (uint32_t j = 0; j <= A.dring; j++) A.docc[(uint64_t)i * (A.dring + 1) + j] = 0;
                A.ctl[i] = make_ulonglong2(base >= INF64 / W - 1 ? INF64 : (base + 1) * W - 1, nb);
                if (A.hcap) A.hlim[i] = heavy_limit(mk == INF64 ? base * W : mk, W, A.hwin);
                A.bin[i] = (uint8_t)bin;
                atomicAdd(&A.dcount[2], 1u);
                atomicAdd(&A.stats[ST_DENSE], 1ull);
            }
            continue;
        }
        if (A.dbits && A.dmode[i]) {
            // Dense: stay on the current bucket while it refilled, else move to
            // the next bucket with bits (or, the ring empty, to the smallest
            // key's bucket: those entries sit in the queue); done once every
            // remaining key would be pruned.
            const uint64_t base = A.dbase[i], W = A.dW[i];
            const uint32_t rd = A.dread[i];
            const uint32_t refill = rd == A.dring ? (uint32_t)(base & (A.dring - 1)) : A.dring;
            uint32_t *oc = A.docc + (uint64_t)i * (A.dring + 1);
            uint64_t nbase = INF64;
            uint32_t nread = 0;
            if (oc[refill]) {
                nbase = base;
                nread = refill;
            } else {
                for (uint32_t j = 1; j < A.dring && nbase == INF64; j++)
                    if (oc[(base + j) & (A.dring - 1)]) {
                        nbase = base + j;
                        nread = (uint32_t)((base + j) & (A.dring - 1));
                    }
                if (nbase == INF64) {
                    nbase = mk == INF64 ? base + 1 : (mk / W > base ? mk / W : base + 1);
                    nread = (uint32_t)(nbase & (A.dring - 1));
                }
            }
            const bool prune_all = nb != INF64 && nbase >= (nb + W - 1) / W;   // nbase * W >= bound
            if (w) {
                oc[rd] = 0;                            // read (and cleared) by this round's scan
                if (prune_all) {
                    A.done[i] = 1;
                    A.ctl[i] = make_ulonglong2(th0, 0);
                    A.done_round[i] = r + 1;
                } else {
                    A.dbase[i] = nbase;
                    A.dread[i] = (uint8_t)nread;
                    const uint64_t th = nbase >= INF64 / W - 1 ? INF64 : (nbase + 1) * W - 1;
                    A.ctl[i] = make_ulonglong2(th, nb);
                    // hubs wait for the low end of the window above the smallest key
                    // added this round (a hub that waited was re-added, so the
                    // smallest waiting one always qualifies: the bucket drains)
                    if (A.hcap) A.hlim[i] = heavy_limit(mk == INF64 || mk < nbase * W ? nbase * W : mk, W, A.hwin);
                    atomicAdd(&A.dcount[2], 1u);
                    if (oc[nread]) A.dlist[(uint64_t)np * A.nsearch + atomicAdd(&A.dcount[np], 1u)] = i;
                }
            }
            continue;
        }
        if (w) {
            if (A.trace) {
                const unsigned long long row = atomicAdd(A.trace_n, 1ull);
                if (row < A.trace_cap) {
                    for (int k = 0; k < MLP_F; k++) A.trace[row * MLP_F + k] = f[k];
                    A.trace_s[row] = i;
                    if (A.trace_r) A.trace_r[row] = r;
                    if (A.trace_b) A.trace_b[row] = (uint8_t)bin;
                }
            }
            A.bin[i] = (uint8_t)bin;
            uint64_t d = (db << bin) >> 4;
            if (d == 0) d = 1;
            A.ctl[i] = make_ulonglong2(step_threshold(A.theta_mode, th0, mk, d), nb);
            if (A.hcap) A.hlim[i] = heavy_limit(mk, d, A.hwin);
        }
    }
}

// Init() of Table 2 for every search: delta[root] = 0, root in the frontier.
// The host has cleared the state, the queue counters and the round counter.
__global__ __launch_bounds__(BLOCK) void k_init(RoundArgs A) {
    const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= A.nsearch) return;
    const SearchDesc sd = A.sd[i];
    const uint32_t s = sd.src;
    A.S[state_index(A.G, A.n, i, s)] = 0;                   // distance 0, stamp 0
    const int32_t hk = hterm(A, sd, s);
    const uint32_t x = i % NSEG;
    const uint32_t pos = atomicAdd(&A.qcount[x], 1u);
    if (pos < A.qseg) A.q0[(uint64_t)x * A.qseg + pos] = make_uint4(i, s, 0u, (uint32_t)hk);
    else atomicOr(A.err, ERR_QUEUE);
    const uint64_t k = key_of(sd.kind, 0, hk);
    A.ctl[i] = make_ulonglong2(k, INF64);
    if (A.hcap) A.hlim[i] = k;
    A.alive[i] = 1;
    A.alive[(uint64_t)A.nsearch + i] = 0;
    A.minkey[i] = k;
    A.minkey[(uint64_t)A.nsearch + i] = INF64;
    A.done[i] = 0;
    A.exh[i] = 0;
    if (A.dbits) A.dmode[i] = 0;
}

// Serving: Init() for the searches listed in ids[0..k), inserted between
// rounds into a running round loop. Their state slabs were cleared by the
// host; their roots join the frontier the next round reads, and their
// per-search control words are set for that round's parity.
__global__ __launch_bounds__(BLOCK) void k_admit(RoundArgs A, const uint32_t *ids, uint32_t k) {
    const uint32_t j = blockIdx.x * BLOCK + threadIdx.x;
    if (j >= k) return;
    const uint32_t i = ids[j];
    const uint32_t r = A.round[0];
    const uint32_t par = r & 1, np = par ^ 1;
    const SearchDesc sd = A.sd[i];
    const uint32_t s = sd.src;
    A.S[state_index(A.G, A.n, i, s)] = 0;                   // distance 0, stamp 0
    const int32_t hk = hterm(A, sd, s);
    const uint32_t x = i % NSEG;
    const uint32_t pos = atomicAdd(&A.qcount[par * NSEG + x], 1u);
    uint4 *q = par ? A.q1 : A.q0;
    if (pos < A.qseg) q[(uint64_t)x * A.qseg + pos] = make_uint4(i, s, 0u, (uint32_t)hk);
    else atomicOr(A.err, ERR_QUEUE);
    A.ctl[i] = make_ulonglong2(key_of(sd.kind, 0, hk), INF64);
    if (A.hcap) A.hlim[i] = key_of(sd.kind, 0, hk);
    A.alive[(uint64_t)par * A.nsearch + i] = 0;
    A.alive[(uint64_t)np * A.nsearch + i] = 0;
    A.minkey[(uint64_t)par * A.nsearch + i] = INF64;
    A.minkey[(uint64_t)np * A.nsearch + i] = INF64;
    A.done[i] = 0;
    A.exh[i] = 0;
    for (uint32_t p = sd.pbeg; p < sd.pend; p++) A.mu[A.partners[p].pair] = INF64;
    if (A.sc) {
        // the learned schedule: fresh counters, the base multiplier until the network's next decision
        for (uint32_t q = 0; q < 2; q++) {
            A.sc[((uint64_t)q * A.nsearch + i) * 2] = 0;
            A.sc[((uint64_t)q * A.nsearch + i) * 2 + 1] = 0;
        }
        A.bin[i] = (uint8_t)(MLP_K / 2);
    }
}

// Serving: chunk layout of the queue the next round reads, after admissions.
__global__ __launch_bounds__(WAVE) void k_reprefix(RoundArgs A) { chunk_prefix(A, A.round[0] & 1); }

// Serving: every search idle (finished, nothing to prune against).
__global__ __launch_bounds__(BLOCK) void k_idle(RoundArgs A) {
    const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= A.nsearch) return;
    A.ctl[i] = make_ulonglong2(0, 0);
    A.done[i] = 1;
    A.exh[i] = 0;
    A.alive[i] = 0;
    A.alive[(uint64_t)A.nsearch + i] = 0;
    A.minkey[i] = INF64;
    A.minkey[(uint64_t)A.nsearch + i] = INF64;
}

__device__ __forceinline__ uint32_t dist_of(const RoundArgs &A, uint32_t i, uint32_t v) {
    return (uint32_t)(A.S[state_index(A.G, A.n, i, v)] >> 32);
}

// A predecessor of v on a shortest path from the root of search i: an
// in-neighbour p with delta[p] + w(p,v) = delta[v] (exists for every exact
// v != root; see ppsp_dev.h), or INF32. A search over the reversed graph
// takes its predecessors among the out-neighbours.
__device__ uint32_t tight_pred(const RoundArgs &A, uint32_t i, uint32_t v) {
    const uint32_t dv = dist_of(A, i, v);
    const bool rev = A.sd[i].rev != 0;
    const uint32_t *rp = rev ? A.row_ptr : A.in_row_ptr;
    const uint2 *arcs = rev ? A.arcs : A.in_arcs;
    for (uint32_t e = rp[v]; e < rp[v + 1]; e++) {
        const uint2 a = arcs[e];
        const uint32_t dp = dist_of(A, i, a.x);
        if (dp != INF32 && (uint64_t)dp + a.y == dv) return a.x;
    }
    return INF32;
}

// Length of the tight-arc walk from v back to the root of search i (vertices
// counted, both ends included), or 0 if it does not reach the root within n
// steps.
__device__ uint32_t walk_len(const RoundArgs &A, uint32_t i, uint32_t v) {
    const uint32_t root = A.sd[i].src;
    uint32_t len = 1;
    while (v != root) {
        v = tight_pred(A, i, v);
        if (v == INF32 || ++len > A.n) return 0;
    }
    return len;
}

// Path lengths of every query slot (0: no path).
__global__ void k_path_len(RoundArgs A, const PairDesc *pd, uint32_t *len) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= A.npair) return;
    const uint64_t mu = A.mu[p];
    if ((mu >> 32) == INF32) { len[p] = 0; return; }
    const uint32_t m = (uint32_t)mu;
    const PairDesc d = pd[p];
    const uint32_t la = walk_len(A, d.a, m);
    const uint32_t lb = (d.b & TARGET_BIT) ? 1u : walk_len(A, d.b, m);
    if (la == 0 || lb == 0) { atomicOr(A.err, ERR_PATH); len[p] = 0; return; }
    len[p] = la + lb - 1;
}

// Writes root(a) -> ... -> meet -> ... -> root(b) at out + off[p].
__global__ void k_path_write(RoundArgs A, const PairDesc *pd, const uint32_t *len, const uint64_t *off,
                             uint32_t *out) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= A.npair || len[p] == 0) return;
    const uint32_t m = (uint32_t)A.mu[p];
    const PairDesc d = pd[p];
    uint32_t *o = out + off[p];
    const uint32_t la = walk_len(A, d.a, m);
    uint32_t v = m;
    const uint32_t ra = A.sd[d.a].src;
    for (uint32_t k = la; k-- > 0;) {        // forward half, written back to front
        o[k] = v;
        if (v == ra) break;
        v = tight_pred(A, d.a, v);
    }
    if (d.b & TARGET_BIT) return;
    const uint32_t rb = A.sd[d.b].src;
    v = m;
    uint32_t k = la;
    while (v != rb) {
        v = tight_pred(A, d.b, v);
        o[k++] = v;
    }
}

// A query answered by a search without pruning: its distance and meeting
// vertex (the target) are read off the root's state after the rounds.
__global__ void k_gather(RoundArgs A, const PairDesc *pd) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= A.npair) return;
    const PairDesc d = pd[p];
    if (!(d.b & TARGET_BIT)) return;
    const uint32_t t = d.b & ~TARGET_BIT;
    const uint32_t dt = dist_of(A, d.a, t);
    A.mu[p] = dt == INF32 ? INF64 : (((uint64_t)dt << 32) | t);
}

// ---- host-side launchers (the engine lives in another translation unit) ----

hipError_t launch_init(const RoundArgs &A, hipStream_t st) {
    k_init<<<(A.nsearch + BLOCK - 1) / BLOCK, BLOCK, 0, st>>>(A);
    k_seed_prefix<<<1, WAVE, 0, st>>>(A);
    return hipGetLastError();
}

hipError_t launch_admit(const RoundArgs &A, const uint32_t *ids, uint32_t k, hipStream_t st) {
    if (k) k_admit<<<(k + BLOCK - 1) / BLOCK, BLOCK, 0, st>>>(A, ids, k);
    k_reprefix<<<1, WAVE, 0, st>>>(A);
    return hipGetLastError();
}

hipError_t launch_idle(const RoundArgs &A, hipStream_t st) {
    k_idle<<<(A.nsearch + BLOCK - 1) / BLOCK, BLOCK, 0, st>>>(A);
    return hipGetLastError();
}

// With events, the launch carries them in its own dispatch (start and end
// of the kernel itself): no marker packets are queued between the rounds.
template <bool PULL, bool MEMO, bool REV, bool DENSE = false>
static hipError_t launch_round_t(const RoundArgs &A, uint32_t grid, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    if (e0)
        hipExtLaunchKernelGGL(k_round<PULL, MEMO, REV, DENSE>, dim3(grid), dim3(WAVE), 0, st, e0, e1, 0, A);
    else
        k_round<PULL, MEMO, REV, DENSE><<<grid, WAVE, 0, st>>>(A);
    return hipGetLastError();
}

hipError_t launch_round(const RoundArgs &A, uint32_t grid, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    // The default path (symmetric graph, no pull pass, no heuristic memo, no
    // dense frontiers) is compiled without those branches, which would
    // otherwise cost it registers and occupancy. A directed graph has a
    // separate transpose. Dense frontiers exclude the pull pass.
    const bool rev = A.in_row_ptr != A.row_ptr;
    if (A.dbits) {
        if (rev) return A.memo ? launch_round_t<false, true, true, true>(A, grid, st, e0, e1)
                               : launch_round_t<false, false, true, true>(A, grid, st, e0, e1);
        return A.memo ? launch_round_t<false, true, false, true>(A, grid, st, e0, e1)
                      : launch_round_t<false, false, false, true>(A, grid, st, e0, e1);
    }
    if (rev) return A.memo ? launch_round_t<false, true, true>(A, grid, st, e0, e1)
                           : launch_round_t<false, false, true>(A, grid, st, e0, e1);
    if (A.pull) return A.memo ? launch_round_t<true, true, false>(A, grid, st, e0, e1)
                              : launch_round_t<true, false, false>(A, grid, st, e0, e1);
    return A.memo ? launch_round_t<false, true, false>(A, grid, st, e0, e1)
                  : launch_round_t<false, false, false>(A, grid, st, e0, e1);
}

template <bool MEMO, bool REV>
static hipError_t launch_heavy_t(const RoundArgs &A, uint32_t grid, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    if (e0)
        hipExtLaunchKernelGGL(k_heavy<MEMO, REV>, dim3(grid), dim3(WAVE), 0, st, e0, e1, 0, A);
    else
        k_heavy<MEMO, REV><<<grid, WAVE, 0, st>>>(A);
    return hipGetLastError();
}

template <bool MEMO>
static hipError_t launch_heavy_grouped_t(const RoundArgs &A, uint32_t grid, hipStream_t st, hipEvent_t e0,
                                         hipEvent_t e1) {
    if (e0)
        hipExtLaunchKernelGGL(k_heavy_grouped<MEMO>, dim3(grid), dim3(WAVE), 0, st, e0, e1, 0, A);
    else
        k_heavy_grouped<MEMO><<<grid, WAVE, 0, st>>>(A);
    return hipGetLastError();
}

hipError_t launch_heavy(const RoundArgs &A, uint32_t grid, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    if (A.hgrouped)
        return A.memo ? launch_heavy_grouped_t<true>(A, grid, st, e0, e1) : launch_heavy_grouped_t<false>(A, grid, st, e0, e1);
    const bool rev = A.in_row_ptr != A.row_ptr;
    if (rev) return A.memo ? launch_heavy_t<true, true>(A, grid, st, e0, e1) : launch_heavy_t<false, true>(A, grid, st, e0, e1);
    return A.memo ? launch_heavy_t<true, false>(A, grid, st, e0, e1) : launch_heavy_t<false, false>(A, grid, st, e0, e1);
}

hipError_t launch_control(const RoundArgs &A, hipStream_t st) {
    if (A.sc) {
        const uint32_t nb = A.nsearch < 4096 ? A.nsearch : 4096;
        k_control_ml<<<nb ? nb : 1, WAVE, 0, st>>>(A);
    } else {
        const uint32_t nb = (A.nsearch + BLOCK - 1) / BLOCK;
        k_control<<<nb, BLOCK, 0, st>>>(A);
    }
    return hipGetLastError();
}

hipError_t launch_gather(const RoundArgs &A, const PairDesc *pd, hipStream_t st) {
    if (A.npair) k_gather<<<(A.npair + 255) / 256, 256, 0, st>>>(A, pd);
    return hipGetLastError();
}

hipError_t launch_path_len(const RoundArgs &A, const PairDesc *pd, uint32_t *len, hipStream_t st) {
    k_path_len<<<(A.npair + 127) / 128, 128, 0, st>>>(A, pd, len);
    return hipGetLastError();
}

hipError_t launch_path_write(const RoundArgs &A, const PairDesc *pd, const uint32_t *len, const uint64_t *off,
                             uint32_t *out, hipStream_t st) {
    k_path_write<<<(A.npair + 127) / 128, 128, 0, st>>>(A, pd, len, off, out);
    return hipGetLastError();
}

}  // namespace ppsp
