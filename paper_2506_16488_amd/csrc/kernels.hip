// gfx950 kernels of the point-to-point shortest-path engine.
//
// One stepping round (the loop body of Algorithm 2) is one launch of
// k_round followed by one launch of k_control:
//
//   k_round     for every frontier entry u^(i):
//                 - UpdateDistance for u^(i) against the other copies of u
//                   (the deferred meeting check, see below);
//                 - Prune(u^(i)): key >= bound  -> drop;
//                 - Extract(theta): key > theta -> keep for a later round;
//                 - otherwise relax every arc (u, v, w) with a 64-bit
//                   atomicMin on the packed (distance, parent) word; on a
//                   strict decrease run UpdateDistance for v^(i) at once,
//                   then Prune(v^(i)) and Add(v^(i)) to the next frontier.
//   k_control   per search: next threshold theta += Delta (Delta*-stepping,
//               Section 2), raised to the smallest key in the next frontier
//               when steps would be empty; mumax bound over the search's
//               queries (Table 2); termination when the frontier is empty;
//               the disconnected-query rule of Appendix B.
//
// Meeting checks. UpdateDistance(v) needs delta of the other copies of v.
// A value written by another wave in the same launch may not be visible
// (per-XCD L2s are only coherent at kernel boundaries), so the check runs
// twice: immediately after a successful relaxation (sees every earlier
// round) and again when the entry is processed in the next round (sees the
// whole previous round). For the meeting vertex of the correctness proofs
// (Theorems bids-correctness and bdastar-correctness) one of its two copies
// is unpruned when it becomes exact, so that copy is added to the frontier
// and the next-round check covers the case where both copies became exact
// in the same round.
//
// Frontier building. Appends are aggregated per wave (ballot + mbcnt prefix,
// one LDS atomic per wave), staged in LDS, and written to the global queue
// with one global atomic per block and coalesced stores. Per-search counts
// and minimum keys are reduced across the wave before their atomics.
// Vertices of degree > HEAVY_DEG are relaxed by a whole wave (coalesced arc
// reads), lower degrees by one lane each.
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

__device__ __forceinline__ uint32_t *flag_word(const RoundArgs &A, uint32_t par, uint32_t i, uint32_t v) {
    return A.flags + ((uint64_t)par * A.nsearch + i) * A.fw + (v >> 5);
}

// Key of vertex v at tentative distance d for a search (see ppsp_dev.h).
__device__ __forceinline__ uint64_t make_key(const RoundArgs &A, const SearchDesc &sd, uint64_t d, uint32_t v) {
    switch (sd.kind) {
        case K_DIST: return d;
        case K_2DIST: return 2 * d;
        case K_ASTAR: {
            int2 p = A.xy[v];
            return d + heur(p.x, p.y, sd.tx, sd.ty, A.ws2, A.fb);
        }
        default: {
            int2 p = A.xy[v];
            int64_t h2 = (int64_t)heur(p.x, p.y, sd.tx, sd.ty, A.ws2, A.fb) -
                         (int64_t)heur(p.x, p.y, sd.sx, sd.sy, A.ws2, A.fb);
            int64_t k = (int64_t)(2 * d) + (sd.kind == K_BIDA_F ? h2 : -h2);
            return k < 0 ? 0 : (uint64_t)k;   // never negative for a consistent heuristic
        }
    }
}

// UpdateDistance (Table 2) of copy v^(i) at distance d.
__device__ __forceinline__ void meet_check(const RoundArgs &A, const SearchDesc &sd, uint32_t d, uint32_t v) {
    for (uint32_t p = sd.pbeg; p < sd.pend; p++) {
        Partner pt = A.partners[p];
        uint64_t sum;
        if (pt.other & TARGET_BIT) {
            if (v != (pt.other & ~TARGET_BIT)) continue;
            sum = d;
        } else {
            uint32_t dj = (uint32_t)(A.S[(uint64_t)pt.other * A.n + v] >> 32);
            if (dj == INF32) continue;
            sum = (uint64_t)d + dj;
        }
        if (sum >= INF32) { atomicOr(A.err, ERR_OVERFLOW); continue; }
        unsigned long long *mp = (unsigned long long *)(A.mu + pt.pair);
        if (sum < (*mp >> 32)) atomicMin(mp, (sum << 32) | v);
    }
}

// LDS staging area of one block.
struct Stage {
    uint64_t buf[STAGE_CAP];
    uint32_t count;   // slots handed out
    uint32_t fail;    // first slot of a wave that did not fit (valid prefix length)
    uint32_t base;    // global position of this flush
};

// Wave-aggregated append of the lanes with pred set. Must be reached by
// every lane of the wave.
__device__ __forceinline__ void stage_push(Stage &st, bool pred, uint64_t entry, uint64_t *qout,
                                           uint32_t *qcout, uint64_t qcap, uint32_t *err) {
    uint64_t mask = __ballot(pred);
    if (mask == 0) return;
    uint32_t c = __popcll(mask);
    uint32_t off = mbcnt64(mask);
    int leader = __ffsll((unsigned long long)mask) - 1;
    uint32_t pos = 0;
    if ((int)lane_id() == leader) pos = atomicAdd(&st.count, c);
    pos = __shfl(pos, leader);
    if (pos + c <= (uint32_t)STAGE_CAP) {
        if (pred) st.buf[pos + off] = entry;
    } else {
        uint32_t g = 0;
        if ((int)lane_id() == leader) {
            atomicMin(&st.fail, pos);
            g = atomicAdd(qcout, c);
        }
        g = __shfl(g, leader);
        if (pred) {
            uint64_t at = (uint64_t)g + off;
            if (at < qcap) qout[at] = entry; else atomicOr(err, ERR_QUEUE);
        }
    }
}

// Block-wide flush of the staged entries. Every thread of the block calls it.
__device__ __forceinline__ void stage_flush(Stage &st, uint64_t *qout, uint32_t *qcout, uint64_t qcap,
                                            uint32_t *err) {
    __syncthreads();
    uint32_t c = min(st.count, st.fail);
    if (threadIdx.x == 0) st.base = c ? atomicAdd(qcout, c) : 0u;
    __syncthreads();
    uint64_t b = st.base;
    for (uint32_t j = threadIdx.x; j < c; j += BLOCK) {
        if (b + j < qcap) qout[b + j] = st.buf[j]; else atomicOr(err, ERR_QUEUE);
    }
    __syncthreads();
    if (threadIdx.x == 0) { st.count = 0; st.fail = STAGE_CAP; }
    __syncthreads();
}

// Per-search frontier statistics of the appends of this wave: one atomic
// per wave when the appending lanes share a search.
__device__ __forceinline__ void search_stats(const RoundArgs &A, uint32_t np, uint32_t i, uint32_t cnt,
                                             uint64_t mink) {
    bool has = cnt > 0;
    uint64_t mask = __ballot(has);
    if (mask == 0) return;
    int leader = __ffsll((unsigned long long)mask) - 1;
    uint32_t i0 = __shfl(i, leader);
    if (__all(!has || i == i0)) {
        uint32_t tot = wave_sum_u32(cnt);
        uint64_t mn = wave_min_u64(has ? mink : INF64);
        if ((int)lane_id() == leader) {
            atomicAdd(&A.cnt[(uint64_t)np * A.nsearch + i0], tot);
            atomicMin((unsigned long long *)&A.minkey[(uint64_t)np * A.nsearch + i0], mn);
        }
    } else if (has) {
        atomicAdd(&A.cnt[(uint64_t)np * A.nsearch + i], cnt);
        atomicMin((unsigned long long *)&A.minkey[(uint64_t)np * A.nsearch + i], mink);
    }
}

// Relaxation of arc e out of u^(i) (Algorithm 2, inner loop). Returns true
// if v^(i) must be added to the next frontier (*vout, key folded into *lmin).
__device__ __forceinline__ bool relax_arc(const RoundArgs &A, const SearchDesc &sd, uint32_t i, uint32_t u,
                                          uint32_t du, uint64_t bnd, uint32_t e, uint32_t np,
                                          uint32_t *vout, uint64_t *lmin, unsigned long long *succ) {
    uint2 a = A.arcs[e];
    uint32_t v = a.x;
    uint64_t cand = (uint64_t)du + a.y;
    if (cand >= INF32) { atomicOr(A.err, ERR_OVERFLOW); return false; }
    unsigned long long *sv = (unsigned long long *)(A.S + (uint64_t)i * A.n + v);
    uint64_t cur = *sv;                 // possibly stale, never below the true value
    if (cand >= (cur >> 32)) return false;
    uint64_t old = atomicMin(sv, (cand << 32) | u);
    if (cand >= (old >> 32)) return false;
    (*succ)++;
    meet_check(A, sd, (uint32_t)cand, v);
    uint64_t kv = make_key(A, sd, cand, v);
    if (kv >= bnd) return false;        // Prune(v) before Add(v)
    uint32_t bit = 1u << (v & 31);
    uint32_t ob = atomicOr(flag_word(A, np, i, v), bit);
    if (ob & bit) return false;         // already in the next frontier
    *vout = v;
    if (kv < *lmin) *lmin = kv;
    return true;
}

__global__ __launch_bounds__(BLOCK) void k_round(RoundArgs A, uint32_t par) {
    __shared__ Stage st;
    if (threadIdx.x == 0) { st.count = 0; st.fail = STAGE_CAP; }
    __syncthreads();
    // entries past the capacity were never stored (the overflow is reported)
    const uint32_t nent = (uint32_t)min((uint64_t)A.qcount[par], A.qcap);
    const uint64_t *qin = par ? A.q1 : A.q0;
    uint64_t *qout = par ? A.q0 : A.q1;
    uint32_t *qcout = &A.qcount[par ^ 1];
    const uint32_t np = par ^ 1;
    if (blockIdx.x == 0 && threadIdx.x == 0 && nent > 0) atomicAdd(&A.stats[ST_ROUNDS], 1ull);
    unsigned long long c_ent = 0, c_sv = 0, c_se = 0, c_succ = 0;

    for (uint64_t base = (uint64_t)blockIdx.x * BLOCK; base < nent; base += (uint64_t)gridDim.x * BLOCK) {
        const uint64_t idx = base + threadIdx.x;
        uint32_t i = 0, u = 0, du = 0, rb = 0, re = 0;
        uint64_t key = 0, bnd = 0;
        int action = 0;  // 0 nothing, 1 keep for a later round, 2 relax
        SearchDesc sd = {};
        if (idx < nent) {
            const uint64_t ent = qin[idx];
            i = (uint32_t)(ent >> 32);
            u = (uint32_t)ent;
            c_ent++;
            atomicAnd(flag_word(A, par, i, u), ~(1u << (u & 31)));
            if (!A.done[i]) {
                sd = A.sd[i];
                du = (uint32_t)(A.S[(uint64_t)i * A.n + u] >> 32);
                meet_check(A, sd, du, u);
                key = make_key(A, sd, du, u);
                bnd = A.bound[i];
                if (key < bnd) action = (key > A.theta[i]) ? 1 : 2;
                if (action == 2) {
                    rb = A.row_ptr[u];
                    re = A.row_ptr[u + 1];
                    c_sv++;
                    c_se += re - rb;
                }
            }
        }
        // Entries above the threshold stay in the frontier.
        bool keep = false;
        if (action == 1) {
            uint32_t bit = 1u << (u & 31);
            keep = !(atomicOr(flag_word(A, np, i, u), bit) & bit);
        }
        uint32_t lcnt = keep ? 1u : 0u;
        uint64_t lmin = keep ? key : INF64;
        stage_push(st, keep, ((uint64_t)i << 32) | u, qout, qcout, A.qcap, A.err);

        // Light vertices: one lane per vertex.
        const uint32_t deg = (action == 2) ? re - rb : 0u;
        const uint32_t ldeg = deg <= HEAVY_DEG ? deg : 0u;
        for (uint32_t k = 0; __any(k < ldeg); k++) {
            bool app = false;
            uint32_t v = 0;
            if (k < ldeg) app = relax_arc(A, sd, i, u, du, bnd, rb + k, np, &v, &lmin, &c_succ);
            lcnt += app;
            stage_push(st, app, ((uint64_t)i << 32) | v, qout, qcout, A.qcap, A.err);
        }
        search_stats(A, np, i, lcnt, lmin);

        // Heavy vertices: the whole wave walks one arc list at a time.
        uint64_t hmask = __ballot(deg > HEAVY_DEG);
        while (hmask) {
            const int L = __ffsll((unsigned long long)hmask) - 1;
            hmask &= hmask - 1;
            const uint32_t hi = __shfl(i, L), hu = __shfl(u, L), hdu = __shfl(du, L);
            const uint32_t hrb = __shfl(rb, L), hre = __shfl(re, L);
            const uint64_t hbnd = __shfl(bnd, L);
            const SearchDesc hsd = A.sd[hi];
            uint32_t hcnt = 0;
            uint64_t hmin = INF64;
            for (uint32_t e0 = hrb; e0 < hre; e0 += WAVE) {
                const uint32_t e = e0 + lane_id();
                bool app = false;
                uint32_t v = 0;
                if (e < hre) app = relax_arc(A, hsd, hi, hu, hdu, hbnd, e, np, &v, &hmin, &c_succ);
                hcnt += app;
                stage_push(st, app, ((uint64_t)hi << 32) | v, qout, qcout, A.qcap, A.err);
            }
            search_stats(A, np, hi, hcnt, hmin);
        }
        stage_flush(st, qout, qcout, A.qcap, A.err);
    }
    c_ent = wave_sum_u64(c_ent);
    c_sv = wave_sum_u64(c_sv);
    c_se = wave_sum_u64(c_se);
    c_succ = wave_sum_u64(c_succ);
    if (lane_id() == 0 && c_ent) {
        atomicAdd(&A.stats[ST_ENTRIES], c_ent);
        atomicAdd(&A.stats[ST_SCANV], c_sv);
        atomicAdd(&A.stats[ST_SCANE], c_se);
        atomicAdd(&A.stats[ST_SUCC], c_succ);
    }
}

// Per-search step control after a round (see the file comment).
__global__ __launch_bounds__(BLOCK) void k_control(RoundArgs A, uint32_t par) {
    const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
    if (i == 0) A.qcount[par] = 0;           // the queue just consumed becomes the next output
    if (i >= A.nsearch) return;
    const uint32_t np = par ^ 1;
    const uint32_t c = A.cnt[(uint64_t)np * A.nsearch + i];
    const uint64_t mk = A.minkey[(uint64_t)np * A.nsearch + i];
    A.cnt[(uint64_t)par * A.nsearch + i] = 0;
    A.minkey[(uint64_t)par * A.nsearch + i] = INF64;
    if (A.done[i]) return;
    const SearchDesc sd = A.sd[i];
    // A frontier that ran dry while nothing could be pruned has covered the
    // whole component of its root (Appendix B, disconnected queries).
    uint32_t ex = A.exh[i];
    if (c == 0 && A.bound[i] == INF64 && !ex) { ex = 1; A.exh[i] = 1; }
    uint64_t mx = 0;
    bool open = false;
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
    A.bound[i] = sd.noprune ? INF64 : (open ? mx : 0);
    if (c == 0 || !open) { A.done[i] = 1; return; }
    uint64_t th = A.theta[i] + A.delta[i];
    if (th < A.theta[i]) th = INF64;
    if (mk != INF64 && mk > th) th = mk;
    A.theta[i] = th;
}

// Init() of Table 2 for every search: delta[root] = 0, root in the frontier.
__global__ __launch_bounds__(BLOCK) void k_init(RoundArgs A) {
    const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= A.nsearch) return;
    const SearchDesc sd = A.sd[i];
    const uint32_t s = sd.src;
    A.S[(uint64_t)i * A.n + s] = (uint64_t)s;             // distance 0, parent = itself
    *flag_word(A, 0, i, s) = 1u << (s & 31);             // bitmaps were cleared; one word per search
    A.q0[i] = ((uint64_t)i << 32) | s;
    const uint64_t k = make_key(A, sd, 0, s);
    A.theta[i] = k;
    A.cnt[i] = 1;
    A.cnt[(uint64_t)A.nsearch + i] = 0;
    A.minkey[i] = k;
    A.minkey[(uint64_t)A.nsearch + i] = INF64;
    A.done[i] = 0;
    A.exh[i] = 0;
    A.bound[i] = INF64;
}

// Length of the parent walk from v back to the root of search i (vertices
// counted, both ends included), or 0 if the walk does not reach the root
// within n steps.
__device__ uint32_t walk_len(const RoundArgs &A, uint32_t i, uint32_t v) {
    const uint32_t root = A.sd[i].src;
    uint32_t len = 1;
    while (v != root) {
        v = (uint32_t)A.S[(uint64_t)i * A.n + v];
        if (++len > A.n) return 0;
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
    uint32_t la = walk_len(A, d.a, m);
    uint32_t lb = (d.b & TARGET_BIT) ? 1u : walk_len(A, d.b, m);
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
    // forward half, written back to front
    uint32_t v = m;
    const uint32_t ra = A.sd[d.a].src;
    for (uint32_t k = la; k-- > 0;) {
        o[k] = v;
        if (v == ra) break;
        v = (uint32_t)A.S[(uint64_t)d.a * A.n + v];
    }
    if (d.b & TARGET_BIT) return;
    const uint32_t rb = A.sd[d.b].src;
    v = m;
    uint32_t k = la;
    while (v != rb) {
        v = (uint32_t)A.S[(uint64_t)d.b * A.n + v];
        o[k++] = v;
    }
}

// ---- host-side launchers (the engine lives in another translation unit) ----

hipError_t launch_init(const RoundArgs &A, hipStream_t st) {
    k_init<<<(A.nsearch + BLOCK - 1) / BLOCK, BLOCK, 0, st>>>(A);
    return hipGetLastError();
}

hipError_t launch_round(const RoundArgs &A, uint32_t par, uint32_t grid, hipStream_t st) {
    k_round<<<grid, BLOCK, 0, st>>>(A, par);
    return hipGetLastError();
}

hipError_t launch_control(const RoundArgs &A, uint32_t par, hipStream_t st) {
    k_control<<<(A.nsearch + BLOCK - 1) / BLOCK, BLOCK, 0, st>>>(A, par);
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
