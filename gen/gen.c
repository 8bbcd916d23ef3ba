/*
 * Seeded synthetic input generators for point-to-point shortest-path workloads.
 *
 * This module produces graphs (CSR), vertex coordinates and s-t query pairs.
 * It contains none of the shortest-path method's arithmetic: no relaxation,
 * no pruning, no heuristic. It is shared by the CPU oracle tests and by the
 * GPU path, which are otherwise independent.
 *
 * Randomness: every random draw is a pure function of (seed, stream, index)
 * (counter-based splitmix64 mixing), so construction is order independent
 * and reproducible from any language.
 *
 * Workload families (the paper's real datasets are replaced by synthetic
 * stand-ins; see the experiment setup of Section 6 and Table 3):
 *   grid     R x C 4-neighbour grid, integer weights uniform in [wlo, whi]
 *   lattice  L x L jittered lattice with fixed-point coordinates (8 fractional
 *            bits per cell unit), 4-neighbour edges plus, with probability
 *            p_diag per cell, one of the cell's two diagonals; the weight is
 *            ceil(1000 * Euclidean length) computed exactly in integers
 *   rmat     R-MAT(a,b,c,d) scale S, edge factor EF, random relabelling,
 *            symmetrised, self-loops dropped, duplicates merged, the weight
 *            of an unordered pair is a hash of that pair (so both directions
 *            agree), uniform in [wlo, whi]
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

typedef uint64_t u64;
typedef uint32_t u32;
typedef int32_t i32;

/* ---- counter-based random numbers -------------------------------------- */

/* splitmix64 output function (Steele, Lea, Flood 2014). */
static inline u64 mix64(u64 z) {
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Key of stream `stream` under `seed`, and word number `idx` of a keyed stream. */
static inline u64 stream_key(u64 seed, u64 stream) { return mix64(seed ^ mix64(stream * 0xD1B54A32D192ED03ULL)); }
static inline u64 keyed_rand(u64 key, u64 idx) { return mix64(key + idx * 0x9E3779B97F4A7C15ULL); }

/* Random 64-bit word number `idx` of stream `stream` under `seed`. */
u64 gen_rand(u64 seed, u64 stream, u64 idx) { return keyed_rand(stream_key(seed, stream), idx); }

/* Uniform integer in [0, range) from a 64-bit word (multiply-shift). */
static inline u64 below(u64 r, u64 range) {
    return (u64)(((unsigned __int128)r * range) >> 64);
}

enum {
    ST_WEIGHT = 1, ST_JX = 2, ST_JY = 3, ST_DIAG = 4, ST_DIAGDIR = 5,
    ST_RMAT = 6, ST_PERM = 7, ST_SRC = 8, ST_DST = 9, ST_HUB = 10, ST_HUBPICK = 11
};

/* ---- exact integer square roots (weights only) ---------------------------- */

/* floor(sqrt(x)) for x < 2^64, exact. */
static u64 isqrt_floor_u64(u64 x) {
    if (x == 0) return 0;
    u64 r = (u64)sqrtl((long double)x);
    /* correct the estimate by +-1 steps with exact 128-bit products */
    while ((unsigned __int128)r * r > x) r--;
    while ((unsigned __int128)(r + 1) * (r + 1) <= x) r++;
    return r;
}

/* ceil(sqrt(x)), exact. */
static u64 isqrt_ceil_u64(u64 x) {
    u64 r = isqrt_floor_u64(x);
    return ((unsigned __int128)r * r == x) ? r : r + 1;
}

u64 gen_isqrt_floor(u64 x) { return isqrt_floor_u64(x); }
u64 gen_isqrt_ceil(u64 x) { return isqrt_ceil_u64(x); }

/* Lattice edge weight: ceil(1000 * len) with len = sqrt(dx^2+dy^2) / 2^fb,
 * i.e. the smallest integer w with (w * 2^fb)^2 >= 10^6 (dx^2 + dy^2). */
u32 gen_lattice_weight(i32 dx, i32 dy, u32 frac_bits) {
    u64 d2 = (u64)((int64_t)dx * dx) + (u64)((int64_t)dy * dy);
    u64 q = 1000000ULL * d2;
    u64 k = isqrt_ceil_u64(q);
    u64 unit = 1ULL << frac_bits;
    return (u32)((k + unit - 1) / unit);
}

/* ---- grid ------------------------------------------------------------- */

/* Number of arcs of an R x C 4-neighbour grid. */
u64 gen_grid_arcs(u32 R, u32 C) {
    return 2ULL * ((u64)R * (C - 1) + (u64)(R - 1) * C);
}

/* Fills row_ptr[n+1], col[m], w[m]; neighbours of each vertex sorted by id.
 * Vertex id = r*C + c. Undirected edge ids: horizontal (r,c)-(r,c+1) -> r*(C-1)+c,
 * vertical (r,c)-(r+1,c) -> R*(C-1) + r*C + c. */
void gen_grid(u32 R, u32 C, u32 wlo, u32 whi, u64 seed,
              u64 *row_ptr, u32 *col, u32 *w) {
    u64 n = (u64)R * C;
    u64 H = (u64)R * (C - 1);
    u64 span = (u64)whi - wlo + 1;
    /* degrees */
    row_ptr[0] = 0;
    for (u64 v = 0; v < n; v++) {
        u32 r = (u32)(v / C), c = (u32)(v % C);
        u32 d = (r > 0) + (c > 0) + (c + 1 < C) + (r + 1 < R);
        row_ptr[v + 1] = row_ptr[v] + d;
    }
    #pragma omp parallel for schedule(static)
    for (long long vv = 0; vv < (long long)n; vv++) {
        u64 v = (u64)vv;
        u32 r = (u32)(v / C), c = (u32)(v % C);
        u64 p = row_ptr[v];
        if (r > 0) { u64 e = H + (u64)(r - 1) * C + c; col[p] = (u32)(v - C); w[p++] = wlo + (u32)below(gen_rand(seed, ST_WEIGHT, e), span); }
        if (c > 0) { u64 e = (u64)r * (C - 1) + (c - 1); col[p] = (u32)(v - 1); w[p++] = wlo + (u32)below(gen_rand(seed, ST_WEIGHT, e), span); }
        if (c + 1 < C) { u64 e = (u64)r * (C - 1) + c; col[p] = (u32)(v + 1); w[p++] = wlo + (u32)below(gen_rand(seed, ST_WEIGHT, e), span); }
        if (r + 1 < R) { u64 e = H + (u64)r * C + c; col[p] = (u32)(v + C); w[p++] = wlo + (u32)below(gen_rand(seed, ST_WEIGHT, e), span); }
    }
}

/* ---- jittered lattice ---------------------------------------------------- */

/* Cell (a,b), 0 <= a,b < L-1, owns corners (a,b),(a+1,b),(a,b+1),(a+1,b+1).
 * Returns -1 (no diagonal), 0 ((a,b)-(a+1,b+1)) or 1 ((a+1,b)-(a,b+1)). */
static inline int cell_diag(u32 L, u32 a, u32 b, u64 seed, u64 p_thresh) {
    u64 cell = (u64)b * (L - 1) + a;
    if ((gen_rand(seed, ST_DIAG, cell) >> 11) >= p_thresh) return -1;
    return (int)(gen_rand(seed, ST_DIAGDIR, cell) & 1);
}

static inline u64 diag_threshold(double p_diag) {
    if (p_diag <= 0) return 0;
    if (p_diag >= 1) return 1ULL << 53;
    return (u64)(p_diag * 9007199254740992.0);  /* p * 2^53 */
}

/* Coordinates in fixed point: X = 2^fb * i + U, Y = 2^fb * j + U', U,U' uniform
 * in [0, 2^fb). Vertex id = j*L + i (row j, column i). */
void gen_lattice_coords(u32 L, u32 frac_bits, u64 seed, i32 *xy) {
    u64 n = (u64)L * L;
    u64 unit = 1ULL << frac_bits;
    #pragma omp parallel for schedule(static)
    for (long long vv = 0; vv < (long long)n; vv++) {
        u64 v = (u64)vv;
        u32 i = (u32)(v % L), j = (u32)(v / L);
        xy[2 * v] = (i32)(unit * i + below(gen_rand(seed, ST_JX, v), unit));
        xy[2 * v + 1] = (i32)(unit * j + below(gen_rand(seed, ST_JY, v), unit));
    }
}

/* Neighbours of lattice vertex (i,j), unsorted; returns count (<= 8). */
static int lattice_nbrs(u32 L, u32 i, u32 j, u64 seed, u64 pt, u32 *out) {
    int k = 0;
    if (j > 0) out[k++] = (j - 1) * L + i;
    if (i > 0) out[k++] = j * L + (i - 1);
    if (i + 1 < L) out[k++] = j * L + (i + 1);
    if (j + 1 < L) out[k++] = (j + 1) * L + i;
    /* diagonals from the (up to) four cells that have (i,j) as a corner */
    if (i + 1 < L && j + 1 < L && cell_diag(L, i, j, seed, pt) == 0) out[k++] = (j + 1) * L + (i + 1);
    if (i > 0 && j + 1 < L && cell_diag(L, i - 1, j, seed, pt) == 1) out[k++] = (j + 1) * L + (i - 1);
    if (i + 1 < L && j > 0 && cell_diag(L, i, j - 1, seed, pt) == 1) out[k++] = (j - 1) * L + (i + 1);
    if (i > 0 && j > 0 && cell_diag(L, i - 1, j - 1, seed, pt) == 0) out[k++] = (j - 1) * L + (i - 1);
    /* sort ascending (insertion sort, k <= 8) */
    for (int a = 1; a < k; a++) {
        u32 x = out[a]; int b = a - 1;
        while (b >= 0 && out[b] > x) { out[b + 1] = out[b]; b--; }
        out[b + 1] = x;
    }
    return k;
}

/* Pass 1: degrees into row_ptr (prefix-summed). Returns m. */
u64 gen_lattice_rowptr(u32 L, double p_diag, u64 seed, u64 *row_ptr) {
    u64 n = (u64)L * L;
    u64 pt = diag_threshold(p_diag);
    u32 *deg = (u32 *)malloc(n * sizeof(u32));
    #pragma omp parallel for schedule(static)
    for (long long vv = 0; vv < (long long)n; vv++) {
        u32 tmp[8];
        deg[vv] = (u32)lattice_nbrs(L, (u32)(vv % L), (u32)(vv / L), seed, pt, tmp);
    }
    row_ptr[0] = 0;
    for (u64 v = 0; v < n; v++) row_ptr[v + 1] = row_ptr[v] + deg[v];
    free(deg);
    return row_ptr[n];
}

/* Pass 2: arcs. xy are the coordinates from gen_lattice_coords. */
void gen_lattice_arcs(u32 L, double p_diag, u64 seed, const i32 *xy, u32 frac_bits,
                      const u64 *row_ptr, u32 *col, u32 *w) {
    u64 n = (u64)L * L;
    u64 pt = diag_threshold(p_diag);
    #pragma omp parallel for schedule(static)
    for (long long vv = 0; vv < (long long)n; vv++) {
        u64 v = (u64)vv;
        u32 nb[8];
        int k = lattice_nbrs(L, (u32)(v % L), (u32)(v / L), seed, pt, nb);
        u64 p = row_ptr[v];
        for (int a = 0; a < k; a++) {
            u32 x = nb[a];
            col[p + a] = x;
            w[p + a] = gen_lattice_weight(xy[2 * x] - xy[2 * v], xy[2 * x + 1] - xy[2 * v + 1], frac_bits);
        }
    }
}

/* ---- R-MAT ------------------------------------------------------------------ */

/* Parallel LSD radix sort of u64 keys on their low key_bits bits (16-bit
 * digits; stable: every thread scatters its own contiguous slice, in order,
 * after the slices of lower threads). tmp has the same size as a. */
static void radix_sort_u64(u64 *a, u64 *tmp, u64 n, int key_bits) {
    const u64 NB = 65536;
    const int passes = (key_bits + 15) / 16;
    const int T = omp_get_max_threads();
    u64 *cnt = (u64 *)malloc((u64)T * NB * sizeof(u64));
    u64 *src = a, *dst = tmp;
    for (int p = 0; p < passes; p++) {
        const int sh = 16 * p;
        #pragma omp parallel num_threads(T)
        {
            const int t = omp_get_thread_num(), nt = omp_get_num_threads();
            const u64 lo = n * (u64)t / (u64)nt, hi = n * (u64)(t + 1) / (u64)nt;
            u64 *c = cnt + (u64)t * NB;
            memset(c, 0, NB * sizeof(u64));
            for (u64 i = lo; i < hi; i++) c[(src[i] >> sh) & (NB - 1)]++;
            #pragma omp barrier
            #pragma omp single
            {
                u64 s = 0;
                for (u64 d = 0; d < NB; d++)
                    for (int tt = 0; tt < nt; tt++) {
                        const u64 x = cnt[(u64)tt * NB + d];
                        cnt[(u64)tt * NB + d] = s;
                        s += x;
                    }
            }
            for (u64 i = lo; i < hi; i++) dst[c[(src[i] >> sh) & (NB - 1)]++] = src[i];
        }
        u64 *t = src; src = dst; dst = t;
    }
    if (src != a) memcpy(a, src, n * sizeof(u64));
    free(cnt);
}

/* First index i of the sorted a[0..n) with a[i] >= x. */
static u64 lower_bound_u64(const u64 *a, u64 n, u64 x) {
    u64 lo = 0, hi = n;
    while (lo < hi) {
        const u64 mid = lo + (hi - lo) / 2;
        if (a[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* Generates the R-MAT graph; returns a malloc'd array of unique canonical
 * undirected edges (key = min << scale | max, ascending), count in *n_edges. */
static u64 *rmat_edges(u32 scale, u32 edge_factor, double a, double b, double c,
                       u64 seed, u64 *n_edges) {
    u64 n = 1ULL << scale;
    u64 E = n * edge_factor;
    u64 *keys = (u64 *)malloc(E * sizeof(u64));
    u64 ta = (u64)(a * 9007199254740992.0);
    u64 tb = (u64)((a + b) * 9007199254740992.0);
    u64 tc = (u64)((a + b + c) * 9007199254740992.0);
    /* random relabelling: perm = order of vertices by a random key */
    u64 *pk = (u64 *)malloc(n * sizeof(u64));
    u64 *ptmp = (u64 *)malloc(n * sizeof(u64));
    #pragma omp parallel for schedule(static)
    for (long long v = 0; v < (long long)n; v++)
        pk[v] = ((gen_rand(seed, ST_PERM, (u64)v) >> scale) << scale) | (u64)v;
    radix_sort_u64(pk, ptmp, n, 64);
    u32 *perm = (u32 *)malloc(n * sizeof(u32));
    #pragma omp parallel for schedule(static)
    for (long long r = 0; r < (long long)n; r++) perm[pk[r] & (n - 1)] = (u32)r;  /* vertex -> new id */
    free(pk); free(ptmp);
    /* self-loops get the all-ones key, above every edge key in its low 2 * scale bits */
    const u64 kr = stream_key(seed, ST_RMAT);
    #pragma omp parallel for schedule(static)
    for (long long ee = 0; ee < (long long)E; ee++) {
        u64 u = 0, v = 0;
        for (u32 lvl = 0; lvl < scale; lvl++) {
            u64 r = keyed_rand(kr, (u64)ee * scale + lvl) >> 11;
            int q = (r < ta) ? 0 : (r < tb) ? 1 : (r < tc) ? 2 : 3;
            u = (u << 1) | (u64)(q >> 1);
            v = (v << 1) | (u64)(q & 1);
        }
        u32 pu = perm[u], pv = perm[v];
        if (pu == pv) { keys[ee] = ~0ULL; continue; }
        u64 lo = pu < pv ? pu : pv, hi = pu < pv ? pv : pu;
        keys[ee] = (lo << scale) | hi;
    }
    free(perm);
    u64 *tmp = (u64 *)malloc(E * sizeof(u64));
    radix_sort_u64(keys, tmp, E, 2 * (int)scale);
    free(tmp);
    u64 k = 0;
    for (u64 i = 0; i < E; i++) {
        if (keys[i] == ~0ULL) break;
        if (k == 0 || keys[k - 1] != keys[i]) keys[k++] = keys[i];
    }
    *n_edges = k;
    return keys;
}

/* Opaque holder so Python can size buffers before the fill. */
typedef struct { u64 *edges; u64 ne; u32 scale; u64 seed; u32 wlo, whi; } rmat_state;

void *gen_rmat_begin(u32 scale, u32 edge_factor, double a, double b, double c,
                     u32 wlo, u32 whi, u64 seed, u64 *m_out) {
    rmat_state *st = (rmat_state *)malloc(sizeof(rmat_state));
    st->edges = rmat_edges(scale, edge_factor, a, b, c, seed, &st->ne);
    st->scale = scale; st->seed = seed; st->wlo = wlo; st->whi = whi;
    *m_out = 2 * st->ne;
    return st;
}

/* Builds the symmetric CSR and frees the state. Row v holds its neighbours
 * below v (ascending), then those above v (ascending); the weight of edge
 * {lo, hi} is drawn from the hash of (lo << 32 | hi). The neighbours above v
 * are the edges keyed (v, hi), contiguous in the sorted edge list; those
 * below v come from a copy of the list keyed (hi, lo) and sorted again. */
void gen_rmat_finish(void *h, u64 *row_ptr, u32 *col, u32 *w) {
    rmat_state *st = (rmat_state *)h;
    const u32 s = st->scale;
    const u64 n = 1ULL << s, ne = st->ne, mask = n - 1;
    const u64 span = (u64)st->whi - st->wlo + 1;
    const u64 *e1 = st->edges;
    const u64 kw = stream_key(st->seed, ST_WEIGHT);
    u64 *e2 = (u64 *)malloc((ne ? ne : 1) * sizeof(u64));
    u64 *tmp = (u64 *)malloc((ne ? ne : 1) * sizeof(u64));
    #pragma omp parallel for schedule(static)
    for (long long i = 0; i < (long long)ne; i++) e2[i] = ((e1[i] & mask) << s) | (e1[i] >> s);
    radix_sort_u64(e2, tmp, ne, 2 * (int)s);
    free(tmp);
    u64 *a1 = (u64 *)malloc((n + 1) * sizeof(u64));   /* first edge (v, .) in e1 */
    u64 *a2 = (u64 *)malloc((n + 1) * sizeof(u64));   /* first edge (v, .) in e2 */
    #pragma omp parallel for schedule(static)
    for (long long v = 0; v < (long long)n; v++) {
        a1[v] = lower_bound_u64(e1, ne, (u64)v << s);
        a2[v] = lower_bound_u64(e2, ne, (u64)v << s);
    }
    a1[n] = ne;
    a2[n] = ne;
    row_ptr[0] = 0;
    for (u64 v = 0; v < n; v++) row_ptr[v + 1] = row_ptr[v] + (a1[v + 1] - a1[v]) + (a2[v + 1] - a2[v]);
    #pragma omp parallel for schedule(dynamic, 4096)
    for (long long vv = 0; vv < (long long)n; vv++) {
        const u64 v = (u64)vv;
        u64 p = row_ptr[v];
        for (u64 j = a2[v]; j < a2[v + 1]; j++, p++) {
            const u64 lo = e2[j] & mask;
            col[p] = (u32)lo;
            w[p] = st->wlo + (u32)below(keyed_rand(kw, (lo << 32) | v), span);
        }
        for (u64 j = a1[v]; j < a1[v + 1]; j++, p++) {
            const u64 hi = e1[j] & mask;
            col[p] = (u32)hi;
            w[p] = st->wlo + (u32)below(keyed_rand(kw, (v << 32) | hi), span);
        }
    }
    free(a1); free(a2); free(e2);
    free(st->edges);
    free(st);
}

/* ---- components and pairs ------------------------------------------------------- */

static u32 uf_find(u32 *p, u32 x) {
    while (p[x] != x) { p[x] = p[p[x]]; x = p[x]; }
    return x;
}

/* Writes the vertices of the largest connected component (ascending) to out,
 * returns their count. out must hold n entries. */
u64 gen_lcc(u64 n, const u64 *row_ptr, const u32 *col, u32 *out) {
    u32 *p = (u32 *)malloc(n * sizeof(u32));
    for (u64 v = 0; v < n; v++) p[v] = (u32)v;
    for (u64 v = 0; v < n; v++)
        for (u64 e = row_ptr[v]; e < row_ptr[v + 1]; e++) {
            u32 a = uf_find(p, (u32)v), b = uf_find(p, col[e]);
            if (a != b) { if (a < b) p[b] = a; else p[a] = b; }
        }
    u32 *sz = (u32 *)calloc(n, sizeof(u32));
    u32 best = 0;
    for (u64 v = 0; v < n; v++) { u32 r = uf_find(p, (u32)v); sz[r]++; }
    for (u64 v = 0; v < n; v++) if (sz[v] > sz[best]) best = (u32)v;
    u64 k = 0;
    for (u64 v = 0; v < n; v++) if (uf_find(p, (u32)v) == best) out[k++] = (u32)v;
    free(p); free(sz);
    return k;
}

/* k uniform pairs over the vertex list cand[0..nc) (cand == NULL: all of [0,nc)).
 * distinct != 0 forces s != t. pairs[2i] = s, pairs[2i+1] = t. */
void gen_pairs_uniform(u64 nc, const u32 *cand, u64 k, int distinct, u64 seed, u64 stream_base,
                       u32 *pairs) {
    for (u64 i = 0; i < k; i++) {
        u64 a = below(gen_rand(seed, ST_SRC + stream_base, i), nc);
        u64 b;
        if (distinct && nc > 1) {
            b = below(gen_rand(seed, ST_DST + stream_base, i), nc - 1);
            if (b >= a) b++;
        } else {
            b = below(gen_rand(seed, ST_DST + stream_base, i), nc);
        }
        pairs[2 * i] = cand ? cand[a] : (u32)a;
        pairs[2 * i + 1] = cand ? cand[b] : (u32)b;
    }
}

/* Hub batch: the first k_hub pairs take s from n_hubs hub vertices (hubs are
 * uniform over the candidates and fixed by the seed), t uniform; the remaining
 * k - k_hub pairs are uniform. Batch number `batch` selects fresh draws. */
void gen_pairs_hub(u64 nc, const u32 *cand, u64 n_hubs, u64 k_hub, u64 k, u64 seed, u64 batch,
                   u32 *pairs) {
    for (u64 i = 0; i < k; i++) {
        u64 idx = batch * k + i;
        u64 a, b;
        if (i < k_hub) {
            u64 h = below(gen_rand(seed, ST_HUBPICK, idx), n_hubs);
            a = below(gen_rand(seed, ST_HUB, h), nc);
        } else {
            a = below(gen_rand(seed, ST_SRC + 100, idx), nc);
        }
        b = below(gen_rand(seed, ST_DST + 100, idx), nc);
        pairs[2 * i] = cand ? cand[a] : (u32)a;
        pairs[2 * i + 1] = cand ? cand[b] : (u32)b;
    }
}
