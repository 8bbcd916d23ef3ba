/*
 * CPU oracle for point-to-point shortest paths. TEST INFRASTRUCTURE ONLY:
 * it is used by the test suite, by the smoke check and by the benchmark's
 * CPU baseline, never by the product path. It shares no code with the GPU
 * library.
 *
 * What it computes is the plain definition of the result: d(s,t) is the
 * minimum over s->t paths of the summed non-negative integer weights, 0 when
 * s = t and "infinity" (UINT64_MAX) when t is unreachable (problem statement
 * of Section 1, notation of Section 2). Every search mode of the method (early
 * termination, A*, bidirectional search, bidirectional A*, and the batch
 * query-graph search of Section 4) is exact, so the oracle does not replay the
 * method; it computes the definition with textbook algorithms:
 *   - Dijkstra with a binary heap and lazy deletion (the stepping framework of
 *     Section 2 with the threshold set to the minimum frontier key), stopping
 *     when t is popped;
 *   - Floyd-Warshall (all pairs, tiny graphs) and Bellman-Ford (single source),
 *     used only to pin Dijkstra;
 *   - an SSSP optimality certificate: d[s] = 0, every arc feasible
 *     (d[v] <= d[u] + w), every reached v != s has a tight in-arc, and d is
 *     finite exactly on the vertices reachable from s. With weights >= 1 these
 *     together prove d is the exact distance function;
 *   - a path validator (arcs exist, weights sum to the distance, endpoints).
 * Integer arithmetic throughout, uint64 distances.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

typedef uint64_t u64;
typedef uint32_t u32;

#define INF UINT64_MAX

/* ---- binary min-heap of (key, vertex) ------------------------------------ */

typedef struct { u64 key; u32 v; } item;
typedef struct { item *a; u64 size, cap; } heap;

static void heap_push(heap *h, u64 key, u32 v) {
    if (h->size == h->cap) {
        h->cap = h->cap ? 2 * h->cap : 1024;
        h->a = (item *)realloc(h->a, h->cap * sizeof(item));
    }
    u64 i = h->size++;
    while (i > 0) {
        u64 p = (i - 1) / 2;
        if (h->a[p].key <= key) break;
        h->a[i] = h->a[p];
        i = p;
    }
    h->a[i].key = key; h->a[i].v = v;
}

static item heap_pop(heap *h) {
    item top = h->a[0];
    item last = h->a[--h->size];
    u64 i = 0;
    for (;;) {
        u64 c = 2 * i + 1;
        if (c >= h->size) break;
        if (c + 1 < h->size && h->a[c + 1].key < h->a[c].key) c++;
        if (h->a[c].key >= last.key) break;
        h->a[i] = h->a[c];
        i = c;
    }
    if (h->size > 0) h->a[i] = last;
    return top;
}

/* ---- Dijkstra ----------------------------------------------------------------- */

/* Dijkstra from s over the out-arcs of the CSR. If t < n, stops as soon as t
 * is popped (its distance is final then) and returns d(s,t); otherwise runs to
 * completion and returns 0. dist[n] receives tentative distances (exact for
 * every popped vertex), parent[n] (optional) the predecessor set on each strict
 * improvement (UINT32_MAX for none). */
u64 oracle_dijkstra(u64 n, const u64 *row_ptr, const u32 *col, const u32 *w,
                    u32 s, u32 t, u64 *dist, u32 *parent) {
    for (u64 v = 0; v < n; v++) dist[v] = INF;
    if (parent) for (u64 v = 0; v < n; v++) parent[v] = UINT32_MAX;
    heap h = {0, 0, 0};
    dist[s] = 0;
    heap_push(&h, 0, s);
    u64 result = (t < n) ? INF : 0;
    while (h.size > 0) {
        item it = heap_pop(&h);
        if (it.key != dist[it.v]) continue;          /* stale entry */
        if (it.v == t) { result = it.key; break; }
        for (u64 e = row_ptr[it.v]; e < row_ptr[it.v + 1]; e++) {
            u32 x = col[e];
            u64 nd = it.key + w[e];
            if (nd < dist[x]) {
                dist[x] = nd;
                if (parent) parent[x] = it.v;
                heap_push(&h, nd, x);
            }
        }
    }
    free(h.a);
    return result;
}

/* ---- batch runner: one Dijkstra per pair, queries spread over threads ----------- */

typedef struct {
    u64 n; const u64 *rp; const u32 *col; const u32 *w;
    u64 k; const u32 *pairs; u64 *out;
    int tid, nthreads;
} job;

static void *worker(void *arg) {
    job *j = (job *)arg;
    u64 *dist = (u64 *)malloc(j->n * sizeof(u64));
    for (u64 q = (u64)j->tid; q < j->k; q += (u64)j->nthreads) {
        u32 s = j->pairs[2 * q], t = j->pairs[2 * q + 1];
        j->out[q] = oracle_dijkstra(j->n, j->rp, j->col, j->w, s, t, dist, NULL);
    }
    free(dist);
    return NULL;
}

/* d(s_q, t_q) for k pairs; pairs[2q] = s, pairs[2q+1] = t. Uses nthreads
 * POSIX threads (each with its own distance array of n words). */
void oracle_pp_batch(u64 n, const u64 *row_ptr, const u32 *col, const u32 *w,
                     u64 k, const u32 *pairs, u64 *out, int nthreads) {
    if (nthreads < 1) nthreads = 1;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * nthreads);
    job *jobs = (job *)malloc(sizeof(job) * nthreads);
    for (int i = 0; i < nthreads; i++) {
        jobs[i] = (job){n, row_ptr, col, w, k, pairs, out, i, nthreads};
        pthread_create(&th[i], NULL, worker, &jobs[i]);
    }
    for (int i = 0; i < nthreads; i++) pthread_join(th[i], NULL);
    free(th); free(jobs);
}

/* ---- brute force pins ----------------------------------------------------------- */

/* All-pairs distances D[u*n+v] by Floyd-Warshall (n small). */
void oracle_floyd_warshall(u64 n, const u64 *row_ptr, const u32 *col, const u32 *w, u64 *D) {
    for (u64 i = 0; i < n * n; i++) D[i] = INF;
    for (u64 u = 0; u < n; u++) {
        D[u * n + u] = 0;
        for (u64 e = row_ptr[u]; e < row_ptr[u + 1]; e++)
            if (w[e] < D[u * n + col[e]]) D[u * n + col[e]] = w[e];
    }
    for (u64 k = 0; k < n; k++)
        for (u64 i = 0; i < n; i++) {
            u64 dik = D[i * n + k];
            if (dik == INF) continue;
            for (u64 j = 0; j < n; j++) {
                u64 dkj = D[k * n + j];
                if (dkj != INF && dik + dkj < D[i * n + j]) D[i * n + j] = dik + dkj;
            }
        }
}

/* Single-source distances by Bellman-Ford (repeat full passes over all arcs
 * until nothing changes; at most n-1 passes are needed). Returns #passes. */
u64 oracle_bellman_ford(u64 n, const u64 *row_ptr, const u32 *col, const u32 *w, u32 s, u64 *dist) {
    for (u64 v = 0; v < n; v++) dist[v] = INF;
    dist[s] = 0;
    u64 pass = 0;
    for (int changed = 1; changed && pass < n; pass++) {
        changed = 0;
        for (u64 u = 0; u < n; u++) {
            if (dist[u] == INF) continue;
            for (u64 e = row_ptr[u]; e < row_ptr[u + 1]; e++)
                if (dist[u] + w[e] < dist[col[e]]) { dist[col[e]] = dist[u] + w[e]; changed = 1; }
        }
    }
    return pass;
}

/* ---- certificates ------------------------------------------------------------- */

/* Checks that dist[] is the exact single-source distance function from s.
 * Requires weights >= 1. Returns 0 on success, otherwise
 *   1: dist[s] != 0
 *   2: an arc u->v with dist[u] finite and dist[v] > dist[u] + w (infeasible)
 *   3: a vertex v != s with finite dist[v] and no tight in-arc
 *   4: finiteness of dist disagrees with reachability from s (BFS)
 * and writes the offending vertex to *bad. */
int oracle_check_sssp(u64 n, const u64 *row_ptr, const u32 *col, const u32 *w,
                      u32 s, const u64 *dist, u64 *bad) {
    if (dist[s] != 0) { *bad = s; return 1; }
    unsigned char *tight = (unsigned char *)calloc(n, 1);
    for (u64 u = 0; u < n; u++) {
        if (dist[u] == INF) continue;
        for (u64 e = row_ptr[u]; e < row_ptr[u + 1]; e++) {
            u32 v = col[e];
            if (dist[v] > dist[u] + w[e]) { free(tight); *bad = v; return 2; }
            if (dist[v] == dist[u] + w[e]) tight[v] = 1;
        }
    }
    for (u64 v = 0; v < n; v++)
        if (v != s && dist[v] != INF && !tight[v]) { free(tight); *bad = v; return 3; }
    /* reachability by BFS */
    unsigned char *seen = tight;
    memset(seen, 0, n);
    u32 *q = (u32 *)malloc(n * sizeof(u32));
    u64 head = 0, tail = 0;
    q[tail++] = s; seen[s] = 1;
    while (head < tail) {
        u32 u = q[head++];
        for (u64 e = row_ptr[u]; e < row_ptr[u + 1]; e++)
            if (!seen[col[e]]) { seen[col[e]] = 1; q[tail++] = col[e]; }
    }
    int rc = 0;
    for (u64 v = 0; v < n; v++)
        if ((dist[v] != INF) != (seen[v] != 0)) { *bad = v; rc = 4; break; }
    free(q); free(seen);
    return rc;
}

/* Validates an s->t path: path[0] = s, path[len-1] = t, each consecutive pair
 * is an arc, and the sum of the (minimum, if parallel) arc weights equals d.
 * Returns 0 if valid; 1 bad endpoints; 2 missing arc (index in *bad);
 * 3 weight sum differs (sum in *bad). */
int oracle_check_path(u64 n, const u64 *row_ptr, const u32 *col, const u32 *w,
                      const u32 *path, u64 len, u32 s, u32 t, u64 d, u64 *bad) {
    (void)n;
    if (len == 0 || path[0] != s || path[len - 1] != t) { *bad = 0; return 1; }
    u64 sum = 0;
    for (u64 i = 0; i + 1 < len; i++) {
        u32 a = path[i], b = path[i + 1];
        u64 best = INF;
        for (u64 e = row_ptr[a]; e < row_ptr[a + 1]; e++)
            if (col[e] == b && w[e] < best) best = w[e];
        if (best == INF) { *bad = i; return 2; }
        sum += best;
    }
    if (sum != d) { *bad = sum; return 3; }
    return 0;
}
