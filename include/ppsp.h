/*
 * ppsp.h - C interface of the MI355X (gfx950) point-to-point shortest-path
 * library.
 *
 * The library answers exact s-t shortest-path distance queries on a graph
 * with non-negative integer arc weights, single or batched, with the
 * parallel point-to-point framework of "Parallel Point-to-Point Shortest
 * Paths and Batch Queries" (SPAA 2025):
 *   - Algorithm 2 (the PPSP framework built on the stepping framework of
 *     Algorithm 1), with the Init / Prune / UpdateDistance rules of Table 2:
 *     early termination (Section 3.2), A* (Section 3.3), bidirectional search
 *     (Section 3.4, Theorem bids-correctness) and bidirectional A*
 *     (Section 3.5, Theorem bdastar-correctness);
 *   - Delta*-stepping thresholds (Section 2: the i-th threshold is i*Delta);
 *   - batch queries through the query graph (Section 4.1) and the Plain,
 *     Plain*, Multi-BiDS (Section 4.2), Plain-SSSP and VC-SSSP (Section 4.3) strategies,
 *     with the paper's adaptation to directed graphs (bipartite query graph,
 *     backward searches on the transposed graph);
 *   - single-source distances (ppsp_sssp), an autotuner, a learned step
 *     schedule and a continuous-batching server around the same kernels.
 * Every mode computes exact distances; the threshold schedule only decides
 * the order of work.
 *
 * Conventions for every function:
 *   - The return value is a status: PPSP_OK (0) or a negative PPSP_E_* code.
 *     On error, caller-owned outputs are left untouched unless stated.
 *   - Host pointers are owned by the caller and are only read (or written, for
 *     outputs) during the call. Device memory is owned by the library and is
 *     released by ppsp_graph_destroy.
 *   - `hip_stream` is a hipStream_t (NULL = the default stream). Work is
 *     ordered on that stream; functions with host outputs synchronise it
 *     before returning.
 *   - A graph handle is not thread-safe: calls on one handle must not
 *     overlap.
 *   - Distances are uint64; PPSP_INF marks an unreachable target. Internally
 *     distances are 32-bit: a distance that would reach 2^32-1 returns
 *     PPSP_E_OVERFLOW instead of a wrong value.
 */
#ifndef PPSP_H
#define PPSP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PPSP_INF UINT64_MAX

/* Status codes. */
enum {
    PPSP_OK = 0,
    PPSP_E_INVALID = -1,   /* null pointer, bad enum value, bad size, inconsistent CSR */
    PPSP_E_RANGE = -2,     /* a vertex id >= n, m >= 2^32, or coordinates too far apart */
    PPSP_E_OOM = -3,       /* device memory (or the search-state budget) is exhausted */
    PPSP_E_OVERFLOW = -4,  /* a tentative distance reached 2^32-1 */
    PPSP_E_NOCOORD = -5,   /* A* mode on a graph without consistent coordinates */
    PPSP_E_NOTSYM = -6,    /* reserved: no call returns it (every mode runs on directed graphs) */
    PPSP_E_DEVICE = -7,    /* a HIP runtime error */
    PPSP_E_BUSY = -8,      /* (serving) the request has not finished, or the graph belongs to a server */
    PPSP_E_PATHCAP = -9,   /* the caller's path buffer is too small; *path_len gets the need */
    PPSP_E_NOPATH = -10,   /* paths were requested on a graph with a zero-weight arc */
    PPSP_E_TIMEOUT = -11   /* the round loop ran longer than the "timeout_ms" option */
};

/* Search algorithm: the rows of Table 2 plus plain single-source search. */
enum ppsp_algo {
    PPSP_SSSP = 0,      /* Delta*-stepping from s without pruning; reports d(s,t) */
    PPSP_ET = 1,        /* early termination: prune delta[v] >= mu (Section 3.2) */
    PPSP_ASTAR = 2,     /* A*: prune delta[v] + h_t(v) >= mu (Section 3.3) */
    PPSP_BIDS = 3,      /* bidirectional: prune 2*delta >= mu (Section 3.4) */
    PPSP_BIDASTAR = 4   /* bidirectional A*: prune 2*delta +/- (h_t - h_s) >= mu (Section 3.5) */
};

/* Batch strategy: the BiDS-based strategies of Section 4.2 and the SSSP-based ones of Section 4.3. */
enum ppsp_batch {
    PPSP_BATCH_PLAIN = 0,      /* one query after another */
    PPSP_BATCH_PLAINSTAR = 1,  /* all queries at once, each with its own searches */
    PPSP_BATCH_MULTI = 2,      /* one search per query-graph vertex, shared (Multi-BiDS) */
    PPSP_BATCH_SSSP = 3,       /* Plain-SSSP: one full SSSP per distinct source */
    PPSP_BATCH_VC = 4,         /* VC-SSSP: one full SSSP per vertex of a vertex cover of the query graph */
    PPSP_BATCH_AUTO = 5        /* VC-SSSP when a cover is small against the query graph, else Multi-BiDS */
};

/* Threshold schedule. */
enum ppsp_sched {
    PPSP_SCHED_FIXED = 0,      /* Delta*-stepping with opts.delta (0: graph default) */
    PPSP_SCHED_AUTOTUNED = 1,  /* the Delta and launch shape chosen by ppsp_tune (defaults until then) */
    PPSP_SCHED_LEARNED = 2,    /* per-round Delta multiplier chosen by the loaded MLP */
    PPSP_SCHED_RHO = 3         /* rho-stepping style (Section 2): each search's step is halved when its
                                  next frontier holds more than 2 rho entries and doubled below rho / 2
                                  (multipliers 2^-4 .. 2^3 of Delta; option "rho", default 4096) */
};

/* ppsp_graph_create flags. */
#define PPSP_SYMMETRIC 1u      /* every arc (u,v,w) has a reverse arc (v,u,w) */
#define PPSP_REORDER 4u        /* graph_create: store vertices in a locality order (see ppsp_graph_create) */

/* ppsp_opts.flags. */
#define PPSP_WANT_PATH 1u      /* also return an s->t vertex path per query */
#define PPSP_PULL 4u           /* pull relaxation (Appendix B): before an extracted vertex u pushes,
                                  delta[u] <- min over its arcs (v, u) of delta[v] + w; symmetric graphs
                                  only (ignored otherwise). Results are identical with or without it. */
#define PPSP_MEMO_H 2u         /* memoise the heuristic per query and vertex (Section 5): A* and BiD-A*,
                                  Plain / Plain*; one 8-byte word per query and vertex, shared by the
                                  query's two searches. Results are identical with or without it. */
#define PPSP_DEVICE_IO 8u      /* ppsp_batch_query: `pairs` and `dist` are device pointers (on the graph's
                                  device), read and written in order on the caller's stream; paths stay
                                  host arrays. The batch is planned on the host, so the call copies the
                                  pairs to host memory and the distances back (8 B each per query) and
                                  synchronises with the caller's stream to do so */

typedef struct {
    uint32_t algo;     /* enum ppsp_algo */
    uint32_t batch;    /* enum ppsp_batch (ignored by ppsp_query) */
    uint32_t sched;    /* enum ppsp_sched */
    uint32_t flags;    /* PPSP_WANT_PATH | PPSP_MEMO_H | PPSP_PULL | PPSP_DEVICE_IO */
    uint64_t delta;    /* Delta in distance units for PPSP_SCHED_FIXED; 0 = graph default */
} ppsp_opts;

/* Counters of the last query or batch on a graph. */
typedef struct {
    uint64_t rounds;           /* stepping rounds (threshold steps) executed */
    uint64_t entries;          /* frontier entries processed (incl. pruned and carried) */
    uint64_t scanned_vertices; /* extracted, unpruned search-vertices whose arcs were relaxed */
    uint64_t scanned_arcs;     /* arcs relaxed */
    uint64_t relax_success;    /* successful write_min operations */
    uint64_t searches;         /* searches (frontier copies) in the batch */
    uint64_t waves;            /* memory waves the batch was split into */
    double wall_ms;            /* host wall time of the call */
    double relax_kernel_ms;    /* summed duration of the timed round-kernel launches ("profile"), else 0 */
    uint64_t relax_launches;   /* number of round-kernel launches */
    uint64_t carried;          /* entries kept for a later round (key above the threshold) */
    uint64_t retries;          /* waves rerun after growing an overflowed frontier queue */
    uint64_t relax_timed;      /* round-kernel launches timed ("profile"): relax_kernel_ms covers these */
    double heavy_kernel_ms;    /* summed duration of the hub-list kernel launches of the same timed rounds
                                  (graphs with vertices of degree > 512), else 0 */
    uint64_t heavy_arcs;       /* arcs of extracted vertices of degree > 512, relaxed by the hub-list kernel
                                  (included in scanned_arcs) */
    uint64_t heavy_chunks;     /* hub-list chunk records (at most 2,048 arcs of one vertex each) */
    uint64_t heavy_success;    /* successful write_min operations of the hub-list kernel (in relax_success) */
    uint64_t dense_searches;   /* searches whose frontier switched to dense bitmaps (options "dense_min",
                                  "dense_force", "dense_learned") */
} ppsp_stats;

typedef struct ppsp_graph_s *ppsp_graph;

/*
 * Uploads a CSR graph (Section 2 notation: G = (V, E, w), N(v) = the arcs of
 * v) to device `device` and returns a handle.
 *   n          number of vertices (ids 0..n-1)
 *   m          number of arcs; must be < 2^32
 *   row_ptr    host, n+1 entries, nondecreasing, row_ptr[0] = 0, row_ptr[n] = m
 *   col, w     host, m entries: arc e goes from its row's vertex to col[e] with
 *              weight w[e] (non-negative integer)
 *   coord_fx   host, 2n int32 fixed-point coordinates (x0,y0,x1,y1,...) with
 *              coord_frac_bits fractional bits, or NULL. They define the
 *              heuristic h_t(v) = floor(w_scale * |p_v - p_t|) used by A* and
 *              bidirectional A* (Sections 3.3, 3.5). The heuristic is consistent
 *              iff every arc satisfies w >= w_scale * |p_u - p_v|; this is checked
 *              here exactly in integers, and A* modes return PPSP_E_NOCOORD on a
 *              graph where it fails.
 *   flags      PPSP_SYMMETRIC if the graph is undirected (required by the
 *              query-graph batch strategies; on directed graphs the backward
 *              search of a bidirectional query walks the transpose).
 *              PPSP_REORDER: the device copy numbers the vertices in a
 *              locality order (Morton order of the coordinates when given,
 *              else the vertices of degree above 128 first, ranked by
 *              descending degree with runs of 8 interleaved by quarter of
 *              that ranking, then the rest breadth-first from the
 *              highest-degree vertex), so that vertices close in the graph,
 *              and the hubs that most arcs lead to, share cache lines of the
 *              search state; each row's arcs are then sorted by new head id.
 *              Vertex ids at the interface stay the caller's (pairs and
 *              paths are translated); results are identical.
 *   out        receives the handle
 * Errors: PPSP_E_INVALID (bad CSR), PPSP_E_RANGE (col >= n, m too large,
 * coordinate span too large for exact 64-bit arithmetic, or a heuristic
 * value across the coordinates' bounding box of 2^31 or more: the kernels
 * carry heuristic terms as signed 32-bit values), PPSP_E_OOM, PPSP_E_DEVICE.
 */
int ppsp_graph_create(int device, uint32_t n, uint64_t m, const uint64_t *row_ptr,
                      const uint32_t *col, const uint32_t *w, const int32_t *coord_fx,
                      uint32_t coord_frac_bits, uint32_t w_scale, uint32_t flags,
                      void *hip_stream, ppsp_graph *out);

/* Releases all device memory of the graph. NULL is accepted. */
int ppsp_graph_destroy(ppsp_graph g);

/*
 * One s-t query (Algorithm 2 with the Table 2 row named by opts->algo).
 *   dist      host, 1 entry: d(s,t), 0 if s = t, PPSP_INF if unreachable
 *             (the disconnected-query rule of Appendix B)
 *   path      host buffer of path_cap vertex ids, or NULL; filled with an
 *             s->t shortest path (s first, t last) when opts->flags has
 *             PPSP_WANT_PATH; *path_len gets its length (0 if unreachable)
 * On a graph not flagged PPSP_SYMMETRIC the backward search of BiDS and
 * BiD-A* walks the transposed graph.
 * Errors: PPSP_E_RANGE (s or t >= n), PPSP_E_NOCOORD,
 * PPSP_E_OVERFLOW, PPSP_E_PATHCAP (path_cap too small; *path_len = need),
 * PPSP_E_NOPATH, PPSP_E_OOM, PPSP_E_DEVICE.
 */
int ppsp_query(ppsp_graph g, uint32_t s, uint32_t t, const ppsp_opts *opts, void *hip_stream,
               uint64_t *dist, uint32_t *path, uint32_t path_cap, uint32_t *path_len);

/*
 * Single-source shortest paths from s (the SSSP row of Table 2: one search
 * without pruning, run until its frontier is empty), with the stepping
 * schedule of opts (delta, sched other than PPSP_SCHED_LEARNED; algo,
 * batch and flags are ignored).
 *   dist      host, n entries: d(s, v), PPSP_INF where v is unreachable
 * Errors: PPSP_E_RANGE (s >= n), PPSP_E_INVALID, PPSP_E_BUSY (served
 * graph), PPSP_E_OVERFLOW, PPSP_E_OOM, PPSP_E_DEVICE.
 */
int ppsp_sssp(ppsp_graph g, uint32_t s, const ppsp_opts *opts, void *hip_stream, uint64_t *dist);

/*
 * A batch of k queries (Section 4): pairs[2q] = s_q, pairs[2q+1] = t_q (host, or
 * device memory with PPSP_DEVICE_IO, as is dist).
 * Duplicate pairs, (t,s) mirrors and s = t are allowed.
 *   dist      host, k entries, in input order
 *   path_off  host, k+1 entries or NULL: with PPSP_WANT_PATH, the path of query
 *             q is path_vtx[path_off[q] .. path_off[q+1])
 *   path_vtx  host buffer of path_cap vertex ids, or NULL
 * opts->batch selects Plain, Plain* or Multi-BiDS; Multi-BiDS requires
 * algo = PPSP_BIDS (the paper defines no batched heuristic search).
 * The SSSP-based strategies of Section 4.3 run one search without pruning per
 * root and read every query's distance off its root's search: Plain-SSSP
 * (PPSP_BATCH_SSSP) roots one search at every distinct source; VC-SSSP
 * (PPSP_BATCH_VC) at the vertices of a vertex cover of the query graph
 * (ppsp_query_cover: exact minimum per component of at most 16 query-graph
 * vertices, greedy by uncovered degree above that; on a directed graph the
 * query graph is bipartite and the cover an exact minimum, a covered target
 * running a backward search on the transpose), each query answered by a
 * cover endpoint. Both take algo = PPSP_SSSP. On a directed graph Multi-BiDS
 * starts a forward search from every source and a backward search from every
 * target (a vertex that is both gets both). PPSP_BATCH_AUTO (algo =
 * PPSP_BIDS) runs VC-SSSP when the cover has at most a quarter of the
 * query-graph vertices (star- and fork-like batches, where one search
 * answers many queries), else Multi-BiDS.
 * Batches whose search state exceeds the memory budget are split into waves
 * of whole query-graph components.
 * Errors: as ppsp_query; PPSP_E_INVALID for Multi with another algorithm.
 */
int ppsp_batch_query(ppsp_graph g, const uint32_t *pairs, uint32_t k, const ppsp_opts *opts,
                     void *hip_stream, uint64_t *dist, uint64_t *path_off, uint32_t *path_vtx,
                     uint64_t path_cap);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * ppsp_batch_query for Plain and Plain* batches without any allocation.
 * Every workspace buffer of the call (search state, frontier queues, heavy
 * list, control words) is carved from a fixed device array of
 * PPSP_NOALLOC_SCRATCH_BYTES that each GPU holds from the first such call
 * until the process ends; the graph's own workspace is left as it was.
 * Batches whose state does not fit run in several waves of whole queries
 * inside it. Work is ordered on hip_stream itself (NULL = the default
 * stream), which is synchronised before returning. Calls on one GPU share
 * the array: calls that overlap on one GPU race, and must not be issued
 * concurrently (each call clears what it reads before use).
 *   pairs, dist   as ppsp_batch_query (host, or device with PPSP_DEVICE_IO)
 *   opts          batch PPSP_BATCH_PLAIN or PPSP_BATCH_PLAINSTAR, sched
 *                 PPSP_SCHED_FIXED or PPSP_SCHED_AUTOTUNED; flags may hold
 *                 PPSP_PULL and PPSP_DEVICE_IO (no paths, no memo)
 * Errors: PPSP_E_INVALID (another strategy, schedule or flag), PPSP_E_OOM
 * with ppsp_last_error() saying so when one query on the graph (two searches
 * of 8 bytes per vertex each, plus its queues) does not fit the scratch, and
 * the errors of ppsp_batch_query.
 */
#define PPSP_NOALLOC_SCRATCH_BYTES (128ull << 20)
int ppsp_batch_query_noalloc(ppsp_graph g, const uint32_t *pairs, uint32_t k, const ppsp_opts *opts,
                             void *hip_stream, uint64_t *dist);

/* Result of ppsp_tune. */
typedef struct {
    uint64_t delta;        /* chosen Delta (distance units) */
    uint32_t theta_mode;   /* chosen threshold rule (see "theta_mode") */
    uint32_t grid_blocks;  /* chosen round-kernel workgroups (0 = default) */
    double ms;             /* wall time of the sample batch with the choice */
    double default_ms;     /* wall time of the sample batch with the defaults */
    uint32_t trials;       /* configurations timed */
    uint32_t from_cache;   /* 1 if read from cache_path */
    uint32_t heavy_window; /* chosen "heavy_window" (graphs with vertices of degree > 512) */
    uint32_t local_chunks; /* chosen "local_chunks" (A* and BiD-A*; else the graph's setting) */
    uint64_t dense_min;    /* chosen "dense_min" (0: sparse frontiers only) */
    uint32_t dense_ring;   /* chosen "dense_ring" */
} ppsp_tune_result;

/*
 * Chooses the threshold schedule and launch shape for (opts->algo,
 * opts->batch) by timing the sample batch `pairs` (k pairs, host). Delta is
 * first swept by doubling from a small start while the time improves (the
 * tuning procedure of Section 6.1), then the hub window ("heavy_window", on
 * graphs with vertices of degree > 512), the threshold rule, Delta between the
 * doublings, the number of round-kernel workgroups, dense frontiers ("dense_min"
 * 2^16 or 2^18, then "dense_ring" 16, 32 or 64 together with the step, a half
 * or a quarter of it) and, for A* and BiD-A*,
 * the local-chunk budget ("local_chunks") are refined. The choice
 * is kept in the handle and used by PPSP_SCHED_AUTOTUNED. With cache_path
 * (or NULL) the choice is read from / appended to a text file keyed by a hash
 * of the graph, so a later process can skip the timing. Results of queries are
 * identical under every choice; only their speed differs.
 */
int ppsp_tune(ppsp_graph g, const uint32_t *pairs, uint32_t k, const ppsp_opts *opts, const char *cache_path,
              ppsp_tune_result *out);

/*
 * Learned step schedule (PPSP_SCHED_LEARNED). The stepping framework of
 * Section 2 lets any threshold sequence through (Theorems bids-correctness
 * and bdastar-correctness hold for every stepping rule), and the best Delta
 * depends on the query (Section 2's discussion of Delta and rho). With a
 * network loaded on the graph, every search picks its own step each round:
 * a 12 -> 64 -> 64 -> 9 perceptron (ReLU; parameters in bf16 on the device,
 * fp32 arithmetic) maps 12 features of the search's state to one of 8
 * multipliers 2^(b-4) of the base Delta (the argmax of outputs 0..7); the
 * threshold rule stays the graph's "theta_mode". Output 8 > 0 switches the
 * search's frontier to dense bitmaps (the dense mode of Appendix B, option
 * "dense_learned"). Distances are exact whatever the network says.
 *
 * Parameters: PPSP_MLP_PARAMS floats, row-major, in this order:
 *   W1 [64][12], b1 [64], W2 [64][64], b2 [64], W3 [9][64], b3 [9].
 * Features (per search after each round; Delta = its base Delta, in key units):
 *   0 log2(1+extracted)/16  1 log2(1+arcs scanned)/16  2 log2(1+next frontier)/16
 *   3 (log2(1+next) - log2(1+partner's next))/8   4 log2(1+(bound-minkey)/Delta)/16 (0 if bound infinite)
 *   5 bound infinite (1/0)  6 log2(1+(minkey-theta)/Delta)/8  7 log2(1+(theta-root key)/Delta)/16
 *   8 log2(1+heuristic s-t distance/Delta)/16  9 log2(1+round)/16
 *   10 progress (theta-root key)/(bound-root key) in [0,1] (0 if bound infinite)  11 log2(m/n)/4
 * Labels y (< PPSP_MLP_LABELS): y = bin + 8 * m, bin the best multiplier,
 * m = 0 (no mode label), 1 (sparse frontier best) or 2 (dense frontier best).
 * Loss per row: softmax cross-entropy of outputs 0..7 against bin, plus for
 * m > 0 the logistic loss log(1 + e^z8) - [m = 2] z8.
 *
 * ppsp_mlp_forward  outputs [n][9] of feature rows x [n][12] (device `device`).
 * ppsp_mlp_grad     mean loss of labels y and its gradient with respect to
 *                   the parameters (grad: PPSP_MLP_PARAMS).
 * ppsp_mlp_train    Adam (lr, beta 0.9/0.999) on mini-batches of `batch` rows,
 *                   reshuffled every epoch from `seed`; params is the initial
 *                   value on entry and the result on return; losses are the
 *                   full-data mean before and after.
 * ppsp_mlp_load     installs params on g (rounded to bf16); enables
 *                   PPSP_SCHED_LEARNED there.
 * ppsp_sched_trace  runs a Plain or Plain* batch with the multiplier bin of
 *                   each pair fixed (bins[k], NULL = 4, i.e. the base Delta),
 *                   records up to cap feature rows (feat [cap][12], row_pair:
 *                   the pair each row belongs to; *nrows = rows produced,
 *                   possibly more than cap) and per pair the rounds its
 *                   searches ran and the arcs they scanned.
 * ppsp_mlp_fit      the whole training recipe on sample pairs, then
 *                   ppsp_mlp_load. Labels: label_mode 0 times every pair
 *                   alone under each of the 8 fixed multipliers (the fastest
 *                   wins); label_mode 1 runs the sample batch under each fixed
 *                   multiplier, fits batch time = c0 + c_round * rounds +
 *                   c_arc * arcs, and labels a pair with the bin minimising
 *                   c_arc * its arcs + c_round * its rounds beyond the best
 *                   fixed batch's (rounds that end before the batch does are
 *                   free). Feature rows are traced along the labelled and the
 *                   default trajectories; training starts from `init`
 *                   (caller-drawn). Fixed-Delta stepping then referees the
 *                   result: the sample batch is timed under the trained
 *                   network and under constant networks that always pick the
 *                   base multiplier (bin 4) or, in label_mode 1, the fastest
 *                   fixed one; a faster constant network is installed and
 *                   returned in params_out instead (rep->fallback_bin).
 *                   label_mode 2 (counterfactual): the first three quarters
 *                   of the pairs (all of them below 8 pairs) train, the rest
 *                   referee. Every training pair runs under each fixed bin
 *                   (batch time fitted as c0 + c_round * rounds + c_arc *
 *                   arcs + c_entry * frontier entries, non-negative
 *                   coefficients, with the rounds term whenever a fit with it
 *                   exists) and under replays that follow the base
 *                   multiplier up to one of six decision rounds spread over
 *                   its run and switch there to each bin, with a sparse or a
 *                   dense frontier; the label of a (pair, decision round) is
 *                   the bin and mode of lowest fitted cost (c_arc * arcs +
 *                   c_entry * entries + c_round * rounds beyond the best fixed
 *                   batch's, plus for a dense frontier the bitmap each of its
 *                   searches reads every round from the switch on, n / 8
 *                   bytes at 4 TB/s), the base (bin 4, sparse) unless another is at
 *                   least 1% cheaper, and it holds until the next switch
 *                   point. "dense_learned" is set when some label chose dense. The rows are the base trajectory's
 *                   features at those decision rounds. The referee times the
 *                   held-out pairs under the trained network and through
 *                   the plain fixed-Delta path (base Delta, the graph's
 *                   threshold rule); if the plain path is faster,
 *                   PPSP_SCHED_LEARNED runs it on this graph until the next
 *                   ppsp_mlp_load (rep->plain_fallback = 1).
 * Errors: PPSP_E_INVALID (null pointers, label >= PPSP_MLP_LABELS, a non-finite
 * parameter, a strategy other than Plain / Plain* for tracing or fitting),
 * the errors of ppsp_batch_query.
 */
#define PPSP_MLP_FEATURES 12
#define PPSP_MLP_BINS 8
#define PPSP_MLP_OUTPUTS 9
#define PPSP_MLP_LABELS 24
#define PPSP_MLP_PARAMS 5577

typedef struct {
    uint32_t label_hist[8];   /* pairs per label bin */
    uint64_t rows;            /* training rows */
    double loss_first;        /* mean loss before training */
    double loss_last;         /* after */
    double train_acc;         /* fraction of rows whose argmax is the label */
    double label_ms;          /* time spent labelling */
    double train_ms;          /* time spent training */
    double c_round_ms;        /* label_mode 1: fitted cost of a batch round (ms) */
    double c_arc_ns;          /* label_mode 1: fitted cost of a scanned arc (ns) */
    uint32_t best_fixed_bin;  /* label_mode 1: the fastest fixed multiplier bin for the sample batch */
    uint32_t fallback_bin;    /* PPSP_MLP_BINS: the trained network was installed; else the bin of the
                                 constant network installed instead (fixed-Delta fallback) */
    double learned_ms;        /* sample batch under the trained network (best of two runs) */
    double fixed_ms;          /* sample batch under the fastest constant network tried (best of two) */
    /* label_mode 2 (counterfactual replays; see ppsp_mlp_fit) */
    double c_entry_ns;        /* fitted cost of a frontier entry (ns) */
    uint32_t variants;        /* replays run (pair x switch round x bin x frontier mode) */
    uint32_t heldout;         /* held-out pairs the referee timed */
    double heldout_learned_ms;    /* held-out batch under the trained network (best of two) */
    double heldout_fixed_ms;      /* held-out batch through the plain fixed-Delta path (best of two) */
    double heldout_learned_cost;  /* fitted cost (ms) of the held-out run's rounds, arcs and entries, learned */
    double heldout_fixed_cost;    /* the same for the base multiplier (bin 4) */
    uint32_t plain_fallback;  /* 1: the plain fixed path won the referee's comparison: PPSP_SCHED_LEARNED then runs it */
    uint32_t dense_labels;    /* label_mode 2: (pair, decision round) labels that chose a dense frontier */
} ppsp_fit_report;

int ppsp_mlp_forward(int device, const float *params, const float *x, uint32_t n, float *logits);
int ppsp_mlp_grad(int device, const float *params, const float *x, const uint32_t *y, uint32_t n, float *grad,
                  double *loss);
int ppsp_mlp_train(int device, float *params, const float *x, const uint32_t *y, uint32_t n, uint32_t epochs,
                   uint32_t batch, float lr, uint64_t seed, double *loss_first, double *loss_last);
int ppsp_mlp_load(ppsp_graph g, const float *params);
int ppsp_sched_trace(ppsp_graph g, const uint32_t *pairs, uint32_t k, const ppsp_opts *opts, const uint8_t *bins,
                     float *feat, uint32_t *row_pair, uint64_t cap, uint64_t *nrows, uint32_t *pair_rounds,
                     uint64_t *pair_arcs);
int ppsp_mlp_fit(ppsp_graph g, const uint32_t *pairs, uint32_t k, const ppsp_opts *opts, const float *init,
                 uint32_t epochs, uint64_t seed, uint32_t label_mode, float *params_out, ppsp_fit_report *rep);

/*
 * ppsp_sched_trace_ex: a traced Plain or Plain* batch (exact distances, like
 * any other schedule) with the step schedule given per pair:
 *   bins[k] (NULL: bin 4 = the base Delta) until the step for round
 *   switch_round[k], bins_after[k] from that step on (8..15: bin - 8 with the
 *   frontier switched to dense there; both NULL: no switch; the
 *   counterfactual replays behind the learned schedule's labels), or,
 *   with network = 1, the bins the loaded network picks (bins ignored; the
 *   rows then record its inputs and choices, for checking its inference).
 *   distinct = 1 keeps equal pairs apart (each pair its own query).
 * Outputs (caller-owned; NULL skips): cap feature rows feat [cap][12] with
 * row_pair, row_round (the round after which the step was chosen), row_side
 * (0: the pair's forward or only search, 1: its backward search), row_bin
 * (the bin chosen); nrows = rows produced (may exceed cap); per pair the
 * rounds its searches ran, the arcs they scanned, the entries they put in
 * their next frontiers (carried entries included) and the distance.
 * Errors: PPSP_E_INVALID (a bin >= 8, a bins_after entry >= 16, one of
 * switch_round / bins_after without the other, network = 1 with no network loaded, another strategy),
 * the errors of ppsp_batch_query.
 */
typedef struct {
    const uint8_t *bins;
    const uint8_t *bins_after;
    const uint32_t *switch_round;
    uint32_t network;
    uint32_t distinct;
    uint64_t cap;
    float *feat;
    uint32_t *row_pair;
    uint32_t *row_round;
    uint8_t *row_side;
    uint8_t *row_bin;
    uint64_t nrows;          /* out */
    uint32_t *pair_rounds;
    uint64_t *pair_arcs;
    uint64_t *pair_entries;
    uint64_t *dist;
} ppsp_trace_spec;

int ppsp_sched_trace_ex(ppsp_graph g, const uint32_t *pairs, uint32_t k, const ppsp_opts *opts,
                        ppsp_trace_spec *spec);

/*
 * Serving (continuous batching). A server owns one or more resident graphs
 * (all on one device) and a worker thread that keeps their round loops
 * running. Each graph gets a fixed pool of query slots (one forward and one
 * backward search each) sized from state_budget (bytes of search state,
 * shared in proportion to the graphs' vertex counts). Submitted queries wait
 * in FIFO order and are admitted into free slots between rounds, so requests
 * that arrive while others run join them on the device; results are the same
 * distances ppsp_batch_query returns. A graph attached to a server is
 * reserved: ppsp_query, ppsp_batch_query, ppsp_set_option and
 * ppsp_graph_destroy on it return PPSP_E_BUSY until ppsp_server_destroy.
 *   opts          one per graph: opts[i].algo is PPSP_BIDS or PPSP_BIDASTAR
 *                 (one query = two searches), opts[i].delta its Delta (0 = the
 *                 graph's default), opts[i].sched PPSP_SCHED_FIXED or
 *                 PPSP_SCHED_LEARNED (the network loaded on the graph picks
 *                 every search's step, as in ppsp_batch_query; the plain path
 *                 when the fit's referee chose it); other fields are ignored
 * ppsp_server_submit copies the pairs and returns a request id.
 * ppsp_server_poll returns PPSP_E_BUSY until every query of the request has
 * finished; then it copies the k distances (input order) and the latency
 * (submit to last result, ms) and forgets the request. ppsp_server_wait blocks
 * up to timeout_ms. When a frontier queue or the heavy list overflows, the
 * queries on the device start again with twice (four times) the capacity; a
 * graph's explicit "queue_cap" option is the queue's starting size. Errors:
 * PPSP_E_RANGE (vertex id), PPSP_E_INVALID (unknown request), PPSP_E_OOM
 * (buffers can grow no further; the server stops).
 */
typedef struct ppsp_server_s *ppsp_server;

typedef struct {
    uint64_t admitted;    /* queries admitted into slots */
    uint64_t completed;   /* requests completed */
    uint64_t chunks;      /* worker iterations (admit, rounds, collect) */
    uint64_t rounds;      /* rounds run, summed over graphs */
    uint64_t running;     /* queries on the device now */
    uint64_t slots;       /* query slots, summed over graphs */
    uint64_t pending;     /* requests with queries not yet admitted */
    uint64_t restarts;    /* frontier-buffer overflows: the queries on the device were restarted
                             with larger buffers (and count again in `admitted`) */
    uint64_t renumbers;   /* the round loop was renumbered from round 0 before its round stamps
                             reached the reserved values (about every 4.29e9 rounds); the queries
                             then on the device were restarted (and count again in `admitted`) */
} ppsp_server_counters;

int ppsp_server_create(const ppsp_graph *graphs, uint32_t ngraphs, const ppsp_opts *opts, uint64_t state_budget,
                       ppsp_server *out);
int ppsp_server_submit(ppsp_server srv, uint32_t graph_id, const uint32_t *pairs, uint32_t k, uint64_t *req_id);
int ppsp_server_poll(ppsp_server srv, uint64_t req_id, uint64_t *dist, double *latency_ms);
int ppsp_server_wait(ppsp_server srv, uint64_t req_id, uint64_t *dist, double *latency_ms, uint32_t timeout_ms);
int ppsp_server_stats(ppsp_server srv, ppsp_server_counters *out);
int ppsp_server_destroy(ppsp_server srv);

/* Counters of the last ppsp_query / ppsp_batch_query on g (see ppsp_stats). */
int ppsp_last_stats(ppsp_graph g, ppsp_stats *stats);

/*
 * Tuning knobs of a graph handle (not part of the method; they only change
 * launch shapes and bookkeeping):
 *   "profile"         K >= 1: time every K-th round-kernel launch (1: all), and the
 *                     hub-list kernel of the same rounds, with HIP events carried by the
 *                     launches themselves (hipExtLaunchKernel: no extra packets); 0: off
 *   "rounds_per_sync" rounds launched between host checks for termination
 *   "grid_blocks"     single-wave workgroups of the round kernel (0 = 20 per compute unit)
 *   "mem_budget_mb"   cap on the search-state memory of one wave (0 = auto)
 *   "default_delta"   Delta (distance units) used when opts.delta = 0 (0 = 2 x mean arc weight)
 *   "theta_mode"      0: Delta*-stepping, the threshold grows by Delta every round
 *                     (raised to the smallest frontier key when a step would be
 *                     empty); 1: the threshold is the end of the Delta-wide bucket
 *                     holding the smallest frontier key (Delta-stepping buckets);
 *                     2 (default): the smallest frontier key + Delta - 1;
 *                     3: infinite (every frontier entry is extracted each round: the
 *                     Bellman-Ford instance of the stepping framework)
 *   "use_graph"       1: replay rounds through a captured hipGraph
 *   "timeout_ms"      host-side limit on one wave's round loop (0 = none)
 *   "queue_cap"       frontier queue capacity in entries (grows x4, with a rerun of
 *                     the wave, whenever a round overflows it)
 *   "heavy_cap"       heavy-list capacity in arc chunks (grows the same way)
 *   "heavy_window"    vertices of degree > 512 are extracted only from the low 1/heavy_window
 *                     of the step window (smallest key + Delta/heavy_window), where their
 *                     distance is close to final, so their long arc lists are pushed fewer
 *                     times (default 64; 1 = the whole window)
 *   "multi_group"     Multi-BiDS state layout: this many consecutive query-graph vertices
 *                     keep their words of a vertex side by side (a power of two up to 64;
 *                     default 32; 1 = search-major)
 *   "plain_group"     bidirectional Plain* state layout: the words of a vertex for this many
 *                     searches (half as many queries) side by side (a power of two, 2 to 64;
 *                     default 2: one query's forward and backward copies)
 *   "list_deg"        extracted vertices of higher degree have their arcs relaxed by the
 *                     hub-list kernel, in chunks of at most 2,048 arcs shared by all waves (16 to
 *                     512; default 128; vertices above 512 also wait for the low end of the
 *                     step window, "heavy_window"); graphs without a vertex above 512 have no
 *                     hub list
 *   "heavy_claim"     hub-list records (chunks of at most 2,048 arcs) a wave of the hub-list
 *                     kernel claims at a time from a shared counter (1 to 64; default 4)
 *   "heavy_waves"     single-wave workgroups per CU of the hub-list kernel (1 to 32; default
 *                     24; 0: the round kernel's grid)
 *   "heavy_grouped"   1 (default): on a symmetric graph with vertices of degree > 512 and a
 *                     state layout of 4 or more searches per group ("plain_group",
 *                     "multi_group"), the hub-list kernel relaxes each chunk of a hub's
 *                     arcs once for all searches of a group that extracted it in the round
 *                     (arcs read once, the group's words of a head in shared lines); 0: one
 *                     pass per search
 *   "rho"             target next-frontier size per search of PPSP_SCHED_RHO (default 4096)
 *   "ml_every"        rounds between evaluations of the learned schedule's network (default 4;
 *                     a search keeps its multiplier in between)
 *   "local_chunks"    up to this many chunks of 64 entries per wave per round are taken
 *                     from the wave's own additions whose key is within the round's
 *                     threshold, in the same launch, for heuristic searches (A*, BiD-A*):
 *                     a frontier advances several hops per round (default 16; 0 = off)
 *   "local_chunks_plain" the same for the other searches (ET, SSSP, BiDS, Multi-BiDS;
 *                     default 0: measured neutral to slower there)
 *   "local_chunks_small" the budget instead in rounds whose frontier is small enough for
 *                     chunks below 64 entries (default 4: single queries; a long serial
 *                     chain per wave would set the round's length)
 *   "local_time_pct"  in rounds of full chunks a wave stops taking local chunks once it has run
 *                     this percentage of the previous round's mean wave time, and its listed
 *                     entries go to the next round, so one long chain does not hold the round
 *                     open (default 90; 0 = no limit)
 *   "defer_time_pct"  in rounds of full chunks a wave that has run this percentage of the
 *                     previous round's mean wave time hands its remaining queue chunks to the
 *                     next round unprocessed; its first chunk is always processed (default
 *                     105; 0 = never; otherwise at least 100)
 *   "min_chunk"       entries per chunk of the round kernel while the frontier is too small
 *                     to give every workgroup a 64-entry chunk: the smallest power of two
 *                     from min_chunk up that covers it (default 16; 64 = always 64)
 *   "local_fill"      local chunks only in rounds whose frontier holds fewer entries than
 *                     this (default 0 = every round)
 *   "dense_min"       dense frontiers (the dense mode of Appendix B): a search whose next
 *                     frontier reaches this many entries (sampled per-search counts) keeps
 *                     its frontier from then on as bitmaps of n bits, one per step bucket
 *                     (the bucket of Delta at the switch holding the smallest key, and
 *                     "dense_ring" buckets ahead; later entries stay in the queue), so that entries
 *                     waiting for a later bucket cost nothing per round; its threshold is
 *                     then the end of its current bucket. 0 (default) = off. Not with
 *                     PPSP_PULL; not in ppsp_batch_query_noalloc or the server. Results are
 *                     identical. Memory: (dense_ring + 1) * n / 8 bytes per search more.
 *   "dense_force"     1: every search switches to dense frontiers after its first round
 *   "dense_ring"      step buckets a dense frontier keeps ahead of its current one (a power
 *                     of two from 2 to 64, default 16)
 *   "dense_learned"   1: under PPSP_SCHED_LEARNED the network's mode output may switch a
 *                     search to dense frontiers (set by ppsp_mlp_fit label_mode 2; default 0)
 *   "server_round_base" the round number a server's round loop on this graph starts at
 *                     (default 0; below 0xFFFFFF00). A server renumbers its rounds from 0
 *                     before they reach 0xFFFFFF00, restarting the queries then running;
 *                     a high base exercises that without billions of rounds
 * Returns PPSP_E_INVALID for an unknown name.
 */
int ppsp_set_option(ppsp_graph g, const char *name, int64_t value);
int ppsp_get_option(ppsp_graph g, const char *name, int64_t *value);

/*
 * The query-graph vertex cover that PPSP_BATCH_VC runs on (Section 4.3 and
 * the adaptation to directed graphs): the k pairs (pairs[2q], pairs[2q+1])
 * are the edges of the query graph. Undirected (directed = 0): (s, t) and
 * (t, s) are one edge; the cover is an exact minimum in every connected
 * component of at most 16 vertices and greedy by uncovered degree in larger
 * ones. Directed: the query graph is bipartite (sources, targets) and the
 * cover is an exact minimum (Hopcroft-Karp matching and Koenig's theorem).
 * root[q] receives the endpoint whose single-source search answers pair q
 * and from_target[q] 1 when that endpoint is the pair's target (on a
 * directed graph: a backward search on the transpose). A pair with s = t
 * needs no search: root[q] = s, not counted. *cover_size receives the number
 * of searches (distinct roots, with their direction when directed). Host
 * function; caller-owned arrays of k entries. Errors: PPSP_E_INVALID.
 */
int ppsp_query_cover(const uint32_t *pairs, uint32_t k, uint32_t directed, uint32_t *root, uint8_t *from_target,
                     uint32_t *cover_size);

/*
 * The heuristic of Sections 3.3 and 3.5 on fixed-point coordinates,
 * computed exactly in integers: floor(w_scale * sqrt(dx^2 + dy^2) / 2^frac_bits)
 * with (dx, dy) = (x1 - x0, y1 - y0). Host function, for checking.
 * Requires w_scale^2 * (dx^2 + dy^2) < 2^63; returns UINT64_MAX otherwise.
 */
uint64_t ppsp_heuristic_fx(int32_t x0, int32_t y0, int32_t x1, int32_t y1, uint32_t w_scale,
                           uint32_t frac_bits);

/* Static description of a status code. */
const char *ppsp_status_str(int status);

/* Detail of the most recent PPSP_E_DEVICE / PPSP_E_OOM on this thread (the
 * failing HIP call and its error name), or "" . Valid until the next call. */
const char *ppsp_last_error(void);

/* Library version, e.g. "0.1.0". */
const char *ppsp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PPSP_H */
