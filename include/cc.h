/*
 * cc.h -- colourful subgraph counting for queries of treewidth <= 2 on one
 * MI355X (gfx950) GPU.
 *
 * The library computes, for a data graph G (n vertices, m undirected edges)
 * and a query Q with k nodes, the number of colourful matches of Q in G
 * under random colourings of G with k colours (Preliminaries: matches are
 * injective, edge-preserving maps V_Q -> V_G; a match is colourful when its
 * k images carry k distinct colours), and the colour-coding estimate of the
 * number of matches scaled to subgraph copies (Section 2: (k^k/k!) times the
 * mean colourful count is an unbiased estimate of n(G,Q); dividing by aut(Q)
 * turns matches into copies).
 *
 * The counts come from the degree-based dynamic program of Section 5: the
 * query is decomposed into leaf-edge and cycle blocks (Section 4.1), and each
 * cycle is solved by partitioning its colourful matches by the highest
 * matched vertex in the degree order (Eq. (1)) and joining high-starting
 * path tables (NodeJoin / EdgeJoin, Section 5.2).  All arithmetic is exact
 * unsigned integer arithmetic; overflow is detected, never wrapped.
 *
 * Conventions for every call:
 *   - Every call returns a cc_status; on error the outputs are left untouched
 *     unless stated otherwise, and cc_last_error() describes the failure.
 *   - The caller owns every buffer it passes.  Input arrays are copied before
 *     the call returns; outputs are written before it returns (all calls are
 *     synchronous with respect to the host, even when a stream is given).
 *   - Arrays documented "host" must be host memory.  `stream` is a
 *     hipStream_t (or NULL for the library's own stream); the device work of
 *     a call is ordered on that stream.
 *   - Handles are opaque, immutable after creation, and freed only by the
 *     matching *_destroy call.  A graph may be shared by concurrent calls on
 *     different streams; a cc_server is not thread-safe.
 *   - Vertex ids are int32 in [0, n); colours are uint8 in [0, k); counts are
 *     uint64.
 */
#ifndef CC_H
#define CC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CC_OK = 0,
  CC_E_ARG = 1,                /* a pointer is null, a size is negative or out of range */
  CC_E_GRAPH = 2,              /* malformed CSR: not symmetric, self-loop, duplicate edge, id out of range */
  CC_E_QUERY_TW = 3,           /* no decomposition into blocks: the query has treewidth > 2 (Lemma 4.1) */
  CC_E_QUERY_DISCONNECTED = 4, /* the query is not connected */
  CC_E_K_RANGE = 5,            /* k < 2 or k > 12 */
  CC_E_UNSUPPORTED = 6,        /* a plan the library cannot run (tables wider than one workgroup's row) */
  CC_E_NOMEM = 7,              /* the work does not fit the device memory budget */
  CC_E_DEVICE = 8,             /* a HIP runtime call failed */
  CC_E_BUSY = 9                /* a server's request table is full */
} cc_status;

typedef struct cc_graph_s *cc_graph;
typedef struct cc_query_s *cc_query;
typedef struct cc_server_s *cc_server;

/* An unsigned 128-bit integer, lo + 2^64 * hi. */
typedef struct {
  uint64_t lo, hi;
} cc_u128;

/* Tuning knobs; zero means "choose automatically". */
typedef struct {
  int32_t group_sources;   /* high-degree sources processed together per launch (<= 64) */
  int32_t trial_group;     /* colourings processed together */
  int32_t light_max_keys;  /* per-level key capacity of the one-workgroup-per-source path */
  int32_t use_graphs;      /* 1: capture the launch sequence of a solve in a hipGraph and replay it */
  int32_t dense_sources;   /* highest sources run as dense groups; -1: the library's cost-model cut */
} cc_tuning;

/* ------------------------------------------------------------------ graphs */

/* Flags for cc_graph_create. */
#define CC_GRAPH_CLEAN 1u         /* drop self-loops and duplicate edges instead of failing */
#define CC_GRAPH_REVERSE_TIES 2u  /* break degree ties by larger id first (the total is unchanged, Eq. (1)) */

/*
 * Make a data graph resident on the current device.
 *   n        number of vertices, 1 <= n < 2^31.
 *   row_ptr  host, int64[n+1], row_ptr[0] = 0, non-decreasing.
 *   col      host, int32[row_ptr[n]]: neighbours of v are col[row_ptr[v] .. row_ptr[v+1]).
 *            Every undirected edge {u,v} appears as v in u's row and u in v's row.
 * The library orders vertices by (degree, id) ascending (Section 5.1, degree
 * ordering), relabels them by that rank and sorts every neighbour list, so the
 * lower neighbours of a vertex form a prefix of its list.
 * Errors: CC_E_ARG, CC_E_GRAPH (see CC_GRAPH_CLEAN), CC_E_NOMEM, CC_E_DEVICE.
 */
cc_status cc_graph_create(int64_t n, const int64_t *row_ptr, const int32_t *col, uint32_t flags,
                          void *stream, cc_graph *out);
cc_status cc_graph_destroy(cc_graph g);
/* n, m (undirected edges) and the maximum degree of a resident graph. */
cc_status cc_graph_info(cc_graph g, int64_t *n, int64_t *m, int64_t *max_degree);

/* ------------------------------------------------------------------ queries */

/*
 * Plan a query: k nodes 0..k-1, num_edges undirected edges given as pairs in
 * `edges` (host, int32[2*num_edges]).  The query must be simple and connected
 * with 2 <= k <= 12.  The planner enumerates decomposition trees (Section 4.1,
 * Cases 1-3) and picks one by the heuristic of Section 6 (shortest longest
 * cycle, then fewest boundary nodes, then fewest annotations), preferring trees
 * whose two-boundary blocks have adjacent boundary nodes.  A block whose two
 * boundary nodes are not adjacent (Configuration (B) of Section 5.1: K_{2,3},
 * theta graphs, the worked example of Section 4.1) produces a table keyed by
 * pairs of vertices that need not be adjacent in the data graph; it is
 * computed by splitting its cycle at the two boundary nodes (the paper's
 * path-splitting procedure, Procedures 1-2 of Section 5.1) and stored as a
 * graph of its own over the nonzero pairs; a count whose pair table does not
 * fit the device memory fails with CC_E_NOMEM.
 * Errors: CC_E_ARG, CC_E_K_RANGE, CC_E_QUERY_DISCONNECTED, CC_E_QUERY_TW.
 */
cc_status cc_query_create(int32_t k, int32_t num_edges, const int32_t *edges, cc_query *out);

/* Flags for cc_query_create_ex. */
#define CC_QUERY_PATH_SPLITTING 1u /* the baseline: every cycle split at its boundary nodes, no degree order */

/*
 * cc_query_create with choices:
 *   flags  0: the degree-based procedure (Section 5.1, DB) for every block
 *          whose boundary nodes allow it; CC_QUERY_PATH_SPLITTING: the
 *          path-splitting baseline of Section 5.1 (PS, equivalent to the
 *          colour-coding procedure of Alon et al.) for every cycle block --
 *          the cycle is split at its boundary nodes (a root cycle at its first
 *          node and the node opposite), the two paths start at the first
 *          boundary node's image and take any vertex (no degree-order
 *          filter), and every match is counted once.  Same counts as DB.
 *   tree   -1: the heuristic's tree; else the index of a tree in the
 *          planner's enumeration (0 .. num_trees - 1, see cc_query_tree_info),
 *          e.g. to time every tree of a query (Section 8: the choice of tree).
 * Errors: as cc_query_create; CC_E_ARG for an unknown flag or tree index.
 */
cc_status cc_query_create_ex(int32_t k, int32_t num_edges, const int32_t *edges, uint32_t flags, int32_t tree,
                             cc_query *out);
/* The chosen tree's index, the number of distinct trees enumerated (at most
 * 4096 are kept), and the number of pair-keyed blocks in the chosen tree.
 * Any output may be NULL. */
cc_status cc_query_tree_info(cc_query q, int32_t *tree, int32_t *num_trees, int32_t *pair_keyed_blocks);
cc_status cc_query_destroy(cc_query q);
/* aut(Q) (Preliminaries), the number of blocks and the longest cycle of the chosen tree. */
cc_status cc_query_info(cc_query q, uint64_t *aut, int32_t *num_blocks, int32_t *longest_cycle);
/*
 * Describe the chosen decomposition tree as ints (host buffer `out`, capacity
 * `cap`): [nblocks, then per block: kind (0 leaf, 1 cycle, 2 root cycle,
 * 3 root singleton), size of its subquery, L, nodes[L], nboundary, boundary[],
 * nchildren, children[]].  *len receives the number of ints needed.
 */
cc_status cc_query_plan(cc_query q, int32_t *out, int32_t cap, int32_t *len);

/* Device bytes a count of `trials` colourings would use (tables and frontiers). */
cc_status cc_footprint(cc_graph g, cc_query q, int32_t trials, uint64_t *bytes);

/* ------------------------------------------------------------------ colourings */

/*
 * The colouring contract (the paper asks only for uniform random colours,
 * Preliminaries): for trial t, chi_t(v) = ((mix(mix(seed + t) ^ v) >> 32) * k) >> 32
 * where v is the caller's (original) vertex id and mix is the splitmix64
 * output function.  Computed on the device; `out` is host, uint8[n], indexed
 * by original vertex id.
 */
cc_status cc_colors(cc_graph g, int32_t k, uint64_t seed, int32_t trial, uint8_t *out);

/* ------------------------------------------------------------------ counting */

/*
 * Count colourful matches of q in g for `trials` colourings drawn by the
 * contract above from `seed` (trial t uses seed + t): the colour-coding count
 * of Section 2, computed over the decomposition tree (Sections 4.1-4.3) with
 * the degree-based cycle solution (Section 5.1, Eq. (1)), and its estimate.
 *   counts    host, uint64[trials]: exact counts; UINT64_MAX when overflow[t] = 1.
 *   overflow  host, uint8[trials]: 1 if the count is >= 2^64 or a table entry
 *             left 64 bits during the computation (sticky per trial).
 *   exact     host, cc_u128[trials] or NULL: the exact count whenever no table
 *             entry overflowed (also when only the final sum exceeds 2^64);
 *             {UINT64_MAX, UINT64_MAX} otherwise.
 *   estimate  host, double or NULL: (sum_t N_t) * k^k / (trials * k! * aut(q)),
 *             from the exact sums, rounded once to double; NaN if any trial
 *             overflowed.
 * Errors: CC_E_ARG, CC_E_NOMEM, CC_E_DEVICE.
 */
cc_status cc_count(cc_graph g, cc_query q, uint64_t seed, int32_t trials, uint64_t *counts,
                   uint8_t *overflow, cc_u128 *exact, double *estimate, void *stream);

/*
 * As cc_count (Section 2, Sections 4.1-5.2), with the colourings given:
 * `colors` is host, uint8[trials*n],
 * trial-major, indexed by original vertex id, values in [0, k).
 * `per_source` (host, cc_u128[trials*n] or NULL) receives, for a query whose
 * root block is a cycle, the count of colourful matches whose highest root
 * cycle vertex (in the degree order) is each vertex, indexed by original id;
 * for a singleton root, each vertex's share of the root sum.
 * Errors: as cc_count, plus CC_E_ARG for a colour >= k.
 */
cc_status cc_count_colors(cc_graph g, cc_query q, int32_t trials, const uint8_t *colors,
                          uint64_t *counts, uint8_t *overflow, cc_u128 *exact, cc_u128 *per_source,
                          void *stream);

/*
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, results and errors as cc_count, but the call allocates nothing
 * on the device (no hipMalloc / hipFree, no stream or event creation): every
 * device buffer of the solve is carved from a static scratch of
 * CC_STATIC_SCRATCH_BYTES per device, held by the library from its first use
 * on that device until the process ends.  Solves whose buffers do not fit
 * fail with CC_E_NOMEM (before any device work).  Calls on one device share
 * its scratch, so the library runs them one at a time (a call waits for the
 * previous one on that device); overlapping calls from other threads are
 * serialised, never interleaved.  Every buffer is cleared or written by the
 * solve before it is read, so the scratch's earlier contents do not matter.
 * The sources with small reach run in the grouped path (the one-workgroup
 * tier's scratch would not fit), and profiling is ignored.  `stream` NULL:
 * the null stream.  The device tables of the kernels (colex and slot maps)
 * live in static device memory as well.
 */
#define CC_STATIC_SCRATCH_BYTES (256ull << 20)
cc_status cc_count_static(cc_graph g, cc_query q, uint64_t seed, int32_t trials, uint64_t *counts,
                          uint8_t *overflow, cc_u128 *exact, double *estimate, void *stream);

/*
 * Batched form: nq queries on one graph, query i with trials[i] colourings
 * from seeds[i] (trial t of query i uses the colouring (seeds[i], t) of the
 * contract, so the counts equal cc_count's).  The trials are the independent
 * colourings whose counts the estimate averages (Section 2; the number of
 * trials sets its precision, Section 8).  The colourings of a query are
 * solved in trial groups that form the batch dimension of every launch; the
 * launch sequence of a trial group is captured once in a hipGraph and
 * replayed for the next groups (use_graphs).  With several queries, up to
 * four run side by side, each on a stream of the library's with a quarter of
 * the free device memory (the call first waits for `stream`).
 *   counts / overflow  host, concatenated per query in order (sum of trials[i]).
 *   estimates          host, double[nq] or NULL.
 *   tuning             NULL: the trial-group size is tuned online on the
 *                      query's first trials (see cc_last_tune_report) and
 *                      graphs are used; else the given choices.
 * Errors: as cc_count.
 */
cc_status cc_count_batch(cc_graph g, int32_t nq, const cc_query *qs, const uint64_t *seeds,
                         const int32_t *trials, uint64_t *counts, uint8_t *overflow, double *estimates,
                         const cc_tuning *tuning, void *stream);

/*
 * What the calling thread's last cc_count_batch chose for its last query
 * (online tuning when `tuning` was NULL): first the decomposition tree, when
 * the query has several and at least 32 colourings are asked for (up to four
 * trees, the heuristic's first, each timed on colourings of the call, the
 * fastest kept; Section 8 reports trees of one query differing by up to an
 * order of magnitude), then the dense cut (the model's, half and double, one
 * colouring per group) and the trial-group size (not tried when one
 * colouring takes 0.25 s or more), the candidates timed and their seconds per
 * colouring, and the graph replays.
 */
typedef struct {
  int32_t trial_group;
  int32_t candidates;
  int32_t tried_trial_group[8];
  double tried_seconds_per_colouring[8];
  uint64_t graph_replays;
  int32_t dense_sources;         /* chosen dense cut (sources run as dense groups) */
  int32_t tried_dense_sources[8];
  int32_t tree;                  /* chosen decomposition tree (index as in cc_query_create_ex) */
  int32_t trees_tried;           /* trees timed (0: the query's own tree only) */
  int32_t tried_tree[8];
  double tried_tree_seconds[8];  /* seconds per colouring of each tree timed */
} cc_tune_report;
cc_status cc_last_tune_report(cc_tune_report *out);

/*
 * How the calling thread's last counting call (cc_count, cc_count_colors,
 * cc_count_static, or the last query of cc_count_batch) split the sources of
 * the root block -- the vertices that can be the highest vertex of a cycle
 * match (at least two lower neighbours, Section 5.1) -- over the execution
 * tiers: dense groups (the sources with the widest reach, a row for every
 * lower vertex), the one-workgroup-per-source tier, and the sources that tier
 * handed back to grouped launches (their frontier did not fit).  Also the
 * colourings per trial group and the sources per group.
 */
typedef struct {
  int64_t sources;
  int64_t dense_sources;
  int64_t light_sources;
  int64_t handed_back;
  int32_t trial_group;
  int32_t group_sources;
} cc_solve_stats;
cc_status cc_last_solve_stats(cc_solve_stats *out);

/* ------------------------------------------------------------------ serving */

/*
 * A request loop over resident graphs.  Requests (graph, query, seed, trials)
 * are admitted while their device footprint fits the budget and fewer than
 * `max_inflight` are running; admitted requests run concurrently on a pool of
 * streams (continuous batching: a request arriving while others run starts as
 * soon as a stream slot and memory are free).  Requests start in arrival
 * order, but while the oldest waiting one does not fit, later ones that fit
 * may start ahead of it (at most 8 per waiting request, so none waits without
 * bound).  A request whose footprint
 * exceeds the budget runs alone within the budget (smaller trial and source
 * groups).  Results are identical to cc_count on the same arguments.
 */
cc_status cc_server_create(uint64_t hbm_budget_bytes, int32_t max_inflight, cc_server *out);
/* Register a resident graph; the server does not take ownership. */
cc_status cc_server_add_graph(cc_server s, cc_graph g, int32_t *graph_id);
/* Enqueue a request; the query must outlive it.  CC_E_BUSY if the request table is full. */
cc_status cc_server_submit(cc_server s, int32_t graph_id, cc_query q, uint64_t seed, int32_t trials,
                           uint64_t *ticket);
/*
 * Poll a ticket: *done = 1 when finished, then counts/overflow (host,
 * [trials]) and *estimate are filled and *latency_s is completion minus
 * submission time.  Any output pointer may be NULL.  A finished ticket is
 * released by the poll that reports it.
 */
cc_status cc_server_poll(cc_server s, uint64_t ticket, int32_t *done, uint64_t *counts, uint8_t *overflow,
                         double *estimate, double *latency_s);
/* Block until every submitted request has finished. */
cc_status cc_server_drain(cc_server s);
cc_status cc_server_destroy(cc_server s);

/* ------------------------------------------------------------------ profiling */

/*
 * Per-kernel timing, for measurement only.  Level 1: every kernel launch of
 * cc_count* (eager runs; graph replays are not split) is bracketed by HIP
 * events on the call's stream and the elapsed times are summed per operation.
 * Level 2: in addition the kernels count the algorithmic bytes they move
 * (Section 5 procedures, the bytes the method itself must read and write):
 *   EdgeJoin  4 B per (key, trial, lower neighbour) triple scanned -- a key
 *             being an input row of a source at a neighbour below that source
 *             -- plus 8 B per slot of every input row relaxed (and of the
 *             annotating edge's row) plus 8 B per slot of every output row
 *             actually written (live rows only);
 *   NodeJoin, AXPY chains, path init, root merge, level builds: the bytes of
 *             the rows they read and write (8 B per slot, 8-16 B per vertex
 *             word), counted by the kernels themselves;
 *   leaf join: computed on the host from the CSR and the table sizes;
 *   one-workgroup-per-source tier: the same per-operation bytes for the rows
 *             it keeps in its scratch, plus 4 B per neighbour scanned while
 *             it builds its key lists.
 * The merges into non-root tables report no bytes.  The counters slow the kernels down: time with level 1.
 * Level 3: events around the EdgeJoin launches only (the least timing overhead
 * for the dominant kernel's launch durations).  Level 0 turns all off.
 */
typedef struct {
  char name[32];
  uint64_t launches;
  double seconds;  /* summed event-measured duration */
  double bytes;    /* algorithmic bytes (level 2; see above) */
  uint64_t work[3]; /* EdgeJoin: (key, trial, lower neighbour) triples scanned, input rows relaxed,
                       output rows written; other kernels: bytes read, bytes written, 0 */
} cc_kernel_stat;

cc_status cc_profile_enable(int32_t level);

/*
 * A plain streaming copy between two device buffers of `bytes` (a multiple
 * of 16) that the library allocates, repeated `reps` times on a stream of its
 * own; *gbps = 2 * bytes * reps / elapsed (bytes read + written per second).
 * A kernel of known traffic: it calibrates hardware byte counters, and its
 * rate is the bandwidth a streaming kernel reaches on this device.
 */
cc_status cc_probe_copy(uint64_t bytes, int32_t reps, double *gbps);
/* Copy up to `cap` entries into `out` (host), set *len to the number of
 * kernels recorded, and reset the statistics. */
cc_status cc_profile_read(cc_kernel_stat *out, int32_t cap, int32_t *len);

/* ------------------------------------------------------------------ errors */

const char *cc_status_str(cc_status st);
/* Text of the last error raised on the calling thread ("" if none). */
const char *cc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CC_H */
