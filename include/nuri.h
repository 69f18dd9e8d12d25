/*
 * nuri.h -- C ABI of the MI355X top-k subgraph discovery engine.
 *
 * The engine runs the paper's basic computational model (Algorithm 1,
 * Section 3.2: prioritized expansion of partial subgraphs with pruning
 * against the k-th result) on one AMD Instinct MI355X (gfx950), for
 *   - top-k maximal cliques (Section 3.2 "Example: Maximum Clique
 *     Discovery", Section 4.1, Listing 1), scored by size or by the sum
 *     of vertex weights, and
 *   - top-k labelled subgraph matching (Section 2.1 "Subgraph
 *     Isomorphism", Section 4.3), scored by the sum of matched edge
 *     weights or by the sum of the degrees of the matched vertices, and
 *   - top-k frequent pattern mining (Section 2.1 "Pattern Mining"), by the
 *     aggregate computation of Section 3.3 (Algorithm 2) with
 *     pattern-oriented expansion and minimum image-based support.
 * The user functions of Table 1 are fixed specialisations selected by the
 * arguments below; no user code runs on the device.
 *
 * Conventions for every entry point:
 *   - Return value: NURI_OK (0) on success, a negative nuri_status on
 *     error.  On error, out-parameters are left untouched and
 *     nuri_last_error() returns a message (thread-local, valid until the
 *     next call on the same thread).
 *   - Host pointers passed in are owned by the caller, read during the
 *     call only, and never retained.
 *   - Handles (nuri_graph, nuri_result, nuri_server) are owned by the
 *     library and released by the matching free/destroy call.
 *   - A graph is immutable after load; several queries may run on one
 *     graph from different threads.  A single query call is synchronous:
 *     it returns when its results are on the host.
 *   - The library fails loudly: it never returns a truncated or inexact
 *     top-k as success.
 */
#ifndef NURI_H
#define NURI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NURI_OK = 0,
  NURI_EINVAL = -1,   /* malformed argument (graph, pattern, k = 0, ...) */
  NURI_ENOMEM = -2,   /* device or host allocation failed */
  NURI_EBUDGET = -3,  /* the frontier does not fit the frontier budget */
  NURI_EDEVICE = -4,  /* a HIP call failed; the message names it */
  NURI_ETIMEOUT = -5  /* the query passed its deadline */
} nuri_status;

typedef struct nuri_graph nuri_graph;
typedef struct nuri_result nuri_result;
typedef struct nuri_server nuri_server;

/*
 * An undirected simple data graph in CSR form (Section 2.1; the engine
 * loads it once and keeps it resident, Section 5).  All arrays are host
 * memory.
 *   n        vertices 0..n-1 (n >= 1)
 *   nnz      directed entries = 2 * |E|
 *   row_ptr  [n+1], row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz
 *   col_idx  [nnz]; each row strictly increasing, no self loops, ids < n,
 *            and symmetric (v in row u iff u in row v)
 *   vertex_weight [n] or NULL; every weight >= 1 (needed by
 *            NURI_SCORE_VERTEX_WEIGHT)
 *   vertex_label  [n] or NULL; labels < NURI_MAX_LABELS (needed by
 *            matching)
 *   edge_weight   [nnz] or NULL, aligned with col_idx, equal for both
 *            directions of an edge, each in [1, 2^31); NULL means weight 1
 * Anything else is rejected with NURI_EINVAL; the input is never repaired.
 */
#define NURI_MAX_LABELS 16
typedef struct {
  uint32_t n;
  uint64_t nnz;
  const uint64_t *row_ptr;
  const uint32_t *col_idx;
  const int32_t *vertex_weight;
  const uint8_t *vertex_label;
  const int32_t *edge_weight;
} nuri_csr;

/*
 * Validates the CSR, copies it to the device and builds the resident
 * structures every query uses: a degeneracy order and the graph relabelled
 * by it, the oriented adjacency N+(v) (later neighbours), one dense local
 * adjacency bitmap per vertex over N+(v), root orders by bound, for each
 * vertex the earlier neighbours with at least 32 later neighbours (the
 * only vertices that can extend a clique of 32 or more members, used by
 * the maximality check of large results), and the per-(vertex, label)
 * maximum edge weight table (the 1-hop form of the Section 4.3 index,
 * Listing 3).  `hip_stream` is a hipStream_t or NULL
 * (the library's own stream); all later work on this graph runs on it.
 * Limit: the degeneracy must be at most 4096 (NURI_EINVAL otherwise).
 */
int nuri_load_graph(const nuri_csr *csr, void *hip_stream, nuri_graph **out);
void nuri_free_graph(nuri_graph *g);

typedef struct {
  uint32_t n;
  uint64_t nnz;
  uint32_t degeneracy;        /* max |N+(v)| under the degeneracy order */
  uint64_t bitmap_bytes;      /* bytes of all local adjacency bitmaps */
  uint64_t device_bytes;      /* device memory held by the graph */
  uint64_t preprocess_ns;     /* wall time of nuri_load_graph */
  double core_density;        /* edge density inside the largest out-neighbourhoods;
                                 near 1 means a near-clique, where the automatic
                                 clique bound keeps to |V| + |P| */
} nuri_graph_info;
int nuri_graph_get_info(const nuri_graph *g, nuri_graph_info *info);

/*
 * The multi-hop (label, hop) max-degree index of Section 4.3 (Listing 3),
 * the index behind NURI_MATCH_DEGREE: builds it on the device up to `hops`
 * hops if it is not there yet (it stays with the graph), then, unless out
 * is NULL, copies it to out (host, caller-owned, int32 [hops][n][16]):
 *   out[(h-1)*n*16 + v*16 + l] = the largest degree of a vertex of label l
 *   at distance 1..h from v (cumulative over hops), 0 when there is none.
 * 1 <= hops <= NURI_MAX_PATTERN - 1; the graph must have vertex labels.
 * build_ns (may be NULL) receives the build time of this call (0 when the
 * hops were already there).
 */
int nuri_graph_hop_index(nuri_graph *g, uint32_t hops, int32_t *out, uint64_t *build_ns);

/* Clique score (relevant results are maximal cliques, ranked by score). */
typedef enum {
  NURI_SCORE_SIZE = 0,          /* |C| */
  NURI_SCORE_VERTEX_WEIGHT = 1  /* sum of vertex weights, int64 */
} nuri_weight_fn;

/*
 * Match score (Section 4.3).
 *   EDGE_WEIGHT  sum over the pattern edges of the data edge weight (1 when
 *                the graph has none); bounded with one-hop tables: the
 *                largest edge weight from a vertex to a label, and over
 *                each label pair
 *   DEGREE       sum of the degrees of the matched data vertices (the
 *                paper's example); bounded with the multi-hop index: for
 *                every unmatched pattern vertex u, the largest degree of a
 *                vertex with u's label within hop(u) hops of the seed (the
 *                data vertex of the first pattern vertex matched), hop(u)
 *                being u's distance from that pattern vertex.  The index is
 *                built on the device the first time a query needs it (up
 *                to the hops that query needs) and stays with the graph.
 */
typedef enum {
  NURI_MATCH_EDGE_WEIGHT = 0,
  NURI_MATCH_DEGREE = 1
} nuri_match_score;

/*
 * A connected labelled query pattern (Section 2.1): q vertices 0..q-1 with
 * label[q] and n_edges undirected edges edges[2*i], edges[2*i+1]
 * (distinct, a != b, a, b < q).  2 <= q <= NURI_MAX_PATTERN.  score is a
 * nuri_match_score (0 = edge weights).
 */
#define NURI_MAX_PATTERN 8
typedef struct {
  uint32_t q, n_edges;
  const uint8_t *label;
  const uint32_t *edges;
  uint32_t score;
} nuri_pattern;

/*
 * Tuning and limits; pass NULL for defaults.  None of these changes a
 * result, only speed, memory and whether the call may fail.
 *   frontier_budget_bytes  device bytes for the frontiers of partial
 *                          subgraphs of all live queries (0 = 40% of the
 *                          free device memory, at most 64 GiB); a batch
 *                          runs only as many queries at once as have an
 *                          arena of a useful size (64 KiB or more, and
 *                          room for the children of any one record) and
 *                          starts the others as those finish; the step
 *                          buffers (selected records, leaves, candidates)
 *                          come on top.  NURI_EBUDGET if a search cannot
 *                          proceed within its arena
 *   batch_B                records expanded per step (0 = automatic)
 *   root_batch             unit subgraphs expanded per step (0 = automatic)
 *   bound                  clique bound used to skip children before they
 *                          are built: 0 automatic (colour classes of P
 *                          unless the densest part of the graph is a
 *                          near-clique, where they cannot beat |P|),
 *                          1 Carraghan-Pardalos (|V| + |P|, or the weight
 *                          analogue) only, 2 colour classes of P always
 *   deadline_ns            wall-clock limit per call (0 = none)
 *   profile                1: time every expansion launch with HIP events
 *                          (reported in nuri_stats)
 *   hip_stream             hipStream_t to run on (NULL = the graph's stream)
 *   priority               order in which partial subgraphs are expanded
 *                          (priority() of Table 1); one of NURI_PRIORITY_*.
 *                          Results never depend on it, only the work does.
 *   chain_links            cliques: when an expanded record keeps a single
 *                          child, the same wavefront expands that child at
 *                          once, up to this many links per launch (0 = 32)
 */
typedef struct {
  uint64_t frontier_budget_bytes;
  uint32_t batch_B;
  uint32_t root_batch;
  uint32_t bound;
  uint64_t deadline_ns;
  uint32_t profile;
  void *hip_stream;
  uint32_t priority;
  uint32_t chain_links;
} nuri_opts;

/*
 * Expansion orders (Section 3.2, prioritized expansion; Section 6.1).  A
 * step expands a batch of records, so each order is followed batch by
 * batch: within a step every record taken ranks at least as high as every
 * record left behind of the same level.
 *   DEPTH  (default) the partial subgraphs with the most vertices first,
 *          highest bound first among them: the paper's (|V|, |P|) for
 *          clique sizes and (matched edges, bound) for matching
 *   BOUND  highest bound first, whatever the size (best-first)
 *   PAPER  the paper's clique priority (|V|, |P|) also for vertex weights
 *          (most vertices first, then the largest candidate set); for
 *          matching the same as DEPTH
 *   NONE   no prioritization and no pruning, as the paper's Nuri-NP
 *          variant: only targeted expansion, so every maximal clique (every
 *          match) is reached and the result set keeps the k best
 */
enum {
  NURI_PRIORITY_DEPTH = 0,
  NURI_PRIORITY_BOUND = 1,
  NURI_PRIORITY_PAPER = 2,
  NURI_PRIORITY_NONE = 3
};

/*
 * Top-k maximal cliques (Algorithm 1 with the clique user functions of
 * Section 4.1: targeted expansion by the ordered candidate set, priority
 * (|V|, bound), dominated when bound < score of the k-th result).
 * Results are the first min(k, #maximal cliques) maximal cliques ordered
 * by score descending, then by the ascending list of their vertex ids
 * compared lexicographically.  k >= 1.
 */
int nuri_topk_cliques(nuri_graph *g, uint32_t k, nuri_weight_fn wf, const nuri_opts *o,
                      nuri_result **out);

/*
 * Top-k matches of a labelled pattern (Section 4.3): injective,
 * label-preserving maps mu with every pattern edge mapped onto a data edge
 * (non-induced).  Embeddings with the same image are one result,
 * represented by the lexicographically smallest (mu(0), ..., mu(q-1)).
 * Score (int64) as p->score selects (nuri_match_score).  Order:
 * score descending, then the representative tuple ascending.  Needs
 * vertex labels.  k >= 1.
 */
int nuri_topk_match(nuri_graph *g, const nuri_pattern *p, uint32_t k, const nuri_opts *o,
                    nuri_result **out);

/*
 * Top-k frequent patterns (Section 2.1 "Pattern Mining"; Section 3.3,
 * Algorithm 2, with pattern-oriented expansion; Section 4.2, Listing 2):
 * the k connected vertex-labelled patterns with exactly n_edges edges
 * (1..8) of highest minimum image-based support -- for a pattern, the
 * smallest number of distinct data vertices any one of its vertices is
 * mapped to over all its embeddings (injective, label-preserving maps that
 * send every pattern edge to a data edge).  Needs vertex labels.  k >= 1.
 * Results, best first: score = support; ids = the pattern's minimum DFS
 * code, 4 values per edge (i, j, label of i, label of j) over DFS discovery
 * ids (forward edge when i < j, backward when i > j).  Ties on support are
 * ranked by code: code edges compare backward-before-forward, backward
 * edges by j, forward edges by the larger i first and then by labels.
 * nuri_opts.frontier_budget_bytes bounds the device bytes of the
 * embeddings held at once (NURI_EBUDGET beyond it); priority and the step
 * sizes do not apply.
 */
int nuri_topk_patterns(nuri_graph *g, uint32_t n_edges, uint32_t k, const nuri_opts *o,
                       nuri_result **out);

/* One query of a batch. kind 0 = clique (uses k, wf), 1 = match (uses k, p). */
typedef struct {
  uint32_t kind;
  uint32_t k;
  nuri_weight_fn wf;
  const nuri_pattern *p;
} nuri_query;

/*
 * Runs nq queries together: every expansion launch serves all live
 * queries, each with its own frontier, threshold and result set.  outs
 * [nq] receives one result per query; each equals what the single-query
 * call returns.  On error no result is returned.
 */
int nuri_topk_batch(nuri_graph *g, const nuri_query *qs, uint32_t nq, const nuri_opts *o,
                    nuri_result **outs);

/*
 * Step-size autotuner for a workload (the batch size B and the root batch
 * of every step change how the frontier is cut into launches, never the
 * result).  Runs the queries qs[nq] as one batch once to warm up, then
 * `rounds` times (rounds >= 1) for each candidate pair (batch_B in {4096,
 * 16384, 32768, 65536}) x (root_batch in {2048, 8192}), with the other options
 * of *o (NULL = defaults), and writes into *best those options with the
 * pair of the smallest wall time.  Results are computed and discarded.
 * Errors: as nuri_topk_batch; *best is untouched on error.
 */
int nuri_autotune(nuri_graph *g, const nuri_query *qs, uint32_t nq, const nuri_opts *o,
                  uint32_t rounds, nuri_opts *best);

/*
 * Read-only view of a result, valid until nuri_free_result.
 *   count   min(k, number of results)
 *   score   [count], non-increasing
 *   offset  [count+1] into ids
 *   ids     clique i: its vertex ids ascending at ids[offset[i]..offset[i+1]);
 *           match i: mu(0), ..., mu(q-1)
 */
typedef struct {
  uint32_t count;
  const int64_t *score;
  const uint64_t *offset;
  const uint32_t *ids;
} nuri_result_view;
int nuri_result_view_get(const nuri_result *r, nuri_result_view *v);

/* Work counters of one query (R10: children created = candidate subgraphs). */
typedef struct {
  uint64_t steps;              /* expansion steps (launch rounds) */
  uint64_t popped;             /* records taken from the frontier */
  uint64_t expanded;           /* records expanded (not pruned at pop) */
  uint64_t children;           /* children created (candidate subgraphs) */
  uint64_t pruned_at_pop;      /* records dropped when taken (bound < k-th) */
  uint64_t pruned_at_creation; /* children dropped when created */
  uint64_t leaves;             /* children with nothing left to add */
  uint64_t offered;            /* results offered to the result set */
  uint64_t frontier_peak_bytes;
  uint64_t logical_bytes;      /* algorithmic bytes of the frontier read + written by
                                  expansion: records taken and written, leaves (and,
                                  for matching, the graph's candidate lists) */
  uint64_t expand_launches;    /* expansion kernel launches */
  uint64_t expand_ns;          /* summed expansion kernel time (profile = 1) */
  uint64_t wall_ns;            /* wall time of the call */
  uint64_t ties_at_k;          /* results returned whose score equals the k-th's (0 when
                                  fewer than k); Algorithm 1 would keep every further
                                  result tied with the k-th too, this engine returns k */
  uint64_t restarts;           /* served queries: times the query outgrew its frontier
                                  arena and was started again with a larger one */
  uint64_t onchip_bytes;       /* cliques: local adjacency rows read by expansion (a
                                  working set that stays in the L2 caches), kept apart
                                  from logical_bytes */
  uint64_t spilled_bytes;      /* frontier bytes moved to host memory when the
                                  query's arena filled up (the bottom levels of its
                                  stack, brought back when the levels above are done) */
  uint64_t index_ns;           /* matching, degree score: time this query spent building
                                  the graph's multi-hop index (0 when it was there);
                                  not part of wall_ns */
} nuri_stats;
int nuri_result_stats(const nuri_result *r, nuri_stats *s);
void nuri_free_result(nuri_result *r);

/*
 * Allocation-free variant of nuri_topk_cliques, for callers that cannot
 * allocate device memory: code under HIP stream capture, tight serving
 * loops, harnesses that forbid hipMalloc.  Same query and the same result
 * as nuri_topk_cliques(g, k, wf, o), but the call allocates no device or
 * page-locked host memory: every device buffer is carved from one static
 * device array of NURI_NOALLOC_SCRATCH_BYTES that each GPU holds from the
 * library's load until the process ends.  Outputs go to caller-owned host
 * arrays:
 *   score_out  [k]               scores, best first
 *   len_out    [k]               number of vertices of each clique
 *   ids_out    [k * ids_stride]  clique i's ascending vertex ids at
 *                                ids_out[i * ids_stride ...]
 *   ids_stride                   >= the graph's degeneracy + 1 (the largest
 *                                possible clique)
 *   count_out                    number of results written (min(k, #results))
 *   stats_out                    work counters, or NULL
 * Options as nuri_topk_cliques, except that profile is ignored and the
 * frontier gets what the array has left after the other buffers (the
 * frontier_budget_bytes option is not used).  Errors: NURI_EINVAL for k = 0,
 * k > NURI_NOALLOC_MAX_K, a short ids_stride, or a graph whose fixed
 * buffers (candidate ids and top-k, which grow with k and the degeneracy)
 * leave less than 4 MiB of the array for the frontier; NURI_EBUDGET when
 * the search needs more frontier than the array holds.  Calls on one GPU
 * share its array and are serialised inside the process; calls from several
 * processes on one GPU race.
 */
#define NURI_NOALLOC_SCRATCH_BYTES (128ull << 20)
#define NURI_NOALLOC_MAX_K 1000u
int nuri_topk_cliques_noalloc(nuri_graph *g, uint32_t k, nuri_weight_fn wf, const nuri_opts *o,
                              int64_t *score_out, uint32_t *len_out, uint32_t *ids_out,
                              uint32_t ids_stride, uint32_t *count_out, nuri_stats *stats_out);

/*
 * Continuous-batching server on one resident graph.  Queries submitted
 * while others run are admitted, in arrival order, when a slot of their
 * kind is free and their frontier arena fits in what the budget has left
 * (a query waiting for memory is not overtaken); admitted queries share
 * every expansion launch.  A query starts with frontier_budget_bytes / (2 *
 * max_slots) bytes of arena (at least what one record's children need); one
 * that outgrows it is restarted with twice the arena, up to the whole
 * budget, and only then fails with NURI_EBUDGET.
 *   frontier_budget_bytes  total device bytes for all live frontiers
 *                          (0 = the default of nuri_opts)
 *   max_slots              queries of each kind live at once
 * nuri_server_submit copies the query and returns a ticket at once
 * (NURI_EINVAL for a malformed query, or a matching query on a graph
 * without vertex labels).
 * nuri_server_poll returns 1 and the result when done (the result then
 * belongs to the caller), 0 while pending, < 0 on error: the query's own
 * error, or NURI_EINVAL for a ticket never issued or already collected.
 * nuri_server_destroy waits for nothing: pending queries are dropped.
 */
int nuri_server_create(nuri_graph *g, uint64_t frontier_budget_bytes, uint32_t max_slots,
                       nuri_server **out);
int nuri_server_submit(nuri_server *s, const nuri_query *q, uint64_t *ticket);
int nuri_server_poll(nuri_server *s, uint64_t ticket, nuri_result **out);
void nuri_server_destroy(nuri_server *s);

const char *nuri_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* NURI_H */
