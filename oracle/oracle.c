/*
 * CPU oracle for top-k subgraph discovery (test infrastructure only).
 *
 * This is a plain, slow, deliberately unoptimised rendering of the paper's
 * basic computational model (Algorithm 1, Section 3.2) for two
 * computations:
 *
 *   - top-k maximal cliques (Section 3.2 "Example: Maximum Clique
 *     Discovery", Section 4.1, Listing 1), and
 *   - top-k labelled subgraph matching (Section 2.1 "Subgraph Isomorphism",
 *     Section 4.3), scored by the sum of matched edge weights, or by the
 *     sum of the degrees of the matched vertices with the multi-hop
 *     (label, hop) max-degree index of Section 4.3 (Listing 3), and
 *   - top-k frequent pattern mining (Section 2.1 "Pattern Mining",
 *     Section 3.3 Algorithm 2 with pattern-oriented expansion, Listing 2):
 *     by its definition on tiny graphs, and by Algorithm 2.
 *
 * It exists to check the GPU engine.  It shares no code with it: no
 * headers, helpers or tables.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it.
 *
 * Readings of the paper this file takes (each is also listed with the
 * design notes):
 *   - A clique result is a *maximal* clique (relevant(s) is true only when
 *     nothing can extend s).  Its score is |V| or the int64 sum of vertex
 *     weights.
 *   - The result set holds exactly min(k, #results) entries ranked by
 *     score descending, then by the ascending-sorted original ids
 *     compared lexicographically (ascending).  The queue priority only
 *     orders exploration.
 *   - Candidate sets are ordered: P_s holds only vertices later than every
 *     member of s in a fixed total order pi (the duplicate-free generation
 *     of Section 3.2).  X_s holds the earlier common neighbours, so that
 *     maximality can be decided when P_s is empty.
 *   - dominated(s, kth) is strict: bound(s) < score(kth) (Section 3.2
 *     footnote on Carraghan-Pardalos; Section 4.1).
 *   - Matching is non-induced (a monomorphism); two embeddings with the
 *     same image are one result, represented by the lexicographically
 *     smallest tuple (mu(0), ..., mu(q-1)) in its automorphism orbit.
 *   - The multi-hop index entry for hop h covers every vertex at distance
 *     1..h (not exactly h): the image of a pattern vertex h hops from the
 *     seed's pattern vertex can lie closer to the seed than h, so only the
 *     cumulative entry bounds it.  The seed itself (distance 0) is never
 *     counted.  Degree = number of neighbours in the data graph.
 *
 * All arithmetic is integer.  parity pins: see tests/test_oracle_*.py.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  uint32_t n;
  const uint64_t *row_ptr;
  const uint32_t *col;
  const int32_t *vw;   /* vertex weights or NULL */
  const uint8_t *lab;  /* vertex labels or NULL */
  const int32_t *ew;   /* edge weights aligned with col, or NULL */
  uint64_t *adj;       /* optional n x n adjacency bit matrix (small graphs) */
} graph_t;

/* ------------------------------------------------------------------ */
/* small helpers                                                       */
/* ------------------------------------------------------------------ */

static void *xmalloc(size_t n) {
  void *p = malloc(n ? n : 1);
  if (!p) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
  return p;
}

static int is_adjacent(const graph_t *g, uint32_t u, uint32_t v) {
  if (g->adj) return (int)((g->adj[(uint64_t)u * ((g->n + 63) / 64) + v / 64] >> (v % 64)) & 1u);
  uint64_t lo = g->row_ptr[u], hi = g->row_ptr[u + 1];
  while (lo < hi) {
    uint64_t mid = lo + (hi - lo) / 2;
    if (g->col[mid] == v) return 1;
    if (g->col[mid] < v) lo = mid + 1; else hi = mid;
  }
  return 0;
}

/* weight of edge {u,v}; 0 if absent */
static int64_t edge_weight(const graph_t *g, uint32_t u, uint32_t v) {
  uint64_t lo = g->row_ptr[u], hi = g->row_ptr[u + 1];
  while (lo < hi) {
    uint64_t mid = lo + (hi - lo) / 2;
    if (g->col[mid] == v) return g->ew ? g->ew[mid] : 1;
    if (g->col[mid] < v) lo = mid + 1; else hi = mid;
  }
  return 0;
}

static int cmp_u32(const void *a, const void *b) {
  uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
  return x < y ? -1 : x > y;
}

/* lexicographic comparison of two id sequences */
static int lex_cmp(const uint32_t *a, uint32_t na, const uint32_t *b, uint32_t nb) {
  uint32_t n = na < nb ? na : nb;
  for (uint32_t i = 0; i < n; ++i)
    if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
  return na < nb ? -1 : (na > nb);
}

/* ------------------------------------------------------------------ */
/* the priority queue Q: a binary max-heap (Algorithm 1, lines 3, 5, 16) */
/* ------------------------------------------------------------------ */

/*
 * Priorities are compared as lexicographic tuples of up to 3 int64 values.
 * Ties are broken by insertion sequence, earlier first, which fixes the
 * exploration order but never the result.
 */
typedef struct {
  int64_t key[3];
  uint64_t seq;
  void *item;
} pq_entry;

typedef struct {
  pq_entry *a;
  uint64_t n, cap, next_seq;
} pq_t;

static int pq_higher(const pq_entry *x, const pq_entry *y) {
  for (int i = 0; i < 3; ++i)
    if (x->key[i] != y->key[i]) return x->key[i] > y->key[i];
  return x->seq < y->seq;
}

static void pq_insert(pq_t *q, const int64_t key[3], void *item) {
  if (q->n == q->cap) {
    q->cap = q->cap ? 2 * q->cap : 1024;
    q->a = (pq_entry *)realloc(q->a, q->cap * sizeof(pq_entry));
    if (!q->a) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
  }
  pq_entry e;
  memcpy(e.key, key, sizeof(e.key));
  e.seq = q->next_seq++;
  e.item = item;
  uint64_t i = q->n++;
  while (i > 0) {
    uint64_t p = (i - 1) / 2;
    if (!pq_higher(&e, &q->a[p])) break;
    q->a[i] = q->a[p];
    i = p;
  }
  q->a[i] = e;
}

static void *pq_remove_max(pq_t *q) {
  void *top = q->a[0].item;
  pq_entry last = q->a[--q->n];
  uint64_t i = 0;
  for (;;) {
    uint64_t l = 2 * i + 1, r = l + 1, b = i;
    const pq_entry *best = &last;
    if (l < q->n && pq_higher(&q->a[l], best)) { b = l; best = &q->a[l]; }
    if (r < q->n && pq_higher(&q->a[r], best)) { b = r; best = &q->a[r]; }
    if (b == i) break;
    q->a[i] = q->a[b];
    i = b;
  }
  if (q->n) q->a[i] = last;
  return top;
}

/* ------------------------------------------------------------------ */
/* the result set R: exactly min(k, #results) entries                   */
/* ------------------------------------------------------------------ */

typedef struct {
  int64_t score;
  uint32_t len;
  uint32_t *ids; /* cliques: ascending original ids; matches: mu(0..q-1) */
} result_t;

typedef struct {
  result_t *e; /* sorted best first */
  uint32_t n, k;
} rset_t;

/* -1 if (s1, ids1) ranks before (s2, ids2) */
static int rank_cmp(int64_t s1, const uint32_t *a, uint32_t na, int64_t s2, const uint32_t *b,
                    uint32_t nb) {
  if (s1 != s2) return s1 > s2 ? -1 : 1;
  return lex_cmp(a, na, b, nb);
}

/* offer a result; returns 1 if it entered R */
static int rset_offer(rset_t *R, int64_t score, const uint32_t *ids, uint32_t len) {
  if (R->n == R->k) {
    const result_t *kth = &R->e[R->k - 1];
    if (rank_cmp(score, ids, len, kth->score, kth->ids, kth->len) >= 0) return 0;
    free(R->e[R->k - 1].ids);
    R->n--;
  }
  uint32_t i = R->n;
  while (i > 0 && rank_cmp(score, ids, len, R->e[i - 1].score, R->e[i - 1].ids, R->e[i - 1].len) < 0) {
    R->e[i] = R->e[i - 1];
    --i;
  }
  R->e[i].score = score;
  R->e[i].len = len;
  R->e[i].ids = (uint32_t *)xmalloc(len * sizeof(uint32_t));
  memcpy(R->e[i].ids, ids, len * sizeof(uint32_t));
  R->n++;
  return 1;
}

/* dominated(s, kth(R)) with the strict rule: bound < score of the k-th */
static int rset_dominates(const rset_t *R, int64_t bound) {
  return R->n == R->k && bound < R->e[R->k - 1].score;
}

typedef struct {
  uint64_t popped, expanded, children, pruned_at_creation, pruned_at_pop, offered;
} ostats_t;

/*
 * Optional cap on the children one clique search may create (0 = none).
 * A capped search stops early and reports -3 instead of a result; it only
 * serves to time the oracle on a bounded sample of a large workload.
 */
static uint64_t g_work_limit = 0;
void oracle_set_work_limit(uint64_t max_children) { g_work_limit = max_children; }

/* flatten R into caller buffers; returns count */
static uint32_t rset_export(rset_t *R, int64_t *score_out, uint64_t *off_out, uint32_t *ids_out,
                            uint64_t ids_cap) {
  uint64_t t = 0;
  off_out[0] = 0;
  for (uint32_t i = 0; i < R->n; ++i) {
    score_out[i] = R->e[i].score;
    for (uint32_t j = 0; j < R->e[i].len; ++j) {
      if (t < ids_cap) ids_out[t] = R->e[i].ids[j];
      ++t;
    }
    off_out[i + 1] = t;
    free(R->e[i].ids);
  }
  uint32_t c = R->n;
  free(R->e);
  return c;
}

/* ------------------------------------------------------------------ */
/* vertex order pi                                                     */
/* ------------------------------------------------------------------ */

/*
 * order_kind 0: pi = vertex id.
 * order_kind 1: degeneracy order (repeatedly remove a vertex of minimum
 * remaining degree); pi(v) = removal position.  Among vertices of equal
 * remaining degree the one at the head of that degree's list goes first,
 * which makes the order deterministic.  Any order yields the same result
 * set; this one keeps candidate sets small (at most the degeneracy).
 */
static uint32_t *vertex_order(const graph_t *g, int order_kind) {
  uint32_t n = g->n;
  uint32_t *pi = (uint32_t *)xmalloc((uint64_t)n * sizeof(uint32_t));
  if (order_kind == 0) {
    for (uint32_t v = 0; v < n; ++v) pi[v] = v;
    return pi;
  }
  uint32_t *deg = (uint32_t *)xmalloc((uint64_t)n * sizeof(uint32_t));
  uint32_t maxd = 0;
  for (uint32_t v = 0; v < n; ++v) {
    deg[v] = (uint32_t)(g->row_ptr[v + 1] - g->row_ptr[v]);
    if (deg[v] > maxd) maxd = deg[v];
  }
  /* one doubly linked list of vertices per remaining degree */
  uint32_t NIL = 0xFFFFFFFFu;
  uint32_t *head = (uint32_t *)xmalloc(((uint64_t)maxd + 1) * sizeof(uint32_t));
  uint32_t *nxt = (uint32_t *)xmalloc((uint64_t)n * sizeof(uint32_t));
  uint32_t *prv = (uint32_t *)xmalloc((uint64_t)n * sizeof(uint32_t));
  uint8_t *gone = (uint8_t *)calloc(n ? n : 1, 1);
  for (uint32_t d = 0; d <= maxd; ++d) head[d] = NIL;
  for (uint32_t v = n; v-- > 0;) {
    uint32_t d = deg[v];
    nxt[v] = head[d];
    prv[v] = NIL;
    if (head[d] != NIL) prv[head[d]] = v;
    head[d] = v;
  }
  uint32_t cur = 0;
  for (uint32_t pos = 0; pos < n; ++pos) {
    if (cur > 0) cur--; /* a removal lowers neighbour degrees by at most one */
    while (head[cur] == NIL) cur++;
    uint32_t v = head[cur];
    /* unlink v */
    if (prv[v] != NIL) nxt[prv[v]] = nxt[v]; else head[cur] = nxt[v];
    if (nxt[v] != NIL) prv[nxt[v]] = prv[v];
    gone[v] = 1;
    pi[v] = pos;
    for (uint64_t e = g->row_ptr[v]; e < g->row_ptr[v + 1]; ++e) {
      uint32_t u = g->col[e];
      if (gone[u]) continue;
      uint32_t d = deg[u];
      if (prv[u] != NIL) nxt[prv[u]] = nxt[u]; else head[d] = nxt[u];
      if (nxt[u] != NIL) prv[nxt[u]] = prv[u];
      deg[u] = d - 1;
      nxt[u] = head[d - 1];
      prv[u] = NIL;
      if (head[d - 1] != NIL) prv[head[d - 1]] = u;
      head[d - 1] = u;
    }
  }
  free(deg); free(head); free(nxt); free(prv); free(gone);
  return pi;
}

/* ------------------------------------------------------------------ */
/* top-k cliques                                                       */
/* ------------------------------------------------------------------ */

/* A clique subgraph s: V_s, the ordered candidate set P_s, and X_s. */
typedef struct {
  uint32_t nv, np, nx;
  uint32_t *V; /* original ids, in insertion order */
  uint32_t *P; /* sorted by pi */
  uint32_t *X; /* sorted by pi */
  int64_t score, bound;
} clique_rec;

static void clique_free(clique_rec *s) {
  free(s->V); free(s->P); free(s->X); free(s);
}

static int64_t vweight(const graph_t *g, int weighted, uint32_t v) {
  return weighted ? (int64_t)g->vw[v] : 1;
}

/*
 * Upper bound on the score of any clique s can expand into.
 * bound_kind 0 (Carraghan-Pardalos, Section 3.2): score(V) + score(P),
 *   i.e. |V| + |P| for size scores.
 * bound_kind 1 (greedy colouring, the tighter bound the paper leaves to
 *   future work): colour P greedily in pi order with the smallest colour
 *   not used by an adjacent earlier vertex; a clique takes at most one
 *   vertex per colour, so score(V) + sum over colours of the largest
 *   weight in that colour is a bound.
 */
static int64_t clique_bound(const graph_t *g, int weighted, int bound_kind, const clique_rec *s) {
  int64_t b = s->score;
  if (bound_kind == 0) {
    for (uint32_t i = 0; i < s->np; ++i) b += vweight(g, weighted, s->P[i]);
    return b;
  }
  uint32_t np = s->np;
  uint32_t *color = (uint32_t *)xmalloc(np * sizeof(uint32_t));
  uint32_t ncol = 0;
  uint8_t *used = (uint8_t *)xmalloc(np + 1);
  for (uint32_t i = 0; i < np; ++i) {
    memset(used, 0, np + 1);
    for (uint32_t j = 0; j < i; ++j)
      if (is_adjacent(g, s->P[i], s->P[j])) used[color[j]] = 1;
    uint32_t c = 0;
    while (used[c]) ++c;
    color[i] = c;
    if (c + 1 > ncol) ncol = c + 1;
  }
  int64_t *cmax = (int64_t *)calloc(ncol ? ncol : 1, sizeof(int64_t));
  for (uint32_t i = 0; i < np; ++i) {
    int64_t w = vweight(g, weighted, s->P[i]);
    if (w > cmax[color[i]]) cmax[color[i]] = w;
  }
  for (uint32_t c = 0; c < ncol; ++c) b += cmax[c];
  free(color); free(used); free(cmax);
  return b;
}

/*
 * Queue priority of a clique subgraph.
 * priority_kind 0: the paper's (|V_s|, |P_s|) compared lexicographically
 *   (Section 3.2, prioritized expansion).
 * priority_kind 1: (bound) - best bound first.
 * priority_kind 2: FIFO - no prioritisation, as in the paper's Nuri-NP
 *   variant (Section 6.1), keyed by insertion order alone.
 */
static void clique_priority(int priority_kind, const clique_rec *s, int64_t key[3]) {
  key[0] = key[1] = key[2] = 0;
  if (priority_kind == 0) { key[0] = s->nv; key[1] = s->np; }
  else if (priority_kind == 1) { key[0] = s->bound; }
}

/*
 * Targeted-expansion test for maximal cliques: true when some x in X_s is
 * adjacent to every vertex of P_s.  Every clique s can grow into lies
 * between V_s and V_s + P_s, so x would extend each of them: none is
 * maximal, and s need not be created (expandable() of Table 1 is false).
 */
static int has_extension_witness(const graph_t *g, const clique_rec *s) {
  for (uint32_t a = 0; a < s->nx; ++a) {
    int all = 1;
    for (uint32_t b = 0; b < s->np && all; ++b)
      if (!is_adjacent(g, s->X[a], s->P[b])) all = 0;
    if (all) return 1;
  }
  return 0;
}

/*
 * Top-k maximal cliques by Algorithm 1.
 *   weighted: 0 score = |C|; 1 score = sum of vertex weights (int64).
 *   xprune: 1 applies has_extension_witness() to unit subgraphs and
 *   children (it never changes the result, only the work).
 * Outputs up to k results: score_out[i], ids_out[off_out[i]..off_out[i+1])
 * holding the ascending original ids.  Returns the count, or -1 if the id
 * buffer was too small (ids_needed then holds the size required).
 */
int64_t oracle_topk_cliques(uint32_t n, const uint64_t *row_ptr, const uint32_t *col,
                            const int32_t *vw, uint32_t k, int weighted, int bound_kind,
                            int priority_kind, int order_kind, int xprune,
                            int64_t *score_out, uint64_t *off_out, uint32_t *ids_out,
                            uint64_t ids_cap, uint64_t *stats_out) {
  graph_t G = {n, row_ptr, col, vw, NULL, NULL, NULL};
  const graph_t *g = &G;
  if (k == 0) return -2;
  /* adjacency tests by bit lookup when the n x n matrix is small */
  if (n <= 32768) {
    uint64_t words = (n + 63) / 64;
    uint64_t cells = (uint64_t)n * words;
    G.adj = (uint64_t *)calloc(cells ? cells : 1, sizeof(uint64_t));
    for (uint32_t u = 0; u < n; ++u)
      for (uint64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e)
        G.adj[(uint64_t)u * words + col[e] / 64] |= 1ull << (col[e] % 64);
  }
  uint32_t *pi = vertex_order(g, order_kind);
  pq_t Q = {0};
  rset_t R = {(result_t *)xmalloc((uint64_t)k * sizeof(result_t)), 0, k};
  ostats_t st = {0};

  /* lines 1-3: one unit subgraph per vertex */
  for (uint32_t v = 0; v < n; ++v) {
    clique_rec *s = (clique_rec *)xmalloc(sizeof(clique_rec));
    uint64_t deg = row_ptr[v + 1] - row_ptr[v];
    s->V = (uint32_t *)xmalloc(sizeof(uint32_t));
    s->P = (uint32_t *)xmalloc(deg * sizeof(uint32_t));
    s->X = (uint32_t *)xmalloc(deg * sizeof(uint32_t));
    s->nv = 1; s->V[0] = v; s->np = 0; s->nx = 0;
    for (uint64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
      uint32_t u = col[e];
      if (pi[u] > pi[v]) s->P[s->np++] = u; else s->X[s->nx++] = u;
    }
    /* sort P and X by pi (insertion sort on pi keys) */
    for (int which = 0; which < 2; ++which) {
      uint32_t *a = which ? s->X : s->P, m = which ? s->nx : s->np;
      for (uint32_t i = 1; i < m; ++i) {
        uint32_t x = a[i], j = i;
        while (j > 0 && pi[a[j - 1]] > pi[x]) { a[j] = a[j - 1]; --j; }
        a[j] = x;
      }
    }
    s->score = vweight(g, weighted, v);
    if (xprune && has_extension_witness(g, s)) { clique_free(s); continue; }
    s->bound = clique_bound(g, weighted, bound_kind, s);
    int64_t key[3];
    clique_priority(priority_kind, s, key);
    pq_insert(&Q, key, s);
  }

  uint32_t *tmp_ids = (uint32_t *)xmalloc(((uint64_t)n + 1) * sizeof(uint32_t));
  int capped = 0;
  while (Q.n > 0) {                                   /* line 4 */
    if (g_work_limit && st.children >= g_work_limit) { capped = 1; break; }
    clique_rec *s = (clique_rec *)pq_remove_max(&Q);   /* line 5 */
    st.popped++;
    /* lines 6-10: relevant(s) iff s is a maximal clique (P and X empty) */
    if (s->np == 0 && s->nx == 0) {
      memcpy(tmp_ids, s->V, s->nv * sizeof(uint32_t));
      qsort(tmp_ids, s->nv, sizeof(uint32_t), cmp_u32);
      st.offered++;
      rset_offer(&R, s->score, tmp_ids, s->nv);
    }
    /* line 11: skip s when dominated by the k-th result */
    if (rset_dominates(&R, s->bound)) { st.pruned_at_pop++; clique_free(s); continue; }
    if (s->np > 0) st.expanded++;
    /* lines 12-16: expand by every p in P_s, in pi order */
    for (uint32_t i = 0; i < s->np; ++i) {
      uint32_t p = s->P[i];
      clique_rec *c = (clique_rec *)xmalloc(sizeof(clique_rec));
      c->nv = s->nv + 1;
      c->V = (uint32_t *)xmalloc(c->nv * sizeof(uint32_t));
      memcpy(c->V, s->V, s->nv * sizeof(uint32_t));
      c->V[s->nv] = p;
      /* P' = {u in P_s after p} intersect N(p) */
      c->P = (uint32_t *)xmalloc((s->np - i) * sizeof(uint32_t));
      c->np = 0;
      for (uint32_t j = i + 1; j < s->np; ++j)
        if (is_adjacent(g, p, s->P[j])) c->P[c->np++] = s->P[j];
      /* X' = (X_s union {u in P_s before p}) intersect N(p), kept pi-sorted */
      c->X = (uint32_t *)xmalloc((s->nx + i + 1) * sizeof(uint32_t));
      c->nx = 0;
      uint32_t a = 0, b = 0;
      while (a < s->nx || b < i) {
        uint32_t u;
        if (b >= i || (a < s->nx && pi[s->X[a]] < pi[s->P[b]])) u = s->X[a++];
        else u = s->P[b++];
        if (is_adjacent(g, p, u)) c->X[c->nx++] = u;
      }
      c->score = s->score + vweight(g, weighted, p);
      st.children++;
      /* line 13: expandable(s, p) */
      if (xprune && has_extension_witness(g, c)) {
        st.pruned_at_creation++;
        clique_free(c);
        continue;
      }
      c->bound = clique_bound(g, weighted, bound_kind, c);
      /* line 15: insert unless dominated */
      if (rset_dominates(&R, c->bound)) { st.pruned_at_creation++; clique_free(c); continue; }
      int64_t key[3];
      clique_priority(priority_kind, c, key);
      pq_insert(&Q, key, c);                          /* line 16 */
    }
    clique_free(s);
  }
  free(tmp_ids);
  while (Q.n > 0) clique_free((clique_rec *)pq_remove_max(&Q));
  free(Q.a);
  free(pi);
  free(G.adj);

  uint64_t need = 0;
  for (uint32_t i = 0; i < R.n; ++i) need += R.e[i].len;
  if (stats_out) {
    stats_out[0] = st.popped; stats_out[1] = st.expanded; stats_out[2] = st.children;
    stats_out[3] = st.pruned_at_creation; stats_out[4] = st.pruned_at_pop; stats_out[5] = st.offered;
    stats_out[6] = need;
  }
  if (capped) {
    for (uint32_t i = 0; i < R.n; ++i) free(R.e[i].ids);
    free(R.e);
    return -3;
  }
  if (need > ids_cap) {
    for (uint32_t i = 0; i < R.n; ++i) free(R.e[i].ids);
    free(R.e);
    return -1;
  }
  return (int64_t)rset_export(&R, score_out, off_out, ids_out, ids_cap);
}

/*
 * Paper-trace mode (Section 3.2 worked example): every clique is relevant,
 * priority is (|V_s|, |P_s|), R ranks entries by that priority and keeps
 * every entry tied with the k-th (lines 7-10), dominated(s, s') is
 * |V_s| + |P_s| < |V_s'|, pi = vertex id.
 *
 * Logs, for each pop in order: the popped vertex set (sorted ids, -1
 * terminated), whether it entered R, whether it was pruned at pop, and the
 * number of children inserted.  Writes R's final vertex sets the same way.
 * Returns the number of pops.
 */
int64_t oracle_clique_trace(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, uint32_t k,
                            int32_t *pop_log, uint64_t pop_log_cap, int32_t *r_log,
                            uint64_t r_log_cap, uint64_t *stats_out) {
  graph_t G = {n, row_ptr, col, NULL, NULL, NULL, NULL};
  const graph_t *g = &G;
  if (n > 64 || k == 0) return -2; /* trace mode is for tiny worked examples */
  pq_t Q = {0};
  /* R holds pointers to vertex sets with their priority */
  typedef struct { int64_t p0, p1; uint32_t nv; uint32_t *V; } tentry;
  tentry *R = (tentry *)xmalloc(((uint64_t)n * n + 8) * sizeof(tentry));
  uint64_t rn = 0, lt = 0, npop = 0;
  ostats_t st = {0};
  for (uint32_t v = 0; v < n; ++v) {
    clique_rec *s = (clique_rec *)xmalloc(sizeof(clique_rec));
    uint64_t deg = row_ptr[v + 1] - row_ptr[v];
    s->V = (uint32_t *)xmalloc(sizeof(uint32_t));
    s->P = (uint32_t *)xmalloc(deg * sizeof(uint32_t));
    s->X = NULL;
    s->nv = 1; s->V[0] = v; s->np = 0; s->nx = 0;
    for (uint64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e)
      if (col[e] > v) s->P[s->np++] = col[e];
    s->score = 1;
    s->bound = 1 + s->np;
    int64_t key[3] = {s->nv, s->np, 0};
    pq_insert(&Q, key, s);
  }
  while (Q.n > 0) {
    clique_rec *s = (clique_rec *)pq_remove_max(&Q);
    st.popped++;
    npop++;
    int inserted = 0, pruned = 0, nchild = 0;
    /* k-th(R): the k-th entry when R is ordered by priority, best first */
    /* R is kept sorted by priority descending (stable for equal keys) */
    int admit = (rn < k);
    if (!admit) {
      tentry *kth = &R[k - 1];
      admit = (s->nv > kth->p0) || (s->nv == kth->p0 && (int64_t)s->np >= kth->p1);
    }
    if (admit) {
      uint64_t i = rn;
      while (i > 0 && (R[i - 1].p0 < s->nv || (R[i - 1].p0 == s->nv && R[i - 1].p1 < (int64_t)s->np))) {
        R[i] = R[i - 1];
        --i;
      }
      R[i].p0 = s->nv; R[i].p1 = s->np; R[i].nv = s->nv;
      R[i].V = (uint32_t *)xmalloc(s->nv * sizeof(uint32_t));
      memcpy(R[i].V, s->V, s->nv * sizeof(uint32_t));
      qsort(R[i].V, s->nv, sizeof(uint32_t), cmp_u32);
      rn++;
      inserted = 1;
      if (rn > k) {
        int64_t k0 = R[k - 1].p0, k1 = R[k - 1].p1;
        uint64_t w = 0;
        for (uint64_t j = 0; j < rn; ++j) {
          int lower = (R[j].p0 < k0) || (R[j].p0 == k0 && R[j].p1 < k1);
          if (lower) free(R[j].V); else R[w++] = R[j];
        }
        rn = w;
      }
    }
    if (rn >= k && (int64_t)(s->nv + s->np) < R[k - 1].p0) {
      pruned = 1;
      st.pruned_at_pop++;
    } else {
      for (uint32_t i = 0; i < s->np; ++i) {
        uint32_t p = s->P[i];
        clique_rec *c = (clique_rec *)xmalloc(sizeof(clique_rec));
        c->nv = s->nv + 1;
        c->V = (uint32_t *)xmalloc(c->nv * sizeof(uint32_t));
        memcpy(c->V, s->V, s->nv * sizeof(uint32_t));
        c->V[s->nv] = p;
        c->P = (uint32_t *)xmalloc((s->np - i) * sizeof(uint32_t));
        c->np = 0;
        c->X = NULL; c->nx = 0;
        for (uint32_t j = i + 1; j < s->np; ++j)
          if (is_adjacent(g, p, s->P[j])) c->P[c->np++] = s->P[j];
        c->score = c->nv;
        c->bound = c->nv + c->np;
        st.children++;
        if (rn >= k && (int64_t)(c->nv + c->np) < R[k - 1].p0) {
          st.pruned_at_creation++;
          clique_free(c);
          continue;
        }
        int64_t key[3] = {c->nv, c->np, 0};
        pq_insert(&Q, key, c);
        nchild++;
      }
    }
    /* log: sorted V, -1, inserted, pruned, nchild */
    uint32_t tmp[64];
    uint32_t nv = s->nv < 64 ? s->nv : 64;
    memcpy(tmp, s->V, nv * sizeof(uint32_t));
    qsort(tmp, nv, sizeof(uint32_t), cmp_u32);
    for (uint32_t i = 0; i < nv; ++i) if (lt < pop_log_cap) pop_log[lt++] = (int32_t)tmp[i];
    int32_t tail[4] = {-1, inserted, pruned, nchild};
    for (int i = 0; i < 4; ++i) if (lt < pop_log_cap) pop_log[lt++] = tail[i];
    clique_free(s);
  }
  uint64_t rt = 0;
  for (uint64_t j = 0; j < rn; ++j) {
    for (uint32_t i = 0; i < R[j].nv; ++i) if (rt < r_log_cap) r_log[rt++] = (int32_t)R[j].V[i];
    if (rt < r_log_cap) r_log[rt++] = -1;
    free(R[j].V);
  }
  free(R);
  free(Q.a);
  if (stats_out) {
    stats_out[0] = st.popped; stats_out[1] = st.children; stats_out[2] = st.pruned_at_creation;
    stats_out[3] = st.pruned_at_pop; stats_out[4] = rn;
  }
  return (int64_t)npop;
}

/* ------------------------------------------------------------------ */
/* top-k labelled subgraph matching                                    */
/* ------------------------------------------------------------------ */

#define QMAX 8

/* a partial embedding: mu(order[0..depth-1]) assigned */
typedef struct {
  uint32_t depth;
  uint32_t mu[QMAX]; /* indexed by pattern vertex; valid for matched ones */
  int64_t score, bound;
} match_rec;

typedef struct {
  uint32_t q, ne;
  uint8_t label[QMAX];
  uint32_t ea[QMAX * QMAX], eb[QMAX * QMAX];
  uint8_t adj[QMAX][QMAX];
  uint32_t order[QMAX], pos[QMAX];
  uint32_t hop[QMAX]; /* distance from order[0] in the pattern */
  uint32_t naut;
  uint8_t *aut; /* naut x q permutations */
} pattern_t;

/*
 * The automorphisms of the labelled pattern: every permutation s of
 * {0..q-1} with label(s(a)) = label(a) and {s(a), s(b)} an edge for every
 * edge {a, b}.  Brute force over all q! permutations (q <= 8).
 */
static void pattern_automorphisms(pattern_t *P) {
  uint32_t q = P->q;
  uint32_t perm[QMAX], c[QMAX];
  uint64_t cap = 1;
  for (uint32_t i = 2; i <= q; ++i) cap *= i;
  P->aut = (uint8_t *)xmalloc(cap * q);
  P->naut = 0;
  for (uint32_t i = 0; i < q; ++i) { perm[i] = i; c[i] = 0; }
  /* Heap's algorithm enumerates every permutation once */
  for (;;) {
    int ok = 1;
    for (uint32_t a = 0; a < q && ok; ++a)
      if (P->label[perm[a]] != P->label[a]) ok = 0;
    for (uint32_t e = 0; e < P->ne && ok; ++e)
      if (!P->adj[perm[P->ea[e]]][perm[P->eb[e]]]) ok = 0;
    if (ok) { for (uint32_t a = 0; a < q; ++a) P->aut[P->naut * q + a] = (uint8_t)perm[a]; P->naut++; }
    uint32_t i = 1;
    while (i < q && c[i] >= i) { c[i] = 0; ++i; }
    if (i >= q) break;
    uint32_t j = (i % 2) ? c[i] : 0;
    uint32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    c[i]++;
  }
}

/* bound tables: best[v*nl + l] = max weight of an edge from v to a label-l vertex */
typedef struct {
  uint32_t nl;
  int64_t *best;     /* n x nl */
  int64_t *pairmax;  /* nl x nl */
} tables_t;

static void build_tables(const graph_t *g, uint32_t nl, tables_t *T) {
  T->nl = nl;
  T->best = (int64_t *)calloc((uint64_t)g->n * nl, sizeof(int64_t));
  T->pairmax = (int64_t *)calloc((uint64_t)nl * nl, sizeof(int64_t));
  for (uint32_t v = 0; v < g->n; ++v)
    for (uint64_t e = g->row_ptr[v]; e < g->row_ptr[v + 1]; ++e) {
      uint32_t u = g->col[e];
      int64_t w = g->ew ? g->ew[e] : 1;
      uint32_t lu = g->lab[u], lv = g->lab[v];
      if (w > T->best[(uint64_t)v * nl + lu]) T->best[(uint64_t)v * nl + lu] = w;
      if (w > T->pairmax[lv * nl + lu]) T->pairmax[lv * nl + lu] = w;
    }
}

/*
 * Upper bound on the final score of any completion of r (Section 4.3:
 * current score plus an index-based bound for what is still unmatched).
 * Per pattern edge {a,b}: its weight if both ends are matched; the
 * largest weight from mu(a) to a vertex labelled label(b) if only a is
 * matched; the largest weight over all edges with that label pair if
 * neither is.  Returns -1 when an unmatched edge has no possible data
 * edge (no completion exists).
 */
static int64_t match_bound(const graph_t *g, const pattern_t *P, const tables_t *T,
                           const match_rec *r) {
  int64_t b = 0;
  uint8_t matched[QMAX] = {0};
  for (uint32_t i = 0; i < r->depth; ++i) matched[P->order[i]] = 1;
  for (uint32_t e = 0; e < P->ne; ++e) {
    uint32_t a = P->ea[e], c = P->eb[e];
    int64_t ub;
    if (matched[a] && matched[c]) ub = edge_weight(g, r->mu[a], r->mu[c]);
    else if (matched[a]) ub = T->best[(uint64_t)r->mu[a] * T->nl + P->label[c]];
    else if (matched[c]) ub = T->best[(uint64_t)r->mu[c] * T->nl + P->label[a]];
    else ub = T->pairmax[P->label[a] * T->nl + P->label[c]];
    if (ub <= 0) return -1;
    b += ub;
  }
  return b;
}

static int64_t degree_of(const graph_t *g, uint32_t v) {
  return (int64_t)(g->row_ptr[v + 1] - g->row_ptr[v]);
}

/*
 * The Section 4.3 index (Listing 3), cumulative over hops:
 * out[(h-1)*n*nl + v*nl + l] = the largest degree of a label-l vertex x
 * with 1 <= dist(v, x) <= h, or 0 when there is none, for h = 1..H.  A
 * breadth-first search from every vertex, cut at depth H.
 */
static void hop_index(const graph_t *g, uint32_t nl, uint32_t H, int32_t *out) {
  const uint32_t n = g->n;
  memset(out, 0, (uint64_t)H * n * nl * sizeof(int32_t));
  int32_t *dist = (int32_t *)xmalloc((uint64_t)n * sizeof(int32_t));
  uint32_t *queue = (uint32_t *)xmalloc((uint64_t)n * sizeof(uint32_t));
  int32_t *layer = (int32_t *)xmalloc((uint64_t)(H + 1) * nl * sizeof(int32_t));
  for (uint32_t v = 0; v < n; ++v) dist[v] = -1;
  for (uint32_t v = 0; v < n; ++v) {
    memset(layer, 0, (uint64_t)(H + 1) * nl * sizeof(int32_t));
    uint64_t head = 0, tail = 0;
    queue[tail++] = v;
    dist[v] = 0;
    while (head < tail) {
      uint32_t x = queue[head++];
      if (dist[x] > 0) {
        int32_t *m = &layer[(uint64_t)dist[x] * nl + g->lab[x]];
        if (degree_of(g, x) > *m) *m = (int32_t)degree_of(g, x);
      }
      if ((uint32_t)dist[x] == H) continue;
      for (uint64_t e = g->row_ptr[x]; e < g->row_ptr[x + 1]; ++e) {
        uint32_t y = g->col[e];
        if (dist[y] < 0) { dist[y] = dist[x] + 1; queue[tail++] = y; }
      }
    }
    for (uint64_t i = 0; i < tail; ++i) dist[queue[i]] = -1;
    /* entry for hop h = max over the layers 1..h */
    for (uint32_t l = 0; l < nl; ++l) {
      int32_t run = 0;
      for (uint32_t h = 1; h <= H; ++h) {
        if (layer[(uint64_t)h * nl + l] > run) run = layer[(uint64_t)h * nl + l];
        out[((uint64_t)(h - 1) * n + v) * nl + l] = run;
      }
    }
  }
  free(dist);
  free(queue);
  free(layer);
}

/*
 * Degree-score bound (Section 4.3): the current score plus, for every
 * pattern vertex u not yet matched, index(seed, label(u), hop(u)), where
 * the seed is the data vertex of the unit subgraph (mu(order[0])) and
 * hop(u) is u's distance from order[0] in the pattern.  A pattern path of
 * length h maps onto a data walk of length h, so mu(u) lies within hop(u)
 * of the seed and is not the seed.  Returns -1 when an entry is 0 (no
 * vertex of that label within reach: no completion exists).
 */
static int64_t match_bound_degree(const graph_t *g, const pattern_t *P, const int32_t *hidx,
                                  uint32_t nl, const match_rec *r) {
  uint8_t matched[QMAX] = {0};
  for (uint32_t i = 0; i < r->depth; ++i) matched[P->order[i]] = 1;
  const uint32_t seed = r->mu[P->order[0]];
  int64_t b = r->score;
  for (uint32_t u = 0; u < P->q; ++u) {
    if (matched[u]) continue;
    int32_t x = hidx[((uint64_t)(P->hop[u] - 1) * g->n + seed) * nl + P->label[u]];
    if (x <= 0) return -1;
    b += x;
  }
  return b;
}

/*
 * True when the complete embedding mu is the lexicographically smallest
 * tuple (mu(0), ..., mu(q-1)) among mu o s for all automorphisms s.
 */
static int match_is_canonical(const pattern_t *P, const uint32_t *mu) {
  for (uint32_t t = 0; t < P->naut; ++t) {
    const uint8_t *s = &P->aut[t * P->q];
    for (uint32_t i = 0; i < P->q; ++i) {
      uint32_t x = mu[s[i]];
      if (x < mu[i]) return 0;
      if (x > mu[i]) break;
    }
  }
  return 1;
}

/*
 * Partial check of the same condition: mu can still be completed into the
 * smallest tuple of its orbit only if, for each automorphism s, the
 * comparison of mu o s against mu over the leading positions whose values
 * are all known does not already come out smaller.  (A full embedding
 * passes this test exactly when match_is_canonical holds.)
 */
static int match_may_be_canonical(const pattern_t *P, const match_rec *r) {
  uint8_t matched[QMAX] = {0};
  for (uint32_t i = 0; i < r->depth; ++i) matched[P->order[i]] = 1;
  for (uint32_t t = 0; t < P->naut; ++t) {
    const uint8_t *s = &P->aut[t * P->q];
    for (uint32_t i = 0; i < P->q; ++i) {
      if (!matched[i] || !matched[s[i]]) break;
      uint32_t x = r->mu[s[i]];
      if (x < r->mu[i]) return 0;
      if (x > r->mu[i]) break;
    }
  }
  return 1;
}

/*
 * Reads the pattern (q vertices, edges as pairs), checks it, and fixes the
 * matching order: first the vertex whose label is rarest in the graph
 * (ties: larger pattern degree, then smaller id); then repeatedly the
 * vertex with the most edges to the ones already ordered (ties: smaller
 * id).  hop[u] = distance of u from order[0].  Returns 0, or -2 for an
 * invalid pattern.
 */
static int pattern_setup(pattern_t *P, const graph_t *g, uint32_t n_labels, uint32_t q,
                         const uint8_t *plabel, uint32_t ne, const uint32_t *pedges) {
  memset(P, 0, sizeof(*P));
  if (q < 2 || q > QMAX) return -2;
  P->q = q;
  P->ne = ne;
  for (uint32_t a = 0; a < q; ++a) P->label[a] = plabel[a];
  for (uint32_t e = 0; e < ne; ++e) {
    uint32_t a = pedges[2 * e], b = pedges[2 * e + 1];
    if (a >= q || b >= q || a == b || P->adj[a][b]) return -2;
    P->ea[e] = a; P->eb[e] = b;
    P->adj[a][b] = P->adj[b][a] = 1;
  }
  /* connectivity */
  {
    uint8_t seen[QMAX] = {1};
    for (uint32_t round = 0; round < q; ++round)
      for (uint32_t a = 0; a < q; ++a)
        if (seen[a]) for (uint32_t b = 0; b < q; ++b) if (P->adj[a][b]) seen[b] = 1;
    for (uint32_t a = 0; a < q; ++a) if (!seen[a]) return -2;
  }
  uint64_t *lcount = (uint64_t *)calloc(n_labels ? n_labels : 1, sizeof(uint64_t));
  for (uint32_t v = 0; v < g->n; ++v) if (g->lab[v] < n_labels) lcount[g->lab[v]]++;
  {
    uint8_t used[QMAX] = {0};
    uint32_t best = 0;
    for (uint32_t a = 1; a < q; ++a) {
      uint32_t da = 0, db = 0;
      for (uint32_t x = 0; x < q; ++x) { da += P->adj[a][x]; db += P->adj[best][x]; }
      uint64_t ca = P->label[a] < n_labels ? lcount[P->label[a]] : 0;
      uint64_t cb = P->label[best] < n_labels ? lcount[P->label[best]] : 0;
      if (ca < cb || (ca == cb && da > db)) best = a;
    }
    P->order[0] = best; used[best] = 1;
    for (uint32_t i = 1; i < q; ++i) {
      uint32_t pick = q, pc = 0;
      for (uint32_t a = 0; a < q; ++a) {
        if (used[a]) continue;
        uint32_t c = 0;
        for (uint32_t j = 0; j < i; ++j) c += P->adj[a][P->order[j]];
        if (pick == q || c > pc) { pick = a; pc = c; }
      }
      P->order[i] = pick; used[pick] = 1;
    }
    for (uint32_t i = 0; i < q; ++i) P->pos[P->order[i]] = i;
  }
  free(lcount);
  /* distances from order[0] by breadth-first search over the pattern */
  {
    uint32_t queue[QMAX], head = 0, tail = 0;
    uint8_t seen[QMAX] = {0};
    queue[tail++] = P->order[0];
    seen[P->order[0]] = 1;
    P->hop[P->order[0]] = 0;
    while (head < tail) {
      uint32_t a = queue[head++];
      for (uint32_t b = 0; b < q; ++b)
        if (P->adj[a][b] && !seen[b]) { seen[b] = 1; P->hop[b] = P->hop[a] + 1; queue[tail++] = b; }
    }
  }
  pattern_automorphisms(P);
  return 0;
}

static uint32_t pattern_max_hop(const pattern_t *P) {
  uint32_t H = 1;
  for (uint32_t u = 0; u < P->q; ++u) if (P->hop[u] > H) H = P->hop[u];
  return H;
}

/* what the search needs to score and bound a partial match */
typedef struct {
  int degree;      /* 0: edge-weight score, 1: degree score */
  uint32_t nl;
  tables_t T;      /* edge-weight bound tables */
  int32_t *hidx;   /* multi-hop index (degree score) */
} scoring_t;

static void scoring_init(scoring_t *S, const graph_t *g, const pattern_t *P, uint32_t nl,
                         int degree) {
  memset(S, 0, sizeof(*S));
  S->degree = degree;
  S->nl = nl;
  if (degree) {
    uint32_t H = pattern_max_hop(P);
    S->hidx = (int32_t *)xmalloc((uint64_t)H * g->n * nl * sizeof(int32_t));
    hop_index(g, nl, H, S->hidx);
  } else {
    build_tables(g, nl, &S->T);
  }
}

static void scoring_free(scoring_t *S) {
  free(S->hidx);
  free(S->T.best);
  free(S->T.pairmax);
}

static int64_t scoring_bound(const scoring_t *S, const graph_t *g, const pattern_t *P,
                             const match_rec *r) {
  return S->degree ? match_bound_degree(g, P, S->hidx, S->nl, r) : match_bound(g, P, &S->T, r);
}

/* a unit subgraph: v hosts order[0]; its score is deg(v) under the degree score */
static void match_root(const scoring_t *S, const graph_t *g, const pattern_t *P, uint32_t v,
                       match_rec *r) {
  memset(r, 0, sizeof(*r));
  r->depth = 1;
  r->mu[P->order[0]] = v;
  r->score = S->degree ? degree_of(g, v) : 0;
  r->bound = scoring_bound(S, g, P, r);
}

/*
 * Top-k matches of the labelled pattern by Algorithm 1 with
 * vertex-at-a-time expansion in the fixed matching order.  Score = the sum
 * of the data-edge weights under the pattern's edges, or (degree) the sum
 * of the degrees of the matched vertices (int64).  Results: score_out[i]
 * and mu(0..q-1) at ids_out[i*q ..].  Returns count, or -2 for an invalid
 * pattern or k.
 */
static int64_t topk_match(const graph_t *g, uint32_t n_labels, uint32_t q, const uint8_t *plabel,
                          uint32_t ne, const uint32_t *pedges, uint32_t k, int priority_kind,
                          int degree, int64_t *score_out, uint32_t *ids_out,
                          uint64_t *stats_out) {
  const uint32_t n = g->n;
  const uint64_t *row_ptr = g->row_ptr;
  const uint32_t *col = g->col;
  const uint8_t *lab = g->lab;
  if (k == 0) return -2;
  pattern_t P;
  if (pattern_setup(&P, g, n_labels, q, plabel, ne, pedges) != 0) return -2;

  scoring_t S;
  scoring_init(&S, g, &P, n_labels, degree);
  pq_t Q = {0};
  rset_t R = {(result_t *)xmalloc((uint64_t)k * sizeof(result_t)), 0, k};
  ostats_t st = {0};

  /* lines 1-3: unit subgraphs = data vertices that can host order[0] */
  uint32_t first = P.order[0];
  for (uint32_t v = 0; v < n; ++v) {
    if (lab[v] != P.label[first]) continue;
    match_rec *r = (match_rec *)xmalloc(sizeof(match_rec));
    match_root(&S, g, &P, v, r);
    if (r->bound < 0) { free(r); continue; }
    int64_t key[3] = {priority_kind == 2 ? 0 : 1, priority_kind == 2 ? 0 : r->bound, 0};
    if (priority_kind == 1) { key[0] = r->bound; key[1] = 0; }
    pq_insert(&Q, key, r);
  }

  while (Q.n > 0) {
    match_rec *r = (match_rec *)pq_remove_max(&Q);
    st.popped++;
    if (r->depth == q && match_is_canonical(&P, r->mu)) {
      st.offered++;
      rset_offer(&R, r->score, r->mu, q);
    }
    if (rset_dominates(&R, r->bound)) { st.pruned_at_pop++; free(r); continue; }
    if (r->depth == q) { free(r); continue; }
    st.expanded++;
    uint32_t a = P.order[r->depth];
    /* candidates: neighbours of the matched pattern-neighbour that comes
       first in the order, filtered by label, injectivity and adjacency to
       every other matched pattern-neighbour (Ullmann-style refinement) */
    uint32_t anchor = q;
    for (uint32_t i = 0; i < r->depth; ++i)
      if (P.adj[a][P.order[i]]) { anchor = P.order[i]; break; }
    uint32_t av = r->mu[anchor];
    for (uint64_t e = row_ptr[av]; e < row_ptr[av + 1]; ++e) {
      uint32_t c = col[e];
      if (lab[c] != P.label[a]) continue;
      int ok = 1;
      int64_t add = 0;
      for (uint32_t i = 0; i < r->depth && ok; ++i) {
        uint32_t b = P.order[i];
        if (r->mu[b] == c) ok = 0;
        else if (P.adj[a][b]) {
          int64_t w = edge_weight(g, c, r->mu[b]);
          if (w == 0) ok = 0; else add += w;
        }
      }
      if (!ok) continue;
      if (degree) add = degree_of(g, c);
      match_rec *ch = (match_rec *)xmalloc(sizeof(match_rec));
      *ch = *r;
      ch->mu[a] = c;
      ch->depth = r->depth + 1;
      ch->score = r->score + add;
      st.children++;
      if (!match_may_be_canonical(&P, ch)) { free(ch); continue; }
      ch->bound = scoring_bound(&S, g, &P, ch);
      if (ch->bound < 0 || rset_dominates(&R, ch->bound)) {
        st.pruned_at_creation++;
        free(ch);
        continue;
      }
      int64_t key[3] = {ch->depth, ch->bound, 0};
      if (priority_kind == 1) { key[0] = ch->bound; key[1] = 0; }
      if (priority_kind == 2) { key[0] = 0; key[1] = 0; }
      pq_insert(&Q, key, ch);
    }
    free(r);
  }
  free(Q.a);
  scoring_free(&S);
  free(P.aut);
  if (stats_out) {
    stats_out[0] = st.popped; stats_out[1] = st.expanded; stats_out[2] = st.children;
    stats_out[3] = st.pruned_at_creation; stats_out[4] = st.pruned_at_pop; stats_out[5] = st.offered;
    stats_out[6] = P.naut;
  }
  uint32_t cnt = R.n;
  for (uint32_t i = 0; i < cnt; ++i) {
    score_out[i] = R.e[i].score;
    memcpy(&ids_out[(uint64_t)i * q], R.e[i].ids, q * sizeof(uint32_t));
    free(R.e[i].ids);
  }
  free(R.e);
  return cnt;
}

/* top-k matches scored by the sum of matched edge weights (ew NULL: 1 each) */
int64_t oracle_topk_match(uint32_t n, const uint64_t *row_ptr, const uint32_t *col,
                          const uint8_t *lab, const int32_t *ew, uint32_t n_labels, uint32_t q,
                          const uint8_t *plabel, uint32_t ne, const uint32_t *pedges, uint32_t k,
                          int priority_kind, int64_t *score_out, uint32_t *ids_out,
                          uint64_t *stats_out) {
  graph_t G = {n, row_ptr, col, NULL, lab, ew, NULL};
  return topk_match(&G, n_labels, q, plabel, ne, pedges, k, priority_kind, 0, score_out, ids_out,
                    stats_out);
}

/* top-k matches scored by the sum of the degrees of the matched vertices */
int64_t oracle_topk_match_degree(uint32_t n, const uint64_t *row_ptr, const uint32_t *col,
                                 const uint8_t *lab, uint32_t n_labels, uint32_t q,
                                 const uint8_t *plabel, uint32_t ne, const uint32_t *pedges,
                                 uint32_t k, int priority_kind, int64_t *score_out,
                                 uint32_t *ids_out, uint64_t *stats_out) {
  graph_t G = {n, row_ptr, col, NULL, lab, NULL, NULL};
  return topk_match(&G, n_labels, q, plabel, ne, pedges, k, priority_kind, 1, score_out, ids_out,
                    stats_out);
}

/* the multi-hop index for hops 1..H, [H][n][n_labels] */
void oracle_hop_index(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, const uint8_t *lab,
                      uint32_t n_labels, uint32_t H, int32_t *out) {
  graph_t G = {n, row_ptr, col, NULL, lab, NULL, NULL};
  hop_index(&G, n_labels, H, out);
}

/*
 * Bounds of the unit subgraphs (Algorithm 1, lines 1-3): bound_out[v] for
 * every vertex v that can host the first pattern vertex of the matching
 * order, -1 for the others and for roots with no completion.  Returns that
 * pattern vertex, or -2 for an invalid pattern.
 */
int64_t oracle_match_root_bounds(uint32_t n, const uint64_t *row_ptr, const uint32_t *col,
                                 const uint8_t *lab, const int32_t *ew, uint32_t n_labels,
                                 uint32_t q, const uint8_t *plabel, uint32_t ne,
                                 const uint32_t *pedges, int degree, int64_t *bound_out) {
  graph_t G = {n, row_ptr, col, NULL, lab, degree ? NULL : ew, NULL};
  pattern_t P;
  if (pattern_setup(&P, &G, n_labels, q, plabel, ne, pedges) != 0) return -2;
  scoring_t S;
  scoring_init(&S, &G, &P, n_labels, degree);
  for (uint32_t v = 0; v < n; ++v) {
    bound_out[v] = -1;
    if (lab[v] != P.label[P.order[0]]) continue;
    match_rec r;
    match_root(&S, &G, &P, v, &r);
    bound_out[v] = r.bound;
  }
  scoring_free(&S);
  free(P.aut);
  return P.order[0];
}

/* order used by the clique oracle, exposed for tests */
void oracle_vertex_order(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, int order_kind,
                         uint32_t *pi_out) {
  graph_t G = {n, row_ptr, col, NULL, NULL, NULL, NULL};
  uint32_t *pi = vertex_order(&G, order_kind);
  memcpy(pi_out, pi, (uint64_t)n * sizeof(uint32_t));
  free(pi);
}

/*
 * Core numbers (the largest c such that v belongs to the c-core, the
 * maximal subgraph of minimum degree c), by repeatedly removing a vertex of
 * minimum remaining degree and recording the running maximum of the
 * degrees at removal.  Used by the tests: every clique of size s lies in
 * the (s-1)-core, and so does every vertex that could extend it.
 */
void oracle_core_numbers(uint32_t n, const uint64_t *row_ptr, const uint32_t *col,
                         uint32_t *core_out) {
  graph_t G = {n, row_ptr, col, NULL, NULL, NULL, NULL};
  uint32_t *pi = vertex_order(&G, 1);
  uint32_t *by_pos = (uint32_t *)xmalloc((uint64_t)n * sizeof(uint32_t));
  for (uint32_t v = 0; v < n; ++v) by_pos[pi[v]] = v;
  uint32_t run = 0;
  for (uint32_t i = 0; i < n; ++i) {
    uint32_t v = by_pos[i], later = 0;
    for (uint64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e)
      if (pi[col[e]] > i) later++;
    if (later > run) run = later;
    core_out[v] = run;
  }
  free(by_pos);
  free(pi);
}

/* ------------------------------------------------------------------ */
/* top-k frequent pattern mining                                       */
/* ------------------------------------------------------------------ */

/*
 * Patterns are connected, vertex-labelled, with no edge labels.  A pattern
 * is written as its minimum DFS code (Section 3.3, pattern-oriented
 * expansion, after gSpan): a sequence of edges (i, j, L(i), L(j)) over
 * DFS discovery ids, forward when i < j (j is a new vertex), backward when
 * i > j.  Code edges compare by the key
 *   backward: (0, j, 0, 0)      forward: (1, -i, L(i), L(j))
 * (backward before forward; among backward edges the smaller target
 * first; among forward edges the one leaving the deeper vertex first, then
 * by labels), and codes compare edge by edge.  For two codes that agree up
 * to some edge this is the DFS lexicographic order of gSpan; results with
 * equal support are ranked by it too.
 *
 * Support (Section 2.1): minimum image-based support, the smallest number
 * of distinct data vertices any one pattern vertex is mapped to over all
 * embeddings (injective, label-preserving maps sending every pattern edge
 * to a data edge).
 */

#define PM_MAXE 8
#define PM_MAXV (PM_MAXE + 1)

typedef struct { uint8_t i, j, li, lj; } pm_edge;
typedef struct { uint32_t ne, nv; pm_edge e[PM_MAXE]; } pm_code;

static void pm_key(const pm_edge *e, int k[4]) {
  if (e->i > e->j) { k[0] = 0; k[1] = e->j; k[2] = 0; k[3] = 0; }
  else { k[0] = 1; k[1] = -(int)e->i; k[2] = e->li; k[3] = e->lj; }
}

static int pm_edge_cmp(const pm_edge *a, const pm_edge *b) {
  int ka[4], kb[4];
  pm_key(a, ka);
  pm_key(b, kb);
  for (int t = 0; t < 4; ++t)
    if (ka[t] != kb[t]) return ka[t] < kb[t] ? -1 : 1;
  return 0;
}

/* codes edge by edge; a proper prefix is smaller */
static int pm_code_cmp(const pm_code *a, const pm_code *b) {
  uint32_t n = a->ne < b->ne ? a->ne : b->ne;
  for (uint32_t t = 0; t < n; ++t) {
    int c = pm_edge_cmp(&a->e[t], &b->e[t]);
    if (c) return c;
  }
  return a->ne < b->ne ? -1 : (a->ne > b->ne);
}

/* a small labelled graph (the pattern behind a code) */
typedef struct {
  uint32_t nv, ne;
  uint8_t lab[PM_MAXV];
  uint8_t adj[PM_MAXV][PM_MAXV];
} pm_graph;

static void pm_graph_of(const pm_code *c, pm_graph *p) {
  memset(p, 0, sizeof(*p));
  p->nv = c->nv;
  p->ne = c->ne;
  for (uint32_t t = 0; t < c->ne; ++t) {
    p->lab[c->e[t].i] = c->e[t].li;
    p->lab[c->e[t].j] = c->e[t].lj;
    p->adj[c->e[t].i][c->e[t].j] = p->adj[c->e[t].j][c->e[t].i] = 1;
  }
}

/*
 * Every DFS code of p: a depth-first traversal from any start vertex, with
 * every choice of the next unvisited neighbour; a vertex's edges to
 * vertices already visited (other than its discoverer) follow the forward
 * edge that discovers it, by ascending id.  The smallest is kept in *best.
 */
typedef struct {
  const pm_graph *p;
  int id[PM_MAXV];        /* discovery id per pattern vertex, -1 unvisited */
  uint32_t who[PM_MAXV];  /* pattern vertex per discovery id */
  uint32_t nvis;
  pm_code cur, best;
  int have;
} pm_dfs;

/* path[0..sp) is the current DFS path (the rightmost path), root first */
static void pm_dfs_rec(pm_dfs *D, const uint32_t *path, uint32_t sp) {
  const pm_graph *p = D->p;
  if (D->cur.ne == p->ne) {
    if (!D->have || pm_code_cmp(&D->cur, &D->best) < 0) { D->best = D->cur; D->have = 1; }
    return;
  }
  /* the deepest vertex on the path with an unvisited neighbour */
  while (sp > 0) {
    uint32_t u = path[sp - 1], any = 0;
    for (uint32_t w = 0; w < p->nv; ++w) if (p->adj[u][w] && D->id[w] < 0) { any = 1; break; }
    if (any) break;
    --sp;
  }
  if (sp == 0) return; /* cannot happen for a connected pattern */
  uint32_t u = path[sp - 1];
  uint32_t next[PM_MAXV];
  memcpy(next, path, sp * sizeof(uint32_t));
  uint32_t saved_ne = D->cur.ne;
  for (uint32_t w = 0; w < p->nv; ++w) {
    if (!p->adj[u][w] || D->id[w] >= 0) continue;
    uint32_t nid = D->nvis;
    D->id[w] = (int)nid;
    D->who[nid] = w;
    D->nvis++;
    pm_edge f = {(uint8_t)D->id[u], (uint8_t)nid, p->lab[u], p->lab[w]};
    D->cur.e[D->cur.ne++] = f;
    for (uint32_t k = 0; k < nid; ++k) {
      uint32_t x = D->who[k];
      if (x != u && p->adj[w][x]) {
        pm_edge b = {(uint8_t)nid, (uint8_t)k, p->lab[w], p->lab[x]};
        D->cur.e[D->cur.ne++] = b;
      }
    }
    D->cur.nv = D->nvis;
    next[sp] = w;
    pm_dfs_rec(D, next, sp + 1);
    D->cur.ne = saved_ne;
    D->nvis--;
    D->id[w] = -1;
  }
}

static void pm_min_code(const pm_graph *p, pm_code *out) {
  pm_dfs D;
  memset(&D, 0, sizeof(D));
  D.p = p;
  for (uint32_t s = 0; s < p->nv; ++s) {
    for (uint32_t v = 0; v < PM_MAXV; ++v) D.id[v] = -1;
    D.id[s] = 0;
    D.who[0] = s;
    D.nvis = 1;
    D.cur.ne = 0;
    D.cur.nv = 1;
    uint32_t path[1] = {s};
    pm_dfs_rec(&D, path, 1);
  }
  *out = D.best;
  out->nv = p->nv;
}

static int pm_is_min(const pm_code *c) {
  pm_graph p;
  pm_code m;
  pm_graph_of(c, &p);
  pm_min_code(&p, &m);
  return pm_code_cmp(&m, c) == 0;
}

/* support by definition: every embedding of the code's pattern */
typedef struct {
  const graph_t *g;
  const pm_code *c;
  uint32_t par[PM_MAXV];   /* discoverer of each code vertex */
  uint32_t phi[PM_MAXV];
  uint8_t *seen;           /* nv x n image marks */
  uint64_t count[PM_MAXV];
} pm_sup;

static void pm_sup_rec(pm_sup *S, uint32_t x) {
  const pm_code *c = S->c;
  const graph_t *g = S->g;
  if (x == c->nv) {
    for (uint32_t v = 0; v < c->nv; ++v) {
      uint8_t *m = &S->seen[(uint64_t)v * g->n + S->phi[v]];
      if (!*m) { *m = 1; S->count[v]++; }
    }
    return;
  }
  /* candidates: neighbours of the discoverer's image (all vertices for 0) */
  uint8_t lx = 0;
  for (uint32_t t = 0; t < c->ne; ++t) {
    if (c->e[t].i == x) lx = c->e[t].li;
    if (c->e[t].j == x) lx = c->e[t].lj;
  }
  uint64_t b = 0, e = g->n;
  if (x > 0) { b = g->row_ptr[S->phi[S->par[x]]]; e = g->row_ptr[S->phi[S->par[x]] + 1]; }
  for (uint64_t it = b; it < e; ++it) {
    uint32_t w = x > 0 ? g->col[it] : (uint32_t)it;
    if (g->lab[w] != lx) continue;
    int ok = 1;
    for (uint32_t v = 0; v < x && ok; ++v) if (S->phi[v] == w) ok = 0;
    /* every code edge between x and an earlier vertex must be a data edge */
    for (uint32_t t = 0; t < c->ne && ok; ++t) {
      uint32_t a = c->e[t].i, d = c->e[t].j;
      if (a == x && d < x) ok = is_adjacent(g, w, S->phi[d]);
      else if (d == x && a < x) ok = is_adjacent(g, w, S->phi[a]);
    }
    if (!ok) continue;
    S->phi[x] = w;
    pm_sup_rec(S, x + 1);
  }
}

static uint64_t pm_support(const graph_t *g, const pm_code *c) {
  pm_sup S;
  memset(&S, 0, sizeof(S));
  S.g = g;
  S.c = c;
  for (uint32_t t = 0; t < c->ne; ++t)
    if (c->e[t].i < c->e[t].j) S.par[c->e[t].j] = c->e[t].i;
  S.seen = (uint8_t *)calloc((uint64_t)c->nv * g->n, 1);
  pm_sup_rec(&S, 0);
  free(S.seen);
  uint64_t f = UINT64_MAX;
  for (uint32_t v = 0; v < c->nv; ++v) if (S.count[v] < f) f = S.count[v];
  return c->nv ? f : 0;
}

/* result set of patterns: support descending, then code ascending */
typedef struct { uint64_t f; pm_code c; } pm_res;

static int pm_res_before(const pm_res *a, const pm_res *b) {
  if (a->f != b->f) return a->f > b->f;
  return pm_code_cmp(&a->c, &b->c) < 0;
}

static void pm_offer(pm_res *R, uint32_t *n, uint32_t k, const pm_res *x) {
  if (*n == k && !pm_res_before(x, &R[k - 1])) return;
  uint32_t at = *n < k ? (*n)++ : k - 1;
  while (at > 0 && pm_res_before(x, &R[at - 1])) { R[at] = R[at - 1]; --at; }
  R[at] = *x;
}

static void pm_write(const pm_res *R, uint32_t n, uint32_t M, uint64_t *support_out,
                     uint32_t *code_out) {
  for (uint32_t r = 0; r < n; ++r) {
    support_out[r] = R[r].f;
    for (uint32_t t = 0; t < M; ++t) {
      uint32_t *o = &code_out[((uint64_t)r * M + t) * 4];
      o[0] = R[r].c.e[t].i; o[1] = R[r].c.e[t].j; o[2] = R[r].c.e[t].li; o[3] = R[r].c.e[t].lj;
    }
  }
}

/*
 * The definition, for tiny graphs: every connected set of M data edges
 * gives a pattern (its minimum DFS code); each distinct pattern is scored
 * by its support over all embeddings; the top k are returned.  Returns the
 * count, or -2 for bad arguments / a graph too large to enumerate.
 */
int64_t oracle_topk_patterns_definition(uint32_t n, const uint64_t *row_ptr, const uint32_t *col,
                                        const uint8_t *lab, uint32_t M, uint32_t k,
                                        uint64_t *support_out, uint32_t *code_out) {
  graph_t G = {n, row_ptr, col, NULL, lab, NULL, NULL};
  if (M < 1 || M > PM_MAXE || k == 0) return -2;
  uint32_t m = 0;
  for (uint32_t u = 0; u < n; ++u)
    for (uint64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) if (u < col[e]) m++;
  if (m > 64) return -2;
  uint32_t *eu = (uint32_t *)xmalloc(m * 4), *ev = (uint32_t *)xmalloc(m * 4);
  m = 0;
  for (uint32_t u = 0; u < n; ++u)
    for (uint64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e)
      if (u < col[e]) { eu[m] = u; ev[m] = col[e]; m++; }
  pm_code *seen = NULL;
  uint64_t nseen = 0, cap = 0;
  uint32_t pick[PM_MAXE];
  /* every M-subset of the edges, in lexicographic order */
  if (M <= m) {
    for (uint32_t t = 0; t < M; ++t) pick[t] = t;
    for (;;) {
      /* the subset's vertices, relabelled 0..nv-1 */
      uint32_t vs[2 * PM_MAXE], nv = 0;
      pm_graph p;
      memset(&p, 0, sizeof(p));
      for (uint32_t t = 0; t < M; ++t) {
        uint32_t ends[2] = {eu[pick[t]], ev[pick[t]]}, id[2];
        for (int s = 0; s < 2; ++s) {
          uint32_t q = 0;
          while (q < nv && vs[q] != ends[s]) ++q;
          if (q == nv) vs[nv++] = ends[s];
          id[s] = q;
        }
        if (nv <= PM_MAXV) p.adj[id[0]][id[1]] = p.adj[id[1]][id[0]] = 1;
      }
      if (nv <= PM_MAXV) {
        p.nv = nv;
        p.ne = M;
        for (uint32_t q = 0; q < nv; ++q) p.lab[q] = lab[vs[q]];
        /* connected? */
        uint32_t reach = 1, grow = 1;
        while (grow) {
          grow = 0;
          for (uint32_t a = 0; a < nv; ++a)
            if (reach >> a & 1)
              for (uint32_t b = 0; b < nv; ++b)
                if (p.adj[a][b] && !(reach >> b & 1)) { reach |= 1u << b; grow = 1; }
        }
        if (reach == (1u << nv) - 1) {
          pm_code c;
          pm_min_code(&p, &c);
          int dup = 0;
          for (uint64_t s = 0; s < nseen && !dup; ++s) dup = pm_code_cmp(&seen[s], &c) == 0;
          if (!dup) {
            if (nseen == cap) {
              cap = cap ? 2 * cap : 64;
              seen = (pm_code *)realloc(seen, cap * sizeof(pm_code));
            }
            seen[nseen++] = c;
          }
        }
      }
      /* next subset */
      int t = (int)M - 1;
      while (t >= 0 && pick[t] == m - M + (uint32_t)t) --t;
      if (t < 0) break;
      pick[t]++;
      for (uint32_t s = (uint32_t)t + 1; s < M; ++s) pick[s] = pick[s - 1] + 1;
    }
  }
  pm_res *R = (pm_res *)xmalloc((uint64_t)k * sizeof(pm_res));
  uint32_t nr = 0;
  for (uint64_t s = 0; s < nseen; ++s) {
    pm_res x;
    x.c = seen[s];
    x.f = pm_support(&G, &seen[s]);
    pm_offer(R, &nr, k, &x);
  }
  pm_write(R, nr, M, support_out, code_out);
  free(R);
  free(seen);
  free(eu);
  free(ev);
  return nr;
}

/* support of one pattern given as a code (4 u32 per edge), by definition */
int64_t oracle_pattern_support(uint32_t n, const uint64_t *row_ptr, const uint32_t *col,
                               const uint8_t *lab, uint32_t ne, const uint32_t *code) {
  graph_t G = {n, row_ptr, col, NULL, lab, NULL, NULL};
  if (ne < 1 || ne > PM_MAXE) return -2;
  pm_code c;
  memset(&c, 0, sizeof(c));
  c.ne = ne;
  for (uint32_t t = 0; t < ne; ++t) {
    c.e[t].i = (uint8_t)code[4 * t]; c.e[t].j = (uint8_t)code[4 * t + 1];
    c.e[t].li = (uint8_t)code[4 * t + 2]; c.e[t].lj = (uint8_t)code[4 * t + 3];
    if (c.e[t].i + 1u > c.nv) c.nv = c.e[t].i + 1u;
    if (c.e[t].j + 1u > c.nv) c.nv = c.e[t].j + 1u;
  }
  return (int64_t)pm_support(&G, &c);
}

/* minimum DFS code of a small labelled graph (nv vertices, edges as pairs) */
int64_t oracle_min_dfs_code(uint32_t nv, const uint8_t *plab, uint32_t ne, const uint32_t *pedges,
                            uint32_t *code_out) {
  if (nv < 2 || nv > PM_MAXV || ne < 1 || ne > PM_MAXE) return -2;
  pm_graph p;
  memset(&p, 0, sizeof(p));
  p.nv = nv;
  p.ne = ne;
  for (uint32_t v = 0; v < nv; ++v) p.lab[v] = plab[v];
  for (uint32_t t = 0; t < ne; ++t) {
    uint32_t a = pedges[2 * t], b = pedges[2 * t + 1];
    if (a >= nv || b >= nv || a == b || p.adj[a][b]) return -2;
    p.adj[a][b] = p.adj[b][a] = 1;
  }
  pm_code c;
  pm_min_code(&p, &c);
  if (c.ne != ne) return -2; /* not connected */
  for (uint32_t t = 0; t < ne; ++t) {
    code_out[4 * t] = c.e[t].i; code_out[4 * t + 1] = c.e[t].j;
    code_out[4 * t + 2] = c.e[t].li; code_out[4 * t + 3] = c.e[t].lj;
  }
  return ne;
}

/*
 * Algorithm 2 (Section 3.3) for top-k frequent patterns, in the paper's
 * order: one-edge subgraphs grouped by pattern (lines 1-8), then groups
 * taken by priority (number of edges, support) (line 10); a group whose
 * pattern has M edges is relevant and offered to R (lines 11-15); a group
 * with support below the k-th result's is dominated (line 16; minimum
 * image-based support never grows when a pattern grows); otherwise every
 * subgraph of the group grows by one edge by pattern-oriented expansion
 * (lines 17-24): rightmost-path extensions of its DFS code, kept only when
 * the new code is minimal, grouped by the new code; groups that are not
 * dominated enter Q (lines 25-27).
 */
typedef struct {
  pm_code c;
  uint64_t f;
  uint32_t *emb; /* count x c.nv data vertices, by code vertex */
  uint64_t count, cap;
} pm_group;

static pm_group *pm_group_new(const pm_code *c) {
  pm_group *G = (pm_group *)calloc(1, sizeof(pm_group));
  G->c = *c;
  return G;
}

static void pm_group_add(pm_group *G, const uint32_t *phi) {
  if (G->count == G->cap) {
    G->cap = G->cap ? 2 * G->cap : 16;
    G->emb = (uint32_t *)realloc(G->emb, G->cap * G->c.nv * sizeof(uint32_t));
    if (!G->emb) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
  }
  memcpy(&G->emb[G->count * G->c.nv], phi, G->c.nv * sizeof(uint32_t));
  G->count++;
}

static void pm_group_free(pm_group *G) {
  free(G->emb);
  free(G);
}

/* minimum image-based support over the group's subgraphs (Listing 2) */
static uint64_t pm_group_support(const pm_group *G, uint32_t n, uint8_t *mark) {
  uint64_t f = UINT64_MAX;
  for (uint32_t v = 0; v < G->c.nv; ++v) {
    uint64_t distinct = 0;
    for (uint64_t s = 0; s < G->count; ++s) {
      uint32_t x = G->emb[s * G->c.nv + v];
      if (!mark[x]) { mark[x] = 1; distinct++; }
    }
    for (uint64_t s = 0; s < G->count; ++s) mark[G->emb[s * G->c.nv + v]] = 0;
    if (distinct < f) f = distinct;
  }
  (void)n;
  return f;
}

int64_t oracle_topk_patterns(uint32_t n, const uint64_t *row_ptr, const uint32_t *col,
                             const uint8_t *lab, uint32_t M, uint32_t k, uint64_t *support_out,
                             uint32_t *code_out, uint64_t *stats_out) {
  graph_t G = {n, row_ptr, col, NULL, lab, NULL, NULL};
  const graph_t *g = &G;
  if (M < 1 || M > PM_MAXE || k == 0) return -2;
  uint8_t *mark = (uint8_t *)calloc(n ? n : 1, 1);
  pm_res *R = (pm_res *)xmalloc((uint64_t)k * sizeof(pm_res));
  uint32_t nr = 0;
  uint64_t st_popped = 0, st_expanded = 0, st_children = 0, st_pruned_pop = 0,
           st_pruned_new = 0, st_nonmin = 0, st_groups = 0;
  pq_t Q = {0};

  /* lines 1-8: one-edge subgraphs (u, v), kept when (0, 1, L(u), L(v)) is
     minimal, i.e. L(u) <= L(v); one group per label pair */
  pm_group **first = (pm_group **)calloc(256 * 256, sizeof(pm_group *));
  for (uint32_t u = 0; u < n; ++u)
    for (uint64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
      uint32_t v = col[e];
      if (lab[u] > lab[v]) continue;
      uint32_t key = lab[u] * 256u + lab[v];
      if (!first[key]) {
        pm_code c;
        memset(&c, 0, sizeof(c));
        c.ne = 1;
        c.nv = 2;
        pm_edge e0 = {0, 1, lab[u], lab[v]};
        c.e[0] = e0;
        first[key] = pm_group_new(&c);
      }
      uint32_t phi[2] = {u, v};
      pm_group_add(first[key], phi);
      st_children++;
    }
  for (uint32_t key = 0; key < 256 * 256; ++key)
    if (first[key]) {
      first[key]->f = pm_group_support(first[key], n, mark);
      int64_t pk[3] = {1, (int64_t)first[key]->f, 0};
      pq_insert(&Q, pk, first[key]);
      st_groups++;
    }
  free(first);

  /* lines 9-27 */
  pm_group **kids = NULL;
  uint32_t nkids = 0;
  while (Q.n > 0) {
    pm_group *S = (pm_group *)pq_remove_max(&Q);
    st_popped++;
    if (S->c.ne == M) {
      pm_res x;
      x.f = S->f;
      x.c = S->c;
      pm_offer(R, &nr, k, &x);
    }
    if (nr == k && S->f < R[k - 1].f) { st_pruned_pop++; pm_group_free(S); continue; }
    if (S->c.ne == M) { pm_group_free(S); continue; } /* expandable() is false at M edges */
    st_expanded++;
    const pm_code *c = &S->c;
    const uint32_t nv = c->nv, rm = nv - 1;
    /* the rightmost path: rm and its discoverers back to 0 */
    uint32_t par[PM_MAXV], onpath[PM_MAXV] = {0}, path[PM_MAXV], np = 0;
    for (uint32_t t = 0; t < c->ne; ++t) if (c->e[t].i < c->e[t].j) par[c->e[t].j] = c->e[t].i;
    for (uint32_t x = rm;; x = par[x]) { path[np++] = x; onpath[x] = 1; if (x == 0) break; }
    uint8_t has[PM_MAXV][PM_MAXV] = {{0}};
    for (uint32_t t = 0; t < c->ne; ++t) has[c->e[t].i][c->e[t].j] = has[c->e[t].j][c->e[t].i] = 1;
    /* child groups by the new code edge: backward to x -> x; forward from
       path vertex x with label l -> nv + x * 256 + l */
    uint32_t nk = nv + nv * 256;
    if (nk > nkids) { kids = (pm_group **)realloc(kids, nk * sizeof(pm_group *)); nkids = nk; }
    memset(kids, 0, nk * sizeof(pm_group *));
    for (uint64_t s = 0; s < S->count; ++s) {
      const uint32_t *phi = &S->emb[s * nv];
      uint32_t child[PM_MAXV];
      memcpy(child, phi, nv * sizeof(uint32_t));
      /* backward edges from the rightmost vertex */
      for (uint32_t x = 0; x < rm; ++x) {
        if (!onpath[x] || has[rm][x]) continue;
        if (!is_adjacent(g, phi[rm], phi[x])) continue;
        if (!kids[x]) {
          pm_code c2 = *c;
          pm_edge b = {(uint8_t)rm, (uint8_t)x, lab[phi[rm]], lab[phi[x]]};
          c2.e[c2.ne++] = b;
          kids[x] = pm_group_new(&c2);
        }
        pm_group_add(kids[x], child);
      }
      /* forward edges from every vertex of the rightmost path */
      for (uint32_t q = 0; q < np; ++q) {
        uint32_t x = path[q], dx = phi[x];
        for (uint64_t e = row_ptr[dx]; e < row_ptr[dx + 1]; ++e) {
          uint32_t w = col[e];
          int used = 0;
          for (uint32_t y = 0; y < nv && !used; ++y) used = phi[y] == w;
          if (used) continue;
          uint32_t key = nv + x * 256u + lab[w];
          if (!kids[key]) {
            pm_code c2 = *c;
            pm_edge f = {(uint8_t)x, (uint8_t)nv, lab[dx], lab[w]};
            c2.e[c2.ne++] = f;
            c2.nv = nv + 1;
            kids[key] = pm_group_new(&c2);
          }
          child[nv] = w;
          pm_group_add(kids[key], child);
        }
      }
    }
    for (uint32_t key = 0; key < nk; ++key) {
      pm_group *C = kids[key];
      if (!C) continue;
      if (!pm_is_min(&C->c)) { st_nonmin++; pm_group_free(C); continue; }
      /* subgraphs are constructed only for minimal codes: count those */
      st_children += C->count;
      C->f = pm_group_support(C, n, mark);
      if (nr == k && C->f < R[k - 1].f) { st_pruned_new++; pm_group_free(C); continue; }
      int64_t pk[3] = {(int64_t)C->c.ne, (int64_t)C->f, 0};
      pq_insert(&Q, pk, C);
      st_groups++;
    }
    pm_group_free(S);
  }
  free(kids);
  free(Q.a);
  free(mark);
  pm_write(R, nr, M, support_out, code_out);
  free(R);
  if (stats_out) {
    stats_out[0] = st_popped; stats_out[1] = st_expanded; stats_out[2] = st_children;
    stats_out[3] = st_pruned_new; stats_out[4] = st_pruned_pop; stats_out[5] = st_nonmin;
    stats_out[6] = st_groups;
  }
  return nr;
}
