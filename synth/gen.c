/*
 * Seeded synthetic graph generators.
 *
 * These produce the inputs that both the CPU oracle and the GPU engine are
 * run on.  Nothing here computes any part of the subgraph-discovery method:
 * the file only draws random graphs, weights and labels and returns them as
 * CSR arrays.
 *
 * Randomness: every draw is splitmix64 used as a counter-based generator.
 * Value number i of a stream with seed s is mix64(s + (i + 1) * GAMMA),
 * where mix64 is the splitmix64 finaliser (Steele, Lea, Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014).  A stream seed
 * is mix64(master ^ stream_id).  Because a draw depends only on its index,
 * results do not depend on thread count or scheduling.
 *
 * Output convention (all generators): an undirected simple graph on
 * vertices 0..n-1 as CSR with row_ptr[n+1] (uint64) and col[nnz] (uint32),
 * every row strictly increasing, no self loops, symmetric.  Arrays are
 * malloc'ed here and released by the caller with synth_free().
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* value number i of the stream with seed s */
static inline uint64_t draw(uint64_t s, uint64_t i) { return mix64(s + (i + 1) * GAMMA); }

/* uniform double in [0,1) from the top 53 bits */
static inline double unif(uint64_t s, uint64_t i) {
  return (double)(draw(s, i) >> 11) * (1.0 / 9007199254740992.0);
}

/* uniform integer in [0, m) by 128-bit multiply-shift (Lemire) */
static inline uint64_t below(uint64_t s, uint64_t i, uint64_t m) {
  return (uint64_t)(((unsigned __int128)draw(s, i) * m) >> 64);
}

uint64_t synth_stream_seed(uint64_t master, uint64_t stream_id) { return mix64(master ^ stream_id); }
uint64_t synth_draw(uint64_t s, uint64_t i) { return draw(s, i); }

void synth_free(void *p) { free(p); }

/* ---------------------------------------------------------------- */
/* edge-list -> CSR                                                  */
/* ---------------------------------------------------------------- */

/* LSD radix sort of 64-bit keys, 16 bits per pass */
static void radix_sort_u64(uint64_t *a, uint64_t n, uint64_t *tmp) {
  uint64_t *src = a, *dst = tmp;
  for (int pass = 0; pass < 4; ++pass) {
    int sh = pass * 16;
    uint64_t *cnt = (uint64_t *)calloc(65536, sizeof(uint64_t));
    for (uint64_t i = 0; i < n; ++i) cnt[(src[i] >> sh) & 0xFFFF]++;
    uint64_t run = 0;
    for (int b = 0; b < 65536; ++b) { uint64_t c = cnt[b]; cnt[b] = run; run += c; }
    for (uint64_t i = 0; i < n; ++i) dst[cnt[(src[i] >> sh) & 0xFFFF]++] = src[i];
    free(cnt);
    uint64_t *t = src; src = dst; dst = t;
  }
  /* four passes: result is back in a */
}

/*
 * keys: packed (u << 32 | v) for undirected pairs, in any order, possibly
 * with duplicates, both orientations allowed, self loops allowed (dropped).
 * Builds the symmetric CSR.  Consumes (frees) keys.
 */
static int build_csr(uint32_t n, uint64_t *keys, uint64_t m, uint64_t **row_ptr_out,
                     uint32_t **col_out, uint64_t *nnz_out) {
  uint64_t cap = 2 * m;
  uint64_t *all = (uint64_t *)malloc((cap ? cap : 1) * sizeof(uint64_t));
  if (!all) return -1;
  uint64_t t = 0;
  for (uint64_t i = 0; i < m; ++i) {
    uint32_t u = (uint32_t)(keys[i] >> 32), v = (uint32_t)keys[i];
    if (u == v) continue;
    all[t++] = ((uint64_t)u << 32) | v;
    all[t++] = ((uint64_t)v << 32) | u;
  }
  free(keys);
  uint64_t *tmp = (uint64_t *)malloc((t ? t : 1) * sizeof(uint64_t));
  if (!tmp) { free(all); return -1; }
  radix_sort_u64(all, t, tmp);
  free(tmp);
  uint64_t w = 0;
  for (uint64_t i = 0; i < t; ++i)
    if (i == 0 || all[i] != all[i - 1]) all[w++] = all[i];
  uint64_t *rp = (uint64_t *)calloc((uint64_t)n + 1, sizeof(uint64_t));
  uint32_t *col = (uint32_t *)malloc((w ? w : 1) * sizeof(uint32_t));
  if (!rp || !col) { free(all); free(rp); free(col); return -1; }
  for (uint64_t i = 0; i < w; ++i) {
    rp[(all[i] >> 32) + 1]++;
    col[i] = (uint32_t)all[i];
  }
  for (uint32_t v = 0; v < n; ++v) rp[v + 1] += rp[v];
  free(all);
  *row_ptr_out = rp; *col_out = col; *nnz_out = w;
  return 0;
}

/* seeded Fisher-Yates permutation of 0..n-1 */
static uint32_t *permutation(uint32_t n, uint64_t s) {
  uint32_t *p = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
  if (!p) return NULL;
  for (uint32_t i = 0; i < n; ++i) p[i] = i;
  for (uint32_t i = n; i > 1; --i) {
    uint32_t j = (uint32_t)below(s, i - 1, i);
    uint32_t t = p[i - 1]; p[i - 1] = p[j]; p[j] = t;
  }
  return p;
}

uint32_t *synth_permutation(uint32_t n, uint64_t s) { return permutation(n, s); }

/*
 * Plants n_cliques vertex-disjoint cliques with sizes uniform in [lo, hi].
 * The member sets are consecutive chunks of a seeded permutation of the
 * vertices.  Appends their pairs to *keys (realloc'ed), and writes the
 * member lists (sorted ascending per clique) to planted[] with offsets
 * planted_off[n_cliques+1] when those are non-NULL.
 */
static int plant(uint32_t n, uint32_t n_cliques, uint32_t lo, uint32_t hi, uint64_t s_perm,
                 uint64_t s_size, uint64_t **keys, uint64_t *m, uint32_t **planted_out,
                 uint64_t **planted_off_out) {
  uint32_t *perm = permutation(n, s_perm);
  if (!perm) return -1;
  uint64_t *off = (uint64_t *)malloc(((uint64_t)n_cliques + 1) * sizeof(uint64_t));
  off[0] = 0;
  for (uint32_t c = 0; c < n_cliques; ++c)
    off[c + 1] = off[c] + lo + below(s_size, c, (uint64_t)hi - lo + 1);
  if (off[n_cliques] > n) { free(perm); free(off); return -2; }
  uint64_t extra = 0;
  for (uint32_t c = 0; c < n_cliques; ++c) {
    uint64_t sz = off[c + 1] - off[c];
    extra += sz * (sz - 1) / 2;
  }
  uint64_t *k2 = (uint64_t *)realloc(*keys, (*m + extra + 1) * sizeof(uint64_t));
  if (!k2) { free(perm); free(off); return -1; }
  *keys = k2;
  uint32_t *members = (uint32_t *)malloc((off[n_cliques] + 1) * sizeof(uint32_t));
  for (uint32_t c = 0; c < n_cliques; ++c) {
    for (uint64_t i = off[c]; i < off[c + 1]; ++i)
      for (uint64_t j = i + 1; j < off[c + 1]; ++j)
        (*keys)[(*m)++] = ((uint64_t)perm[i] << 32) | perm[j];
    /* sorted member list: insertion sort (sizes are small) */
    for (uint64_t i = off[c]; i < off[c + 1]; ++i) {
      uint32_t x = perm[i];
      uint64_t j = i;
      while (j > off[c] && members[j - 1] > x) { members[j] = members[j - 1]; --j; }
      members[j] = x;
    }
  }
  free(perm);
  if (planted_out) *planted_out = members; else free(members);
  if (planted_off_out) *planted_off_out = off; else free(off);
  return 0;
}

/* ---------------------------------------------------------------- */
/* Erdos-Renyi G(n, p) with planted cliques                          */
/* ---------------------------------------------------------------- */

/*
 * Each of the C(n,2) pairs (i<j) is an edge with probability p, decided by
 * draw number (pair index) of stream s_edges.  Then planted cliques are added.
 */
int synth_er_planted(uint32_t n, double p, uint32_t n_cliques, uint32_t lo, uint32_t hi,
                     uint64_t master, uint64_t **row_ptr, uint32_t **col, uint64_t *nnz,
                     uint32_t **planted, uint64_t **planted_off) {
  uint64_t s_edges = synth_stream_seed(master, 1);
  uint64_t s_perm = synth_stream_seed(master, 2);
  uint64_t s_size = synth_stream_seed(master, 3);
  uint64_t cap = 1024, m = 0;
  uint64_t *keys = (uint64_t *)malloc(cap * sizeof(uint64_t));
  uint64_t idx = 0;
  for (uint32_t i = 0; i < n; ++i)
    for (uint32_t j = i + 1; j < n; ++j, ++idx) {
      if (unif(s_edges, idx) < p) {
        if (m == cap) { cap *= 2; keys = (uint64_t *)realloc(keys, cap * sizeof(uint64_t)); }
        keys[m++] = ((uint64_t)i << 32) | j;
      }
    }
  int rc = plant(n, n_cliques, lo, hi, s_perm, s_size, &keys, &m, planted, planted_off);
  if (rc) { free(keys); return rc; }
  return build_csr(n, keys, m, row_ptr, col, nnz);
}

/* ---------------------------------------------------------------- */
/* Chung-Lu power-law graph                                          */
/* ---------------------------------------------------------------- */

/*
 * Expected degrees w_i = min(cap, c * (i+1)^(-1/(beta-1))), with c found by
 * bisection so that sum_i w_i = 2 * m_target.  Pair (u,v) is an edge with
 * probability min(1, w_u w_v / sum w), sampled in O(n + m) with the
 * skipping method of Miller and Hagberg ("Efficient generation of networks
 * with given expected degrees", WAW 2011), which needs w non-increasing
 * (it is, by construction).  Vertex u's draws come from stream
 * mix64(s_edges ^ u), so rows are independent.  Then planted cliques are
 * added and the ids are shuffled by a seeded permutation.
 */
int synth_chung_lu(uint32_t n, double beta, double m_target, double cap, uint32_t n_cliques,
                   uint32_t lo, uint32_t hi, uint64_t master, uint64_t **row_ptr,
                   uint32_t **col, uint64_t *nnz, double *c_out) {
  double ex = -1.0 / (beta - 1.0);
  double target = 2.0 * m_target;
  double clo = 0.0, chi = 1.0;
  double *w = (double *)malloc((uint64_t)n * sizeof(double));
  for (;;) {
    double s = 0;
    for (uint32_t i = 0; i < n; ++i) s += fmin(cap, chi * pow((double)i + 1.0, ex));
    if (s >= target) break;
    chi *= 2.0;
  }
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (clo + chi), s = 0;
    for (uint32_t i = 0; i < n; ++i) s += fmin(cap, mid * pow((double)i + 1.0, ex));
    if (s < target) clo = mid; else chi = mid;
  }
  double c = 0.5 * (clo + chi), S = 0;
  for (uint32_t i = 0; i < n; ++i) { w[i] = fmin(cap, c * pow((double)i + 1.0, ex)); S += w[i]; }
  if (c_out) *c_out = c;
  uint64_t s_edges = synth_stream_seed(master, 11);
  uint64_t cap_k = (uint64_t)(m_target * 1.2) + 1024, m = 0;
  uint64_t *keys = (uint64_t *)malloc(cap_k * sizeof(uint64_t));
  for (uint32_t u = 0; u + 1 < n; ++u) {
    uint64_t su = mix64(s_edges ^ (uint64_t)u), j = 0;
    uint64_t v = (uint64_t)u + 1;
    double p = fmin(w[u] * w[v] / S, 1.0);
    while (v < n && p > 0) {
      if (p != 1.0) {
        double r = unif(su, j++);
        if (r <= 0.0) r = 1e-300;
        v += (uint64_t)floor(log(r) / log1p(-p));
      }
      if (v < n) {
        double q = fmin(w[u] * w[v] / S, 1.0);
        double r = unif(su, j++);
        if (r < q / p) {
          if (m == cap_k) { cap_k *= 2; keys = (uint64_t *)realloc(keys, cap_k * sizeof(uint64_t)); }
          keys[m++] = ((uint64_t)u << 32) | (uint32_t)v;
        }
        p = q;
        v += 1;
      }
    }
  }
  free(w);
  int rc = plant(n, n_cliques, lo, hi, synth_stream_seed(master, 12), synth_stream_seed(master, 13),
                 &keys, &m, NULL, NULL);
  if (rc) { free(keys); return rc; }
  uint32_t *perm = permutation(n, synth_stream_seed(master, 14));
  for (uint64_t i = 0; i < m; ++i) {
    uint32_t a = perm[keys[i] >> 32], b = perm[(uint32_t)keys[i]];
    keys[i] = ((uint64_t)a << 32) | b;
  }
  free(perm);
  return build_csr(n, keys, m, row_ptr, col, nnz);
}

/* ---------------------------------------------------------------- */
/* R-MAT                                                             */
/* ---------------------------------------------------------------- */

/*
 * R-MAT (Chakrabarti, Zhan, Faloutsos, SDM 2004): n = 2^scale vertices and
 * edge_factor * n generated tuples.  Tuple t descends `scale` levels; at
 * level l it picks quadrant (0,0),(0,1),(1,0),(1,1) with probabilities
 * a, b, c, 1-a-b-c using draw number t*scale+l.  Self loops and duplicates
 * are dropped, the result is symmetrised, and ids are shuffled by a seeded
 * permutation.
 */
int synth_rmat(uint32_t scale, uint32_t edge_factor, double a, double b, double c, uint64_t master,
               uint64_t **row_ptr, uint32_t **col, uint64_t *nnz) {
  uint32_t n = 1u << scale;
  uint64_t T = (uint64_t)edge_factor << scale;
  uint64_t s = synth_stream_seed(master, 21);
  uint64_t *keys = (uint64_t *)malloc(T * sizeof(uint64_t));
  if (!keys) return -1;
  uint32_t *perm = permutation(n, synth_stream_seed(master, 22));
  double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
  for (uint64_t t = 0; t < T; ++t) {
    uint32_t u = 0, v = 0;
    for (uint32_t l = 0; l < scale; ++l) {
      double r = unif(s, t * scale + l);
      uint32_t bu = 0, bv = 0;
      if (r < a) { }
      else if (r < ab) bv = 1;
      else if (r < abc) bu = 1;
      else { bu = 1; bv = 1; }
      u = (u << 1) | bu;
      v = (v << 1) | bv;
    }
    keys[t] = ((uint64_t)perm[u] << 32) | perm[v];
  }
  free(perm);
  return build_csr(n, keys, T, row_ptr, col, nnz);
}

/* ---------------------------------------------------------------- */
/* weights and labels                                                */
/* ---------------------------------------------------------------- */

/* vertex weights uniform in [lo, hi], draw number = vertex id */
void synth_vertex_weights(uint32_t n, int32_t lo, int32_t hi, uint64_t s, int32_t *out) {
  for (uint32_t v = 0; v < n; ++v) out[v] = lo + (int32_t)below(s, v, (uint64_t)(hi - lo + 1));
}

/*
 * Edge weights uniform in [lo, hi], one per undirected edge {u,v}: the draw
 * index is the packed pair (min << 32 | max), so both CSR directions get the
 * same value.
 */
void synth_edge_weights(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, int32_t lo,
                        int32_t hi, uint64_t s, int32_t *out) {
#pragma omp parallel for schedule(dynamic, 4096)
  for (uint32_t u = 0; u < n; ++u)
    for (uint64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
      uint32_t v = col[e];
      uint64_t key = u < v ? (((uint64_t)u << 32) | v) : (((uint64_t)v << 32) | u);
      out[e] = lo + (int32_t)below(s, key, (uint64_t)(hi - lo + 1));
    }
}

/*
 * iid labels from a truncated Zipf law over n_labels values:
 * P(l) proportional to (l+1)^(-s), by inverse CDF of draw number v.
 */
void synth_zipf_labels(uint32_t n, uint32_t n_labels, double s_exp, uint64_t s, uint8_t *out) {
  double cdf[256];
  double z = 0;
  for (uint32_t l = 0; l < n_labels; ++l) z += pow((double)l + 1.0, -s_exp);
  double run = 0;
  for (uint32_t l = 0; l < n_labels; ++l) { run += pow((double)l + 1.0, -s_exp) / z; cdf[l] = run; }
  cdf[n_labels - 1] = 1.0;
  for (uint32_t v = 0; v < n; ++v) {
    double r = unif(s, v);
    uint32_t l = 0;
    while (l + 1 < n_labels && r >= cdf[l]) ++l;
    out[v] = (uint8_t)l;
  }
}
