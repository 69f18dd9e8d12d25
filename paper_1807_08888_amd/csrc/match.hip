// Top-k labelled subgraph matching on the GPU.
//
// The paper's basic computational model (Algorithm 1, Section 3.2) with the
// subgraph-isomorphism user functions of Section 4.3, scored by the sum of
// matched edge weights, or by the sum of the matched vertices' degrees (the
// paper's example, bounded with its multi-hop index; see below):
//
//   targeted expansion  a partial match grows by one pattern vertex at a
//                       time (in a fixed matching order), taking only data
//                       vertices with the right label that are adjacent to
//                       every already-matched pattern neighbour (Ullmann-
//                       style refinement) and distinct from the matched ones;
//   bound               score + an upper bound for every pattern edge not yet
//                       matched, from a one-hop index (the Section 4.3 index
//                       at hop 1): max edge weight from a matched vertex to
//                       a label, or from any vertex of one label to another;
//   priority            (matched vertices, bound): the deepest level first,
//                       highest bound first within it;
//   dominated           bound < score of the k-th result (strict).
//
// Degree score: a unit subgraph {v} scores deg(v), a child adds the
// degree of its new vertex, and the bound is the score plus, for every
// unmatched pattern vertex u, the multi-hop index entry of the seed
// mu(order[0]) for label(u) at hop(u), u's distance from order[0].
//
// Matches are non-induced.  Embeddings with the same image are one result:
// symmetry-breaking constraints mu(i) < mu(j), for j in the orbit of i under
// the automorphisms fixing 0..i-1, keep exactly the lexicographically
// smallest tuple of each orbit.
#include <algorithm>
#include <climits>
#include <cstring>
#include <numeric>

#include "device_common.h"

namespace nuri {
namespace {

constexpr int QM = NURI_MAX_PATTERN;

struct MRec {  // 64 B partial match
  long long score;
  long long bound;
  uint32_t mu[QM];    // data vertex (original id) per pattern vertex; valid if matched
  uint32_t qid;
  uint32_t depth;     // matched vertices: order[0..depth-1]
  uint32_t nchild;    // upper bound on its children (smallest anchor segment)
  uint32_t pad;
};
static_assert(sizeof(MRec) == 64, "match record must stay 64 bytes");

// mu[b] for a pattern vertex b known only at run time
__device__ inline uint32_t mu_at(const MRec &r, uint32_t b) { return r.mu[b]; }

struct MPlan {  // per query pattern plan
  uint32_t q, k;
  uint8_t label[QM];
  uint8_t order[QM];  // matching order
  uint8_t pos[QM];    // position of each pattern vertex in the order
  uint8_t nbr[QM];    // pattern adjacency bitmasks
  uint8_t sb_lt[QM];  // sb_lt[a] bit b: a result needs mu(a) < mu(b)
  int32_t pmx[QM][QM];  // max data edge weight for the label pair of pattern edge {a,b}
  long long rest0;    // bound contribution of edges not touching order[0], all unmatched
  uint8_t hop[QM];    // distance from order[0] in the pattern
  uint32_t degree;    // 1: degree score, 0: edge-weight score
  uint32_t max_hop;
};

struct MView {
  const uint64_t *orow;
  const uint32_t *lcol;
  const int32_t *lew;
  const uint32_t *loff;
  const int32_t *best;
  const uint32_t *lab_vert;
  const int32_t *hidx[QM - 1];  // multi-hop index, per hop: [v * 16 + label]
};

__device__ inline long long vdeg(const MView &m, uint32_t v) {
  return (long long)(m.orow[v + 1] - m.orow[v]);
}

// multi-hop index entry of seed v for label l within h >= 1 hops
__device__ inline int32_t hop_entry(const MView &m, uint32_t h, uint32_t v, uint32_t l) {
  return m.hidx[h - 1][(u64)v * NURI_MAX_LABELS + l];
}

struct MCfg {  // per query, per step
  MRec *hdr;
  uint32_t out_hdr, hdr_cap;
  uint32_t prio, pad;  // NURI_PRIORITY_*: no pruning for NONE
};

// the k-th score the search prunes against (none in the Nuri-NP order)
__device__ inline long long mprune_theta(const MCfg &c, const QRes &r) {
  return c.prio == NURI_PRIORITY_NONE ? LLONG_MIN : r.theta;
}

struct MStep {  // per query, this step's counters
  unsigned int n_out, n_kept, overflow, cand_n;
  u64 out_cost;        // sum of nchild over appended records
  long long out_max_bound;
  u64 out_max_cost;
  long long cand_max;  // best score among this step's complete matches
};

struct CPre {  // per query: score histogram window for the candidate prefilter
  long long top;
  uint32_t shift;
  int tbin;  // candidates in bins >= tbin are kept
};

// per query, cumulative counters (kCtrSlots copies, one cache line each)
struct alignas(128) MCtr {
  u64 popped, expanded, children, pruned_pop, pruned_new, leaves, offered, logical_bytes;
};

struct MSeg {
  uint32_t qid, begin, count, take_all;
  uint32_t shift, temp_off;
  long long top;
  u64 max_records, max_children, maxcost;
};

__device__ inline uint32_t seg_len(const MView &m, uint32_t v, uint32_t l) {
  const uint32_t *lo = m.loff + (u64)v * 17;
  return lo[l + 1] - lo[l];
}

// index of x in the label-l segment of row v, or -1
__device__ inline long long seg_find(const MView &m, uint32_t v, uint32_t l, uint32_t x) {
  const uint32_t *lo = m.loff + (u64)v * 17;
  u64 a = m.orow[v] + lo[l], z = m.orow[v] + lo[l + 1];
  while (a < z) {
    u64 mid = (a + z) >> 1;
    if (m.lcol[mid] < x) a = mid + 1; else z = mid;
  }
  return (a < m.orow[v] + lo[l + 1] && m.lcol[a] == x) ? (long long)a : -1ll;
}

// upper bound on the children of a record whose next pattern vertex is a
__device__ inline uint32_t child_bound(const MView &m, const MPlan &P, const MRec &r) {
  if (r.depth >= P.q) return 0;
  const uint32_t a = P.order[r.depth];
  uint32_t best = 0xFFFFFFFFu;
  for (uint32_t i = 0; i < r.depth; ++i) {
    const uint32_t b = P.order[i];
    if (P.nbr[a] >> b & 1) {
      uint32_t s = seg_len(m, mu_at(r, b), P.label[a]);
      best = s < best ? s : best;
    }
  }
  return best == 0xFFFFFFFFu ? 0 : best;
}

// ------------------------------------------------------------------
// unit subgraphs: every vertex with the label of order[0] (lines 1-3)
// grid: (x, index into the list of slots being started)
// ------------------------------------------------------------------
__global__ void k_match_roots(MView m, const MPlan *plans, const uint64_t *lab_off, MCfg *cfg,
                              MStep *ms, const uint32_t *slots) {
  const uint32_t q = slots[blockIdx.y];
  const MPlan &P = plans[q];
  const uint32_t a0 = P.order[0];
  const uint32_t l0 = P.label[a0];
  const u64 b = lab_off[l0], e = lab_off[l0 + 1];
  for (u64 i = b + blockIdx.x * (u64)blockDim.x + threadIdx.x; i < e;
       i += (u64)gridDim.x * blockDim.x) {
    const uint32_t v = m.lab_vert[i];
    long long bound = P.rest0, score = 0;
    bool ok = true;
    if (P.degree) {
      score = vdeg(m, v);
      bound = score;
      for (uint32_t u = 0; u < P.q; ++u)
        if (u != a0) {
          const int32_t x = hop_entry(m, P.hop[u], v, P.label[u]);
          ok &= x > 0;
          bound += x;
        }
    } else {
      for (uint32_t u = 0; u < P.q; ++u)
        if (P.nbr[a0] >> u & 1) {
          int32_t w = m.best[(u64)v * NURI_MAX_LABELS + P.label[u]];
          ok &= w > 0;
          bound += w;
        }
    }
    if (!ok) continue;
    MRec r;
    r.score = score;
    r.bound = bound;
    for (int t = 0; t < QM; ++t) r.mu[t] = 0;
    r.mu[a0] = v;
    r.qid = q;
    r.depth = 1;
    r.nchild = child_bound(m, P, r);
    r.pad = 0;
    if (r.nchild == 0 && P.q > 1) continue;
    unsigned int slot = atomicAdd(&ms[q].n_out, 1u);
    if (slot < cfg[q].hdr_cap) {
      cfg[q].hdr[slot] = r;
      atomicAdd(&ms[q].out_cost, (u64)r.nchild);
      atomicMax(&ms[q].out_max_bound, r.bound);
      atomicMax(&ms[q].out_max_cost, (u64)r.nchild);
    } else {
      atomicAdd(&ms[q].overflow, 1u);
    }
  }
}

// ------------------------------------------------------------------
// select (as for cliques): histogram of bounds, threshold, partition
// ------------------------------------------------------------------
__global__ void __launch_bounds__(256)
    k_msel_hist(const MSeg *segs, const MCfg *cfg, const QRes *res, unsigned int *hist,
                u64 *hcost) {
  __shared__ unsigned int s_h[kBins];
  __shared__ u64 s_c[kBins];
  const uint32_t s = blockIdx.y;
  const MSeg sg = segs[s];
  if (sg.take_all) return;
  for (int b = threadIdx.x; b < kBins; b += blockDim.x) {
    s_h[b] = 0;
    s_c[b] = 0;
  }
  __syncthreads();
  const long long theta = mprune_theta(cfg[sg.qid], res[sg.qid]);
  const MRec *h = cfg[sg.qid].hdr + sg.begin;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < sg.count;
       i += gridDim.x * blockDim.x) {
    const long long bound = h[i].bound;
    if (bound < theta) continue;
    int b = bin_of(bound, sg.top, sg.shift);
    atomicAdd(&s_h[b], 1u);
    atomicAdd(&s_c[b], (u64)h[i].nchild);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kBins; b += blockDim.x)
    if (s_h[b]) {
      atomicAdd(&hist[(size_t)s * kBins + b], s_h[b]);
      atomicAdd(&hcost[(size_t)s * kBins + b], s_c[b]);
    }
}

__global__ void __launch_bounds__(kSelThreads)
    k_msel_thresh(const MSeg *segs, uint32_t nseg, unsigned int *hist, u64 *hcost, int *thr,
                  unsigned int *quota) {
  const uint32_t s = blockIdx.x;
  if (s >= nseg) return;
  const MSeg sg = segs[s];
  if (sg.take_all) return;
  unsigned int *h = hist + (size_t)s * kBins;
  u64 *hc = hcost + (size_t)s * kBins;
  const SelLimits lim{sg.max_records, sg.max_children, ~0ull, 0, sg.maxcost};
  block_select_threshold(h, hc, lim, &thr[s], &quota[s]);
  __syncthreads();
  for (int b = threadIdx.x; b < kBins; b += blockDim.x) {
    h[b] = 0;
    hc[b] = 0;
  }
}

__global__ void k_msel_part(const MSeg *segs, const MCfg *cfg, const QRes *res, const int *thr,
                            const unsigned int *quota, unsigned int *taken, MRec *batch,
                            StepHdr *hdr, MRec *temp, unsigned int *temp_count, MCtr *ctr) {
  const uint32_t s = blockIdx.y;
  const MSeg sg = segs[s];
  const long long theta = mprune_theta(cfg[sg.qid], res[sg.qid]);
  const MRec *h = cfg[sg.qid].hdr + sg.begin;
  const int t = sg.take_all ? -1 : thr[s];
  const unsigned int qt = sg.take_all ? 0 : quota[s];
  unsigned int pruned = 0;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < sg.count;
       i += gridDim.x * blockDim.x) {
    const MRec c = h[i];
    int where;
    if (c.bound < theta) {
      where = 3;
    } else if (sg.take_all) {
      where = 1;
    } else {
      int b = bin_of(c.bound, sg.top, sg.shift);
      if (b > t) where = 1;
      else if (b < t) where = 2;
      else where = atomicAdd(&taken[s], 1u) < qt ? 1 : 2;
    }
    if (where == 1) batch[atomicAdd(&hdr->batch_count, 1u)] = c;
    else if (where == 2) temp[sg.temp_off + atomicAdd(&temp_count[s], 1u)] = c;
    else ++pruned;
  }
  if (pruned) {
    MCtr &C = ctr[sg.qid * kCtrSlots + (blockIdx.x & (kCtrSlots - 1))];
    atomicAdd(&C.popped, (u64)pruned);
    atomicAdd(&C.pruned_pop, (u64)pruned);
  }
}

__global__ void k_mcopy_back(const MSeg *segs, const MCfg *cfg, const MRec *temp,
                             const unsigned int *temp_count, MStep *ms) {
  const uint32_t s = blockIdx.y;
  const MSeg sg = segs[s];
  const unsigned int kept = sg.take_all ? 0u : temp_count[s];
  MRec *h = cfg[sg.qid].hdr + sg.begin;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < kept; i += gridDim.x * blockDim.x)
    h[i] = temp[sg.temp_off + i];
  if (blockIdx.x == 0 && threadIdx.x == 0) ms[sg.qid].n_kept = kept;
}

// ------------------------------------------------------------------
// expand (Algorithm 1, lines 11-16)
// ------------------------------------------------------------------
// One wavefront per record; lanes walk the candidates of the smallest
// label segment among the matched neighbours of the next pattern vertex a
// (coalesced reads of ids and weights), and test each candidate against
// the other matched neighbours by binary search in their label-a segments.
//
// A hub's label segment can hold tens of thousands of ids, and one
// wavefront walking it alone would keep a launch running long after the
// rest of the device is idle.  So a wavefront walks at most kMatchChunk
// candidates of its record; the rest of a longer segment is cut into
// chunks of kMatchChunk that k_match_expand_big shares out between all its
// wavefronts.
constexpr int kMatchWaves = 4;
constexpr uint32_t kMatchChunk = 2048;
constexpr uint32_t kBigBlocks = 1024;

// what a wavefront needs to walk candidates of one record
struct MWork {
  uint32_t a, la, anchor, alen;
  u64 base;          // first entry of the anchor's label-la segment
  long long bound0;  // record bound without the terms the candidate replaces
  bool last;         // children are complete matches
};

__device__ inline MWork match_work(const MView &m, const MPlan &P, const MRec &p) {
  MWork w;
  w.a = P.order[p.depth];
  w.la = P.label[w.a];
  // anchor: the matched neighbour of a with the shortest label-la segment
  w.anchor = QM;
  w.alen = 0xFFFFFFFFu;
  for (uint32_t i = 0; i < p.depth; ++i) {
    const uint32_t b = P.order[i];
    if (P.nbr[w.a] >> b & 1) {
      uint32_t s = seg_len(m, mu_at(p, b), w.la);
      if (s < w.alen) {
        w.alen = s;
        w.anchor = b;
      }
    }
  }
  if (w.anchor == QM) w.alen = 0;  // cannot happen for a connected pattern
  const uint32_t av = w.anchor == QM ? 0 : mu_at(p, w.anchor);
  w.base = m.orow[av] + m.loff[(u64)av * 17 + w.la];
  w.last = p.depth + 1 == P.q;
  w.bound0 = p.bound;
  if (P.degree) {
    // a's index term is replaced by the candidate's degree
    w.bound0 -= hop_entry(m, P.hop[w.a], mu_at(p, P.order[0]), w.la);
    return w;
  }
  // the anchor's own bound term is replaced by the candidate's weight
  for (uint32_t i = 0; i < p.depth; ++i) {
    const uint32_t b = P.order[i];
    if (P.nbr[w.a] >> b & 1) w.bound0 -= m.best[(u64)mu_at(p, b) * NURI_MAX_LABELS + w.la];
  }
  for (uint32_t u = 0; u < P.q; ++u)
    if ((P.nbr[w.a] >> u & 1) && P.pos[u] > p.depth) w.bound0 -= P.pmx[w.a][u];
  return w;
}

// per-wavefront counters of the candidates it walked
struct MTally {
  u64 pruned_new = 0, leaves = 0, offered = 0, bytes = 0, cost = 0, maxcost = 0;
  long long maxb = LLONG_MIN;
};

// candidates [t_begin, t_end) of record p's anchor segment
__device__ inline void match_walk(const MView &m, const MPlan &P, const MRec &p, const MWork &w,
                                  uint32_t t_begin, uint32_t t_end, long long theta, uint32_t q,
                                  const MCfg &cf, MStep *ms, StepHdr *hdr, Cand *cands,
                                  uint32_t *cand_ids, uint32_t cand_cap, int lane, MTally &st) {
  const uint32_t a = w.a, la = w.la, anchor = w.anchor;
  const bool dg = P.degree != 0;
  for (uint32_t t0 = t_begin; t0 < t_end; t0 += 64) {
    const uint32_t t = t0 + lane;
    bool ok = t < t_end;
    uint32_t c = 0;
    long long score2 = p.score, bound2 = w.bound0;
    if (ok) {
      c = m.lcol[w.base + t];
      const long long wa = dg ? vdeg(m, c) : (long long)m.lew[w.base + t];
      score2 += wa;
      bound2 += wa;
      // injectivity and symmetry breaking against every matched vertex
      for (uint32_t i = 0; i < p.depth && ok; ++i) {
        const uint32_t b = P.order[i];
        const uint32_t mb = mu_at(p, b);
        ok = c != mb;
        if ((P.sb_lt[a] >> b & 1) && !(c < mb)) ok = false;
        if ((P.sb_lt[b] >> a & 1) && !(mb < c)) ok = false;
      }
      // adjacency to the other matched neighbours
      for (uint32_t i = 0; i < p.depth && ok; ++i) {
        const uint32_t b = P.order[i];
        if (b == anchor || !(P.nbr[a] >> b & 1)) continue;
        long long at = seg_find(m, mu_at(p, b), la, c);
        if (at < 0) {
          ok = false;
        } else if (!dg) {
          const int32_t wt = m.lew[at];
          score2 += wt;
          bound2 += wt;
        }
      }
      // edges from a to unmatched pattern vertices: one-hop bound from c
      // (under the degree score only the test that c has a neighbour of
      // each needed label)
      for (uint32_t u = 0; u < P.q && ok; ++u)
        if ((P.nbr[a] >> u & 1) && P.pos[u] > p.depth) {
          const int32_t wt = m.best[(u64)c * NURI_MAX_LABELS + P.label[u]];
          if (wt <= 0) ok = false;
          if (!dg) bound2 += wt;
        }
    }
    const bool valid = t < t_end;
    const bool prune = valid && (!ok || bound2 < theta);
    const bool complete = ok && !prune && w.last;
    const bool offer = complete && score2 >= theta;
    const bool keep = ok && !prune && !w.last;
    st.pruned_new += __popcll(__ballot(prune));
    st.leaves += __popcll(__ballot(complete));
    // children
    MRec ch;
    uint32_t nch = 0;
    if (keep) {
      ch = p;
      ch.mu[a] = c;
      ch.score = score2;
      ch.bound = bound2;
      ch.depth = p.depth + 1;
      nch = child_bound(m, P, ch);
      ch.nchild = nch;
    }
    const bool keep2 = keep && nch > 0;  // a child with no possible candidate is dead
    st.pruned_new += __popcll(__ballot(keep && !keep2));
    const u64 km = __ballot(keep2);
    if (km) {
      unsigned int h0 = 0;
      if (lane == 0) h0 = atomicAdd(&ms[q].n_out, (unsigned int)__popcll(km));
      h0 = __shfl(h0, 0, 64);
      if (keep2) {
        const uint32_t rk = __popcll(km & ((1ull << lane) - 1ull));
        const u64 slot = (u64)cf.out_hdr + h0 + rk;
        if (slot < cf.hdr_cap) {
          cf.hdr[slot] = ch;
          st.cost += nch;
          st.maxcost = nch > st.maxcost ? nch : st.maxcost;
          st.maxb = bound2 > st.maxb ? bound2 : st.maxb;
          st.bytes += 64;
        } else {
          atomicAdd(&ms[q].overflow, 1u);
        }
      }
    }
    const u64 fm = __ballot(offer);
    if (fm) {
      long long cm = offer ? score2 : LLONG_MIN;
      cm = wave_max(cm);
      if (lane == 0) {
        atomicAdd(&ms[q].cand_n, (unsigned int)__popcll(fm));
        atomicMax(&ms[q].cand_max, cm);
      }
      unsigned int c0 = 0;
      if (lane == 0) c0 = atomicAdd(&hdr->leaf_count, (unsigned int)__popcll(fm));
      c0 = __shfl(c0, 0, 64);
      if (offer) {
        const uint32_t slot = c0 + __popcll(fm & ((1ull << lane) - 1ull));
        if (slot < cand_cap) {
          Cand cd;
          cd.score = score2;
          cd.qid = q;
          cd.len = P.q;
          cands[slot] = cd;
          uint32_t *dst = cand_ids + (u64)slot * QM;
          for (uint32_t i = 0; i < P.q; ++i) dst[i] = (i == a) ? c : p.mu[i];
          st.offered++;
        } else {
          atomicAdd(&ms[q].overflow, 1u);
        }
      }
    }
  }
}

// flush one wavefront's tally into the query's counters
__device__ inline void match_flush(MTally &st, MCtr &C, MStep &S, int lane) {
  st.cost = wave_sum(st.cost);
  st.maxcost = wave_max_u64(st.maxcost);
  st.bytes = wave_sum(st.bytes);
  st.offered = wave_sum(st.offered);
  st.maxb = wave_max(st.maxb);
  if (lane == 0) {
    if (st.pruned_new) atomicAdd(&C.pruned_new, st.pruned_new);
    if (st.leaves) atomicAdd(&C.leaves, st.leaves);
    if (st.offered) atomicAdd(&C.offered, st.offered);
    if (st.bytes) atomicAdd(&C.logical_bytes, st.bytes);
    if (st.cost) {
      atomicAdd(&S.out_cost, st.cost);
      atomicMax(&S.out_max_cost, st.maxcost);
    }
    if (st.maxb != LLONG_MIN) atomicMax(&S.out_max_bound, st.maxb);
  }
}

__global__ void __launch_bounds__(64 * kMatchWaves)
    k_match_expand(MView m, const MPlan *plans, const MRec *__restrict__ batch, StepHdr *hdr,
                   const MCfg *cfg, MStep *ms, MCtr *ctr, const QRes *res, Cand *cands,
                   uint32_t *cand_ids, uint32_t cand_cap, uint32_t *big_rec, uint32_t *big_base) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint32_t rec = blockIdx.x * kMatchWaves + wv;
  if (rec >= hdr->batch_count) return;
  const MRec p = batch[rec];
  const uint32_t q = p.qid;
  const MPlan &P = plans[q];
  const MCfg cf = cfg[q];
  const long long theta = mprune_theta(cf, res[q]);
  MTally st;
  u64 children = 0;
  const bool pruned_pop = p.bound < theta;
  if (!pruned_pop && p.depth < P.q) {
    const MWork w = match_work(m, P, p);
    children = w.alen;
    if (lane == 0) st.bytes += 64 + 8ull * w.alen;
    if (w.alen > kMatchChunk && lane == 0) {
      // the chunks past the first go to k_match_expand_big; one 64-bit
      // atomic reserves both the list slot and the chunk numbers, so the
      // list stays sorted by its first chunk
      const u64 nrest = (w.alen - 1) / kMatchChunk;
      const u64 old = atomicAdd(&hdr->big_packed, (1ull << 32) | nrest);
      const uint32_t slot = (uint32_t)(old >> 32);
      big_rec[slot] = rec;
      big_base[slot] = (uint32_t)old;
    }
    match_walk(m, P, p, w, 0, min(w.alen, kMatchChunk), theta, q, cf, ms, hdr, cands, cand_ids,
               cand_cap, lane, st);
  }
  MCtr &C = ctr[q * kCtrSlots + (rec & (kCtrSlots - 1))];
  match_flush(st, C, ms[q], lane);
  if (lane == 0) {
    atomicAdd(&C.popped, 1ull);
    if (pruned_pop) atomicAdd(&C.pruned_pop, 1ull);
    if (children) {
      atomicAdd(&C.expanded, 1ull);
      atomicAdd(&C.children, children);
    }
  }
}

// The chunks of long anchor segments: wavefronts take chunk numbers from a
// shared counter until none is left; a chunk's record is found by binary
// search in the list (sorted by first chunk).  grid: kBigBlocks blocks.
__global__ void __launch_bounds__(64 * kMatchWaves)
    k_match_expand_big(MView m, const MPlan *plans, const MRec *__restrict__ batch, StepHdr *hdr,
                       const MCfg *cfg, MStep *ms, MCtr *ctr, const QRes *res, Cand *cands,
                       uint32_t *cand_ids, uint32_t cand_cap, const uint32_t *big_rec,
                       const uint32_t *big_base) {
  const int lane = threadIdx.x & 63;
  const u64 packed = hdr->big_packed;
  const uint32_t nbig = (uint32_t)(packed >> 32), nchunks = (uint32_t)packed;
  for (;;) {
    uint32_t c = 0;
    if (lane == 0) c = atomicAdd(&hdr->big_next, 1u);
    c = __shfl(c, 0, 64);
    if (c >= nchunks) break;
    uint32_t lo = 0, hi = nbig;  // last slot whose first chunk is <= c
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (big_base[mid] <= c) lo = mid;
      else hi = mid;
    }
    const MRec p = batch[big_rec[lo]];
    const uint32_t q = p.qid;
    const MPlan &P = plans[q];
    const MCfg cf = cfg[q];
    const long long theta = mprune_theta(cf, res[q]);
    const MWork w = match_work(m, P, p);
    const uint32_t t0 = (c - big_base[lo] + 1) * kMatchChunk;
    MTally st;
    match_walk(m, P, p, w, t0, min(w.alen, t0 + kMatchChunk), theta, q, cf, ms, hdr, cands,
               cand_ids, cand_cap, lane, st);
    match_flush(st, ctr[q * kCtrSlots + (c & (kCtrSlots - 1))], ms[q], lane);
  }
}

// ------------------------------------------------------------------
// candidate prefilter: complete matches are results, so at most k of
// them can matter per query; a histogram of scores over the new
// candidates and the current top-k gives a score below which none can
// enter, and only the rest go to the exact merge
// ------------------------------------------------------------------
__device__ inline int cbin(long long score, const CPre &c) {
  long long gap = (c.top - score) >> c.shift;
  long long b = kBins - 1 - gap;
  return b < 0 ? 0 : (b > kBins - 1 ? kBins - 1 : (int)b);
}

__global__ void k_cand_hist(const Cand *cands, uint32_t ncand, const CPre *pre,
                            unsigned int *hist) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ncand) {
    const Cand c = cands[i];
    atomicAdd(&hist[(size_t)c.qid * kBins + cbin(c.score, pre[c.qid])], 1u);
  }
}

// the current top-k entries count too: one block per query

__global__ void k_cand_hist_topk(const QRes *res, const CPre *pre, unsigned int *hist) {
  const uint32_t q = blockIdx.x;
  const QRes R = res[q];
  for (uint32_t i = threadIdx.x; i < R.tk_n; i += blockDim.x)
    atomicAdd(&hist[(size_t)q * kBins + cbin(R.tk_score[R.cur][i], pre[q])], 1u);
}

__global__ void k_cand_thresh(const uint32_t *ks, CPre *pre, unsigned int *hist) {
  const uint32_t q = blockIdx.x;
  if (threadIdx.x == 0) {
    u64 n = 0;
    int t = 0;
    for (int b = kBins - 1; b >= 0; --b) {
      n += hist[(size_t)q * kBins + b];
      if (n >= ks[q]) {
        t = b;
        break;
      }
    }
    pre[q].tbin = t;
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kBins; b += blockDim.x) hist[(size_t)q * kBins + b] = 0;
}

__global__ void k_cand_compact(const Cand *cands, const uint32_t *ids, uint32_t ncand,
                               const CPre *pre, Cand *out, uint32_t *out_ids,
                               unsigned int *count) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ncand) return;
  const Cand c = cands[i];
  if (cbin(c.score, pre[c.qid]) < pre[c.qid].tbin) return;
  const unsigned int slot = atomicAdd(count, 1u);
  out[slot] = c;
  for (int t = 0; t < QM; ++t) out_ids[(u64)slot * QM + t] = ids[(u64)i * QM + t];
}

// ------------------------------------------------------------------
// host: pattern planning
// ------------------------------------------------------------------
void plan_pattern(const Graph &g, const nuri_pattern &pt, uint32_t k, MPlan &P) {
  const uint32_t q = pt.q;
  if (q < 2 || q > (uint32_t)QM) throw Error{NURI_EINVAL, "pattern size must be 2..8"};
  if (k == 0) throw Error{NURI_EINVAL, "k must be >= 1"};
  if (pt.score > NURI_MATCH_DEGREE) throw Error{NURI_EINVAL, "unknown match score"};
  memset(&P, 0, sizeof(P));
  P.q = q;
  P.k = k;
  P.degree = pt.score == NURI_MATCH_DEGREE;
  uint8_t adj[QM][QM] = {};
  for (uint32_t a = 0; a < q; ++a) {
    if (pt.label[a] >= NURI_MAX_LABELS) throw Error{NURI_EINVAL, "pattern label out of range"};
    P.label[a] = pt.label[a];
  }
  for (uint32_t e = 0; e < pt.n_edges; ++e) {
    uint32_t a = pt.edges[2 * e], b = pt.edges[2 * e + 1];
    if (a >= q || b >= q || a == b) throw Error{NURI_EINVAL, "bad pattern edge"};
    if (adj[a][b]) throw Error{NURI_EINVAL, "duplicate pattern edge"};
    adj[a][b] = adj[b][a] = 1;
  }
  for (uint32_t a = 0; a < q; ++a)
    for (uint32_t b = 0; b < q; ++b)
      if (adj[a][b]) P.nbr[a] |= (uint8_t)(1u << b);
  // connectivity
  uint32_t seen = 1, grow = 1;
  while (grow) {
    grow = 0;
    for (uint32_t a = 0; a < q; ++a)
      if ((seen >> a & 1) && (P.nbr[a] & ~seen)) {
        seen |= P.nbr[a];
        grow = 1;
      }
  }
  if (seen != (1u << q) - 1) throw Error{NURI_EINVAL, "pattern must be connected"};
  // automorphisms (brute force over q! permutations)
  std::vector<std::vector<uint8_t>> aut;
  std::vector<uint8_t> perm(q);
  std::iota(perm.begin(), perm.end(), 0);
  do {
    bool ok = true;
    for (uint32_t a = 0; a < q && ok; ++a) ok = P.label[perm[a]] == P.label[a];
    for (uint32_t a = 0; a < q && ok; ++a)
      for (uint32_t b = a + 1; b < q && ok; ++b)
        if (adj[a][b]) ok = adj[perm[a]][perm[b]];
    if (ok) aut.push_back(perm);
  } while (std::next_permutation(perm.begin(), perm.end()));
  // symmetry breaking: mu(i) < mu(j) for j in the orbit of i under the
  // automorphisms that fix 0..i-1
  for (uint32_t i = 0; i < q; ++i)
    for (const auto &s : aut) {
      bool fixes = true;
      for (uint32_t t = 0; t < i && fixes; ++t) fixes = s[t] == t;
      if (fixes && s[i] != i) P.sb_lt[i] |= (uint8_t)(1u << s[i]);
    }
  // matching order: rarest label first (ties: larger degree, smaller id),
  // then most edges into the ordered prefix (ties: smaller id)
  uint32_t used = 0;
  auto deg = [&](uint32_t a) { return (uint32_t)__builtin_popcount(P.nbr[a]); };
  uint32_t first = 0;
  for (uint32_t a = 1; a < q; ++a) {
    uint64_t ca = g.h_label_count[P.label[a]], cb = g.h_label_count[P.label[first]];
    if (ca < cb || (ca == cb && deg(a) > deg(first))) first = a;
  }
  P.order[0] = (uint8_t)first;
  used = 1u << first;
  for (uint32_t i = 1; i < q; ++i) {
    uint32_t pick = q, pc = 0;
    for (uint32_t a = 0; a < q; ++a) {
      if (used >> a & 1) continue;
      uint32_t c = __builtin_popcount(P.nbr[a] & used);
      if (pick == q || c > pc) {
        pick = a;
        pc = c;
      }
    }
    P.order[i] = (uint8_t)pick;
    used |= 1u << pick;
  }
  for (uint32_t i = 0; i < q; ++i) P.pos[P.order[i]] = (uint8_t)i;
  // distances from order[0] (breadth-first over the pattern)
  {
    uint32_t reached = 1u << first, frontier = reached;
    P.hop[first] = 0;
    P.max_hop = 1;
    for (uint32_t h = 1; frontier; ++h) {
      uint32_t nxt = 0;
      for (uint32_t a = 0; a < q; ++a)
        if (frontier >> a & 1) nxt |= P.nbr[a];
      nxt &= ~reached;
      for (uint32_t a = 0; a < q; ++a)
        if (nxt >> a & 1) {
          P.hop[a] = (uint8_t)h;
          P.max_hop = std::max(P.max_hop, h);
        }
      reached |= nxt;
      frontier = nxt;
    }
  }
  // label-pair maxima of the pattern edges, and the bound part of the
  // edges that do not touch order[0]
  P.rest0 = 0;
  bool possible = true;
  for (uint32_t a = 0; a < q; ++a)
    for (uint32_t b = 0; b < q; ++b)
      if (adj[a][b]) {
        P.pmx[a][b] = g.h_pairmax[P.label[a] * NURI_MAX_LABELS + P.label[b]];
        if (P.pmx[a][b] <= 0) possible = false;
        if (a < b && a != first && b != first) P.rest0 += P.pmx[a][b];
      }
  if (!possible) P.rest0 = LLONG_MIN / 4;  // marks: no match can exist
}

// ------------------------------------------------------------------
// host: engine
// ------------------------------------------------------------------
struct MLevel {
  uint32_t begin = 0, count = 0;
  uint32_t depth = 1;  // matched pattern vertices of its records
  u64 cost = 0, maxcost = 0;
  long long max_bound = LLONG_MIN;
};

// Bottom levels of a query's stack moved to host memory (the paper's
// virtual priority queue, Section 5): the records of the arena range
// [0, n) they occupied, returned to the same offsets when the levels above
// have drained.
struct MSpill {
  std::vector<MLevel> levels;
  std::vector<MRec> recs;
};

struct MQHost {
  bool active = false;  // the slot holds a query
  bool done = true;     // the query needs no more steps
  bool rooted = false;  // its unit subgraphs are in place
  int error = 0;
  std::string errmsg;
  uint32_t k = 1;
  std::vector<MLevel> stack;
  long long theta = LLONG_MIN;
  long long top_seen = LLONG_MIN;  // best score ever offered (bounds the top-k)
  uint32_t hdr_cap = 0;
  uint64_t t_admit = 0, steps = 0, launches = 0, expand_ns = 0, peak_bytes = 0;
  uint64_t index_ns = 0;  // multi-hop index built for this query
  int plan = 0;
  uint32_t new_begin = 0;
  int seg = -1;
  int lvl = -1;  // stack index of the level this step takes from
  std::vector<std::shared_ptr<MSpill>> spill;  // spilled chunks, the last spilled last
  uint64_t spilled_bytes = 0;
};

// per-slot top-k buffers and frontier arena, taken at admission
struct MSlotTopk {
  PoolBuf<long long> score;
  PoolBuf<unsigned int> len, ids;
  PoolBuf<MRec> hdr;
};

struct MStepLayout {
  size_t ms, cfg, seg, taken, tempc, thr, quota, total;
  explicit MStepLayout(uint32_t nq) {
    size_t o = sizeof(StepHdr);
    ms = o;
    o += nq * sizeof(MStep);
    cfg = o;
    o += nq * sizeof(MCfg);
    seg = o;
    o += nq * sizeof(MSeg);
    taken = o;
    o += nq * 4;
    tempc = o;
    o += nq * 4;
    thr = o;
    o += nq * 4;
    quota = o;
    o += nq * 4;
    total = (o + 255) & ~size_t(255);
  }
  size_t readback() const { return cfg; }
};

struct MatchEngine {
  Graph &g;
  QueryOpts o;
  hipStream_t s;
  bool server_mode = false;
  uint32_t nq = 0;  // slots
  std::vector<MQHost> qh;
  std::vector<MPlan> plans;
  std::vector<MCfg> cfg;
  std::vector<std::unique_ptr<MSlotTopk>> tk;
  PoolBuf<MPlan> d_plans;
  PoolBuf<uint64_t> d_lab_off;
  PoolBuf<MRec> batch, temp;
  u64 arena_bytes = 0;  // frontier arena of a slot unless admit() is given one
  PoolBuf<uint32_t> big_rec, big_base;  // records whose candidates are shared out in chunks
  PoolBuf<MCtr> d_ctr;
  PoolBuf<QRes> d_res;
  PoolBuf<uint32_t> d_k, d_rootq;
  PoolBuf<Cand> cands, cands2;
  MergeBufs mbuf;  // top-k merge: candidate positions and survivor lists
  PoolBuf<uint32_t> cand_ids, cand_ids2;
  PoolBuf<CPre> d_pre;
  PinBuf<CPre> h_pre;
  PoolBuf<unsigned int> d_chist, d_ccount;
  PinBuf<unsigned int> h_ccount;  // [0] candidates kept; [1..] merge chunk sizes
  bool theta_pending = false;     // h_res holds k-th scores not yet taken
  PoolBuf<unsigned int> d_hist;
  PoolBuf<u64> d_hcost;
  PoolBuf<unsigned char> d_step;
  PinBuf<unsigned char> h_step;
  PinBuf<QRes> h_res;
  PinBuf<MCtr> h_ctr;
  PinBuf<uint32_t> h_k, h_rootq;
  PinBuf<MPlan> h_plan;
  std::unique_ptr<MStepLayout> L;
  uint32_t batch_cap = 0, cand_cap = 0, B = 0;
  u64 step_children = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  uint32_t rr = 0;  // round-robin start of the per-step planning

  MatchEngine(Graph &g_, const QueryOpts &o_) : g(g_), o(o_), s(o_.stream ? o_.stream : g_.stream) {}
  ~MatchEngine() {
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
  }

  MView view() const {
    MView v;
    v.orow = g.orow.p;
    v.lcol = g.lcol.p;
    v.lew = g.lew.p;
    v.loff = g.loff.p;
    v.best = g.best.p;
    v.lab_vert = g.lab_vert.p;
    for (int h = 0; h < QM - 1; ++h) v.hidx[h] = g.hidx[h].p;
    return v;
  }
  StepHdr *sh() { return (StepHdr *)h_step.p; }
  MStep *sms() { return (MStep *)(h_step.p + L->ms); }
  MSeg *sseg() { return (MSeg *)(h_step.p + L->seg); }
  template <class T>
  T *dev(size_t off) {
    return (T *)(d_step.p + off);
  }

  void fail(uint32_t i, int code, const std::string &msg) {
    if (!server_mode) throw Error{code, msg};
    qh[i].error = code;
    qh[i].errmsg = msg;
    qh[i].done = true;
  }

  void setup(uint32_t slots) {
    nq = slots;
    qh.assign(nq, MQHost{});
    plans.assign(nq, MPlan{});
    cfg.assign(nq, MCfg{});
    tk.clear();
    for (uint32_t i = 0; i < nq; ++i) tk.emplace_back(new MSlotTopk);
    L.reset(new MStepLayout(nq));
    arena_bytes = o.frontier_budget / nq;
    for (uint32_t i = 0; i < nq; ++i) {
      cfg[i].out_hdr = 0;
      cfg[i].prio = o.priority;
      cfg[i].pad = 0;
    }
    d_plans.alloc(g.pool, nq);
    h_plan.alloc(1);
    d_lab_off.alloc(g.pool, NURI_MAX_LABELS + 1);
    NURI_HIP(hipMemcpyAsync(d_lab_off.p, g.h_lab_off.data(), (NURI_MAX_LABELS + 1) * 8,
                            hipMemcpyHostToDevice, s));
    NURI_HIP(hipStreamSynchronize(s));  // the host vector is not pinned
    h_res.alloc(nq);
    h_ctr.alloc((u64)nq * kCtrSlots);
    h_k.alloc(nq);
    h_rootq.alloc(nq);
    for (uint32_t i = 0; i < nq; ++i) {
      memset(&h_res.p[i], 0, sizeof(QRes));
      h_res.p[i].theta = LLONG_MIN;
      h_k.p[i] = 1;
    }
    d_ctr.alloc(g.pool, (u64)nq * kCtrSlots);
    d_res.alloc(g.pool, nq);
    d_k.alloc(g.pool, nq);
    d_rootq.alloc(g.pool, nq);
    NURI_HIP(hipMemcpyAsync(d_res.p, h_res.p, nq * sizeof(QRes), hipMemcpyHostToDevice, s));
    NURI_HIP(hipMemcpyAsync(d_k.p, h_k.p, nq * 4, hipMemcpyHostToDevice, s));
    NURI_HIP(hipMemsetAsync(d_ctr.p, 0, (u64)nq * kCtrSlots * sizeof(MCtr), s));
    B = o.batch_B ? o.batch_B : 16384;
    step_children = std::max<u64>(1ull << 16, std::min<u64>(o.frontier_budget / 8 / sizeof(MRec),
                                                            8ull << 20));
    cand_cap = (uint32_t)std::min<u64>(step_children, 1ull << 22);
    batch_cap = (uint32_t)std::min<u64>((u64)nq * B, 1u << 24);
    batch.alloc(g.pool, batch_cap);
    big_rec.alloc(g.pool, batch_cap);
    big_base.alloc(g.pool, batch_cap);
    cands.alloc(g.pool, cand_cap);
    cand_ids.alloc(g.pool, (u64)cand_cap * QM);
    cands2.alloc(g.pool, cand_cap);
    mbuf.alloc(g.pool, nq, s);
    cand_ids2.alloc(g.pool, (u64)cand_cap * QM);
    d_pre.alloc(g.pool, nq);
    h_pre.alloc(nq);
    d_chist.alloc(g.pool, (u64)nq * kBins);
    NURI_HIP(hipMemsetAsync(d_chist.p, 0, d_chist.bytes(), s));
    d_ccount.alloc(g.pool, 1);
    h_ccount.alloc(1 + (cand_cap + kCandChunk - 1) / kCandChunk);
    d_hist.alloc(g.pool, (u64)nq * kBins);
    d_hcost.alloc(g.pool, (u64)nq * kBins);
    NURI_HIP(hipMemsetAsync(d_hist.p, 0, d_hist.bytes(), s));
    NURI_HIP(hipMemsetAsync(d_hcost.p, 0, d_hcost.bytes(), s));
    d_step.alloc(g.pool, L->total);
    h_step.alloc(L->total);
    if (o.profile) {
      NURI_HIP(hipEventCreate(&ev0));
      NURI_HIP(hipEventCreate(&ev1));
    }
  }

  // records in an arena of `bytes`
  static u64 arena_records(u64 bytes) {
    return std::min<u64>(std::max<u64>(4096, bytes / sizeof(MRec)), 0x7FFFFFFFull);
  }

  // start a query in a free slot (its unit subgraphs are made on the next
  // step) with a frontier arena of `bytes` (0: the slot default)
  void admit(uint32_t i, const nuri_pattern &pt, uint32_t k, u64 bytes = 0) {
    // the copy of every query's k-th score still in flight would land on
    // top of this slot's new entry: let it land and take it while the slot
    // still holds the old query (which no longer counts), before resetting it
    if (theta_pending) {
      NURI_HIP(hipStreamSynchronize(s));
      take_theta();
    }

    MPlan P;
    plan_pattern(g, pt, k, P);  // throws on an invalid pattern
    uint64_t index_ns = 0;
    if (P.degree) {
      const uint64_t t0 = now_ns();
      ensure_hop_index(g, P.max_hop, s);
      index_ns = now_ns() - t0;
    }
    MQHost &Q = qh[i];
    Q = MQHost{};
    Q.index_ns = index_ns;
    Q.active = true;
    Q.k = k;
    const u64 cap = arena_records(bytes ? bytes : arena_bytes);
    tk[i]->hdr.alloc(g.pool, cap);
    cfg[i].hdr = tk[i]->hdr.p;
    cfg[i].hdr_cap = (uint32_t)cap;
    Q.hdr_cap = (uint32_t)cap;
    Q.t_admit = now_ns();
    Q.done = P.rest0 == LLONG_MIN / 4;  // some pattern edge has no data edge
    Q.rooted = Q.done;
    plans[i] = P;
    *h_plan.p = P;
    NURI_HIP(hipMemcpyAsync(&d_plans.p[i], h_plan.p, sizeof(MPlan), hipMemcpyHostToDevice, s));
    MSlotTopk &T = *tk[i];
    T.score.alloc(g.pool, 2ull * k);
    T.len.alloc(g.pool, 2ull * k);
    T.ids.alloc(g.pool, 2ull * k * QM);
    QRes &R = h_res.p[i];
    R.theta = LLONG_MIN;
    R.tk_n = 0;
    R.cur = 0;
    for (int b = 0; b < 2; ++b) {
      R.tk_score[b] = T.score.p + (u64)b * k;
      R.tk_len[b] = T.len.p + (u64)b * k;
      R.tk_ids[b] = T.ids.p + (u64)b * k * QM;
    }
    h_k.p[i] = k;
    NURI_HIP(hipMemcpyAsync(&d_res.p[i], &h_res.p[i], sizeof(QRes), hipMemcpyHostToDevice, s));
    NURI_HIP(hipMemcpyAsync(&d_k.p[i], &h_k.p[i], 4, hipMemcpyHostToDevice, s));
    NURI_HIP(hipMemsetAsync(&d_ctr.p[(u64)i * kCtrSlots], 0, kCtrSlots * sizeof(MCtr), s));
    NURI_HIP(hipStreamSynchronize(s));  // h_plan is reused by the next admission
  }

  bool slot_free(uint32_t i) const { return !qh[i].active; }
  bool finished(uint32_t i) const { return qh[i].active && qh[i].done; }
  bool any_live() const {
    for (auto &Q : qh)
      if (Q.active && !Q.done) return true;
    return false;
  }

  void upload_step() {
    for (uint32_t i = 0; i < nq; ++i) {
      cfg[i].out_hdr = qh[i].new_begin;
      sms()[i].out_max_bound = LLONG_MIN;
      sms()[i].cand_max = LLONG_MIN;
    }
    memcpy(h_step.p + L->cfg, cfg.data(), nq * sizeof(MCfg));
    memset(h_step.p + L->taken, 0, 8ull * nq);
    NURI_HIP(hipMemcpyAsync(d_step.p, h_step.p, L->total, hipMemcpyHostToDevice, s));
  }

  void read_step() {
    NURI_HIP(hipMemcpyAsync(h_step.p, d_step.p, L->readback(), hipMemcpyDeviceToHost, s));
    NURI_HIP(hipStreamSynchronize(s));
    take_theta();
  }

  // after a synchronisation: take the k-th scores copied back last
  void take_theta() {
    if (!theta_pending) return;
    theta_pending = false;
    for (uint32_t i = 0; i < nq; ++i)
      if (qh[i].active) qh[i].theta = h_res.p[i].theta;
  }

  // unit subgraphs of newly admitted queries become their first level,
  // unsorted: the select step orders them by bound
  void make_roots() {
    uint32_t n = 0;
    for (uint32_t i = 0; i < nq; ++i)
      if (qh[i].active && !qh[i].rooted) h_rootq.p[n++] = i;
    if (!n) return;
    memset(h_step.p, 0, L->cfg);
    for (uint32_t t = 0; t < n; ++t) qh[h_rootq.p[t]].new_begin = 0;
    upload_step();
    NURI_HIP(hipMemcpyAsync(d_rootq.p, h_rootq.p, n * 4, hipMemcpyHostToDevice, s));
    uint32_t maxn = 1;
    for (int l = 0; l < NURI_MAX_LABELS; ++l)
      maxn = std::max<uint32_t>(maxn, (uint32_t)(g.h_lab_off[l + 1] - g.h_lab_off[l]));
    const uint32_t bx = std::min<uint32_t>((maxn + 255) / 256, 2048);
    hipLaunchKernelGGL(k_match_roots, dim3(bx, n), dim3(256), 0, s, view(), d_plans.p,
                       d_lab_off.p, dev<MCfg>(L->cfg), dev<MStep>(L->ms), d_rootq.p);
    NURI_HIP(hipGetLastError());
    read_step();
    for (uint32_t t = 0; t < n; ++t) {
      const uint32_t i = h_rootq.p[t];
      MQHost &Q = qh[i];
      const MStep &c = sms()[i];
      Q.rooted = true;
      if (c.overflow) {
        fail(i, NURI_EBUDGET, "frontier budget too small for the unit subgraphs");
        continue;
      }
      if (c.n_out) {
        MLevel Lv;
        Lv.begin = 0;
        Lv.depth = 1;
        Lv.count = c.n_out;
        Lv.cost = c.out_cost;
        Lv.maxcost = c.out_max_cost;
        Lv.max_bound = c.out_max_bound;
        Q.stack.push_back(Lv);
      } else {
        Q.done = true;
      }
    }
  }

  // When a query's arena is nearly full its bottom levels -- at least half
  // of the used records, never the top level -- are copied to host memory
  // and the levels above moved down.  Returns false when there is nothing
  // to spill.
  bool spill_bottom(uint32_t i) {
    MQHost &Q = qh[i];
    if (Q.stack.size() < 2) return false;
    const MLevel &T = Q.stack.back();
    const u64 used = (u64)T.begin + T.count;
    size_t m = 1;  // levels [0, m) go to the host
    while (m + 1 < Q.stack.size() && (u64)Q.stack[m].begin * 2 < used) ++m;
    const u64 shift = Q.stack[m].begin;
    if (shift == 0) return false;
    auto C = std::make_shared<MSpill>();
    C->levels.assign(Q.stack.begin(), Q.stack.begin() + m);
    C->recs.resize(shift);
    MRec *arena = cfg[i].hdr;
    NURI_HIP(hipMemcpyAsync(C->recs.data(), arena, shift * sizeof(MRec), hipMemcpyDeviceToHost,
                            s));
    const u64 rest = used - shift;
    if (rest) {
      if (shift >= rest) {
        NURI_HIP(hipMemcpyAsync(arena, arena + shift, rest * sizeof(MRec),
                                hipMemcpyDeviceToDevice, s));
      } else {
        PoolBuf<MRec> tmp;  // the ranges overlap: through a scratch copy
        tmp.alloc(g.pool, rest);
        NURI_HIP(hipMemcpyAsync(tmp.p, arena + shift, rest * sizeof(MRec),
                                hipMemcpyDeviceToDevice, s));
        NURI_HIP(hipMemcpyAsync(arena, tmp.p, rest * sizeof(MRec), hipMemcpyDeviceToDevice, s));
        NURI_HIP(hipStreamSynchronize(s));  // before the scratch returns to the pool
      }
    }
    NURI_HIP(hipStreamSynchronize(s));
    Q.stack.erase(Q.stack.begin(), Q.stack.begin() + m);
    for (MLevel &L : Q.stack) L.begin -= (uint32_t)shift;
    Q.spilled_bytes += shift * sizeof(MRec);
    Q.spill.push_back(C);
    return true;
  }

  // the stack is empty: the last spilled chunk comes back to its offsets
  void reload(uint32_t i) {
    MQHost &Q = qh[i];
    std::shared_ptr<MSpill> C = Q.spill.back();
    Q.spill.pop_back();
    NURI_HIP(hipMemcpyAsync(cfg[i].hdr, C->recs.data(), C->recs.size() * sizeof(MRec),
                            hipMemcpyHostToDevice, s));
    NURI_HIP(hipStreamSynchronize(s));  // the host copy is freed below
    Q.stack = C->levels;
  }

  bool plan(uint32_t &nseg, uint32_t &batch_ub, u64 &temp_need, uint32_t &max_count,
            bool &any_sel) {
    nseg = 0;
    batch_ub = 0;
    temp_need = 0;
    max_count = 0;
    any_sel = false;
    uint32_t live = 0;
    for (auto &Q : qh) live += Q.active && !Q.done;
    if (!live) return false;
    const uint64_t now = o.deadline_ns ? now_ns() : 0;
    // a query's children go to its own arena, so only its free space and a
    // per-step cap limit it; complete matches go to the shared candidate
    // buffer, which is split between the queries that produce them
    const u64 cand_share = std::max<u64>(cand_cap / live, 1);
    u64 left_cand = cand_cap;
    bool any = false;
    for (uint32_t i = 0; i < nq; ++i) {
      qh[i].plan = 0;
      qh[i].seg = -1;
    }
    rr = (rr + 1) % nq;  // the query served first rotates between steps
    for (uint32_t t = 0; t < nq; ++t) {
      const uint32_t i = (rr + t) % nq;
      MQHost &Q = qh[i];
      if (!Q.active || Q.done) continue;
      if (o.deadline_ns && now - Q.t_admit > o.deadline_ns) {
        fail(i, NURI_ETIMEOUT, "query deadline passed");
        continue;
      }
      while (!Q.stack.empty() && Q.stack.back().count == 0) Q.stack.pop_back();
      while (Q.stack.empty() && !Q.spill.empty()) {
        reload(i);
        while (!Q.stack.empty() && Q.stack.back().count == 0) Q.stack.pop_back();
      }
      if (Q.stack.empty()) {
        Q.done = true;
        continue;
      }
      // when the children of one record of some level no longer fit, the
      // bottom levels go to host memory (spilling earlier, while smaller
      // steps still fit, copied gigabytes through the host for nothing)
      {
        u64 need = 1;
        for (const MLevel &Lx : Q.stack)
          if (Lx.count) need = std::max<u64>(need, Lx.maxcost);
        const MLevel &T0 = Q.stack.back();
        const u64 f0 = Q.hdr_cap - (u64)(T0.begin + T0.count);
        if (f0 < need) spill_bottom(i);
      }
      // the level to take from: the deepest, or (best-first) the one with the
      // highest bound (ties: the deeper)
      int li = (int)Q.stack.size() - 1;
      if (o.priority == NURI_PRIORITY_BOUND)
        for (int t2 = li - 1; t2 >= 0; --t2)
          if (Q.stack[t2].count && Q.stack[t2].max_bound > Q.stack[li].max_bound) li = t2;
      MLevel &Lv = Q.stack[li];
      const MLevel &Top = Q.stack.back();
      const u64 free_h = Q.hdr_cap - (u64)(Top.begin + Top.count);
      const bool to_leaves = Lv.depth + 1 == plans[i].q;  // children are complete matches
      const u64 rec = std::max<u64>(1, Lv.maxcost);
      if ((to_leaves ? cand_cap : free_h) < rec) {
        fail(i, NURI_EBUDGET, "frontier budget exhausted");
        continue;
      }
      // a step's children take at most three quarters of the query's free
      // arena, so the (at most q) deeper levels always keep room to go on
      const u64 lim = to_leaves ? std::min<u64>(left_cand, std::max(cand_share, rec))
                                : std::min<u64>(step_children,
                                                std::max<u64>(free_h - free_h / 4, rec));
      if (lim < rec) continue;
      const uint32_t room = batch_cap - batch_ub;
      if (room == 0) continue;
      MSeg &sg = sseg()[nseg];
      sg = MSeg{};
      sg.qid = i;
      sg.begin = Lv.begin;
      sg.count = Lv.count;
      sg.max_records = std::min<u64>(B, room);
      sg.max_children = lim;
      sg.maxcost = Lv.maxcost;
      sg.take_all = Lv.count <= sg.max_records && Lv.cost <= lim;
      sg.top = Lv.max_bound;
      const long long floor_b =
          Q.theta == LLONG_MIN || o.priority == NURI_PRIORITY_NONE ? 0 : Q.theta;
      const long long span = Lv.max_bound - floor_b;
      uint32_t shift = 0;
      while (span > 0 && (span >> shift) >= kBins - 1) ++shift;
      sg.shift = shift;
      sg.temp_off = (uint32_t)temp_need;
      if (!sg.take_all) {
        temp_need += Lv.count;
        any_sel = true;
      }
      max_count = std::max(max_count, Lv.count);
      Q.seg = (int)nseg++;
      Q.lvl = li;
      Q.plan = 1;
      Q.new_begin = Top.begin + Top.count;
      batch_ub += (uint32_t)(sg.take_all ? Lv.count : sg.max_records);
      const u64 used = sg.take_all ? Lv.cost : lim;
      if (to_leaves) left_cand -= std::min(left_cand, used);
      any = true;
    }
    if (!any)
      for (uint32_t i = 0; i < nq; ++i)
        if (qh[i].active && !qh[i].done)
          fail(i, NURI_EBUDGET, "frontier budget too small to make progress");
    return any;
  }

  void step(uint32_t nseg, uint32_t batch_ub, u64 temp_need, uint32_t max_count, bool any_sel) {
    memset(h_step.p, 0, L->cfg);
    upload_step();
    StepHdr *dh = dev<StepHdr>(0);
    MStep *dms = dev<MStep>(L->ms);
    MCfg *dcfg = dev<MCfg>(L->cfg);
    MSeg *dseg = dev<MSeg>(L->seg);
    if (temp_need && temp.n < temp_need) temp.alloc(g.pool, temp_need * 2);
    const uint32_t bx = std::max(1u, std::min<uint32_t>((max_count + 255) / 256, 2048));
    if (any_sel) {
      hipLaunchKernelGGL(k_msel_hist, dim3(std::min(bx, 512u), nseg), dim3(256), 0, s, dseg, dcfg,
                         d_res.p, d_hist.p, d_hcost.p);
      NURI_HIP(hipGetLastError());
      hipLaunchKernelGGL(k_msel_thresh, dim3(nseg), dim3(256), 0, s, dseg, nseg, d_hist.p,
                         d_hcost.p, dev<int>(L->thr), dev<unsigned int>(L->quota));
      NURI_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_msel_part, dim3(bx, nseg), dim3(256), 0, s, dseg, dcfg, d_res.p,
                       dev<int>(L->thr), dev<unsigned int>(L->quota), dev<unsigned int>(L->taken),
                       batch.p, dh, temp.p, dev<unsigned int>(L->tempc), d_ctr.p);
    NURI_HIP(hipGetLastError());
    if (any_sel) {
      hipLaunchKernelGGL(k_mcopy_back, dim3(bx, nseg), dim3(256), 0, s, dseg, dcfg, temp.p,
                         dev<unsigned int>(L->tempc), dms);
      NURI_HIP(hipGetLastError());
    }
    if (o.profile) NURI_HIP(hipEventRecord(ev0, s));
    hipLaunchKernelGGL(k_match_expand, dim3((batch_ub + kMatchWaves - 1) / kMatchWaves),
                       dim3(64 * kMatchWaves), 0, s, view(), d_plans.p, batch.p, dh, dcfg, dms,
                       d_ctr.p, d_res.p, cands.p, cand_ids.p, cand_cap, big_rec.p, big_base.p);
    NURI_HIP(hipGetLastError());
    // long candidate lists were cut into chunks: share those out
    bool any_big = false;
    for (uint32_t t = 0; t < nseg; ++t) any_big |= sseg()[t].maxcost > kMatchChunk;
    if (any_big) {
      hipLaunchKernelGGL(k_match_expand_big, dim3(kBigBlocks), dim3(64 * kMatchWaves), 0, s,
                         view(), d_plans.p, batch.p, dh, dcfg, dms, d_ctr.p, d_res.p, cands.p,
                         cand_ids.p, cand_cap, big_rec.p, big_base.p);
      NURI_HIP(hipGetLastError());
    }
    if (o.profile) NURI_HIP(hipEventRecord(ev1, s));
    read_step();
    uint64_t ens = 0;
    if (o.profile) {
      float ms = 0;
      NURI_HIP(hipEventElapsedTime(&ms, ev0, ev1));
      ens = (uint64_t)(ms * 1e6);
    }
    for (uint32_t i = 0; i < nq; ++i) {
      MQHost &Q = qh[i];
      if (!Q.plan) continue;
      const MStep &c = sms()[i];
      Q.steps++;
      Q.launches++;
      Q.expand_ns += ens;
      if (c.overflow) {
        fail(i, NURI_EBUDGET, "frontier overflow (internal accounting error)");
        continue;
      }
      MLevel &Lv = Q.stack[Q.lvl];
      Lv.count = sseg()[Q.seg].take_all ? 0 : c.n_kept;
      if (c.n_out) {
        MLevel N;
        N.depth = Lv.depth + 1;
        N.begin = Q.new_begin;
        N.count = c.n_out;
        N.cost = c.out_cost;
        N.maxcost = c.out_max_cost;
        N.max_bound = c.out_max_bound;
        Q.stack.push_back(N);
      }
      const MLevel &T = Q.stack.back();
      Q.peak_bytes = std::max<u64>(Q.peak_bytes, (u64)(T.begin + T.count) * sizeof(MRec));
    }
    merge_candidates(dh);
  }

  // complete matches -> top-k merge in chunks (the threshold rises between chunks)
  void merge_candidates(StepHdr *dh) {
    uint32_t ncand = sh()->leaf_count;
    if (ncand > cand_cap) throw Error{NURI_EBUDGET, "candidate buffer overflow (internal)"};
    if (!ncand) return;
    uint32_t kmax = 0;
    for (auto &Q : qh)
      if (Q.active) kmax = std::max(kmax, Q.k);
    const Cand *mc = cands.p;
    const uint32_t *mids = cand_ids.p;
    if (ncand > kCandChunk) {
      // prefilter by score: keep, per query, the candidates in score bins
      // at or above the bin of the k-th best among candidates and top-k
      for (uint32_t i = 0; i < nq; ++i) {
        const MStep &c = sms()[i];
        CPre &P = h_pre.p[i];
        P.top = c.cand_n ? c.cand_max : 0;
        // the current top-k can hold higher scores than this step's best
        if (qh[i].active && h_res.p[i].tk_n) P.top = std::max<long long>(P.top, qh[i].top_seen);
        const long long floor_s = qh[i].theta == LLONG_MIN ? 0 : qh[i].theta;
        const long long span = std::max<long long>(0, P.top - floor_s);
        uint32_t shift = 0;
        while ((span >> shift) >= kBins - 1) ++shift;
        P.shift = shift;
        P.tbin = 0;
        if (c.cand_n) qh[i].top_seen = std::max(qh[i].top_seen, c.cand_max);
      }
      NURI_HIP(hipMemcpyAsync(d_pre.p, h_pre.p, nq * sizeof(CPre), hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_cand_hist, dim3((ncand + 255) / 256), dim3(256), 0, s, cands.p, ncand,
                         d_pre.p, d_chist.p);
      NURI_HIP(hipGetLastError());
      hipLaunchKernelGGL(k_cand_hist_topk, dim3(nq), dim3(256), 0, s, d_res.p, d_pre.p,
                         d_chist.p);
      NURI_HIP(hipGetLastError());
      hipLaunchKernelGGL(k_cand_thresh, dim3(nq), dim3(256), 0, s, d_k.p, d_pre.p, d_chist.p);
      NURI_HIP(hipGetLastError());
      NURI_HIP(hipMemsetAsync(d_ccount.p, 0, 4, s));
      hipLaunchKernelGGL(k_cand_compact, dim3((ncand + 255) / 256), dim3(256), 0, s, cands.p,
                         cand_ids.p, ncand, d_pre.p, cands2.p, cand_ids2.p, d_ccount.p);
      NURI_HIP(hipGetLastError());
      NURI_HIP(hipMemcpyAsync(h_ccount.p, d_ccount.p, 4, hipMemcpyDeviceToHost, s));
      NURI_HIP(hipStreamSynchronize(s));
      ncand = h_ccount.p[0];
      mc = cands2.p;
      mids = cand_ids2.p;
    } else {
      for (uint32_t i = 0; i < nq; ++i)
        if (sms()[i].cand_n) qh[i].top_seen = std::max(qh[i].top_seen, sms()[i].cand_max);
    }
    for (uint32_t f = 0, c = 1; f < ncand; f += kCandChunk, ++c) {
      // the merge kernels read the chunk size through StepHdr::cand_count;
      // each chunk's size has its own pinned slot, so nothing waits here
      h_ccount.p[c] = std::min<uint32_t>(kCandChunk, ncand - f);
      NURI_HIP(hipMemcpyAsync(&dh->cand_count, &h_ccount.p[c], 4, hipMemcpyHostToDevice, s));
      launch_merge(mc + f, dh, mids + (u64)f * QM, (uint32_t)QM, d_res.p, d_k.p, mbuf, nq, kmax,
                   h_ccount.p[c], s);
    }
    // the k-th scores come back with the next step's read-back (the host
    // plans one step with the previous ones, which only prunes less)
    NURI_HIP(hipMemcpyAsync(h_res.p, d_res.p, nq * sizeof(QRes), hipMemcpyDeviceToHost, s));
    theta_pending = true;
  }

  bool step_all() {
    make_roots();
    uint32_t nseg, batch_ub, maxc;
    u64 temp_need;
    bool any_sel;
    if (!plan(nseg, batch_ub, temp_need, maxc, any_sel)) return false;
    step(nseg, batch_ub, temp_need, maxc, any_sel);
    return true;
  }

  void harvest(uint32_t i, Result &res) {
    MQHost &Q = qh[i];
    NURI_HIP(hipMemcpyAsync(&h_res.p[i], &d_res.p[i], sizeof(QRes), hipMemcpyDeviceToHost, s));
    NURI_HIP(hipMemcpyAsync(&h_ctr.p[(u64)i * kCtrSlots], &d_ctr.p[(u64)i * kCtrSlots],
                            kCtrSlots * sizeof(MCtr), hipMemcpyDeviceToHost, s));
    NURI_HIP(hipStreamSynchronize(s));
    const QRes &R = h_res.p[i];
    const uint32_t n = Q.error ? 0 : R.tk_n, q = plans[i].q;
    std::vector<long long> sc(n);
    std::vector<unsigned int> ids((u64)n * QM);
    if (n) {
      NURI_HIP(hipMemcpyAsync(sc.data(), R.tk_score[R.cur], n * 8, hipMemcpyDeviceToHost, s));
      NURI_HIP(hipMemcpyAsync(ids.data(), R.tk_ids[R.cur], (u64)n * QM * 4,
                              hipMemcpyDeviceToHost, s));
      NURI_HIP(hipStreamSynchronize(s));
    }
    res.error = Q.error;
    res.errmsg = Q.errmsg;
    res.score.assign(sc.begin(), sc.end());
    res.offset.assign(1, 0);
    res.ids.clear();
    for (uint32_t t = 0; t < n; ++t) {
      res.ids.insert(res.ids.end(), ids.begin() + (u64)t * QM, ids.begin() + (u64)t * QM + q);
      res.offset.push_back(res.ids.size());
    }
    MCtr c;
    memset(&c, 0, sizeof(c));
    for (uint32_t t = 0; t < kCtrSlots; ++t) {
      const MCtr &e = h_ctr.p[(u64)i * kCtrSlots + t];
      c.popped += e.popped;
      c.expanded += e.expanded;
      c.children += e.children;
      c.pruned_pop += e.pruned_pop;
      c.pruned_new += e.pruned_new;
      c.leaves += e.leaves;
      c.offered += e.offered;
      c.logical_bytes += e.logical_bytes;
    }
    nuri_stats &st = res.stats;
    memset(&st, 0, sizeof(st));
    st.steps = Q.steps;
    st.popped = c.popped;
    st.expanded = c.expanded;
    st.children = c.children;
    st.pruned_at_pop = c.pruned_pop;
    st.pruned_at_creation = c.pruned_new;
    st.leaves = c.leaves;
    st.offered = c.offered;
    st.frontier_peak_bytes = Q.peak_bytes;
    st.spilled_bytes = Q.spilled_bytes;
    st.logical_bytes = c.logical_bytes;
    st.expand_launches = Q.launches;
    st.expand_ns = Q.expand_ns;
    st.wall_ns = now_ns() - Q.t_admit;
    st.ties_at_k = ties_at_k(res.score, Q.k);
    st.index_ns = Q.index_ns;
    Q.active = false;
    Q.stack.clear();
    tk[i]->score.release();
    tk[i]->len.release();
    tk[i]->ids.release();
    tk[i]->hdr.release();
    cfg[i].hdr = nullptr;
  }
};

}  // namespace

void run_matches(Graph &g, const std::vector<const nuri_pattern *> &ps,
                 const std::vector<uint32_t> &ks, const QueryOpts &o, std::vector<Result> &out) {
  if (ps.empty()) return;
  if (!g.has_lab) throw Error{NURI_EINVAL, "labelled matching needs vertex labels"};
  if (ps.size() > 65535) throw Error{NURI_EINVAL, "at most 65535 queries per batch"};
  // as many patterns live at once as the frontier budget holds arenas of
  // at least kMinArena bytes; the others wait for a slot
  constexpr u64 kMinArena = 4096 * sizeof(MRec);
  const uint32_t nq = (uint32_t)ps.size();
  const u64 per = std::max<u64>(kMinArena, o.frontier_budget / nq);
  const uint32_t slots = (uint32_t)std::max<u64>(1, std::min<u64>(nq, o.frontier_budget / per));
  MatchEngine e(g, o);
  e.setup(slots);
  e.arena_bytes = o.frontier_budget / slots;
  std::vector<uint32_t> slot_query(slots, UINT32_MAX);
  uint32_t next = 0;
  out.resize(nq);
  auto fill = [&] {
    for (uint32_t s = 0; s < slots && next < nq; ++s)
      if (e.slot_free(s)) {
        e.admit(s, *ps[next], ks[next]);
        slot_query[s] = next++;
      }
  };
  fill();
  for (;;) {
    const bool more = e.step_all();
    bool freed = false;
    for (uint32_t s = 0; s < slots; ++s)
      if (e.finished(s)) {
        e.harvest(s, out[slot_query[s]]);
        slot_query[s] = UINT32_MAX;
        freed = true;
      }
    if (freed) fill();
    if (!more && !e.any_live() && next >= nq) break;
  }
}

// ------------------------------------------------------------------
// slot interface for the server
// ------------------------------------------------------------------
struct MatchSlots::Impl {
  MatchEngine e;
  Impl(Graph &g, const QueryOpts &o) : e(g, o) {}
};

MatchSlots::MatchSlots(Graph &g, const QueryOpts &o, uint32_t slots) : impl(new Impl(g, o)) {
  if (!g.has_lab) throw Error{NURI_EINVAL, "labelled matching needs vertex labels"};
  impl->e.server_mode = true;
  impl->e.setup(slots);
}
MatchSlots::~MatchSlots() = default;
uint32_t MatchSlots::slots() const { return impl->e.nq; }
bool MatchSlots::free(uint32_t i) const { return impl->e.slot_free(i); }
bool MatchSlots::finished(uint32_t i) const { return impl->e.finished(i); }
bool MatchSlots::live() const { return impl->e.any_live(); }
void MatchSlots::admit(uint32_t i, const nuri_pattern &p, uint32_t k, uint64_t bytes) {
  impl->e.admit(i, p, k, bytes);
}
uint64_t MatchSlots::min_arena_bytes() const { return 4096 * sizeof(MRec); }
bool MatchSlots::step() { return impl->e.step_all(); }
void MatchSlots::harvest(uint32_t i, Result &r) { impl->e.harvest(i, r); }

}  // namespace nuri
