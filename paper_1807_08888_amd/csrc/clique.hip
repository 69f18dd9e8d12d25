// Top-k maximal clique discovery on the GPU.
//
// The paper's basic computational model (Algorithm 1, Section 3.2) with the
// clique user functions (Section 4.1, Listing 1), run as batched
// best-first steps:
//
//   select   the next records to expand: the deepest non-empty level of a
//            query's frontier, highest bound first (a radix-bucket select),
//            or the next unit subgraphs in bound order (lines 1-5);
//   expand   every record by every vertex of its ordered candidate set
//            (lines 12-14) with wavefront-wide bitmap intersections;
//   prune    children whose bound is below the current k-th score
//            (dominated, lines 11 and 15) -- strictly below, so ties survive;
//   offer    children with nothing left to add to the maximality check,
//            then merge the maximal ones into the top-k (lines 6-10);
//   append   the other children to the next level (line 16).
//
// Frontier records.  Vertices are ranks in a degeneracy order.  A partial
// clique s is kept as (root r, one bitmap over the local universe N+(r),
// last): r is its lowest-ranked vertex, bits at local positions <= last are
// the other members V_s, and bits above last are the candidate set P_s
// (common later neighbours, the ordered form of Listing 1's p()).  Since
// every member sits at or before `last` and every candidate after it, one
// bitmap of W = ceil(|N+(r)|/64) words holds both.  A second bitmap holds
// X_s: local positions outside s adjacent to all of s that were passed
// over earlier.  If some x in X_s is adjacent to all of P_s, x extends every
// clique s can grow into, none of them is maximal, and s is not created
// (targeted expansion, expandable() of Table 1).  A record is therefore a
// 32-byte header plus 2W words.
//
// A level holds records of one size |V|.  Priority is (|V|, bound): the
// deepest level is expanded first (the paper's (|V_s|, |P_s|) order for
// cliques), the highest bounds within it first.  The result never depends
// on the priority, the batch size or scheduling: pruning is strict and the
// top-k is merged under a total order.
#include <algorithm>
#include <climits>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "device_common.h"

namespace nuri {
namespace {


struct CRec {
  long long score;
  long long bound;
  u64 woff;       // low 48 bits: word offset of the bitmap in the query's word
                  // arena; high 16 bits: |P|, the number of candidates
  uint32_t root;  // rank of the root vertex
  int16_t last;   // local position of the last added vertex; -1 for a unit subgraph
  uint16_t qid;
};
static_assert(sizeof(CRec) == 32, "frontier record must stay 32 bytes");

constexpr uint32_t kWoffBits = 48;
constexpr u64 kWoffMask = (1ull << kWoffBits) - 1;
__device__ inline u64 pack_woff(u64 woff, uint32_t np) { return woff | ((u64)np << kWoffBits); }
__device__ inline uint32_t rec_np(const CRec &c) { return (uint32_t)(c.woff >> kWoffBits); }

struct LRec {  // a child with an empty candidate set, awaiting the maximality check
  long long score;
  u64 woff;  // word offset of its member bitmap in the leaf word arena
  uint32_t root;
  int16_t last;
  uint16_t qid;
};

struct QCfg {  // per query, written by the host each step
  CRec *hdr;
  u64 *words;
  u64 out_word;  // first word of the level this step appends to
  u64 word_cap;
  uint32_t out_hdr;  // first header slot of the level this step appends to
  uint32_t hdr_cap;
  uint32_t weighted;
  uint32_t k;
  uint32_t colour_min;  // colour cutoff for records with at least this many live
                        // children after the size cutoff (0 = never)
  uint32_t prio;        // NURI_PRIORITY_*: the selection key, and no pruning for NONE
};

// the k-th score the search prunes against: none without prioritization
// and pruning (the Nuri-NP order), where only the result set keeps the k best
__device__ inline long long prune_theta(const QCfg &c, const QRes &r) {
  return c.prio == NURI_PRIORITY_NONE ? LLONG_MIN : r.theta;
}

// selection key inside a level: the bound, or |P| for the paper's
// (|V|, |P|) clique priority
__device__ inline long long sel_key(const QCfg &c, const CRec &r) {
  return c.prio == NURI_PRIORITY_PAPER ? (long long)rec_np(r) : r.bound;
}

// per query, this step's counters (zeroed by the step upload); the two
// that wavefronts reserve child slots with have a cache line each
struct QStep {
  alignas(128) unsigned int n_out, pad;
  alignas(128) u64 out_words;
  alignas(128) u64 out_cost_children, out_cost_words;
  long long out_max_bound;
  u64 out_max_cc;  // largest children bound of one appended record
  unsigned int out_max_w, overflow;
};

// per query, this step's totals over the children written (kCtrSlots
// copies, one cache line each, added to when wavefronts end); k_qflush
// folds them into the QStep after the expansion and resets them
struct alignas(128) QFlush {
  u64 cost_children, cost_words, max_cc;
  long long max_bound;
  unsigned int max_w;
};

// per query, cumulative counters (kCtrSlots copies, one cache line each)
struct alignas(128) QCtr {
  u64 popped, expanded, children, pruned_pop, pruned_new, leaves, offered, logical_bytes;
  u64 onchip_bytes;  // adjacency rows read (cache-resident), apart from logical_bytes
};

struct GView {
  const uint32_t *dplus, *split, *oplus, *orig, *rcol, *hcol;
  const uint64_t *ooff, *bm_off, *rrow, *hrow;
  const u64 *bm;
  const int32_t *wloc, *vw;
  const int64_t *wplus;
  const uint32_t *root_order[2];
  uint32_t *wit;  // [n] a vertex u was found not adjacent to (~0u: none)
};

struct SelSeg {  // one query's level to take records from this step
  uint32_t qid, begin, count, take_all;
  uint32_t shift, temp_off;
  long long top;  // upper bound of every bound in the level
  u64 max_records, max_children, max_words;
  u64 maxcc;      // largest children bound of one record in the level
  u64 wpc;        // bitmap words per child, at most, in the level (2 W)
};

struct RootSeg {
  uint32_t qid, kind;
  uint32_t first, count;  // positions in the root order
};

// ------------------------------------------------------------------
// unit subgraphs (Algorithm 1, lines 1-3), taken in root-bound order
// grid: (x, segment)
// ------------------------------------------------------------------
__global__ void k_make_roots(GView g, const RootSeg *segs, CRec *batch, StepHdr *hdr) {
  const RootSeg sg = segs[blockIdx.y];
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < sg.count;
       i += gridDim.x * blockDim.x) {
    uint32_t r = g.root_order[sg.kind][sg.first + i];
    CRec c;
    c.score = sg.kind ? (long long)g.vw[r] : 1;
    c.bound = sg.kind ? c.score + g.wplus[r] : 1 + (long long)g.dplus[r];
    c.woff = pack_woff(0, g.dplus[r]);
    c.root = r;
    c.last = -1;
    c.qid = (uint16_t)sg.qid;
    batch[atomicAdd(&hdr->batch_count, 1u)] = c;
  }
}

// ------------------------------------------------------------------
// select: histogram of bounds, threshold, partition.  grid: (x, segment)
// ------------------------------------------------------------------
// A record at `last` in a universe of d can create at most d-last-1
// children.
__device__ inline u64 rec_children(const GView &g, const CRec &c) {
  return (u64)(g.dplus[c.root] - (uint32_t)(c.last + 1));
}

// per-block histograms in LDS, flushed with one atomic per non-empty bin
__global__ void __launch_bounds__(256)
    k_sel_hist(GView g, const SelSeg *segs, const QCfg *cfg, const QRes *res, unsigned int *hist,
               u64 *hchild) {
  __shared__ unsigned int s_h[kBins];
  __shared__ u64 s_c[kBins];
  const uint32_t s = blockIdx.y;
  const SelSeg sg = segs[s];
  if (sg.take_all) return;
  for (int b = threadIdx.x; b < kBins; b += blockDim.x) {
    s_h[b] = 0;
    s_c[b] = 0;
  }
  __syncthreads();
  const QCfg cf = cfg[sg.qid];
  const long long theta = prune_theta(cf, res[sg.qid]);
  const CRec *h = cf.hdr + sg.begin;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < sg.count;
       i += gridDim.x * blockDim.x) {
    const CRec c = h[i];
    if (c.bound < theta) continue;
    int b = bin_of(sel_key(cf, c), sg.top, sg.shift);
    atomicAdd(&s_h[b], 1u);
    atomicAdd(&s_c[b], rec_children(g, c));
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kBins; b += blockDim.x)
    if (s_h[b]) {
      atomicAdd(&hist[(size_t)s * kBins + b], s_h[b]);
      atomicAdd(&hchild[(size_t)s * kBins + b], s_c[b]);
    }
}

// threshold bin and quota of each segment (block_select_threshold), then
// the bins are cleared for the next step.  grid: (segment), 256 threads
__global__ void __launch_bounds__(kSelThreads)
    k_sel_thresh(const SelSeg *segs, uint32_t nseg, unsigned int *hist, u64 *hchild, int *thr,
                 unsigned int *quota) {
  const uint32_t s = blockIdx.x;
  if (s >= nseg) return;
  const SelSeg sg = segs[s];
  if (sg.take_all) return;
  unsigned int *h = hist + (size_t)s * kBins;
  u64 *hc = hchild + (size_t)s * kBins;
  const SelLimits lim{sg.max_records, sg.max_children, sg.max_words, sg.wpc, sg.maxcc};
  block_select_threshold(h, hc, lim, &thr[s], &quota[s]);
  __syncthreads();
  for (int b = threadIdx.x; b < kBins; b += blockDim.x) {
    h[b] = 0;
    hc[b] = 0;
  }
}

__global__ void k_sel_part(const SelSeg *segs, const QCfg *cfg, const QRes *res, const int *thr,
                           const unsigned int *quota, unsigned int *taken, CRec *batch,
                           StepHdr *hdr, CRec *temp, unsigned int *temp_count, QCtr *ctr) {
  const uint32_t s = blockIdx.y;
  const SelSeg sg = segs[s];
  const QCfg cf = cfg[sg.qid];
  const long long theta = prune_theta(cf, res[sg.qid]);
  const CRec *h = cf.hdr + sg.begin;
  const int t = sg.take_all ? -1 : thr[s];
  const unsigned int qt = sg.take_all ? 0 : quota[s];
  unsigned int pruned = 0;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < sg.count;
       i += gridDim.x * blockDim.x) {
    const CRec c = h[i];
    int where;  // 1 batch, 2 keep, 3 pruned
    if (c.bound < theta) {
      where = 3;
    } else if (sg.take_all) {
      where = 1;
    } else {
      int b = bin_of(sel_key(cf, c), sg.top, sg.shift);
      if (b > t) where = 1;
      else if (b < t) where = 2;
      else where = atomicAdd(&taken[s], 1u) < qt ? 1 : 2;
    }
    if (where == 1) batch[atomicAdd(&hdr->batch_count, 1u)] = c;
    else if (where == 2) temp[sg.temp_off + atomicAdd(&temp_count[s], 1u)] = c;
    else ++pruned;
  }
  if (pruned) {
    QCtr &C = ctr[sg.qid * kCtrSlots + (blockIdx.x & (kCtrSlots - 1))];
    atomicAdd(&C.popped, (u64)pruned);
    atomicAdd(&C.pruned_pop, (u64)pruned);
  }
}

// records moved down in their arena by the frontier spill: their word
// offsets move down by the same shift (the |P| bits above stay as they are)
__global__ void k_rebase(CRec *h, u64 n, u64 wshift) {
  for (u64 i = blockIdx.x * (u64)blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x)
    h[i].woff -= wshift;
}

__global__ void k_copy_back(const SelSeg *segs, const QCfg *cfg, const CRec *temp,
                            const unsigned int *temp_count) {
  const uint32_t s = blockIdx.y;
  const SelSeg sg = segs[s];
  const unsigned int kept = sg.take_all ? 0u : temp_count[s];
  CRec *h = cfg[sg.qid].hdr + sg.begin;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < kept; i += gridDim.x * blockDim.x)
    h[i] = temp[sg.temp_off + i];
}

// ------------------------------------------------------------------
// seed cliques: an early k-th score
// ------------------------------------------------------------------
// Before the search, one wavefront per root (the first `count` roots in
// bound order) builds a clique greedily: starting from the root's later
// neighbours it adds the highest remaining position (with vertex weights,
// also the heaviest remaining candidate, keeping the heavier clique) and
// keeps the positions adjacent to it, until none is left.  The result goes through
// the same maximality check and merge as any leaf, so the k-th score
// starts at the k-th best of these cliques instead of at minus infinity;
// any k maximal cliques give a valid lower bound of the final k-th score.
// The search later finds these cliques again; the merge drops a candidate
// equal to an item already in the top-k.
struct SeedSeg {
  uint32_t qid, kind, count, pad;
};

__global__ void __launch_bounds__(256)
    k_seed_dive(GView g, const SeedSeg *segs, LRec *leaves, u64 *leaf_words, StepHdr *hdr,
                uint32_t leaf_cap, u64 leaf_word_cap, QStep *qs) {
  const int lane = threadIdx.x & 63;
  const SeedSeg sg = segs[blockIdx.y];
  const uint32_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= sg.count) return;
  const uint32_t r = g.root_order[sg.kind][i];
  const uint32_t d = g.dplus[r];
  const uint32_t W = words_of(d);
  const int32_t *wl = g.wloc + g.ooff[r];
  const u64 *rows = g.bm + g.bm_off[r];
  // one greedy clique: add the highest remaining position (by_weight:
  // the heaviest remaining candidate, ties to the highest position)
  auto dive = [&](bool by_weight, u64 &V, int &last) -> long long {
    long long score = sg.kind ? (long long)g.vw[r] : 1ll;
    u64 P = (lane < (int)W) ? lt_mask(lane, d) : 0ull;
    V = 0;
    last = -1;
    while (__ballot(P != 0)) {
      int hb;
      if (by_weight) {
        // (weight, position) maximum: this lane's word, then the wave
        long long best = -1;
        for (u64 t = P; t; t &= t - 1) {
          const int pos = lane * 64 + __ffsll((long long)t) - 1;
          const long long key = ((long long)wl[pos] << 13) | pos;
          best = key > best ? key : best;
        }
        for (int o2 = 32; o2 > 0; o2 >>= 1) {
          const long long y = __shfl_xor(best, o2, 64);
          best = y > best ? y : best;
        }
        hb = (int)(best & 8191);
      } else {
        hb = wave_highest_bit(P);
      }
      last = hb;
      score += sg.kind ? (long long)wl[hb] : 1ll;
      if (lane == (hb >> 6)) {
        V |= 1ull << (hb & 63);
        P &= ~(1ull << (hb & 63));
      }
      if (lane < (int)W) P &= rows[(u64)hb * W + lane];
    }
    return score;
  };
  u64 V = 0;
  int last = -1;
  long long score = dive(false, V, last);
  if (sg.kind) {
    // vertex weights: keep the heavier of the two greedy cliques
    u64 V2 = 0;
    int last2 = -1;
    const long long score2 = dive(true, V2, last2);
    if (score2 > score) {
      score = score2;
      V = V2;
      last = last2;
    }
  }
  unsigned int slot = 0;
  u64 w0 = 0;
  if (lane == 0) {
    slot = atomicAdd(&hdr->leaf_count, 1u);
    w0 = atomicAdd(&hdr->leaf_word_count, (u64)W);
  }
  slot = __shfl(slot, 0, 64);
  w0 = __shfl(w0, 0, 64);
  if (slot >= leaf_cap || w0 + W > leaf_word_cap) {
    if (lane == 0) atomicAdd(&qs[sg.qid].overflow, 1u);
    return;
  }
  if (lane < (int)W) leaf_words[w0 + lane] = V;
  if (lane == 0) {
    LRec l;
    l.score = score;
    l.woff = w0;
    l.root = r;
    l.last = (int16_t)last;
    l.qid = (uint16_t)sg.qid;
    leaves[slot] = l;
  }
}

// ------------------------------------------------------------------
// expand (Algorithm 1, lines 11-16)
// ------------------------------------------------------------------
// One wavefront per record.  The record's candidate positions are listed
// in LDS.  Child idx (the idx-th candidate) can reach at most
// score + (weight of candidates idx, idx+1, ...), so every child past the
// first idx where that falls below the k-th score is dominated before it
// is built (the Carraghan-Pardalos cutoff); those are counted as created
// and pruned without touching memory.  The remaining children are built
// one per lane, 64 at a time: a lane ANDs the parent's bitmap words with
// its child vertex's local adjacency row, word by word, and gets |P'|
// (or w(P')), the first vertex of X' and the witness test without
// reductions between lanes; the survivors of a round are compacted with a
// ballot, placed with one atomic per wave and written by their lanes.
//
// Whole records: when at most one candidate may be left out and the k-th
// score still be reached, the subtree's only possible results are V + P
// and V + P minus one vertex; one pass over all candidates' rows finds
// them (see below).
//
// Chains: when a record keeps exactly one child, the wave expands that
// child at once instead of writing it to the frontier and waiting for a
// later step.  Dense regions make such chains hundreds of vertices long
// (one per clique member), so this turns hundreds of steps into one.  The
// order in which records are expanded does not change the result: every
// expansion prunes against a valid lower bound of the k-th score.
//
// LDS per wave (dynamic, sized by the largest local row of the graph):
// five bitmaps of wst words (parent P, parent V, parent X, carried child
// V+P, carried child X), a candidate list of lst u16 positions and, for
// vertex-weight scores, the root's lst local weights.
// one wavefront per workgroup: a record's wavefront frees its slot as soon
// as it ends, instead of waiting for the slowest of its group
constexpr int kExpandWaves = 1;
// links one wavefront chains (by default) before it writes the held child
// to the frontier instead: a launch lasts as long as its longest chain, and
// an unbounded chain (hundreds of links down a near-clique) leaves most of
// the device idle at the end of every launch
constexpr uint32_t kMaxLinks = 32;

// f(w, row[w]) for the W words of a local adjacency row, in order.  Rows
// of up to 16 words (1,024 local positions) are loaded whole before the
// first word is used, so that all their loads are in flight together
// instead of in dependent groups.
template <class F>
__device__ inline void row_words(const u64 *row, uint32_t W, F &&f) {
  if (W <= 16) {
    u64 v[16];
#pragma unroll
    for (uint32_t w = 0; w < 16; ++w) v[w] = w < W ? row[w] : 0ull;
#pragma unroll
    for (uint32_t w = 0; w < 16; ++w)
      if (w < W) f(w, v[w]);
  } else {
    for (uint32_t w = 0; w < W; ++w) f(w, row[w]);
  }
}

// f(w, row[w]) and f(w, r1[w], r2[w]) in a plain loop: the expansion
// kernel's occupancy is bound by its registers, and there these keep
// fewer of them live than row_words
template <class F>
__device__ inline void row_loop(const u64 *row, uint32_t W, F &&f) {
#pragma unroll 4
  for (uint32_t w = 0; w < W; ++w) f(w, row[w]);
}

template <class F>
__device__ inline void row_loop2(const u64 *r1, const u64 *r2, uint32_t W, F &&f) {
#pragma unroll 4
  for (uint32_t w = 0; w < W; ++w) f(w, r1[w], r2[w]);
}

__device__ inline void put_crec(CRec *hdr, u64 slot, long long score, long long bound, u64 woff,
                                uint32_t np, uint32_t root, int j, uint32_t q) {
  CRec ch;
  ch.score = score;
  ch.bound = bound;
  ch.woff = pack_woff(woff, np);
  ch.root = root;
  ch.last = (int16_t)j;
  ch.qid = (uint16_t)q;
  hdr[slot] = ch;
}

__global__ void __launch_bounds__(64 * kExpandWaves)
    k_expand(GView g, const CRec *__restrict__ batch, StepHdr *hdr, const QCfg *__restrict__ cfg,
             QStep *qs, QCtr *ctr, QFlush *flush, const QRes *__restrict__ res, LRec *leaves,
             u64 *leaf_words,
             uint32_t leaf_cap, u64 leaf_word_cap, uint32_t wst, uint32_t lst, u64 chain_cap,
             uint32_t max_links) {
  extern __shared__ u64 s_dyn[];
  __shared__ long long s_cscore[kExpandWaves], s_cbound[kExpandWaves];
  __shared__ int s_cj[kExpandWaves];
  __shared__ uint32_t s_ccnt[kExpandWaves];
  __shared__ u64 s_cost[kExpandWaves], s_maxcc[kExpandWaves];
  __shared__ long long s_maxb[kExpandWaves];
  __shared__ u64 s_st[kExpandWaves][9];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  u64 *s_pw = s_dyn + (u64)wv * 5 * wst;
  u64 *s_vw = s_pw + wst;
  u64 *s_xw = s_vw + wst;
  u64 *s_cv = s_xw + wst;  // carried child: V + P bitmap
  u64 *s_cx = s_cv + wst;  // carried child: X bitmap
  uint16_t *s_list = (uint16_t *)(s_dyn + (u64)kExpandWaves * 5 * wst) + (u64)wv * lst;
  // the root's local vertex weights (vertex-weight scores only)
  int32_t *s_wl = (int32_t *)((uint16_t *)(s_dyn + (u64)kExpandWaves * 5 * wst) +
                              (u64)kExpandWaves * lst) + (u64)wv * lst;
  const uint32_t rec = blockIdx.x * kExpandWaves + wv;
  if (rec >= hdr->batch_count) return;
  CRec p = batch[rec];
  const uint32_t q = p.qid;
  const QCfg cf = cfg[q];
  const long long theta = prune_theta(cf, res[q]);
  const bool weighted = cf.weighted != 0;
  // wave-uniform work counters, kept in LDS by lane 0 rather than in
  // registers (they live across the whole kernel, and every register counts
  // against occupancy); the per-child ones of written children are gathered
  // in LDS by the lanes that write them
  enum {
    ST_POPPED, ST_PRUNED_POP, ST_EXPANDED, ST_CHILDREN, ST_PRUNED_NEW, ST_LEAVES,
    ST_BYTES,   // frontier records and leaves read and written
    ST_ONCHIP,  // local adjacency rows read (L2-resident)
    ST_MARK,    // pruned count before this record's children (undone by absorption)
    ST_N
  };
  u64 *st = s_st[wv];
  auto stat = [&](int i, u64 v) {
    if (lane == 0) st[i] += v;
  };
  if (lane == 0) {
    for (int i = 0; i < ST_N; ++i) st[i] = 0;
    s_cost[wv] = 0;
    s_maxcc[wv] = 0;
    s_maxb[wv] = LLONG_MIN;
  }

  const uint32_t r = p.root;
  const uint32_t d = g.dplus[r];
  const uint32_t W = words_of(d);
  // every record and chained link of this wavefront has root r: with vertex
  // weights, the root's local weights are read into LDS once, so that the
  // per-child sums over P' (one lane per child, a bit at a time) read LDS.
  // Not for a record pruned when popped (or without later neighbours): the
  // wavefront ends with it.
  if (weighted && p.bound >= theta && d) {
    const int32_t *gwl = g.wloc + g.ooff[r];
#pragma unroll 8
    for (uint32_t t = lane; t < d; t += 64) s_wl[t] = gwl[t];
    wave_sync();
  }
  const int32_t *wl = s_wl;
  const u64 *rows = g.bm + g.bm_off[r];
  uint32_t G = 1;
  while (G < W) G <<= 1;
  const uint32_t per = 64 / G;
  const int wi = lane & (G - 1);
  bool carried = false;  // p is a kept child carried over from the previous link
  u64 credit = 0;        // leaf slots reserved for chained links, not yet used (lane 0)
  uint32_t links = 0;    // chained links expanded by this wave
  // write the held child (s_cv, s_cx, s_c*) to header slot hs, word slot ws
  auto write_held = [&](u64 hs, u64 ws) {
    if (lane < (int)W) {
      cf.words[ws + lane] = s_cv[lane];
      cf.words[ws + W + lane] = s_cx[lane];
    }
    if (lane == 0) {
      const int jc = s_cj[wv];
      put_crec(cf.hdr, hs, s_cscore[wv], s_cbound[wv], ws, s_ccnt[wv], r, jc, q);
      const u64 cc = (u64)(d - jc - 1);
      atomicAdd(&s_cost[wv], cc);
      atomicMax(&s_maxcc[wv], cc);
      atomicMax(&s_maxb[wv], s_cbound[wv]);
    }
    stat(ST_BYTES, 32 + 16ull * W);
  };

  for (;;) {
    stat(ST_POPPED, 1);
    if (p.bound < theta) {
      stat(ST_PRUNED_POP, 1);
      break;
    }
    if (d == 0) {
      // a unit subgraph with no later neighbour: itself a leaf
      stat(ST_LEAVES, 1);
      if (p.score >= theta && lane == 0) {
        unsigned int slot = atomicAdd(&hdr->leaf_count, 1u);
        if (slot < leaf_cap) {
          LRec l;
          l.score = p.score;
          l.woff = 0;
          l.root = r;
          l.last = -1;
          l.qid = (uint16_t)q;
          leaves[slot] = l;
        } else {
          atomicAdd(&qs[q].overflow, 1u);
        }
      }
      break;
    }
    const int last = p.last;
    u64 word = 0, xword = 0;
    if (lane < (int)W) {
      if (carried) {
        word = s_cv[lane];
        xword = s_cx[lane];
      } else {
        const u64 wo = p.woff & kWoffMask;
        word = last < 0 ? lt_mask(lane, d) : cf.words[wo + lane];
        xword = last < 0 ? 0ull : cf.words[wo + W + lane];
      }
    }
    const u64 pw = word & gt_mask(lane, last);
    const u64 vwd = word & ~gt_mask(lane, last);
    wave_sync();  // every lane has read the carried child before it is replaced
    if (lane < (int)W) {
      s_pw[lane] = pw;
      s_vw[lane] = vwd;
      s_xw[lane] = xword;
    }
    // candidates in increasing position: this lane holds positions
    // [off, off + c) of the list
    const uint32_t c = __popcll(pw);
    const uint32_t off = wave_excl_scan(c, lane);
    const uint32_t nchild = __shfl(off + c, 63, 64);
    // cutoff: child idx reaches at most score + (weight of candidates
    // idx, idx+1, ...); past the first idx where that is below theta every
    // child is dominated
    uint32_t n_eff = nchild;
    // whole: at most one candidate may be left out and theta still be
    // reached, so the subtree's only possible results are V + P and V + P
    // minus one vertex, found directly
    bool whole = false;
    int wslack = 0;         // whole: how many candidates may be left out (0 or 1)
    long long wR = 0;       // whole, vertex weights: a left-out candidate weighs at most wR
    long long wP = nchild;  // weight of the candidate set
    if (theta != LLONG_MIN) {
      if (!weighted) {
        // each candidate weighs 1: child idx reaches score + nchild - idx
        const long long R = p.score + (long long)nchild - theta;
        n_eff = R < 0 ? 0u : (uint32_t)(R + 1 < (long long)nchild ? R + 1 : nchild);
        whole = (R == 0 || R == 1) && nchild > 0;
        wslack = (int)R;
      } else {
        // one word at a time, one lane per bit: coalesced weight loads and
        // wave reductions instead of a serial walk over each word's bits
        long long total = 0;
        uint32_t m1 = INT32_MAX, m2 = INT32_MAX;  // the two smallest weights
        for (uint32_t w = 0; w < W; ++w) {
          const u64 word = readlane64(pw, (int)w);
          const bool set = (word >> lane) & 1ull;
          const int32_t x = set ? wl[w * 64 + lane] : 0;
          total += (long long)wave_sum((u64)x);
          const uint32_t xv = set ? (uint32_t)x : (uint32_t)INT32_MAX;
          const uint32_t a = wave_min_u32(xv);
          const uint32_t b = __popcll(__ballot(set && xv == a)) >= 2
                                 ? a
                                 : wave_min_u32(xv == a ? (uint32_t)INT32_MAX : xv);
          if (a < m1) {
            m2 = min(m1, b);
            m1 = a;
          } else {
            m2 = min(m2, a);
          }
        }
        wP = total;
        const long long R = total + p.score - theta;
        // at most one candidate can be left out when any two weigh more
        // than the slack R
        whole = R >= 0 && R < (long long)m1 + (long long)m2 && nchild > 0;
        wslack = R >= (long long)m1 ? 1 : 0;
        wR = R;
        // first candidate index whose preceding candidates weigh more than R
        uint32_t cut = 0xFFFFFFFFu;
        if (R < 0) {
          cut = 0;
        } else if (total > R) {
          long long run = 0;
          uint32_t base = 0;
          for (uint32_t w = 0; w < W; ++w) {
            const u64 word = readlane64(pw, (int)w);
            const bool set = (word >> lane) & 1ull;
            const long long x = set ? (long long)wl[w * 64 + lane] : 0ll;
            const long long excl = wave_excl_scan64(x, lane);
            const u64 hit = __ballot(set && run + excl > R);
            if (hit) {
              const int f = __ffsll((long long)hit) - 1;
              cut = base + (uint32_t)__popcll(word & ((1ull << f) - 1ull));
              break;
            }
            run += (long long)__shfl(excl + x, 63, 64);
            base += (uint32_t)__popcll(word);
          }
        }
        cut = wave_min_u32(cut);
        if (cut < n_eff) n_eff = cut;
      }
      // colour-class cutoff (a tighter bound than Carraghan-Pardalos, the
      // direction the paper leaves to future work): split the candidates
      // into independent sets, each built greedily from the highest
      // remaining position down.  The first vertex of class c is the
      // highest uncoloured one, so class tops decrease; a clique in the
      // subtree of child j uses at most one vertex of each class that
      // reaches position j, so child j can score at most
      // score + (sum of the max weights of classes whose top is >= j).
      // Classes are built until that sum reaches theta - score; children
      // above the top of the last class built are dominated.
      const long long need = theta - p.score;
      if (!whole && cf.colour_min && n_eff >= cf.colour_min && need > 0) {
        // Once the classes built so far plus the weight of everything not
        // yet coloured fall below need, no child survives: stop there
        // (most records that reach this point are such dead ends).
        u64 U = pw, Q = 0;
        long long run = 0, wU = wP;
        bool dead = false;
        int cut_pos = -1;  // children at positions <= cut_pos survive
        while (__ballot(U != 0)) {
          Q = U;
          long long cmax = 0;
          int top = -1;
          while (__ballot(Q != 0)) {
            const int hb = wave_highest_bit(Q);
            if (top < 0) top = hb;
            const long long wv2 = weighted ? (long long)wl[hb] : 1ll;
            cmax = wv2 > cmax ? wv2 : cmax;
            wU -= wv2;
            if (lane == (hb >> 6)) {
              const u64 bit = 1ull << (hb & 63);
              U &= ~bit;
              Q &= ~bit;
            }
            if (lane < (int)W) Q &= ~rows[(u64)hb * W + lane];
            if (run + cmax + wU < need) {
              dead = true;
              break;
            }
          }
          if (dead) break;
          run += cmax;
          if (run >= need) {
            cut_pos = top;
            break;
          }
        }
        // children surviving: candidates at positions <= cut_pos
        uint32_t keep_n = 0;
        if (cut_pos >= 0) {
          const u64 m = (lane < (int)W) ? (pw & ~gt_mask(lane, cut_pos)) : 0ull;
          keep_n = (uint32_t)wave_sum((u64)__popcll(m));
        }
        if (keep_n < n_eff) n_eff = keep_n;
      }
    }
    // list the positions of the children that get built
    const uint32_t n_list = whole ? nchild : n_eff;
    {
      uint32_t o = off;
      for (u64 t = pw; t && o < n_list; t &= t - 1)
        s_list[o++] = (uint16_t)(lane * 64 + __ffsll((long long)t) - 1);
    }
    wave_sync();
    if (last >= 0) stat(ST_BYTES, 32 + 16ull * W);  // the parent record
    if (nchild) stat(ST_EXPANDED, 1);
    stat(ST_CHILDREN, nchild);
    if (whole) {
      // Every candidate's row at once (the loads are independent): for each
      // candidate the number of other candidates it is not adjacent to.
      // With slack 0 the only possible result is V + P (P a clique); with
      // slack 1 it is V + P or V + P - {x}, and P - {x} is a clique iff
      // every non-adjacent pair of P contains x.  Also a vertex of X
      // adjacent to all of P extends V + P, which is then not maximal.
      u64 xacc = (wi < (int)W) ? s_xw[wi] : 0ull;
      uint32_t zc = 0, msum = 0, zlo = 0xFFFFFFFFu, zhi = 0, mbest = 0, mpos = 0;
      // With slack 1, V + P - {x} needs every non-adjacent pair of P to
      // contain x (the pairs form a star around x), so two candidates with
      // two or more misses each rule out every x: the pass stops there,
      // as it stops with slack 0 at the first miss.
      uint32_t n2 = 0;     // candidates seen with two or more misses
      bool dead = false;   // no result is possible
      u64 rows_read = 0;   // candidates whose rows were read
      if (W >= 2) {
        // one candidate per lane, its W words in sequence (independent
        // loads): 64 candidates per round and no group reductions
        for (uint32_t b0 = 0; b0 < nchild; b0 += 64) {
          const uint32_t ci = b0 + lane;
          uint32_t miss = 0;
          rows_read += nchild - b0 < 64 ? nchild - b0 : 64;
          if (ci < nchild) {
            const uint32_t j = s_list[ci];
            const uint32_t jw = j >> 6;
            const u64 jb = 1ull << (j & 63);
            const u64 *rj = rows + (u64)j * W;
            row_loop(rj, W, [&](uint32_t w, u64 rw) {
              miss += __popcll(s_pw[w] & ~(w == jw ? jb : 0ull) & ~rw);
            });
            if (miss) {
              ++zc;
              msum += miss;
              zlo = j < zlo ? j : zlo;
              zhi = j > zhi ? j : zhi;
              if (miss > mbest) {
                mbest = miss;
                mpos = j;
              }
            }
          }
          if (wslack == 0 && __ballot(zc != 0)) break;  // P is not a clique
          n2 += __popcll(__ballot(miss >= 2));
          if (n2 >= 2) {
            dead = true;
            break;
          }
        }
        xacc = 0;  // X is tested below, only if P is a clique
      } else
      for (uint32_t b0 = 0; b0 < nchild; b0 += 8 * per) {
        rows_read += nchild - b0 < 8 * per ? nchild - b0 : 8 * per;
        for (uint32_t u = 0; u < 8; ++u) {
          const uint32_t ci = b0 + u * per + lane / G;
          const bool valid = ci < nchild;
          uint32_t miss = 0, j = 0;
          if (valid && wi < (int)W) {
            j = s_list[ci];
            const u64 own = (wi == (int)(j >> 6)) ? (1ull << (j & 63)) : 0ull;
            const u64 row = rows[(u64)j * W + wi];
            miss = __popcll(s_pw[wi] & ~own & ~row);
            xacc &= row;
          }
          for (uint32_t o2 = 1; o2 < G; o2 <<= 1) miss += __shfl_xor(miss, o2, 64);
          n2 += __popcll(__ballot(valid && wi == 0 && miss >= 2));
          if (valid && wi == 0 && miss) {
            ++zc;
            msum += miss;
            zlo = j < zlo ? j : zlo;
            zhi = j > zhi ? j : zhi;
            if (miss > mbest) {
              mbest = miss;
              mpos = j;
            }
          }
        }
        if (wslack == 0 && __ballot(zc != 0)) break;  // P is not a clique
        if (n2 >= 2) {
          dead = true;
          break;
        }
      }
      stat(ST_ONCHIP, 8ull * W * rows_read);
      zc = (uint32_t)wave_sum((u64)zc);
      msum = (uint32_t)wave_sum((u64)msum);
      zlo = wave_min_u32(zlo);
      zhi = (uint32_t)wave_max_u64((u64)zhi);
      {
        const u64 key = wave_max_u64(((u64)mbest << 32) | mpos);
        mbest = (uint32_t)(key >> 32);
        mpos = (uint32_t)key;
      }
      // AND the X accumulators of the lane groups holding the same word
      for (uint32_t o2 = G; o2 < 64; o2 <<= 1) xacc &= __shfl_xor(xacc, o2, 64);
      int drop0 = -2, drop1 = -2;  // dropped position per leaf; -1 none, -2 no leaf
      if (zc == 0 && W >= 2) {
        // P is a clique: V + P is maximal unless a vertex of X is adjacent
        // to all of P.  X's positions go to the candidate list (no longer
        // needed), one per lane, each tested against P word by word.
        wave_sync();
        const u64 xw = (lane < (int)W) ? s_xw[lane] : 0ull;
        const uint32_t xc = __popcll(xw);
        const uint32_t xo = wave_excl_scan(xc, lane);
        const uint32_t nx = __shfl(xo + xc, 63, 64);
        {
          uint32_t o = xo;
          for (u64 t = xw; t; t &= t - 1) s_list[o++] = (uint16_t)(lane * 64 + __ffsll((long long)t) - 1);
        }
        wave_sync();
        bool ext = false;
        for (uint32_t b0 = 0; b0 < nx && !ext; b0 += 64) {
          bool all = false;
          if (b0 + lane < nx) {
            const u64 *rx = rows + (u64)s_list[b0 + lane] * W;
            u64 out = 0;
            row_loop(rx, W, [&](uint32_t w, u64 rxw) { out |= s_pw[w] & ~rxw; });
            all = out == 0;
          }
          ext = __ballot(all) != 0;
        }
        stat(ST_ONCHIP, 8ull * W * nx);
        if (!ext) drop0 = -1;
      } else if (zc == 0) {
        if (!__ballot(wi < (int)W && xacc != 0ull)) drop0 = -1;
      } else if (!dead && wslack >= 1 && msum / 2 == mbest) {
        if (mbest == 1) {
          drop0 = (int)zlo;
          drop1 = (int)zhi;
        } else {
          drop0 = (int)mpos;
        }
        // with vertex weights a left-out candidate must weigh at most the slack
        if (weighted) {
          if (drop1 >= 0 && (long long)wl[drop1] > wR) drop1 = -2;
          if (drop0 >= 0 && (long long)wl[drop0] > wR) {
            drop0 = drop1;
            drop1 = -2;
          }
        }
      }
      const uint32_t nl = (drop0 != -2) + (drop1 != -2);
      stat(ST_PRUNED_NEW, nchild - (nl ? 1 : 0));
      stat(ST_LEAVES, nl);
      n_eff = 0;  // no child is built one by one
      if (nl) {
        const long long tot = weighted ? wP : (long long)nchild;
        unsigned int l0 = 0;
        u64 w0 = 0;
        if (lane == 0) {
          l0 = atomicAdd(&hdr->leaf_count, nl);
          w0 = atomicAdd(&hdr->leaf_word_count, (u64)nl * W);
        }
        l0 = __shfl(l0, 0, 64);
        w0 = __shfl(w0, 0, 64);
        if (l0 + nl <= leaf_cap && w0 + (u64)nl * W <= leaf_word_cap) {
          for (uint32_t t = 0; t < nl; ++t) {
            const int dp = t == 0 ? drop0 : drop1;
            const u64 dbit = (dp >= 0 && lane == (dp >> 6)) ? (1ull << (dp & 63)) : 0ull;
            if (lane < (int)W) leaf_words[w0 + (u64)t * W + lane] = (s_vw[lane] | s_pw[lane]) & ~dbit;
            if (lane == 0) {
              LRec l;
              l.score = p.score + tot - (dp >= 0 ? (weighted ? (long long)wl[dp] : 1ll) : 0ll);
              l.woff = w0 + (u64)t * W;
              l.root = r;
              l.last = (int16_t)last;
              l.qid = (uint16_t)q;
              leaves[l0 + t] = l;
            }
          }
          stat(ST_BYTES, (24 + 8ull * W) * nl);
        } else if (lane == 0) {
          atomicAdd(&qs[q].overflow, 1u);
        }
      }
    } else {
      if (lane == 0) st[ST_MARK] = st[ST_PRUNED_NEW];
      stat(ST_PRUNED_NEW, nchild - n_eff);
    }
    // Screening, for records with more than 64/G children (G = the power
    // of two >= W): one child per lane, as in the build below but without
    // writing anything, gives |P'| -- with vertex weights an upper bound of
    // w(P'): the bits of each word times the heaviest candidate in that
    // word, which spares the exact sum for most children -- and the first
    // vertex of X' with the test whether it is adjacent to all of P'.
    // Children that this bound or the witness rule out are counted as
    // pruned here; the others, in order, replace the list and are built
    // below, where the exact test is repeated.
    // A run of first candidates each adjacent to all the others is in every
    // maximal clique below the record (any clique of the subtree extends by
    // them), and a chain would add them one link at a time; the screening's
    // first round finds such a run (candidate i, in position order, sees
    // all nchild - 1 - i later candidates) and absorbs it below.
    bool absorbed = false, absorb_keep = false;
    uint32_t absorb_n = 0;  // length of the run
    if (!whole && n_eff > per && W >= 2) {
      int32_t wmx = 0;  // lane w: heaviest candidate of word w
      if (weighted)
        for (uint32_t w = 0; w < W; ++w) {
          const u64 word = readlane64(pw, (int)w);
          const uint32_t x = ((word >> lane) & 1ull) ? (uint32_t)wl[w * 64 + lane] : 0u;
          const uint32_t m = (uint32_t)wave_max_u64((u64)x);
          if (lane == (int)w) wmx = (int32_t)m;
        }
      uint32_t kept = 0;
      bool uni0 = false;  // first round: this lane's candidate sees all later ones
      for (uint32_t b0 = 0; b0 < n_eff; b0 += 64) {
        const uint32_t ci = b0 + lane;
        const bool valid = ci < n_eff;
        const uint32_t j = valid ? s_list[ci] : 0;
        const u64 *rj = rows + (u64)j * W;
        uint32_t cnt = 0;
        long long wub = 0;
        int x0 = -1;
        if (valid) {
          row_loop(rj, W, [&](uint32_t w, u64 row) {
            const u64 pv = s_pw[w];
            const u64 a = pv & row & gt_mask((int)w, (int)j);
            const uint32_t c = __popcll(a);
            cnt += c;
            if (weighted) wub += (long long)c * __builtin_amdgcn_readlane(wmx, (int)w);
            const u64 xc = (s_xw[w] | (pv & ~gt_mask((int)w, (int)j - 1))) & row;
            if (x0 < 0 && xc) x0 = (int)w * 64 + __ffsll((long long)xc) - 1;
          });
        }
        if (b0 == 0) uni0 = valid && cnt == nchild - 1 - ci;
        const long long score2 = p.score + (weighted ? (long long)wl[j] : 1ll);
        bool pass = valid && score2 + (weighted ? wub : (long long)cnt) >= theta;
        if (pass && x0 >= 0) {
          const u64 *rx = rows + (u64)x0 * W;
          u64 out = 0;
          row_loop2(rj, rx, W, [&](uint32_t w, u64 rjw, u64 rxw) {
            out |= s_pw[w] & rjw & gt_mask((int)w, (int)j) & ~rxw;
          });
          pass = out != 0;  // covered when x0 is adjacent to all of P'
        }
        const u64 pm = __ballot(pass);
        stat(ST_PRUNED_NEW, __popcll(__ballot(valid && !pass)));
        stat(ST_ONCHIP, 8ull * W * (__popcll(__ballot(valid)) + __popcll(__ballot(valid && x0 >= 0))));
        wave_sync();  // every lane has read its entry before the list is rewritten
        if (pass) s_list[kept + __popcll(pm & ((1ull << lane) - 1ull))] = (uint16_t)j;
        kept += __popcll(pm);
        wave_sync();
      }
      if (nchild >= 3) {
        const u64 um = __ballot(uni0);
        const uint32_t run = um == ~0ull ? 64u : (uint32_t)__ffsll((long long)~um) - 1;
        absorb_n = run < nchild - 1 ? run : nchild - 1;  // keep a candidate
      }
      absorbed = absorb_n >= 2;
      if (absorbed) {
        // the screened list was rewritten: the run is the first absorb_n
        // candidates in position order again
        const u64 mw = (lane < (int)W) ? pw : 0ull;
        const uint32_t c2 = __popcll(mw);
        uint32_t o = wave_excl_scan(c2, lane);
        wave_sync();
        for (u64 t = mw; t && o < absorb_n; t &= t - 1)
          s_list[o++] = (uint16_t)(lane * 64 + __ffsll((long long)t) - 1);
        wave_sync();
      } else {
        n_eff = kept;
      }
    }
    if (absorbed) {
      // The record grows by the run (positions s_list[0 .. absorb_n)): it
      // keeps its bound, its members reach the run's last position, and X
      // keeps only what is adjacent to the whole run.  If some vertex of
      // that X is adjacent to all remaining candidates, no clique below is
      // maximal and the record is dropped; otherwise it is held as the
      // record's only child and goes on as a chained link (or is written
      // to the frontier) below.  It is one child (R10), the candidates it
      // replaces are not.
      const uint32_t jl = s_list[absorb_n - 1];
      const bool mine = (uint32_t)lane < absorb_n;
      const uint32_t jm = mine ? s_list[lane] : 0;
      long long add = mine ? (weighted ? (long long)wl[jm] : 1ll) : 0ll;
      add = (long long)wave_sum((u64)add);
      u64 xa = 0;  // lane w: word w of X and the run's rows
      for (uint32_t w = 0; w < W; ++w) {
        u64 v = mine ? rows[(u64)jm * W + w] : ~0ull;
        for (int o2 = 32; o2 > 0; o2 >>= 1) v &= __shfl_xor(v, o2, 64);
        if (lane == (int)w) xa = s_xw[w] & v;
      }
      stat(ST_ONCHIP, 8ull * W * absorb_n);
      const u64 pnew = (lane < (int)W) ? (pw & gt_mask(lane, (int)jl)) : 0ull;
      // exhaustive witness: each vertex of the new X, one per lane
      const uint32_t xcn = __popcll(xa);
      const uint32_t xo = wave_excl_scan(xcn, lane);
      const uint32_t nx = __shfl(xo + xcn, 63, 64);
      wave_sync();  // the list is no longer read
      {
        uint32_t o = xo;
        for (u64 t = xa; t; t &= t - 1) s_list[o++] = (uint16_t)(lane * 64 + __ffsll((long long)t) - 1);
      }
      wave_sync();
      if (lane < (int)W) s_cx[lane] = pnew;  // staging: P' for the broadcast reads below
      wave_sync();
      bool ext = false;
      for (uint32_t b0 = 0; b0 < nx && !ext; b0 += 64) {
        bool all = false;
        if (b0 + lane < nx) {
          const u64 *rx = rows + (u64)s_list[b0 + lane] * W;
          u64 out = 0;
          row_loop(rx, W, [&](uint32_t w, u64 rxw) { out |= s_cx[w] & ~rxw; });
          all = out == 0;
        }
        ext = __ballot(all) != 0;
      }
      stat(ST_ONCHIP, 8ull * W * nx);
      wave_sync();
      // children: the absorbed record replaces the nchild counted above
      if (lane == 0) {
        st[ST_CHILDREN] -= nchild - 1;
        st[ST_PRUNED_NEW] = st[ST_MARK];
      }
      absorb_keep = !ext;
      if (ext) {
        stat(ST_PRUNED_NEW, 1);
      } else {
        if (lane < (int)W) {
          s_cv[lane] = s_vw[lane] | s_pw[lane];  // members up to jl, candidates after
          s_cx[lane] = xa;
        }
        if (lane == 0) {
          s_cscore[wv] = p.score + add;
          s_cbound[wv] = p.bound;
          s_cj[wv] = (int)jl;
          s_ccnt[wv] = nchild - absorb_n;
        }
        wave_sync();
      }
      n_eff = 0;  // nothing is built one by one
    }
    // kept children: the first is held back (in s_cv/s_cx) in case it
    // stays the only one; `spilled` once it has been written out
    bool held = absorb_keep, spilled = false;
    // One child per lane, its W words in sequence: 64 children per round,
    // independent loads and no reductions between lanes.  A kept child's
    // words (V + P' and X') are recomputed from its row (a cache hit) as
    // they are stored rather than held in registers.
    const u64 lanes_below = (1ull << lane) - 1ull;
    for (uint32_t base = 0; base < n_eff; base += 64) {
      const uint32_t ci = base + (uint32_t)lane;
      const bool valid = ci < n_eff;
      const uint32_t j = valid ? s_list[ci] : 0;
      const uint32_t jw = j >> 6;
      const u64 jb = 1ull << (j & 63);
      const u64 *rj = rows + (u64)j * W;
      uint32_t cnt = 0;
      long long wsum = 0;
      int x0 = -1;  // extension witness: the first vertex of X'
      if (valid) {
        row_loop(rj, W, [&](uint32_t w, u64 row) {
          const u64 pv = s_pw[w];
          const u64 a = pv & row & gt_mask((int)w, (int)j);  // P'
          cnt += __popcll(a);
          if (weighted)
            for (u64 t = a; t; t &= t - 1) wsum += wl[w * 64 + __ffsll((long long)t) - 1];
          const u64 xc = (s_xw[w] | (pv & ~gt_mask((int)w, (int)j - 1))) & row;  // X'
          if (x0 < 0 && xc) x0 = (int)w * 64 + __ffsll((long long)xc) - 1;
        });
      }
      // the child is covered when the witness is adjacent to all of P':
      // then no clique below it is maximal
      bool covered = false;
      if (x0 >= 0) {
        const u64 *rx = rows + (u64)x0 * W;
        u64 out = 0;
        row_loop2(rj, rx, W, [&](uint32_t w, u64 rjw, u64 rxw) {
          out |= s_pw[w] & rjw & gt_mask((int)w, (int)j) & ~rxw;
        });
        covered = out == 0;
      }
      const long long score2 = p.score + (weighted ? (long long)wl[j] : 1ll);
      const long long bound2 = score2 + (weighted ? wsum : (long long)cnt);
      const bool prune = valid && (bound2 < theta || covered);
      const bool leaf = valid && !prune && cnt == 0;
      const bool keep = valid && !prune && cnt > 0;
      const bool offer = leaf && score2 >= theta;
      const u64 km = __ballot(keep);
      const u64 fm = __ballot(offer);
      stat(ST_PRUNED_NEW, __popcll(__ballot(prune)));
      stat(ST_LEAVES, __popcll(__ballot(leaf)));
      // adjacency rows read: the children's and the witnesses'
      stat(ST_ONCHIP, 8ull * W * (__popcll(__ballot(valid)) + __popcll(__ballot(x0 >= 0))));
      // this lane's child: V + P' to vo[0..W), X' to xo[0..W)
      auto put_child = [&](u64 *vo, u64 *xo) {
        row_loop(rj, W, [&](uint32_t w, u64 row) {
          const u64 pv = s_pw[w];
          vo[w] = s_vw[w] | (pv & row & gt_mask((int)w, (int)j)) | (w == jw ? jb : 0ull);
          xo[w] = (s_xw[w] | (pv & ~gt_mask((int)w, (int)j - 1))) & row;
        });
      };
      if (km) {
        if (!held && __popcll(km) == 1) {
          // the first kept child: hold it back
          held = true;
          if (keep) {
            put_child(s_cv, s_cx);
            s_cscore[wv] = score2;
            s_cbound[wv] = bound2;
            s_cj[wv] = (int)j;
            s_ccnt[wv] = cnt;
          }
          wave_sync();
        } else {
          // write these children, and the held one if it is still held
          const uint32_t extra = (held && !spilled) ? 1u : 0u;
          const uint32_t nk = __popcll(km) + extra;
          unsigned int h0 = 0;
          u64 w0 = 0;
          if (lane == 0) {
            h0 = atomicAdd(&qs[q].n_out, nk);
            w0 = atomicAdd(&qs[q].out_words, (u64)nk * 2 * W);
          }
          h0 = __shfl(h0, 0, 64);
          w0 = __shfl(w0, 0, 64);
          const bool fits0 = (u64)cf.out_hdr + h0 + nk <= cf.hdr_cap &&
                             cf.out_word + w0 + (u64)nk * 2 * W <= cf.word_cap;
          if (!fits0) {
            if (lane == 0) atomicAdd(&qs[q].overflow, 1u);
          } else {
            if (extra) {
              write_held((u64)cf.out_hdr + h0, cf.out_word + w0);
              spilled = true;
            }
            if (keep) {
              const uint32_t rk = extra + __popcll(km & lanes_below);
              const u64 slot_w = cf.out_word + w0 + (u64)rk * 2 * W;
              put_child(cf.words + slot_w, cf.words + slot_w + W);
              put_crec(cf.hdr, (u64)cf.out_hdr + h0 + rk, score2, bound2, slot_w, cnt, r, (int)j, q);
              const u64 cc = (u64)(d - j - 1);
              atomicAdd(&s_cost[wv], cc);
              atomicMax(&s_maxcc[wv], cc);
              atomicMax(&s_maxb[wv], bound2);
            }
            stat(ST_BYTES, (32 + 16ull * W) * __popcll(km));
          }
          held = true;
          spilled = true;
        }
      }
      if (fm) {
        const uint32_t nf = __popcll(fm);
        stat(ST_BYTES, (24 + 8ull * W) * nf);
        unsigned int l0 = 0;
        u64 w0 = 0;
        if (lane == 0) {
          l0 = atomicAdd(&hdr->leaf_count, nf);
          w0 = atomicAdd(&hdr->leaf_word_count, (u64)nf * W);
        }
        l0 = __shfl(l0, 0, 64);
        w0 = __shfl(w0, 0, 64);
        if (offer) {
          const uint32_t rk = __popcll(fm & lanes_below);
          const u64 slot_l = (u64)l0 + rk;
          const u64 slot_w = w0 + (u64)rk * W;
          if (slot_l < leaf_cap && slot_w + W <= leaf_word_cap) {
            for (uint32_t w = 0; w < W; ++w) leaf_words[slot_w + w] = s_vw[w] | (w == jw ? jb : 0ull);
            LRec l;
            l.score = score2;
            l.woff = slot_w;
            l.root = r;
            l.last = (int16_t)j;
            l.qid = (uint16_t)q;
            leaves[slot_l] = l;
          } else {
            atomicAdd(&qs[q].overflow, 1u);
          }
        }
      }
    }
    if (!held || spilled) break;
    // exactly one kept child.  Expand it next, in this wave, if a k-th
    // score is known (without one nothing is cut, and thousands of chains
    // would each run to full depth unpruned), the chain is shorter than
    // max_links and the leaf buffer has room for every leaf it can offer
    // (at most one per candidate); otherwise write it to the frontier like
    // any other child.
    {
      // leaf slots are reserved in chunks of several links' worth; unused
      // credit is handed back when the chain ends
      const u64 m = s_ccnt[wv];
      int ok = 0;
      if (lane == 0 && theta != LLONG_MIN && links < max_links) {
        if (credit < m) {
          for (u64 want = 8 * m; want >= m && !ok; want = want == m ? 0 : m) {
            const u64 oc = atomicAdd(&hdr->chain_c, want);
            if (oc + want <= chain_cap) {
              credit += want;
              ok = 1;
            } else {
              atomicSub(&hdr->chain_c, want);
            }
          }
        } else {
          ok = 1;
        }
        if (ok) credit -= m;
      }
      ok = __shfl(ok, 0, 64);
      if (!ok) {
        unsigned int h0 = 0;
        u64 w0 = 0;
        if (lane == 0) {
          h0 = atomicAdd(&qs[q].n_out, 1u);
          w0 = atomicAdd(&qs[q].out_words, 2ull * W);
        }
        h0 = __shfl(h0, 0, 64);
        w0 = __shfl(w0, 0, 64);
        if ((u64)cf.out_hdr + h0 + 1 <= cf.hdr_cap && cf.out_word + w0 + 2ull * W <= cf.word_cap)
          write_held((u64)cf.out_hdr + h0, cf.out_word + w0);
        else if (lane == 0)
          atomicAdd(&qs[q].overflow, 1u);
        break;
      }
    }
    p.score = s_cscore[wv];
    p.bound = s_cbound[wv];
    p.last = (int16_t)s_cj[wv];
    carried = true;
    ++links;
  }
  if (lane == 0 && credit) atomicSub(&hdr->chain_c, credit);
  // flush per-wave statistics with one atomic each
  wave_sync();
  if (lane == 0) {
    const uint32_t slot = (blockIdx.x * kExpandWaves + wv) & (kCtrSlots - 1);
    QCtr &C = ctr[q * kCtrSlots + slot];
    atomicAdd(&C.popped, st[ST_POPPED]);
    if (st[ST_PRUNED_POP]) atomicAdd(&C.pruned_pop, st[ST_PRUNED_POP]);
    if (st[ST_EXPANDED]) atomicAdd(&C.expanded, st[ST_EXPANDED]);
    if (st[ST_CHILDREN]) atomicAdd(&C.children, st[ST_CHILDREN]);
    if (st[ST_PRUNED_NEW]) atomicAdd(&C.pruned_new, st[ST_PRUNED_NEW]);
    if (st[ST_LEAVES]) atomicAdd(&C.leaves, st[ST_LEAVES]);
    if (st[ST_BYTES]) atomicAdd(&C.logical_bytes, st[ST_BYTES]);
    if (st[ST_ONCHIP]) atomicAdd(&C.onchip_bytes, st[ST_ONCHIP]);
    QFlush &F = flush[q * kCtrSlots + slot];
    const u64 cost = s_cost[wv];
    if (cost) {
      atomicAdd(&F.cost_children, cost);
      atomicAdd(&F.cost_words, cost * 2 * W);
      atomicMax(&F.max_cc, s_maxcc[wv]);
      atomicMax(&F.max_w, W);
    }
    if (s_maxb[wv] != LLONG_MIN) atomicMax(&F.max_bound, s_maxb[wv]);
  }
}

// the QFlush copies of query blockIdx.x into its QStep, then back to
// their neutral values.  grid: (queries), one wavefront
static_assert(kCtrSlots == 64, "one QFlush copy per lane");
__global__ void __launch_bounds__(64) k_qflush(QFlush *flush, QStep *qs) {
  const int lane = threadIdx.x;
  QFlush &e = flush[(u64)blockIdx.x * kCtrSlots + lane];
  const u64 cc = wave_sum(e.cost_children), cw = wave_sum(e.cost_words);
  const u64 mc = wave_max_u64(e.max_cc), mw = wave_max_u64(e.max_w);
  const long long mb = wave_max(e.max_bound);
  e.cost_children = 0;
  e.cost_words = 0;
  e.max_cc = 0;
  e.max_bound = LLONG_MIN;
  e.max_w = 0;
  if (lane == 0) {
    QStep &S = qs[blockIdx.x];
    S.out_cost_children = cc;
    S.out_cost_words = cw;
    S.out_max_cc = mc;
    S.out_max_bound = mb;
    S.out_max_w = (unsigned int)mw;
  }
}

// ------------------------------------------------------------------
// maximality check of leaves (relevant(s) of Table 1 for cliques)
// ------------------------------------------------------------------
// A leaf C = {r} + members has no common later neighbour.  It is maximal
// iff no other vertex is adjacent to all of C:
//  (a) no local position outside C adjacent to every member (AND of the
//      members' local rows), and
//  (b) no vertex u ranked below r adjacent to all of C: u is scanned in
//      the lower neighbour list N-(c*) of the member with the shortest one
//      and tested against every other member by binary search in N+(u).
// A vertex of C that u is not adjacent to rules u out; the first one a
// test finds is kept in a per-graph table (wit[u]), and later checks try
// it first: leaves of one dense region share most members, so most u are
// ruled out by one lookup instead of a search.  Any entry is a fact about
// the graph, so concurrent writers cannot make it wrong.
constexpr int kLeafCap = kMaxLocal + 1;
// wavefronts per leaf: (a) is done by wave 0, the candidates of (b) are
// shared out between all of them, and all of them sort the output
constexpr int kLeafWaves = 8;
constexpr uint32_t kNoWit = 0xFFFFFFFFu;

__global__ void __launch_bounds__(64 * kLeafWaves)
    k_leaf_check(GView g, const LRec *leaves, uint32_t first, const u64 *leaf_words,
                 const QRes *res, Cand *cands, unsigned int *cand_count, uint32_t *cand_ids,
                 uint32_t lmax, QCtr *ctr) {
  __shared__ uint32_t s_rank[kLeafCap];
  __shared__ uint32_t s_id[kLeafCap];
  __shared__ uint32_t s_sorted[kLeafCap];
  __shared__ int s_ext;  // an extender was found: the leaf is not maximal
  __shared__ uint32_t s_nc, s_nu, s_cs;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const LRec L = leaves[first + blockIdx.x];
  const uint32_t q = L.qid;
  if (L.score < res[q].theta) return;
  const uint32_t r = L.root;
  const uint32_t d = g.dplus[r];
  const uint32_t W = words_of(d);
  if (wv == 0) {
    u64 v = 0;
    if (d && lane < (int)W) v = leaf_words[L.woff + lane];
    // member positions -> ranks
    const uint32_t c = __popcll(v);
    const uint32_t off = wave_excl_scan(c, lane);
    const uint32_t nm = __shfl(off + c, 63, 64);
    const uint32_t *np = g.oplus + g.ooff[r];
    {
      u64 t = v;
      uint32_t o = off;
      while (t) {
        int b = __ffsll((long long)t) - 1;
        s_rank[o] = np[lane * 64 + b];
        s_sorted[o++] = lane * 64 + b;  // local positions, for (a)
        t &= t - 1;
      }
    }
    if (lane == 0) s_rank[nm] = r;
    wave_sync();
    const uint32_t nc = nm + 1;  // clique size
    int ext = 0;
    // (a) local extension: the AND of the members' rows.  Rows of up to 16
    // words: one member per lane, a whole row's loads in flight together,
    // then one reduction per word; wider rows: groups of G lanes, one word
    // per lane, 64/G members per round.
    if (d) {
      const u64 *rows = g.bm + g.bm_off[r];
      u64 accw = ~0ull;  // lane w < W: word w of the AND
      if (W <= 16) {
        u64 acc[16];
#pragma unroll
        for (int w = 0; w < 16; ++w) acc[w] = ~0ull;
        for (uint32_t b0 = 0; b0 < nm; b0 += 64) {
          if (b0 + lane < nm)
            row_words(rows + (u64)s_sorted[b0 + lane] * W, W,
                      [&](uint32_t w, u64 rw) { acc[w] &= rw; });
        }
#pragma unroll
        for (int w = 0; w < 16; ++w) {
          if ((uint32_t)w < W) {
            u64 a = acc[w];
            for (int o2 = 32; o2 > 0; o2 >>= 1) a &= __shfl_xor(a, o2, 64);
            if (lane == w) accw = a;
          }
        }
      } else {
        uint32_t G = 1;
        while (G < W) G <<= 1;
        const uint32_t per = 64 / G;
        const int wi = lane & (G - 1);
#pragma unroll 8
        for (uint32_t b0 = 0; b0 < nm; b0 += per) {
          const uint32_t ci = b0 + lane / G;
          if (ci < nm && wi < (int)W) accw &= rows[(u64)s_sorted[ci] * W + wi];
        }
        for (uint32_t o2 = G; o2 < 64; o2 <<= 1) accw &= __shfl_xor(accw, o2, 64);
      }
      const u64 x = (lane < (int)W) ? (~v & lt_mask(lane, d) & accw) : 0ull;
      ext = __ballot(x != 0) != 0;
    }
    // (b) set-up: an extender u ranked below r has |N+(u)| >= nc; for
    // nc >= kHeavy only the heavy part of the lower neighbour lists can
    // hold one.  Scan the list of the member with the fewest entries.
    const bool heavy = nc >= kHeavy;
    uint32_t bestc = 0xFFFFFFFFu, besti = 0;
    for (uint32_t t = lane; t < nc; t += 64) {
      const uint32_t m = s_rank[t];
      const uint32_t sz = heavy ? (uint32_t)(g.hrow[m + 1] - g.hrow[m]) : g.split[m];
      if (sz < bestc) { bestc = sz; besti = t; }
    }
    for (int o2 = 32; o2 > 0; o2 >>= 1) {
      uint32_t oc = __shfl_xor(bestc, o2, 64), oi = __shfl_xor(besti, o2, 64);
      if (oc < bestc || (oc == bestc && oi < besti)) { bestc = oc; besti = oi; }
    }
    const uint32_t cs = s_rank[besti];
    const uint32_t *lo_list = heavy ? g.hcol + g.hrow[cs] : g.rcol + g.rrow[cs];
    // entries below r form a prefix (lists are sorted by rank)
    uint32_t lo = 0, hi = bestc;
    while (lo < hi) {
      uint32_t mid = (lo + hi) >> 1;
      if (lo_list[mid] < r) lo = mid + 1; else hi = mid;
    }
    if (lane == 0) {
      s_ext = ext;
      s_nc = nc;
      s_nu = lo;
      s_cs = cs;
    }
  }
  __syncthreads();
  if (s_ext) return;
  const uint32_t nc = s_nc, nu = s_nu;
  {
    const uint32_t cs = s_cs;
    const bool heavy = nc >= kHeavy;
    const uint32_t *lo_list = heavy ? g.hcol + g.hrow[cs] : g.rcol + g.rrow[cs];
    // (b): |N+(u)| >= nc rejects almost every u with one load.  Each
    // remaining u is tested by a whole wave, 64 members at a time; the
    // waves take turns over the list and stop once one finds an extender.
    const uint32_t nmem = nc - 1;  // s_rank[0 .. nmem): members above r, ascending
    for (uint32_t b0 = wv * 64; b0 < nu; b0 += 64 * kLeafWaves) {
      if (*(volatile int *)&s_ext) break;
      const uint32_t t = b0 + lane;
      const uint32_t u = t < nu ? lo_list[t] : 0u;
      bool live = t < nu && g.dplus[u] >= nc;
      const uint32_t xw = live ? g.wit[u] : kNoWit;
      if (xw != kNoWit) {
        // is the stored non-neighbour of u in C?
        bool inc = xw == r;
        if (!inc) {
          uint32_t a = 0, z = nmem;
          while (a < z) {
            const uint32_t mid = (a + z) >> 1;
            if (s_rank[mid] < xw) a = mid + 1; else z = mid;
          }
          inc = a < nmem && s_rank[a] == xw;
        }
        live = !inc;
      }
      u64 cand = __ballot(live);
      bool found = false;
      while (cand && !found) {
        const int src = __ffsll((long long)cand) - 1;
        cand &= cand - 1;
        const uint32_t uu = __shfl(u, src, 64);
        const uint32_t *up = g.oplus + g.ooff[uu];
        const uint32_t du = g.dplus[uu];
        bool all = true;
        for (uint32_t m0 = 0; m0 < nc && all; m0 += 64) {
          const uint32_t m = m0 + lane;
          bool miss = false;
          if (m < nc) {
            const uint32_t x = s_rank[m];
            uint32_t a = 0, z = du;
            while (a < z) {
              const uint32_t mid = (a + z) >> 1;
              if (up[mid] < x) a = mid + 1; else z = mid;
            }
            miss = !(a < du && up[a] == x);
          }
          const u64 mm = __ballot(miss);
          all = mm == 0;
          if (!all && lane == __ffsll((long long)mm) - 1) g.wit[uu] = s_rank[m];
        }
        found = all;
      }
      if (found) {
        if (lane == 0) s_ext = 1;
        break;
      }
    }
  }
  __syncthreads();
  if (s_ext) return;
  // maximal: emit (score, ascending original ids), ranked by counting
  // (ids are distinct) over all the block's threads
  for (uint32_t t = threadIdx.x; t < nc; t += 64 * kLeafWaves) s_id[t] = g.orig[s_rank[t]];
  __syncthreads();
  for (uint32_t t = threadIdx.x; t < nc; t += 64 * kLeafWaves) {
    const uint32_t x = s_id[t];
    uint32_t rk = 0;
    for (uint32_t u = 0; u < nc; ++u) rk += s_id[u] < x;
    s_sorted[rk] = x;
  }
  __syncthreads();
  if (wv != 0) return;
  unsigned int slot = 0;
  if (lane == 0) {
    slot = atomicAdd(cand_count, 1u);
    Cand cd;
    cd.score = L.score;
    cd.qid = q;
    cd.len = nc;
    cands[slot] = cd;
    atomicAdd(&ctr[q * kCtrSlots + (blockIdx.x & (kCtrSlots - 1))].offered, 1ull);
  }
  slot = __shfl(slot, 0, 64);
  for (uint32_t t = lane; t < nc; t += 64) cand_ids[(u64)slot * lmax + t] = s_sorted[t];
}

// ------------------------------------------------------------------
// host side
// ------------------------------------------------------------------
struct Level {
  uint32_t begin = 0, count = 0;
  u64 wbegin = 0, wend = 0;
  u64 cost_children = 0, cost_words = 0;
  long long max_bound = LLONG_MIN;
  u64 maxcc = 0;
  uint32_t maxw = 0;
};

// Frontier levels moved to host memory (the paper's virtual priority queue,
// Section 5): the bottom of a query's level stack -- its shallowest, lowest
// priority records -- with the arena range they occupied, which always
// starts at offset 0, so a chunk returns to the same offsets.  Held in
// ordinary (pageable) host memory: page-locking every chunk costs more than
// the copies it would speed up.
struct SpillChunk {
  std::vector<Level> levels;
  u64 n_hdr = 0, n_words = 0;  // header slots and words from offset 0
  std::vector<CRec> hdr;
  std::vector<u64> words;
};

struct QHost {
  bool active = false;  // the slot holds a query
  bool done = true;     // the query needs no more steps
  int error = 0;        // nuri_status of a failed query
  std::string errmsg;
  uint32_t k = 1;
  int kind = 0;  // 0 size, 1 vertex weight
  std::vector<Level> stack;
  uint64_t cursor = 0;
  long long theta = LLONG_MIN;
  bool seeded = false;  // seed cliques offered
  uint32_t hdr_cap = 0;
  u64 word_cap = 0;
  uint64_t t_admit = 0, steps = 0, expand_ns = 0, launches = 0, peak_bytes = 0;
  std::vector<std::shared_ptr<SpillChunk>> spill;  // spilled chunks, the last spilled last
  uint64_t spilled_bytes = 0;
  // this step
  int plan = 0;  // 0 idle, 1 roots, 2 level
  uint32_t new_begin = 0;
  u64 new_wbegin = 0;
  uint32_t seg0 = 0, nsegs = 0;  // this step's segments: seg0 .. seg0 + nsegs - 1
};

// per-slot top-k buffers (two of each, switched by every merge) and the
// slot's frontier arena (record headers and bitmap words), all taken when a
// query is admitted and returned when it is harvested
struct SlotTopk {
  PoolBuf<long long> score;
  PoolBuf<unsigned int> len, ids;
  PoolBuf<CRec> hdr;
  PoolBuf<u64> words;
};

// Layout of the per-step block that one host-to-device copy uploads and
// one device-to-host copy (of its first part) reads back.
struct StepLayout {
  // StepHdr | QStep[nq] | tempc[ns] (read back) | cfg[nq] | rseg[nq] |
  // taken[ns] | thr[ns] | quota[ns] | seg[ns] (uploaded up to the last used)
  size_t qs, tempc, cfg, rseg, taken, thr, quota, seg, total;
  uint32_t nseg_cap;
  StepLayout(uint32_t nq, uint32_t ns) : nseg_cap(ns) {
    size_t o = sizeof(StepHdr);
    qs = o;
    o += nq * sizeof(QStep);
    tempc = o;
    o += ns * 4;
    o = (o + 15) & ~size_t(15);
    cfg = o;
    o += nq * sizeof(QCfg);
    rseg = o;
    o += nq * sizeof(RootSeg);
    taken = o;
    o += ns * 4;
    thr = o;
    o += ns * 4;
    quota = o;
    o += ns * 4;
    o = (o + 15) & ~size_t(15);
    seg = o;
    o += ns * sizeof(SelSeg);
    total = (o + 255) & ~size_t(255);
  }
  size_t readback() const { return cfg; }  // StepHdr + QStep[nq] + tempc[ns]
  size_t upload(uint32_t nseg) const { return seg + nseg * sizeof(SelSeg); }
};

struct Engine {
  Graph &g;
  QueryOpts o;
  hipStream_t s;
  bool server_mode = false;  // per-query failures mark the query instead of throwing
  uint32_t nq = 0;           // slots
  uint32_t lmax = 0;
  std::vector<QHost> qh;
  std::vector<QCfg> cfg;
  std::vector<std::unique_ptr<SlotTopk>> tk;

  u64 arena_bytes = 0;  // frontier arena of a slot unless admit() is given one
  PoolBuf<QCtr> d_ctr;
  PoolBuf<QFlush> d_flush;
  PoolBuf<QRes> d_res;
  PoolBuf<uint32_t> d_k;
  PoolBuf<CRec> batch, temp;
  PoolBuf<LRec> leaves;
  PoolBuf<u64> leaf_words;
  PoolBuf<Cand> cands;
  MergeBufs mbuf;  // top-k merge: candidate positions and survivor lists
  PinBuf<SeedSeg> h_seed;
  PoolBuf<SeedSeg> d_seed;
  PoolBuf<uint32_t> cand_ids;
  // selection segments: up to kSegPerQuery levels of one query per step
  static constexpr uint32_t kSegPerQuery = 8;
  uint32_t seg_cap = 0;
  std::vector<uint32_t> seg_level;  // level index (in its query's stack) of each segment
  PoolBuf<unsigned int> d_hist;
  PoolBuf<u64> d_hchild;
  PoolBuf<unsigned char> d_step;
  PinBuf<unsigned char> h_step;
  PinBuf<QRes> h_res;
  PinBuf<QCtr> h_ctr;
  PinBuf<uint32_t> h_k;
  uint32_t batch_cap = 0, leaf_cap = 0;
  u64 leaf_word_cap = 0;
  uint32_t B = 0, root_B = 0;
  u64 step_children = 0, step_words = 0;
  u64 plan_c = 0, plan_w = 0;  // children and words the current step may write
  uint32_t ex_wst = 0, ex_lst = 0;
  size_t expand_lds = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::unique_ptr<StepLayout> L;
  // NURI_TRACE=n: one line on stderr every n steps (1: every step)
  uint64_t trace = 0, trace_steps = 0;
  bool theta_pending = false;  // h_res holds k-th scores not yet taken
  uint32_t rr = 0;     // round-robin start of the per-step planning
  std::vector<int> level_order;  // scratch of plan()

  // device memory of every buffer: the graph's pool, or a fixed region
  // (the allocation-free entry point), from which nothing is allocated
  MemPool *mp;
  uint64_t fixed_topk_bytes = 0;  // fixed region: bytes kept for the top-k buffers

  Engine(Graph &g_, const QueryOpts &o_, MemPool *pool = nullptr)
      : g(g_), o(o_), s(o_.stream ? o_.stream : g_.stream), mp(pool ? pool : &g_.pool) {
    const char *t = getenv("NURI_TRACE");
    trace = t ? strtoull(t, nullptr, 10) : 0;
    const bool pinned = mp->fixed_base == nullptr;
    h_seed.pinned = h_step.pinned = h_res.pinned = h_ctr.pinned = h_k.pinned = pinned;
  }
  ~Engine() {
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
  }

  GView view() const {
    GView v;
    v.dplus = g.dplus.p;
    v.split = g.split.p;
    v.oplus = g.oplus.p;
    v.orig = g.orig.p;
    v.rcol = g.rcol.p;
    v.ooff = g.ooff.p;
    v.bm_off = g.bm_off.p;
    v.rrow = g.rrow.p;
    v.hrow = g.hrow.p;
    v.hcol = g.hcol.p;
    v.bm = (const u64 *)g.bm.p;
    v.wloc = g.wloc.p;
    v.vw = g.vw.p;
    v.wplus = g.wplus.p;
    v.root_order[0] = g.root_order[0].p;
    v.root_order[1] = g.root_order[1].p;
    v.wit = g.leaf_wit.p;
    return v;
  }

  StepHdr *sh() { return (StepHdr *)h_step.p; }
  QStep *sq() { return (QStep *)(h_step.p + L->qs); }
  SelSeg *sseg() { return (SelSeg *)(h_step.p + L->seg); }
  RootSeg *srseg() { return (RootSeg *)(h_step.p + L->rseg); }
  template <class T>
  T *dev(size_t off) {
    return (T *)(d_step.p + off);
  }

  // A query failed: in a batch the whole call fails; in the server only
  // that query does.
  void fail(uint32_t i, int code, const std::string &msg) {
    if (!server_mode) throw Error{code, msg};
    qh[i].error = code;
    qh[i].errmsg = msg;
    qh[i].done = true;
  }

  // allocate `slots` query slots sharing the frontier budget equally
  void setup(uint32_t slots) {
    nq = slots;
    lmax = g.degeneracy + 1;
    qh.assign(nq, QHost{});
    cfg.assign(nq, QCfg{});
    tk.clear();
    for (uint32_t i = 0; i < nq; ++i) tk.emplace_back(new SlotTopk);
    seg_cap = std::min<uint32_t>(nq * kSegPerQuery, std::max<uint32_t>(nq, 1024));
    L.reset(new StepLayout(nq, seg_cap));
    seg_level.assign(seg_cap, 0);
    const bool fixed = mp->fixed_base != nullptr;
    B = o.batch_B ? o.batch_B : 16384;
    root_B = o.root_batch ? o.root_batch : 8192;
    // LDS of k_expand: five bitmaps of the widest local row, a candidate
    // list and the local weights as long as the largest out-degree, per wave
    ex_wst = std::max<uint32_t>(1, (g.degeneracy + 63) / 64);
    ex_lst = (g.degeneracy + 8) & ~7u;
    u64 budget = o.frontier_budget;
    if (fixed) {
      // a fixed region: small steps, and the frontier gets what is left
      // after every other buffer (temp, which holds a level being
      // selected from, is sized with the headers)
      B = std::min<uint32_t>(B, 4096);
      root_B = std::min<uint32_t>(root_B, 4096);
      step_words = 1ull << 17;
      step_children = 1ull << 16;
      batch_cap = nq * std::max(B, root_B);
      leaf_cap = (uint32_t)(2 * step_children + batch_cap);
      leaf_word_cap = 2 * step_words;
      const u64 other = MemPool::align_up(batch_cap * sizeof(CRec)) +
                        MemPool::align_up((u64)leaf_cap * sizeof(LRec)) +
                        MemPool::align_up(leaf_word_cap * 8) +
                        MemPool::align_up(kCandChunk * sizeof(Cand)) +
                        MemPool::align_up((u64)kCandChunk * lmax * 4) +
                        MemPool::align_up((u64)seg_cap * kBins * 4) +
                        MemPool::align_up((u64)seg_cap * kBins * 8) +
                        MemPool::align_up(L->total) + 16 * 4096 + fixed_topk_bytes +
                        (u64)nq * (kCandChunk * 4 + 1024);
      const u64 have = mp->fixed_size - MemPool::align_up(mp->fixed_used);
      if (have < other + (4ull << 20))
        throw Error{NURI_EINVAL, "query too large for the fixed scratch region: needs more than " +
                                     std::to_string(other + (4ull << 20)) + " of " +
                                     std::to_string(have) + " bytes"};
      budget = have - other;
    }
    arena_bytes = budget / nq;
    h_res.alloc(nq);
    h_ctr.alloc((u64)nq * kCtrSlots);
    h_k.alloc(nq);
    for (uint32_t i = 0; i < nq; ++i) {
      QRes &R = h_res.p[i];
      memset(&R, 0, sizeof(R));
      R.theta = LLONG_MIN;
      h_k.p[i] = 1;
    }
    d_ctr.alloc(*mp, (u64)nq * kCtrSlots);
    d_res.alloc(*mp, nq);
    d_k.alloc(*mp, nq);
    NURI_HIP(hipMemcpyAsync(d_res.p, h_res.p, nq * sizeof(QRes), hipMemcpyHostToDevice, s));
    NURI_HIP(hipMemcpyAsync(d_k.p, h_k.p, nq * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    NURI_HIP(hipMemsetAsync(d_ctr.p, 0, (u64)nq * kCtrSlots * sizeof(QCtr), s));
    if (!fixed) {
      step_words = std::max<u64>(1ull << 20, std::min<u64>(budget / 16 / 8, 64ull << 20));
      step_children = std::max<u64>(1ull << 16, std::min<u64>(step_words, 32ull << 20));
      // records per step; k_expand runs 64 threads per record and a launch
      // must stay below 2^31 threads
      batch_cap = (uint32_t)std::min<u64>((u64)nq * std::max(B, root_B), 1u << 24);
      // leaves of one step: at most one per planned child plus one per unit
      // subgraph, and the reserve that chained expansion draws from
      leaf_cap = (uint32_t)(2 * step_children + batch_cap);
      leaf_word_cap = 2 * step_words;
    }
    batch.alloc(*mp, batch_cap);
    if (fixed) temp.alloc(*mp, arena_caps(arena_bytes).first);  // every level fits
    // per wavefront: five bitmaps, the candidate list and the root's weights
    expand_lds = (size_t)kExpandWaves * (5ull * 8 * ex_wst + 2ull * ex_lst + 4ull * ex_lst);
    leaves.alloc(*mp, leaf_cap);
    leaf_words.alloc(*mp, leaf_word_cap);
    cands.alloc(*mp, kCandChunk);
    mbuf.alloc(*mp, nq, s);
    h_seed.alloc(nq);
    d_seed.alloc(*mp, nq);
    cand_ids.alloc(*mp, (u64)kCandChunk * lmax);
    d_hist.alloc(*mp, (u64)seg_cap * kBins);
    d_hchild.alloc(*mp, (u64)seg_cap * kBins);
    NURI_HIP(hipMemsetAsync(d_hist.p, 0, d_hist.bytes(), s));
    NURI_HIP(hipMemsetAsync(d_hchild.p, 0, d_hchild.bytes(), s));
    d_step.alloc(*mp, L->total);
    h_step.alloc(L->total);
    // k_qflush leaves the copies neutral; a first pass over the zeroed
    // buffer sets them so (what it writes to the QSteps is overwritten by
    // every step's upload)
    d_flush.alloc(*mp, (u64)nq * kCtrSlots);
    NURI_HIP(hipMemsetAsync(d_flush.p, 0, (u64)nq * kCtrSlots * sizeof(QFlush), s));
    hipLaunchKernelGGL(k_qflush, dim3(nq), dim3(64), 0, s, d_flush.p, dev<QStep>(L->qs));
    NURI_HIP(hipGetLastError());
    if (o.profile) {
      NURI_HIP(hipEventCreate(&ev0));
      NURI_HIP(hipEventCreate(&ev1));
    }
  }

  // (headers, words) of an arena of `bytes`: a third headers, the rest
  // words; in a fixed region a quarter headers, a quarter their selection
  // copy (temp) and half words
  std::pair<u64, u64> arena_caps(u64 bytes) const {
    const bool fixed = mp->fixed_base != nullptr;
    u64 h = std::max<u64>(1024, bytes / (fixed ? 4 : 3) / sizeof(CRec));
    h = std::min<u64>(h, 0x7FFFFFFFull);
    const u64 hb = h * sizeof(CRec) * (fixed ? 2 : 1);
    const u64 w = std::max<u64>(4096, bytes > hb ? (bytes - hb) / 8 : 0);
    return {h, w};
  }
  // bytes of the smallest arena that holds the children of any one record
  u64 min_arena_bytes() const {
    const u64 W = (g.degeneracy + 63) / 64;
    return std::max<u64>(64ull << 10, 4ull * g.degeneracy * (sizeof(CRec) + 16 * W));
  }

  // start query (k, score kind) in a free slot with a frontier arena of
  // `bytes` (0: the slot default)
  void admit(uint32_t i, uint32_t k, int kind, u64 bytes = 0) {
    // the copy of every query's k-th score still in flight would land on
    // top of this slot's new entry: let it land and take it while the slot
    // still holds the old query (which no longer counts), before resetting it
    if (theta_pending) {
      NURI_HIP(hipStreamSynchronize(s));
      take_theta();
    }
    // the maximality checks' table of non-neighbours starts empty whenever
    // the engine takes work with no query in flight, so that a query run
    // on its own does not gain from the ones before it
    bool busy = false;
    for (const auto &O : qh) busy |= O.active;
    if (!busy) NURI_HIP(hipMemsetAsync(g.leaf_wit.p, 0xFF, g.leaf_wit.bytes(), s));
    QHost &Q = qh[i];
    Q = QHost{};
    Q.active = true;
    Q.done = false;
    Q.k = k;
    Q.kind = kind;
    const auto caps = arena_caps(bytes ? bytes : arena_bytes);
    SlotTopk &A = *tk[i];
    A.hdr.alloc(*mp, caps.first);
    A.words.alloc(*mp, caps.second);
    Q.hdr_cap = (uint32_t)caps.first;
    Q.word_cap = caps.second;
    Q.t_admit = now_ns();
    QCfg &c = cfg[i];
    c.hdr = A.hdr.p;
    c.words = A.words.p;
    c.hdr_cap = (uint32_t)caps.first;
    c.word_cap = caps.second;
    c.weighted = kind;
    c.k = k;
    // automatic: colour classes unless the densest region is a near-clique
    const bool colour = o.bound == 2 || (o.bound == 0 && g.core_density < 0.9);
    c.colour_min = colour ? 1u : 0u;
    c.prio = o.priority;
    SlotTopk &T = *tk[i];
    T.score.alloc(*mp, 2ull * k);
    T.len.alloc(*mp, 2ull * k);
    T.ids.alloc(*mp, 2ull * k * lmax);
    QRes &R = h_res.p[i];
    R.theta = LLONG_MIN;
    R.tk_n = 0;
    R.cur = 0;
    for (int b = 0; b < 2; ++b) {
      R.tk_score[b] = T.score.p + (u64)b * k;
      R.tk_len[b] = T.len.p + (u64)b * k;
      R.tk_ids[b] = T.ids.p + (u64)b * k * lmax;
    }
    h_k.p[i] = k;
    NURI_HIP(hipMemcpyAsync(&d_res.p[i], &h_res.p[i], sizeof(QRes), hipMemcpyHostToDevice, s));
    NURI_HIP(hipMemcpyAsync(&d_k.p[i], &h_k.p[i], sizeof(uint32_t), hipMemcpyHostToDevice, s));
    NURI_HIP(hipMemsetAsync(&d_ctr.p[(u64)i * kCtrSlots], 0, kCtrSlots * sizeof(QCtr), s));
  }

  bool slot_free(uint32_t i) const { return !qh[i].active; }
  bool finished(uint32_t i) const { return qh[i].active && qh[i].done; }
  bool any_live() const {
    for (auto &Q : qh)
      if (Q.active && !Q.done) return true;
    return false;
  }

  // one record of output at most: d children of 2W words
  u64 max_rec_children() const { return g.degeneracy; }
  u64 max_rec_words() const { return (u64)g.degeneracy * 2 * ((g.degeneracy + 63) / 64); }

  // The frontier spill (not in a fixed region, where nothing may be
  // allocated): when a query's arena is nearly full, its bottom levels --
  // at least half of the used headers and words, never the top level --
  // are copied to host memory and the levels above are moved
  // down (their word offsets rebased).  Returns false when there is
  // nothing to spill.
  bool spill_bottom(uint32_t i) {
    QHost &Q = qh[i];
    if (mp->fixed_base || Q.stack.size() < 2) return false;
    const Level &T = Q.stack.back();
    const u64 used_h = (u64)T.begin + T.count, used_w = T.wend;
    size_t m = 1;  // levels [0, m) go to the host
    while (m + 1 < Q.stack.size() &&
           ((u64)Q.stack[m].begin * 2 < used_h || Q.stack[m].wbegin * 2 < used_w))
      ++m;
    const u64 hshift = Q.stack[m].begin, wshift = Q.stack[m].wbegin;
    if (hshift == 0 && wshift == 0) return false;
    auto C = std::make_shared<SpillChunk>();
    C->levels.assign(Q.stack.begin(), Q.stack.begin() + m);
    C->n_hdr = hshift;
    C->n_words = wshift;
    C->hdr.resize(std::max<u64>(1, hshift));
    C->words.resize(std::max<u64>(1, wshift));
    QCfg &c = cfg[i];
    NURI_HIP(hipMemcpyAsync(C->hdr.data(), c.hdr, hshift * sizeof(CRec), hipMemcpyDeviceToHost,
                            s));
    NURI_HIP(hipMemcpyAsync(C->words.data(), c.words, wshift * 8, hipMemcpyDeviceToHost, s));
    // move the rest down; the source and destination may overlap, so
    // through a scratch copy when they do
    const u64 mh = used_h - hshift, mw = used_w - wshift;
    auto move = [&](void *base, u64 shift_b, u64 bytes) {
      if (!bytes) return;
      char *b = (char *)base;
      if (shift_b >= bytes) {
        NURI_HIP(hipMemcpyAsync(b, b + shift_b, bytes, hipMemcpyDeviceToDevice, s));
      } else {
        PoolBuf<unsigned char> tmp;
        tmp.alloc(*mp, bytes);
        NURI_HIP(hipMemcpyAsync(tmp.p, b + shift_b, bytes, hipMemcpyDeviceToDevice, s));
        NURI_HIP(hipMemcpyAsync(b, tmp.p, bytes, hipMemcpyDeviceToDevice, s));
        NURI_HIP(hipStreamSynchronize(s));  // before the scratch returns to the pool
      }
    };
    move(c.hdr, hshift * sizeof(CRec), mh * sizeof(CRec));
    move(c.words, wshift * 8, mw * 8);
    if (mh && wshift) {
      const uint32_t blocks = (uint32_t)std::min<u64>((mh + 255) / 256, 4096);
      hipLaunchKernelGGL(k_rebase, dim3(blocks), dim3(256), 0, s, c.hdr, mh, wshift);
      NURI_HIP(hipGetLastError());
    }
    NURI_HIP(hipStreamSynchronize(s));
    Q.stack.erase(Q.stack.begin(), Q.stack.begin() + m);
    for (Level &L : Q.stack) {
      L.begin -= (uint32_t)hshift;
      L.wbegin -= wshift;
      L.wend -= wshift;
    }
    Q.spilled_bytes += hshift * sizeof(CRec) + wshift * 8;
    Q.spill.push_back(C);
    return true;
  }

  // the stack is empty: the last spilled chunk comes back to its offsets
  void reload(uint32_t i) {
    QHost &Q = qh[i];
    std::shared_ptr<SpillChunk> C = Q.spill.back();
    Q.spill.pop_back();
    QCfg &c = cfg[i];
    NURI_HIP(hipMemcpyAsync(c.hdr, C->hdr.data(), C->n_hdr * sizeof(CRec), hipMemcpyHostToDevice,
                            s));
    NURI_HIP(hipMemcpyAsync(c.words, C->words.data(), C->n_words * 8, hipMemcpyHostToDevice, s));
    NURI_HIP(hipStreamSynchronize(s));  // the host copy is freed below
    Q.stack = C->levels;
  }

  // plan this step for every live query into the staging block; returns
  // false when no query has work
  bool plan(uint32_t &nseg, uint32_t &nrseg, uint32_t &batch_ub, u64 &temp_need,
            uint32_t &max_seg_count, uint32_t &max_rseg_count) {
    nseg = nrseg = 0;
    batch_ub = 0;
    temp_need = 0;
    max_seg_count = max_rseg_count = 0;
    uint32_t live = 0;
    for (auto &Q : qh) live += Q.active && !Q.done;
    if (!live) return false;
    const uint64_t now = o.deadline_ns ? now_ns() : 0;
    // each live query may use an equal share of this step's output limits,
    // and at most an eighth of its own arena: a step that fills the arena
    // leaves the deeper levels so little room that the search then crawls
    // forward a few records per step
    const u64 step_share_c = step_children / live, step_share_w = step_words / live;
    u64 left_c = step_children, left_w = step_words;
    bool any = false;
    for (uint32_t i = 0; i < nq; ++i) {
      qh[i].plan = 0;
      qh[i].nsegs = 0;
    }
    rr = (rr + 1) % nq;  // the query served first rotates between steps
    for (uint32_t t = 0; t < nq; ++t) {
      const uint32_t i = (rr + t) % nq;
      QHost &Q = qh[i];
      if (!Q.active || Q.done) continue;
      if (o.deadline_ns && now - Q.t_admit > o.deadline_ns) {
        fail(i, NURI_ETIMEOUT, "query deadline passed");
        continue;
      }
      while (!Q.stack.empty() && Q.stack.back().count == 0) Q.stack.pop_back();
      while (Q.stack.empty() && !Q.spill.empty()) {
        // spilled levels are deeper than any unit subgraph: they go first
        reload(i);
        while (!Q.stack.empty() && Q.stack.back().count == 0) Q.stack.pop_back();
      }
      const u64 share_c =
          std::max<u64>(std::min<u64>(step_share_c, Q.hdr_cap / 8), max_rec_children());
      const u64 share_w =
          std::max<u64>(std::min<u64>(step_share_w, Q.word_cap / 8), max_rec_words());
      const u64 cap_c = std::min(left_c, share_c), cap_w = std::min(left_w, share_w);
      const bool prune = o.priority != NURI_PRIORITY_NONE;
      // unit subgraphs left: the next roots in bound order with bound >= theta
      const auto &rb = g.h_root_bound[Q.kind];
      const auto &ro = g.h_root_order[Q.kind];
      u64 end = g.n;
      if (Q.theta != LLONG_MIN && prune)
        end = std::lower_bound(rb.begin(), rb.end(), Q.theta,
                               [](long long a, long long t) { return a >= t; }) -
              rb.begin();
      // best-first: unit subgraphs come before records of lower bound
      long long level_best = LLONG_MIN;
      for (const Level &Lv : Q.stack)
        if (Lv.count) level_best = std::max(level_best, Lv.max_bound);
      bool roots_first = o.priority == NURI_PRIORITY_BOUND && !Q.stack.empty() &&
                         Q.cursor < end && rb[Q.cursor] > level_best;
      if (roots_first) {
        // the next unit subgraph goes on top of the stack: with too little
        // room above it, the bottom levels go to host memory first, and
        // when that is not possible the levels are expanded this step
        const u64 d = g.h_dplus[ro[Q.cursor]], w = d * 2 * ((d + 63) / 64);
        auto fits = [&]() {
          const Level &T = Q.stack.back();
          return d <= Q.hdr_cap - ((u64)T.begin + T.count) && w <= Q.word_cap - T.wend;
        };
        if (!fits() && !(spill_bottom(i) && fits())) roots_first = false;
      }
      if (Q.stack.empty() || roots_first) {
        if (Q.cursor >= end) {
          Q.done = true;
          continue;
        }
        const u64 new_h = Q.stack.empty() ? 0 : (u64)Q.stack.back().begin + Q.stack.back().count;
        const u64 new_w = Q.stack.empty() ? 0 : Q.stack.back().wend;
        u64 cc = 0, cw = 0, cnt = 0;
        const u64 lim_c = std::min<u64>(cap_c, Q.hdr_cap - new_h),
                  lim_w = std::min<u64>(cap_w, Q.word_cap - new_w);
        while (Q.cursor + cnt < end && cnt < root_B && batch_ub + cnt < batch_cap) {
          const uint32_t r = ro[Q.cursor + cnt];
          const u64 d = g.h_dplus[r];
          const u64 w = d * 2 * ((d + 63) / 64);
          if (cnt > 0 && (cc + d > lim_c || cw + w > lim_w)) break;
          cc += d;
          cw += w;
          ++cnt;
        }
        if (cc > Q.hdr_cap - new_h || cw > Q.word_cap - new_w) {
          fail(i, NURI_EBUDGET, "frontier budget too small for one unit subgraph");
          continue;
        }
        if (cnt == 0) continue;
        RootSeg &rs = srseg()[nrseg++];
        rs.qid = i;
        rs.kind = Q.kind;
        rs.first = (uint32_t)Q.cursor;
        rs.count = (uint32_t)cnt;
        max_rseg_count = std::max(max_rseg_count, rs.count);
        Q.cursor += cnt;
        Q.plan = 1;
        Q.new_begin = (uint32_t)new_h;
        Q.new_wbegin = new_w;
        batch_ub += (uint32_t)cnt;
        left_c -= std::min(left_c, cc);
        left_w -= std::min(left_w, cw);
        any = true;
        continue;
      }
      // one record of the top level must always fit; with less room than
      // one step's share left, the bottom levels go to host memory
      {
        const Level &T0 = Q.stack.back();
        const u64 rc = std::max<u64>(1, T0.maxcc), rw = rc * 2 * std::max(1u, T0.maxw);
        const u64 fh = Q.hdr_cap - (u64)(T0.begin + T0.count), fw = Q.word_cap - T0.wend;
        if (fh < std::max(rc, share_c) || fw < std::max(rw, share_w)) spill_bottom(i);
      }
      const Level &Top = Q.stack.back();
      const u64 free_h = Q.hdr_cap - (u64)(Top.begin + Top.count);
      const u64 free_w = Q.word_cap - Top.wend;
      u64 lim_c = std::min<u64>(cap_c, free_h), lim_w = std::min<u64>(cap_w, free_w);
      const u64 rec_c = std::max<u64>(1, Top.maxcc), rec_w = rec_c * 2 * std::max(1u, Top.maxw);
      if (free_h < rec_c || free_w < rec_w) {
        fail(i, NURI_EBUDGET, "frontier budget exhausted");
        continue;
      }
      if (lim_c < rec_c || lim_w < rec_w) continue;  // next step
      // levels from the top down: whole levels while they fit, then a
      // selection of the best records of the next one.  Taking from more
      // than the deepest level keeps the device busy when the deepest
      // levels are narrow; the new level still goes on top of the stack.
      Q.seg0 = nseg;
      Q.nsegs = 0;
      u64 rec_left = B;
      // levels in priority order: the deepest first, or the highest bound
      // first (ties: the deeper)
      std::vector<int> &lorder = level_order;
      lorder.resize(Q.stack.size());
      for (size_t t2 = 0; t2 < lorder.size(); ++t2) lorder[t2] = (int)(lorder.size() - 1 - t2);
      if (o.priority == NURI_PRIORITY_BOUND)
        std::stable_sort(lorder.begin(), lorder.end(), [&](int a, int b) {
          return Q.stack[a].max_bound > Q.stack[b].max_bound;
        });
      for (int li : lorder) {
        if (nseg >= L->nseg_cap || Q.nsegs >= kSegPerQuery || rec_left == 0) break;
        const Level &Lv = Q.stack[li];
        if (Lv.count == 0) continue;
        const uint32_t room = batch_cap - batch_ub;
        if (room == 0) break;
        const u64 lrc = std::max<u64>(1, Lv.maxcc), lrw = lrc * 2 * std::max(1u, Lv.maxw);
        if (lim_c < lrc || lim_w < lrw) break;
        SelSeg &sg = sseg()[nseg];
        sg = SelSeg{};
        sg.qid = i;
        sg.begin = Lv.begin;
        sg.count = Lv.count;
        sg.max_records = std::min<u64>(rec_left, room);
        sg.max_children = lim_c;
        sg.max_words = lim_w;
        sg.take_all =
            Lv.count <= sg.max_records && Lv.cost_children <= lim_c && Lv.cost_words <= lim_w;
        sg.top = Lv.max_bound;
        sg.maxcc = Lv.maxcc;
        sg.wpc = 2ull * Lv.maxw;
        long long floor_b = Q.theta == LLONG_MIN || !prune ? 0 : Q.theta;
        if (o.priority == NURI_PRIORITY_PAPER) {
          // key |P| <= the largest out-neighbourhood
          sg.top = g.degeneracy;
          floor_b = 0;
        }
        const long long span = sg.top - floor_b;
        uint32_t shift = 0;
        while (span > 0 && (span >> shift) >= kBins - 1) ++shift;
        sg.shift = shift;
        sg.temp_off = (uint32_t)temp_need;
        if (!sg.take_all) temp_need += Lv.count;
        max_seg_count = std::max(max_seg_count, Lv.count);
        seg_level[nseg] = (uint32_t)li;
        ++nseg;
        ++Q.nsegs;
        const u64 nb = sg.take_all ? Lv.count : sg.max_records;
        batch_ub += (uint32_t)nb;
        rec_left -= std::min(rec_left, nb);
        const u64 uc = sg.take_all ? Lv.cost_children : lim_c;
        const u64 uw = sg.take_all ? Lv.cost_words : lim_w;
        lim_c -= std::min(lim_c, uc);
        lim_w -= std::min(lim_w, uw);
        left_c -= std::min(left_c, uc);
        left_w -= std::min(left_w, uw);
        if (!sg.take_all) break;  // a selection uses up this query's limits
      }
      if (Q.nsegs == 0) continue;
      Q.plan = 2;
      Q.new_begin = Top.begin + Top.count;
      Q.new_wbegin = Top.wend;
      any = true;
    }
    if (!any)
      for (uint32_t i = 0; i < nq; ++i)
        if (qh[i].active && !qh[i].done)
          fail(i, NURI_EBUDGET, "frontier budget too small to make progress");
    plan_c = step_children - left_c;
    plan_w = step_words - left_w;
    return any;
  }

  void step(uint32_t nseg, uint32_t nrseg, uint32_t batch_ub, u64 temp_need,
            uint32_t max_seg_count, uint32_t max_rseg_count) {
    GView gv = view();
    // counters start at zero; configuration for this step
    memset(h_step.p, 0, L->cfg);
    for (uint32_t i = 0; i < nq; ++i) {
      cfg[i].out_hdr = qh[i].new_begin;
      cfg[i].out_word = qh[i].new_wbegin;
      sq()[i].out_max_bound = LLONG_MIN;
    }
    memcpy(h_step.p + L->cfg, cfg.data(), nq * sizeof(QCfg));
    memset(h_step.p + L->taken, 0, 4ull * L->nseg_cap);  // taken (tempc is in the zeroed part)
    NURI_HIP(hipMemcpyAsync(d_step.p, h_step.p, L->upload(nseg), hipMemcpyHostToDevice, s));
    StepHdr *dh = dev<StepHdr>(0);
    QStep *dqs = dev<QStep>(L->qs);
    QCfg *dcfg = dev<QCfg>(L->cfg);
    SelSeg *dseg = dev<SelSeg>(L->seg);
    if (nrseg) {
      const uint32_t bx = std::min<uint32_t>((max_rseg_count + 255) / 256, 1024);
      hipLaunchKernelGGL(k_make_roots, dim3(std::max(1u, bx), nrseg), dim3(256), 0, s, gv,
                         dev<RootSeg>(L->rseg), batch.p, dh);
      NURI_HIP(hipGetLastError());
    }
    if (nseg) {
      bool any_sel = false;
      for (uint32_t i = 0; i < nseg; ++i) any_sel |= !sseg()[i].take_all;
      if (temp_need && temp.n < temp_need) temp.alloc(*mp, temp_need * 2);
      const uint32_t bx = std::max(1u, std::min<uint32_t>((max_seg_count + 255) / 256, 2048));
      if (any_sel) {
        hipLaunchKernelGGL(k_sel_hist, dim3(std::min(bx, 512u), nseg), dim3(256), 0, s, gv, dseg,
                           dcfg, d_res.p, d_hist.p, d_hchild.p);
        NURI_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_sel_thresh, dim3(nseg), dim3(256), 0, s, dseg, nseg, d_hist.p,
                           d_hchild.p, dev<int>(L->thr), dev<unsigned int>(L->quota));
        NURI_HIP(hipGetLastError());
      }
      hipLaunchKernelGGL(k_sel_part, dim3(bx, nseg), dim3(256), 0, s, dseg, dcfg, d_res.p,
                         dev<int>(L->thr), dev<unsigned int>(L->quota),
                         dev<unsigned int>(L->taken), batch.p, dh, temp.p,
                         dev<unsigned int>(L->tempc), d_ctr.p);
      NURI_HIP(hipGetLastError());
      if (any_sel) {
        hipLaunchKernelGGL(k_copy_back, dim3(bx, nseg), dim3(256), 0, s, dseg, dcfg, temp.p,
                           dev<unsigned int>(L->tempc));
        NURI_HIP(hipGetLastError());
      }
    }
    uint64_t ens = 0;
    if (batch_ub) {
      if (o.profile) NURI_HIP(hipEventRecord(ev0, s));
      const uint32_t blocks = (batch_ub + kExpandWaves - 1) / kExpandWaves;
      hipLaunchKernelGGL(k_expand, dim3(blocks), dim3(64 * kExpandWaves), expand_lds, s, gv,
                         batch.p, dh, dcfg, dqs, d_ctr.p, d_flush.p, d_res.p, leaves.p,
                         leaf_words.p,
                         leaf_cap, leaf_word_cap, ex_wst, ex_lst,
                         std::min<u64>((u64)leaf_cap - plan_c - batch_ub,
                                       (leaf_word_cap - plan_w) / ex_wst),
                         o.chain_links ? o.chain_links : kMaxLinks);
      NURI_HIP(hipGetLastError());
      if (o.profile) NURI_HIP(hipEventRecord(ev1, s));
      hipLaunchKernelGGL(k_qflush, dim3(nq), dim3(64), 0, s, d_flush.p, dqs);
      NURI_HIP(hipGetLastError());
    }
    NURI_HIP(hipMemcpyAsync(h_step.p, d_step.p, L->readback(), hipMemcpyDeviceToHost, s));
    NURI_HIP(hipStreamSynchronize(s));
    take_theta();
    if (o.profile && batch_ub) {
      float ms = 0;
      NURI_HIP(hipEventElapsedTime(&ms, ev0, ev1));
      ens = (uint64_t)(ms * 1e6);
    }
    // update the level stacks
    for (uint32_t i = 0; i < nq; ++i) {
      QHost &Q = qh[i];
      if (!Q.plan) continue;
      const QStep &c = sq()[i];
      Q.steps++;
      Q.launches++;
      Q.expand_ns += ens;
      if (c.overflow) {
        fail(i, NURI_EBUDGET, "frontier overflow (internal accounting error)");
        continue;
      }
      if (Q.plan == 2) {
        const unsigned int *kept = (const unsigned int *)(h_step.p + L->tempc);
        for (uint32_t t = 0; t < Q.nsegs; ++t) {
          const uint32_t sx = Q.seg0 + t;
          Q.stack[seg_level[sx]].count = sseg()[sx].take_all ? 0 : kept[sx];
        }
      }
      if (c.n_out) {
        Level N;
        N.begin = Q.new_begin;
        N.count = c.n_out;
        N.wbegin = Q.new_wbegin;
        N.wend = Q.new_wbegin + c.out_words;
        N.cost_children = c.out_cost_children;
        N.cost_words = c.out_cost_words;
        N.max_bound = c.out_max_bound;
        N.maxcc = c.out_max_cc;
        N.maxw = c.out_max_w;
        Q.stack.push_back(N);
      }
      if (!Q.stack.empty()) {
        const Level &T = Q.stack.back();
        Q.peak_bytes = std::max<u64>(Q.peak_bytes, (u64)(T.begin + T.count) * sizeof(CRec) +
                                                        T.wend * 8);
      }
    }
    offer_leaves(sh()->leaf_count);
  }

  // leaves in the leaf buffer -> maximality check -> merge, in chunks;
  // then every query's k-th score is read back
  void offer_leaves(uint32_t nleaf) {
    if (nleaf > leaf_cap) throw Error{NURI_EBUDGET, "leaf buffer overflow (internal)"};
    if (!nleaf) return;
    GView gv = view();
    StepHdr *dh = dev<StepHdr>(0);
    uint32_t kmax = 0;
    for (auto &Q : qh)
      if (Q.active) kmax = std::max(kmax, Q.k);
    for (uint32_t f = 0; f < nleaf; f += kCandChunk) {
      const uint32_t cnt = std::min<uint32_t>(kCandChunk, nleaf - f);
      NURI_HIP(hipMemsetAsync(&dh->cand_count, 0, sizeof(unsigned int), s));
      hipLaunchKernelGGL(k_leaf_check, dim3(cnt), dim3(64 * kLeafWaves), 0, s, gv, leaves.p, f, leaf_words.p,
                         d_res.p, cands.p, &dh->cand_count, cand_ids.p, lmax, d_ctr.p);
      NURI_HIP(hipGetLastError());
      launch_merge(cands.p, dh, cand_ids.p, lmax, d_res.p, d_k.p, mbuf, nq, kmax, cnt, s);
    }
    // the k-th scores come back with the next step's read-back: the host
    // plans one step with the previous ones, which are never above the
    // current ones, so it prunes less, never wrongly (the kernels read the
    // current ones from device memory)
    NURI_HIP(hipMemcpyAsync(h_res.p, d_res.p, nq * sizeof(QRes), hipMemcpyDeviceToHost, s));
    theta_pending = true;
  }

  // after a synchronisation: take the k-th scores copied back last
  void take_theta() {
    if (!theta_pending) return;
    theta_pending = false;
    for (uint32_t i = 0; i < nq; ++i)
      if (qh[i].active) qh[i].theta = h_res.p[i].theta;
  }

  // seed cliques for queries that have none yet (see k_seed_dive)
  void seed_new() {
    uint32_t ns = 0, maxc = 0;
    u64 total = 0;
    for (uint32_t i = 0; i < nq; ++i) {
      QHost &Q = qh[i];
      if (!Q.active || Q.done || Q.seeded) continue;
      if (o.priority == NURI_PRIORITY_NONE) {
        Q.seeded = true;  // no pruning: an early k-th score would not be used
        continue;
      }
      const u64 want = std::min<u64>(g.n, std::max<u64>(2ull * Q.k, 512));
      const u64 room = std::min<u64>(leaf_cap, leaf_word_cap / ex_wst);
      if (total + want > room) break;  // the rest seed at the next step
      Q.seeded = true;
      SeedSeg &sg = h_seed.p[ns++];
      sg.qid = i;
      sg.kind = (uint32_t)Q.kind;
      sg.count = (uint32_t)want;
      sg.pad = 0;
      total += want;
      maxc = std::max<uint32_t>(maxc, sg.count);
    }
    if (!ns) return;
    StepHdr *dh = dev<StepHdr>(0);
    QStep *dqs = dev<QStep>(L->qs);
    NURI_HIP(hipMemsetAsync(d_step.p, 0, L->cfg, s));  // counters and overflow flags
    NURI_HIP(hipMemcpyAsync(d_seed.p, h_seed.p, ns * sizeof(SeedSeg), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_seed_dive, dim3((maxc + 3) / 4, ns), dim3(256), 0, s, view(), d_seed.p,
                       leaves.p, leaf_words.p, dh, leaf_cap, leaf_word_cap, dqs);
    NURI_HIP(hipGetLastError());
    NURI_HIP(hipMemcpyAsync(h_step.p, d_step.p, L->readback(), hipMemcpyDeviceToHost, s));
    NURI_HIP(hipStreamSynchronize(s));
    for (uint32_t t = 0; t < ns; ++t)
      if (sq()[h_seed.p[t].qid].overflow)
        throw Error{NURI_EBUDGET, "leaf buffer overflow while seeding (internal)"};
    offer_leaves(sh()->leaf_count);
  }

  // one step for every live query; false when none has work left
  bool step_all() {
    uint32_t nseg, nrseg, batch_ub, mseg, mrseg;
    u64 temp_need;
    seed_new();
    const uint64_t t0 = trace ? now_ns() : 0;
    if (!plan(nseg, nrseg, batch_ub, temp_need, mseg, mrseg)) return false;
    const uint64_t t1 = trace ? now_ns() : 0;
    step(nseg, nrseg, batch_ub, temp_need, mseg, mrseg);
    if (trace && ++trace_steps % trace == 0) {
      uint32_t live = 0;
      for (auto &Q : qh) live += Q.active && !Q.done;
      size_t depth = 0;
      for (auto &Q : qh) depth = std::max(depth, Q.stack.size());
      fprintf(stderr, "[nuri] step live=%u segs=%u roots=%u batch<=%u maxlevel=%u temp=%llu "
              "leaves=%u plan_us=%llu step_us=%llu theta0=%lld depth=%zu\n", live, nseg, nrseg,
              batch_ub, mseg, (unsigned long long)temp_need, sh()->leaf_count,
              (unsigned long long)(t1 - t0) / 1000, (unsigned long long)(now_ns() - t1) / 1000,
              qh[0].theta, depth);
    }
    return true;
  }

  // result of a finished query; frees its slot
  void harvest(uint32_t i, Result &res) {
    QHost &Q = qh[i];
    NURI_HIP(hipMemcpyAsync(&h_res.p[i], &d_res.p[i], sizeof(QRes), hipMemcpyDeviceToHost, s));
    NURI_HIP(hipMemcpyAsync(&h_ctr.p[(u64)i * kCtrSlots], &d_ctr.p[(u64)i * kCtrSlots],
                            kCtrSlots * sizeof(QCtr), hipMemcpyDeviceToHost, s));
    NURI_HIP(hipStreamSynchronize(s));
    const QRes &R = h_res.p[i];
    const uint32_t n = Q.error ? 0 : R.tk_n;
    std::vector<long long> sc(n);
    std::vector<unsigned int> ln(n), ids((u64)n * lmax);
    if (n) {
      NURI_HIP(hipMemcpyAsync(sc.data(), R.tk_score[R.cur], n * 8, hipMemcpyDeviceToHost, s));
      NURI_HIP(hipMemcpyAsync(ln.data(), R.tk_len[R.cur], n * 4, hipMemcpyDeviceToHost, s));
      NURI_HIP(hipMemcpyAsync(ids.data(), R.tk_ids[R.cur], (u64)n * lmax * 4,
                              hipMemcpyDeviceToHost, s));
      NURI_HIP(hipStreamSynchronize(s));
    }
    res.error = Q.error;
    res.errmsg = Q.errmsg;
    res.score.assign(sc.begin(), sc.end());
    res.offset.assign(1, 0);
    res.ids.clear();
    for (uint32_t t = 0; t < n; ++t) {
      res.ids.insert(res.ids.end(), ids.begin() + (u64)t * lmax,
                     ids.begin() + (u64)t * lmax + ln[t]);
      res.offset.push_back(res.ids.size());
    }
    QCtr c;
    memset(&c, 0, sizeof(c));
    for (uint32_t t = 0; t < kCtrSlots; ++t) {
      const QCtr &e = h_ctr.p[(u64)i * kCtrSlots + t];
      c.popped += e.popped;
      c.expanded += e.expanded;
      c.children += e.children;
      c.pruned_pop += e.pruned_pop;
      c.pruned_new += e.pruned_new;
      c.leaves += e.leaves;
      c.offered += e.offered;
      c.logical_bytes += e.logical_bytes;
      c.onchip_bytes += e.onchip_bytes;
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
    st.logical_bytes = c.logical_bytes;
    st.onchip_bytes = c.onchip_bytes;
    st.expand_launches = Q.launches;
    st.expand_ns = Q.expand_ns;
    st.wall_ns = now_ns() - Q.t_admit;
    st.ties_at_k = ties_at_k(res.score, Q.k);
    st.spilled_bytes = Q.spilled_bytes;
    Q.active = false;
    Q.stack.clear();
    Q.spill.clear();
    tk[i]->score.release();
    tk[i]->len.release();
    tk[i]->ids.release();
    tk[i]->hdr.release();
    tk[i]->words.release();
    cfg[i].hdr = nullptr;
    cfg[i].words = nullptr;
  }
};

}  // namespace

void check_clique_query(const Graph &g, uint32_t k, int kind) {
  if (k == 0) throw Error{NURI_EINVAL, "k must be >= 1"};
  if (kind != 0 && kind != 1) throw Error{NURI_EINVAL, "unknown weight_fn"};
  if (kind == 1 && !g.has_vw)
    throw Error{NURI_EINVAL, "NURI_SCORE_VERTEX_WEIGHT needs vertex weights"};
}

void run_cliques(Graph &g, const std::vector<uint32_t> &ks, const std::vector<int> &kinds,
                 const QueryOpts &o, std::vector<Result> &out) {
  if (ks.empty()) return;
  if (ks.size() > 65535) throw Error{NURI_EINVAL, "at most 65535 queries per batch"};
  for (size_t i = 0; i < ks.size(); ++i) check_clique_query(g, ks[i], kinds[i]);
  // as many queries live at once as the frontier budget holds arenas of at
  // least the smallest useful size; the others wait for a slot and run
  // when one is harvested
  const uint32_t nq = (uint32_t)ks.size();
  Engine e(g, o);
  const u64 per = std::max<u64>(e.min_arena_bytes(), o.frontier_budget / nq);
  const uint32_t slots = (uint32_t)std::max<u64>(1, std::min<u64>(nq, o.frontier_budget / per));
  e.setup(slots);
  e.arena_bytes = o.frontier_budget / slots;
  std::vector<uint32_t> slot_query(slots, UINT32_MAX);
  uint32_t next = 0;
  out.resize(nq);
  auto fill = [&] {
    for (uint32_t s = 0; s < slots && next < nq; ++s)
      if (e.slot_free(s)) {
        e.admit(s, ks[next], kinds[next]);
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

// One clique query whose device buffers all come from the caller's fixed
// region [base, base + bytes): nothing is allocated on the device and no
// host memory is page-locked.  The region's previous contents are never
// read: every buffer that must start at zero is cleared by the query.
void run_clique_fixed(Graph &g, uint32_t k, int kind, const QueryOpts &o, void *base, size_t bytes,
                      Result &out) {
  check_clique_query(g, k, kind);
  MemPool region;
  region.fixed_base = static_cast<unsigned char *>(base);
  region.fixed_size = bytes;
  QueryOpts q = o;
  q.profile = false;  // no HIP events either
  Engine e(g, q, &region);
  const u64 lmax = g.degeneracy + 1;
  e.fixed_topk_bytes = MemPool::align_up(2ull * k * 8) + MemPool::align_up(2ull * k * 4) +
                       MemPool::align_up(2ull * k * lmax * 4);
  e.setup(1);
  e.admit(0, k, kind);
  while (e.step_all()) {
  }
  e.harvest(0, out);
  if (out.error) throw Error{out.error, out.errmsg};
}

// ------------------------------------------------------------------
// slot interface for the server
// ------------------------------------------------------------------
struct CliqueSlots::Impl {
  Engine e;
  Impl(Graph &g, const QueryOpts &o) : e(g, o) {}
};

CliqueSlots::CliqueSlots(Graph &g, const QueryOpts &o, uint32_t slots) : impl(new Impl(g, o)) {
  impl->e.server_mode = true;
  impl->e.setup(slots);
}
CliqueSlots::~CliqueSlots() = default;
uint32_t CliqueSlots::slots() const { return impl->e.nq; }
bool CliqueSlots::free(uint32_t i) const { return impl->e.slot_free(i); }
bool CliqueSlots::finished(uint32_t i) const { return impl->e.finished(i); }
bool CliqueSlots::live() const { return impl->e.any_live(); }
void CliqueSlots::admit(uint32_t i, uint32_t k, int kind, uint64_t bytes) {
  check_clique_query(impl->e.g, k, kind);
  impl->e.admit(i, k, kind, bytes);
}
uint64_t CliqueSlots::min_arena_bytes() const { return impl->e.min_arena_bytes(); }
bool CliqueSlots::step() { return impl->e.step_all(); }
void CliqueSlots::harvest(uint32_t i, Result &r) { impl->e.harvest(i, r); }

}  // namespace nuri
