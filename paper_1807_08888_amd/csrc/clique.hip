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
#include <cstring>

#include "nuri_internal.h"

namespace nuri {
namespace {

typedef unsigned long long u64;

struct CRec {
  long long score;
  long long bound;
  u64 woff;       // word offset of the bitmap in the query's word arena
  uint32_t root;  // rank of the root vertex
  int16_t last;   // local position of the last added vertex; -1 for a unit subgraph
  uint16_t qid;
};
static_assert(sizeof(CRec) == 32, "frontier record must stay 32 bytes");

struct LRec {  // a child with an empty candidate set, awaiting the maximality check
  long long score;
  u64 woff;  // word offset of its member bitmap in the leaf word arena
  uint32_t root;
  int16_t last;
  uint16_t qid;
};

struct Cand {  // a maximal clique offered to the result set
  long long score;
  uint32_t qid;
  uint32_t len;
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
};

struct QCtr {  // per query, device counters
  // per step (cleared before each step)
  unsigned int n_out, n_kept;
  u64 out_words, out_cost_children, out_cost_words;
  long long out_max_bound;
  unsigned int overflow, pad;
  // cumulative
  u64 popped, expanded, children, pruned_pop, pruned_new, leaves, offered, logical_bytes;
};

struct QRes {  // per query result state
  long long theta;  // score of the k-th result; LLONG_MIN while fewer than k results
  unsigned int tk_n, cur;
  long long *tk_score[2];
  unsigned int *tk_len[2];
  unsigned int *tk_ids[2];  // stride lmax
};

struct GView {
  const uint32_t *dplus, *split, *oplus, *orig, *rcol;
  const uint64_t *ooff, *bm_off, *rrow;
  const u64 *bm;
  const int32_t *wloc, *vw;
  const int64_t *wplus;
  const uint32_t *root_order[2];
};

struct SelSeg {  // one query's level to take records from this step
  uint32_t qid, begin, count, take_all;
  uint32_t shift, nbins_used;
  long long top;  // upper bound of every bound in the level
  uint32_t temp_off, max_records;
  u64 max_children, max_words;
};

struct RootSeg {
  uint32_t qid, kind;
  uint32_t first, count;  // positions in the root order
};

constexpr int kBins = 2048;
constexpr uint32_t kCandChunk = 2048;

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// bits of word w whose position w*64+b is greater than pos (pos may be -1)
__device__ inline u64 gt_mask(int w, int pos) {
  int lo = w * 64;
  if (pos < lo) return ~0ull;
  if (pos >= lo + 63) return 0ull;
  return ~0ull << (pos - lo + 1);
}

// bits of word w whose position is below d
__device__ inline u64 lt_mask(int w, uint32_t d) {
  int lo = w * 64;
  if ((int)d >= lo + 64) return ~0ull;
  if ((int)d <= lo) return 0ull;
  return (1ull << (d - lo)) - 1ull;
}

__device__ inline uint32_t words_of(uint32_t d) { return (d + 63) >> 6; }

// exclusive prefix sum over the 64 lanes of a wave
__device__ inline uint32_t wave_excl_scan(uint32_t x, int lane) {
  uint32_t inc = x;
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t t = __shfl_up(inc, off, 64);
    if (lane >= off) inc += t;
  }
  return inc - x;
}

__device__ inline u64 wave_sum(u64 x) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

__device__ inline long long wave_max(long long x) {
  for (int off = 32; off > 0; off >>= 1) {
    long long y = __shfl_xor(x, off, 64);
    x = y > x ? y : x;
  }
  return x;
}

// ------------------------------------------------------------------
// unit subgraphs (Algorithm 1, lines 1-3), taken in root-bound order
// ------------------------------------------------------------------
__global__ void k_make_roots(GView g, const RootSeg *segs, uint32_t nseg, CRec *batch,
                             unsigned int *batch_count) {
  // one block per segment chunk of 256 roots is simpler than a map: loop
  for (uint32_t s = 0; s < nseg; ++s) {
    RootSeg sg = segs[s];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < sg.count;
         i += gridDim.x * blockDim.x) {
      uint32_t r = g.root_order[sg.kind][sg.first + i];
      CRec c;
      c.score = sg.kind ? (long long)g.vw[r] : 1;
      c.bound = sg.kind ? c.score + g.wplus[r] : 1 + (long long)g.dplus[r];
      c.woff = 0;
      c.root = r;
      c.last = -1;
      c.qid = (uint16_t)sg.qid;
      unsigned int slot = atomicAdd(batch_count, 1u);
      batch[slot] = c;
    }
  }
}

// ------------------------------------------------------------------
// select: histogram of bounds, threshold, partition
// ------------------------------------------------------------------
// Record cost bounds: a record at `last` in a universe of d can create at
// most d-last-1 children, each 2W words.
__device__ inline void rec_cost(const GView &g, const CRec &c, u64 &children, u64 &words) {
  uint32_t d = g.dplus[c.root];
  u64 ch = (u64)(d - (uint32_t)(c.last + 1));
  children = ch;
  words = ch * 2 * words_of(d);
}

__device__ inline int bin_of(long long bound, long long top, uint32_t shift) {
  long long gap = (top - bound) >> shift;
  long long b = kBins - 1 - gap;
  return b < 0 ? 0 : (b > kBins - 1 ? kBins - 1 : (int)b);
}

__global__ void k_sel_hist(GView g, const SelSeg *segs, const uint32_t *blk_seg,
                           const uint32_t *blk_off, const QCfg *cfg, const QRes *res,
                           unsigned int *hist, u64 *hchild, u64 *hword, u64 *hmaxc, u64 *hmaxw) {
  uint32_t s = blk_seg[blockIdx.x];
  SelSeg sg = segs[s];
  if (sg.take_all) return;
  uint32_t i = blk_off[blockIdx.x] + threadIdx.x;
  if (i >= sg.count) return;
  const CRec c = cfg[sg.qid].hdr[sg.begin + i];
  if (c.bound < res[sg.qid].theta) return;
  int b = bin_of(c.bound, sg.top, sg.shift);
  u64 ch, w;
  rec_cost(g, c, ch, w);
  size_t o = (size_t)s * kBins + b;
  atomicAdd(&hist[o], 1u);
  atomicAdd(&hchild[o], ch);
  atomicAdd(&hword[o], w);
  atomicMax(&hmaxc[o], ch);
  atomicMax(&hmaxw[o], w);
}

// one wave per segment: scan bins from the top until a limit is reached
__global__ void k_sel_thresh(const SelSeg *segs, uint32_t nseg, const unsigned int *hist,
                             const u64 *hchild, const u64 *hword, const u64 *hmaxc,
                             const u64 *hmaxw, int *thr, unsigned int *quota) {
  uint32_t s = blockIdx.x;
  if (s >= nseg || threadIdx.x != 0) return;
  SelSeg sg = segs[s];
  if (sg.take_all) return;
  u64 n = 0, c = 0, w = 0;
  int t = -1;
  unsigned int q = 0;
  for (int b = kBins - 1; b >= 0; --b) {
    size_t o = (size_t)s * kBins + b;
    u64 hn = hist[o];
    if (!hn) continue;
    if (n + hn <= sg.max_records && c + hchild[o] <= sg.max_children &&
        w + hword[o] <= sg.max_words) {
      n += hn;
      c += hchild[o];
      w += hword[o];
      continue;
    }
    u64 qa = sg.max_records - n;
    u64 mc = hmaxc[o] ? (sg.max_children - c) / hmaxc[o] : qa;
    u64 mw = hmaxw[o] ? (sg.max_words - w) / hmaxw[o] : qa;
    qa = qa < mc ? qa : mc;
    qa = qa < mw ? qa : mw;
    if (qa == 0 && n == 0) qa = 1;  // the host guarantees one record always fits
    t = b;
    q = (unsigned int)(qa < hn ? qa : hn);
    break;
  }
  thr[s] = t;
  quota[s] = q;
}

__global__ void k_sel_part(GView g, const SelSeg *segs, const uint32_t *blk_seg,
                           const uint32_t *blk_off, const QCfg *cfg, const QRes *res,
                           const int *thr, const unsigned int *quota, unsigned int *taken,
                           CRec *batch, unsigned int *batch_count, CRec *temp,
                           unsigned int *temp_count, QCtr *ctr) {
  uint32_t s = blk_seg[blockIdx.x];
  SelSeg sg = segs[s];
  uint32_t i = blk_off[blockIdx.x] + threadIdx.x;
  bool valid = i < sg.count;
  CRec c;
  int where = 0;  // 0 none, 1 batch, 2 keep, 3 pruned
  if (valid) {
    c = cfg[sg.qid].hdr[sg.begin + i];
    if (c.bound < res[sg.qid].theta) {
      where = 3;
    } else if (sg.take_all) {
      where = 1;
    } else {
      int b = bin_of(c.bound, sg.top, sg.shift);
      int t = thr[s];
      if (b > t) where = 1;
      else if (b < t) where = 2;
      else where = atomicAdd(&taken[s], 1u) < quota[s] ? 1 : 2;
    }
  }
  if (where == 1) batch[atomicAdd(batch_count, 1u)] = c;
  if (where == 2) temp[sg.temp_off + atomicAdd(&temp_count[s], 1u)] = c;
  if (where == 3) {
    atomicAdd(&ctr[sg.qid].popped, 1ull);
    atomicAdd(&ctr[sg.qid].pruned_pop, 1ull);
  }
}

// clear the per-step counters of every query
__global__ void k_reset_step(QCtr *ctr, uint32_t nq) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq) return;
  QCtr &c = ctr[i];
  c.n_out = c.n_kept = 0;
  c.out_words = c.out_cost_children = c.out_cost_words = 0;
  c.out_max_bound = LLONG_MIN;
  c.overflow = 0;
}

__global__ void k_copy_back(const SelSeg *segs, uint32_t nseg, const QCfg *cfg, const CRec *temp,
                            const unsigned int *temp_count, QCtr *ctr) {
  for (uint32_t s = 0; s < nseg; ++s) {
    SelSeg sg = segs[s];
    unsigned int kept = sg.take_all ? 0u : temp_count[s];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < kept;
         i += gridDim.x * blockDim.x)
      cfg[sg.qid].hdr[sg.begin + i] = temp[sg.temp_off + i];
    if (blockIdx.x == 0 && threadIdx.x == 0) ctr[sg.qid].n_kept = kept;
  }
}

// ------------------------------------------------------------------
// expand (Algorithm 1, lines 11-16)
// ------------------------------------------------------------------
// One wavefront per record.  The record's candidate positions are listed
// in LDS; its children are then processed 64/G at a time, G = the power of
// two >= W lanes per child, each lane ANDing one word of the parent's
// candidate bitmap with one word of the child vertex's local adjacency
// row.  Group reductions give |P'| (or w(P')); survivors are compacted
// with a ballot and one atomic per wave and written with coalesced stores.
constexpr int kExpandWaves = 4;

__global__ void __launch_bounds__(64 * kExpandWaves)
    k_expand(GView g, const CRec *__restrict__ batch, const unsigned int *batch_count,
             const QCfg *__restrict__ cfg, QCtr *ctr, const QRes *__restrict__ res, LRec *leaves,
             unsigned int *leaf_count, u64 *leaf_words, u64 *leaf_word_count, uint32_t leaf_cap,
             u64 leaf_word_cap) {
  __shared__ uint16_t s_list[kExpandWaves][kMaxLocal];
  __shared__ u64 s_pw[kExpandWaves][kMaxWords];
  __shared__ u64 s_vw[kExpandWaves][kMaxWords];
  __shared__ u64 s_xw[kExpandWaves][kMaxWords];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint32_t rec = blockIdx.x * kExpandWaves + wv;
  if (rec >= *batch_count) return;
  const CRec p = batch[rec];
  const uint32_t q = p.qid;
  const QCfg cf = cfg[q];
  const long long theta = res[q].theta;
  u64 st_popped = 1, st_pruned_pop = 0, st_expanded = 0, st_children = 0, st_pruned_new = 0,
      st_leaves = 0, st_bytes = 0, st_cost_c = 0, st_cost_w = 0;
  long long st_maxb = LLONG_MIN;

  const uint32_t r = p.root;
  const uint32_t d = g.dplus[r];
  const uint32_t W = words_of(d);
  if (p.bound < theta) {
    st_pruned_pop = 1;
  } else if (d == 0) {
    // a unit subgraph with no later neighbour: itself a leaf
    st_leaves = 1;
    if (p.score >= theta && lane == 0) {
      unsigned int slot = atomicAdd(leaf_count, 1u);
      if (slot < leaf_cap) {
        LRec l;
        l.score = p.score;
        l.woff = 0;
        l.root = r;
        l.last = -1;
        l.qid = (uint16_t)q;
        leaves[slot] = l;
      } else {
        atomicAdd(&ctr[q].overflow, 1u);
      }
    }
  } else {
    const int last = p.last;
    u64 word = 0, xword = 0;
    if (lane < (int)W) {
      word = last < 0 ? lt_mask(lane, d) : cf.words[p.woff + lane];
      xword = last < 0 ? 0ull : cf.words[p.woff + W + lane];
    }
    const u64 pw = word & gt_mask(lane, last);
    const u64 vwd = word & ~gt_mask(lane, last);
    if (lane < (int)W) {
      s_pw[wv][lane] = pw;
      s_vw[wv][lane] = vwd;
      s_xw[wv][lane] = xword;
    }
    // list the candidate positions in increasing order
    uint32_t c = __popcll(pw);
    uint32_t off = wave_excl_scan(c, lane);
    uint32_t nchild = __shfl(off + c, 63, 64);
    {
      u64 t = pw;
      uint32_t o = off;
      while (t) {
        int b = __ffsll((long long)t) - 1;
        s_list[wv][o++] = (uint16_t)(lane * 64 + b);
        t &= t - 1;
      }
    }
    wave_sync();
    if (last >= 0 && lane == 0) st_bytes += 32 + 16ull * W;  // the parent record
    if (nchild) st_expanded = 1;
    const u64 *rows = g.bm + g.bm_off[r];
    const int32_t *wl = g.wloc + g.ooff[r];
    const bool weighted = cf.weighted != 0;
    uint32_t G = 1;
    while (G < W) G <<= 1;
    const uint32_t per = 64 / G;
    const int wi = lane & (G - 1);
    const int gl = lane & ~(int)(G - 1);  // lane of this group's leader
    for (uint32_t base = 0; base < nchild; base += per) {
      const uint32_t ci = base + lane / G;
      const bool valid = ci < nchild;
      const uint32_t j = valid ? s_list[wv][ci] : 0;
      u64 a = 0, xc = 0;
      if (valid && wi < (int)W) {
        const u64 row = rows[(u64)j * W + wi];
        const u64 pv = s_pw[wv][wi];
        a = pv & row & gt_mask(wi, (int)j);                              // P'
        xc = (s_xw[wv][wi] | (pv & ~gt_mask(wi, (int)j - 1))) & row;     // X'
      }
      // extension witness: the first vertex of X'; if it is adjacent to all
      // of P', no clique below this child is maximal
      int x0 = xc ? wi * 64 + __ffsll((long long)xc) - 1 : 0x7FFFFFFF;
      for (uint32_t o2 = 1; o2 < G; o2 <<= 1) {
        int y = __shfl_xor(x0, o2, 64);
        x0 = y < x0 ? y : x0;
      }
      bool covered = false;
      if (x0 != 0x7FFFFFFF) {
        int miss = (wi < (int)W) ? ((a & ~rows[(u64)x0 * W + wi]) != 0ull) : 0;
        for (uint32_t o2 = 1; o2 < G; o2 <<= 1) miss |= __shfl_xor(miss, o2, 64);
        covered = miss == 0;
      }
      uint32_t cnt = __popcll(a);
      long long wsum = 0;
      if (weighted) {
        u64 t = a;
        while (t) {
          int b = __ffsll((long long)t) - 1;
          wsum += wl[wi * 64 + b];
          t &= t - 1;
        }
      }
      for (uint32_t o2 = 1; o2 < G; o2 <<= 1) {
        cnt += __shfl_xor(cnt, o2, 64);
        if (weighted) wsum += __shfl_xor(wsum, o2, 64);
      }
      const long long score2 = p.score + (weighted ? (long long)wl[j] : 1ll);
      const long long bound2 = score2 + (weighted ? wsum : (long long)cnt);
      const bool leader = valid && wi == 0;
      const bool prune = bound2 < theta || covered;
      const bool leaf = valid && !prune && cnt == 0;
      const bool keep = valid && !prune && cnt > 0;
      const bool offer = leaf && score2 >= theta;
      const u64 lm = __ballot(leader);
      const u64 km = __ballot(leader && keep);
      const u64 fm = __ballot(leader && offer);
      st_children += __popcll(lm);
      st_pruned_new += __popcll(__ballot(leader && prune));
      st_leaves += __popcll(__ballot(leader && leaf));
      if (lane == 0) st_bytes += 8ull * W * __popcll(lm);  // adjacency rows read
      if (wi == 0 && valid && x0 != 0x7FFFFFFF) st_bytes += 8ull * W;  // witness row
      const u64 below = gl ? ((1ull << gl) - 1ull) : 0ull;
      const u64 jbit = (wi == (int)(j >> 6)) ? (1ull << (j & 63)) : 0ull;
      if (km) {
        const uint32_t nk = __popcll(km);
        unsigned int h0 = 0;
        u64 w0 = 0;
        if (lane == 0) {
          h0 = atomicAdd(&ctr[q].n_out, nk);
          w0 = atomicAdd(&ctr[q].out_words, (u64)nk * 2 * W);
        }
        h0 = __shfl(h0, 0, 64);
        w0 = __shfl(w0, 0, 64);
        if (keep) {
          const uint32_t rk = __popcll(km & below);
          const u64 slot_h = (u64)cf.out_hdr + h0 + rk;
          const u64 slot_w = cf.out_word + w0 + (u64)rk * 2 * W;
          if (slot_h < cf.hdr_cap && slot_w + 2 * W <= cf.word_cap) {
            if (wi < (int)W) {
              cf.words[slot_w + wi] = s_vw[wv][wi] | a | jbit;
              cf.words[slot_w + W + wi] = xc;
            }
            if (wi == 0) {
              CRec ch;
              ch.score = score2;
              ch.bound = bound2;
              ch.woff = slot_w;
              ch.root = r;
              ch.last = (int16_t)j;
              ch.qid = (uint16_t)q;
              cf.hdr[slot_h] = ch;
            }
          } else if (wi == 0) {
            atomicAdd(&ctr[q].overflow, 1u);
          }
          if (wi == 0) {
            u64 cc = (u64)(d - j - 1);
            st_cost_c += cc;
            st_cost_w += cc * 2 * W;
            st_maxb = bound2 > st_maxb ? bound2 : st_maxb;
            st_bytes += 32 + 16ull * W;
          }
        }
      }
      if (fm) {
        const uint32_t nf = __popcll(fm);
        unsigned int l0 = 0;
        u64 w0 = 0;
        if (lane == 0) {
          l0 = atomicAdd(leaf_count, nf);
          w0 = atomicAdd(leaf_word_count, (u64)nf * W);
        }
        l0 = __shfl(l0, 0, 64);
        w0 = __shfl(w0, 0, 64);
        if (offer) {
          const uint32_t rk = __popcll(fm & below);
          const u64 slot_l = (u64)l0 + rk;
          const u64 slot_w = w0 + (u64)rk * W;
          if (slot_l < leaf_cap && slot_w + W <= leaf_word_cap) {
            if (wi < (int)W) leaf_words[slot_w + wi] = s_vw[wv][wi] | jbit;
            if (wi == 0) {
              LRec l;
              l.score = score2;
              l.woff = slot_w;
              l.root = r;
              l.last = (int16_t)j;
              l.qid = (uint16_t)q;
              leaves[slot_l] = l;
              st_bytes += 24 + 8ull * W;
            }
          } else if (wi == 0) {
            atomicAdd(&ctr[q].overflow, 1u);
          }
        }
      }
    }
  }
  // flush per-wave statistics with one atomic each
  st_cost_c = wave_sum(st_cost_c);
  st_cost_w = wave_sum(st_cost_w);
  st_bytes = wave_sum(st_bytes);
  st_maxb = wave_max(st_maxb);
  if (lane == 0) {
    QCtr &C = ctr[q];
    atomicAdd(&C.popped, st_popped);
    if (st_pruned_pop) atomicAdd(&C.pruned_pop, st_pruned_pop);
    if (st_expanded) atomicAdd(&C.expanded, st_expanded);
    if (st_children) atomicAdd(&C.children, st_children);
    if (st_pruned_new) atomicAdd(&C.pruned_new, st_pruned_new);
    if (st_leaves) atomicAdd(&C.leaves, st_leaves);
    if (st_bytes) atomicAdd(&C.logical_bytes, st_bytes);
    if (st_cost_c) atomicAdd(&C.out_cost_children, st_cost_c);
    if (st_cost_w) atomicAdd(&C.out_cost_words, st_cost_w);
    if (st_maxb != LLONG_MIN) atomicMax(&C.out_max_bound, st_maxb);
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
constexpr int kLeafCap = kMaxLocal + 1;

__global__ void __launch_bounds__(64)
    k_leaf_check(GView g, const LRec *leaves, uint32_t first, const u64 *leaf_words,
                 const QRes *res, Cand *cands, unsigned int *cand_count, uint32_t *cand_ids,
                 uint32_t lmax, QCtr *ctr) {
  __shared__ uint32_t s_rank[kLeafCap];
  __shared__ uint32_t s_id[kLeafCap];
  __shared__ uint32_t s_sorted[kLeafCap];
  const int lane = threadIdx.x;
  const LRec L = leaves[first + blockIdx.x];
  const uint32_t q = L.qid;
  if (L.score < res[q].theta) return;
  const uint32_t r = L.root;
  const uint32_t d = g.dplus[r];
  const uint32_t W = words_of(d);
  u64 v = 0;
  if (d && lane < (int)W) v = leaf_words[L.woff + lane];
  // member positions -> ranks
  uint32_t c = __popcll(v);
  uint32_t off = wave_excl_scan(c, lane);
  const uint32_t nm = __shfl(off + c, 63, 64);
  const uint32_t *np = g.oplus + g.ooff[r];
  {
    u64 t = v;
    uint32_t o = off;
    while (t) {
      int b = __ffsll((long long)t) - 1;
      s_rank[o++] = np[lane * 64 + b];
      t &= t - 1;
    }
  }
  if (lane == 0) s_rank[nm] = r;
  wave_sync();
  const uint32_t nc = nm + 1;  // clique size
  // (a) local extension
  if (d) {
    u64 x = (lane < (int)W) ? (~v & lt_mask(lane, d)) : 0ull;
    const u64 *rows = g.bm + g.bm_off[r];
    // walk members in position order via their bits
    for (int w = 0; w < (int)W && __ballot(x != 0); ++w) {
      u64 mw = __shfl(v, w, 64);
      while (mw && __ballot(x != 0)) {
        int b = __ffsll((long long)mw) - 1;
        uint32_t i = w * 64 + b;
        if (lane < (int)W) x &= rows[(u64)i * W + lane];
        mw &= mw - 1;
      }
    }
    if (__ballot(x != 0)) return;
  }
  // (b) extension by a vertex ranked below r
  {
    // member with the fewest lower neighbours
    uint32_t bestc = 0xFFFFFFFFu, besti = 0;
    for (uint32_t t = lane; t < nc; t += 64) {
      uint32_t s = g.split[s_rank[t]];
      if (s < bestc) { bestc = s; besti = t; }
    }
    for (int o2 = 32; o2 > 0; o2 >>= 1) {
      uint32_t oc = __shfl_xor(bestc, o2, 64), oi = __shfl_xor(besti, o2, 64);
      if (oc < bestc || (oc == bestc && oi < besti)) { bestc = oc; besti = oi; }
    }
    const uint32_t cs = s_rank[besti];
    const uint32_t *lo_list = g.rcol + g.rrow[cs];
    // entries of N-(cs) below r form a prefix (rows are sorted)
    uint32_t lo = 0, hi = g.split[cs];
    while (lo < hi) {
      uint32_t mid = (lo + hi) >> 1;
      if (lo_list[mid] < r) lo = mid + 1; else hi = mid;
    }
    const uint32_t nu = lo;
    for (uint32_t b0 = 0; b0 < nu; b0 += 64) {
      bool ext = false;
      uint32_t t = b0 + lane;
      if (t < nu) {
        uint32_t u = lo_list[t];
        const uint32_t *up = g.oplus + g.ooff[u];
        uint32_t du = g.dplus[u];
        ext = true;
        for (uint32_t m = 0; m < nc && ext; ++m) {
          if (m == besti) continue;
          uint32_t x = s_rank[m];
          uint32_t a = 0, z = du;
          while (a < z) {
            uint32_t mid = (a + z) >> 1;
            if (up[mid] < x) a = mid + 1; else z = mid;
          }
          ext = a < du && up[a] == x;
        }
      }
      if (__ballot(ext)) return;
    }
  }
  // maximal: emit (score, ascending original ids)
  for (uint32_t t = lane; t < nc; t += 64) s_id[t] = g.orig[s_rank[t]];
  wave_sync();
  for (uint32_t t = lane; t < nc; t += 64) {
    uint32_t x = s_id[t], rk = 0;
    for (uint32_t u = 0; u < nc; ++u) rk += s_id[u] < x;
    s_sorted[rk] = x;
  }
  wave_sync();
  unsigned int slot = 0;
  if (lane == 0) {
    slot = atomicAdd(cand_count, 1u);
    Cand cd;
    cd.score = L.score;
    cd.qid = q;
    cd.len = nc;
    cands[slot] = cd;
    atomicAdd(&ctr[q].offered, 1ull);
  }
  slot = __shfl(slot, 0, 64);
  for (uint32_t t = lane; t < nc; t += 64) cand_ids[(u64)slot * lmax + t] = s_sorted[t];
}

// ------------------------------------------------------------------
// top-k merge (Algorithm 1, lines 6-10) under the total order
// (score descending, then ascending id list lexicographically)
// ------------------------------------------------------------------
__device__ inline bool before(long long sa, const uint32_t *a, uint32_t la, long long sb,
                              const uint32_t *b, uint32_t lb) {
  if (sa != sb) return sa > sb;
  uint32_t n = la < lb ? la : lb;
  for (uint32_t i = 0; i < n; ++i)
    if (a[i] != b[i]) return a[i] < b[i];
  return la < lb;
}

__global__ void __launch_bounds__(1024)
    k_merge(const Cand *cands, const unsigned int *cand_count, const uint32_t *cand_ids,
            uint32_t lmax, QRes *res, const uint32_t *ks) {
  __shared__ uint32_t s_idx[kCandChunk];
  __shared__ unsigned int s_n;
  const uint32_t q = blockIdx.x;
  if (threadIdx.x == 0) s_n = 0;
  __syncthreads();
  const uint32_t nc_all = *cand_count;
  for (uint32_t i = threadIdx.x; i < nc_all; i += blockDim.x)
    if (cands[i].qid == q) s_idx[atomicAdd(&s_n, 1u)] = i;
  __syncthreads();
  const uint32_t nc = s_n;
  if (nc == 0) return;
  QRes R = res[q];
  const uint32_t k = ks[q];
  const uint32_t cur = R.cur, alt = cur ^ 1u;
  const uint32_t N = R.tk_n + nc;
  for (uint32_t i = threadIdx.x; i < N; i += blockDim.x) {
    long long si;
    const uint32_t *ai;
    uint32_t li;
    if (i < R.tk_n) {
      si = R.tk_score[cur][i];
      ai = R.tk_ids[cur] + (u64)i * lmax;
      li = R.tk_len[cur][i];
    } else {
      uint32_t c = s_idx[i - R.tk_n];
      si = cands[c].score;
      ai = cand_ids + (u64)c * lmax;
      li = cands[c].len;
    }
    uint32_t rank = 0;
    for (uint32_t j = 0; j < N && rank < k; ++j) {
      if (j == i) continue;
      long long sj;
      const uint32_t *aj;
      uint32_t lj;
      if (j < R.tk_n) {
        sj = R.tk_score[cur][j];
        aj = R.tk_ids[cur] + (u64)j * lmax;
        lj = R.tk_len[cur][j];
      } else {
        uint32_t c = s_idx[j - R.tk_n];
        sj = cands[c].score;
        aj = cand_ids + (u64)c * lmax;
        lj = cands[c].len;
      }
      rank += before(sj, aj, lj, si, ai, li);
    }
    if (rank < k) {
      R.tk_score[alt][rank] = si;
      R.tk_len[alt][rank] = li;
      uint32_t *dst = R.tk_ids[alt] + (u64)rank * lmax;
      for (uint32_t t = 0; t < li; ++t) dst[t] = ai[t];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t nn = N < k ? N : k;
    res[q].tk_n = nn;
    res[q].cur = alt;
    res[q].theta = nn == k ? R.tk_score[alt][k - 1] : LLONG_MIN;
  }
}

// ------------------------------------------------------------------
// host side
// ------------------------------------------------------------------
struct Level {
  uint32_t begin = 0, count = 0;
  u64 wbegin = 0, wend = 0;
  u64 cost_children = 0, cost_words = 0;
  long long max_bound = LLONG_MIN;
};

struct QHost {
  uint32_t k = 1;
  int kind = 0;  // 0 size, 1 vertex weight
  std::vector<Level> stack;
  uint64_t cursor = 0;
  long long theta = LLONG_MIN;
  bool done = false;
  uint32_t hdr_cap = 0;
  u64 word_cap = 0;
  // this step
  int plan = 0;  // 0 idle, 1 roots, 2 level
  uint32_t new_begin = 0;
  u64 new_wbegin = 0;
  int sel_seg = -1;
};

struct Engine {
  Graph &g;
  const QueryOpts &o;
  hipStream_t s;
  uint32_t nq;
  uint32_t lmax;
  std::vector<QHost> qh;

  DevBuf<CRec> hdr;
  DevBuf<u64> words;
  DevBuf<QCfg> d_cfg;
  DevBuf<QCtr> d_ctr;
  DevBuf<QRes> d_res;
  DevBuf<uint32_t> d_k;
  DevBuf<long long> tk_score;
  DevBuf<unsigned int> tk_len, tk_ids;
  DevBuf<CRec> batch, temp;
  DevBuf<unsigned int> counters;  // [0] batch, [1] leaf, [2] cand
  DevBuf<u64> leaf_word_count;
  DevBuf<LRec> leaves;
  DevBuf<u64> leaf_words;
  DevBuf<Cand> cands;
  DevBuf<uint32_t> cand_ids;
  DevBuf<SelSeg> d_seg;
  DevBuf<RootSeg> d_rseg;
  DevBuf<uint32_t> d_blk_seg, d_blk_off;
  DevBuf<unsigned int> d_hist, d_taken, d_tempc, d_quota;
  DevBuf<u64> d_hchild, d_hword, d_hmaxc, d_hmaxw;
  DevBuf<int> d_thr;
  std::vector<QCfg> h_cfg;
  std::vector<QCtr> h_ctr;
  std::vector<QRes> h_res;
  uint32_t batch_cap = 0, leaf_cap = 0;
  u64 leaf_word_cap = 0;
  uint32_t B = 0, root_B = 0;
  u64 step_children = 0, step_words = 0;
  uint64_t steps = 0, launches = 0, expand_ns = 0, peak_bytes = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;

  Engine(Graph &g_, const QueryOpts &o_) : g(g_), o(o_), s(o_.stream ? o_.stream : g_.stream) {}
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
    v.bm = (const u64 *)g.bm.p;
    v.wloc = g.wloc.p;
    v.vw = g.vw.p;
    v.wplus = g.wplus.p;
    v.root_order[0] = g.root_order[0].p;
    v.root_order[1] = g.root_order[1].p;
    return v;
  }

  void setup(const std::vector<uint32_t> &ks, const std::vector<int> &kinds) {
    nq = (uint32_t)ks.size();
    lmax = g.degeneracy + 1;
    qh.resize(nq);
    // frontier budget: a third for headers, the rest for bitmap words,
    // split evenly between the queries
    u64 budget = o.frontier_budget;
    u64 per_q = budget / nq;
    u64 hdr_per_q = std::max<u64>(1024, per_q / 3 / sizeof(CRec));
    u64 word_per_q = std::max<u64>(4096, (per_q - hdr_per_q * sizeof(CRec)) / 8);
    hdr_per_q = std::min<u64>(hdr_per_q, 0x7FFFFFFFull);
    hdr.alloc(hdr_per_q * nq);
    words.alloc(word_per_q * nq);
    h_cfg.resize(nq);
    h_ctr.assign(nq, QCtr{});
    h_res.resize(nq);
    u64 tk_total = 0;
    for (uint32_t i = 0; i < nq; ++i) tk_total += ks[i];
    tk_score.alloc(2 * tk_total);
    tk_len.alloc(2 * tk_total);
    tk_ids.alloc(2 * tk_total * lmax);
    u64 tko = 0;
    for (uint32_t i = 0; i < nq; ++i) {
      QHost &Q = qh[i];
      Q.k = ks[i];
      Q.kind = kinds[i];
      Q.hdr_cap = (uint32_t)hdr_per_q;
      Q.word_cap = word_per_q;
      QCfg &c = h_cfg[i];
      c.hdr = hdr.p + (u64)i * hdr_per_q;
      c.words = words.p + (u64)i * word_per_q;
      c.out_word = 0;
      c.word_cap = word_per_q;
      c.out_hdr = 0;
      c.hdr_cap = (uint32_t)hdr_per_q;
      c.weighted = kinds[i];
      c.k = ks[i];
      QRes &R = h_res[i];
      R.theta = LLONG_MIN;
      R.tk_n = 0;
      R.cur = 0;
      for (int b = 0; b < 2; ++b) {
        R.tk_score[b] = tk_score.p + 2 * tko + (u64)b * ks[i];
        R.tk_len[b] = tk_len.p + 2 * tko + (u64)b * ks[i];
        R.tk_ids[b] = tk_ids.p + (2 * tko + (u64)b * ks[i]) * lmax;
      }
      tko += ks[i];
    }
    d_cfg.alloc(nq);
    d_ctr.alloc(nq);
    d_res.alloc(nq);
    d_k.alloc(nq);
    NURI_HIP(hipMemcpyAsync(d_res.p, h_res.data(), nq * sizeof(QRes), hipMemcpyHostToDevice, s));
    NURI_HIP(hipMemcpyAsync(d_k.p, ks.data(), nq * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    NURI_HIP(hipMemsetAsync(d_ctr.p, 0, nq * sizeof(QCtr), s));
    // per-step limits
    B = o.batch_B ? o.batch_B : 16384;
    root_B = o.root_batch ? o.root_batch : 8192;
    step_words = std::max<u64>(1ull << 20, std::min<u64>(budget / 16 / 8, 64ull << 20));
    step_children = std::max<u64>(1ull << 16, std::min<u64>(step_words, 32ull << 20));
    batch_cap = (uint32_t)std::min<u64>((u64)nq * std::max(B, root_B), 1u << 26);
    batch.alloc(batch_cap);
    leaf_cap = (uint32_t)step_children;
    leaf_word_cap = step_words;
    leaves.alloc(leaf_cap);
    leaf_words.alloc(leaf_word_cap);
    counters.alloc(4);
    leaf_word_count.alloc(1);
    cands.alloc(kCandChunk);
    cand_ids.alloc((u64)kCandChunk * lmax);
    d_seg.alloc(nq);
    d_rseg.alloc(nq);
    d_hist.alloc((u64)nq * kBins);
    d_hchild.alloc((u64)nq * kBins);
    d_hword.alloc((u64)nq * kBins);
    d_hmaxc.alloc((u64)nq * kBins);
    d_hmaxw.alloc((u64)nq * kBins);
    d_thr.alloc(nq);
    d_quota.alloc(nq);
    d_taken.alloc(nq);
    d_tempc.alloc(nq);
    if (o.profile) {
      NURI_HIP(hipEventCreate(&ev0));
      NURI_HIP(hipEventCreate(&ev1));
    }
  }

  // largest possible output of one record: d * (header + W words)
  u64 max_rec_children() const { return g.degeneracy; }
  u64 max_rec_words() const { return (u64)g.degeneracy * 2 * ((g.degeneracy + 63) / 64); }

  // plan this step for every live query; returns false if nothing to do
  bool plan(std::vector<SelSeg> &segs, std::vector<RootSeg> &rsegs, uint32_t &batch_ub,
            u64 &temp_need) {
    segs.clear();
    rsegs.clear();
    batch_ub = 0;
    temp_need = 0;
    u64 left_c = step_children, left_w = step_words;
    bool any = false;
    for (uint32_t i = 0; i < nq; ++i) {
      QHost &Q = qh[i];
      Q.plan = 0;
      Q.sel_seg = -1;
      if (Q.done) continue;
      while (!Q.stack.empty() && Q.stack.back().count == 0) Q.stack.pop_back();
      if (Q.stack.empty()) {
        // unit subgraphs: the next roots in bound order with bound >= theta
        const auto &rb = g.h_root_bound[Q.kind];
        const auto &ro = g.h_root_order[Q.kind];
        u64 end = g.n;
        if (Q.theta != LLONG_MIN) {
          // first position with bound < theta (bounds are non-increasing)
          end = std::lower_bound(rb.begin(), rb.end(), Q.theta,
                                 [](long long a, long long t) { return a >= t; }) -
                rb.begin();
        }
        if (Q.cursor >= end) {
          Q.done = true;
          continue;
        }
        u64 cc = 0, cw = 0, cnt = 0;
        u64 lim_c = std::min<u64>(left_c, Q.hdr_cap), lim_w = std::min<u64>(left_w, Q.word_cap);
        while (Q.cursor + cnt < end && cnt < root_B && batch_ub + cnt < batch_cap) {
          uint32_t r = ro[Q.cursor + cnt];
          u64 d = g.h_dplus[r];
          u64 w = d * 2 * ((d + 63) / 64);
          if (cnt > 0 && (cc + d > lim_c || cw + w > lim_w)) break;
          cc += d;
          cw += w;
          ++cnt;
        }
        if (cc > lim_c || cw > lim_w)
          throw Error{NURI_EBUDGET, "frontier budget too small for one unit subgraph"};
        if (cnt == 0) continue;
        RootSeg rs;
        rs.qid = i;
        rs.kind = Q.kind;
        rs.first = (uint32_t)Q.cursor;
        rs.count = (uint32_t)cnt;
        rsegs.push_back(rs);
        Q.cursor += cnt;
        Q.plan = 1;
        Q.new_begin = 0;
        Q.new_wbegin = 0;
        batch_ub += (uint32_t)cnt;
        left_c -= cc;
        left_w -= cw;
        any = true;
        continue;
      }
      Level &L = Q.stack.back();
      u64 free_h = Q.hdr_cap - (u64)(L.begin + L.count);
      u64 free_w = Q.word_cap - L.wend;
      u64 lim_c = std::min<u64>(left_c, free_h), lim_w = std::min<u64>(left_w, free_w);
      if (lim_c < max_rec_children() || lim_w < max_rec_words()) {
        if (left_c < step_children || left_w < step_words) continue;  // retry next step
        throw Error{NURI_EBUDGET, "frontier budget exhausted"};
      }
      uint32_t room = batch_cap - batch_ub;
      if (room == 0) continue;
      SelSeg sg{};
      sg.qid = i;
      sg.begin = L.begin;
      sg.count = L.count;
      sg.max_records = std::min<u64>(B, room);
      sg.max_children = lim_c;
      sg.max_words = lim_w;
      sg.take_all = L.count <= sg.max_records && L.cost_children <= lim_c && L.cost_words <= lim_w;
      sg.top = L.max_bound;
      long long floor_b = Q.theta == LLONG_MIN ? 0 : Q.theta;
      long long span = L.max_bound - floor_b;
      uint32_t shift = 0;
      while (span > 0 && (span >> shift) >= kBins - 1) ++shift;
      sg.shift = shift;
      sg.temp_off = (uint32_t)temp_need;
      if (!sg.take_all) temp_need += L.count;
      Q.sel_seg = (int)segs.size();
      segs.push_back(sg);
      Q.plan = 2;
      Q.new_begin = L.begin + L.count;
      Q.new_wbegin = L.wend;
      u64 take = sg.take_all ? L.count : sg.max_records;
      batch_ub += (uint32_t)take;
      u64 uc = sg.take_all ? L.cost_children : lim_c;
      u64 uw = sg.take_all ? L.cost_words : lim_w;
      left_c -= std::min(left_c, uc);
      left_w -= std::min(left_w, uw);
      any = true;
    }
    return any;
  }

  void step(const std::vector<SelSeg> &segs, const std::vector<RootSeg> &rsegs, uint32_t batch_ub,
            u64 temp_need) {
    GView gv = view();
    for (uint32_t i = 0; i < nq; ++i) {
      h_cfg[i].out_hdr = qh[i].new_begin;
      h_cfg[i].out_word = qh[i].new_wbegin;
    }
    NURI_HIP(hipMemcpyAsync(d_cfg.p, h_cfg.data(), nq * sizeof(QCfg), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_reset_step, dim3((nq + 255) / 256), dim3(256), 0, s, d_ctr.p, nq);
    NURI_HIP(hipGetLastError());
    NURI_HIP(hipMemsetAsync(counters.p, 0, 4 * sizeof(unsigned int), s));
    NURI_HIP(hipMemsetAsync(leaf_word_count.p, 0, sizeof(u64), s));
    if (!rsegs.empty()) {
      NURI_HIP(hipMemcpyAsync(d_rseg.p, rsegs.data(), rsegs.size() * sizeof(RootSeg),
                              hipMemcpyHostToDevice, s));
      uint32_t mx = 0;
      for (auto &r : rsegs) mx = std::max(mx, r.count);
      uint32_t blocks = std::min<uint32_t>((mx + 255) / 256, 4096);
      hipLaunchKernelGGL(k_make_roots, dim3(std::max(1u, blocks)), dim3(256), 0, s, gv,
                         d_rseg.p, (uint32_t)rsegs.size(), batch.p, counters.p);
      NURI_HIP(hipGetLastError());
    }
    if (!segs.empty()) {
      uint32_t ns = (uint32_t)segs.size();
      NURI_HIP(hipMemcpyAsync(d_seg.p, segs.data(), ns * sizeof(SelSeg), hipMemcpyHostToDevice, s));
      std::vector<uint32_t> bs, bo;
      bool any_sel = false;
      for (uint32_t i = 0; i < ns; ++i) {
        for (uint32_t off = 0; off < segs[i].count; off += 256) {
          bs.push_back(i);
          bo.push_back(off);
        }
        any_sel |= !segs[i].take_all;
      }
      if (d_blk_seg.n < bs.size()) {
        d_blk_seg.alloc(bs.size() * 2);
        d_blk_off.alloc(bs.size() * 2);
      }
      NURI_HIP(hipMemcpyAsync(d_blk_seg.p, bs.data(), bs.size() * 4, hipMemcpyHostToDevice, s));
      NURI_HIP(hipMemcpyAsync(d_blk_off.p, bo.data(), bo.size() * 4, hipMemcpyHostToDevice, s));
      if (temp_need && temp.n < temp_need) temp.alloc(temp_need * 2);
      NURI_HIP(hipMemsetAsync(d_taken.p, 0, ns * 4, s));
      NURI_HIP(hipMemsetAsync(d_tempc.p, 0, ns * 4, s));
      if (any_sel) {
        NURI_HIP(hipMemsetAsync(d_hist.p, 0, (u64)ns * kBins * 4, s));
        NURI_HIP(hipMemsetAsync(d_hchild.p, 0, (u64)ns * kBins * 8, s));
        NURI_HIP(hipMemsetAsync(d_hword.p, 0, (u64)ns * kBins * 8, s));
        NURI_HIP(hipMemsetAsync(d_hmaxc.p, 0, (u64)ns * kBins * 8, s));
        NURI_HIP(hipMemsetAsync(d_hmaxw.p, 0, (u64)ns * kBins * 8, s));
        hipLaunchKernelGGL(k_sel_hist, dim3((uint32_t)bs.size()), dim3(256), 0, s, gv, d_seg.p,
                           d_blk_seg.p, d_blk_off.p, d_cfg.p, d_res.p, d_hist.p, d_hchild.p,
                           d_hword.p, d_hmaxc.p, d_hmaxw.p);
        NURI_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_sel_thresh, dim3(ns), dim3(64), 0, s, d_seg.p, ns, d_hist.p,
                           d_hchild.p, d_hword.p, d_hmaxc.p, d_hmaxw.p, d_thr.p, d_quota.p);
        NURI_HIP(hipGetLastError());
      }
      hipLaunchKernelGGL(k_sel_part, dim3((uint32_t)bs.size()), dim3(256), 0, s, gv, d_seg.p,
                         d_blk_seg.p, d_blk_off.p, d_cfg.p, d_res.p, d_thr.p, d_quota.p,
                         d_taken.p, batch.p, counters.p, temp.p, d_tempc.p, d_ctr.p);
      NURI_HIP(hipGetLastError());
      hipLaunchKernelGGL(k_copy_back, dim3(1024), dim3(256), 0, s, d_seg.p, ns, d_cfg.p, temp.p,
                         d_tempc.p, d_ctr.p);
      NURI_HIP(hipGetLastError());
    }
    if (batch_ub) {
      if (o.profile) NURI_HIP(hipEventRecord(ev0, s));
      uint32_t blocks = (batch_ub + kExpandWaves - 1) / kExpandWaves;
      hipLaunchKernelGGL(k_expand, dim3(blocks), dim3(64 * kExpandWaves), 0, s, gv, batch.p,
                         counters.p, d_cfg.p, d_ctr.p, d_res.p, leaves.p, counters.p + 1,
                         leaf_words.p, leaf_word_count.p, leaf_cap, leaf_word_cap);
      NURI_HIP(hipGetLastError());
      if (o.profile) NURI_HIP(hipEventRecord(ev1, s));
      launches++;
    }
    unsigned int hc[4];
    NURI_HIP(hipMemcpyAsync(h_ctr.data(), d_ctr.p, nq * sizeof(QCtr), hipMemcpyDeviceToHost, s));
    NURI_HIP(hipMemcpyAsync(hc, counters.p, sizeof(hc), hipMemcpyDeviceToHost, s));
    NURI_HIP(hipStreamSynchronize(s));
    if (o.profile && batch_ub) {
      float ms = 0;
      NURI_HIP(hipEventElapsedTime(&ms, ev0, ev1));
      expand_ns += (uint64_t)(ms * 1e6);
    }
    steps++;
    // update the level stacks
    u64 live = 0;
    for (uint32_t i = 0; i < nq; ++i) {
      QHost &Q = qh[i];
      const QCtr &c = h_ctr[i];
      if (c.overflow)
        throw Error{NURI_EBUDGET, "frontier overflow (internal accounting error)"};
      if (Q.plan == 2) {
        Level &L = Q.stack.back();
        const SelSeg &sg = segs[Q.sel_seg];
        if (sg.take_all) {
          L.count = 0;
        } else {
          L.count = c.n_kept;
        }
      }
      if (Q.plan && c.n_out) {
        Level N;
        N.begin = Q.new_begin;
        N.count = c.n_out;
        N.wbegin = Q.new_wbegin;
        N.wend = Q.new_wbegin + c.out_words;
        N.cost_children = c.out_cost_children;
        N.cost_words = c.out_cost_words;
        N.max_bound = c.out_max_bound;
        Q.stack.push_back(N);
      }
      if (!Q.stack.empty()) {
        const Level &T = Q.stack.back();
        live += (u64)(T.begin + T.count) * sizeof(CRec) + T.wend * 8;
      }
    }
    peak_bytes = std::max<uint64_t>(peak_bytes, live);
    // leaves -> maximality check -> merge, in chunks
    uint32_t nleaf = hc[1];
    if (nleaf > leaf_cap) throw Error{NURI_EBUDGET, "leaf buffer overflow (internal)"};
    for (uint32_t f = 0; f < nleaf; f += kCandChunk) {
      uint32_t cnt = std::min<uint32_t>(kCandChunk, nleaf - f);
      NURI_HIP(hipMemsetAsync(counters.p + 2, 0, sizeof(unsigned int), s));
      hipLaunchKernelGGL(k_leaf_check, dim3(cnt), dim3(64), 0, s, gv, leaves.p, f,
                         leaf_words.p, d_res.p, cands.p, counters.p + 2, cand_ids.p, lmax,
                         d_ctr.p);
      NURI_HIP(hipGetLastError());
      hipLaunchKernelGGL(k_merge, dim3(nq), dim3(1024), 0, s, cands.p, counters.p + 2,
                         cand_ids.p, lmax, d_res.p, d_k.p);
      NURI_HIP(hipGetLastError());
    }
    if (nleaf) {
      NURI_HIP(hipMemcpyAsync(h_res.data(), d_res.p, nq * sizeof(QRes), hipMemcpyDeviceToHost, s));
      NURI_HIP(hipStreamSynchronize(s));
      for (uint32_t i = 0; i < nq; ++i) qh[i].theta = h_res[i].theta;
    }
  }

  void run() {
    std::vector<SelSeg> segs;
    std::vector<RootSeg> rsegs;
    uint32_t batch_ub;
    u64 temp_need;
    uint64_t t0 = now_ns();
    while (plan(segs, rsegs, batch_ub, temp_need)) {
      if (o.deadline_ns && now_ns() - t0 > o.deadline_ns)
        throw Error{NURI_ETIMEOUT, "query deadline passed"};
      step(segs, rsegs, batch_ub, temp_need);
    }
  }

  void collect(std::vector<Result> &out, uint64_t wall) {
    NURI_HIP(hipMemcpyAsync(h_res.data(), d_res.p, nq * sizeof(QRes), hipMemcpyDeviceToHost, s));
    NURI_HIP(hipMemcpyAsync(h_ctr.data(), d_ctr.p, nq * sizeof(QCtr), hipMemcpyDeviceToHost, s));
    NURI_HIP(hipStreamSynchronize(s));
    out.resize(nq);
    for (uint32_t i = 0; i < nq; ++i) {
      const QRes &R = h_res[i];
      Result &res = out[i];
      uint32_t n = R.tk_n;
      std::vector<long long> sc(n);
      std::vector<unsigned int> ln(n), ids((u64)n * lmax);
      if (n) {
        NURI_HIP(hipMemcpyAsync(sc.data(), R.tk_score[R.cur], n * 8, hipMemcpyDeviceToHost, s));
        NURI_HIP(hipMemcpyAsync(ln.data(), R.tk_len[R.cur], n * 4, hipMemcpyDeviceToHost, s));
        NURI_HIP(hipMemcpyAsync(ids.data(), R.tk_ids[R.cur], (u64)n * lmax * 4,
                                hipMemcpyDeviceToHost, s));
        NURI_HIP(hipStreamSynchronize(s));
      }
      res.score.assign(sc.begin(), sc.end());
      res.offset.assign(1, 0);
      res.ids.clear();
      for (uint32_t t = 0; t < n; ++t) {
        res.ids.insert(res.ids.end(), ids.begin() + (u64)t * lmax,
                       ids.begin() + (u64)t * lmax + ln[t]);
        res.offset.push_back(res.ids.size());
      }
      const QCtr &c = h_ctr[i];
      nuri_stats &st = res.stats;
      memset(&st, 0, sizeof(st));
      st.steps = steps;
      st.popped = c.popped;
      st.expanded = c.expanded;
      st.children = c.children;
      st.pruned_at_pop = c.pruned_pop;
      st.pruned_at_creation = c.pruned_new;
      st.leaves = c.leaves;
      st.offered = c.offered;
      st.frontier_peak_bytes = peak_bytes;
      st.logical_bytes = c.logical_bytes;
      st.expand_launches = launches;
      st.expand_ns = expand_ns;
      st.wall_ns = wall;
    }
  }
};

}  // namespace

void run_cliques(Graph &g, const std::vector<uint32_t> &ks, const std::vector<int> &kinds,
                 const QueryOpts &o, std::vector<Result> &out) {
  uint64_t t0 = now_ns();
  if (ks.size() > 65535) throw Error{NURI_EINVAL, "at most 65535 queries per batch"};
  for (size_t i = 0; i < ks.size(); ++i) {
    if (ks[i] == 0) throw Error{NURI_EINVAL, "k must be >= 1"};
    if (kinds[i] != 0 && kinds[i] != 1) throw Error{NURI_EINVAL, "unknown weight_fn"};
    if (kinds[i] == 1 && !g.has_vw)
      throw Error{NURI_EINVAL, "NURI_SCORE_VERTEX_WEIGHT needs vertex weights"};
  }
  Engine e(g, o);
  e.setup(ks, kinds);
  e.run();
  e.collect(out, now_ns() - t0);
}

}  // namespace nuri
