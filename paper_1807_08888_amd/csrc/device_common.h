// Device-side pieces shared by the clique and matching engines: wavefront
// helpers, the per-step counters, the result-set state and the top-k merge
// (Algorithm 1, lines 6-10) under the total order of results.
#pragma once

#include <climits>
#include <new>

#include "nuri_internal.h"

namespace nuri {
namespace {

typedef unsigned long long u64;

struct Cand {  // a result offered to the result set (its ids are stored apart)
  long long score;
  uint32_t qid;
  uint32_t len;
};

// Global counters of one step (zeroed by the step upload).  The ones that
// every wavefront of an expansion launch reserves space with get a cache
// line each: atomics on one line are serialised.
struct StepHdr {
  alignas(128) unsigned int batch_count;
  unsigned int cand_count, big_next;
  alignas(128) unsigned int leaf_count;
  alignas(128) u64 leaf_word_count;
  alignas(128) u64 chain_c;     // leaf slots reserved by chained expansion (each with the widest row)
  alignas(128) u64 big_packed;  // matching: records with long candidate lists (high 32 bits)
                                // and their extra chunks (low 32 bits)
};

struct QRes {  // per query result state
  long long theta;  // score of the k-th result; LLONG_MIN while fewer than k results
  unsigned int tk_n, cur;
  long long *tk_score[2];
  unsigned int *tk_len[2];
  unsigned int *tk_ids[2];  // stride lmax
};

constexpr int kBins = 2048;
constexpr uint32_t kCandChunk = 2048;

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// lane l's 64-bit value, read by every lane (l wave-uniform)
__device__ inline u64 readlane64(u64 x, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), l);
  return ((u64)hi << 32) | lo;
}

// highest set position over a wave's words (lane l holds word l); the
// caller guarantees that some lane's word is non-zero.  The lane comes from
// a ballot and the word from a scalar read of that lane, so the result is
// wave-uniform without a shuffle reduction.
__device__ inline int wave_highest_bit(u64 x) {
  const u64 m = __ballot(x != 0);
  const int l = 63 - (int)__clzll(m);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), l);
  const u64 w = ((u64)hi << 32) | lo;
  return l * 64 + 63 - (int)__clzll(w);
}

// lowest set position over a wave's words (lane l holds word l), or -1
__device__ inline int wave_lowest_bit(u64 x) {
  const u64 m = __ballot(x != 0);
  if (!m) return -1;
  const int l = __ffsll((long long)m) - 1;
  return l * 64 + __ffsll((long long)readlane64(x, l)) - 1;
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

__device__ inline long long wave_excl_scan64(long long x, int lane) {
  long long inc = x;
  for (int off = 1; off < 64; off <<= 1) {
    long long t = __shfl_up(inc, off, 64);
    if (lane >= off) inc += t;
  }
  return inc - x;
}

__device__ inline u64 wave_max_u64(u64 x) {
  for (int off = 32; off > 0; off >>= 1) {
    u64 y = __shfl_xor(x, off, 64);
    x = y > x ? y : x;
  }
  return x;
}

__device__ inline uint32_t wave_min_u32(uint32_t x) {
  for (int off = 32; off > 0; off >>= 1) {
    uint32_t y = __shfl_xor(x, off, 64);
    x = y < x ? y : x;
  }
  return x;
}

__device__ inline int bin_of(long long bound, long long top, uint32_t shift) {
  long long gap = (top - bound) >> shift;
  long long b = kBins - 1 - gap;
  return b < 0 ? 0 : (b > kBins - 1 ? kBins - 1 : (int)b);
}

// ------------------------------------------------------------------
// selection threshold over a bound histogram (one 256-thread block per
// segment).  Bins are taken from the top while the records, the children
// they may create and those children's bitmap words all stay within the
// step's limits; the first bin (from the top) that would break a limit is
// the threshold bin t, of which only `quota` records are taken.  Running
// totals from the top are a suffix scan over the bins: each thread owns 8
// consecutive bins, the block scans the per-thread totals, and every thread
// tests its own bins.  A bin can only break a limit if it holds records
// (an empty bin adds nothing to the totals), so t is never empty.
// ------------------------------------------------------------------
constexpr int kSelThreads = 256;
constexpr int kBinsPerThread = kBins / kSelThreads;
static_assert(kBins % kSelThreads == 0, "bins are shared evenly by the threads");

struct SelLimits {
  u64 max_records, max_children, max_words;
  u64 wpc;    // bitmap words per child (0: no word limit)
  u64 maxcc;  // most children one record of the level can create
};

// hist/hchild: this segment's kBins counters (records, children) per bin.
// Writes (t, quota) from thread 0; every thread must call it.
__device__ inline void block_select_threshold(const unsigned int *hist, const u64 *hchild,
                                              const SelLimits lim, int *t_out,
                                              unsigned int *q_out) {
  __shared__ u64 s_n[kSelThreads], s_c[kSelThreads];
  __shared__ int s_t;
  const int tid = threadIdx.x;
  // this thread's bins: b0 .. b0 + 7; thread 0 holds the top bins
  const int b0 = kBins - (tid + 1) * kBinsPerThread;
  u64 hn[kBinsPerThread], hc[kBinsPerThread];
  u64 tn = 0, tc = 0;
  for (int i = 0; i < kBinsPerThread; ++i) {
    hn[i] = hist[b0 + i];
    hc[i] = hchild[b0 + i];
    tn += hn[i];
    tc += hc[i];
  }
  s_n[tid] = tn;
  s_c[tid] = tc;
  if (tid == 0) s_t = -1;
  __syncthreads();
  // inclusive scan over threads (Hillis-Steele in LDS)
  for (int off = 1; off < kSelThreads; off <<= 1) {
    const u64 an = tid >= off ? s_n[tid - off] : 0, ac = tid >= off ? s_c[tid - off] : 0;
    __syncthreads();
    s_n[tid] += an;
    s_c[tid] += ac;
    __syncthreads();
  }
  // totals of the bins above this thread's bins
  u64 n = s_n[tid] - tn, c = s_c[tid] - tc;
  auto fits = [&](u64 nn, u64 cc) {
    return nn <= lim.max_records && cc <= lim.max_children &&
           (lim.wpc == 0 || cc * lim.wpc <= lim.max_words);
  };
  int mine = -1;  // highest bin of this thread that breaks a limit
  u64 n_at = 0, c_at = 0;
  for (int i = kBinsPerThread - 1; i >= 0; --i) {
    if (hn[i] && !fits(n + hn[i], c + hc[i])) {
      mine = b0 + i;
      n_at = n;
      c_at = c;
      break;
    }
    n += hn[i];
    c += hc[i];
  }
  if (mine >= 0) atomicMax(&s_t, mine);
  __syncthreads();
  if (mine >= 0 && mine == s_t) {
    u64 qa = lim.max_records - n_at;
    const u64 mc = lim.maxcc ? (lim.max_children - c_at) / lim.maxcc : qa;
    const u64 mw = (lim.maxcc && lim.wpc) ? (lim.max_words - c_at * lim.wpc) / (lim.maxcc * lim.wpc)
                                          : qa;
    qa = qa < mc ? qa : mc;
    qa = qa < mw ? qa : mw;
    if (qa == 0 && n_at == 0) qa = 1;  // the host guarantees one record always fits
    const u64 h = hist[mine];
    *t_out = mine;
    *q_out = (unsigned int)(qa < h ? qa : h);
  } else if (tid == 0 && s_t < 0) {
    *t_out = -1;
    *q_out = 0;
  }
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

// The same order, decided by a whole wavefront: 64 ids are compared per
// load, so lists that share a long prefix (cliques of one dense region)
// cost a few wave steps instead of hundreds of serial loads.  Every lane
// returns the same value.
__device__ inline bool wave_before(long long sa, const uint32_t *a, uint32_t la, long long sb,
                                   const uint32_t *b, uint32_t lb, int lane) {
  if (sa != sb) return sa > sb;
  const uint32_t n = la < lb ? la : lb;
  for (uint32_t base = 0; base < n; base += 64) {
    const uint32_t i = base + lane;
    const bool diff = i < n && a[i] != b[i];
    const u64 m = __ballot(diff);
    if (m) {
      const uint32_t f = base + __ffsll((long long)m) - 1;
      return a[f] < b[f];
    }
  }
  return la < lb;
}

// The merge of one chunk of candidates into each query's top-k takes
// three launches.
//   k_merge_pos: one wave per candidate finds, by binary search, how many
//     current top-k items precede it.  A candidate preceded by k or more
//     can never enter (everything that will precede a member of the new
//     top-k precedes it too), so it is dropped; so is a candidate equal to
//     a top-k item (a result offered twice).  Survivors are appended to
//     their query's list (the order of a list does not matter).
//   k_merge_rank: one wave per item of (top-k, survivors) of a query
//     counts the survivors that precede it; with its position in the
//     top-k that is its rank in the union.  Items ranked below k are
//     written to the other top-k buffer at their rank.
//   k_merge_finish: switches to the merged buffer, sets the threshold and
//     empties the survivor list.
constexpr int kMergeWaves = 4;

// device buffers of the merge: position of each candidate of a chunk, and
// per query a survivor list (count zero between merges)
struct MergeBufs {
  PoolBuf<uint32_t> pos, list, count;
  void alloc(MemPool &pool, uint32_t nq, hipStream_t s) {
    pos.alloc(pool, kCandChunk);
    list.alloc(pool, (u64)nq * kCandChunk);
    count.alloc(pool, nq);
    NURI_HIP(hipMemsetAsync(count.p, 0, nq * sizeof(uint32_t), s));
  }
};

__global__ void __launch_bounds__(64 * kMergeWaves)
    k_merge_pos(const Cand *cands, const StepHdr *hdr, const uint32_t *cand_ids, uint32_t lmax,
                const QRes *res, const uint32_t *ks, uint32_t *pos, uint32_t *slist,
                uint32_t *scount) {
  const int lane = threadIdx.x & 63;
  const uint32_t c = blockIdx.x * kMergeWaves + (threadIdx.x >> 6);
  if (c >= hdr->cand_count) return;
  const Cand cd = cands[c];
  const QRes &R = res[cd.qid];
  const uint32_t cur = R.cur, n = R.tk_n;
  const uint32_t *ids = cand_ids + (u64)c * lmax;
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (wave_before(R.tk_score[cur][mid], R.tk_ids[cur] + (u64)mid * lmax, R.tk_len[cur][mid],
                    cd.score, ids, cd.len, lane))
      lo = mid + 1;
    else
      hi = mid;
  }
  // an item equal to the candidate (it was offered before) drops it
  const bool dup = lo < n && !wave_before(cd.score, ids, cd.len, R.tk_score[cur][lo],
                                          R.tk_ids[cur] + (u64)lo * lmax, R.tk_len[cur][lo], lane);
  if (lane == 0) {
    pos[c] = lo;
    if (lo < ks[cd.qid] && !dup)
      slist[(u64)cd.qid * kCandChunk + atomicAdd(&scount[cd.qid], 1u)] = c;
  }
}

__global__ void __launch_bounds__(64 * kMergeWaves)
    k_merge_rank(const Cand *cands, const uint32_t *cand_ids, uint32_t lmax, const QRes *res,
                 const uint32_t *ks, const uint32_t *pos, const uint32_t *slist,
                 const uint32_t *scount) {
  const uint32_t q = blockIdx.y;
  const uint32_t ns = scount[q];
  if (ns == 0) return;
  const uint32_t *sl = slist + (u64)q * kCandChunk;
  const int lane = threadIdx.x & 63;
  const QRes &R = res[q];
  const uint32_t k = ks[q];
  const uint32_t cur = R.cur, alt = cur ^ 1u;
  const uint32_t nt = R.tk_n < k ? R.tk_n : k;
  for (uint32_t it = blockIdx.x * kMergeWaves + (threadIdx.x >> 6); it < nt + ns;
       it += gridDim.x * kMergeWaves) {
    long long si;
    const uint32_t *ai;
    uint32_t li, rank;
    if (it < nt) {
      si = R.tk_score[cur][it];
      ai = R.tk_ids[cur] + (u64)it * lmax;
      li = R.tk_len[cur][it];
      rank = it;
    } else {
      const uint32_t c = sl[it - nt];
      si = cands[c].score;
      ai = cand_ids + (u64)c * lmax;
      li = cands[c].len;
      rank = pos[c];
    }
    // survivors that precede this item: scores decide 64 at a time, ties
    // are settled one by one by the whole wave
    for (uint32_t base = 0; base < ns && rank < k; base += 64) {
      const uint32_t j = base + lane;
      long long sj = 0;
      uint32_t cj = 0;
      if (j < ns) {
        cj = sl[j];
        sj = cands[cj].score;
      }
      const bool self = it >= nt && j == it - nt;
      rank += __popcll(__ballot(j < ns && !self && sj > si));
      u64 tie = __ballot(j < ns && !self && sj == si);
      while (tie) {
        const int t = __ffsll((long long)tie) - 1;
        tie &= tie - 1;
        const uint32_t ct = __shfl(cj, t, 64);
        rank += wave_before(si, cand_ids + (u64)ct * lmax, cands[ct].len, si, ai, li, lane);
      }
    }
    if (rank < k) {
      if (lane == 0) {
        R.tk_score[alt][rank] = si;
        R.tk_len[alt][rank] = li;
      }
      uint32_t *dst = R.tk_ids[alt] + (u64)rank * lmax;
      for (uint32_t t = lane; t < li; t += 64) dst[t] = ai[t];
    }
  }
}

// one thread per query: switch to the merged buffer and set the threshold
__global__ void k_merge_finish(QRes *res, const uint32_t *ks, uint32_t *scount, uint32_t nq) {
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  const uint32_t ns = scount[q];
  if (ns == 0) return;
  scount[q] = 0;
  QRes &R = res[q];
  const uint32_t k = ks[q];
  const uint32_t N = (R.tk_n < k ? R.tk_n : k) + ns;
  const uint32_t nn = N < k ? N : k;
  const uint32_t alt = R.cur ^ 1u;
  R.tk_n = nn;
  R.cur = alt;
  R.theta = nn == k ? R.tk_score[alt][k - 1] : LLONG_MIN;
}

// launch the three merge kernels for a chunk of at most `ub` candidates
// (the exact count is read on the device from hdr->cand_count)
inline void launch_merge(const Cand *cands, const StepHdr *hdr, const uint32_t *ids,
                         uint32_t lmax, QRes *res, const uint32_t *ks, MergeBufs &mb, uint32_t nq,
                         uint32_t kmax, uint32_t ub, hipStream_t s) {
  if (!ub) return;
  hipLaunchKernelGGL(k_merge_pos, dim3((ub + kMergeWaves - 1) / kMergeWaves),
                     dim3(64 * kMergeWaves), 0, s, cands, hdr, ids, lmax, res, ks, mb.pos.p,
                     mb.list.p, mb.count.p);
  NURI_HIP(hipGetLastError());
  // blocks per query: enough waves for the items, at most 32 blocks (each
  // wave then walks several items)
  const uint32_t items = kmax + std::min<uint32_t>(ub, kCandChunk);
  const uint32_t bx = std::min<uint32_t>((items + kMergeWaves - 1) / kMergeWaves, 32);
  hipLaunchKernelGGL(k_merge_rank, dim3(bx, nq), dim3(64 * kMergeWaves), 0, s, cands, ids, lmax,
                     res, ks, mb.pos.p, mb.list.p, mb.count.p);
  NURI_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_merge_finish, dim3((nq + 255) / 256), dim3(256), 0, s, res, ks, mb.count.p,
                     nq);
  NURI_HIP(hipGetLastError());
}

// host staging buffer: page-locked, or (pinned = false, for the
// allocation-free entry point) ordinary pageable host memory
template <class T>
struct PinBuf {
  // byte buffers hold structures with cache-line aligned members
  static constexpr size_t kAlign = alignof(T) > 128 ? alignof(T) : 128;
  T *p = nullptr;
  size_t n = 0;
  bool pinned = true;
  PinBuf() = default;
  PinBuf(const PinBuf &) = delete;
  PinBuf &operator=(const PinBuf &) = delete;
  ~PinBuf() { release(); }
  void release() {
    if (p) {
      if (pinned) (void)hipHostFree(p);
      else ::operator delete(p, std::align_val_t(kAlign));
    }
    p = nullptr;
  }
  void alloc(size_t count) {
    release();
    if (pinned) NURI_HIP(hipHostMalloc((void **)&p, count * sizeof(T), 0));
    else p = static_cast<T *>(::operator new(count * sizeof(T), std::align_val_t(kAlign)));
    n = count;
  }
};

}  // namespace
}  // namespace nuri
