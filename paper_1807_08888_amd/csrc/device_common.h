// Device-side pieces shared by the clique and matching engines: wavefront
// helpers, the per-step counters, the result-set state and the top-k merge
// (Algorithm 1, lines 6-10) under the total order of results.
#pragma once

#include <climits>

#include "nuri_internal.h"

namespace nuri {
namespace {

typedef unsigned long long u64;

struct Cand {  // a result offered to the result set (its ids are stored apart)
  long long score;
  uint32_t qid;
  uint32_t len;
};

struct StepHdr {  // global counters of one step (zeroed by the step upload)
  unsigned int batch_count, leaf_count, cand_count, pad;
  u64 leaf_word_count;
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

// Ranks are computed against the current top-k plus this chunk's
// candidates of the query (all-pairs comparison, one thread per item,
// grid (x, query)); items ranked below k are written to the other top-k
// buffer at their rank, so the order of candidates in the buffer never
// matters.
__global__ void __launch_bounds__(256)
    k_merge_rank(const Cand *cands, const StepHdr *hdr, const uint32_t *cand_ids, uint32_t lmax,
                 const QRes *res, const uint32_t *ks) {
  __shared__ uint32_t s_idx[kCandChunk];
  __shared__ uint32_t s_cnt[256];
  __shared__ uint32_t s_nc;
  constexpr uint32_t per = kCandChunk / 256;
  const uint32_t q = blockIdx.y;
  const uint32_t nc_all = hdr->cand_count;
  const uint32_t b0 = threadIdx.x * per;
  uint32_t mine = 0;
  for (uint32_t i = b0; i < b0 + per && i < nc_all; ++i) mine += cands[i].qid == q;
  s_cnt[threadIdx.x] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int t = 0; t < 256; ++t) {
      uint32_t c = s_cnt[t];
      s_cnt[t] = run;
      run += c;
    }
    s_nc = run;
  }
  __syncthreads();
  uint32_t o = s_cnt[threadIdx.x];
  for (uint32_t i = b0; i < b0 + per && i < nc_all; ++i)
    if (cands[i].qid == q) s_idx[o++] = i;
  __syncthreads();
  const uint32_t nc = s_nc;
  if (nc == 0) return;
  const QRes R = res[q];
  const uint32_t k = ks[q];
  const uint32_t cur = R.cur, alt = cur ^ 1u;
  const uint32_t N = R.tk_n + nc;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
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

// one block per query: switch to the merged buffer and set the threshold
__global__ void __launch_bounds__(256)
    k_merge_finish(const Cand *cands, const StepHdr *hdr, QRes *res, const uint32_t *ks) {
  __shared__ uint32_t s_n;
  const uint32_t q = blockIdx.x;
  if (threadIdx.x == 0) s_n = 0;
  __syncthreads();
  const uint32_t nc_all = hdr->cand_count;
  uint32_t mine = 0;
  for (uint32_t i = threadIdx.x; i < nc_all; i += blockDim.x) mine += cands[i].qid == q;
  if (mine) atomicAdd(&s_n, mine);
  __syncthreads();
  if (threadIdx.x != 0 || s_n == 0) return;
  QRes &R = res[q];
  const uint32_t k = ks[q];
  const uint32_t N = R.tk_n + s_n;
  const uint32_t nn = N < k ? N : k;
  const uint32_t alt = R.cur ^ 1u;
  R.tk_n = nn;
  R.cur = alt;
  R.theta = nn == k ? R.tk_score[alt][k - 1] : LLONG_MIN;
}

// page-locked host staging buffer
template <class T>
struct PinBuf {
  T *p = nullptr;
  size_t n = 0;
  PinBuf() = default;
  PinBuf(const PinBuf &) = delete;
  PinBuf &operator=(const PinBuf &) = delete;
  ~PinBuf() {
    if (p) (void)hipHostFree(p);
  }
  void alloc(size_t count) {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    NURI_HIP(hipHostMalloc((void **)&p, count * sizeof(T), 0));
    n = count;
  }
};

}  // namespace
}  // namespace nuri
