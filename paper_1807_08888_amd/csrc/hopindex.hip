// The multi-hop (label, hop) max-degree index of Section 4.3 (Listing 3),
// built on the GPU for the degree score of labelled matching.
//
//   entry (h, v, l) = the largest degree of a vertex with label l whose
//                     distance from v is 1..h; 0 when there is none.
//
// The index is cumulative over hops: the image of a pattern vertex h hops
// from the seed's pattern vertex can lie nearer than h to the seed, so only
// the cumulative entry bounds it.  The paper computes the entries vertex by
// vertex on the CPU and notes that the vertices are independent.
//
// Here each hop is one gather over the adjacency.  The vertices that walks
// of 1..h edges reach from v are its ball of radius h, minus v for h = 1
// and plus v itself for h >= 2 (v -> w -> v).  That set is N(v) together
// with the hop-(h-1) sets of v's neighbours.  To leave v out, every
// (vertex, label) carries its two best distinct vertices, keyed by degree
// and then by the smaller id: the two best of a union are among the two
// best of each part, and the entry is the better of v's two that is not v.
//
// Threads: 16 lanes per vertex, lane l for label l, so the 16 states of a
// neighbour (256 bytes) are read in one coalesced access.  Vertices of
// degree above kSmallDeg are cut into chunks of kChunk neighbours, one
// 256-thread block each (16 lane groups striding the chunk), and their
// partial states are merged by a third kernel.
#include <algorithm>
#include <chrono>

#include "device_common.h"

namespace nuri {
namespace {

constexpr uint32_t kL = NURI_MAX_LABELS;  // 16 labels, one lane each
constexpr uint32_t kSmallDeg = 1024;
constexpr uint32_t kChunk = 4096;

struct Top2 {
  u64 a, b;  // best, second best; 0 = empty
};

// key of vertex w: its degree, then the smaller id first
__device__ inline u64 vkey(const uint64_t *orow, uint32_t w) {
  return ((orow[w + 1] - orow[w]) << 32) | (u64)(0xFFFFFFFFu - w);
}

// fold key k into the pair (a > b): a key already there (the same vertex)
// or 0 changes nothing; written with selects so a and b stay in registers
__device__ inline void top2_add(u64 &a, u64 &b, u64 k) {
  const bool dup = (k == a) | (k == b);
  const u64 hi = k > a ? k : a;
  const u64 lo = k > a ? a : (k > b ? k : b);
  a = dup ? a : hi;
  b = dup ? b : lo;
}

// the entry of v: the better of its two that is not v itself
__device__ inline int32_t entry_of(u64 a, u64 b, uint32_t v) {
  const u64 k = ((uint32_t)a == 0xFFFFFFFFu - v) ? b : a;
  return (int32_t)(k >> 32);
}

// neighbours [j0, j1) of row v, stepping by `step`: lane l folds in every
// neighbour of label l and (hop >= 2) every neighbour's hop-(h-1) state
__device__ inline void fold(const uint64_t *orow, const uint32_t *lcol, const uint32_t *loff,
                            const Top2 *prev, uint32_t v, u64 j0, u64 j1, u64 step, uint32_t l,
                            u64 &a, u64 &b) {
  const u64 r0 = orow[v];
  const u64 sb = r0 + loff[(u64)v * 17 + l], se = r0 + loff[(u64)v * 17 + l + 1];
  for (u64 j = j0; j < j1; j += step) {
    const uint32_t w = lcol[j];
    if (j >= sb && j < se) top2_add(a, b, vkey(orow, w));
    if (prev) {
      const Top2 t = prev[(u64)w * kL + l];
      top2_add(a, b, t.a);
      top2_add(a, b, t.b);
    }
  }
}

// vertices of degree <= kSmallDeg: 16 lanes each
__global__ void __launch_bounds__(256)
    k_hop_small(const uint64_t *orow, const uint32_t *lcol, const uint32_t *loff, uint32_t n,
                const Top2 *prev, Top2 *next, int32_t *entry) {
  const uint32_t l = threadIdx.x & (kL - 1);
  for (u64 v = (blockIdx.x * (u64)blockDim.x + threadIdx.x) / kL; v < n;
       v += (u64)gridDim.x * blockDim.x / kL) {
    const u64 r0 = orow[v], r1 = orow[v + 1];
    if (r1 - r0 > kSmallDeg) continue;
    u64 a = 0, b = 0;
    fold(orow, lcol, loff, prev, (uint32_t)v, r0, r1, 1, l, a, b);
    next[v * kL + l] = Top2{a, b};
    entry[v * kL + l] = entry_of(a, b, (uint32_t)v);
  }
}

struct Piece {  // a chunk of a high-degree row
  uint32_t v, pad;
  u64 j0, j1;
};

// one 256-thread block per chunk: 16 groups of 16 lanes stride the chunk,
// then the 16 partial states per label are merged through LDS
__global__ void __launch_bounds__(256)
    k_hop_chunk(const uint64_t *orow, const uint32_t *lcol, const uint32_t *loff,
                const Piece *pieces, const Top2 *prev, Top2 *partial) {
  __shared__ u64 sa[16][kL], sb[16][kL];
  const Piece pc = pieces[blockIdx.x];
  const uint32_t l = threadIdx.x & (kL - 1), grp = threadIdx.x / kL;
  u64 a = 0, b = 0;
  fold(orow, lcol, loff, prev, pc.v, pc.j0 + grp, pc.j1, 16, l, a, b);
  sa[grp][l] = a;
  sb[grp][l] = b;
  __syncthreads();
  if (threadIdx.x < kL) {
    u64 x = 0, y = 0;
    for (int g2 = 0; g2 < 16; ++g2) {
      top2_add(x, y, sa[g2][threadIdx.x]);
      top2_add(x, y, sb[g2][threadIdx.x]);
    }
    partial[(u64)blockIdx.x * kL + threadIdx.x] = Top2{x, y};
  }
}

// merge the chunks of each high-degree row: 16 lanes per row
__global__ void __launch_bounds__(256)
    k_hop_merge(const uint32_t *big_v, const uint32_t *big_first, uint32_t nbig,
                const Top2 *partial, Top2 *next, int32_t *entry) {
  const uint32_t l = threadIdx.x & (kL - 1);
  const u64 i = (blockIdx.x * (u64)blockDim.x + threadIdx.x) / kL;
  if (i >= nbig) return;
  const uint32_t v = big_v[i];
  u64 a = 0, b = 0;
  for (uint32_t p = big_first[i]; p < big_first[i + 1]; ++p) {
    const Top2 t = partial[(u64)p * kL + l];
    top2_add(a, b, t.a);
    top2_add(a, b, t.b);
  }
  next[(u64)v * kL + l] = Top2{a, b};
  entry[(u64)v * kL + l] = entry_of(a, b, v);
}

}  // namespace

void ensure_hop_index(Graph &g, uint32_t hops, hipStream_t s) {
  if (hops > NURI_MAX_PATTERN - 1) throw Error{NURI_EINVAL, "hop index: too many hops"};
  std::lock_guard<std::mutex> lk(g.hidx_mu);
  if (g.hidx_hops >= hops) return;
  if (!g.has_lab) throw Error{NURI_EINVAL, "the degree score needs vertex labels"};
  const auto t0 = std::chrono::steady_clock::now();
  const uint32_t n = g.n;
  // rows above kSmallDeg, cut into chunks
  std::vector<uint64_t> row(n + 1);
  NURI_HIP(hipMemcpyAsync(row.data(), g.orow.p, (n + 1) * sizeof(uint64_t),
                          hipMemcpyDeviceToHost, s));
  NURI_HIP(hipStreamSynchronize(s));
  std::vector<Piece> pieces;
  std::vector<uint32_t> big_v, big_first;
  for (uint32_t v = 0; v < n; ++v) {
    const u64 d = row[v + 1] - row[v];
    if (d <= kSmallDeg) continue;
    big_v.push_back(v);
    big_first.push_back((uint32_t)pieces.size());
    for (u64 j = row[v]; j < row[v + 1]; j += kChunk)
      pieces.push_back(Piece{v, 0, j, std::min<u64>(j + kChunk, row[v + 1])});
  }
  big_first.push_back((uint32_t)pieces.size());
  DevBuf<Piece> d_pieces;
  DevBuf<uint32_t> d_big_v, d_big_first;
  DevBuf<Top2> partial, st0, st1;
  d_pieces.alloc(pieces.size());
  d_big_v.alloc(big_v.size());
  d_big_first.alloc(big_first.size());
  partial.alloc(pieces.size() * kL);
  st0.alloc((size_t)n * kL);
  st1.alloc((size_t)n * kL);
  if (!pieces.empty()) {
    NURI_HIP(hipMemcpyAsync(d_pieces.p, pieces.data(), pieces.size() * sizeof(Piece),
                            hipMemcpyHostToDevice, s));
    NURI_HIP(hipMemcpyAsync(d_big_v.p, big_v.data(), big_v.size() * 4, hipMemcpyHostToDevice, s));
  }
  NURI_HIP(hipMemcpyAsync(d_big_first.p, big_first.data(), big_first.size() * 4,
                          hipMemcpyHostToDevice, s));
  // hops already built are recomputed (their states are not kept) but not
  // rewritten: their entry arrays stay valid for queries running meanwhile
  Top2 *prev = nullptr, *next = st0.p;
  DevBuf<int32_t> scratch_entry;
  for (uint32_t h = 1; h <= hops; ++h) {
    int32_t *entry;
    if (h <= g.hidx_hops) {
      if (!scratch_entry.p) scratch_entry.alloc((size_t)n * kL);
      entry = scratch_entry.p;
    } else {
      g.hidx[h - 1].alloc((size_t)n * kL);
      entry = g.hidx[h - 1].p;
    }
    const uint32_t small_blocks =
        (uint32_t)std::min<u64>(((u64)n * kL + 255) / 256, 1u << 20);
    hipLaunchKernelGGL(k_hop_small, dim3(std::max(1u, small_blocks)), dim3(256), 0, s,
                       g.orow.p, g.lcol.p, g.loff.p, n, prev, next, entry);
    NURI_HIP(hipGetLastError());
    if (!pieces.empty()) {
      hipLaunchKernelGGL(k_hop_chunk, dim3((uint32_t)pieces.size()), dim3(256), 0, s, g.orow.p,
                         g.lcol.p, g.loff.p, d_pieces.p, prev, partial.p);
      NURI_HIP(hipGetLastError());
      const uint32_t mb = (uint32_t)(((u64)big_v.size() * kL + 255) / 256);
      hipLaunchKernelGGL(k_hop_merge, dim3(mb), dim3(256), 0, s, d_big_v.p, d_big_first.p,
                         (uint32_t)big_v.size(), partial.p, next, entry);
      NURI_HIP(hipGetLastError());
    }
    prev = next;
    next = (next == st0.p) ? st1.p : st0.p;
  }
  NURI_HIP(hipStreamSynchronize(s));
  g.hidx_hops = hops;
  g.hidx_ns += (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
                   std::chrono::steady_clock::now() - t0)
                   .count();
}

}  // namespace nuri
