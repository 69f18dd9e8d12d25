// Top-k frequent pattern mining on the GPU: the aggregate computation of
// Section 3.3 (Algorithm 2) with the pattern-mining user functions of
// Sections 3.3 and 4.2 (Listing 2):
//
//   key(s)        the pattern of subgraph s, as its minimum DFS code
//                 (pattern-oriented expansion);
//   relevant(S)   the pattern has exactly M edges;
//   priority(S)   (edges of the pattern, support), compared in that order;
//   dominated     support below that of the k-th result (strict); minimum
//                 image-based support never grows when a pattern grows, so
//                 nothing below a dominated group can reach the result set.
//
// A subgraph group is the set of embeddings of one DFS code: for every
// subgraph, the data vertex of each code vertex.  The host keeps the queue
// of groups (a few thousand at most) and the result set; the device holds
// the embeddings and does the per-embedding work:
//
//   k_pm_first      one-edge subgraphs (u, v) with L(u) <= L(v) (the only
//                   minimal one-edge codes), counted and then written by
//                   label pair;
//   k_pm_extend     one thread per embedding of the group being
//                   expanded: the rightmost-path extensions of its code --
//                   backward edges from the rightmost vertex, forward edges
//                   from every vertex of the rightmost path to a data
//                   neighbour not yet in the embedding -- restricted to the
//                   extensions whose new code the host found minimal;
//                   counted in one pass, written in a second into one slice
//                   per new code (per-block counts in LDS, one global
//                   atomic per block and code);
//   k_pm_mark,      minimum image-based support of every new group at
//   k_pm_count      once: one byte per data vertex and (group, code
//                   vertex), set by the embeddings that map the code vertex
//                   there, then counted.
//
// Results: the k patterns of highest support (ties: smaller code first,
// under the code order below), each with its support.
#include <algorithm>
#include <climits>
#include <cstring>
#include <memory>
#include <queue>

#include "device_common.h"

namespace nuri {
namespace {

constexpr uint32_t kPMaxE = 8;             // edges of a pattern
constexpr uint32_t kPMaxV = kPMaxE + 1;    // vertices of a pattern
constexpr uint32_t kL = NURI_MAX_LABELS;   // vertex labels
constexpr uint32_t kMaxKeys = kPMaxV + kPMaxV * kL;  // extension keys of one group
constexpr uint32_t kKeyCap = kL * kL;                 // one-edge label pairs
static_assert(kKeyCap >= kMaxKeys, "key buffers hold either kind of key");

struct CodeEdge {
  uint8_t i, j, li, lj;
};

// Code edges compare by (backward first; backward by target; forward by the
// deeper source first, then by labels); codes compare edge by edge.  For
// codes that agree up to some edge this is gSpan's DFS lexicographic order.
inline void edge_key(const CodeEdge &e, int k[4]) {
  if (e.i > e.j) {
    k[0] = 0;
    k[1] = e.j;
    k[2] = k[3] = 0;
  } else {
    k[0] = 1;
    k[1] = -(int)e.i;
    k[2] = e.li;
    k[3] = e.lj;
  }
}

inline int edge_cmp(const CodeEdge &a, const CodeEdge &b) {
  int x[4], y[4];
  edge_key(a, x);
  edge_key(b, y);
  for (int t = 0; t < 4; ++t)
    if (x[t] != y[t]) return x[t] < y[t] ? -1 : 1;
  return 0;
}

inline int code_cmp(const std::vector<CodeEdge> &a, const std::vector<CodeEdge> &b) {
  const size_t n = std::min(a.size(), b.size());
  for (size_t t = 0; t < n; ++t) {
    const int c = edge_cmp(a[t], b[t]);
    if (c) return c;
  }
  return a.size() < b.size() ? -1 : (a.size() > b.size());
}

// Is `code` the minimum DFS code of its own pattern?  Depth-first
// traversals of the pattern are grown edge by edge and compared with the
// code as they grow: a traversal that falls below it proves it is not
// minimal, one that rises above it is abandoned.
struct MinCheck {
  const std::vector<CodeEdge> &code;
  uint32_t nv;
  uint8_t lab[kPMaxV];
  uint16_t adj[kPMaxV];  // adjacency bitmasks
  int id[kPMaxV];        // discovery id, -1 unvisited
  uint32_t who[kPMaxV];
  uint32_t nvis = 0;
  bool smaller = false;

  explicit MinCheck(const std::vector<CodeEdge> &c) : code(c) {
    nv = 0;
    for (const auto &e : c) nv = std::max<uint32_t>(nv, std::max(e.i, e.j) + 1u);
    memset(adj, 0, sizeof(adj));
    for (const auto &e : c) {
      lab[e.i] = e.li;
      lab[e.j] = e.lj;
      adj[e.i] |= (uint16_t)(1u << e.j);
      adj[e.j] |= (uint16_t)(1u << e.i);
    }
  }

  // pos: code edges matched so far; path: the current DFS path
  void grow(size_t pos, const uint32_t *path, uint32_t sp) {
    if (smaller || pos == code.size()) return;
    while (sp > 0) {
      uint32_t open = 0;
      for (uint32_t w = 0; w < nv; ++w)
        if ((adj[path[sp - 1]] >> w & 1) && id[w] < 0) open = 1;
      if (open) break;
      --sp;
    }
    if (sp == 0) return;
    const uint32_t u = path[sp - 1];
    uint32_t next[kPMaxV];
    memcpy(next, path, sp * sizeof(uint32_t));
    for (uint32_t w = 0; w < nv && !smaller; ++w) {
      if (!(adj[u] >> w & 1) || id[w] >= 0) continue;
      const uint32_t nid = nvis;
      // the forward edge, then w's edges back to visited vertices
      CodeEdge run[kPMaxV + 1];
      uint32_t nrun = 0;
      run[nrun++] = CodeEdge{(uint8_t)id[u], (uint8_t)nid, lab[u], lab[w]};
      for (uint32_t k = 0; k < nid; ++k)
        if (who[k] != u && (adj[w] >> who[k] & 1))
          run[nrun++] = CodeEdge{(uint8_t)nid, (uint8_t)k, lab[w], lab[who[k]]};
      int c = 0;
      uint32_t t = 0;
      for (; t < nrun && pos + t < code.size(); ++t) {
        c = edge_cmp(run[t], code[pos + t]);
        if (c) break;
      }
      if (c < 0) {
        smaller = true;
        return;
      }
      if (c > 0) continue;  // this traversal is already larger
      id[w] = (int)nid;
      who[nid] = w;
      ++nvis;
      next[sp] = w;
      grow(pos + nrun, next, sp + 1);
      --nvis;
      id[w] = -1;
    }
  }

  bool is_min() {
    for (uint32_t s = 0; s < nv && !smaller; ++s) {
      if (lab[s] != code[0].li) continue;  // a smaller first label would already win
      for (uint32_t v = 0; v < kPMaxV; ++v) id[v] = -1;
      id[s] = 0;
      who[0] = s;
      nvis = 1;
      uint32_t path[1] = {s};
      grow(0, path, 1);
    }
    // a start vertex with a smaller label than the code's first vertex
    for (uint32_t s = 0; s < nv; ++s)
      for (uint32_t w = 0; w < nv; ++w)
        if ((adj[s] >> w & 1) &&
            edge_cmp(CodeEdge{0, 1, lab[s], lab[w]}, code[0]) < 0)
          return false;
    return !smaller;
  }
};

// the extensions of one group, as the kernels need them
struct PMExt {
  uint32_t nv, rm, np, nkeys;
  uint32_t back_mask;          // bit x: backward edge rm -> x is a minimal extension
  uint32_t pad;
  uint8_t path[kPMaxV];        // rightmost path, rm first
  uint8_t lab[kPMaxV];         // code vertex labels
  uint16_t fwd_mask[kPMaxV];   // per code vertex: bit l, forward edge to a new label-l vertex
};

struct PMView {
  const uint64_t *orow;
  const uint32_t *lcol;
  const uint32_t *loff;
  const uint8_t *lab;
  uint32_t n;
};

__device__ inline bool pm_adjacent(const PMView &m, uint32_t v, uint32_t l, uint32_t x) {
  const uint32_t *lo = m.loff + (u64)v * 17;
  u64 a = m.orow[v] + lo[l], z = m.orow[v] + lo[l + 1];
  while (a < z) {
    const u64 mid = (a + z) >> 1;
    if (m.lcol[mid] < x) a = mid + 1;
    else z = mid;
  }
  return a < m.orow[v] + lo[l + 1] && m.lcol[a] == x;
}

// one-edge subgraphs: thread per vertex u, every neighbour v with
// L(u) <= L(v); key = L(u) * 16 + L(v).  kWrite: write (u, v) at the
// key's cursor; else count.
template <bool kWrite>
__global__ void __launch_bounds__(256)
    k_pm_first(PMView m, unsigned long long *count, unsigned long long *cursor,
               const unsigned long long *off, uint32_t *out) {
  for (u64 u = blockIdx.x * (u64)blockDim.x + threadIdx.x; u < m.n;
       u += (u64)gridDim.x * blockDim.x) {
    const uint32_t lu = m.lab[u];
    const uint32_t *lo = m.loff + u * 17;
    // neighbours are sorted by (label, id): labels >= lu start at lo[lu]
    for (u64 t = m.orow[u] + lo[lu]; t < m.orow[u + 1]; ++t) {
      const uint32_t v = m.lcol[t];
      const uint32_t key = lu * kL + m.lab[v];
      if (!kWrite) {
        atomicAdd(&count[key], 1ull);
      } else {
        const u64 s = atomicAdd(&cursor[key], 1ull);
        uint32_t *dst = out + off[key] + 2 * s;
        dst[0] = (uint32_t)u;
        dst[1] = v;
      }
    }
  }
}

// x[i] for an index known only at run time, by selects over the slots
// (a run-time index into a register array would put it in scratch memory)
__device__ inline uint32_t pick(const uint32_t *x, uint32_t i) {
  uint32_t r = x[0];
#pragma unroll
  for (uint32_t v = 1; v < kPMaxV; ++v) r = (i == v) ? x[v] : r;
  return r;
}

// every minimal rightmost-path extension of embedding phi, in a fixed
// order: emit(key, w) with w the new vertex (forward) or ~0u (backward)
template <class F>
__device__ inline void pm_extensions(const PMView &m, const PMExt &x, const uint32_t *phi, F emit) {
  const uint32_t prm = pick(phi, x.rm);
  for (uint32_t v = 0; v < x.nv; ++v)
    if ((x.back_mask >> v & 1) && pm_adjacent(m, prm, x.lab[v], pick(phi, v))) emit(v, ~0u);
  for (uint32_t q = 0; q < x.np; ++q) {
    const uint32_t xv = x.path[q];
    const uint32_t mask = x.fwd_mask[xv];
    if (!mask) continue;
    const uint32_t d = pick(phi, xv);
    const uint32_t *lo = m.loff + (u64)d * 17;
    const u64 r0 = m.orow[d];
    for (uint32_t l = 0; l < kL; ++l) {
      if (!(mask >> l & 1)) continue;
      const uint32_t key = x.nv + xv * kL + l;
      for (u64 t = r0 + lo[l], z = r0 + lo[l + 1]; t < z; ++t) {
        const uint32_t w = m.lcol[t];
        bool fresh = true;
#pragma unroll
        for (uint32_t v = 0; v < kPMaxV; ++v)
          if (v < x.nv && phi[v] == w) fresh = false;
        if (fresh) emit(key, w);
      }
    }
  }
}

// rightmost-path extensions of every embedding of one group: one thread
// per embedding.  Counts go to LDS per block and then to the global count
// of each key (!kWrite).  kWrite: each block reserves its run of slots per
// key with one global atomic and writes its children there; children of
// key c go to out + off[c] with stride nv'(c) (nv for backward keys, nv + 1
// for forward keys).
template <bool kWrite>
__global__ void __launch_bounds__(256)
    k_pm_extend(PMView m, const uint32_t *__restrict__ emb, u64 count, PMExt x,
                unsigned long long *cnt, unsigned long long *cursor,
                const unsigned long long *off, uint32_t *out) {
  __shared__ unsigned int s_cnt[kMaxKeys];
  __shared__ unsigned int s_pos[kMaxKeys];
  __shared__ unsigned long long s_base[kMaxKeys];
  for (uint32_t c = threadIdx.x; c < x.nkeys; c += blockDim.x) {
    s_cnt[c] = 0;
    s_pos[c] = 0;
  }
  __syncthreads();
  const u64 e = blockIdx.x * (u64)blockDim.x + threadIdx.x;
  const bool live = e < count;
  uint32_t phi[kPMaxV];
#pragma unroll
  for (uint32_t v = 0; v < kPMaxV; ++v) phi[v] = (live && v < x.nv) ? emb[e * x.nv + v] : ~0u;
  if (live)
    pm_extensions(m, x, phi, [&](uint32_t key, uint32_t) { atomicAdd(&s_cnt[key], 1u); });
  __syncthreads();
  if (!kWrite) {
    for (uint32_t c = threadIdx.x; c < x.nkeys; c += blockDim.x)
      if (s_cnt[c]) atomicAdd(&cnt[c], (unsigned long long)s_cnt[c]);
    return;
  }
  for (uint32_t c = threadIdx.x; c < x.nkeys; c += blockDim.x)
    s_base[c] = s_cnt[c] ? atomicAdd(&cursor[c], (unsigned long long)s_cnt[c]) : 0ull;
  __syncthreads();
  if (!live) return;
  pm_extensions(m, x, phi, [&](uint32_t key, uint32_t w) {
    const u64 slot = s_base[key] + atomicAdd(&s_pos[key], 1u);
    const uint32_t nv2 = key < x.nv ? x.nv : x.nv + 1;
    uint32_t *dst = out + off[key] + slot * nv2;
#pragma unroll
    for (uint32_t v = 0; v < kPMaxV; ++v)
      if (v < x.nv) dst[v] = phi[v];
    if (key >= x.nv) dst[x.nv] = w;
  });
}

// minimum image-based support of every new group, in two kernels.  Each
// (group, code vertex) has a slot: a byte per data vertex, set when some
// embedding maps the code vertex there (a plain store: many embeddings
// share an image, and an atomic per entry would serialise on it), then
// counted.  Group g's entries are [woff[g], woff[g + 1]) with stride
// nvs[g]; its slots start at sbase[g].
__global__ void __launch_bounds__(256)
    k_pm_mark(const uint32_t *__restrict__ ent, const unsigned long long *woff,
              const uint32_t *nvs, const uint32_t *sbase, uint32_t ngroups, uint32_t n,
              uint8_t *marks) {
  const u64 total = woff[ngroups];
  for (u64 i = blockIdx.x * (u64)blockDim.x + threadIdx.x; i < total;
       i += (u64)gridDim.x * blockDim.x) {
    uint32_t lo = 0, hi = ngroups;  // the group holding entry i
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (woff[mid] <= i) lo = mid;
      else hi = mid;
    }
    const uint32_t pos = (uint32_t)((i - woff[lo]) % nvs[lo]);
    marks[(u64)(sbase[lo] + pos) * n + ent[i]] = 1;
  }
}

// one block per slot: the number of marked vertices
__global__ void __launch_bounds__(256)
    k_pm_count(const uint8_t *__restrict__ marks, uint32_t n, unsigned long long *images) {
  __shared__ unsigned long long part[4];
  const uint8_t *row = marks + (u64)blockIdx.x * n;
  unsigned long long c = 0;
  for (uint32_t v = threadIdx.x; v < n; v += blockDim.x) c += row[v];
  c = wave_sum(c);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) images[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

// ------------------------------------------------------------------
// host
// ------------------------------------------------------------------

// embeddings of one or more groups, freed when the last group using them is
struct EmbBlock {
  MemPool *pool = nullptr;
  uint64_t *held = nullptr;  // the engine's count of embedding bytes
  uint32_t *p = nullptr;
  size_t bytes = 0;
  ~EmbBlock() {
    if (p) pool->put(p, bytes);
    if (held) *held -= bytes;
  }
};

struct Group {
  std::vector<CodeEdge> code;
  uint32_t nv = 0;
  uint64_t support = 0;
  uint64_t count = 0;                // embeddings
  std::shared_ptr<EmbBlock> block;   // embeddings at block->p + word_off
  uint64_t word_off = 0;
  uint64_t seq = 0;
};

struct GroupOrder {  // priority (edges, support); earlier first on ties
  bool operator()(const std::shared_ptr<Group> &a, const std::shared_ptr<Group> &b) const {
    if (a->code.size() != b->code.size()) return a->code.size() < b->code.size();
    if (a->support != b->support) return a->support < b->support;
    return a->seq > b->seq;
  }
};

struct PResult {
  uint64_t f;
  std::vector<CodeEdge> code;
};

inline bool presult_before(const PResult &a, const PResult &b) {
  if (a.f != b.f) return a.f > b.f;
  return code_cmp(a.code, b.code) < 0;
}

struct PatternEngine {
  Graph &g;
  QueryOpts o;
  hipStream_t s;
  uint32_t M, k;
  std::vector<PResult> R;
  std::priority_queue<std::shared_ptr<Group>, std::vector<std::shared_ptr<Group>>, GroupOrder> Q;
  uint64_t seq = 0;
  nuri_stats st{};
  uint64_t held = 0, peak = 0;  // embedding bytes on the device
  PinBuf<unsigned long long> h_cnt;
  DevBuf<unsigned long long> d_cnt, d_cursor, d_off, d_woff, d_images;
  DevBuf<uint32_t> d_nvs, d_sbase;
  uint64_t t0 = 0;

  PatternEngine(Graph &g_, const QueryOpts &o_, uint32_t M_, uint32_t k_)
      : g(g_), o(o_), s(o_.stream ? o_.stream : g_.stream), M(M_), k(k_) {
    h_cnt.alloc(kKeyCap + 1);
    d_cnt.alloc(kKeyCap);
    d_cursor.alloc(kKeyCap);
    d_off.alloc(kKeyCap + 1);
    d_woff.alloc(kKeyCap + 1);
    d_images.alloc((size_t)kKeyCap * kPMaxV);
    d_nvs.alloc(kKeyCap);
    d_sbase.alloc(kKeyCap);
  }

  PMView view() const {
    return PMView{g.orow.p, g.lcol.p, g.loff.p, g.vlab.p, g.n};
  }

  bool dominated(uint64_t f) const { return R.size() == k && f < R.back().f; }

  void offer(const Group &G) {
    PResult x{G.support, G.code};
    if (R.size() == k && !presult_before(x, R.back())) return;
    R.insert(std::upper_bound(R.begin(), R.end(), x, presult_before), x);
    if (R.size() > k) R.pop_back();
    st.offered++;
  }

  std::shared_ptr<EmbBlock> alloc_block(uint64_t words) {
    const uint64_t bytes = std::max<uint64_t>(4, words * 4);
    if (held + bytes > o.frontier_budget)
      throw Error{NURI_EBUDGET, "pattern mining: embeddings exceed the frontier budget"};
    auto b = std::make_shared<EmbBlock>();
    b->pool = &g.pool;
    b->p = (uint32_t *)g.pool.get(bytes);
    b->bytes = bytes;
    b->held = &held;
    held += bytes;
    peak = std::max(peak, held);
    return b;
  }

  // support of groups [0, ng) whose embeddings are at `ent` with word
  // offsets woff (ng + 1 entries, host) and strides nvs
  void supports(const uint32_t *ent, const std::vector<uint64_t> &woff,
                const std::vector<uint32_t> &nvs, std::vector<uint64_t> &out) {
    const uint32_t ng = (uint32_t)nvs.size();
    out.assign(ng, 0);
    if (!ng) return;
    std::vector<uint32_t> sbase(ng + 1, 0);
    for (uint32_t c = 0; c < ng; ++c) sbase[c + 1] = sbase[c] + nvs[c];
    const uint32_t slots = sbase[ng];
    PoolBuf<uint8_t> marks;
    marks.alloc(g.pool, (size_t)slots * g.n);
    NURI_HIP(hipMemsetAsync(marks.p, 0, marks.bytes(), s));
    NURI_HIP(hipMemcpyAsync(d_woff.p, woff.data(), (ng + 1) * 8, hipMemcpyHostToDevice, s));
    NURI_HIP(hipMemcpyAsync(d_nvs.p, nvs.data(), ng * 4, hipMemcpyHostToDevice, s));
    NURI_HIP(hipMemcpyAsync(d_sbase.p, sbase.data(), ng * 4, hipMemcpyHostToDevice, s));
    const u64 total = woff[ng];
    const uint32_t blocks = (uint32_t)std::max<u64>(1, std::min<u64>((total + 255) / 256, 1 << 16));
    hipLaunchKernelGGL(k_pm_mark, dim3(blocks), dim3(256), 0, s, ent, d_woff.p, d_nvs.p,
                       d_sbase.p, ng, g.n, marks.p);
    NURI_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_pm_count, dim3(slots), dim3(256), 0, s, marks.p, g.n, d_images.p);
    NURI_HIP(hipGetLastError());
    std::vector<unsigned long long> img(slots);
    NURI_HIP(hipMemcpyAsync(img.data(), d_images.p, slots * 8, hipMemcpyDeviceToHost, s));
    NURI_HIP(hipStreamSynchronize(s));
    for (uint32_t c = 0; c < ng; ++c) {
      uint64_t f = UINT64_MAX;
      for (uint32_t v = sbase[c]; v < sbase[c + 1]; ++v) f = std::min<uint64_t>(f, img[v]);
      out[c] = f;
    }
  }

  // lines 1-8 of Algorithm 2
  void first_groups() {
    const uint32_t nk = kL * kL;
    NURI_HIP(hipMemsetAsync(d_cnt.p, 0, nk * 8, s));
    const uint32_t blocks = (uint32_t)std::max<u64>(1, std::min<u64>((g.n + 255) / 256, 1 << 14));
    hipLaunchKernelGGL(k_pm_first<false>, dim3(blocks), dim3(256), 0, s, view(), d_cnt.p,
                       d_cursor.p, d_off.p, (uint32_t *)nullptr);
    NURI_HIP(hipGetLastError());
    NURI_HIP(hipMemcpyAsync(h_cnt.p, d_cnt.p, nk * 8, hipMemcpyDeviceToHost, s));
    NURI_HIP(hipStreamSynchronize(s));
    std::vector<uint64_t> off(nk + 1, 0);
    for (uint32_t c = 0; c < nk; ++c) off[c + 1] = off[c] + 2 * h_cnt.p[c];
    auto block = alloc_block(off[nk]);
    NURI_HIP(hipMemcpyAsync(d_off.p, off.data(), nk * 8, hipMemcpyHostToDevice, s));
    NURI_HIP(hipMemsetAsync(d_cursor.p, 0, nk * 8, s));
    hipLaunchKernelGGL(k_pm_first<true>, dim3(blocks), dim3(256), 0, s, view(), d_cnt.p,
                       d_cursor.p, d_off.p, block->p);
    NURI_HIP(hipGetLastError());
    std::vector<uint64_t> woff;
    std::vector<uint32_t> nvs, keys;
    for (uint32_t c = 0; c < nk; ++c)
      if (h_cnt.p[c]) {
        woff.push_back(off[c]);
        nvs.push_back(2);
        keys.push_back(c);
      }
    woff.push_back(off[nk]);
    st.children += off[nk] / 2;
    // the groups' slices are contiguous in key order, so woff is the
    // compacted offset list
    std::vector<uint64_t> f;
    supports(block->p, woff, nvs, f);
    for (size_t t = 0; t < keys.size(); ++t) {
      auto G = std::make_shared<Group>();
      G->code = {CodeEdge{0, 1, (uint8_t)(keys[t] / kL), (uint8_t)(keys[t] % kL)}};
      G->nv = 2;
      G->support = f[t];
      G->count = (woff[t + 1] - woff[t]) / 2;
      G->block = block;
      G->word_off = woff[t];
      G->seq = seq++;
      Q.push(G);
    }
  }

  // lines 17-27 for group S
  void expand(const Group &S) {
    st.expanded++;
    PMExt x;
    memset(&x, 0, sizeof(x));
    x.nv = S.nv;
    x.rm = S.nv - 1;
    uint32_t par[kPMaxV] = {};
    bool has[kPMaxV][kPMaxV] = {};
    for (const auto &e : S.code) {
      if (e.i < e.j) par[e.j] = e.i;
      has[e.i][e.j] = has[e.j][e.i] = true;
      x.lab[e.i] = e.li;
      x.lab[e.j] = e.lj;
    }
    bool onpath[kPMaxV] = {};
    for (uint32_t v = x.rm;; v = par[v]) {
      x.path[x.np++] = (uint8_t)v;
      onpath[v] = true;
      if (v == 0) break;
    }
    // the extensions whose new code is minimal (key: backward v -> v;
    // forward from v with label l -> nv + v * 16 + l)
    x.nkeys = x.nv + x.nv * kL;
    std::vector<std::vector<CodeEdge>> kcode(x.nkeys);
    for (uint32_t v = 0; v < x.rm; ++v) {
      if (!onpath[v] || has[x.rm][v]) continue;
      std::vector<CodeEdge> c = S.code;
      c.push_back(CodeEdge{(uint8_t)x.rm, (uint8_t)v, x.lab[x.rm], x.lab[v]});
      if (MinCheck(c).is_min()) {
        x.back_mask |= 1u << v;
        kcode[v] = std::move(c);
      }
    }
    if (S.nv < kPMaxV)
      for (uint32_t q = 0; q < x.np; ++q) {
        const uint32_t v = x.path[q];
        for (uint32_t l = 0; l < kL; ++l) {
          if (!g.h_label_count[l]) continue;
          std::vector<CodeEdge> c = S.code;
          c.push_back(CodeEdge{(uint8_t)v, (uint8_t)x.nv, x.lab[v], (uint8_t)l});
          if (MinCheck(c).is_min()) {
            x.fwd_mask[v] |= (uint16_t)(1u << l);
            kcode[x.nv + v * kL + l] = std::move(c);
          }
        }
      }
    if (!x.back_mask && !std::any_of(x.fwd_mask, x.fwd_mask + kPMaxV, [](uint16_t m) { return m; }))
      return;
    const uint32_t *emb = S.block->p + S.word_off;
    if ((S.count + 255) / 256 > 0x7FFFFFFFull)
      throw Error{NURI_EBUDGET, "pattern mining: a group has too many embeddings for one launch"};
    const uint32_t blocks = (uint32_t)((S.count + 255) / 256);
    NURI_HIP(hipMemsetAsync(d_cnt.p, 0, x.nkeys * 8, s));
    if (o.profile) NURI_HIP(hipEventRecord(ev0, s));
    hipLaunchKernelGGL(k_pm_extend<false>, dim3(blocks), dim3(256), 0, s, view(), emb,
                       (u64)S.count, x, d_cnt.p, d_cursor.p, d_off.p, (uint32_t *)nullptr);
    NURI_HIP(hipGetLastError());
    if (o.profile) NURI_HIP(hipEventRecord(ev1, s));
    NURI_HIP(hipMemcpyAsync(h_cnt.p, d_cnt.p, x.nkeys * 8, hipMemcpyDeviceToHost, s));
    NURI_HIP(hipStreamSynchronize(s));
    std::vector<uint64_t> off(x.nkeys + 1, 0);
    for (uint32_t c = 0; c < x.nkeys; ++c)
      off[c + 1] = off[c] + h_cnt.p[c] * (c < x.nv ? x.nv : x.nv + 1);
    if (!off[x.nkeys]) return;
    auto block = alloc_block(off[x.nkeys]);
    NURI_HIP(hipMemcpyAsync(d_off.p, off.data(), x.nkeys * 8, hipMemcpyHostToDevice, s));
    NURI_HIP(hipMemsetAsync(d_cursor.p, 0, x.nkeys * 8, s));
    if (o.profile) NURI_HIP(hipEventRecord(ev2, s));
    hipLaunchKernelGGL(k_pm_extend<true>, dim3(blocks), dim3(256), 0, s, view(), emb,
                       (u64)S.count, x, d_cnt.p, d_cursor.p, d_off.p, block->p);
    NURI_HIP(hipGetLastError());
    if (o.profile) {
      // the two passes are timed apart: the host works between them
      NURI_HIP(hipEventRecord(ev3, s));
      NURI_HIP(hipEventSynchronize(ev3));
      float a = 0, b = 0;
      NURI_HIP(hipEventElapsedTime(&a, ev0, ev1));
      NURI_HIP(hipEventElapsedTime(&b, ev2, ev3));
      st.expand_ns += (uint64_t)((a + b) * 1e6);
    }
    st.expand_launches += 2;
    std::vector<uint64_t> woff;
    std::vector<uint32_t> nvs, keys;
    for (uint32_t c = 0; c < x.nkeys; ++c)
      if (h_cnt.p[c]) {
        woff.push_back(off[c]);
        nvs.push_back(c < x.nv ? x.nv : x.nv + 1);
        keys.push_back(c);
      }
    woff.push_back(off[x.nkeys]);
    for (uint32_t c = 0; c < x.nkeys; ++c) st.children += h_cnt.p[c];
    // algorithmic bytes of the two passes: the parent group read twice,
    // the children written once (the data rows scanned are not counted)
    st.logical_bytes += 2 * S.count * S.nv * 4 + off[x.nkeys] * 4;
    std::vector<uint64_t> f;
    supports(block->p, woff, nvs, f);
    for (size_t t = 0; t < keys.size(); ++t) {
      if (dominated(f[t])) {
        st.pruned_at_creation++;
        continue;
      }
      auto G = std::make_shared<Group>();
      G->code = kcode[keys[t]];
      G->nv = nvs[t];
      G->support = f[t];
      G->count = (woff[t + 1] - woff[t]) / nvs[t];
      G->block = block;
      G->word_off = woff[t];
      G->seq = seq++;
      Q.push(G);
    }
  }

  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr, ev3 = nullptr;

  ~PatternEngine() {
    for (hipEvent_t ev : {ev0, ev1, ev2, ev3})
      if (ev) (void)hipEventDestroy(ev);
  }

  void run(Result &res) {
    t0 = now_ns();
    if (o.profile) {
      NURI_HIP(hipEventCreate(&ev0));
      NURI_HIP(hipEventCreate(&ev1));
      NURI_HIP(hipEventCreate(&ev2));
      NURI_HIP(hipEventCreate(&ev3));
    }
    first_groups();
    while (!Q.empty()) {
      if (o.deadline_ns && now_ns() - t0 > o.deadline_ns)
        throw Error{NURI_ETIMEOUT, "query deadline passed"};
      std::shared_ptr<Group> S = Q.top();
      Q.pop();
      st.popped++;
      st.steps++;
      if (S->code.size() == M) offer(*S);
      if (dominated(S->support)) {
        st.pruned_at_pop++;
      } else if (S->code.size() < M) {
        expand(*S);
      }
    }
    res.score.clear();
    res.offset.assign(1, 0);
    res.ids.clear();
    for (const auto &r : R) {
      res.score.push_back((int64_t)r.f);
      for (const auto &e : r.code) {
        res.ids.push_back(e.i);
        res.ids.push_back(e.j);
        res.ids.push_back(e.li);
        res.ids.push_back(e.lj);
      }
      res.offset.push_back(res.ids.size());
    }
    st.frontier_peak_bytes = peak;
    st.wall_ns = now_ns() - t0;
    st.ties_at_k = ties_at_k(res.score, k);
    res.stats = st;
  }
};

}  // namespace

void run_patterns(Graph &g, uint32_t n_edges, uint32_t k, const QueryOpts &o, Result &out) {
  if (!g.has_lab) throw Error{NURI_EINVAL, "pattern mining needs vertex labels"};
  if (n_edges < 1 || n_edges > kPMaxE) throw Error{NURI_EINVAL, "n_edges must be 1..8"};
  if (k == 0) throw Error{NURI_EINVAL, "k must be >= 1"};
  PatternEngine e(g, o, n_edges, k);
  e.run(out);
}

}  // namespace nuri
