// Internal declarations of the engine (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/nuri.h"

namespace nuri {

// Largest |N+(v)| the dense local bitmaps support: one 64-bit word per lane
// of a 64-wide wavefront.
constexpr uint32_t kMaxLocal = 4096;
constexpr uint32_t kMaxWords = kMaxLocal / 64;
// copies of each query's work counters, one cache line apiece: every
// wavefront of an expansion launch adds its counts when it ends, and
// thousands of atomics on one line serialise; a kernel adds to the copy
// its workgroup picks and the host sums the copies
constexpr uint32_t kCtrSlots = 64;
constexpr uint32_t kHeavy = 32;

// ------------------------------------------------------------------
// errors
// ------------------------------------------------------------------
void set_error(const std::string &msg);

struct Error {
  int code;
  std::string msg;
};

#define NURI_HIP(call)                                                                    \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      throw ::nuri::Error{e_ == hipErrorOutOfMemory ? NURI_ENOMEM : NURI_EDEVICE,         \
                          std::string(#call) + ": " + hipGetErrorString(e_)};             \
  } while (0)

// Owning device buffer.
template <class T>
struct DevBuf {
  T *p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void alloc(size_t count) {
    release();
    if (count == 0) count = 1;
    NURI_HIP(hipMalloc(&p, count * sizeof(T)));
    n = count;
  }
  size_t bytes() const { return n * sizeof(T); }
};

// Device memory kept for reuse by later queries on the same graph: query
// workspaces (frontier arenas, buffers) are taken from here and returned,
// so repeated queries do not pay for hipMalloc/hipFree of large blocks.
//
// Fixed-region mode (fixed_base set): blocks are carved in order from the
// caller's region [fixed_base, fixed_base + fixed_size), never returned one
// by one, and no device memory is ever allocated; a request past the end
// of the region fails with NURI_EBUDGET.
struct MemPool {
  std::mutex mu;
  std::multimap<size_t, void *> free_blocks;  // size -> block
  unsigned char *fixed_base = nullptr;
  size_t fixed_size = 0, fixed_used = 0;
  ~MemPool() { trim(); }
  static size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }
  void *get(size_t bytes) {
    if (fixed_base) {
      const size_t at = align_up(fixed_used);
      if (at + bytes > fixed_size)
        throw Error{NURI_EBUDGET, "query needs more than the fixed scratch region (" +
                                      std::to_string(fixed_size) + " bytes)"};
      fixed_used = at + bytes;
      return fixed_base + at;
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      auto it = free_blocks.lower_bound(bytes);
      if (it != free_blocks.end() && it->first <= 2 * bytes + (64ull << 20)) {
        void *p = it->second;
        free_blocks.erase(it);
        return p;
      }
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e == hipErrorOutOfMemory) {
      (void)hipGetLastError();
      trim();
      e = hipMalloc(&p, bytes);
    }
    if (e != hipSuccess)
      throw Error{e == hipErrorOutOfMemory ? NURI_ENOMEM : NURI_EDEVICE,
                  std::string("hipMalloc: ") + hipGetErrorString(e)};
    return p;
  }
  void put(void *p, size_t bytes) {
    if (fixed_base) return;
    std::lock_guard<std::mutex> lk(mu);
    free_blocks.emplace(bytes, p);
  }
  void trim() {
    std::lock_guard<std::mutex> lk(mu);
    for (auto &kv : free_blocks) (void)hipFree(kv.second);
    free_blocks.clear();
  }
};

// Device buffer borrowed from a graph's MemPool.  The block returns to the
// pool when the buffer is released; block sizes are remembered exactly so
// a later query asking for the same size reuses it.
template <class T>
struct PoolBuf {
  MemPool *pool = nullptr;
  T *p = nullptr;
  size_t n = 0, cap_bytes = 0;
  PoolBuf() = default;
  PoolBuf(const PoolBuf &) = delete;
  PoolBuf &operator=(const PoolBuf &) = delete;
  ~PoolBuf() { release(); }
  void release() {
    if (p && pool) pool->put(p, cap_bytes);
    p = nullptr;
    n = 0;
    cap_bytes = 0;
  }
  void alloc(MemPool &mp, size_t count) {
    release();
    if (count == 0) count = 1;
    pool = &mp;
    cap_bytes = count * sizeof(T);
    p = (T *)mp.get(cap_bytes);
    n = count;
  }
  size_t bytes() const { return n * sizeof(T); }
};

// ------------------------------------------------------------------
// resident graph
// ------------------------------------------------------------------
//
// Vertices are relabelled by rank in a degeneracy order; "rank" below is a
// vertex id in that relabelled space.  For a vertex r, the local universe
// is its out-list N+(r) (neighbours of higher rank), sorted by rank;
// position j in it is "local position j".  The local bitmap of r holds,
// for every local position i, the row {j : N+(r)[j] adjacent to
// N+(r)[i]} as W(r) = ceil(|N+(r)| / 64) words.
struct Graph {
  uint32_t n = 0;
  uint64_t nnz = 0;
  uint32_t degeneracy = 0;
  uint32_t n_labels = 0;
  bool has_vw = false, has_lab = false, has_ew = false;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  uint64_t preprocess_ns = 0;

  // device: rank-space CSR, rows sorted by rank; N-(r) = first split[r]
  // entries of row r, N+(r) = the rest
  DevBuf<uint64_t> rrow;
  DevBuf<uint32_t> rcol;
  DevBuf<uint32_t> split;
  DevBuf<uint32_t> dplus;     // |N+(r)|
  // heavy lower neighbours: the part of N-(r) whose |N+(u)| >= kHeavy,
  // sorted by rank (a vertex that extends a clique of c >= kHeavy members
  // ranked above it has |N+(u)| >= c)
  DevBuf<uint64_t> hrow;
  DevBuf<uint32_t> hcol;
  // [n] maximality checks of cliques: a vertex that u was found not to be
  // adjacent to (~0u: none yet); filled as queries run
  DevBuf<uint32_t> leaf_wit;
  DevBuf<uint32_t> orig;      // rank -> original id
  DevBuf<int32_t> vw;         // vertex weight by rank
  DevBuf<uint64_t> bm_off;    // [n+1] word offset of r's local bitmap
  DevBuf<uint64_t> bm;        // local adjacency bitmaps
  DevBuf<int64_t> wplus;      // sum of vertex weights over N+(r)

  // labelled matching works on original ids: every row of the input CSR
  // re-sorted by (label, id), with per-row label segment offsets
  DevBuf<uint64_t> orow;      // [n+1] = the input row_ptr
  DevBuf<uint32_t> lcol;      // [nnz] neighbours sorted by (label, id)
  DevBuf<int32_t> lew;        // [nnz] edge weights aligned with lcol
  DevBuf<uint32_t> loff;      // [n * 17] label l of row v: lcol[orow[v] + loff[17v+l] .. 17v+l+1)
  DevBuf<int32_t> best;       // [n * 16] max edge weight from v to a label-l vertex (0: none)
  DevBuf<uint32_t> lab_vert;  // vertices grouped by label, ascending ids within a label
  DevBuf<uint8_t> vlab;       // [n] vertex labels
  std::vector<uint64_t> h_lab_off;  // [17] offsets of the label groups in lab_vert

  // host mirrors used to plan queries
  std::vector<uint32_t> h_dplus;
  std::vector<uint32_t> h_rank;            // original id -> rank
  std::vector<uint32_t> h_orig;            // rank -> original id
  std::vector<uint64_t> h_label_count;     // vertices per label
  std::vector<int32_t> h_pairmax;          // [16*16] max edge weight per label pair
  // root orders: ranks sorted by root bound (descending), per score kind
  std::vector<uint32_t> h_root_order[2];
  std::vector<int64_t> h_root_bound[2];
  DevBuf<uint32_t> root_order[2];
  uint64_t bitmap_words = 0;
  double core_density = 0;  // edge density inside the largest local universes

  // oriented adjacency in a compact layout: N+(r) at oplus[ooff[r] ..
  // ooff[r] + dplus[r]) and the weights of those vertices at wloc[...]
  DevBuf<uint64_t> ooff;
  DevBuf<uint32_t> oplus;
  DevBuf<int32_t> wloc;

  // multi-hop (label, hop) max-degree index for the degree score of
  // matching, built on first use up to the hops a pattern needs:
  // hidx[h-1][v * 16 + l] = largest degree of a label-l vertex 1..h hops
  // from v (0: none).  Arrays of hops already built are never replaced.
  std::mutex hidx_mu;
  DevBuf<int32_t> hidx[NURI_MAX_PATTERN - 1];
  uint32_t hidx_hops = 0;
  uint64_t hidx_ns = 0;  // time spent building it

  MemPool pool;  // query workspaces kept between queries

  uint64_t device_bytes() const;
  uint64_t hop_index_bytes() const;
  Graph() = default;
  Graph(const Graph &) = delete;
  Graph &operator=(const Graph &) = delete;
  ~Graph() {
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
};

Graph *load_graph(const nuri_csr *csr, hipStream_t stream);

// builds the multi-hop index of g up to `hops` hops (1..NURI_MAX_PATTERN-1)
// if it is not there yet; synchronous on stream s
void ensure_hop_index(Graph &g, uint32_t hops, hipStream_t s);

// ------------------------------------------------------------------
// results
// ------------------------------------------------------------------
struct Result {
  int error = 0;  // nuri_status of a failed query (served queries only)
  std::string errmsg;
  std::vector<int64_t> score;
  std::vector<uint64_t> offset;
  std::vector<uint32_t> ids;
  nuri_stats stats{};
};

// results of a full top-k whose score equals the k-th's; 0 when fewer than k
inline uint64_t ties_at_k(const std::vector<int64_t> &score, uint32_t k) {
  if (k == 0 || score.size() < k) return 0;
  uint64_t t = 0;
  for (size_t i = score.size(); i-- > 0 && score[i] == score[k - 1];) ++t;
  return t;
}

struct QueryOpts {
  uint64_t frontier_budget = 8ull << 30;
  uint32_t batch_B = 0;
  uint32_t root_batch = 0;
  uint32_t bound = 0;  // 0 auto, 1 Carraghan-Pardalos only, 2 colour classes always
  uint32_t priority = NURI_PRIORITY_DEPTH;
  uint32_t chain_links = 0;  // 0: the engine's default
  uint64_t deadline_ns = 0;
  bool profile = false;
  hipStream_t stream = nullptr;
};
QueryOpts resolve_opts(const Graph &g, const nuri_opts *o);

uint64_t now_ns();

// clique engine: runs several clique queries (each its own k and score)
// together; results in the same order
void run_cliques(Graph &g, const std::vector<uint32_t> &ks, const std::vector<int> &wfs,
                 const QueryOpts &o, std::vector<Result> &out);

// one clique query with every device buffer carved from [base, base + bytes)
void run_clique_fixed(Graph &g, uint32_t k, int kind, const QueryOpts &o, void *base, size_t bytes,
                      Result &out);

// Query slots for continuous batching: queries are admitted into free
// slots between steps, every step serves all live slots, and finished
// slots are harvested.
struct CliqueSlots {
  struct Impl;
  std::unique_ptr<Impl> impl;
  CliqueSlots(Graph &g, const QueryOpts &o, uint32_t slots);
  ~CliqueSlots();
  uint32_t slots() const;
  bool free(uint32_t i) const;
  bool finished(uint32_t i) const;
  bool live() const;
  // starts a query in slot i with a frontier arena of `bytes`; throws on
  // invalid arguments
  void admit(uint32_t i, uint32_t k, int kind, uint64_t bytes);
  bool step();  // false when no slot has work
  void harvest(uint32_t i, Result &r);
  uint64_t min_arena_bytes() const;  // smallest arena a query can start with
};

struct MatchSlots {
  struct Impl;
  std::unique_ptr<Impl> impl;
  MatchSlots(Graph &g, const QueryOpts &o, uint32_t slots);
  ~MatchSlots();
  uint32_t slots() const;
  bool free(uint32_t i) const;
  bool finished(uint32_t i) const;
  bool live() const;
  void admit(uint32_t i, const nuri_pattern &p, uint32_t k, uint64_t bytes);
  bool step();
  void harvest(uint32_t i, Result &r);
  uint64_t min_arena_bytes() const;
};

// top-k frequent patterns with n_edges edges (Algorithm 2)
void run_patterns(Graph &g, uint32_t n_edges, uint32_t k, const QueryOpts &o, Result &out);

// matching engine
void run_matches(Graph &g, const std::vector<const nuri_pattern *> &ps,
                 const std::vector<uint32_t> &ks, const QueryOpts &o, std::vector<Result> &out);

}  // namespace nuri

// the opaque handles of the C ABI
struct nuri_graph {
  nuri::Graph *g;
};
struct nuri_result {
  nuri::Result r;
};
