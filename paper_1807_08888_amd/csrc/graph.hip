// Graph residency and preprocessing: validation, degeneracy order, the
// rank-space CSR, per-vertex dense local adjacency bitmaps, bound tables
// and root orders.  Runs once per graph (Section 5: the data graph is
// loaded into memory for the computations); queries only read what is
// built here.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <numeric>
#include <thread>

#include "nuri_internal.h"

namespace nuri {

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Runs f(begin, end) over [0, n) split into contiguous chunks on host threads.
template <class F>
static void parallel_chunks(uint64_t n, F f) {
  unsigned t = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 65536 || t == 1) {
    f(0, n);
    return;
  }
  std::vector<std::thread> th;
  uint64_t per = (n + t - 1) / t;
  for (unsigned i = 0; i < t; ++i) {
    uint64_t b = i * per, e = std::min(n, b + per);
    if (b >= e) break;
    th.emplace_back([=] { f(b, e); });
  }
  for (auto &x : th) x.join();
}

static void fail(const std::string &m) { throw Error{NURI_EINVAL, m}; }

// ------------------------------------------------------------------
// validation (the input is rejected, never repaired)
// ------------------------------------------------------------------
static void validate(const nuri_csr &c) {
  if (c.n == 0) fail("graph has no vertices");
  if (!c.row_ptr || (!c.col_idx && c.nnz)) fail("row_ptr/col_idx must be non-NULL");
  if (c.row_ptr[0] != 0) fail("row_ptr[0] must be 0");
  if (c.row_ptr[c.n] != c.nnz) fail("row_ptr[n] must equal nnz");
  for (uint32_t v = 0; v < c.n; ++v)
    if (c.row_ptr[v + 1] < c.row_ptr[v]) fail("row_ptr must be non-decreasing");
  std::atomic<int> bad{0};
  std::string why[4] = {"", "column id out of range", "self loop", "row not strictly increasing"};
  parallel_chunks(c.n, [&](uint64_t b, uint64_t e) {
    for (uint64_t v = b; v < e && !bad.load(); ++v)
      for (uint64_t k = c.row_ptr[v]; k < c.row_ptr[v + 1]; ++k) {
        uint32_t u = c.col_idx[k];
        if (u >= c.n) { bad = 1; return; }
        if (u == v) { bad = 2; return; }
        if (k > c.row_ptr[v] && c.col_idx[k - 1] >= u) { bad = 3; return; }
      }
  });
  if (bad) fail(why[bad.load()]);
  // symmetry, and equal weights in both directions
  parallel_chunks(c.n, [&](uint64_t b, uint64_t e) {
    for (uint64_t v = b; v < e && !bad.load(); ++v)
      for (uint64_t k = c.row_ptr[v]; k < c.row_ptr[v + 1]; ++k) {
        uint32_t u = c.col_idx[k];
        const uint32_t *lo = c.col_idx + c.row_ptr[u], *hi = c.col_idx + c.row_ptr[u + 1];
        const uint32_t *it = std::lower_bound(lo, hi, (uint32_t)v);
        if (it == hi || *it != v) { bad = 1; return; }
        if (c.edge_weight) {
          int32_t w = c.edge_weight[k];
          if (w < 1 || c.edge_weight[it - c.col_idx] != w) { bad = 2; return; }
        }
      }
  });
  if (bad == 1) fail("adjacency is not symmetric");
  if (bad == 2) fail("edge weights must be >= 1 and equal in both directions");
  if (c.vertex_weight)
    for (uint32_t v = 0; v < c.n; ++v)
      if (c.vertex_weight[v] < 1) fail("vertex weights must be >= 1");
  if (c.vertex_label)
    for (uint32_t v = 0; v < c.n; ++v)
      if (c.vertex_label[v] >= NURI_MAX_LABELS) fail("vertex label out of range");
}

// ------------------------------------------------------------------
// degeneracy order (bucket peeling: repeatedly remove a vertex of minimum
// remaining degree), O(n + m)
// ------------------------------------------------------------------
static std::vector<uint32_t> degeneracy_order(const nuri_csr &c) {
  uint32_t n = c.n;
  std::vector<uint32_t> deg(n), bin, pos(n), vert(n);
  uint32_t md = 0;
  for (uint32_t v = 0; v < n; ++v) {
    deg[v] = (uint32_t)(c.row_ptr[v + 1] - c.row_ptr[v]);
    md = std::max(md, deg[v]);
  }
  bin.assign(md + 1, 0);
  for (uint32_t v = 0; v < n; ++v) bin[deg[v]]++;
  uint32_t start = 0;
  for (uint32_t d = 0; d <= md; ++d) {
    uint32_t k = bin[d];
    bin[d] = start;
    start += k;
  }
  for (uint32_t v = 0; v < n; ++v) {
    pos[v] = bin[deg[v]];
    vert[pos[v]] = v;
    bin[deg[v]]++;
  }
  for (uint32_t d = md; d >= 1; --d) bin[d] = bin[d - 1];
  bin[0] = 0;
  for (uint32_t i = 0; i < n; ++i) {
    uint32_t v = vert[i];
    for (uint64_t k = c.row_ptr[v]; k < c.row_ptr[v + 1]; ++k) {
      uint32_t u = c.col_idx[k];
      if (deg[u] > deg[v]) {
        uint32_t du = deg[u], pu = pos[u], pw = bin[du], w = vert[pw];
        if (u != w) {
          pos[u] = pw;
          vert[pu] = w;
          pos[w] = pu;
          vert[pw] = u;
        }
        bin[du]++;
        deg[u]--;
      }
    }
  }
  return vert;  // vert[i] = vertex removed i-th
}

// ------------------------------------------------------------------
// local bitmap construction
// ------------------------------------------------------------------
// One workgroup per root r (with |N+(r)| >= 2).  N+(r) is staged in LDS;
// each wave takes local rows i and, for every x in N+(u) (u = N+(r)[i]),
// binary-searches x among N+(r)[i+1..d).  A hit at position j is the edge
// {u, N+(r)[j]}: bits (i, j) and (j, i) are set.
__global__ void __launch_bounds__(256) k_build_bitmaps(
    const uint32_t *__restrict__ roots, const uint64_t *__restrict__ rrow,
    const uint32_t *__restrict__ rcol, const uint32_t *__restrict__ split,
    const uint32_t *__restrict__ dplus, const uint64_t *__restrict__ bm_off,
    unsigned long long *__restrict__ bm) {
  __shared__ uint32_t loc[kMaxLocal];
  uint32_t r = roots[blockIdx.x];
  uint32_t d = dplus[r];
  const uint32_t *np = rcol + rrow[r] + split[r];
  for (uint32_t t = threadIdx.x; t < d; t += blockDim.x) loc[t] = np[t];
  __syncthreads();
  uint32_t W = (d + 63) >> 6;
  unsigned long long *base = bm + bm_off[r];
  uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  for (uint32_t i = wave; i < d; i += nw) {
    uint32_t u = loc[i];
    const uint32_t *up = rcol + rrow[u] + split[u];
    uint32_t du = dplus[u];
    for (uint32_t t = lane; t < du; t += 64) {
      uint32_t x = up[t];
      // first position > i holding a value >= x
      uint32_t lo = i + 1, hi = d;
      while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (loc[mid] < x) lo = mid + 1; else hi = mid;
      }
      if (lo < d && loc[lo] == x) {
        uint32_t j = lo;
        atomicOr(&base[(uint64_t)i * W + (j >> 6)], 1ull << (j & 63));
        atomicOr(&base[(uint64_t)j * W + (i >> 6)], 1ull << (i & 63));
      }
    }
  }
}

uint64_t Graph::device_bytes() const {
  return rrow.bytes() + rcol.bytes() + split.bytes() + dplus.bytes() + hrow.bytes() +
         hcol.bytes() + leaf_wit.bytes() + orig.bytes() + vw.bytes() +
         bm_off.bytes() + bm.bytes() + wplus.bytes() + best.bytes() +
         orow.bytes() + lcol.bytes() + lew.bytes() + loff.bytes() + lab_vert.bytes() +
         vlab.bytes() +
         root_order[0].bytes() + root_order[1].bytes() + ooff.bytes() + oplus.bytes() +
         wloc.bytes() + hop_index_bytes();
}

uint64_t Graph::hop_index_bytes() const {
  uint64_t b = 0;
  for (const auto &h : hidx) b += h.bytes();
  return b;
}

template <class T>
static void upload(DevBuf<T> &d, const T *h, size_t n, hipStream_t s) {
  d.alloc(n);
  if (n) {
    NURI_HIP(hipMemcpyAsync(d.p, h, n * sizeof(T), hipMemcpyHostToDevice, s));
    NURI_HIP(hipStreamSynchronize(s));  // the host vector may go out of scope next
  }
}

Graph *load_graph(const nuri_csr *csr, hipStream_t stream) {
  if (!csr) fail("csr is NULL");
  uint64_t t0 = now_ns();
  const nuri_csr &c = *csr;
  validate(c);
  auto G = std::make_unique<Graph>();
  Graph &g = *G;
  g.n = c.n;
  g.nnz = c.nnz;
  g.has_vw = c.vertex_weight != nullptr;
  g.has_lab = c.vertex_label != nullptr;
  g.has_ew = c.edge_weight != nullptr;
  if (stream) {
    g.stream = stream;
  } else {
    NURI_HIP(hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking));
    g.own_stream = true;
  }
  uint32_t n = c.n;

  // order and relabelling
  g.h_orig = degeneracy_order(c);
  g.h_rank.resize(n);
  for (uint32_t i = 0; i < n; ++i) g.h_rank[g.h_orig[i]] = i;

  std::vector<uint64_t> rrow(n + 1, 0);
  for (uint32_t r = 0; r < n; ++r) {
    uint32_t v = g.h_orig[r];
    rrow[r + 1] = rrow[r] + (c.row_ptr[v + 1] - c.row_ptr[v]);
  }
  std::vector<uint32_t> rcol(c.nnz), split(n), dplus(n);
  parallel_chunks(n, [&](uint64_t b, uint64_t e) {
    std::vector<uint32_t> tmp;
    for (uint64_t r = b; r < e; ++r) {
      uint32_t v = g.h_orig[r];
      uint64_t k0 = c.row_ptr[v], k1 = c.row_ptr[v + 1];
      tmp.clear();
      for (uint64_t k = k0; k < k1; ++k) tmp.push_back(g.h_rank[c.col_idx[k]]);
      std::sort(tmp.begin(), tmp.end());
      uint64_t o = rrow[r];
      uint32_t s = 0;
      for (size_t i = 0; i < tmp.size(); ++i) {
        rcol[o + i] = tmp[i];
        if (tmp[i] < r) ++s;
      }
      split[r] = s;
      dplus[r] = (uint32_t)tmp.size() - s;
    }
  });
  g.h_dplus = dplus;
  g.degeneracy = n ? *std::max_element(dplus.begin(), dplus.end()) : 0;
  std::vector<uint64_t> hrow(n + 1, 0);
  for (uint32_t r = 0; r < n; ++r) {
    uint64_t h = 0;
    for (uint64_t k = rrow[r]; k < rrow[r] + split[r]; ++k) h += dplus[rcol[k]] >= kHeavy;
    hrow[r + 1] = hrow[r] + h;
  }
  std::vector<uint32_t> hcol(hrow[n]);
  parallel_chunks(n, [&](uint64_t b, uint64_t e) {
    for (uint64_t r = b; r < e; ++r) {
      uint64_t o = hrow[r];
      for (uint64_t k = rrow[r]; k < rrow[r] + split[r]; ++k)
        if (dplus[rcol[k]] >= kHeavy) hcol[o++] = rcol[k];
    }
  });
  if (g.degeneracy > kMaxLocal)
    fail("degeneracy " + std::to_string(g.degeneracy) + " exceeds the supported maximum 4096");

  std::vector<uint64_t> bm_off(n + 1, 0);
  for (uint32_t r = 0; r < n; ++r) {
    uint64_t d = dplus[r];
    bm_off[r + 1] = bm_off[r] + d * ((d + 63) / 64);
  }
  g.bitmap_words = bm_off[n];

  std::vector<int32_t> vwr(n, 1);
  if (c.vertex_weight)
    for (uint32_t r = 0; r < n; ++r) vwr[r] = c.vertex_weight[g.h_orig[r]];
  std::vector<int64_t> wplus(n, 0);
  std::vector<uint64_t> ooff(n + 1, 0);
  for (uint32_t r = 0; r < n; ++r) ooff[r + 1] = ooff[r] + dplus[r];
  std::vector<uint32_t> oplus(ooff[n]);
  std::vector<int32_t> wloc(ooff[n]);
  for (uint32_t r = 0; r < n; ++r) {
    int64_t s = 0;
    uint64_t o = ooff[r];
    for (uint64_t k = rrow[r] + split[r]; k < rrow[r + 1]; ++k, ++o) {
      s += vwr[rcol[k]];
      oplus[o] = rcol[k];
      wloc[o] = vwr[rcol[k]];
    }
    wplus[r] = s;
  }
  g.h_label_count.assign(NURI_MAX_LABELS, 0);
  if (c.vertex_label)
    for (uint32_t v = 0; v < n; ++v) g.h_label_count[c.vertex_label[v]]++;
  // 1-hop index for matching (the one-hop form of the per-vertex index of
  // Section 4.3, Listing 3): best[v][l] = max weight of an edge from v to a
  // label-l vertex; pairmax[l1][l2] = max weight over edges with that label
  // pair.  Rows re-sorted by (label, id) give each label's neighbours as
  // one sorted segment.
  std::vector<int32_t> best(c.vertex_label ? (size_t)n * NURI_MAX_LABELS : 0, 0);
  std::vector<uint32_t> lcol(c.vertex_label ? c.nnz : 0), loff(c.vertex_label ? (size_t)n * 17 : 0);
  std::vector<int32_t> lew(c.vertex_label ? c.nnz : 0);
  std::vector<uint32_t> lab_vert;
  g.h_pairmax.assign(NURI_MAX_LABELS * NURI_MAX_LABELS, 0);
  g.h_lab_off.assign(NURI_MAX_LABELS + 1, 0);
  if (c.vertex_label) {
    const uint8_t *L = c.vertex_label;
    parallel_chunks(n, [&](uint64_t b, uint64_t e) {
      std::vector<std::pair<uint64_t, int32_t>> tmp;
      for (uint64_t v = b; v < e; ++v) {
        uint64_t k0 = c.row_ptr[v], k1 = c.row_ptr[v + 1];
        tmp.clear();
        for (uint64_t k = k0; k < k1; ++k) {
          uint32_t u = c.col_idx[k];
          tmp.emplace_back(((uint64_t)L[u] << 32) | u, c.edge_weight ? c.edge_weight[k] : 1);
        }
        std::sort(tmp.begin(), tmp.end());
        uint32_t *lo = &loff[v * 17];
        for (int l = 0; l <= NURI_MAX_LABELS; ++l) lo[l] = 0;
        for (size_t i = 0; i < tmp.size(); ++i) {
          uint32_t u = (uint32_t)tmp[i].first, lu = (uint32_t)(tmp[i].first >> 32);
          lcol[k0 + i] = u;
          lew[k0 + i] = tmp[i].second;
          lo[lu + 1]++;
          int32_t &bb = best[v * NURI_MAX_LABELS + lu];
          if (tmp[i].second > bb) bb = tmp[i].second;
        }
        for (int l = 0; l < NURI_MAX_LABELS; ++l) lo[l + 1] += lo[l];
      }
    });
    for (uint32_t v = 0; v < n; ++v)
      for (int l = 0; l < NURI_MAX_LABELS; ++l) {
        int32_t w = best[(size_t)v * NURI_MAX_LABELS + l];
        int32_t &pm = g.h_pairmax[L[v] * NURI_MAX_LABELS + l];
        if (w > pm) pm = w;
      }
    for (uint32_t v = 0; v < n; ++v) g.h_lab_off[L[v] + 1]++;
    for (int l = 0; l < NURI_MAX_LABELS; ++l) g.h_lab_off[l + 1] += g.h_lab_off[l];
    lab_vert.resize(n);
    std::vector<uint64_t> fill(g.h_lab_off.begin(), g.h_lab_off.end() - 1);
    for (uint32_t v = 0; v < n; ++v) lab_vert[fill[L[v]]++] = v;
  }
  // root orders by bound, descending (ties: smaller rank first)
  for (int kind = 0; kind < 2; ++kind) {
    std::vector<int64_t> bnd(n);
    for (uint32_t r = 0; r < n; ++r)
      bnd[r] = kind == 0 ? 1 + (int64_t)dplus[r] : (int64_t)vwr[r] + wplus[r];
    std::vector<uint32_t> ord(n);
    std::iota(ord.begin(), ord.end(), 0u);
    std::stable_sort(ord.begin(), ord.end(),
                     [&](uint32_t a, uint32_t b) { return bnd[a] > bnd[b]; });
    g.h_root_bound[kind].resize(n);
    for (uint32_t i = 0; i < n; ++i) g.h_root_bound[kind][i] = bnd[ord[i]];
    g.h_root_order[kind] = std::move(ord);
  }

  hipStream_t s = g.stream;
  upload(g.rrow, rrow.data(), n + 1, s);
  upload(g.rcol, rcol.data(), rcol.size(), s);
  upload(g.split, split.data(), n, s);
  upload(g.dplus, dplus.data(), n, s);
  upload(g.hrow, hrow.data(), n + 1, s);
  if (hcol.empty()) hcol.push_back(0);  // keep the device pointer valid
  upload(g.hcol, hcol.data(), hcol.size(), s);
  g.leaf_wit.alloc(n);
  NURI_HIP(hipMemsetAsync(g.leaf_wit.p, 0xFF, (size_t)n * sizeof(uint32_t), s));
  upload(g.orig, g.h_orig.data(), n, s);
  upload(g.vw, vwr.data(), n, s);
  upload(g.bm_off, bm_off.data(), n + 1, s);
  upload(g.wplus, wplus.data(), n, s);
  upload(g.ooff, ooff.data(), n + 1, s);
  upload(g.oplus, oplus.data(), oplus.size(), s);
  upload(g.wloc, wloc.data(), wloc.size(), s);
  if (c.vertex_label) {
    upload(g.orow, c.row_ptr, (size_t)n + 1, s);
    upload(g.lcol, lcol.data(), lcol.size(), s);
    upload(g.lew, lew.data(), lew.size(), s);
    upload(g.loff, loff.data(), loff.size(), s);
    upload(g.best, best.data(), best.size(), s);
    upload(g.lab_vert, lab_vert.data(), lab_vert.size(), s);
    upload(g.vlab, c.vertex_label, (size_t)n, s);
  }
  for (int kind = 0; kind < 2; ++kind)
    upload(g.root_order[kind], g.h_root_order[kind].data(), n, s);
  g.bm.alloc(g.bitmap_words);
  NURI_HIP(hipMemsetAsync(g.bm.p, 0, g.bm.bytes(), s));
  std::vector<uint32_t> broots;
  for (uint32_t r = 0; r < n; ++r)
    if (dplus[r] >= 2) broots.push_back(r);
  if (!broots.empty()) {
    DevBuf<uint32_t> d_broots;
    upload(d_broots, broots.data(), broots.size(), s);
    // grid.x is limited to 2^31-1 blocks; n < 2^32 roots fits in chunks
    const uint32_t chunk = 1u << 30;
    for (size_t b = 0; b < broots.size(); b += chunk) {
      uint32_t cnt = (uint32_t)std::min<size_t>(chunk, broots.size() - b);
      hipLaunchKernelGGL(k_build_bitmaps, dim3(cnt), dim3(256), 0, s, d_broots.p + b,
                         g.rrow.p, g.rcol.p, g.split.p, g.dplus.p, g.bm_off.p,
                         (unsigned long long *)g.bm.p);
      NURI_HIP(hipGetLastError());
    }
    NURI_HIP(hipStreamSynchronize(s));
  }
  NURI_HIP(hipStreamSynchronize(s));
  // density of the largest local universes (up to 8 roots): a near-clique
  // dense region is where colour classes cannot beat |P|
  {
    std::vector<uint32_t> top(n);
    std::iota(top.begin(), top.end(), 0u);
    const size_t nt = std::min<size_t>(8, n);
    std::partial_sort(top.begin(), top.begin() + nt, top.end(),
                      [&](uint32_t a, uint32_t b) { return dplus[a] > dplus[b]; });
    double edges = 0, pairs = 0;
    for (size_t t = 0; t < nt; ++t) {
      const uint32_t r = top[t];
      const uint64_t d = dplus[r];
      if (d < 2) continue;
      std::vector<uint64_t> rows(bm_off[r + 1] - bm_off[r]);
      NURI_HIP(hipMemcpy(rows.data(), g.bm.p + bm_off[r], rows.size() * 8, hipMemcpyDeviceToHost));
      for (uint64_t w : rows) edges += __builtin_popcountll(w);
      pairs += (double)d * (double)(d - 1);
    }
    g.core_density = pairs > 0 ? edges / pairs : 0.0;
  }
  g.preprocess_ns = now_ns() - t0;
  return G.release();
}

}  // namespace nuri
