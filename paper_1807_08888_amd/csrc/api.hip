// C ABI entry points (include/nuri.h): argument checks, handle ownership,
// error codes and the thread-local error message.
#include <algorithm>
#include <cstring>
#include <exception>
#include <new>

#include <memory>

#include "nuri_internal.h"


namespace nuri {

static thread_local std::string t_err;

void set_error(const std::string &msg) { t_err = msg; }

// Default frontier budget: 40% of the free device memory, at most 64 GiB.
static uint64_t default_budget() {
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess || free_b == 0) return 8ull << 30;
  uint64_t b = (uint64_t)(free_b * 0.4);
  b = std::min<uint64_t>(b, 64ull << 30);
  return std::max<uint64_t>(b, 256ull << 20);
}

QueryOpts resolve_opts(const Graph &g, const nuri_opts *o) {
  QueryOpts q;
  q.stream = g.stream;
  q.frontier_budget = default_budget();
  if (!o) return q;
  if (o->frontier_budget_bytes) q.frontier_budget = o->frontier_budget_bytes;
  q.batch_B = o->batch_B;
  q.root_batch = o->root_batch;
  if (o->bound > 2) throw Error{NURI_EINVAL, "bound must be 0, 1 or 2"};
  q.bound = o->bound;
  q.deadline_ns = o->deadline_ns;
  q.profile = o->profile != 0;
  if (o->priority > NURI_PRIORITY_NONE) throw Error{NURI_EINVAL, "priority must be 0..3"};
  q.priority = o->priority;
  q.chain_links = o->chain_links;
  if (o->hip_stream) q.stream = (hipStream_t)o->hip_stream;
  if (q.frontier_budget < (64ull << 20))
    throw Error{NURI_EINVAL, "frontier_budget_bytes must be at least 64 MiB"};
  return q;
}

// Runs f, turning exceptions into status codes and the error message.
template <class F>
static int guarded(F f) {
  try {
    f();
    return NURI_OK;
  } catch (const Error &e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc &) {
    set_error("host allocation failed");
    return NURI_ENOMEM;
  } catch (const std::exception &e) {
    set_error(e.what());
    return NURI_EDEVICE;
  }
}

static void check_pattern(const nuri_pattern *p) {
  if (!p) throw Error{NURI_EINVAL, "pattern is NULL"};
  if (p->q < 2 || p->q > NURI_MAX_PATTERN) throw Error{NURI_EINVAL, "pattern size must be 2..8"};
  if (!p->label || (!p->edges && p->n_edges)) throw Error{NURI_EINVAL, "pattern arrays are NULL"};
}

}  // namespace nuri

using namespace nuri;

extern "C" {

const char *nuri_last_error(void) { return t_err.c_str(); }

int nuri_load_graph(const nuri_csr *csr, void *hip_stream, nuri_graph **out) {
  if (!out) {
    set_error("out is NULL");
    return NURI_EINVAL;
  }
  return guarded([&] {
    Graph *g = load_graph(csr, (hipStream_t)hip_stream);
    *out = new nuri_graph{g};
  });
}

void nuri_free_graph(nuri_graph *g) {
  if (!g) return;
  delete g->g;
  delete g;
}

int nuri_graph_hop_index(nuri_graph *g, uint32_t hops, int32_t *out, uint64_t *build_ns) {
  if (!g) {
    set_error("NULL argument");
    return NURI_EINVAL;
  }
  return guarded([&] {
    Graph &G = *g->g;
    if (hops < 1 || hops > NURI_MAX_PATTERN - 1)
      throw Error{NURI_EINVAL, "hops must be 1..NURI_MAX_PATTERN-1"};
    const uint64_t t0 = now_ns();
    ensure_hop_index(G, hops, G.stream);
    const uint64_t t1 = now_ns();
    if (build_ns) *build_ns = t1 - t0;
    if (!out) return;
    std::lock_guard<std::mutex> lk(G.hidx_mu);
    const size_t per = (size_t)G.n * NURI_MAX_LABELS;
    for (uint32_t h = 0; h < hops; ++h)
      NURI_HIP(hipMemcpyAsync(out + h * per, G.hidx[h].p, per * sizeof(int32_t),
                              hipMemcpyDeviceToHost, G.stream));
    NURI_HIP(hipStreamSynchronize(G.stream));
  });
}

int nuri_graph_get_info(const nuri_graph *g, nuri_graph_info *info) {
  if (!g || !info) {
    set_error("NULL argument");
    return NURI_EINVAL;
  }
  info->n = g->g->n;
  info->nnz = g->g->nnz;
  info->degeneracy = g->g->degeneracy;
  info->bitmap_bytes = g->g->bitmap_words * 8;
  info->device_bytes = g->g->device_bytes();
  info->preprocess_ns = g->g->preprocess_ns;
  info->core_density = g->g->core_density;
  return NURI_OK;
}

int nuri_topk_cliques(nuri_graph *g, uint32_t k, nuri_weight_fn wf, const nuri_opts *o,
                      nuri_result **out) {
  if (!g || !out) {
    set_error("NULL argument");
    return NURI_EINVAL;
  }
  return guarded([&] {
    QueryOpts qo = resolve_opts(*g->g, o);
    std::vector<Result> res;
    run_cliques(*g->g, {k}, {(int)wf}, qo, res);
    auto *r = new nuri_result;
    r->r = std::move(res[0]);
    *out = r;
  });
}

int nuri_topk_patterns(nuri_graph *g, uint32_t n_edges, uint32_t k, const nuri_opts *o,
                       nuri_result **out) {
  if (!g || !out) {
    set_error("NULL argument");
    return NURI_EINVAL;
  }
  return guarded([&] {
    QueryOpts qo = resolve_opts(*g->g, o);
    std::unique_ptr<nuri_result> r(new nuri_result);
    run_patterns(*g->g, n_edges, k, qo, r->r);
    *out = r.release();
  });
}

int nuri_topk_match(nuri_graph *g, const nuri_pattern *p, uint32_t k, const nuri_opts *o,
                    nuri_result **out) {
  if (!g || !out) {
    set_error("NULL argument");
    return NURI_EINVAL;
  }
  return guarded([&] {
    check_pattern(p);
    QueryOpts qo = resolve_opts(*g->g, o);
    std::vector<Result> res;
    run_matches(*g->g, {p}, {k}, qo, res);
    auto *r = new nuri_result;
    r->r = std::move(res[0]);
    *out = r;
  });
}

int nuri_topk_batch(nuri_graph *g, const nuri_query *qs, uint32_t nq, const nuri_opts *o,
                    nuri_result **outs) {
  if (!g || !outs || (!qs && nq)) {
    set_error("NULL argument");
    return NURI_EINVAL;
  }
  return guarded([&] {
    QueryOpts qo = resolve_opts(*g->g, o);
    std::vector<uint32_t> ck, mk;
    std::vector<int> cw;
    std::vector<const nuri_pattern *> mp;
    std::vector<uint32_t> cidx, midx;
    for (uint32_t i = 0; i < nq; ++i) {
      if (qs[i].kind == 0) {
        ck.push_back(qs[i].k);
        cw.push_back((int)qs[i].wf);
        cidx.push_back(i);
      } else if (qs[i].kind == 1) {
        check_pattern(qs[i].p);
        mk.push_back(qs[i].k);
        mp.push_back(qs[i].p);
        midx.push_back(i);
      } else {
        throw Error{NURI_EINVAL, "query kind must be 0 (clique) or 1 (match)"};
      }
    }
    std::vector<Result> cres, mres;
    if (!ck.empty()) run_cliques(*g->g, ck, cw, qo, cres);
    if (!mk.empty()) run_matches(*g->g, mp, mk, qo, mres);
    std::vector<nuri_result *> made(nq, nullptr);
    for (size_t i = 0; i < cidx.size(); ++i) {
      made[cidx[i]] = new nuri_result;
      made[cidx[i]]->r = std::move(cres[i]);
    }
    for (size_t i = 0; i < midx.size(); ++i) {
      made[midx[i]] = new nuri_result;
      made[midx[i]]->r = std::move(mres[i]);
    }
    for (uint32_t i = 0; i < nq; ++i) outs[i] = made[i];
  });
}

int nuri_autotune(nuri_graph *g, const nuri_query *qs, uint32_t nq, const nuri_opts *o,
                  uint32_t rounds, nuri_opts *best) {
  if (!g || !best || !qs || nq == 0 || rounds == 0) {
    set_error("autotune needs a graph, queries, rounds >= 1 and an output");
    return NURI_EINVAL;
  }
  nuri_opts base{};
  if (o) base = *o;
  std::vector<nuri_result *> outs(nq, nullptr);
  auto run = [&](const nuri_opts &x, uint64_t &ns) -> int {
    const uint64_t t0 = now_ns();
    const int rc = nuri_topk_batch(g, qs, nq, &x, outs.data());
    ns = now_ns() - t0;
    if (rc == NURI_OK)
      for (auto *r : outs) nuri_free_result(r);
    return rc;
  };
  uint64_t ns = 0;
  int rc = run(base, ns);  // warm-up (workspace pool, caches)
  if (rc != NURI_OK) return rc;
  static const uint32_t kB[] = {4096, 16384, 32768, 65536};
  static const uint32_t kRoot[] = {2048, 8192};
  uint64_t best_ns = UINT64_MAX;
  nuri_opts pick = base;
  for (uint32_t b : kB)
    for (uint32_t rb : kRoot) {
      nuri_opts x = base;
      x.batch_B = b;
      x.root_batch = rb;
      uint64_t t = UINT64_MAX;
      for (uint32_t i = 0; i < rounds; ++i) {
        rc = run(x, ns);
        if (rc != NURI_OK) return rc;
        t = std::min(t, ns);
      }
      if (t < best_ns) {
        best_ns = t;
        pick = x;
      }
    }
  *best = pick;
  return NURI_OK;
}

int nuri_result_view_get(const nuri_result *r, nuri_result_view *v) {
  if (!r || !v) {
    set_error("NULL argument");
    return NURI_EINVAL;
  }
  v->count = (uint32_t)r->r.score.size();
  v->score = r->r.score.data();
  v->offset = r->r.offset.data();
  v->ids = r->r.ids.data();
  return NURI_OK;
}

int nuri_result_stats(const nuri_result *r, nuri_stats *s) {
  if (!r || !s) {
    set_error("NULL argument");
    return NURI_EINVAL;
  }
  *s = r->r.stats;
  return NURI_OK;
}

void nuri_free_result(nuri_result *r) { delete r; }

}  // extern "C"
