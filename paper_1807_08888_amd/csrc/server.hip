// Continuous-batching server over one resident graph.
//
// The paper's communication component takes a computation from the user
// and returns its result set (Section 5); here many computations are live
// at once.  A worker thread owns two slot engines (cliques, matching), each
// holding up to max_slots live queries.  All live queries draw their
// frontier arenas from one budget: a queued query is admitted, in arrival
// order, when a slot of its kind is free and its arena fits in what the
// budget has left (a query waiting for memory holds back the ones behind
// it, so a large query is not starved).  A query starts with a base arena
// (the budget over twice the slot count); one that outgrows its arena is
// started again with twice the arena, up to the whole budget, so a served
// result is exact whenever the budget can hold the search at all.  Every
// step serves all live queries of each engine -- their work shares every
// launch -- and finished slots are harvested.  A query's result does not
// depend on what else is in flight: every search is exact.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>
#include <unordered_map>

#include "nuri_internal.h"


namespace nuri {

struct Served {
  uint64_t ticket = 0;
  uint32_t kind = 0, k = 0;
  int wf = 0;
  std::vector<uint8_t> labels;
  std::vector<uint32_t> edges;
  uint32_t mscore = 0;  // nuri_match_score
  uint64_t t_submit = 0;
  uint64_t arena = 0;     // frontier bytes to admit it with (0: the base arena)
  uint32_t restarts = 0;  // times it outgrew its arena and was started again
};

struct Server {
  Graph *g = nullptr;
  QueryOpts opts;
  uint32_t max_slots = 0;
  std::unique_ptr<CliqueSlots> cs;
  std::unique_ptr<MatchSlots> ms;
  std::vector<uint64_t> c_ticket, m_ticket;      // ticket per slot (0 = free)
  std::vector<Served> c_query, m_query;          // the query in each slot
  uint64_t budget = 0, used = 0;                 // frontier bytes: total, held by live queries
  uint64_t base_arena = 0;
  std::unordered_map<uint64_t, uint64_t> submit_t;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Served> queue;
  std::unordered_map<uint64_t, Result> done;
  uint64_t next_ticket = 1;
  bool stop = false;
  int fatal = 0;
  std::string fatal_msg;
  std::thread worker;

  void finish(uint64_t ticket, Result &&r) {
    std::lock_guard<std::mutex> lk(mu);
    auto it = submit_t.find(ticket);
    if (it != submit_t.end()) {
      r.stats.wall_ns = now_ns() - it->second;  // completion - arrival
      submit_t.erase(it);
    }
    done.emplace(ticket, std::move(r));
  }

  void fail_ticket(uint64_t ticket, int code, const std::string &msg) {
    Result r;
    r.error = code;
    r.errmsg = msg;
    r.offset.assign(1, 0);
    finish(ticket, std::move(r));
  }

  uint64_t arena_of(const Served &q) const {
    const uint64_t lo = q.kind == 0 ? cs->min_arena_bytes() : ms->min_arena_bytes();
    return std::min<uint64_t>(budget, std::max<uint64_t>(q.arena ? q.arena : base_arena, lo));
  }

  // move queued queries into free slots, in arrival order: a query is
  // admitted when a slot of its kind is free and its arena fits in the
  // budget; the first query that waits for memory stops the scan
  void admit() {
    std::deque<Served> take;
    {
      std::lock_guard<std::mutex> lk(mu);
      uint32_t cfree = 0, mfree = 0;
      for (auto t : c_ticket) cfree += t == 0;
      for (auto t : m_ticket) mfree += t == 0;
      std::deque<Served> keep;
      bool blocked = false;
      while (!queue.empty()) {
        Served q = std::move(queue.front());
        queue.pop_front();
        const bool slot = q.kind == 0 ? cfree > 0 : mfree > 0;
        const uint64_t need = (q.kind == 1 && !ms) ? 0 : arena_of(q);
        if (!blocked && slot && used + need <= budget) {
          (q.kind == 0 ? cfree : mfree)--;
          used += need;
          q.arena = need;
          take.push_back(std::move(q));
        } else {
          if (slot) blocked = true;  // waits for memory: nothing overtakes it
          keep.push_back(std::move(q));
        }
      }
      queue.swap(keep);
    }
    for (auto &q : take) {
      try {
        if (q.kind == 0) {
          uint32_t i = 0;
          while (c_ticket[i]) ++i;
          cs->admit(i, q.k, q.wf, q.arena);
          c_ticket[i] = q.ticket;
          c_query[i] = q;
        } else {
          if (!ms) throw Error{NURI_EINVAL, "labelled matching needs vertex labels"};
          uint32_t i = 0;
          while (m_ticket[i]) ++i;
          nuri_pattern p{(uint32_t)q.labels.size(), (uint32_t)(q.edges.size() / 2),
                         q.labels.data(), q.edges.data(), q.mscore};
          ms->admit(i, p, q.k, q.arena);
          m_ticket[i] = q.ticket;
          m_query[i] = q;
        }
      } catch (const Error &e) {
        if (e.code == NURI_EINVAL) {
          used -= q.arena;
          fail_ticket(q.ticket, e.code, e.msg);
        } else {
          throw;
        }
      }
    }
  }

  // a finished slot: its arena returns to the budget; a query that outgrew
  // its arena goes back to the head of the queue with twice the arena
  void settle(Served &q, Result &&r) {
    used -= q.arena;
    if (r.error == NURI_EBUDGET && q.arena < budget) {
      q.arena = std::min<uint64_t>(budget, 2 * q.arena);
      q.restarts++;
      std::lock_guard<std::mutex> lk(mu);
      queue.push_front(std::move(q));
      return;
    }
    r.stats.restarts = q.restarts;
    finish(q.ticket, std::move(r));
  }

  void harvest() {
    for (uint32_t i = 0; i < c_ticket.size(); ++i)
      if (c_ticket[i] && cs->finished(i)) {
        Result r;
        cs->harvest(i, r);
        c_ticket[i] = 0;
        settle(c_query[i], std::move(r));
      }
    for (uint32_t i = 0; i < m_ticket.size(); ++i)
      if (m_ticket[i] && ms->finished(i)) {
        Result r;
        ms->harvest(i, r);
        m_ticket[i] = 0;
        settle(m_query[i], std::move(r));
      }
  }

  bool busy() const {
    for (auto t : c_ticket)
      if (t) return true;
    for (auto t : m_ticket)
      if (t) return true;
    return false;
  }

  void loop() {
    try {
      for (;;) {
        {
          std::unique_lock<std::mutex> lk(mu);
          cv.wait(lk, [&] { return stop || !queue.empty() || busy(); });
          if (stop) return;
        }
        admit();
        if (cs && cs->live()) cs->step();
        if (ms && ms->live()) ms->step();
        harvest();
      }
    } catch (const Error &e) {
      fail_all(e.code, e.msg);
    } catch (const std::exception &e) {
      fail_all(NURI_EDEVICE, e.what());
    }
  }

  // a device error ends the server: every pending and live query fails
  void fail_all(int code, const std::string &msg) {
    std::vector<uint64_t> tickets;
    {
      std::lock_guard<std::mutex> lk(mu);
      fatal = code;
      fatal_msg = msg;
      for (auto &q : queue) tickets.push_back(q.ticket);
      queue.clear();
    }
    for (auto t : c_ticket)
      if (t) tickets.push_back(t);
    for (auto t : m_ticket)
      if (t) tickets.push_back(t);
    for (auto t : tickets) fail_ticket(t, code, msg);
  }
};

}  // namespace nuri

using namespace nuri;

struct nuri_server {
  nuri::Server s;
};

extern "C" {

int nuri_server_create(nuri_graph *g, uint64_t frontier_budget_bytes, uint32_t max_slots,
                       nuri_server **out) {
  if (!g || !out || max_slots == 0 || max_slots > 4096) {
    set_error("server needs a graph, an out pointer and 1..4096 slots");
    return NURI_EINVAL;
  }
  try {
    nuri_opts o{};
    o.frontier_budget_bytes = frontier_budget_bytes;
    QueryOpts qo = resolve_opts(*g->g, &o);
    auto *srv = new nuri_server;
    Server &S = srv->s;
    S.g = g->g;
    S.opts = qo;
    S.max_slots = max_slots;
    // one frontier budget shared by all live queries of both engines
    S.budget = qo.frontier_budget;
    S.base_arena = qo.frontier_budget / (2ull * max_slots);
    try {
      S.cs.reset(new CliqueSlots(*g->g, qo, max_slots));
      if (g->g->has_lab) S.ms.reset(new MatchSlots(*g->g, qo, max_slots));
    } catch (...) {
      delete srv;
      throw;
    }
    S.c_ticket.assign(max_slots, 0);
    S.m_ticket.assign(S.ms ? max_slots : 0, 0);
    S.c_query.assign(max_slots, Served{});
    S.m_query.assign(S.ms ? max_slots : 0, Served{});
    S.worker = std::thread([&S] { S.loop(); });
    *out = srv;
    return NURI_OK;
  } catch (const Error &e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::exception &e) {
    set_error(e.what());
    return NURI_EDEVICE;
  }
}

int nuri_server_submit(nuri_server *srv, const nuri_query *q, uint64_t *ticket) {
  if (!srv || !q || !ticket) {
    set_error("NULL argument");
    return NURI_EINVAL;
  }
  Server &S = srv->s;
  Served item;
  item.kind = q->kind;
  item.k = q->k;
  item.wf = (int)q->wf;
  if (q->kind == 1) {
    if (!q->p || !q->p->label || (!q->p->edges && q->p->n_edges) || q->p->q > NURI_MAX_PATTERN) {
      set_error("bad pattern");
      return NURI_EINVAL;
    }
    item.labels.assign(q->p->label, q->p->label + q->p->q);
    item.edges.assign(q->p->edges, q->p->edges + 2 * q->p->n_edges);
    item.mscore = q->p->score;
  } else if (q->kind != 0) {
    set_error("query kind must be 0 (clique) or 1 (match)");
    return NURI_EINVAL;
  }
  if (q->kind == 1 && !S.ms) {
    // no matching engine (and no slot) exists for a graph without labels
    set_error("labelled matching needs vertex labels");
    return NURI_EINVAL;
  }
  {
    std::lock_guard<std::mutex> lk(S.mu);
    if (S.fatal) {
      set_error("server stopped after an error: " + S.fatal_msg);
      return S.fatal;
    }
    item.ticket = S.next_ticket++;
    item.t_submit = now_ns();
    S.submit_t[item.ticket] = item.t_submit;
    *ticket = item.ticket;
    S.queue.push_back(std::move(item));
  }
  S.cv.notify_one();
  return NURI_OK;
}

int nuri_server_poll(nuri_server *srv, uint64_t ticket, nuri_result **out) {
  if (!srv || !out) {
    set_error("NULL argument");
    return NURI_EINVAL;
  }
  Server &S = srv->s;
  std::lock_guard<std::mutex> lk(S.mu);
  auto it = S.done.find(ticket);
  if (it == S.done.end()) {
    if (ticket == 0 || ticket >= S.next_ticket) {
      set_error("unknown ticket");
      return NURI_EINVAL;
    }
    // a ticket is pending until finish() moves it from submit_t to done
    if (!S.submit_t.count(ticket)) {
      set_error("ticket already collected");
      return NURI_EINVAL;
    }
    return 0;
  }
  Result r = std::move(it->second);
  S.done.erase(it);
  if (r.error) {
    set_error(r.errmsg);
    return r.error;
  }
  auto *res = new nuri_result;
  res->r = std::move(r);
  *out = res;
  return 1;
}

void nuri_server_destroy(nuri_server *srv) {
  if (!srv) return;
  Server &S = srv->s;
  {
    std::lock_guard<std::mutex> lk(S.mu);
    S.stop = true;
  }
  S.cv.notify_all();
  if (S.worker.joinable()) S.worker.join();
  delete srv;
}

}  // extern "C"
