"""Serving: continuous batching must not change any result.

Queries are submitted to a server with fewer slots than queries (so most
wait and are admitted while others run) and in staggered waves; every
served result must equal the same query run alone, and the oracle.
"""
import time

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nuri():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1807_08888_amd import nuri as N
    N.lib()
    return N


def _case(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def workload(nuri):
    g = synth.rmat(13)
    synth.add_vertex_weights(g)
    synth.add_edge_weights(g)
    synth.add_zipf_labels(g)
    queries = []
    for i in range(18):
        queries.append({"kind": "clique", "k": synth.log_uniform_k(i, 200), "weight_fn": i % 2})
    for i in range(12):
        p = synth.random_pattern(i, q_lo=3, q_hi=6)
        queries.append({"kind": "match", "k": 10 + (i * 7) % 50, "labels": p.labels,
                        "edges": p.edges})
    G = nuri.Graph.from_synth(g)
    yield g, G, queries
    G.close()


def _alone(nuri, G, q):
    if q["kind"] == "clique":
        return nuri.topk_cliques(G, q["k"], q["weight_fn"]).items
    return nuri.topk_match(G, q["labels"], q["edges"], q["k"]).items


def _wait(nuri, S, tickets, timeout=90.0):
    out = {}
    t0 = last = time.time()
    while len(out) < len(tickets):
        if time.time() - last > 10:
            last = time.time()
            print(f"[wait] {len(tickets) - len(out)} pending after {last - t0:.0f} s", flush=True)
        for t in tickets:
            if t in out:
                continue
            r = S.poll(t)
            if r is not None:
                out[t] = r
        if time.time() - t0 > timeout:
            raise TimeoutError(f"{len(tickets) - len(out)} queries still pending")
        time.sleep(0.002)
    return out


def test_served_equals_alone_and_oracle(nuri, workload):
    g, G, queries = workload
    _case("server: 30 mixed queries, 4 slots per engine")
    alone = [_alone(nuri, G, q) for q in queries]
    S = nuri.Server(G, frontier_budget_bytes=4 << 30, max_slots=4)
    try:
        tickets = [S.submit(q) for q in queries]
        res = _wait(nuri, S, tickets)
    finally:
        S.close()
    for i, t in enumerate(tickets):
        assert res[t].items == alone[i], i
        assert res[t].stats["wall_ns"] > 0
    for i in (0, 1, 18, 19):
        q = queries[i]
        if q["kind"] == "clique":
            want, _ = oracle.topk_cliques(g, q["k"], weighted=bool(q["weight_fn"]))
        else:
            want, _ = oracle.topk_match(g, q["labels"], q["edges"], q["k"])
        assert alone[i] == want, i


def test_staggered_arrivals(nuri, workload):
    g, G, queries = workload
    _case("server: staggered arrivals")
    alone = {i: _alone(nuri, G, queries[i]) for i in range(0, len(queries), 3)}
    S = nuri.Server(G, frontier_budget_bytes=4 << 30, max_slots=2)
    try:
        tickets = {}
        for i in sorted(alone):
            tickets[i] = S.submit(queries[i])
            time.sleep(0.003)  # later queries arrive while earlier ones run
        res = _wait(nuri, S, list(tickets.values()))
    finally:
        S.close()
    for i, t in tickets.items():
        assert res[t].items == alone[i], i


def test_invalid_query_fails_alone(nuri, workload):
    g, G, queries = workload
    _case("server: invalid query among valid ones")
    S = nuri.Server(G, frontier_budget_bytes=2 << 30, max_slots=2)
    try:
        good = S.submit(queries[0])
        bad = S.submit({"kind": "clique", "k": 0, "weight_fn": 0})
        bad2 = S.submit({"kind": "match", "k": 5, "labels": [0, 0, 0], "edges": [(0, 1)]})
        t0 = time.time()
        errors = {}
        while len(errors) < 2 and time.time() - t0 < 30:
            for t in (bad, bad2):
                if t in errors:
                    continue
                try:
                    S.poll(t)
                except nuri.NuriError as e:
                    errors[t] = e.name
            time.sleep(0.002)
        assert errors == {bad: "EINVAL", bad2: "EINVAL"}
        res = _wait(nuri, S, [good])
        assert res[good].items == _alone(nuri, G, queries[0])
    finally:
        S.close()


def test_ticket_errors(nuri):
    """A collected ticket cannot be polled again, and a matching query on a
    graph without vertex labels is refused at submission (there is no
    matching engine to admit it)."""
    _case("server: ticket lifecycle, matching without labels")
    G = nuri.Graph.from_synth(synth.gnp(60, 0.2, 5))
    S = nuri.Server(G, frontier_budget_bytes=1 << 30, max_slots=2)
    try:
        t = S.submit({"kind": "clique", "k": 3, "weight_fn": 0})
        res = _wait(nuri, S, [t])
        assert res[t].items == nuri.topk_cliques(G, 3).items
        with pytest.raises(nuri.NuriError) as e:
            S.poll(t)
        assert e.value.name == "EINVAL"
        with pytest.raises(nuri.NuriError) as e:
            S.poll(t + 100)
        assert e.value.name == "EINVAL"
        with pytest.raises(nuri.NuriError) as e:
            S.submit({"kind": "match", "k": 5, "labels": [0, 0], "edges": [(0, 1)]})
        assert e.value.name == "EINVAL"
    finally:
        S.close()
        G.close()


def test_small_budget_admits_by_memory_and_restarts_exactly(nuri, workload):
    """A 64 MiB budget over 4096 slots gives each query only the smallest
    arena to start with: queries wait for memory, the ones that outgrow
    their arena are started again with twice the arena, and every result
    still equals the query run alone."""
    g, G, queries = workload
    _case("server: 64 MiB budget, 4096 slots")
    alone = [_alone(nuri, G, q) for q in queries]
    S = nuri.Server(G, frontier_budget_bytes=64 << 20, max_slots=4096)
    try:
        tickets = [S.submit(q) for q in queries]
        res = _wait(nuri, S, tickets, timeout=180.0)
    finally:
        S.close()
    for i, t in enumerate(tickets):
        assert res[t].items == alone[i], i


def test_query_that_outgrows_its_arena_restarts_exactly(nuri):
    """A labelled path on a graph where 12,001 vertices carry the pattern's
    label: its unit subgraphs alone (64 bytes each) overflow the smallest
    matching arena (4,096 records), so under a 64 MiB budget over 4096
    slots the query must be restarted with larger arenas -- and its result
    must still equal the query run alone."""
    n = 12001
    rng = np.random.default_rng(5)
    edges = {(0, v) for v in range(1, n)}
    for _ in range(3 * n):
        a, b = (int(x) for x in rng.integers(1, n, 2))
        if a != b:
            edges.add((min(a, b), max(a, b)))
    g = synth.from_edges(n, sorted(edges))
    g.vertex_label = np.zeros(n, np.uint8)
    synth.add_edge_weights(g, 1, 1000, master=5)
    labels, pedges = [0, 0, 0], [(0, 1), (1, 2)]
    _case("server: a query larger than its first arena")
    G = nuri.Graph.from_synth(g)
    try:
        alone = nuri.topk_match(G, labels, pedges, 20, deadline_ns=90 * 10 ** 9).items
        _case("server: the same query served")
        S = nuri.Server(G, frontier_budget_bytes=64 << 20, max_slots=4096)
        try:
            t = S.submit({"kind": "match", "k": 20, "labels": labels, "edges": pedges})
            res = _wait(nuri, S, [t], timeout=120.0)
        finally:
            S.close()
    finally:
        G.close()
    assert res[t].items == alone
    assert res[t].stats["restarts"] >= 1
