"""GPU parity for degree-score matching (Section 4.3): HIP engine vs CPU oracle.

The multi-hop index is compared entry by entry with the oracle's
breadth-first index, including rows long enough to be cut into chunks;
top-k results are compared bit-exactly on (score, mu(0..q-1)).
"""
import numpy as np
import pytest

import oracle
import synth
from tests import bruteforce
from tests.test_oracle_match import PATTERNS, PATTERNS8

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


def _labelled(n, p, seed, n_labels):
    g = synth.gnp(n, p, seed)
    synth.add_zipf_labels(g, n_labels=n_labels, s=0.5, master=seed)
    return g


_R12 = {}


def _rmat12():
    """R-MAT scale 12 with Zipf labels over 16 values (the labelled workload's
    recipe at a size the oracle's breadth-first index finishes in seconds)."""
    if "g" not in _R12:
        g = synth.rmat(12)
        synth.add_zipf_labels(g)
        _R12["g"] = g
    return _R12["g"]


def _rmat12_dev(nuri):
    if "G" not in _R12:
        _R12["G"] = nuri.Graph.from_synth(_rmat12())
    return _R12["G"]


def _hubs():
    """A sparse Chung-Lu graph on 10,000 vertices plus three hubs joined to
    about 95%, 45% and 15% of the vertices: rows of ~9,500, ~4,500 and
    ~1,500 neighbours take the chunked path (three, two and one chunks)."""
    base = synth.chung_lu(n=10000, beta=2.1, m_target=30000, cap=200.0, n_cliques=0)
    edges = []
    for u in range(base.n):
        for v in base.col[base.row_ptr[u]:base.row_ptr[u + 1]]:
            if u < int(v):
                edges.append((u, int(v)))
    s = synth.stream_seed(91, 7)
    for hub, pct in ((0, 95), (1, 45), (2, 15)):
        for j in range(3, base.n):
            if synth.below(s, hub * base.n + j, 100) < pct:
                edges.append((hub, j))
    g = synth.from_edges(base.n, edges, name="chunglu10000_hubs")
    synth.add_zipf_labels(g, n_labels=5, s=0.8, master=77)
    return g


def test_worked_example_on_the_gpu(nuri):
    """Section 4.3: the path v1-v2-v3-v4 (all label a) and the one-edge
    query; top-1 is {v2, v3} with score 4, then the two end edges (3)."""
    g = synth.from_edges(4, [(0, 1), (1, 2), (2, 3)])
    g.vertex_label = np.zeros(4, np.uint8)
    _case("worked example")
    G = nuri.Graph.from_synth(g)
    try:
        r = nuri.topk_match(G, [0, 0], [(0, 1)], 1, score="degree")
        assert r.items == [(4, (1, 2))]
        r = nuri.topk_match(G, [0, 0], [(0, 1)], 5, score="degree")
        assert r.items == [(4, (1, 2)), (3, (0, 1)), (3, (2, 3))]
        idx, _ = G.hop_index(1)
        assert idx[0, :, 0].tolist() == [2, 2, 2, 2]
    finally:
        G.close()


def test_hop_index_equals_oracle_rmat12(nuri):
    g = _rmat12()
    _case("hop index, R-MAT 12, 7 hops")
    want = oracle.hop_index(g, 7, n_labels=16)
    G = _rmat12_dev(nuri)
    got, _ = G.hop_index(7)
    assert np.array_equal(got, want)


def test_hop_index_with_chunked_rows_and_extension(nuri):
    """Rows of up to ~9,000 neighbours (chunked); the index built for 2
    hops first, then extended to 3: the first two hops' arrays are kept and
    the third equals the oracle's."""
    g = _hubs()
    deg = np.diff(g.row_ptr)
    assert deg.max() > 2 * 4096, deg.max()
    _case(f"hop index, Chung-Lu hubs (max degree {deg.max()}), 2 then 3 hops")
    want = oracle.hop_index(g, 3, n_labels=16)
    G = nuri.Graph.from_synth(g)
    try:
        got2, ns2 = G.hop_index(2)
        assert ns2 > 0
        assert np.array_equal(got2, want[:2])
        got3, ns3 = G.hop_index(3)
        assert np.array_equal(got3, want)
        again, ns = G.hop_index(3)
        assert ns < ns3 and np.array_equal(again, want)
    finally:
        G.close()


@pytest.mark.parametrize("pi", range(len(PATTERNS)))
def test_degree_brute_force_corpus(nuri, pi):
    labels, edges = PATTERNS[pi]
    for seed in (1, 2):
        g = _labelled(9 if len(labels) <= 3 else 8, 0.55, 700 + 100 * seed + pi, 2)
        _case(f"degree brute force pattern {pi} seed {seed}")
        G = nuri.Graph.from_synth(g)
        try:
            for k in (1, 3, 10000):
                want, _ = bruteforce.topk_matches(g, labels, edges, k, score="degree")
                assert nuri.topk_match(G, labels, edges, k, score="degree").items == want
        finally:
            G.close()


@pytest.mark.parametrize("pi", [0, 2, 3])
def test_degree_eight_vertex_patterns_vs_brute_force(nuri, pi):
    labels, edges = PATTERNS8[pi]
    n_labels = max(labels) + 1
    g = _labelled(9, 0.9, 860 + pi, n_labels)
    g.vertex_label = np.array([i % n_labels for i in range(9)], np.uint8)[
        np.random.default_rng(pi).permutation(9)]
    want, n_img = bruteforce.topk_matches(g, labels, edges, 10 ** 6, score="degree")
    _case(f"degree eight-vertex pattern {pi}: {n_img} images")
    G = nuri.Graph.from_synth(g)
    try:
        for k in (1, 5, 10 ** 6):
            assert nuri.topk_match(G, labels, edges, k, score="degree").items == want[:k]
    finally:
        G.close()


@pytest.mark.parametrize("idx", range(12))
def test_degree_rmat12_patterns_vs_oracle(nuri, idx):
    g = _rmat12()
    p = synth.random_pattern(idx)
    _case(f"degree rmat12 pattern {idx}: q={p.q} labels={p.labels} edges={p.edges}")
    want, _ = oracle.topk_match(g, p.labels, p.edges, 50, score="degree")
    got = nuri.topk_match(_rmat12_dev(nuri), p.labels, p.edges, 50, score="degree")
    assert got.items == want


@pytest.mark.parametrize("priority", [1, 2, 3])
def test_degree_result_independent_of_priority(nuri, priority):
    g = _rmat12()
    p = synth.random_pattern(3)
    _case(f"degree priority {priority}")
    want, _ = oracle.topk_match(g, p.labels, p.edges, 40, score="degree")
    got = nuri.topk_match(_rmat12_dev(nuri), p.labels, p.edges, 40, score="degree",
                          priority=priority)
    assert got.items == want


def test_mixed_batch_and_server(nuri):
    """Edge-weight and degree queries in one batch, and through the server:
    each equals the oracle."""
    g = synth.rmat(12)
    synth.add_zipf_labels(g)
    synth.add_edge_weights(g)
    G = nuri.Graph.from_synth(g)
    try:
        pats = [synth.random_pattern(200 + i) for i in range(8)]
        qs = [{"kind": "match", "k": 10 + i, "labels": p.labels, "edges": p.edges,
               "score": "degree" if i % 2 else "edge"} for i, p in enumerate(pats)]
        _case("mixed batch of 8 patterns")
        outs = nuri.topk_batch(G, qs)
        for i, p in enumerate(pats):
            want, _ = oracle.topk_match(g, p.labels, p.edges, 10 + i, score=qs[i]["score"])
            assert outs[i].items == want, i
        _case("degree queries through the server")
        srv = nuri.Server(G, max_slots=4)
        try:
            tickets = [srv.submit(q) for q in qs]
            for t, q, i in zip(tickets, qs, range(len(qs))):
                r = None
                while r is None:
                    r = srv.poll(t)
                assert r.items == outs[i].items, i
        finally:
            srv.close()
    finally:
        G.close()


def test_degree_needs_labels_and_a_known_score(nuri):
    g = synth.gnp(30, 0.2, 3)
    _case("degree score edge cases")
    G = nuri.Graph.from_synth(g)
    try:
        with pytest.raises(nuri.NuriError):
            nuri.topk_match(G, [0, 0], [(0, 1)], 3, score="degree")
        with pytest.raises(nuri.NuriError):
            G.hop_index(1)
    finally:
        G.close()
    g.vertex_label = np.zeros(g.n, np.uint8)
    G = nuri.Graph.from_synth(g)
    try:
        with pytest.raises(nuri.NuriError):
            G.hop_index(8)
        with pytest.raises(nuri.NuriError):
            G.hop_index(0)
        # a label no vertex carries: empty result
        assert nuri.topk_match(G, [3, 0], [(0, 1)], 3, score="degree").items == []
        # isolated vertices and k above the number of matches
        want, _ = oracle.topk_match(g, [0, 0, 0], [(0, 1), (1, 2)], 10 ** 5, score="degree")
        got = nuri.topk_match(G, [0, 0, 0], [(0, 1), (1, 2)], 10 ** 5, score="degree")
        assert got.items == want
    finally:
        G.close()
