"""GPU parity for top-k labelled subgraph matching: HIP engine vs CPU oracle.

Bit-exact on (score, mu(0..q-1)) under (score descending, tuple ascending).
Runs only where a GPU is present.
"""
from math import comb

import networkx as nx
import numpy as np
import pytest

import oracle
import synth
from tests import bruteforce

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


def _labelled(n, p, seed, n_labels, w_hi):
    g = synth.gnp(n, p, seed)
    synth.add_zipf_labels(g, n_labels=n_labels, s=0.5, master=seed)
    synth.add_edge_weights(g, 1, w_hi, master=seed)
    return g


PATTERNS = [
    ([0, 0], [(0, 1)]),
    ([0, 1], [(0, 1)]),
    ([0, 0, 0], [(0, 1), (1, 2)]),
    ([0, 0, 0], [(0, 1), (1, 2), (0, 2)]),
    ([1, 0, 1], [(0, 1), (1, 2)]),
    ([0, 1, 0, 1], [(0, 1), (1, 2), (2, 3), (0, 3)]),
    ([0, 0, 0, 0], [(0, 1), (0, 2), (0, 3)]),
    ([0, 1, 1, 0], [(0, 1), (1, 2), (2, 3), (0, 2)]),
    ([0, 0, 0, 0], [(0, 1), (1, 2), (2, 3), (3, 0), (0, 2), (1, 3)]),
]


@pytest.mark.parametrize("pi", range(len(PATTERNS)))
def test_brute_force_corpus(nuri, pi):
    labels, edges = PATTERNS[pi]
    for seed in (1, 2):
        g = _labelled(9 if len(labels) <= 3 else 8, 0.55, 100 * seed + pi, 2, 4)
        _case(f"brute force pattern {pi} seed {seed}")
        G = nuri.Graph.from_synth(g)
        try:
            for k in (1, 3, 10000):
                want, _ = bruteforce.topk_matches(g, labels, edges, k)
                assert nuri.topk_match(G, labels, edges, k).items == want, (pi, seed, k)
        finally:
            G.close()


@pytest.mark.parametrize("idx", range(16))
def test_rmat_patterns_vs_oracle(nuri, idx):
    """R-MAT scale 14 with the labelled workload's labels, weights and pattern recipe."""
    g = _rmat14()
    p = synth.random_pattern(idx)
    _case(f"rmat14 pattern {idx}: q={p.q} labels={p.labels} edges={p.edges}")
    want, _ = oracle.topk_match(g, p.labels, p.edges, 50)
    G = _rmat14_dev(nuri)
    got = nuri.topk_match(G, p.labels, p.edges, 50)
    assert got.items == want


_R14 = {}


def _rmat14():
    if "g" not in _R14:
        g = synth.rmat(14)
        synth.add_zipf_labels(g)
        synth.add_edge_weights(g)
        _R14["g"] = g
    return _R14["g"]


def _rmat14_dev(nuri):
    if "G" not in _R14:
        _R14["G"] = nuri.Graph.from_synth(_rmat14())
    return _R14["G"]


def test_batch_equals_single_queries(nuri):
    g = _rmat14()
    G = _rmat14_dev(nuri)
    pats = [synth.random_pattern(100 + i) for i in range(12)]
    _case("batch of 12 patterns")
    qs = [{"kind": "match", "k": 20 + i, "labels": p.labels, "edges": p.edges}
          for i, p in enumerate(pats)]
    outs = nuri.topk_batch(G, qs)
    for i, p in enumerate(pats):
        want, _ = oracle.topk_match(g, p.labels, p.edges, 20 + i)
        assert outs[i].items == want, i


def test_edge_pattern_is_sorted_edges(nuri):
    g = _labelled(200, 0.05, 7, 3, 50)
    _case("edge patterns")
    G = nuri.Graph.from_synth(g)
    try:
        lab = g.vertex_label
        for la, lb in [(0, 1), (1, 1), (2, 0)]:
            rows = []
            for u in range(g.n):
                for e in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1])):
                    v = int(g.col[e])
                    if lab[u] == la and lab[v] == lb and not (la == lb and u > v):
                        rows.append((int(g.edge_weight[e]), (u, v)))
            want = sorted(rows, key=lambda t: (-t[0], t[1]))
            assert nuri.topk_match(G, [la, lb], [(0, 1)], len(want) + 3).items == want
    finally:
        G.close()


def test_uniform_triangles_and_stars(nuri):
    g = synth.gnp(80, 0.12, 12)
    g.vertex_label = np.zeros(g.n, np.uint8)
    synth.add_edge_weights(g, 1, 9, master=12)
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    for u in range(g.n):
        for e in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1])):
            G.add_edge(u, int(g.col[e]))
    n_tri = sum(nx.triangles(G).values()) // 3
    stars = int(sum(comb(int(d), 3) for d in g.degree()))
    _case("uniform triangles and 3-stars")
    D = nuri.Graph.from_synth(g)
    try:
        tri = nuri.topk_match(D, [0, 0, 0], [(0, 1), (1, 2), (0, 2)], n_tri + 5)
        assert len(tri) == n_tri
        want, _ = oracle.topk_match(g, [0, 0, 0], [(0, 1), (1, 2), (0, 2)], n_tri + 5, n_labels=1)
        assert tri.items == want
        st = nuri.topk_match(D, [0] * 4, [(0, 1), (0, 2), (0, 3)], stars + 5)
        assert len(st) == stars
    finally:
        D.close()


def test_repeated_runs_identical(nuri):
    g = _rmat14()
    G = _rmat14_dev(nuri)
    p = synth.random_pattern(3)
    _case("repeated match runs")
    first = nuri.topk_match(G, p.labels, p.edges, 50).items
    for _ in range(4):
        assert nuri.topk_match(G, p.labels, p.edges, 50).items == first


def test_match_edge_cases(nuri):
    g = _labelled(30, 0.3, 2, 2, 3)
    _case("match edge cases")
    G = nuri.Graph.from_synth(g)
    try:
        assert nuri.topk_match(G, [5, 0], [(0, 1)], 5).items == []       # absent label
        for labels, edges in [([0, 0, 0], [(0, 1)]), ([0] * 9, [(i, i + 1) for i in range(8)]),
                              ([0, 0], [(0, 0)]), ([0, 0], [(0, 1), (1, 0)])]:
            with pytest.raises(nuri.NuriError) as e:
                nuri.topk_match(G, labels, edges, 5)
            assert e.value.name == "EINVAL"
        with pytest.raises(nuri.NuriError):
            nuri.topk_match(G, [0, 0], [(0, 1)], 0)
    finally:
        G.close()


def test_match_deadline_fails_loudly(nuri):
    g = _rmat14()
    G = _rmat14_dev(nuri)
    p = synth.random_pattern(3)
    _case("match deadline")
    with pytest.raises(nuri.NuriError) as e:
        nuri.topk_match(G, p.labels, p.edges, 50, deadline_ns=1)
    assert e.value.name == "ETIMEOUT"
    want, _ = oracle.topk_match(g, p.labels, p.edges, 50)
    assert nuri.topk_match(G, p.labels, p.edges, 50).items == want


# eight-vertex patterns (the largest query size; every bit of the pattern
# masks and all eight matched slots of a record are used): a cycle, a star,
# a labelled path, a cube-like graph, and two joined stars
PATTERNS8 = [
    ([0] * 8, [(i, (i + 1) % 8) for i in range(8)]),
    ([0] * 8, [(0, i) for i in range(1, 8)]),
    ([0, 1, 0, 1, 0, 1, 0, 1], [(i, i + 1) for i in range(7)]),
    ([0, 0, 0, 0, 1, 1, 1, 1], [(0, 1), (1, 2), (2, 3), (3, 0), (4, 5), (5, 6), (6, 7), (7, 4),
                                (0, 4), (1, 5), (2, 6), (3, 7)]),
    ([1, 0, 0, 0, 1, 0, 0, 0], [(0, 1), (0, 2), (0, 3), (0, 4), (4, 5), (4, 6), (4, 7)]),
]


@pytest.mark.parametrize("pi", range(len(PATTERNS8)))
def test_eight_vertex_patterns_vs_brute_force(nuri, pi):
    labels, edges = PATTERNS8[pi]
    n_labels = max(labels) + 1
    g = _labelled(9, 0.92, 800 + pi, n_labels, 6)
    # the pattern's own labels plus one more vertex, shuffled
    g.vertex_label = np.array(list(labels) + [0], np.uint8)[
        np.random.default_rng(pi).permutation(9)]
    want, n_img = bruteforce.topk_matches(g, labels, edges, 10 ** 6)
    assert n_img > 0
    _case(f"eight-vertex pattern {pi}: {n_img} images")
    G = nuri.Graph.from_synth(g)
    try:
        for k in (1, 5, 10 ** 6):
            assert nuri.topk_match(G, labels, edges, k).items == want[:k], k
    finally:
        G.close()


@pytest.mark.parametrize("idx", list(range(6)) + ["cycle", "double_star"])
def test_eight_vertex_rmat_patterns_vs_oracle(nuri, idx):
    """Eight-vertex patterns of the served mix's recipe (q = 8), plus two
    with non-trivial automorphism groups (16 and 72), on R-MAT scale 14."""
    if idx == "cycle":
        labels, edges = PATTERNS8[0]
    elif idx == "double_star":
        labels = [2, 0, 0, 0, 2, 0, 0, 0]
        edges = PATTERNS8[4][1]
    else:
        p = synth.random_pattern(2000 + idx, q_lo=8, q_hi=8)
        labels, edges = p.labels, p.edges
    g = _rmat14()
    _case(f"rmat14 eight-vertex pattern {idx}: labels={labels}")
    want, _ = oracle.topk_match(g, labels, edges, 50)
    got = nuri.topk_match(_rmat14_dev(nuri), labels, edges, 50)
    assert got.items == want


@pytest.mark.parametrize("priority", [0, 1, 2, 3])
def test_match_result_independent_of_priority(nuri, priority):
    """Depth-first, best-first, the paper's order and no pruning (Nuri-NP)
    give the same top-k; without pruning at least as many children."""
    g = _labelled(300, 0.04, 77, 3, 50)
    _case(f"matching priority={priority}")
    G = nuri.Graph.from_synth(g)
    try:
        for labels, edges in PATTERNS[2:] + [([0, 1, 2, 0], [(0, 1), (1, 2), (2, 3), (3, 1)])]:
            for k in (1, 20):
                want, _ = oracle.topk_match(g, labels, edges, k, n_labels=3)
                got = nuri.topk_match(G, labels, edges, k, priority=priority)
                assert got.items == want, (labels, edges, k)
                ties = sum(1 for s, _ in want if s == want[-1][0]) if len(want) == k else 0
                assert got.stats["ties_at_k"] == ties
                if priority == 3:
                    ref = nuri.topk_match(G, labels, edges, k)
                    assert got.stats["children"] >= ref.stats["children"]
    finally:
        G.close()


def test_matching_frontier_spill_is_exact(nuri):
    """128 labelled patterns share the smallest budget (64 MiB), so each gets
    a 512 KiB arena (8,192 records), and run best-first; the
    searches whose frontiers outgrow it move their bottom levels to host
    memory and take them back when the levels above are done.  Every
    result equals the same batch under the default budget, and the oracle
    on four of them.  A deadline bounds both runs."""
    g = synth.rmat(13)
    synth.add_zipf_labels(g)
    synth.add_edge_weights(g)
    pats = [synth.random_pattern(300 + i) for i in range(128)]
    qs = [{"kind": "match", "k": 50, "labels": p.labels, "edges": p.edges} for p in pats]
    limit = 150 * 10 ** 9
    G = nuri.Graph.from_synth(g)
    try:
        _case("128 patterns, R-MAT 13, best-first, default budget")
        full = nuri.topk_batch(G, qs, priority=nuri.PRIORITY_BOUND, deadline_ns=limit)
        peaks = sorted(r.stats["frontier_peak_bytes"] for r in full)
        arena = (64 << 20) // len(qs)
        _case(f"frontier peaks: max {peaks[-1]}, median {peaks[len(peaks) // 2]}, above "
              f"{arena} bytes: {sum(p > arena for p in peaks)}")
        assert peaks[-1] > arena, "no query outgrows its arena: the test would not spill"
        _case("128 patterns, R-MAT 13, best-first, 64 MiB budget: spills")
        small = nuri.topk_batch(G, qs, frontier_budget_bytes=64 << 20,
                                priority=nuri.PRIORITY_BOUND, deadline_ns=limit)
    finally:
        G.close()
    for i in range(len(qs)):
        assert small[i].items == full[i].items, i
    _case(f"spilled bytes: {sum(r.stats['spilled_bytes'] for r in small)} over "
          f"{sum(r.stats['spilled_bytes'] > 0 for r in small)} queries")
    assert sum(r.stats["spilled_bytes"] for r in small) > 0
    for i in (0, 1, 2, 3):
        want, _ = oracle.topk_match(g, pats[i].labels, pats[i].edges, 50)
        assert small[i].items == want, i
