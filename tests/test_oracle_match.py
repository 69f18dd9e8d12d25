"""Pins for the CPU oracle's top-k labelled subgraph matching (no GPU).

Checked against brute force over all injective maps, closed forms (edge,
triangle and star patterns), and networkx's monomorphism enumeration
(|monomorphisms| = |images| x |Aut(P)|).
"""
import itertools
from math import comb

import networkx as nx
import numpy as np
import pytest

import oracle
import synth
from tests import bruteforce


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
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_match_topk_matches_brute_force(pi, seed):
    labels, edges = PATTERNS[pi]
    n = 9 if len(labels) <= 3 else 8
    g = _labelled(n, 0.55, 100 * seed + pi, n_labels=2, w_hi=4)
    for k in (1, 3, 10000):
        want, _ = bruteforce.topk_matches(g, labels, edges, k)
        got, _ = oracle.topk_match(g, labels, edges, k, n_labels=2)
        assert got == want, (pi, seed, k)


@pytest.mark.parametrize("idx", range(12))
def test_random_patterns_match_brute_force(idx):
    pat = synth.random_pattern(idx, q_lo=2, q_hi=5, n_labels=2, s=0.5)
    g = _labelled(8, 0.6, 500 + idx, n_labels=2, w_hi=3)
    want, _ = bruteforce.topk_matches(g, pat.labels, pat.edges, 10000)
    got, st = oracle.topk_match(g, pat.labels, pat.edges, 10000, n_labels=2)
    assert got == want
    assert st["automorphisms"] == bruteforce.automorphism_count(pat.labels, pat.edges)


@pytest.mark.parametrize("priority", [0, 1, 2])
def test_result_independent_of_priority(priority):
    g = _labelled(60, 0.15, 42, n_labels=3, w_hi=20)
    labels, edges = [0, 1, 0, 2], [(0, 1), (1, 2), (2, 3), (1, 3)]
    ref, _ = oracle.topk_match(g, labels, edges, 30, n_labels=3, priority=0)
    got, _ = oracle.topk_match(g, labels, edges, 30, n_labels=3, priority=priority)
    assert got == ref


def test_edge_pattern_is_a_sort_of_edges():
    """q = 2: the results are the edges with the right label pair, by weight."""
    g = _labelled(150, 0.08, 7, n_labels=3, w_hi=50)
    lab = g.vertex_label
    for la, lb in [(0, 1), (1, 1), (2, 0)]:
        rows = []
        for u in range(g.n):
            for e in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1])):
                v = int(g.col[e])
                if lab[u] == la and lab[v] == lb:
                    if la == lb and u > v:
                        continue
                    rows.append((int(g.edge_weight[e]), (u, v)))
        want = sorted(rows, key=lambda t: (-t[0], t[1]))
        got, _ = oracle.topk_match(g, [la, lb], [(0, 1)], len(want) + 5, n_labels=3)
        assert got == want
        got5, _ = oracle.topk_match(g, [la, lb], [(0, 1)], 5, n_labels=3)
        assert got5 == want[:5]


def _nx(g):
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    for u in range(g.n):
        for e in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1])):
            G.add_edge(u, int(g.col[e]))
    return G


def test_uniform_triangle_count():
    g = synth.gnp(80, 0.15, 12)
    g.vertex_label = np.zeros(g.n, np.uint8)
    synth.add_edge_weights(g, 1, 9, master=12)
    n_tri = sum(nx.triangles(_nx(g)).values()) // 3
    got, _ = oracle.topk_match(g, [0, 0, 0], [(0, 1), (1, 2), (0, 2)], n_tri + 10, n_labels=1)
    assert len(got) == n_tri
    for s, mu in got:
        assert mu[0] < mu[1] < mu[2]


@pytest.mark.parametrize("r", [2, 3, 7])
def test_uniform_star_count(r):
    g = synth.gnp(40, 0.15, 13)
    g.vertex_label = np.zeros(g.n, np.uint8)
    synth.add_edge_weights(g, 1, 9, master=13)
    deg = g.degree()
    want = int(sum(comb(int(d), r) for d in deg))
    labels = [0] * (r + 1)
    edges = [(0, i) for i in range(1, r + 1)]
    got, _ = oracle.topk_match(g, labels, edges, want + 10, n_labels=1)
    assert len(got) == want


def test_monomorphisms_equal_images_times_automorphisms():
    g = _labelled(30, 0.25, 21, n_labels=2, w_hi=5)
    G = _nx(g)
    for v in range(g.n):
        G.nodes[v]["l"] = int(g.vertex_label[v])
    for labels, edges in PATTERNS[2:]:
        P = nx.Graph()
        for a, la in enumerate(labels):
            P.add_node(a, l=la)
        P.add_edges_from(edges)
        gm = nx.algorithms.isomorphism.GraphMatcher(
            G, P, node_match=lambda x, y: x["l"] == y["l"])
        monos = sum(1 for _ in gm.subgraph_monomorphisms_iter())
        got, st = oracle.topk_match(g, labels, edges, 10 ** 6, n_labels=2)
        assert monos == len(got) * st["automorphisms"]


def test_scores_are_exact_and_embeddings_valid():
    g = _labelled(100, 0.1, 5, n_labels=3, w_hi=1000)
    labels, edges = [0, 1, 0], [(0, 1), (1, 2)]
    got, _ = oracle.topk_match(g, labels, edges, 200, n_labels=3)
    wmap = {}
    for u in range(g.n):
        for e in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1])):
            wmap[(u, int(g.col[e]))] = int(g.edge_weight[e])
    for s, mu in got:
        assert len(set(mu)) == len(mu)
        assert all(int(g.vertex_label[mu[a]]) == labels[a] for a in range(3))
        assert s == sum(wmap[(mu[a], mu[b])] for a, b in edges)
        # mirror automorphism (0 <-> 2): representative keeps mu(0) < mu(2)
        assert mu[0] < mu[2]
    keys = [(-s, mu) for s, mu in got]
    assert keys == sorted(keys)


def test_invalid_patterns_rejected():
    g = _labelled(10, 0.5, 1, n_labels=2, w_hi=3)
    with pytest.raises(ValueError):
        oracle.topk_match(g, [0, 0, 0], [(0, 1)], 5, n_labels=2)      # disconnected
    with pytest.raises(ValueError):
        oracle.topk_match(g, [0], [], 5, n_labels=2)                  # q < 2
    with pytest.raises(ValueError):
        oracle.topk_match(g, [0] * 9, [(i, i + 1) for i in range(8)], 5, n_labels=2)  # q > 8
    with pytest.raises(ValueError):
        oracle.topk_match(g, [0, 0], [(0, 1)], 0, n_labels=2)        # k = 0


def test_absent_label_gives_empty_result():
    g = _labelled(20, 0.3, 2, n_labels=2, w_hi=3)
    got, _ = oracle.topk_match(g, [5, 0], [(0, 1)], 5, n_labels=16)
    assert got == []


@pytest.mark.parametrize("pi", [2, 4, 5, 6, 7])
def test_topk_equals_networkx_monomorphisms(pi):
    """The whole ranked list, rebuilt from networkx's monomorphism
    enumeration: embeddings grouped by image (the set of data edges the
    pattern edges land on), each image scored by its edge weights and
    represented by its smallest embedding tuple, ranked by score descending
    then tuple ascending.  On graphs larger than brute force reaches."""
    labels, edges = PATTERNS[pi]
    g = _labelled(45, 0.22, 60 + pi, n_labels=2, w_hi=7)
    G = _nx(g)
    for v in range(g.n):
        G.nodes[v]["l"] = int(g.vertex_label[v])
    wmap = {}
    for u in range(g.n):
        for e in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1])):
            wmap[(u, int(g.col[e]))] = int(g.edge_weight[e])
    P = nx.Graph()
    for a, la in enumerate(labels):
        P.add_node(a, l=la)
    P.add_edges_from(edges)
    gm = nx.algorithms.isomorphism.GraphMatcher(G, P, node_match=lambda x, y: x["l"] == y["l"])
    best = {}
    for m in gm.subgraph_monomorphisms_iter():  # data vertex -> pattern vertex
        mu = [0] * len(labels)
        for v, a in m.items():
            mu[a] = v
        mu = tuple(mu)
        image = frozenset(frozenset((mu[a], mu[b])) for a, b in edges)
        if image not in best or mu < best[image]:
            best[image] = mu
    ranked = sorted(((sum(wmap[(mu[a], mu[b])] for a, b in edges), mu) for mu in best.values()),
                    key=lambda t: (-t[0], t[1]))
    for k in (1, 7, 50, len(ranked) + 1):
        got, _ = oracle.topk_match(g, labels, edges, k, n_labels=2)
        assert got == ranked[:k], k


# eight-vertex patterns (the largest size a query may have): a cycle, a star,
# a labelled path and a cube-like graph with many automorphisms
PATTERNS8 = [
    ([0] * 8, [(i, (i + 1) % 8) for i in range(8)]),
    ([0] + [0] * 7, [(0, i) for i in range(1, 8)]),
    ([0, 1, 0, 1, 0, 1, 0, 1], [(i, i + 1) for i in range(7)]),
    ([0, 0, 0, 0, 1, 1, 1, 1], [(0, 1), (1, 2), (2, 3), (3, 0), (4, 5), (5, 6), (6, 7), (7, 4),
                                (0, 4), (1, 5), (2, 6), (3, 7)]),
]


@pytest.mark.parametrize("pi", range(len(PATTERNS8)))
def test_eight_vertex_patterns_match_brute_force(pi):
    labels, edges = PATTERNS8[pi]
    n_labels = max(labels) + 1
    g = _labelled(9, 0.92, 800 + pi, n_labels=n_labels, w_hi=6)
    # every pattern label on at least four data vertices
    g.vertex_label = np.array([i % n_labels for i in range(9)], np.uint8)[
        np.random.default_rng(pi).permutation(9)]
    want, n_img = bruteforce.topk_matches(g, labels, edges, 10 ** 6)
    assert n_img > 0
    got, st = oracle.topk_match(g, labels, edges, 10 ** 6, n_labels=n_labels)
    assert got == want and len(got) == n_img
    assert st["automorphisms"] == bruteforce.automorphism_count(labels, edges)
    for k in (1, 5):
        top, _ = oracle.topk_match(g, labels, edges, k, n_labels=n_labels)
        assert top == want[:k]


@pytest.mark.parametrize("idx", range(4))
def test_random_eight_vertex_patterns_match_brute_force(idx):
    pat = synth.random_pattern(900 + idx, q_lo=8, q_hi=8, n_labels=2, s=0.3)
    assert len(pat.labels) == 8
    g = _labelled(10, 0.85, 900 + idx, n_labels=2, w_hi=9)
    # the pattern's own labels plus one vertex of each label, shuffled
    g.vertex_label = np.array(list(pat.labels) + [0, 1], np.uint8)[
        np.random.default_rng(idx).permutation(10)]
    want, n_img = bruteforce.topk_matches(g, pat.labels, pat.edges, 10 ** 6)
    assert n_img > 0
    got, _ = oracle.topk_match(g, pat.labels, pat.edges, 10 ** 6, n_labels=2)
    assert got == want
