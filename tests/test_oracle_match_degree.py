"""Pins for the CPU oracle's degree-score matching (no GPU).

Section 4.3 scores a match by the sum of the degrees of its vertices and
bounds a partial match with a multi-hop index: for every vertex, hop count
and label, the largest degree among the vertices of that label within that
many hops.  Checked against the section's worked example (Figure 7), the
index rebuilt from scipy's all-pairs shortest paths, brute force over all
injective maps, the soundness of every unit-subgraph bound over every
embedding, and a closed form for one-edge patterns.
"""
import os

import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import shortest_path

import oracle
import synth
from tests import bruteforce
from tests.test_oracle_match import PATTERNS, PATTERNS8

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _labelled(n, p, seed, n_labels):
    g = synth.gnp(n, p, seed)
    synth.add_zipf_labels(g, n_labels=n_labels, s=0.5, master=seed)
    return g


def _read_fixture():
    rows = {}
    with open(os.path.join(GOLDEN, "worked_example_si_degree.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            key, *vals = line.split()
            rows[key] = vals
    return rows


def _pairs(vals):
    return [tuple(int(x) for x in v.split("-")) for v in vals]


def test_section_4_3_worked_example():
    fx = _read_fixture()
    n = int(fx["n"][0])
    g = synth.from_edges(n, _pairs(fx["edges"]))
    g.vertex_label = np.array([int(x) for x in fx["labels"]], np.uint8)
    plabels = [int(x) for x in fx["pattern_labels"]]
    pedges = _pairs(fx["pattern_edges"])
    first, bounds = oracle.match_root_bounds(g, plabels, pedges, n_labels=1, score="degree")
    assert first == 0
    assert bounds.tolist() == [int(x) for x in fx["root_bounds"]]
    deg = np.diff(g.row_ptr)
    assert deg[1] == int(fx["score_s2"][0])
    idx = oracle.hop_index(g, 1, n_labels=1)
    assert idx[0, 1, 0] == int(fx["index_v2_label_a_hop1"][0])
    top, st = oracle.topk_match(g, plabels, pedges, 1, n_labels=1, score="degree")
    want = [int(x) for x in fx["top1"]]
    assert top == [(want[0], tuple(want[1:]))]
    # top-1: the unit subgraphs of bound 3 are discarded once s6 (score 4)
    # is in the result set, so they are never expanded
    assert st["pruned_at_pop"] >= 2


def _index_from_distances(g, hops, n_labels):
    """index[h-1, v, l] from the all-pairs hop distances (scipy)."""
    n = g.n
    A = csr_matrix((np.ones(len(g.col)), g.col.astype(np.int64), g.row_ptr.astype(np.int64)),
                   shape=(n, n))
    D = shortest_path(A, unweighted=True, directed=False)
    deg = np.diff(g.row_ptr).astype(np.int64)
    lab = g.vertex_label.astype(np.int64)
    out = np.zeros((hops, n, n_labels), np.int64)
    for h in range(1, hops + 1):
        within = (D >= 1) & (D <= h)
        for l in range(n_labels):
            m = within & (lab[None, :] == l)
            out[h - 1, :, l] = np.where(m, deg[None, :], 0).max(axis=1)
    return out


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_hop_index_equals_shortest_path_definition(seed):
    g = _labelled(70, 0.04, 300 + seed, n_labels=4)
    want = _index_from_distances(g, 5, 4)
    got = oracle.hop_index(g, 5, n_labels=4)
    assert np.array_equal(got, want)


def test_hop_index_on_a_path_grows_one_hop_at_a_time():
    """On a path 0-1-...-9 with degree-1 ends, vertex 0's label-0 entry
    reaches a degree-2 vertex at hop 1, and the far end (degree 1) never
    raises it; with the labels of vertices 1..8 set to 1, vertex 0 first
    sees label 0 at hop 9."""
    g = synth.from_edges(10, [(i, i + 1) for i in range(9)])
    g.vertex_label = np.array([0] + [1] * 8 + [0], np.uint8)
    idx = oracle.hop_index(g, 9, n_labels=2)
    assert idx[:, 0, 0].tolist() == [0] * 8 + [1]
    assert idx[:, 0, 1].tolist() == [2] * 9
    # the middle vertex sees degree-2 vertices of label 1 one hop away and
    # both ends (label 0, degree 1) from hop 4 (vertex 0) and hop 5 (vertex 9)
    assert idx[:, 4, 0].tolist() == [0, 0, 0, 1, 1, 1, 1, 1, 1]


@pytest.mark.parametrize("pi", range(len(PATTERNS)))
@pytest.mark.parametrize("seed", [1, 2])
def test_degree_topk_matches_brute_force(pi, seed):
    labels, edges = PATTERNS[pi]
    n = 9 if len(labels) <= 3 else 8
    g = _labelled(n, 0.55, 700 + 100 * seed + pi, n_labels=2)
    for k in (1, 3, 10000):
        want, _ = bruteforce.topk_matches(g, labels, edges, k, score="degree")
        got, _ = oracle.topk_match(g, labels, edges, k, n_labels=2, score="degree")
        assert got == want, (pi, seed, k)


@pytest.mark.parametrize("idx", range(10))
def test_degree_random_patterns_match_brute_force(idx):
    pat = synth.random_pattern(40 + idx, q_lo=2, q_hi=5, n_labels=2, s=0.5)
    g = _labelled(8, 0.6, 740 + idx, n_labels=2)
    want, _ = bruteforce.topk_matches(g, pat.labels, pat.edges, 10000, score="degree")
    got, _ = oracle.topk_match(g, pat.labels, pat.edges, 10000, n_labels=2, score="degree")
    assert got == want


@pytest.mark.parametrize("pi", [0, 2])
def test_degree_eight_vertex_patterns_match_brute_force(pi):
    labels, edges = PATTERNS8[pi]
    n_labels = max(labels) + 1
    g = _labelled(9, 0.9, 860 + pi, n_labels=n_labels)
    g.vertex_label = np.array([i % n_labels for i in range(9)], np.uint8)[
        np.random.default_rng(pi).permutation(9)]
    want, n_img = bruteforce.topk_matches(g, labels, edges, 10 ** 6, score="degree")
    assert n_img > 0
    for k in (1, 5, 10 ** 6):
        got, _ = oracle.topk_match(g, labels, edges, k, n_labels=n_labels, score="degree")
        assert got == want[:k]


@pytest.mark.parametrize("pi", [2, 4, 5, 6, 7])
def test_root_bounds_are_sound_over_every_embedding(pi):
    """No embedding scores above the bound of the unit subgraph its first
    pattern vertex (in the matching order) sits on: the multi-hop bound may
    only overestimate.  A pattern vertex h hops from the first can land
    closer than h to the seed, which is why the index is cumulative."""
    import itertools
    labels, edges = PATTERNS[pi]
    g = _labelled(10, 0.5, 900 + pi, n_labels=2)
    first, bounds = oracle.match_root_bounds(g, labels, edges, n_labels=2, score="degree")
    deg = np.diff(g.row_ptr)
    adj = [set(g.col[g.row_ptr[v]:g.row_ptr[v + 1]].tolist()) for v in range(g.n)]
    lab = g.vertex_label.tolist()
    q, seen = len(labels), 0
    for mu in itertools.permutations(range(g.n), q):
        if any(lab[mu[a]] != labels[a] for a in range(q)):
            continue
        if any(mu[b] not in adj[mu[a]] for a, b in edges):
            continue
        seen += 1
        assert bounds[mu[first]] >= sum(int(deg[v]) for v in mu), mu
    assert seen > 0
    # and a root is only dropped (-1) when no embedding uses it
    used = set()
    for mu in itertools.permutations(range(g.n), q):
        if all(lab[mu[a]] == labels[a] for a in range(q)) and \
                all(mu[b] in adj[mu[a]] for a, b in edges):
            used.add(mu[first])
    for v in used:
        assert bounds[v] >= 0


def test_one_edge_pattern_is_a_sort_of_edges_by_degree_sum():
    g = _labelled(80, 0.08, 17, n_labels=2)
    deg = np.diff(g.row_ptr).astype(np.int64)
    lab = g.vertex_label
    want = []
    for u in range(g.n):
        for v in g.col[g.row_ptr[u]:g.row_ptr[u + 1]]:
            v = int(v)
            if lab[u] == 0 and lab[v] == 1:
                want.append((int(deg[u] + deg[v]), (u, v)))
    want.sort(key=lambda t: (-t[0], t[1]))
    got, _ = oracle.topk_match(g, [0, 1], [(0, 1)], len(want) + 3, n_labels=2, score="degree")
    assert got == want


@pytest.mark.parametrize("priority", [0, 1, 2])
def test_degree_result_independent_of_priority(priority):
    g = _labelled(60, 0.15, 42, n_labels=3)
    labels, edges = [0, 1, 0, 2], [(0, 1), (1, 2), (2, 3), (1, 3)]
    ref, _ = oracle.topk_match(g, labels, edges, 30, n_labels=3, priority=0, score="degree")
    got, _ = oracle.topk_match(g, labels, edges, 30, n_labels=3, priority=priority,
                               score="degree")
    assert got == ref and len(got) == 30


def test_degree_score_ignores_edge_weights():
    g = _labelled(40, 0.2, 5, n_labels=2)
    a, _ = oracle.topk_match(g, [0, 1, 0], [(0, 1), (1, 2)], 20, n_labels=2, score="degree")
    synth.add_edge_weights(g, 1, 50, master=5)
    b, _ = oracle.topk_match(g, [0, 1, 0], [(0, 1), (1, 2)], 20, n_labels=2, score="degree")
    assert a == b
