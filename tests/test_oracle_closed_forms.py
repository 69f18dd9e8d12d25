"""Closed-form pins for the oracle (no GPU).

Cliques: the graph families and their maximal cliques are those of
tests/closed_forms.py (complete multipartite and Moon-Moser graphs, cycles,
disjoint complete graphs); the expected top-k is the closed form ranked by
score descending, then ids ascending (the result order of Section 3.2).
Matching: paths and 4-cycles in complete graphs and labelled paths in a
complete bipartite graph, whose images and smallest representatives follow
from the pattern's automorphisms; scores from edge weights given by formula.
"""
import itertools

import numpy as np
import pytest

import oracle
from tests import closed_forms as cf


@pytest.mark.parametrize("sizes,seed", [((3, 3, 3, 3, 3), 1), ((1, 2, 3, 4, 2), 2),
                                        ((5, 1, 1, 4), 3), ((2,) * 9, 4)])
@pytest.mark.parametrize("k", [1, 7, 48, 100000])
def test_complete_multipartite_by_size(sizes, seed, k):
    g, parts = cf.multipartite(sizes, seed)
    want = cf.ranked(cf.transversals(parts))
    assert len(want) == int(np.prod(sizes))
    for bound in (0, 1):
        got, _ = oracle.topk_cliques(g, k, bound=bound)
        assert got == want[:k]


@pytest.mark.parametrize("sizes,seed,w_hi", [((3, 3, 3, 3, 3), 5, 4), ((1, 2, 3, 4, 2), 6, 100),
                                             ((4, 4, 4), 7, 2)])
@pytest.mark.parametrize("k", [1, 5, 60, 100000])
def test_complete_multipartite_by_weight(sizes, seed, w_hi, k):
    g, parts = cf.multipartite(sizes, seed)
    w = np.random.default_rng(seed + 50).integers(1, w_hi + 1, g.n)
    cf.set_weights(g, w)
    want = cf.ranked(cf.transversals(parts), cf.weight_of(w))
    for bound in (0, 1):
        for priority in (0, 1):
            got, _ = oracle.topk_cliques(g, k, weighted=True, bound=bound, priority=priority)
            assert got == want[:k]


@pytest.mark.parametrize("m", [6, 8])
def test_moon_moser_count_and_top1_weight(m):
    """3^m maximal cliques of size m; the heaviest takes each part's heaviest
    vertex, the smallest id among equals (a smaller member gives a
    lexicographically smaller sorted list)."""
    g, parts = cf.multipartite((3,) * m, 10 + m)
    res, _ = oracle.topk_cliques(g, 3 ** m + 1)
    assert len(res) == 3 ** m and all(s == m for s, _ in res)
    assert res[0][1] == tuple(sorted(p[0] for p in parts))
    assert res[-1][1] == tuple(sorted(p[-1] for p in parts))
    w = np.random.default_rng(m).integers(1, 4, g.n)
    cf.set_weights(g, w)
    best = [min(p, key=lambda v: (-int(w[v]), v)) for p in parts]
    got, _ = oracle.topk_cliques(g, 1, weighted=True)
    assert got == [(cf.weight_of(w)(best), tuple(sorted(best)))]


@pytest.mark.parametrize("n", [4, 5, 9, 30])
def test_cycle_edges_are_the_maximal_cliques(n):
    g, edges = cf.cycle(n, n)
    want = cf.ranked(edges)
    for k in (1, 3, n, n + 5):
        got, _ = oracle.topk_cliques(g, k)
        assert got == want[:k]


def test_triangle_is_one_clique():
    import synth
    g = synth.from_edges(3, [(0, 1), (1, 2), (0, 2)])
    assert oracle.topk_cliques(g, 5)[0] == [(3, (0, 1, 2))]


@pytest.mark.parametrize("sizes,seed", [((5, 3, 5, 1, 2, 7), 1), ((4,) * 10, 2)])
def test_disjoint_complete_graphs(sizes, seed):
    g, comps = cf.disjoint_cliques(sizes, seed)
    w = np.random.default_rng(seed + 1).integers(1, 6, g.n)
    want = cf.ranked(comps)
    want_w = cf.ranked(comps, cf.weight_of(w))
    cf.set_weights(g, w)
    for k in (1, 2, len(sizes), 100):
        assert oracle.topk_cliques(g, k)[0] == want[:k]
        assert oracle.topk_cliques(g, k, weighted=True)[0] == want_w[:k]


# ---- labelled matching (Section 4.3; results are images of the pattern,
# each represented by its lexicographically smallest embedding tuple) ----

def _complete(n, weight=None):
    import synth
    g = synth.from_edges(n, [(u, v) for u in range(n) for v in range(u + 1, n)])
    g.vertex_label = np.zeros(n, np.uint8)
    if weight is not None:
        rp = g.row_ptr.astype(np.int64)
        g.edge_weight = np.array([weight(u, int(g.col[e])) for u in range(n)
                                  for e in range(rp[u], rp[u + 1])], np.int32)
    return g


def _ranked_matches(tuples, pattern_edges, weight):
    return sorted(((sum(weight(t[a], t[b]) for a, b in pattern_edges), t) for t in tuples),
                  key=lambda x: (-x[0], x[1]))


@pytest.mark.parametrize("weighted", [False, True])
def test_paths_in_a_complete_graph(weighted):
    """A path a-b-c-d has two automorphisms (itself and its reversal), so its
    images in K_n are the ordered 4-tuples of distinct vertices with a < d:
    n(n-1)(n-2)(n-3)/2 of them."""
    n = 9
    w = (lambda u, v: u + v + 1) if weighted else (lambda u, v: 1)
    g = _complete(n, w if weighted else None)
    edges = [(0, 1), (1, 2), (2, 3)]
    reps = [t for t in itertools.permutations(range(n), 4) if t[0] < t[3]]
    assert len(reps) == n * (n - 1) * (n - 2) * (n - 3) // 2
    want = _ranked_matches(reps, edges, w)
    for k in (1, 17, len(reps), len(reps) + 5):
        got, _ = oracle.topk_match(g, [0] * 4, edges, k, n_labels=1)
        assert got == want[:k]


def test_four_cycles_in_a_complete_graph():
    """A 4-cycle has eight automorphisms; the smallest tuple of an image
    starts at its smallest vertex and goes first to the smaller of that
    vertex's two cycle neighbours."""
    n = 8
    w = lambda u, v: (u * v) % 7 + 1
    g = _complete(n, w)
    edges = [(0, 1), (1, 2), (2, 3), (3, 0)]
    reps = [t for t in itertools.permutations(range(n), 4)
            if t[0] < min(t[1], t[2], t[3]) and t[1] < t[3]]
    assert len(reps) == n * (n - 1) * (n - 2) * (n - 3) // 8
    want = _ranked_matches(reps, edges, w)
    for k in (1, 40, len(reps) + 1):
        got, _ = oracle.topk_match(g, [0] * 4, edges, k, n_labels=1)
        assert got == want[:k]


def test_labelled_paths_in_a_complete_bipartite_graph():
    """K_{a,b} with label 0 on one side and 1 on the other: the pattern
    0-1-0 has one image per (middle vertex, pair of ends); the swap of the
    ends is its only automorphism, so the first end is the smaller one.  The
    pattern 1-0-1-0 (a path with labels alternating) has no automorphism
    preserving labels but the identity."""
    import synth
    a, b = 5, 4
    left, right = list(range(0, 2 * a, 2)), list(range(1, 2 * b + 1, 2))  # interleaved ids
    n = a + b
    ids = sorted(left + right)
    assert ids == list(range(n))
    g = synth.from_edges(n, [(u, v) for u in left for v in right])
    lab = np.zeros(n, np.uint8)
    lab[right] = 1
    g.vertex_label = lab
    w = lambda u, v: 3 * u + 5 * v + (u * v) % 4 + 1
    wsym = lambda u, v: w(min(u, v), max(u, v))
    rp = g.row_ptr.astype(np.int64)
    g.edge_weight = np.array([wsym(u, int(g.col[e])) for u in range(n)
                              for e in range(rp[u], rp[u + 1])], np.int32)
    e3 = [(0, 1), (1, 2)]
    reps = [(x, m, y) for m in right for x in left for y in left if x < y]
    assert len(reps) == b * a * (a - 1) // 2
    want = _ranked_matches(reps, e3, wsym)
    got, _ = oracle.topk_match(g, [0, 1, 0], e3, len(reps) + 3, n_labels=2)
    assert got == want
    e4 = [(0, 1), (1, 2), (2, 3)]
    reps4 = [(p, q, r, s) for p in right for q in left for r in right for s in left
             if p != r and q != s]
    want4 = _ranked_matches(reps4, e4, wsym)
    for k in (1, 9, len(reps4) + 1):
        got, _ = oracle.topk_match(g, [1, 0, 1, 0], e4, k, n_labels=2)
        assert got == want4[:k]
