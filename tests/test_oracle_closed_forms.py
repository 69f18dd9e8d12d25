"""Closed-form pins for the oracle's top-k maximal cliques (no GPU).

The graph families and their maximal cliques are those of
tests/closed_forms.py (complete multipartite and Moon-Moser graphs, cycles,
disjoint complete graphs); the expected top-k is the closed form ranked by
score descending, then ids ascending (the result order of Section 3.2).
"""
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
