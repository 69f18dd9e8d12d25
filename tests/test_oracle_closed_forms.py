"""Closed-form pins for the oracle's top-k maximal cliques (no GPU).

Families whose maximal cliques are known without search:
  - complete multipartite graphs: a set is a maximal clique exactly when it
    takes one vertex from every part, so there are prod(|part|) of them, all
    of size (number of parts); parts of three give the Moon-Moser graphs,
    which have the most maximal cliques of any graph on their vertex count;
  - cycles of length n >= 4: the n edges;
  - disjoint unions of complete graphs: the components.
Vertex ids are shuffled so that parts and components are not id ranges, and
the results of the paper's ranking (score descending, then the ascending id
list lexicographically, readings of Section 3.2) are written out directly.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth


def _multipartite(sizes, seed):
    n = sum(sizes)
    perm = np.random.default_rng(seed).permutation(n)
    parts, at = [], 0
    for s in sizes:
        parts.append(sorted(int(v) for v in perm[at:at + s]))
        at += s
    edges = [(u, v) for a, b in itertools.combinations(range(len(parts)), 2)
             for u in parts[a] for v in parts[b]]
    return synth.from_edges(n, edges), parts


def _weights(g, w):
    g.vertex_weight = np.asarray(w, np.int32)
    return g


def _ranked(cliques, score):
    return sorted(((score(c), c) for c in cliques), key=lambda t: (-t[0], t[1]))


@pytest.mark.parametrize("sizes,seed", [((3, 3, 3, 3, 3), 1), ((1, 2, 3, 4, 2), 2),
                                        ((5, 1, 1, 4), 3), ((2,) * 9, 4)])
@pytest.mark.parametrize("k", [1, 7, 48, 100000])
def test_complete_multipartite_by_size(sizes, seed, k):
    g, parts = _multipartite(sizes, seed)
    want = _ranked([tuple(sorted(t)) for t in itertools.product(*parts)], len)
    assert len(want) == int(np.prod(sizes))
    for bound in (0, 1):
        got, _ = oracle.topk_cliques(g, k, bound=bound)
        assert got == want[:k]


@pytest.mark.parametrize("sizes,seed,w_hi", [((3, 3, 3, 3, 3), 5, 4), ((1, 2, 3, 4, 2), 6, 100),
                                             ((4, 4, 4), 7, 2)])
@pytest.mark.parametrize("k", [1, 5, 60, 100000])
def test_complete_multipartite_by_weight(sizes, seed, w_hi, k):
    g, parts = _multipartite(sizes, seed)
    w = np.random.default_rng(seed + 50).integers(1, w_hi + 1, g.n)
    _weights(g, w)
    want = _ranked([tuple(sorted(t)) for t in itertools.product(*parts)],
                   lambda c: int(sum(int(w[v]) for v in c)))
    for bound in (0, 1):
        for priority in (0, 1):
            got, _ = oracle.topk_cliques(g, k, weighted=True, bound=bound, priority=priority)
            assert got == want[:k]


@pytest.mark.parametrize("m", [6, 8])
def test_moon_moser_count_and_top1_weight(m):
    """3^m maximal cliques of size m; the heaviest takes each part's heaviest
    vertex, the smallest id among equals (a smaller member gives a
    lexicographically smaller sorted list)."""
    g, parts = _multipartite((3,) * m, 10 + m)
    res, _ = oracle.topk_cliques(g, 3 ** m + 1)
    assert len(res) == 3 ** m and all(s == m for s, _ in res)
    assert res[0][1] == tuple(sorted(p[0] for p in parts))
    assert res[-1][1] == tuple(sorted(p[-1] for p in parts))
    w = np.random.default_rng(m).integers(1, 4, g.n)
    _weights(g, w)
    best = [min(p, key=lambda v: (-int(w[v]), v)) for p in parts]
    got, _ = oracle.topk_cliques(g, 1, weighted=True)
    assert got == [(int(sum(int(w[v]) for v in best)), tuple(sorted(best)))]


@pytest.mark.parametrize("n", [4, 5, 9, 30])
def test_cycle_edges_are_the_maximal_cliques(n):
    perm = np.random.default_rng(n).permutation(n)
    edges = [(int(perm[i]), int(perm[(i + 1) % n])) for i in range(n)]
    g = synth.from_edges(n, edges)
    want = sorted((2, tuple(sorted(e))) for e in edges)
    for k in (1, 3, n, n + 5):
        got, _ = oracle.topk_cliques(g, k)
        assert got == want[:k]


def test_triangle_is_one_clique():
    g = synth.from_edges(3, [(0, 1), (1, 2), (0, 2)])
    assert oracle.topk_cliques(g, 5)[0] == [(3, (0, 1, 2))]


@pytest.mark.parametrize("sizes,seed", [((5, 3, 5, 1, 2, 7), 1), ((4,) * 10, 2)])
def test_disjoint_complete_graphs(sizes, seed):
    n = sum(sizes)
    perm = np.random.default_rng(seed).permutation(n)
    comps, edges, at = [], [], 0
    for s in sizes:
        c = sorted(int(v) for v in perm[at:at + s])
        comps.append(tuple(c))
        edges += list(itertools.combinations(c, 2))
        at += s
    g = synth.from_edges(n, edges)
    w = np.random.default_rng(seed + 1).integers(1, 6, n)
    want = _ranked(comps, len)
    want_w = _ranked(comps, lambda c: int(sum(int(w[v]) for v in c)))
    _weights(g, w)
    for k in (1, 2, len(sizes), 100):
        assert oracle.topk_cliques(g, k)[0] == want[:k]
        assert oracle.topk_cliques(g, k, weighted=True)[0] == want_w[:k]
