"""Metamorphic pin for the oracle (no GPU): renaming the vertices.

Scores do not depend on vertex ids, so under a random relabelling of the
data graph the score list of the top-k is unchanged, and every result whose
score is strictly above the k-th score (those are the same set whichever
ids break the ties) maps onto a result of the relabelled run.  Ties at the
k-th score are broken by ids (ascending id list for cliques, smallest
embedding tuple for matches), so the tied results are compared by a fresh
brute force on the relabelled graph instead.
"""
import numpy as np
import pytest

import oracle
import synth
from tests import bruteforce


def _relabel(g, perm):
    """g with vertex v renamed perm[v]; weights and labels move with it."""
    rp = g.row_ptr.astype(np.int64)
    edges = [(int(perm[u]), int(perm[g.col[e]])) for u in range(g.n)
             for e in range(rp[u], rp[u + 1]) if u < g.col[e]]
    h = synth.from_edges(g.n, edges)
    inv = np.argsort(perm)
    if g.vertex_weight is not None:
        h.vertex_weight = np.ascontiguousarray(g.vertex_weight[inv])
    if g.vertex_label is not None:
        h.vertex_label = np.ascontiguousarray(g.vertex_label[inv])
    if g.edge_weight is not None:
        w = {}
        for u in range(g.n):
            for e in range(rp[u], rp[u + 1]):
                w[(int(perm[u]), int(perm[g.col[e]]))] = int(g.edge_weight[e])
        hp = h.row_ptr.astype(np.int64)
        h.edge_weight = np.array([w[(u, int(h.col[e]))] for u in range(h.n)
                                  for e in range(hp[u], hp[u + 1])], np.int32)
    return h


def _above_kth(res):
    if not res:
        return []
    kth = res[-1][0]
    return [r for r in res if r[0] > kth]


@pytest.mark.parametrize("n,p,seed", [(40, 0.3, 1), (60, 0.2, 2), (13, 0.6, 3)])
@pytest.mark.parametrize("weighted", [False, True])
def test_cliques_under_relabelling(n, p, seed, weighted):
    g = synth.gnp(n, p, seed)
    synth.add_vertex_weights(g, 1, 5, master=seed)
    perm = np.random.default_rng(seed).permutation(n)
    h = _relabel(g, perm)
    for k in (1, 5, 30):
        a, _ = oracle.topk_cliques(g, k, weighted=weighted)
        b, _ = oracle.topk_cliques(h, k, weighted=weighted)
        assert [s for s, _ in a] == [s for s, _ in b]
        mapped = {(s, tuple(sorted(int(perm[v]) for v in ids))) for s, ids in _above_kth(a)}
        assert mapped == set(_above_kth(b))
    if n <= 13:
        want = bruteforce.topk_cliques(h, 30, weights=h.vertex_weight if weighted else None)
        assert oracle.topk_cliques(h, 30, weighted=weighted)[0] == want


PATTERNS = [([0, 1, 0], [(0, 1), (1, 2)]), ([0, 0, 0], [(0, 1), (1, 2), (0, 2)]),
            ([1, 0, 1, 0], [(0, 1), (1, 2), (2, 3)])]


@pytest.mark.parametrize("pi", range(len(PATTERNS)))
def test_matches_under_relabelling(pi):
    labels, edges = PATTERNS[pi]
    g = synth.gnp(30, 0.25, 40 + pi)
    synth.add_zipf_labels(g, n_labels=2, s=0.5, master=40 + pi)
    synth.add_edge_weights(g, 1, 6, master=40 + pi)
    perm = np.random.default_rng(pi).permutation(g.n)
    h = _relabel(g, perm)

    def image(mu, f=lambda v: v):
        return frozenset(frozenset((f(mu[a]), f(mu[b]))) for a, b in edges)

    for k in (1, 10, 60):
        a, _ = oracle.topk_match(g, labels, edges, k, n_labels=2)
        b, _ = oracle.topk_match(h, labels, edges, k, n_labels=2)
        assert [s for s, _ in a] == [s for s, _ in b]
        mapped = {(s, image(mu, lambda v: int(perm[v]))) for s, mu in _above_kth(a)}
        assert mapped == {(s, image(mu)) for s, mu in _above_kth(b)}
    want, _ = bruteforce.topk_matches(h, labels, edges, 60)
    assert oracle.topk_match(h, labels, edges, 60, n_labels=2)[0] == want
