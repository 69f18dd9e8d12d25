"""Pins for the CPU oracle's top-k clique search (no GPU).

The oracle is checked against things other than itself: the paper's worked
example (Section 3.2), brute force over every vertex subset, networkx's
Bron-Kerbosch and maximum-weight-clique routines, the planted cliques of the
small planted-clique workload, and invariants (prefix property, independence
of the bound, priority and vertex order).
"""
import os

import networkx as nx
import numpy as np
import pytest

import oracle
import synth
from tests import bruteforce, closed_forms

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load_worked_example():
    spec = {"pops": []}
    with open(os.path.join(GOLDEN, "worked_example_max_clique.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tag, _, rest = line.partition(" ")
            if tag == "n":
                spec["n"] = int(rest)
            elif tag == "k":
                spec["k"] = int(rest)
            elif tag == "edges":
                spec["edges"] = [tuple(int(x) for x in e.split("-")) for e in rest.split()]
            elif tag == "pop":
                ids, _, flags = rest.partition("|")
                spec["pops"].append((tuple(int(x) for x in ids.split()),
                                     *(int(x) for x in flags.split())))
            elif tag == "result":
                spec["result"] = tuple(int(x) for x in rest.split())
            elif tag == "children_created":
                spec["children"] = int(rest)
    return spec


def test_worked_example_trace_matches_paper():
    """Section 3.2: pop order, result set, pruned subgraphs and children."""
    spec = _load_worked_example()
    g = synth.from_edges(spec["n"], spec["edges"])
    pops, R, st = oracle.clique_trace(g, spec["k"])
    assert pops == spec["pops"]
    assert R == [spec["result"]]
    assert st["children"] == spec["children"]
    # the four pruned subgraphs are s6 = {v1, v3}, s2, s3, s4
    pruned = [p[0] for p in pops if p[2] == 1]
    assert pruned == [(0, 2), (1,), (2,), (3,)]


def test_worked_example_graph_has_nine_cliques():
    """Section 2.1: the example graph has 9 cliques of sizes 1 to 3."""
    spec = _load_worked_example()
    g = synth.from_edges(spec["n"], spec["edges"])
    adj = bruteforce.adjacency_masks(g)
    cliques = [m for m in range(1, 16)
               if all((adj[v] | 1 << v) & m == m for v in range(4) if m >> v & 1)]
    assert len(cliques) == 9
    assert max(bin(m).count("1") for m in cliques) == 3


def test_worked_example_maximal_mode():
    spec = _load_worked_example()
    g = synth.from_edges(spec["n"], spec["edges"])
    res, _ = oracle.topk_cliques(g, 5)
    assert res == [(3, (0, 1, 2)), (2, (2, 3))]


def _small_graphs():
    cases = []
    for n in (1, 2, 5, 8, 11, 13):
        for p in (0.0, 0.3, 0.6, 0.9, 1.0):
            cases.append((n, p, 1000 + 17 * n + int(100 * p)))
    return cases


@pytest.mark.parametrize("n,p,seed", _small_graphs())
def test_size_topk_matches_brute_force(n, p, seed):
    g = synth.gnp(n, p, seed)
    for k in (1, 3, 1000):
        want = bruteforce.topk_cliques(g, k)
        for xprune in (False, True):
            got, _ = oracle.topk_cliques(g, k, xprune=xprune)
            assert got == want, (n, p, seed, k, xprune)


@pytest.mark.parametrize("n,p,seed", [c for c in _small_graphs() if c[0] >= 5])
def test_weighted_topk_matches_brute_force(n, p, seed):
    g = synth.gnp(n, p, seed)
    synth.add_vertex_weights(g, 1, 3, master=seed)  # small range: deliberate score ties
    for k in (1, 4, 1000):
        want = bruteforce.topk_cliques(g, k, weights=g.vertex_weight)
        for xprune in (False, True):
            got, _ = oracle.topk_cliques(g, k, weighted=True, xprune=xprune)
            assert got == want, (n, p, seed, k, xprune)


@pytest.mark.parametrize("bound", [0, 1])
@pytest.mark.parametrize("priority", [0, 1, 2])
@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("xprune", [False, True])
def test_result_independent_of_bound_priority_order(bound, priority, order, xprune):
    g = synth.gnp(40, 0.35, 77)
    synth.add_vertex_weights(g, 1, 5, master=77)
    ref_s, _ = oracle.topk_cliques(g, 25)
    ref_w, _ = oracle.topk_cliques(g, 25, weighted=True)
    got_s, _ = oracle.topk_cliques(g, 25, bound=bound, priority=priority, order=order,
                                   xprune=xprune)
    got_w, _ = oracle.topk_cliques(g, 25, weighted=True, bound=bound, priority=priority,
                                   order=order, xprune=xprune)
    assert got_s == ref_s
    assert got_w == ref_w


def test_pruning_reduces_work_but_not_result():
    """Priority + pruning (Nuri) explores less than FIFO order (Nuri-NP-like), same answer."""
    g = synth.gnp(60, 0.4, 5)
    a, sa = oracle.topk_cliques(g, 1, priority=0)
    b, sb = oracle.topk_cliques(g, 1, priority=2)
    assert a == b
    assert sa["children"] < sb["children"]


def test_extension_witness_makes_dense_graphs_tractable():
    """K_40 has one maximal clique; with k > 1 nothing is pruned by bounds,
    so only the maximality witness keeps the search polynomial."""
    kn = synth.from_edges(40, [(i, j) for i in range(40) for j in range(i + 1, 40)])
    res, st = oracle.topk_cliques(kn, 10)
    assert res == [(40, tuple(range(40)))]
    assert st["children"] < 40 * 40
    # near-clique: K_30 minus a perfect matching has 2^15 maximal cliques of size 15
    edges = [(i, j) for i in range(30) for j in range(i + 1, 30) if not (j == i + 1 and i % 2 == 0)]
    g = synth.from_edges(30, edges)
    res, _ = oracle.topk_cliques(g, 5)
    assert [s for s, _ in res] == [15] * 5
    assert res[0][1] == tuple(range(0, 30, 2))


def test_against_networkx_bron_kerbosch():
    g = synth.gnp(120, 0.25, 9)
    synth.add_vertex_weights(g, 1, 100, master=9)
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    for u in range(g.n):
        for e in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1])):
            G.add_edge(u, int(g.col[e]))
    cl = [tuple(sorted(c)) for c in nx.find_cliques(G)]
    w = g.vertex_weight
    for k in (1, 10, 200, 100000):
        want = sorted(((len(c), c) for c in cl), key=lambda t: (-t[0], t[1]))[:k]
        got, _ = oracle.topk_cliques(g, k)
        assert got == want
        want_w = sorted(((int(sum(int(w[v]) for v in c)), c) for c in cl),
                        key=lambda t: (-t[0], t[1]))[:k]
        got_w, _ = oracle.topk_cliques(g, k, weighted=True)
        assert got_w == want_w


def test_top1_weight_matches_networkx_max_weight_clique():
    g = synth.gnp(70, 0.3, 31)
    synth.add_vertex_weights(g, 1, 100, master=31)
    G = nx.Graph()
    for v in range(g.n):
        G.add_node(v, weight=int(g.vertex_weight[v]))
    for u in range(g.n):
        for e in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1])):
            G.add_edge(u, int(g.col[e]))
    _, wmax = nx.max_weight_clique(G, weight="weight")
    got, _ = oracle.topk_cliques(g, 1, weighted=True)
    assert got[0][0] == wmax


def test_planted_cliques_recovered():
    """Planted-clique workload: n=2000, average degree 20, 10 planted cliques of 8..15.

    With p = 20/1999 the background graph almost surely has no clique larger
    than 4, so the 10 largest maximal cliques are exactly the planted ones.
    """
    g = synth.er_planted()
    res, _ = oracle.topk_cliques(g, 10)
    want = sorted(((len(p), tuple(int(x) for x in p)) for p in g.planted),
                  key=lambda t: (-t[0], t[1]))
    assert res == want


def test_prefix_property():
    g = synth.gnp(80, 0.3, 8)
    synth.add_vertex_weights(g, 1, 4, master=8)
    big, _ = oracle.topk_cliques(g, 300, weighted=True)
    for k in (1, 2, 7, 50, 299):
        small, _ = oracle.topk_cliques(g, k, weighted=True)
        assert small == big[:k]


def test_isolated_vertices_and_lone_edges_are_results():
    g = synth.from_edges(5, [(0, 1)])
    res, _ = oracle.topk_cliques(g, 10)
    assert res == [(2, (0, 1)), (1, (2,)), (1, (3,)), (1, (4,))]


def test_results_are_cliques_and_maximal():
    g = synth.gnp(50, 0.5, 3)
    adj = bruteforce.adjacency_masks(g)
    res, _ = oracle.topk_cliques(g, 40)
    for s, ids in res:
        m = sum(1 << v for v in ids)
        assert all((adj[v] | 1 << v) & m == m for v in ids)
        assert not any(adj[u] & m == m for u in range(g.n) if u not in ids)
        assert s == len(ids)
    keys = [(-s, ids) for s, ids in res]
    assert keys == sorted(keys) and len(set(keys)) == len(keys)


def test_k_zero_rejected():
    g = synth.gnp(5, 0.5, 1)
    with pytest.raises(ValueError):
        oracle.topk_cliques(g, 0)


def test_degeneracy_order_is_a_permutation_with_small_out_degree():
    g = synth.gnp(200, 0.1, 4)
    pi = oracle.vertex_order(g, 1)
    assert sorted(pi.tolist()) == list(range(g.n))
    G = nx.Graph()
    for u in range(g.n):
        for e in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1])):
            G.add_edge(u, int(g.col[e]))
    degeneracy = max(nx.core_number(G).values())
    outdeg = [sum(1 for e in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1]))
                  if pi[int(g.col[e])] > pi[u]) for u in range(g.n)]
    assert max(outdeg) == degeneracy


@pytest.mark.parametrize("seed", range(12))
def test_large_clique_kernel_is_exact(seed):
    """The oracle on the reduced graph (core and truss peeling, common
    vertices taken out) gives the same maximal cliques of at least s
    vertices as brute force on the whole graph."""
    g = synth.gnp(13, 0.45 + 0.04 * (seed % 6), seed)
    want_all = bruteforce.topk_cliques(g, 100000)
    for s in (3, 4, 5, 6, 8):
        want = [x for x in want_all if x[0] >= s]
        resid, rid, common = oracle.large_clique_kernel(g, s)
        if resid.n:
            res, _ = oracle.topk_cliques(resid, 100000)
            cand = [common + [int(rid[i]) for i in ids] for _, ids in res]
        else:
            cand = [common] if common else []
        got = sorted(((len(c), tuple(sorted(c))) for c in cand if len(c) >= s),
                     key=lambda t: (-t[0], t[1]))
        assert got == want, (seed, s)


def test_large_clique_kernel_on_planted_workload():
    g = synth.er_planted()
    want, _ = oracle.topk_cliques(g, 10)
    s = min(size for size, _ in want)
    resid, rid, common = oracle.large_clique_kernel(g, s)
    res, _ = oracle.topk_cliques(resid, 10)
    got = sorted(((len(common) + len(ids), tuple(sorted(common + [int(rid[i]) for i in ids])))
                  for _, ids in res), key=lambda t: (-t[0], t[1]))
    assert got == want


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_core_numbers_match_networkx(seed):
    g = synth.gnp(150, 0.05 * seed, seed)
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    for u in range(g.n):
        for e in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1])):
            G.add_edge(u, int(g.col[e]))
    want = nx.core_number(G)
    got = oracle.core_numbers(g)
    assert [int(got[v]) for v in range(g.n)] == [want[v] for v in range(g.n)]


def test_induced_subgraph_keeps_edges_weights_and_id_order():
    g = synth.gnp(60, 0.2, 7)
    synth.add_vertex_weights(g, 1, 50, master=7)
    keep = np.zeros(g.n, bool)
    keep[np.random.default_rng(7).choice(g.n, 35, replace=False)] = True
    sub, old = oracle.induced_subgraph(g, keep)
    assert list(old) == sorted(np.flatnonzero(keep).tolist())
    edges = {(int(old[u]), int(old[sub.col[e]])) for u in range(sub.n)
             for e in range(int(sub.row_ptr[u]), int(sub.row_ptr[u + 1]))}
    want = {(u, int(g.col[e])) for u in range(g.n) if keep[u]
            for e in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1])) if keep[g.col[e]]}
    assert edges == want
    assert list(sub.vertex_weight) == [int(g.vertex_weight[v]) for v in old]


@pytest.mark.parametrize("shape", [
    # (singleton parts, multi-vertex parts, decoy parts, background vertices, seed)
    (290, [2] * 6 + [3] * 4, 148, 3000, 11),
    (400, [2] * 30 + [3] * 20, 224, 3000, 12),
])
def test_large_clique_kernel_on_dense_cores_in_a_sparse_graph(shape):
    """The reduction at the shape it is used on: a dense core of 300-520
    vertices (a complete multipartite graph whose one-vertex parts are
    adjacent to everything else in it) inside a sparse power-law graph,
    next to a decoy core whose vertices pass the degree test but whose
    edges fail the common-neighbour test.  The maximal cliques with s =
    (number of parts) vertices are exactly the singletons plus a transversal
    of the other parts, so the kernel must return the singletons as common
    vertices and, as residual, exactly the other parts with the edges
    between different parts."""
    singletons, multi, decoy_parts, n_bg, seed = shape
    g, s, single, parts, decoys = closed_forms.dense_core_in_background(
        singletons, multi, decoy_parts, n_bg, seed)
    core = oracle.core_numbers(g)
    # the decoys survive core peeling: only the common-neighbour test removes them
    assert all(int(core[v]) >= s - 1 for v in decoys)
    resid, rid, common = oracle.large_clique_kernel(g, s)
    assert common == single
    members = sorted(v for pt in parts for v in pt)
    assert sorted(int(x) for x in rid) == members
    part_of = {v: i for i, pt in enumerate(parts) for v in pt}
    got_edges = {(int(rid[u]), int(rid[resid.col[e]])) for u in range(resid.n)
                 for e in range(int(resid.row_ptr[u]), int(resid.row_ptr[u + 1]))}
    want_edges = {(u, v) for u in members for v in members if part_of[u] != part_of[v]}
    assert got_edges == want_edges
    if len(parts) <= 12:
        # the search on the residual, lifted back, ranks the transversals
        k = 40
        res, _ = oracle.topk_cliques(resid, k)
        got = [(len(common) + len(ids), tuple(sorted(common + [int(rid[i]) for i in ids])))
               for _, ids in res]
        full = [tuple(sorted(single + list(t))) for t in closed_forms.transversals(parts)]
        assert got == closed_forms.ranked(full)[:k]
        assert all(size == s for size, _ in got)


def test_work_limit_stops_the_search_and_resets():
    """A capped search stops once it has created the cap's children and
    returns no result; with the cap removed the same query is exact."""
    g = synth.er_planted()
    want, st_full = oracle.topk_cliques(g, 10)
    cap = st_full["children"] // 4
    oracle.set_work_limit(cap)
    try:
        res, st = oracle.topk_cliques(g, 10)
    finally:
        oracle.set_work_limit(0)
    assert res is None
    assert cap <= st["children"] < st_full["children"]
    again, st2 = oracle.topk_cliques(g, 10)
    assert again == want and st2["children"] == st_full["children"]
