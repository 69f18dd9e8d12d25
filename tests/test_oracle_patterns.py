"""Pins for the CPU oracle's top-k frequent pattern mining (no GPU).

Section 2.1 defines the minimum image-based support of a pattern and
Section 3.3 finds the k most frequent M-edge patterns by Algorithm 2 with
pattern-oriented expansion over minimum DFS codes.  Checked against the
worked example of those sections, networkx (isomorphism classes and
monomorphism images), the definition enumerated over every connected set
of M data edges, anti-monotonicity, and closed forms on one-label graphs.
"""
import itertools
import os

import networkx as nx
import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _fixture():
    rows = {}
    with open(os.path.join(GOLDEN, "worked_example_pattern_mining.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            key, *vals = line.split()
            rows.setdefault(key, []).append(vals)
    return rows


def _code(tokens):
    return tuple(tuple(int(x) for x in t.split("-")) for t in tokens)


def _example_graph(fx):
    n = int(fx["n"][0][0])
    edges = [tuple(int(x) for x in e.split("-")) for e in fx["edges"][0]]
    g = synth.from_edges(n, edges)
    g.vertex_label = np.array([int(x) for x in fx["labels"][0]], np.uint8)
    return g


def test_section_3_3_worked_example():
    fx = _fixture()
    g = _example_graph(fx)
    for name, f, *code in fx["support"]:
        assert oracle.pattern_support(g, _code(code)) == int(f), name
    # 8 one-edge subgraphs, in two groups (p2 first: support 3 > 2)
    res, st = oracle.topk_patterns(g, 1, 10)
    assert st["children"] == int(fx["one_edge_subgraphs"][0][0])
    assert res == [(3, ((0, 1, 1, 1),)), (2, ((0, 1, 0, 1),))]
    # the most frequent 2-edge pattern, and how the search reaches it
    want = fx["top1_two_edges"][0]
    res, st = oracle.topk_patterns(g, 2, 1)
    assert res == [(int(want[0]), _code(want[1:]))]
    trace = fx["top1_trace"][0]
    for key, val in zip(trace[0::2], trace[1::2]):
        assert st[key] == int(val), key
    # minimal code of the a-b-b path, and the order of the two codes
    assert oracle.min_dfs_code([1, 1, 0], [(0, 1), (1, 2)]) == ((0, 1, 0, 1), (1, 2, 1, 1))
    assert oracle.min_dfs_code([0, 1], [(0, 1)]) == ((0, 1, 0, 1),)


def _random_labelled_connected(rng, nv, ne, n_labels):
    while True:
        pairs = list(itertools.combinations(range(nv), 2))
        idx = rng.choice(len(pairs), size=ne, replace=False)
        edges = [pairs[i] for i in idx]
        G = nx.Graph()
        G.add_nodes_from(range(nv))
        G.add_edges_from(edges)
        if nx.is_connected(G):
            labels = [int(x) for x in rng.integers(0, n_labels, nv)]
            return labels, edges


def _nx_pattern(labels, edges):
    P = nx.Graph()
    for v, l in enumerate(labels):
        P.add_node(v, l=l)
    P.add_edges_from(edges)
    return P


@pytest.mark.parametrize("seed", range(6))
def test_min_dfs_code_is_a_canonical_form(seed):
    """Renamed copies of a pattern get its code; two patterns get the same
    code exactly when networkx finds them isomorphic (labels included)."""
    rng = np.random.default_rng(seed)
    pats = []
    for _ in range(14):
        nv = int(rng.integers(2, 6))
        ne = int(rng.integers(nv - 1, min(nv * (nv - 1) // 2, 6) + 1))
        pats.append(_random_labelled_connected(rng, nv, ne, 2))
    codes = []
    for labels, edges in pats:
        c = oracle.min_dfs_code(labels, edges)
        perm = rng.permutation(len(labels))
        lab2 = [0] * len(labels)
        for v, l in enumerate(labels):
            lab2[perm[v]] = l
        e2 = [(int(perm[a]), int(perm[b])) for a, b in edges]
        assert oracle.min_dfs_code(lab2, e2) == c
        assert len(c) == len(edges)
        codes.append(c)
    nm = nx.algorithms.isomorphism.categorical_node_match("l", None)
    for (a, ca), (b, cb) in itertools.combinations(zip(pats, codes), 2):
        iso = nx.is_isomorphic(_nx_pattern(*a), _nx_pattern(*b), node_match=nm)
        assert iso == (ca == cb)


def _nx_support(g, code):
    """Minimum image-based support from networkx's monomorphisms."""
    nv = 1 + max(max(e[0], e[1]) for e in code)
    labels = [0] * nv
    for i, j, li, lj in code:
        labels[i], labels[j] = li, lj
    P = _nx_pattern(labels, [(i, j) for i, j, _, _ in code])
    G = nx.Graph()
    for v in range(g.n):
        G.add_node(v, l=int(g.vertex_label[v]))
    for u in range(g.n):
        for v in g.col[g.row_ptr[u]:g.row_ptr[u + 1]]:
            G.add_edge(u, int(v))
    nm = nx.algorithms.isomorphism.categorical_node_match("l", None)
    images = [set() for _ in range(nv)]
    for m in nx.algorithms.isomorphism.GraphMatcher(G, P, node_match=nm) \
            .subgraph_monomorphisms_iter():
        for dv, pv in m.items():
            images[pv].add(dv)
    return min(len(s) for s in images)


def _labelled(n, p, seed, n_labels):
    g = synth.gnp(n, p, seed)
    synth.add_zipf_labels(g, n_labels=n_labels, s=0.5, master=seed)
    return g


@pytest.mark.parametrize("seed", range(4))
def test_support_equals_networkx_monomorphism_images(seed):
    g = _labelled(14, 0.3, 40 + seed, 2)
    res = oracle.topk_patterns_definition(g, 3, 10 ** 6) if g.m <= 64 else []
    res += oracle.topk_patterns(g, 2, 10 ** 6)[0]
    assert res
    for f, code in res[:25]:
        assert _nx_support(g, code) == f, code


@pytest.mark.parametrize("M", [1, 2, 3, 4])
@pytest.mark.parametrize("seed", range(5))
def test_algorithm_2_equals_the_definition(M, seed):
    n_labels = 1 + seed % 3
    g = _labelled(11, 0.35, 60 + 7 * seed + M, n_labels)
    if g.m > 64:
        pytest.skip("too many edges to enumerate")
    want = oracle.topk_patterns_definition(g, M, 10 ** 6)
    for k in (1, 2, 5, 10 ** 6):
        got, _ = oracle.topk_patterns(g, M, k)
        assert got == want[:k], (M, seed, k)


def test_support_never_grows_with_the_pattern():
    g = _labelled(16, 0.3, 9, 2)
    for M in (2, 3):
        for f, code in oracle.topk_patterns(g, M, 10 ** 6)[0]:
            # every connected sub-pattern with one edge fewer
            for drop in range(M):
                rest = [e for t, e in enumerate(code) if t != drop]
                nv = 1 + max(max(e[0], e[1]) for e in code)
                labels = [0] * nv
                for i, j, li, lj in code:
                    labels[i], labels[j] = li, lj
                used = sorted({v for e in rest for v in e[:2]})
                ren = {v: t for t, v in enumerate(used)}
                sub_edges = [(ren[e[0]], ren[e[1]]) for e in rest]
                try:
                    sub = oracle.min_dfs_code([labels[v] for v in used], sub_edges)
                except ValueError:
                    continue  # not connected
                assert oracle.pattern_support(g, sub) >= f


def test_one_label_closed_forms():
    """One label: the single edge has support = vertices of degree >= 1;
    the two-edge path's middle vertex maps to vertices of degree >= 2 and
    its ends to neighbours of those, and its support is the smaller count;
    the two-edge path is then the only 2-edge pattern."""
    g = synth.gnp(40, 0.08, 3)
    g.vertex_label = np.zeros(g.n, np.uint8)
    deg = np.diff(g.row_ptr).astype(np.int64)
    res, _ = oracle.topk_patterns(g, 1, 5)
    assert res == [(int((deg >= 1).sum()), ((0, 1, 0, 0),))]
    mid = deg >= 2
    ends = np.zeros(g.n, bool)
    for u in range(g.n):
        for v in g.col[g.row_ptr[u]:g.row_ptr[u + 1]]:
            if mid[int(v)]:
                ends[u] = True
    res, _ = oracle.topk_patterns(g, 2, 5)
    assert res == [(int(min(mid.sum(), ends.sum())), ((0, 1, 0, 0), (1, 2, 0, 0)))]


def test_k_larger_than_the_number_of_patterns_and_bad_arguments():
    g = _labelled(12, 0.3, 4, 2)
    allp = oracle.topk_patterns_definition(g, 2, 10 ** 6)
    got, _ = oracle.topk_patterns(g, 2, len(allp) + 50)
    assert got == allp
    with pytest.raises(ValueError):
        oracle.topk_patterns(g, 0, 5)
    with pytest.raises(ValueError):
        oracle.topk_patterns(g, 2, 0)


def _all_dfs_codes(labels, edges):
    """Every DFS code of a small connected labelled graph, in Python: from
    every start vertex, every choice of the next unvisited neighbour of the
    deepest path vertex that has one; a newly reached vertex's edges back to
    visited vertices (other than its discoverer) follow by ascending id."""
    nv = len(labels)
    adj = [set() for _ in range(nv)]
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    out = []

    def grow(ids, order, path, code):
        if len(code) == len(edges):
            out.append(tuple(code))
            return
        while path and not any(w not in ids for w in adj[path[-1]]):
            path = path[:-1]
        u = path[-1]
        for w in sorted(adj[u]):
            if w in ids:
                continue
            nid = len(order)
            ids2 = dict(ids)
            ids2[w] = nid
            code2 = code + [(ids[u], nid, labels[u], labels[w])]
            for k, x in enumerate(order):
                if x != u and x in adj[w]:
                    code2.append((nid, k, labels[w], labels[x]))
            grow(ids2, order + [w], path + [w], code2)

    for s in range(nv):
        grow({s: 0}, [s], [s], [])
    return out


def _key(e):
    i, j, li, lj = e
    return (0, j, 0, 0) if i > j else (1, -i, li, lj)


@pytest.mark.parametrize("seed", range(8))
def test_min_dfs_code_is_the_smallest_of_all_dfs_codes(seed):
    rng = np.random.default_rng(100 + seed)
    for _ in range(12):
        nv = int(rng.integers(2, 7))
        ne = int(rng.integers(nv - 1, min(nv * (nv - 1) // 2, 7) + 1))
        labels, edges = _random_labelled_connected(rng, nv, ne, 3)
        codes = _all_dfs_codes(labels, edges)
        want = min(codes, key=lambda c: [_key(e) for e in c])
        assert oracle.min_dfs_code(labels, edges) == want, (labels, edges)


@pytest.mark.parametrize("seed,M", [(13, 2), (81, 3), (135, 2), (135, 3)])
def test_ties_at_the_kth_support(seed, M):
    """Graphs where several patterns share the k-th support and the one
    with the smallest code sits below a group of exactly that support: the
    group must not be pruned (dominated means strictly below)."""
    n, nl = 8 + seed % 5, 1 + seed % 2
    g = synth.gnp(n, 0.4, 1000 + seed)
    synth.add_zipf_labels(g, n_labels=nl, s=0.5, master=1000 + seed)
    want = oracle.topk_patterns_definition(g, M, 10 ** 6)
    for k in (1, 2, 3):
        assert oracle.topk_patterns(g, M, k)[0] == want[:k], k
