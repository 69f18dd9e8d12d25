"""Brute-force references for tiny graphs (test-only, pure Python).

These enumerate every vertex subset or every injective map, so they are
independent of the best-first search both the oracle and the GPU engine use.
"""
from __future__ import annotations

import itertools
from typing import Dict, List, Sequence, Tuple


def adjacency_masks(g) -> List[int]:
    masks = [0] * g.n
    for u in range(g.n):
        for e in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1])):
            masks[u] |= 1 << int(g.col[e])
    return masks


def all_maximal_cliques(g) -> List[Tuple[int, ...]]:
    """Every maximal clique, by testing all 2^n vertex subsets (n <= ~16)."""
    n = g.n
    adj = adjacency_masks(g)
    out = []
    for mask in range(1, 1 << n):
        members = [v for v in range(n) if mask >> v & 1]
        if any((adj[v] | (1 << v)) & mask != mask for v in members):
            continue
        if any(adj[u] & mask == mask for u in range(n) if not mask >> u & 1):
            continue
        out.append(tuple(members))
    return out


def topk_cliques(g, k: int, weights: Sequence[int] = None):
    """Top-k maximal cliques under (score desc, ascending id tuple asc)."""
    cl = all_maximal_cliques(g)
    def score(c):
        return sum(int(weights[v]) for v in c) if weights is not None else len(c)
    ranked = sorted(cl, key=lambda c: (-score(c), c))
    return [(score(c), c) for c in ranked[:k]]


def all_images(g, labels: Sequence[int], edges: Sequence[Tuple[int, int]],
               score: str = "edge"):
    """Every injective, label- and edge-preserving map, grouped by image.

    score "edge": sum of the weights of the data edges under the pattern
    edges; "degree": sum of the degrees of the matched data vertices.
    Returns {image_key: (score, lexicographically smallest mu tuple)}.
    """
    q = len(labels)
    n = g.n
    adj = [set() for _ in range(n)]
    w: Dict[Tuple[int, int], int] = {}
    for u in range(n):
        for e in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1])):
            v = int(g.col[e])
            adj[u].add(v)
            w[(u, v)] = int(g.edge_weight[e]) if g.edge_weight is not None else 1
    lab = [int(x) for x in g.vertex_label]
    images = {}
    for mu in itertools.permutations(range(n), q):
        if any(lab[mu[a]] != labels[a] for a in range(q)):
            continue
        if any(mu[b] not in adj[mu[a]] for a, b in edges):
            continue
        vs = frozenset(mu)
        es = frozenset(frozenset((mu[a], mu[b])) for a, b in edges)
        key = (vs, es)
        if score == "degree":
            sc = sum(len(adj[v]) for v in mu)
        else:
            sc = sum(w[(mu[a], mu[b])] for a, b in edges)
        if key not in images or mu < images[key][1]:
            images[key] = (sc, mu)
    return images


def topk_matches(g, labels, edges, k, score: str = "edge"):
    imgs = all_images(g, labels, edges, score)
    ranked = sorted(imgs.values(), key=lambda t: (-t[0], t[1]))
    return [(s, mu) for s, mu in ranked[:k]], len(imgs)


def count_monomorphisms(g, labels, edges) -> int:
    q = len(labels)
    n = g.n
    adj = adjacency_masks(g)
    lab = [int(x) for x in g.vertex_label]
    c = 0
    for mu in itertools.permutations(range(n), q):
        if any(lab[mu[a]] != labels[a] for a in range(q)):
            continue
        if any(not (adj[mu[a]] >> mu[b] & 1) for a, b in edges):
            continue
        c += 1
    return c


def automorphism_count(labels, edges) -> int:
    q = len(labels)
    es = set(frozenset(e) for e in edges)
    c = 0
    for p in itertools.permutations(range(q)):
        if all(labels[p[a]] == labels[a] for a in range(q)) and \
                all(frozenset((p[a], p[b])) in es for a, b in edges):
            c += 1
    return c
