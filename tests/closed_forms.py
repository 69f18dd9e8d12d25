"""Graphs whose maximal cliques are known in closed form, with their top-k.

  - complete multipartite graphs: a set is a maximal clique exactly when it
    takes one vertex from every part, so there are prod(|part|) of them, all
    of size (number of parts); parts of three give the Moon-Moser graphs,
    which have the most maximal cliques of any graph on their vertex count;
  - cycles of length n >= 4: the n edges;
  - disjoint unions of complete graphs: the components.
Vertex ids are shuffled (seeded) so that parts and components are not id
ranges.  The ranking is score descending, then the ascending id list
compared lexicographically.
"""
import itertools

import numpy as np

import synth


def multipartite(sizes, seed):
    """(graph, parts): the complete multipartite graph with the given part sizes."""
    n = sum(sizes)
    perm = np.random.default_rng(seed).permutation(n)
    parts, at = [], 0
    for s in sizes:
        parts.append(sorted(int(v) for v in perm[at:at + s]))
        at += s
    edges = [(u, v) for a, b in itertools.combinations(range(len(parts)), 2)
             for u in parts[a] for v in parts[b]]
    return synth.from_edges(n, edges), parts


def transversals(parts):
    """The maximal cliques of a complete multipartite graph, ids ascending."""
    return [tuple(sorted(t)) for t in itertools.product(*parts)]


def cycle(n, seed):
    """(graph, edges): a cycle through all n vertices in a shuffled order."""
    perm = np.random.default_rng(seed).permutation(n)
    edges = [tuple(sorted((int(perm[i]), int(perm[(i + 1) % n])))) for i in range(n)]
    return synth.from_edges(n, edges), edges


def disjoint_cliques(sizes, seed):
    """(graph, components): disjoint complete graphs of the given sizes."""
    n = sum(sizes)
    perm = np.random.default_rng(seed).permutation(n)
    comps, edges, at = [], [], 0
    for s in sizes:
        c = tuple(sorted(int(v) for v in perm[at:at + s]))
        comps.append(c)
        edges += list(itertools.combinations(c, 2))
        at += s
    return synth.from_edges(n, edges), comps


def set_weights(g, w):
    g.vertex_weight = np.asarray(w, np.int32)
    return g


def ranked(cliques, score=len):
    """[(score, ids)] best first."""
    return sorted(((score(c), c) for c in cliques), key=lambda t: (-t[0], t[1]))


def weight_of(w):
    return lambda c: int(sum(int(w[v]) for v in c))
