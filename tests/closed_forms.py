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


def dense_core_in_background(singletons, multi, decoy_parts, n_background, seed):
    """A graph whose large maximal cliques are known in closed form.

    Core A: a complete multipartite graph with `singletons` parts of one
    vertex (adjacent to every other core vertex) and the parts listed in
    `multi` (sizes 2 or 3).  Its maximal cliques are the transversals, of
    size = number of parts s.  Decoy D: a complete multipartite graph with
    `decoy_parts` parts of two vertices (its cliques have decoy_parts < s
    vertices), every decoy vertex also joined to 5 random core vertices, so
    that decoy degrees reach s - 1 while no decoy edge has s - 2 common
    neighbours.  Background: a sparse Chung-Lu graph on n_background
    vertices (expected degrees 2..40), every background vertex also joined
    to 2 random core or decoy vertices.  Ids are shuffled.

    Returns (graph, s, singleton ids, multi parts as id lists, decoy ids).
    """
    rng = np.random.default_rng(seed)
    sizes_a = [1] * singletons + list(multi)
    n_a = sum(sizes_a)
    n_d = 2 * decoy_parts
    n = n_a + n_d + n_background
    perm = rng.permutation(n)
    a_ids = perm[:n_a]
    d_ids = perm[n_a:n_a + n_d]
    b_ids = perm[n_a + n_d:]
    parts, at = [], 0
    for sz in sizes_a:
        parts.append([int(v) for v in a_ids[at:at + sz]])
        at += sz
    dparts = [[int(d_ids[2 * i]), int(d_ids[2 * i + 1])] for i in range(decoy_parts)]
    edges = set()

    def add(u, v):
        u, v = int(u), int(v)
        if u != v:
            edges.add((min(u, v), max(u, v)))

    for group in (parts, dparts):
        flat = [(v, i) for i, pt in enumerate(group) for v in pt]
        for x in range(len(flat)):
            for y in range(x + 1, len(flat)):
                if flat[x][1] != flat[y][1]:
                    add(flat[x][0], flat[y][0])
    for v in d_ids:
        for u in rng.choice(a_ids, 5, replace=False):
            add(v, u)
    # sparse Chung-Lu background: p_uv = w_u w_v / sum(w)
    w = rng.uniform(2.0, 40.0, n_background)
    tot = w.sum()
    for i in range(n_background):
        pr = np.minimum(1.0, w[i] * w[i + 1:] / tot)
        hit = np.flatnonzero(rng.random(n_background - i - 1) < pr)
        for j in hit:
            add(b_ids[i], b_ids[i + 1 + j])
    targets = np.concatenate([a_ids, d_ids])
    for v in b_ids:
        for u in rng.choice(targets, 2, replace=False):
            add(v, u)
    g = synth.from_edges(n, sorted(edges))
    single = sorted(pt[0] for pt in parts if len(pt) == 1)
    multi_parts = [sorted(pt) for pt in parts if len(pt) > 1]
    return g, len(parts), single, multi_parts, sorted(int(v) for v in d_ids)
