"""CPU oracle for top-k subgraph discovery -- test infrastructure only.

A plain, slow rendering of the paper's Algorithm 1 (Section 3.2) for top-k
maximal cliques and top-k labelled subgraph matching, and of Algorithm 2
(Section 3.3) and its definition for top-k frequent patterns, in oracle.c,
plus this ctypes loader.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import it; the GPU engine never does, and the two share
no code.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import List, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build() -> str:
    src = os.path.join(_HERE, "oracle.c")
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, src])
    os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    lib = ctypes.CDLL(_SO)
    vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    lib.oracle_topk_cliques.restype = ctypes.c_int64
    lib.oracle_topk_cliques.argtypes = [u32, vp, vp, vp, u32, i32, i32, i32, i32, i32, vp, vp, vp, u64,
                                        vp]
    lib.oracle_clique_trace.restype = ctypes.c_int64
    lib.oracle_clique_trace.argtypes = [u32, vp, vp, u32, vp, u64, vp, u64, vp]
    lib.oracle_topk_match.restype = ctypes.c_int64
    lib.oracle_topk_match.argtypes = [u32, vp, vp, vp, vp, u32, u32, vp, u32, vp, u32, i32, vp, vp, vp]
    lib.oracle_topk_match_degree.restype = ctypes.c_int64
    lib.oracle_topk_match_degree.argtypes = [u32, vp, vp, vp, u32, u32, vp, u32, vp, u32, i32, vp, vp,
                                             vp]
    lib.oracle_hop_index.argtypes = [u32, vp, vp, vp, u32, u32, vp]
    lib.oracle_match_root_bounds.restype = ctypes.c_int64
    lib.oracle_match_root_bounds.argtypes = [u32, vp, vp, vp, vp, u32, u32, vp, u32, vp, i32, vp]
    lib.oracle_topk_patterns.restype = ctypes.c_int64
    lib.oracle_topk_patterns.argtypes = [u32, vp, vp, vp, u32, u32, vp, vp, vp]
    lib.oracle_topk_patterns_definition.restype = ctypes.c_int64
    lib.oracle_topk_patterns_definition.argtypes = [u32, vp, vp, vp, u32, u32, vp, vp]
    lib.oracle_pattern_support.restype = ctypes.c_int64
    lib.oracle_pattern_support.argtypes = [u32, vp, vp, vp, u32, vp]
    lib.oracle_min_dfs_code.restype = ctypes.c_int64
    lib.oracle_min_dfs_code.argtypes = [u32, vp, u32, vp, vp]
    lib.oracle_vertex_order.argtypes = [u32, vp, vp, i32, vp]
    lib.oracle_core_numbers.argtypes = [u32, vp, vp, vp]
    lib.oracle_set_work_limit.argtypes = [u64]
    _lib = lib
    return lib


def _arr(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


CLIQUE_STATS = ("popped", "expanded", "children", "pruned_at_creation", "pruned_at_pop", "offered",
                "ids")
MATCH_STATS = ("popped", "expanded", "children", "pruned_at_creation", "pruned_at_pop", "offered",
               "automorphisms")


def topk_cliques(g, k: int, weighted: bool = False, bound: int = 0, priority: int = 0,
                 order: int = 1, xprune: bool = True) -> Tuple[List[Tuple[int, Tuple[int, ...]]], dict]:
    """Top-k maximal cliques of g.

    Returns ([(score, ids_ascending), ...] best first, stats).
    bound: 0 Carraghan-Pardalos, 1 greedy colouring.
    priority: 0 paper (|V|, |P|), 1 bound, 2 FIFO.  order: 0 id, 1 degeneracy.
    xprune: skip subgraphs none of whose expansions can be maximal.
    """
    lib = _load()
    rp, col = _arr(g.row_ptr, np.uint64), _arr(g.col, np.uint32)
    vw = _arr(g.vertex_weight, np.int32) if weighted else None
    if weighted and vw is None:
        raise ValueError("weighted cliques need vertex weights")
    cap = max(1024, 64 * k)
    while True:
        scores = np.zeros(k, np.int64)
        off = np.zeros(k + 1, np.uint64)
        ids = np.zeros(cap, np.uint32)
        stats = np.zeros(8, np.uint64)
        c = lib.oracle_topk_cliques(g.n, rp.ctypes.data, col.ctypes.data,
                                    vw.ctypes.data if vw is not None else None, k, int(weighted),
                                    bound, priority, order, int(xprune), scores.ctypes.data,
                                    off.ctypes.data,
                                    ids.ctypes.data, cap, stats.ctypes.data)
        if c == -2:
            raise ValueError("invalid arguments")
        if c == -3:
            return None, dict(zip(CLIQUE_STATS, (int(x) for x in stats[:7])))
        if c == -1:
            cap = int(stats[6]) + 16
            continue
        res = [(int(scores[i]), tuple(int(x) for x in ids[int(off[i]):int(off[i + 1])]))
               for i in range(c)]
        return res, dict(zip(CLIQUE_STATS, (int(x) for x in stats[:7])))


def clique_trace(g, k: int):
    """Paper-trace mode of the clique computation (Section 3.2 worked example).

    Returns (pops, R, stats) where pops is a list of
    (sorted vertex tuple, inserted_into_R, pruned_at_pop, n_children_inserted).
    """
    lib = _load()
    rp, col = _arr(g.row_ptr, np.uint64), _arr(g.col, np.uint32)
    pop_log = np.zeros(1 << 16, np.int32)
    r_log = np.zeros(1 << 12, np.int32)
    stats = np.zeros(8, np.uint64)
    npop = lib.oracle_clique_trace(g.n, rp.ctypes.data, col.ctypes.data, k, pop_log.ctypes.data,
                                   pop_log.size, r_log.ctypes.data, r_log.size, stats.ctypes.data)
    if npop < 0:
        raise ValueError("invalid arguments")
    pops = []
    i = 0
    for _ in range(npop):
        vs = []
        while pop_log[i] != -1:
            vs.append(int(pop_log[i]))
            i += 1
        pops.append((tuple(vs), int(pop_log[i + 1]), int(pop_log[i + 2]), int(pop_log[i + 3])))
        i += 4
    R = []
    cur = []
    for x in r_log:
        if x == -1:
            R.append(tuple(cur))
            cur = []
            if len(R) == int(stats[4]):
                break
        else:
            cur.append(int(x))
    st = dict(zip(("popped", "children", "pruned_at_creation", "pruned_at_pop", "r_size"),
                  (int(x) for x in stats[:5])))
    return pops, R[:st["r_size"]], st


def topk_match(g, labels, edges, k: int, n_labels: int = 16, priority: int = 0,
               score: str = "edge"):
    """Top-k labelled matches of the pattern (labels[q], edges [(a,b)]) in g.

    score: "edge" (sum of matched edge weights) or "degree" (sum of the
    degrees of the matched vertices, bounded with the multi-hop index).
    Returns ([(score, (mu(0), ..., mu(q-1))), ...] best first, stats).
    """
    lib = _load()
    q = len(labels)
    rp, col = _arr(g.row_ptr, np.uint64), _arr(g.col, np.uint32)
    lab = _arr(g.vertex_label, np.uint8)
    ew = _arr(g.edge_weight, np.int32) if g.edge_weight is not None else None
    pl = _arr(labels, np.uint8)
    pe = _arr(np.array(edges, dtype=np.uint32).reshape(-1), np.uint32)
    scores = np.zeros(k, np.int64)
    ids = np.zeros(k * q, np.uint32)
    stats = np.zeros(8, np.uint64)
    if score == "degree":
        c = lib.oracle_topk_match_degree(g.n, rp.ctypes.data, col.ctypes.data, lab.ctypes.data,
                                         n_labels, q, pl.ctypes.data, len(edges), pe.ctypes.data,
                                         k, priority, scores.ctypes.data, ids.ctypes.data,
                                         stats.ctypes.data)
    elif score == "edge":
        c = lib.oracle_topk_match(g.n, rp.ctypes.data, col.ctypes.data, lab.ctypes.data,
                                  ew.ctypes.data if ew is not None else None, n_labels, q,
                                  pl.ctypes.data, len(edges), pe.ctypes.data, k, priority,
                                  scores.ctypes.data, ids.ctypes.data, stats.ctypes.data)
    else:
        raise ValueError("score must be 'edge' or 'degree'")
    if c < 0:
        raise ValueError("invalid pattern or k")
    res = [(int(scores[i]), tuple(int(x) for x in ids[i * q:(i + 1) * q])) for i in range(c)]
    return res, dict(zip(MATCH_STATS, (int(x) for x in stats[:7])))


def hop_index(g, hops: int, n_labels: int = 16) -> np.ndarray:
    """The multi-hop max-degree index, int32 [hops, n, n_labels]: entry
    [h-1, v, l] = largest degree of a label-l vertex 1..h hops from v, 0 if
    none."""
    lib = _load()
    rp, col = _arr(g.row_ptr, np.uint64), _arr(g.col, np.uint32)
    lab = _arr(g.vertex_label, np.uint8)
    out = np.zeros((hops, g.n, n_labels), np.int32)
    lib.oracle_hop_index(g.n, rp.ctypes.data, col.ctypes.data, lab.ctypes.data, n_labels, hops,
                         out.ctypes.data)
    return out


def match_root_bounds(g, labels, edges, n_labels: int = 16, score: str = "edge"):
    """(first pattern vertex of the matching order, int64 bound per data
    vertex of the unit subgraph it hosts; -1 for non-roots and for roots
    with no completion)."""
    lib = _load()
    rp, col = _arr(g.row_ptr, np.uint64), _arr(g.col, np.uint32)
    lab = _arr(g.vertex_label, np.uint8)
    ew = _arr(g.edge_weight, np.int32) if g.edge_weight is not None else None
    pl = _arr(labels, np.uint8)
    pe = _arr(np.array(edges, dtype=np.uint32).reshape(-1), np.uint32)
    out = np.zeros(g.n, np.int64)
    first = lib.oracle_match_root_bounds(g.n, rp.ctypes.data, col.ctypes.data, lab.ctypes.data,
                                         ew.ctypes.data if ew is not None else None, n_labels,
                                         len(labels), pl.ctypes.data, len(edges), pe.ctypes.data,
                                         int(score == "degree"), out.ctypes.data)
    if first < 0:
        raise ValueError("invalid pattern")
    return int(first), out


PATTERN_STATS = ("popped", "expanded", "children", "pruned_at_creation", "pruned_at_pop",
                 "non_minimal", "groups")


def _codes(codes, count, M):
    return [tuple(tuple(int(x) for x in codes[(r * M + t) * 4:(r * M + t) * 4 + 4])
                  for t in range(M)) for r in range(count)]


def topk_patterns(g, n_edges: int, k: int):
    """Top-k frequent patterns with n_edges edges by Algorithm 2.

    Returns ([(support, code)], stats); code = ((i, j, L(i), L(j)), ...),
    the pattern's minimum DFS code.
    """
    lib = _load()
    rp, col = _arr(g.row_ptr, np.uint64), _arr(g.col, np.uint32)
    lab = _arr(g.vertex_label, np.uint8)
    sup = np.zeros(k, np.uint64)
    codes = np.zeros(k * n_edges * 4, np.uint32)
    stats = np.zeros(8, np.uint64)
    c = lib.oracle_topk_patterns(g.n, rp.ctypes.data, col.ctypes.data, lab.ctypes.data, n_edges,
                                 k, sup.ctypes.data, codes.ctypes.data, stats.ctypes.data)
    if c < 0:
        raise ValueError("bad arguments")
    res = [(int(sup[r]), code) for r, code in enumerate(_codes(codes, c, n_edges))]
    return res, dict(zip(PATTERN_STATS, (int(x) for x in stats[:7])))


def topk_patterns_definition(g, n_edges: int, k: int):
    """The same top-k from the definition (every connected set of n_edges
    data edges); graphs of at most 64 edges."""
    lib = _load()
    rp, col = _arr(g.row_ptr, np.uint64), _arr(g.col, np.uint32)
    lab = _arr(g.vertex_label, np.uint8)
    sup = np.zeros(k, np.uint64)
    codes = np.zeros(k * n_edges * 4, np.uint32)
    c = lib.oracle_topk_patterns_definition(g.n, rp.ctypes.data, col.ctypes.data, lab.ctypes.data,
                                            n_edges, k, sup.ctypes.data, codes.ctypes.data)
    if c < 0:
        raise ValueError("bad arguments or graph too large")
    return [(int(sup[r]), code) for r, code in enumerate(_codes(codes, c, n_edges))]


def pattern_support(g, code) -> int:
    """Minimum image-based support of the pattern given by a DFS code."""
    lib = _load()
    rp, col = _arr(g.row_ptr, np.uint64), _arr(g.col, np.uint32)
    lab = _arr(g.vertex_label, np.uint8)
    flat = _arr(np.array(code, dtype=np.uint32).reshape(-1), np.uint32)
    f = lib.oracle_pattern_support(g.n, rp.ctypes.data, col.ctypes.data, lab.ctypes.data,
                                   len(code), flat.ctypes.data)
    if f < 0:
        raise ValueError("bad code")
    return int(f)


def min_dfs_code(labels, edges):
    """Minimum DFS code of a small connected labelled graph."""
    lib = _load()
    pl = _arr(labels, np.uint8)
    pe = _arr(np.array(edges, dtype=np.uint32).reshape(-1), np.uint32)
    out = np.zeros(len(edges) * 4, np.uint32)
    r = lib.oracle_min_dfs_code(len(labels), pl.ctypes.data, len(edges), pe.ctypes.data,
                                out.ctypes.data)
    if r < 0:
        raise ValueError("bad or disconnected pattern")
    return _codes(out, 1, len(edges))[0]


def vertex_order(g, order: int = 1) -> np.ndarray:
    lib = _load()
    rp, col = _arr(g.row_ptr, np.uint64), _arr(g.col, np.uint32)
    pi = np.zeros(g.n, np.uint32)
    lib.oracle_vertex_order(g.n, rp.ctypes.data, col.ctypes.data, order, pi.ctypes.data)
    return pi


def set_work_limit(max_children: int) -> None:
    """Cap the children a clique search may create (0 = no cap).

    A capped search returns (None, stats); it is only for timing the oracle
    on a bounded sample of a large workload.
    """
    _load().oracle_set_work_limit(int(max_children))


def core_numbers(g) -> np.ndarray:
    lib = _load()
    rp, col = _arr(g.row_ptr, np.uint64), _arr(g.col, np.uint32)
    core = np.zeros(g.n, np.uint32)
    lib.oracle_core_numbers(g.n, rp.ctypes.data, col.ctypes.data, core.ctypes.data)
    return core


def induced_subgraph(g, keep: np.ndarray):
    """Subgraph induced by the vertices with keep[v] true.

    Vertices are renumbered in increasing original id, so sorted id lists
    stay sorted and lexicographic order is preserved.  Returns (subgraph,
    new->original id array).
    """
    import synth
    old = np.flatnonzero(keep).astype(np.int64)
    new_of = np.full(g.n, -1, np.int64)
    new_of[old] = np.arange(len(old))
    rp = g.row_ptr.astype(np.int64)
    deg = rp[1:] - rp[:-1]
    src = np.repeat(np.arange(g.n), deg)
    dst = g.col.astype(np.int64)
    m = keep[src] & keep[dst]
    s2, d2 = new_of[src[m]], new_of[dst[m]]
    order = np.lexsort((d2, s2))
    s2, d2 = s2[order], d2[order]
    row = np.zeros(len(old) + 1, np.uint64)
    np.add.at(row, s2 + 1, 1)
    row = np.cumsum(row).astype(np.uint64)
    sub = synth.Graph(len(old), row, d2.astype(np.uint32))
    if g.vertex_weight is not None:
        sub.vertex_weight = np.ascontiguousarray(g.vertex_weight[old], np.int32)
    return sub, old


def large_clique_kernel(g, min_size: int, max_vertices: int = 8192):
    """Exact reduction for the maximal cliques of g with >= min_size vertices.

    Returns (residual graph, residual -> original id array, common ids):
    the maximal cliques of g with s >= min_size vertices are exactly
    common + C for the maximal cliques C of the residual with
    s - len(common) vertices.  Steps, each exact for such cliques:
      1. keep the (min_size-1)-core (every member has min_size-1 neighbours
         inside the clique);
      2. repeatedly drop edges with fewer than min_size-2 common neighbours
         and then vertices with fewer than min_size-1 neighbours (every edge
         of the clique has min_size-2 common neighbours inside it, so
         nothing of the clique is ever dropped);
      3. take out the vertices adjacent to all others that are left: every
         maximal clique of what is left contains them.
    A vertex extending such a clique in g forms a larger one, which the
    same steps keep, so maximality is unchanged by the reduction.  Ids stay
    in increasing original order, so the ranking order is unchanged too
    (the common ids are shared by every result).
    """
    core = core_numbers(g)
    sub, old = induced_subgraph(g, core >= max(0, min_size - 1))
    n = sub.n
    if n > max_vertices:
        raise ValueError(f"core of {n} vertices is larger than {max_vertices}")
    A = np.zeros((n, n), np.float32)  # counts below 2^24 are exact in float32
    rp = sub.row_ptr.astype(np.int64)
    A[np.repeat(np.arange(n), np.diff(rp)), sub.col.astype(np.int64)] = 1.0
    alive = np.ones(n, bool)
    while True:
        support = A @ A  # common neighbours of every pair
        weak = (A > 0) & (support < min_size - 2)
        A[weak] = 0.0
        low = alive & (A.sum(axis=1) < min_size - 1)
        A[low, :] = 0.0
        A[:, low] = 0.0
        alive &= ~low
        if not weak.any() and not low.any():
            break
    idx = np.flatnonzero(alive)
    B = A[np.ix_(idx, idx)]
    universal = B.sum(axis=1) == len(idx) - 1
    common = old[idx[universal]]
    rest = idx[~universal]
    keep = np.zeros(n, bool)
    keep[rest] = True
    # the residual keeps only the edges that survived the peeling
    C = A[np.ix_(rest, rest)]
    import synth
    m = len(rest)
    src, dst = np.nonzero(C)
    row = np.zeros(m + 1, np.uint64)
    np.add.at(row, src + 1, 1)
    resid = synth.Graph(m, np.cumsum(row).astype(np.uint64), dst.astype(np.uint32))
    return resid, old[rest], [int(v) for v in common]
