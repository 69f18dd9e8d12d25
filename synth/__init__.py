"""Seeded synthetic inputs shared by the CPU oracle tests and the GPU engine.

This module draws graphs, weights, labels, query patterns and query
parameters.  It holds none of the subgraph-discovery arithmetic: it never
looks for cliques or matches, never scores and never bounds.

All randomness is splitmix64 used as a counter-based generator (value i of a
stream with seed s is mix64(s + (i+1) * 0x9E3779B97F4A7C15)); the C side
(gen.c) and the small Python helpers below implement the same definition.

Workloads (sizes as the engine's benchmarks use them):

* ``er_planted``   G(n, p) plus vertex-disjoint planted cliques.
* ``chung_lu``     power-law expected-degree graph (Miller-Hagberg sampling)
                   plus planted cliques.
* ``rmat``         R-MAT graph, symmetrised, self loops and duplicates dropped.
* weights / labels / patterns / k draws, each from its own stream.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess
from typing import List, Optional

import numpy as np

MASTER_SEED = 1807088880
_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsynth.so")
_MASK = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15

# stream ids (one per kind of draw)
S_VERTEX_WEIGHT = 101
S_EDGE_WEIGHT = 102
S_LABEL = 103
S_PATTERN = 104
S_K = 105
S_ARRIVAL = 106


def build() -> str:
    """Compile gen.c into libsynth.so (plain gcc, OpenMP)."""
    src = os.path.join(_HERE, "gen.c")
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
    os.replace(tmp, _SO)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    lib = ctypes.CDLL(_SO)
    u64, u32, i32, dbl = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32, ctypes.c_double
    P = ctypes.POINTER
    lib.synth_stream_seed.restype = u64
    lib.synth_stream_seed.argtypes = [u64, u64]
    lib.synth_draw.restype = u64
    lib.synth_draw.argtypes = [u64, u64]
    lib.synth_free.argtypes = [ctypes.c_void_p]
    lib.synth_er_planted.restype = ctypes.c_int
    lib.synth_er_planted.argtypes = [u32, dbl, u32, u32, u32, u64, P(P(u64)), P(P(u32)), P(u64),
                                     P(P(u32)), P(P(u64))]
    lib.synth_chung_lu.restype = ctypes.c_int
    lib.synth_chung_lu.argtypes = [u32, dbl, dbl, dbl, u32, u32, u32, u64, P(P(u64)), P(P(u32)),
                                   P(u64), P(dbl)]
    lib.synth_rmat.restype = ctypes.c_int
    lib.synth_rmat.argtypes = [u32, u32, dbl, dbl, dbl, u64, P(P(u64)), P(P(u32)), P(u64)]
    lib.synth_vertex_weights.argtypes = [u32, i32, i32, u64, ctypes.c_void_p]
    lib.synth_edge_weights.argtypes = [u32, ctypes.c_void_p, ctypes.c_void_p, i32, i32, u64,
                                       ctypes.c_void_p]
    lib.synth_zipf_labels.argtypes = [u32, u32, dbl, u64, ctypes.c_void_p]
    lib.synth_permutation.restype = P(u32)
    lib.synth_permutation.argtypes = [u32, u64]
    _lib = lib
    return lib


def _take(ptr, count, dtype):
    """Copy a malloc'ed C array into numpy and free it."""
    lib = _load()
    if count == 0:
        lib.synth_free(ctypes.cast(ptr, ctypes.c_void_p))
        return np.zeros(0, dtype=dtype)
    buf = np.ctypeslib.as_array(ptr, shape=(count,)).copy().astype(dtype, copy=False)
    lib.synth_free(ctypes.cast(ptr, ctypes.c_void_p))
    return buf


@dataclasses.dataclass
class Graph:
    """Undirected simple graph in CSR form (rows strictly increasing, symmetric)."""
    n: int
    row_ptr: np.ndarray            # uint64 [n+1]
    col: np.ndarray                # uint32 [nnz]
    vertex_weight: Optional[np.ndarray] = None   # int32 [n]
    vertex_label: Optional[np.ndarray] = None    # uint8 [n]
    edge_weight: Optional[np.ndarray] = None     # int32 [nnz], aligned with col
    planted: Optional[List[np.ndarray]] = None   # sorted member lists of planted cliques
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def degree(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)


# ------------------------------------------------------------------
# counter-based draws in Python (same definition as gen.c)
# ------------------------------------------------------------------

def mix64(z: int) -> int:
    z &= _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def stream_seed(master: int, stream_id: int) -> int:
    return mix64((master ^ stream_id) & _MASK)


def draw(s: int, i: int) -> int:
    return mix64((s + (i + 1) * _GAMMA) & _MASK)


def unif(s: int, i: int) -> float:
    return (draw(s, i) >> 11) * (1.0 / 9007199254740992.0)


def below(s: int, i: int, m: int) -> int:
    return (draw(s, i) * m) >> 64


# ------------------------------------------------------------------
# graphs
# ------------------------------------------------------------------

def er_planted(n: int = 2000, avg_degree: float = 20.0, n_cliques: int = 10, lo: int = 8,
               hi: int = 15, master: int = MASTER_SEED) -> Graph:
    """G(n, p = avg_degree/(n-1)) plus n_cliques disjoint planted cliques of sizes U{lo..hi}."""
    lib = _load()
    rp, col = ctypes.POINTER(ctypes.c_uint64)(), ctypes.POINTER(ctypes.c_uint32)()
    nnz = ctypes.c_uint64()
    pl, plo = ctypes.POINTER(ctypes.c_uint32)(), ctypes.POINTER(ctypes.c_uint64)()
    p = avg_degree / (n - 1) if n > 1 else 0.0
    rc = lib.synth_er_planted(n, p, n_cliques, lo, hi, master, ctypes.byref(rp), ctypes.byref(col),
                              ctypes.byref(nnz), ctypes.byref(pl), ctypes.byref(plo))
    if rc != 0:
        raise ValueError(f"synth_er_planted failed ({rc})")
    row_ptr = _take(rp, n + 1, np.uint64)
    colv = _take(col, nnz.value, np.uint32)
    off = _take(plo, n_cliques + 1, np.uint64)
    members = _take(pl, int(off[-1]), np.uint32) if off[-1] > 0 else np.zeros(0, np.uint32)
    planted = [members[int(off[i]):int(off[i + 1])].copy() for i in range(n_cliques)]
    return Graph(n, row_ptr, colv, planted=planted, name=f"er{n}_d{avg_degree:g}_planted{n_cliques}")


def chung_lu(n: int = 1_000_000, beta: float = 2.1, m_target: float = 2e7, cap: float = 20000.0,
             n_cliques: int = 200, lo: int = 20, hi: int = 40, master: int = MASTER_SEED) -> Graph:
    """Chung-Lu expected-degree graph with exponent beta and expected-degree cap, plus planted cliques."""
    lib = _load()
    rp, col = ctypes.POINTER(ctypes.c_uint64)(), ctypes.POINTER(ctypes.c_uint32)()
    nnz = ctypes.c_uint64()
    c = ctypes.c_double()
    rc = lib.synth_chung_lu(n, beta, m_target, cap, n_cliques, lo, hi, master, ctypes.byref(rp),
                            ctypes.byref(col), ctypes.byref(nnz), ctypes.byref(c))
    if rc != 0:
        raise ValueError(f"synth_chung_lu failed ({rc})")
    return Graph(n, _take(rp, n + 1, np.uint64), _take(col, nnz.value, np.uint32),
                 name=f"chunglu{n}_b{beta:g}_m{m_target:g}_cap{cap:g}_planted{n_cliques}")


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         master: int = MASTER_SEED) -> Graph:
    """R-MAT graph with 2^scale vertices and edge_factor * 2^scale generated tuples."""
    lib = _load()
    rp, col = ctypes.POINTER(ctypes.c_uint64)(), ctypes.POINTER(ctypes.c_uint32)()
    nnz = ctypes.c_uint64()
    rc = lib.synth_rmat(scale, edge_factor, a, b, c, master, ctypes.byref(rp), ctypes.byref(col),
                        ctypes.byref(nnz))
    if rc != 0:
        raise ValueError(f"synth_rmat failed ({rc})")
    n = 1 << scale
    return Graph(n, _take(rp, n + 1, np.uint64), _take(col, nnz.value, np.uint32),
                 name=f"rmat{scale}_ef{edge_factor}")


def from_edges(n: int, edges, name: str = "") -> Graph:
    """CSR from an undirected edge list (pairs), dropping duplicates; rejects self loops."""
    adj = [set() for _ in range(n)]
    for u, v in edges:
        u, v = int(u), int(v)
        if u == v:
            raise ValueError("self loop")
        adj[u].add(v)
        adj[v].add(u)
    row_ptr = np.zeros(n + 1, np.uint64)
    cols = []
    for u in range(n):
        row = sorted(adj[u])
        cols.extend(row)
        row_ptr[u + 1] = row_ptr[u] + len(row)
    return Graph(n, row_ptr, np.array(cols, dtype=np.uint32), name=name)


def gnp(n: int, p: float, seed: int) -> Graph:
    """Small G(n, p) drawn in Python (test graphs)."""
    s = stream_seed(seed, 1)
    edges = []
    idx = 0
    for i in range(n):
        for j in range(i + 1, n):
            if unif(s, idx) < p:
                edges.append((i, j))
            idx += 1
    return from_edges(n, edges, name=f"gnp{n}_{p:g}_{seed}")


# ------------------------------------------------------------------
# weights and labels
# ------------------------------------------------------------------

def add_vertex_weights(g: Graph, lo: int = 1, hi: int = 100, master: int = MASTER_SEED) -> Graph:
    out = np.empty(g.n, np.int32)
    _load().synth_vertex_weights(g.n, lo, hi, stream_seed(master, S_VERTEX_WEIGHT),
                                 out.ctypes.data)
    g.vertex_weight = out
    return g


def add_edge_weights(g: Graph, lo: int = 1, hi: int = 1000, master: int = MASTER_SEED) -> Graph:
    out = np.empty(g.nnz, np.int32)
    rp = np.ascontiguousarray(g.row_ptr, np.uint64)
    col = np.ascontiguousarray(g.col, np.uint32)
    _load().synth_edge_weights(g.n, rp.ctypes.data, col.ctypes.data, lo, hi,
                               stream_seed(master, S_EDGE_WEIGHT), out.ctypes.data)
    g.edge_weight = out
    return g


def add_zipf_labels(g: Graph, n_labels: int = 16, s: float = 1.2, master: int = MASTER_SEED) -> Graph:
    out = np.empty(g.n, np.uint8)
    _load().synth_zipf_labels(g.n, n_labels, s, stream_seed(master, S_LABEL), out.ctypes.data)
    g.vertex_label = out
    return g


def zipf_pmf(n_labels: int = 16, s: float = 1.2) -> np.ndarray:
    w = np.array([(l + 1.0) ** (-s) for l in range(n_labels)])
    return w / w.sum()


# ------------------------------------------------------------------
# query patterns and query parameters
# ------------------------------------------------------------------

@dataclasses.dataclass
class Pattern:
    q: int
    labels: List[int]
    edges: List[tuple]     # (a, b) with a < b


def random_pattern(index: int, q_lo: int = 3, q_hi: int = 7, n_labels: int = 16, s: float = 1.2,
                   master: int = MASTER_SEED) -> Pattern:
    """Connected pattern number `index`: a random attachment tree plus random extra edges.

    q ~ U{q_lo..q_hi}; vertex i >= 1 attaches to U{0..i-1}; then
    e_x ~ U{0 .. min(q-1, C(q,2)-(q-1))} distinct non-edges are added,
    chosen uniformly; labels are iid truncated Zipf(s).
    """
    st = mix64(stream_seed(master, S_PATTERN) ^ index)
    c = 0

    def nxt_below(m):
        nonlocal c
        v = below(st, c, m)
        c += 1
        return v

    def nxt_unif():
        nonlocal c
        v = unif(st, c)
        c += 1
        return v

    q = q_lo + nxt_below(q_hi - q_lo + 1)
    edges = set()
    for i in range(1, q):
        j = nxt_below(i)
        edges.add((j, i))
    non_edges = [(a, b) for a in range(q) for b in range(a + 1, q) if (a, b) not in edges]
    max_extra = min(q - 1, q * (q - 1) // 2 - (q - 1))
    ex = nxt_below(max_extra + 1)
    for t in range(ex):
        r = t + nxt_below(len(non_edges) - t)
        non_edges[t], non_edges[r] = non_edges[r], non_edges[t]
        edges.add(non_edges[t])
    pmf = zipf_pmf(n_labels, s)
    cdf = np.cumsum(pmf)
    cdf[-1] = 1.0
    labels = []
    for _ in range(q):
        r = nxt_unif()
        labels.append(int(np.searchsorted(cdf, r, side="right")))
    return Pattern(q, labels, sorted(edges))


def log_uniform_k(index: int, k_max: int = 1000, master: int = MASTER_SEED) -> int:
    """k = clamp(floor(exp(u * ln(k_max+1))), 1, k_max) with u ~ U[0,1) draw number `index`."""
    u = unif(stream_seed(master, S_K), index)
    return max(1, min(k_max, int(math.floor(math.exp(u * math.log(k_max + 1))))))
