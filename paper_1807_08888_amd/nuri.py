"""Thin ctypes binding of libnuri.so (include/nuri.h).

Argument marshalling only: every step of a query runs in the HIP library.
The binding raises if the library is missing; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnuri.so")

NURI_OK = 0
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EBUDGET", -4: "EDEVICE", -5: "ETIMEOUT"}
SCORE_SIZE = 0
SCORE_VERTEX_WEIGHT = 1
PRIORITY_DEPTH, PRIORITY_BOUND, PRIORITY_PAPER, PRIORITY_NONE = 0, 1, 2, 3
MATCH_EDGE_WEIGHT, MATCH_DEGREE = 0, 1


class NuriError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class _CSR(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("nnz", ctypes.c_uint64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("vertex_weight", ctypes.c_void_p), ("vertex_label", ctypes.c_void_p),
                ("edge_weight", ctypes.c_void_p)]


class _GraphInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("nnz", ctypes.c_uint64), ("degeneracy", ctypes.c_uint32),
                ("bitmap_bytes", ctypes.c_uint64), ("device_bytes", ctypes.c_uint64),
                ("preprocess_ns", ctypes.c_uint64), ("core_density", ctypes.c_double)]


class _Pattern(ctypes.Structure):
    _fields_ = [("q", ctypes.c_uint32), ("n_edges", ctypes.c_uint32),
                ("label", ctypes.c_void_p), ("edges", ctypes.c_void_p),
                ("score", ctypes.c_uint32)]


class _Opts(ctypes.Structure):
    _fields_ = [("frontier_budget_bytes", ctypes.c_uint64), ("batch_B", ctypes.c_uint32),
                ("root_batch", ctypes.c_uint32), ("bound", ctypes.c_uint32),
                ("deadline_ns", ctypes.c_uint64), ("profile", ctypes.c_uint32),
                ("hip_stream", ctypes.c_void_p), ("priority", ctypes.c_uint32),
                ("chain_links", ctypes.c_uint32)]


class _Query(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("k", ctypes.c_uint32), ("wf", ctypes.c_int),
                ("p", ctypes.POINTER(_Pattern))]


class _View(ctypes.Structure):
    _fields_ = [("count", ctypes.c_uint32), ("score", ctypes.POINTER(ctypes.c_int64)),
                ("offset", ctypes.POINTER(ctypes.c_uint64)),
                ("ids", ctypes.POINTER(ctypes.c_uint32))]


STAT_FIELDS = ("steps", "popped", "expanded", "children", "pruned_at_pop", "pruned_at_creation",
               "leaves", "offered", "frontier_peak_bytes", "logical_bytes", "expand_launches",
               "expand_ns", "wall_ns", "ties_at_k", "restarts", "onchip_bytes",
               "spilled_bytes", "index_ns")


class _Stats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in STAT_FIELDS]


# every function include/nuri.h declares, with (restype, argtypes)
_VP = ctypes.c_void_p
SIGNATURES = {
    "nuri_load_graph": (ctypes.c_int, [ctypes.POINTER(_CSR), _VP, ctypes.POINTER(_VP)]),
    "nuri_free_graph": (None, [_VP]),
    "nuri_graph_get_info": (ctypes.c_int, [_VP, ctypes.POINTER(_GraphInfo)]),
    "nuri_topk_patterns": (ctypes.c_int, [_VP, ctypes.c_uint32, ctypes.c_uint32, _VP,
                                          ctypes.POINTER(_VP)]),
    "nuri_graph_hop_index": (ctypes.c_int, [_VP, ctypes.c_uint32, _VP,
                                            ctypes.POINTER(ctypes.c_uint64)]),
    "nuri_topk_cliques": (ctypes.c_int, [_VP, ctypes.c_uint32, ctypes.c_int,
                                         ctypes.POINTER(_Opts), ctypes.POINTER(_VP)]),
    "nuri_topk_match": (ctypes.c_int, [_VP, ctypes.POINTER(_Pattern), ctypes.c_uint32,
                                       ctypes.POINTER(_Opts), ctypes.POINTER(_VP)]),
    "nuri_topk_batch": (ctypes.c_int, [_VP, ctypes.POINTER(_Query), ctypes.c_uint32,
                                       ctypes.POINTER(_Opts), ctypes.POINTER(_VP)]),
    "nuri_autotune": (ctypes.c_int, [_VP, ctypes.POINTER(_Query), ctypes.c_uint32,
                                     ctypes.POINTER(_Opts), ctypes.c_uint32,
                                     ctypes.POINTER(_Opts)]),
    "nuri_result_view_get": (ctypes.c_int, [_VP, ctypes.POINTER(_View)]),
    "nuri_result_stats": (ctypes.c_int, [_VP, ctypes.POINTER(_Stats)]),
    "nuri_free_result": (None, [_VP]),
    "nuri_server_create": (ctypes.c_int, [_VP, ctypes.c_uint64, ctypes.c_uint32,
                                          ctypes.POINTER(_VP)]),
    "nuri_server_submit": (ctypes.c_int, [_VP, ctypes.POINTER(_Query),
                                          ctypes.POINTER(ctypes.c_uint64)]),
    "nuri_server_poll": (ctypes.c_int, [_VP, ctypes.c_uint64, ctypes.POINTER(_VP)]),
    "nuri_server_destroy": (None, [_VP]),
    "nuri_topk_cliques_noalloc": (ctypes.c_int, [_VP, ctypes.c_uint32, ctypes.c_int,
                                                 ctypes.POINTER(_Opts), _VP, _VP, _VP,
                                                 ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32),
                                                 ctypes.POINTER(_Stats)]),
    "nuri_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libnuri.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1807_08888_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(rc: int):
    if rc < 0:
        raise NuriError(rc, lib().nuri_last_error().decode(errors="replace"))
    return rc


def _stream_handle(stream) -> Optional[int]:
    """hipStream_t from a torch.cuda.Stream (or an int handle); None = default."""
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def _opts(frontier_budget_bytes=0, batch_B=0, root_batch=0, bound=0, deadline_ns=0,
          profile=False, stream=None, priority=PRIORITY_DEPTH, chain_links=0) -> _Opts:
    return _Opts(frontier_budget_bytes, batch_B, root_batch, bound, deadline_ns,
                 int(bool(profile)), _stream_handle(stream), priority, chain_links)


class Result:
    """A top-k result: list of (score, ids) plus the work counters."""

    def __init__(self, handle):
        self._h = handle
        v = _View()
        _check(lib().nuri_result_view_get(handle, ctypes.byref(v)))
        n = v.count
        scores = [int(v.score[i]) for i in range(n)]
        off = [int(v.offset[i]) for i in range(n + 1)]
        total = off[-1] if n else 0
        ids = np.ctypeslib.as_array(v.ids, shape=(total,)).copy() if total else np.zeros(0, np.uint32)
        self.items: List[Tuple[int, Tuple[int, ...]]] = [
            (scores[i], tuple(int(x) for x in ids[off[i]:off[i + 1]])) for i in range(n)]
        st = _Stats()
        _check(lib().nuri_result_stats(handle, ctypes.byref(st)))
        self.stats: Dict[str, int] = {f: int(getattr(st, f)) for f in STAT_FIELDS}
        lib().nuri_free_result(handle)
        self._h = None

    def __iter__(self):
        return iter(self.items)

    def __len__(self):
        return len(self.items)


class Graph:
    """A graph resident on the GPU (nuri_load_graph)."""

    def __init__(self, row_ptr, col_idx, vertex_weight=None, vertex_label=None, edge_weight=None,
                 stream=None):
        self._keep = [np.ascontiguousarray(row_ptr, np.uint64),
                      np.ascontiguousarray(col_idx, np.uint32)]
        rp, col = self._keep
        n = len(rp) - 1
        vw = None if vertex_weight is None else np.ascontiguousarray(vertex_weight, np.int32)
        lb = None if vertex_label is None else np.ascontiguousarray(vertex_label, np.uint8)
        ew = None if edge_weight is None else np.ascontiguousarray(edge_weight, np.int32)
        csr = _CSR(n, int(rp[-1]) if n >= 0 else 0, rp.ctypes.data, col.ctypes.data,
                   vw.ctypes.data if vw is not None else None,
                   lb.ctypes.data if lb is not None else None,
                   ew.ctypes.data if ew is not None else None)
        h = _VP()
        _check(lib().nuri_load_graph(ctypes.byref(csr), _stream_handle(stream), ctypes.byref(h)))
        self._h = h
        self._keep = None

    @classmethod
    def from_synth(cls, g, stream=None) -> "Graph":
        return cls(g.row_ptr, g.col, g.vertex_weight, g.vertex_label, g.edge_weight, stream=stream)

    def info(self) -> Dict[str, int]:
        i = _GraphInfo()
        _check(lib().nuri_graph_get_info(self._h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in _GraphInfo._fields_}

    def hop_index(self, hops: int, copy: bool = True):
        """(int32 [hops, n, 16] multi-hop index or None when copy is False,
        build ns of this call) (nuri_graph_hop_index)."""
        n = int(self.info()["n"])
        out = np.zeros((hops, n, 16), np.int32) if copy else None
        ns = ctypes.c_uint64(0)
        _check(lib().nuri_graph_hop_index(self._h, hops, out.ctypes.data if copy else None,
                                          ctypes.byref(ns)))
        return out, int(ns.value)

    def close(self):
        if getattr(self, "_h", None):
            lib().nuri_free_graph(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def topk_cliques(graph: Graph, k: int, weight_fn: int = SCORE_SIZE, **opts) -> Result:
    """Top-k maximal cliques (nuri_topk_cliques)."""
    out = _VP()
    o = _opts(**opts)
    _check(lib().nuri_topk_cliques(graph._h, k, weight_fn, ctypes.byref(o), ctypes.byref(out)))
    return Result(out)


def topk_cliques_noalloc(graph: Graph, k: int, weight_fn: int = SCORE_SIZE, **opts):
    """Top-k maximal cliques through the allocation-free entry point
    (nuri_topk_cliques_noalloc); returns (items, stats) like Result."""
    stride = int(graph.info()["degeneracy"]) + 1
    score = np.zeros(max(k, 1), np.int64)
    lens = np.zeros(max(k, 1), np.uint32)
    ids = np.zeros(max(k, 1) * stride, np.uint32)
    count = ctypes.c_uint32(0)
    st = _Stats()
    o = _opts(**opts)
    _check(lib().nuri_topk_cliques_noalloc(graph._h, k, weight_fn, ctypes.byref(o),
                                           score.ctypes.data, lens.ctypes.data, ids.ctypes.data,
                                           stride, ctypes.byref(count), ctypes.byref(st)))
    items = [(int(score[i]), tuple(int(x) for x in ids[i * stride:i * stride + int(lens[i])]))
             for i in range(count.value)]
    return items, {f: int(getattr(st, f)) for f in STAT_FIELDS}


def _match_score(score) -> int:
    if score in ("edge", MATCH_EDGE_WEIGHT):
        return MATCH_EDGE_WEIGHT
    if score in ("degree", MATCH_DEGREE):
        return MATCH_DEGREE
    raise ValueError("match score must be 'edge' or 'degree'")


def _pattern(labels: Sequence[int], edges: Sequence[Tuple[int, int]], score="edge"):
    lb = np.ascontiguousarray(labels, np.uint8)
    ed = np.ascontiguousarray(np.array(edges, dtype=np.uint32).reshape(-1), np.uint32)
    p = _Pattern(len(lb), len(edges), lb.ctypes.data, ed.ctypes.data if len(edges) else None,
                 _match_score(score))
    return p, (lb, ed)


def topk_match(graph: Graph, labels: Sequence[int], edges: Sequence[Tuple[int, int]], k: int,
               score="edge", **opts) -> Result:
    """Top-k labelled matches (nuri_topk_match).  score: "edge" (sum of the
    matched edge weights) or "degree" (sum of the matched vertices'
    degrees, bounded with the multi-hop index)."""
    p, keep = _pattern(labels, edges, score)
    out = _VP()
    o = _opts(**opts)
    _check(lib().nuri_topk_match(graph._h, ctypes.byref(p), k, ctypes.byref(o), ctypes.byref(out)))
    return Result(out)


def topk_patterns(graph: Graph, n_edges: int, k: int, **opts):
    """Top-k frequent patterns with n_edges edges (nuri_topk_patterns).

    Returns ([(support, code)], stats); code = ((i, j, L(i), L(j)), ...),
    the pattern's minimum DFS code."""
    out = _VP()
    o = _opts(**opts)
    _check(lib().nuri_topk_patterns(graph._h, n_edges, k, ctypes.byref(o), ctypes.byref(out)))
    r = Result(out)
    items = [(int(s), tuple(tuple(int(x) for x in ids[4 * t:4 * t + 4])
                           for t in range(len(ids) // 4))) for s, ids in r.items]
    return items, r.stats


def _queries(queries):
    """queries: dicts {"kind": "clique", "k", "weight_fn"} or
    {"kind": "match", "k", "labels", "edges", optional "score"}."""
    qs = (_Query * len(queries))()
    keep = []
    for i, q in enumerate(queries):
        if q["kind"] == "clique":
            qs[i] = _Query(0, q["k"], q.get("weight_fn", SCORE_SIZE), None)
        else:
            p, arrs = _pattern(q["labels"], q["edges"], q.get("score", "edge"))
            keep.append((p, arrs))
            qs[i] = _Query(1, q["k"], 0, ctypes.pointer(p))
    return qs, keep


def topk_batch(graph: Graph, queries, **opts) -> List[Result]:
    """Many queries sharing every launch (nuri_topk_batch)."""
    qs, keep = _queries(queries)
    outs = (_VP * len(queries))()
    o = _opts(**opts)
    _check(lib().nuri_topk_batch(graph._h, qs, len(queries), ctypes.byref(o), outs))
    return [Result(outs[i]) for i in range(len(queries))]


def autotune(graph: Graph, queries, rounds: int = 1, **opts) -> Dict[str, int]:
    """Fastest (batch_B, root_batch) for these queries (nuri_autotune)."""
    qs, keep = _queries(queries)
    o = _opts(**opts)
    best = _Opts()
    _check(lib().nuri_autotune(graph._h, qs, len(queries), ctypes.byref(o), rounds,
                               ctypes.byref(best)))
    return {"batch_B": int(best.batch_B), "root_batch": int(best.root_batch)}


class Server:
    """Continuous-batching server (nuri_server_*)."""

    def __init__(self, graph: Graph, frontier_budget_bytes: int = 0, max_slots: int = 64):
        h = _VP()
        _check(lib().nuri_server_create(graph._h, frontier_budget_bytes, max_slots, ctypes.byref(h)))
        self._h = h
        self._graph = graph

    def submit(self, query) -> int:
        qs, keep = _queries([query])
        t = ctypes.c_uint64()
        _check(lib().nuri_server_submit(self._h, qs, ctypes.byref(t)))
        return int(t.value)

    def poll(self, ticket: int) -> Optional[Result]:
        out = _VP()
        rc = _check(lib().nuri_server_poll(self._h, ticket, ctypes.byref(out)))
        return Result(out) if rc == 1 else None

    def close(self):
        if getattr(self, "_h", None):
            lib().nuri_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
