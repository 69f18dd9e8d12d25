"""MI355X-native top-k subgraph discovery (prioritized, pruned expansion of
partial subgraphs; arXiv 1807.08888).

The engine is the HIP library libnuri.so behind include/nuri.h; `nuri` is
its thin ctypes binding.
"""
from . import nuri  # noqa: F401
from .nuri import (Graph, NuriError, Result, Server, SCORE_SIZE, SCORE_VERTEX_WEIGHT,  # noqa: F401
                   topk_batch, topk_cliques, topk_match)
