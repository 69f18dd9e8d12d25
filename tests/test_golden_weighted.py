"""The stored oracle top-1000 of the batched weighted-clique shape (no GPU).

tests/golden/rmat15_weighted_top1000.txt holds the oracle's 1000 heaviest
maximal cliques of R-MAT scale 15 with vertex weights U{1..100}.  Here the
file is tied to the generator (workload hash), every entry is checked
against the graph (a clique, maximal, its score the sum of its weights,
strictly ordered), and the first three are recomputed with the oracle.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.golden_lists import rmat15_weighted_top1000, workload_sha256


@pytest.fixture(scope="module")
def workload():
    g = synth.rmat(15)
    synth.add_vertex_weights(g)
    return g


def test_stored_list_belongs_to_the_workload_and_is_valid(workload):
    g = workload
    sha, items = rmat15_weighted_top1000()
    assert workload_sha256(g) == sha
    assert len(items) == 1000
    keys = [(-s, ids) for s, ids in items]
    assert keys == sorted(keys) and len(set(keys)) == len(keys)
    rp, col, w = g.row_ptr.astype(np.int64), g.col, g.vertex_weight
    for s, ids in items:
        C = np.array(ids, dtype=np.int64)
        assert s == int(w[C].sum())
        # how many members each vertex is adjacent to: a member must see
        # all the others (a clique), an outside vertex not all (maximal)
        nb = np.concatenate([col[rp[u]:rp[u + 1]] for u in C]).astype(np.int64)
        seen = np.bincount(nb, minlength=g.n)
        assert (seen[C] == len(C) - 1).all(), "not a clique"
        seen[C] = 0
        assert (seen < len(C)).all(), "not maximal"


def test_first_entries_equal_a_fresh_oracle_run(workload):
    _, items = rmat15_weighted_top1000()
    got, _ = oracle.topk_cliques(workload, 3, weighted=True, bound=1)
    assert got == items[:3]
