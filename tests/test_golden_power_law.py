"""The stored top-100 of the power-law workload (no GPU).

tests/golden/power_law_top100.txt is written by
tests/golden/make_power_law_top100.py from the CPU oracle on an exact
reduction of the graph.  Here it is tied to the generator (same graph
hash) and checked against the graph itself: 100 results, each a clique
that no vertex extends, of the stated size, strictly ordered by size
descending, then ids ascending.
"""
import numpy as np
import pytest

import synth
from tests.golden_lists import graph_sha256, power_law_top100


@pytest.fixture(scope="module")
def stored():
    g = synth.chung_lu()
    sha, items = power_law_top100()
    return g, sha, items


def test_stored_list_belongs_to_the_generated_graph(stored):
    g, sha, items = stored
    assert graph_sha256(g) == sha
    assert len(items) == 100


def test_stored_results_are_maximal_cliques_in_order(stored):
    g, _, items = stored
    rp = g.row_ptr.astype(np.int64)
    keys = [(-s, ids) for s, ids in items]
    assert keys == sorted(keys) and len(set(keys)) == len(keys)
    for size, ids in items:
        members = np.array(ids, np.int64)
        assert len(members) == size
        # every member is adjacent to all other members, and no outside
        # vertex is adjacent to all of them
        count = np.zeros(g.n, np.int64)
        for v in members:
            nb = g.col[rp[v]:rp[v + 1]].astype(np.int64)
            count[nb] += 1
        assert np.all(count[members] == size - 1)
        count[members] = 0
        assert count.max() < size
