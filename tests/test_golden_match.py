"""The stored oracle results of the full-size matching workload (no GPU).

tests/golden/rmat22_match_top50.txt holds, for each of the 128 patterns of
the R-MAT scale-22 labelled workload, the length, best score and SHA-256 of
the oracle's top-50 list.  Here the file is tied to the generator (same
workload hash) and two of its fastest patterns are recomputed with the
oracle and must hash the same.
"""
import pytest

import oracle
import synth
from tests.golden_lists import result_sha256, rmat22_match_top50, workload_sha256


@pytest.fixture(scope="module")
def workload():
    g = synth.rmat(22)
    synth.add_vertex_weights(g)
    synth.add_edge_weights(g)
    synth.add_zipf_labels(g)
    return g


def test_stored_file_is_complete_and_belongs_to_the_workload(workload):
    sha, rows = rmat22_match_top50()
    assert workload_sha256(workload) == sha
    assert set(rows) <= set(range(128)) and len(rows) >= 100
    assert all(0 <= n <= 50 and len(h) == 64 for n, _, h in rows.values())


@pytest.mark.parametrize("i", [32, 38])
def test_stored_hash_equals_a_fresh_oracle_run(workload, i):
    _, rows = rmat22_match_top50()
    p = synth.random_pattern(i)
    res, _ = oracle.topk_match(workload, p.labels, p.edges, 50)
    assert (len(res), res[0][0] if res else 0, result_sha256(res)) == rows[i]
