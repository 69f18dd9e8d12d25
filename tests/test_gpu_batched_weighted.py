"""The batched vertex-weighted clique workload's shape, checked in full:
256 queries with k drawn log-uniform in 1..1000, all in one batch (every
expansion launch serves all of them), on R-MAT scale 15 with vertex weights
U{1..100}.  Results are ranked under a total order, so every query's top-k
is the first k entries of the graph's top-1000, which the oracle wrote to
tests/golden/rmat15_weighted_top1000.txt (script beside it).  Every one of
the 256 answers must equal its prefix of that list.
"""
import pytest

import synth
from tests.golden_lists import rmat15_weighted_top1000, workload_sha256

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nuri():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1807_08888_amd import nuri as N
    N.lib()
    return N


def test_256_weighted_queries_in_one_batch_equal_stored_prefixes(nuri):
    sha, top = rmat15_weighted_top1000()
    g = synth.rmat(15)
    synth.add_vertex_weights(g)
    assert workload_sha256(g) == sha, "the generator made a different workload"
    ks = [synth.log_uniform_k(i, 1000) for i in range(256)]
    qs = [{"kind": "clique", "k": k, "weight_fn": 1} for k in ks]
    print(f"[case] R-MAT 15, 256 weighted queries, k in {min(ks)}..{max(ks)}", flush=True)
    G = nuri.Graph.from_synth(g)
    try:
        outs = nuri.topk_batch(G, qs)
    finally:
        G.close()
    bad = [i for i, k in enumerate(ks) if outs[i].items != top[:k]]
    assert not bad, f"queries whose top-k is not the stored prefix: {bad[:10]}"
