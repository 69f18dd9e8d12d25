"""GPU parity for top-k frequent pattern mining (Sections 2.1, 3.3, 4.2):
HIP engine vs CPU oracle, bit-exact on (support, minimum DFS code) lists
under (support descending, code ascending)."""
import numpy as np
import pytest

import oracle
import synth
from tests.test_oracle_patterns import _example_graph, _fixture, _code

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nuri():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1807_08888_amd import nuri as N
    N.lib()
    return N


def _case(msg):
    print(f"[case] {msg}", flush=True)


def _labelled(n, p, seed, n_labels):
    g = synth.gnp(n, p, seed)
    synth.add_zipf_labels(g, n_labels=n_labels, s=0.5, master=seed)
    return g


def test_worked_example_on_the_gpu(nuri):
    fx = _fixture()
    g = _example_graph(fx)
    _case("pattern mining worked example")
    G = nuri.Graph.from_synth(g)
    try:
        res, st = nuri.topk_patterns(G, 1, 10)
        assert res == [(3, ((0, 1, 1, 1),)), (2, ((0, 1, 0, 1),))]
        assert st["children"] == int(fx["one_edge_subgraphs"][0][0])
        want = fx["top1_two_edges"][0]
        res, st = nuri.topk_patterns(G, 2, 1)
        assert res == [(int(want[0]), _code(want[1:]))]
        # only p2's group is expanded; p1's is dominated when taken
        assert st["expanded"] == 1 and st["pruned_at_pop"] == 1
        res, _ = nuri.topk_patterns(G, 2, 5)
        assert res == [(3, _code(["0-1-1-1", "1-2-1-1"])), (2, _code(["0-1-0-1", "1-2-1-1"]))]
    finally:
        G.close()


@pytest.mark.parametrize("M", [1, 2, 3, 4])
@pytest.mark.parametrize("seed", range(4))
def test_small_graphs_vs_definition(nuri, M, seed):
    n_labels = 1 + seed % 3
    g = _labelled(11, 0.35, 60 + 7 * seed + M, n_labels)
    if g.m > 64:
        pytest.skip("too many edges to enumerate")
    want = oracle.topk_patterns_definition(g, M, 10 ** 6)
    _case(f"patterns M={M} seed={seed}: {len(want)} patterns")
    G = nuri.Graph.from_synth(g)
    try:
        for k in (1, 2, 5, 10 ** 6):
            assert nuri.topk_patterns(G, M, k)[0] == want[:k], k
    finally:
        G.close()


@pytest.mark.parametrize("seed,M", [(13, 2), (81, 3), (135, 2), (135, 3)])
def test_ties_at_the_kth_support(nuri, seed, M):
    g = synth.gnp(8 + seed % 5, 0.4, 1000 + seed)
    synth.add_zipf_labels(g, n_labels=1 + seed % 2, s=0.5, master=1000 + seed)
    want = oracle.topk_patterns_definition(g, M, 10 ** 6)
    _case(f"pattern ties seed={seed} M={M}")
    G = nuri.Graph.from_synth(g)
    try:
        for k in (1, 2, 3):
            assert nuri.topk_patterns(G, M, k)[0] == want[:k], k
    finally:
        G.close()


_CS = {}


def _citeseer_like(n_labels):
    """Chung-Lu stand-in for the citation graph the paper mines (3,300
    vertices, ~4,400 edges, expected degrees capped at 100) with Zipf
    labels."""
    if n_labels not in _CS:
        g = synth.chung_lu(n=3300, m_target=4500, cap=100, n_cliques=0)
        synth.add_zipf_labels(g, n_labels=n_labels, s=0.8, master=31)
        _CS[n_labels] = g
    return _CS[n_labels]


@pytest.mark.parametrize("n_labels,M", [(6, 1), (6, 2), (6, 3), (16, 3), (16, 4)])
def test_citeseer_like_vs_oracle(nuri, n_labels, M):
    g = _citeseer_like(n_labels)
    _case(f"citeseer-like, {n_labels} labels, M={M}")
    G = nuri.Graph.from_synth(g)
    try:
        for k in (1, 10, 100):
            want, ost = oracle.topk_patterns(g, M, k)
            got, st = nuri.topk_patterns(G, M, k)
            assert got == want, k
            # the same groups are taken and expanded in the same order
            assert st["popped"] == ost["popped"] and st["expanded"] == ost["expanded"]
            assert st["children"] == ost["children"]
            assert st["pruned_at_pop"] == ost["pruned_at_pop"]
            assert st["pruned_at_creation"] == ost["pruned_at_creation"]
    finally:
        G.close()


def test_rmat12_two_edges_vs_oracle(nuri):
    g = synth.rmat(12)
    synth.add_zipf_labels(g)
    want, _ = oracle.topk_patterns(g, 2, 50)
    _case("R-MAT 12, 16 labels, M=2")
    G = nuri.Graph.from_synth(g)
    try:
        assert nuri.topk_patterns(G, 2, 50)[0] == want
    finally:
        G.close()


def test_pattern_edge_cases(nuri):
    _case("pattern mining edge cases")
    g = synth.gnp(30, 0.2, 3)
    G = nuri.Graph.from_synth(g)
    try:
        with pytest.raises(nuri.NuriError):
            nuri.topk_patterns(G, 2, 5)  # no labels
    finally:
        G.close()
    g.vertex_label = np.zeros(g.n, np.uint8)
    G = nuri.Graph.from_synth(g)
    try:
        for bad in ((0, 5), (9, 5), (2, 0)):
            with pytest.raises(nuri.NuriError):
                nuri.topk_patterns(G, *bad)
        deg = np.diff(g.row_ptr)
        assert nuri.topk_patterns(G, 1, 3)[0] == [(int((deg >= 1).sum()), ((0, 1, 0, 0),))]
        want = oracle.topk_patterns_definition(g, 2, 100) if g.m <= 64 else \
            oracle.topk_patterns(g, 2, 100)[0]
        assert nuri.topk_patterns(G, 2, 100)[0] == want
    finally:
        G.close()
    # no edges: no pattern
    g = synth.from_edges(5, [])
    g.vertex_label = np.zeros(5, np.uint8)
    G = nuri.Graph.from_synth(g)
    try:
        assert nuri.topk_patterns(G, 1, 3)[0] == []
    finally:
        G.close()


def test_pattern_budget_and_deadline_fail_loudly(nuri):
    """The embeddings of 4-edge patterns on the 6-label stand-in held at
    once exceed 64 MiB: under the smallest budget (64 MiB) the query fails with
    EBUDGET; a deadline that has passed at the first group fails with
    ETIMEOUT; the graph still answers exactly afterwards."""
    g = _citeseer_like(6)
    _case("pattern mining budget and deadline")
    G = nuri.Graph.from_synth(g)
    try:
        _, st = nuri.topk_patterns(G, 4, 10)
        assert st["frontier_peak_bytes"] > 64 << 20, st["frontier_peak_bytes"]
        with pytest.raises(nuri.NuriError) as e:
            nuri.topk_patterns(G, 4, 10, frontier_budget_bytes=64 << 20)
        assert "EBUDGET" in str(e.value)
        with pytest.raises(nuri.NuriError) as e:
            nuri.topk_patterns(G, 3, 10, deadline_ns=1)
        assert "ETIMEOUT" in str(e.value)
        want, _ = oracle.topk_patterns(g, 2, 10)
        assert nuri.topk_patterns(G, 2, 10)[0] == want
    finally:
        G.close()
