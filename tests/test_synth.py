"""The seeded input generators (no GPU): the recipes the workloads are
built from hold what they state, and every draw is reproducible.

Randomness is splitmix64 used as a counter-based generator (value i of a
stream with seed s is the splitmix64 finaliser of s + (i+1) * golden
gamma), so the first draws from seed 0 are the published splitmix64
sequence.
"""
import numpy as np
import pytest

import synth


def _check_simple(g):
    rp = g.row_ptr.astype(np.int64)
    assert rp[0] == 0 and rp[-1] == len(g.col) and np.all(np.diff(rp) >= 0)
    rows = np.repeat(np.arange(g.n), np.diff(rp))
    col = g.col.astype(np.int64)
    assert np.all(col < g.n) and not np.any(col == rows)
    same_row = rows[1:] == rows[:-1]
    assert np.all(col[1:][same_row] > col[:-1][same_row])  # strictly increasing rows
    fwd = rows * g.n + col
    bwd = col * g.n + rows
    assert np.array_equal(np.sort(fwd), np.sort(bwd))  # symmetric
    return rows, col


def test_splitmix64_reference_sequence():
    assert [synth.draw(0, i) for i in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                                     0x06C45D188009454F]
    lib = synth._load()
    for s in (0, 1, 0xDEADBEEF, synth.stream_seed(synth.MASTER_SEED, 3)):
        for i in (0, 1, 1000, 2 ** 40):
            assert lib.synth_draw(s, i) == synth.draw(s, i)  # C and Python agree


def test_planted_clique_workload():
    g = synth.er_planted()
    assert g.n == 2000
    _check_simple(g)
    assert abs(g.degree().mean() - 20.0) < 1.5
    seen = set()
    rp = g.row_ptr.astype(np.int64)
    for p in g.planted:
        assert 8 <= len(p) <= 15 and not (seen & set(p.tolist()))
        seen |= set(p.tolist())
        for u in p:
            row = set(g.col[rp[u]:rp[u + 1]].tolist())
            assert set(p.tolist()) - {int(u)} <= row
    h = synth.er_planted()
    assert np.array_equal(g.col, h.col) and np.array_equal(g.row_ptr, h.row_ptr)
    other = synth.er_planted(master=synth.MASTER_SEED + 1)
    assert not np.array_equal(g.col, other.col)


def test_rmat_shape_and_skew():
    g = synth.rmat(12)
    assert g.n == 4096
    _check_simple(g)
    deg = g.degree()
    assert g.nnz <= 2 * 16 * g.n
    assert deg.max() > 20 * deg.mean()  # (0.57, 0.19, 0.19) concentrates edges on low ids


def test_weights_in_range_and_symmetric():
    g = synth.rmat(10)
    synth.add_vertex_weights(g)
    synth.add_edge_weights(g)
    assert g.vertex_weight.min() >= 1 and g.vertex_weight.max() <= 100
    assert g.edge_weight.min() >= 1 and g.edge_weight.max() <= 1000
    rows, col = _check_simple(g)
    key = {}
    for r, c, w in zip(rows.tolist(), col.tolist(), g.edge_weight.tolist()):
        key[(r, c)] = w
    assert all(key[(c, r)] == w for (r, c), w in key.items())
    assert len(set(g.vertex_weight.tolist())) > 90  # uniform over 1..100


def test_zipf_labels_follow_the_pmf():
    g = synth.rmat(16)
    synth.add_zipf_labels(g)
    freq = np.bincount(g.vertex_label, minlength=16) / g.n
    pmf = synth.zipf_pmf()
    sigma = np.sqrt(pmf * (1 - pmf) / g.n)
    assert np.all(np.abs(freq - pmf) < 5 * sigma)
    assert g.vertex_label.max() < 16


@pytest.mark.parametrize("q_lo,q_hi", [(3, 7), (3, 8), (2, 5)])
def test_random_patterns_are_valid(q_lo, q_hi):
    sizes = set()
    for i in range(300):
        p = synth.random_pattern(i, q_lo=q_lo, q_hi=q_hi)
        assert q_lo <= p.q <= q_hi and len(p.labels) == p.q
        sizes.add(p.q)
        assert all(0 <= a < b < p.q for a, b in p.edges) and len(set(p.edges)) == len(p.edges)
        assert p.q - 1 <= len(p.edges) <= p.q - 1 + min(p.q - 1, p.q * (p.q - 1) // 2 - (p.q - 1))
        reach, frontier = {0}, [0]
        while frontier:
            v = frontier.pop()
            for a, b in p.edges:
                for x, y in ((a, b), (b, a)):
                    if x == v and y not in reach:
                        reach.add(y)
                        frontier.append(y)
        assert reach == set(range(p.q))  # connected
        assert all(0 <= l < 16 for l in p.labels)
        assert synth.random_pattern(i, q_lo=q_lo, q_hi=q_hi) == p
    assert sizes == set(range(q_lo, q_hi + 1))


def test_log_uniform_k():
    ks = np.array([synth.log_uniform_k(i) for i in range(4000)])
    assert ks.min() >= 1 and ks.max() <= 1000
    # log-uniform on [1, 1001): about half of the draws fall below sqrt(1001)
    assert abs(np.mean(ks < np.sqrt(1001.0)) - 0.5) < 0.05


def test_power_law_workload_as_stated():
    """The benchmark's graph: n = 1M, 19,541,719 edges, degeneracy 602."""
    import oracle
    g = synth.chung_lu()
    assert g.n == 1_000_000 and g.nnz == 2 * 19_541_719
    rank = oracle.vertex_order(g, 1).astype(np.int64)  # position of each vertex
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr.astype(np.int64)))
    later = rank[g.col.astype(np.int64)] > rank[rows]
    assert np.bincount(rows[later], minlength=g.n).max() == 602
