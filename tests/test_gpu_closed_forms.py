"""GPU results against closed forms (no oracle involved): complete
multipartite and Moon-Moser graphs (thousands of maximal cliques that tie on
size), cycles and disjoint complete graphs, by size and by vertex weight,
under every clique bound setting.  Bit-exact on (score, ascending ids).
"""
import numpy as np
import pytest

from tests import closed_forms as cf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nuri():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1807_08888_amd import nuri as N
    N.lib()
    return N


def _run(nuri, g, queries):
    G = nuri.Graph.from_synth(g)
    try:
        return [nuri.topk_cliques(G, k, wf, bound=b).items for k, wf, b in queries]
    finally:
        G.close()


@pytest.mark.parametrize("sizes,seed", [((3,) * 7, 1), ((1, 2, 3, 4, 2), 2), ((5, 1, 1, 4), 3)])
def test_complete_multipartite(nuri, sizes, seed):
    print(f"[case] multipartite {sizes}", flush=True)
    g, parts = cf.multipartite(sizes, seed)
    w = np.random.default_rng(seed + 50).integers(1, 4, g.n)
    cf.set_weights(g, w)
    want = {0: cf.ranked(cf.transversals(parts)),
            1: cf.ranked(cf.transversals(parts), cf.weight_of(w))}
    n_all = int(np.prod(sizes))
    qs = [(k, wf, b) for k in (1, 100, n_all, n_all + 7) for wf in (0, 1) for b in (0, 1, 2)]
    for (k, wf, b), got in zip(qs, _run(nuri, g, qs)):
        assert got == want[wf][:k], (k, wf, b)


def test_cycle_and_disjoint_cliques(nuri):
    print("[case] cycle n=30 and disjoint complete graphs", flush=True)
    g, edges = cf.cycle(30, 30)
    for (k, _, _), got in zip([(k, 0, 0) for k in (1, 30, 40)],
                              _run(nuri, g, [(k, 0, 0) for k in (1, 30, 40)])):
        assert got == cf.ranked(edges)[:k]
    g, comps = cf.disjoint_cliques((5, 3, 5, 1, 2, 7, 70), 1)
    w = np.random.default_rng(2).integers(1, 6, g.n)
    cf.set_weights(g, w)
    qs = [(k, wf, 0) for k in (1, 3, 7, 100) for wf in (0, 1)]
    for (k, wf, _), got in zip(qs, _run(nuri, g, qs)):
        want = cf.ranked(comps, cf.weight_of(w) if wf else len)
        assert got == want[:k], (k, wf)
