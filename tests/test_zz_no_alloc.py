"""The allocation-free clique entry point (nuri_topk_cliques_noalloc)
against nuri_topk_cliques, through the C ABI: two calls in a row on the
device's static scratch array, the second with a smaller input, each
bit-exact with the allocating entry point."""
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nuri():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1807_08888_amd import nuri as N
    N.lib()
    return N


def _both(nuri, g, k, wf, **opts):
    G = nuri.Graph.from_synth(g)
    try:
        items, stats = nuri.topk_cliques_noalloc(G, k, wf, **opts)
        ref = nuri.topk_cliques(G, k, wf, **opts)
    finally:
        G.close()
    return items, stats, ref


def test_noalloc_equals_allocating_entry_point_twice(nuri):
    big = synth.rmat(12)
    synth.add_vertex_weights(big)
    print("[case] noalloc: R-MAT 12, top-100 by vertex weight", flush=True)
    items, stats, ref = _both(nuri, big, 100, 1)
    assert items == ref.items and len(items) == 100
    assert stats["children"] > 0
    small = synth.gnp(120, 0.1, 5)
    print("[case] noalloc: G(120, 0.1), top-7 by size", flush=True)
    items2, _, ref2 = _both(nuri, small, 7, 0)
    assert items2 == ref2.items and len(items2) == 7


def test_noalloc_rejects_sizes_beyond_its_limits(nuri):
    g = synth.gnp(50, 0.2, 1)
    G = nuri.Graph.from_synth(g)
    try:
        with pytest.raises(nuri.NuriError) as e:
            nuri.topk_cliques_noalloc(G, 1001, 0)
        assert e.value.name == "EINVAL"
        with pytest.raises(nuri.NuriError) as e:
            nuri.topk_cliques_noalloc(G, 0, 0)
        assert e.value.name == "EINVAL"
        # still usable after the refusals
        items, _ = nuri.topk_cliques_noalloc(G, 5, 0)
        assert items == nuri.topk_cliques(G, 5, 0).items
    finally:
        G.close()
