"""Readers for stored expected results under tests/golden/."""
import hashlib
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def graph_sha256(g) -> str:
    """Hash of a graph's CSR arrays (ties a stored list to the generator's output)."""
    h = hashlib.sha256()
    h.update(g.row_ptr.astype("<u8").tobytes())
    h.update(g.col.astype("<u4").tobytes())
    return h.hexdigest()


def power_law_top100():
    """(graph_sha256, [(size, ids ascending)]) from power_law_top100.txt."""
    common, residual, items, sha = [], [], [], None
    with open(os.path.join(GOLDEN, "power_law_top100.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            tag, _, rest = line.strip().partition(" ")
            if tag == "graph_sha256":
                sha = rest
            elif tag == "common":
                common = [int(x) for x in rest.split()]
            elif tag == "residual":
                residual = [int(x) for x in rest.split()]
            elif tag == "result":
                size, mask = rest.split()
                m = int(mask, 16)
                ids = sorted(common + [residual[j] for j in range(len(residual)) if m >> j & 1])
                assert len(ids) == int(size)
                items.append((int(size), tuple(ids)))
    return sha, items
