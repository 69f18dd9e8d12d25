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


def workload_sha256(g) -> str:
    """Hash of a graph's CSR arrays and of whichever of vertex weights,
    vertex labels and edge weights it carries."""
    h = hashlib.sha256()
    h.update(g.row_ptr.astype("<u8").tobytes())
    h.update(g.col.astype("<u4").tobytes())
    for name, arr, dt in (("vertex_weight", g.vertex_weight, "<i4"),
                          ("vertex_label", g.vertex_label, "u1"),
                          ("edge_weight", g.edge_weight, "<i4")):
        if arr is not None:
            h.update(name.encode())
            h.update(arr.astype(dt).tobytes())
    return h.hexdigest()


def result_sha256(items) -> str:
    """Hash of a result list [(score, ids tuple)] in its canonical text."""
    canon = [(int(s), tuple(int(x) for x in ids)) for s, ids in items]
    return hashlib.sha256(repr(canon).encode()).hexdigest()


def rmat22_match_top50():
    """(workload_sha256, {pattern index: (count, best score, result sha256)});
    patterns the oracle did not finish are absent."""
    rows, sha = {}, None
    with open(os.path.join(GOLDEN, "rmat22_match_top50.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            if parts[0] == "workload_sha256":
                sha = parts[1]
            elif parts[0] == "pattern" and parts[2] != "unfinished":
                rows[int(parts[1])] = (int(parts[2]), int(parts[3]), parts[4])
    return sha, rows


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


def rmat15_weighted_top1000():
    """(workload_sha256, [(score, ids ascending)]) from rmat15_weighted_top1000.txt."""
    items, sha, base = [], None, []
    with open(os.path.join(GOLDEN, "rmat15_weighted_top1000.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            if parts[0] == "workload_sha256":
                sha = parts[1]
            elif parts[0] == "base":
                base = [int(x) for x in parts[1:]]
            elif parts[0] == "result":
                m = int(parts[2], 16)
                items.append((int(parts[1]), tuple(base[j] for j in range(len(base)) if m >> j & 1)))
    return sha, items
