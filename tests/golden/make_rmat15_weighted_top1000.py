"""Writes rmat15_weighted_top1000.txt: the CPU oracle's top-1000 maximal
cliques by vertex weight on R-MAT scale 15 (a = 0.57, b = c = 0.19, vertex
weights U{1..100}, the generator's default seed), with the graph's hash.

Every top-k list of this graph for k <= 1000 is a prefix of this list (the
results are ranked under a total order), so one stored list checks all the
queries of a batch with k drawn in 1..1000.  Run from anywhere:
python tests/golden/make_rmat15_weighted_top1000.py
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402
from tests.golden_lists import workload_sha256  # noqa: E402

SCALE, K = 15, 1000
OUT = os.path.join(HERE, "rmat15_weighted_top1000.txt")


def workload():
    g = synth.rmat(SCALE)
    synth.add_vertex_weights(g)
    return g


def main():
    g = workload()
    t = time.time()
    res, st = oracle.topk_cliques(g, K, weighted=True, bound=1)
    print(f"oracle: {len(res)} results in {time.time() - t:.1f} s, {st['children']} children")
    # the results share most of their vertices: store the sorted union once
    # and each result as a hex mask over it
    base = sorted({v for _, ids in res for v in ids})
    at = {v: i for i, v in enumerate(base)}
    with open(OUT, "w") as f:
        f.write("# Top-1000 maximal cliques by vertex weight, R-MAT scale 15, from the CPU\n"
                "# oracle; written by make_rmat15_weighted_top1000.py.  base <the sorted\n"
                "# vertices of all results>; result <score> <hex mask over base>\n")
        f.write(f"workload_sha256 {workload_sha256(g)}\n")
        f.write(f"base {' '.join(str(v) for v in base)}\n")
        for s, ids in res:
            f.write(f"result {s} {sum(1 << at[v] for v in ids):x}\n")
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
