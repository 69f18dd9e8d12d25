"""Writes power_law_top100.txt: the exact top-100 maximal cliques by size of
the power-law workload (Chung-Lu, n = 1,000,000, exponent 2.1, expected
degree cap 20,000, 200 planted cliques; the benchmark's graph), computed by
the CPU oracle alone.

The oracle cannot search the whole graph in reasonable time, so it runs on
the exact large-clique kernel of oracle.large_clique_kernel: for cliques of
at least MIN_SIZE vertices, the core/truss peeling and the vertices common
to every such clique reduce the graph to a residual of a few hundred
vertices.  If the oracle's top-100 on the residual all reach MIN_SIZE once
the common vertices are added, they are the top-100 of the whole graph
(every clique of MIN_SIZE or more vertices is represented in the residual,
and every smaller one ranks below them).  MIN_SIZE only sets how far the
reduction goes; a value too large would leave fewer than 100 results and
the script would fail rather than write a wrong list.

Run from the repository root: python tests/golden/make_power_law_top100.py
(under a minute on one core).
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402
from tests.golden_lists import graph_sha256  # noqa: E402

K = 100
MIN_SIZE = 501
OUT = os.path.join(HERE, "power_law_top100.txt")


def main():
    t0 = time.time()
    g = synth.chung_lu()
    resid, rid, common = oracle.large_clique_kernel(g, MIN_SIZE)
    print(f"kernel: {resid.n} residual vertices, {resid.nnz // 2} edges, "
          f"{len(common)} common ({time.time() - t0:.0f} s)", flush=True)
    # bound-first priority and the colouring bound: the result does not
    # depend on either (tests/test_oracle_clique.py), the time does (about
    # 15 s; the paper's (|V|, |P|) priority takes about 15 minutes here)
    res, st = oracle.topk_cliques(resid, K, bound=1, priority=1)
    print(f"oracle on the residual: {st} ({time.time() - t0:.0f} s)", flush=True)
    if len(res) < K or any(len(common) + len(ids) < MIN_SIZE for _, ids in res):
        sys.exit("fewer than K maximal cliques reach MIN_SIZE: lower MIN_SIZE")
    rid = [int(v) for v in rid]
    with open(OUT, "w") as f:
        f.write("# Top-100 maximal cliques by size of the power-law workload\n"
                "# (synth.chung_lu() defaults), written by make_power_law_top100.py\n"
                "# from the CPU oracle on the exact large-clique kernel.\n"
                "# Result i = sorted(common + [residual[j] for each bit j of mask i]).\n")
        f.write(f"graph_sha256 {graph_sha256(g)}\n")
        f.write(f"k {K}\n")
        f.write("common " + " ".join(map(str, common)) + "\n")
        f.write("residual " + " ".join(map(str, rid)) + "\n")
        for score, ids in res:
            mask = 0
            for j in ids:
                mask |= 1 << int(j)
            f.write(f"result {len(common) + score} {mask:x}\n")
    print(f"wrote {OUT} ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
