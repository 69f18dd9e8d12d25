"""Benchmark: top-k maximal clique discovery on the power-law workload.

Workload (one "step" = one full top-k query through the HIP engine, inputs
resident in HBM): Chung-Lu graph, 1,000,000 vertices, ~20M undirected
edges, degree exponent 2.1, expected degree capped at 20,000, 200 planted
cliques of 20..40 vertices; top-100 maximal cliques by size.

Prints one JSON line with the throughput in expanded subgraphs (children
created, the paper's candidate-subgraph count) per second, the query time,
the expansion kernel's roofline figures and the CPU oracle timed on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "chung_lu_n1M_m20M_beta2.1_cap20k_planted200x20-40_top100_maximal_cliques_size"


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(g, k: int, seconds: float) -> dict:
    """The oracle on the same workload, stopped after a bounded amount of work.

    The oracle is single-threaded; its children-per-second rate is measured
    on a child cap sized from a short calibration run to take about
    `seconds` of CPU time.
    """
    import oracle
    oracle.set_work_limit(200_000)
    t = time.perf_counter()
    _, st = oracle.topk_cliques(g, k)
    dt = max(time.perf_counter() - t, 1e-6)
    rate = st["children"] / dt
    cap = max(200_000, int(rate * seconds))
    oracle.set_work_limit(cap)
    t = time.perf_counter()
    _, st = oracle.topk_cliques(g, k)
    dt = time.perf_counter() - t
    oracle.set_work_limit(0)
    return {"value": st["children"] / dt, "unit": "subgraphs/s", "cores": 1, "kind": "oracle",
            "sample": f"first {st['children']} children of the same top-{k} query "
                      f"(search capped, {dt:.1f} s, one host core)"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--k", type=int, default=100)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB device copy first (scales HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the engine has no multi-GPU path)", file=sys.stderr)
        return 2

    import torch
    import synth
    from paper_1807_08888_amd import nuri

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()

    t = time.perf_counter()
    g = synth.chung_lu()
    _log(f"generated graph n={g.n} m={g.m} in {time.perf_counter() - t:.1f}s")
    G = nuri.Graph.from_synth(g, stream=stream)
    info = G.info()
    _log(f"loaded: {info}")

    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
        src.fill_(1)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        _log("copy calibration: 1 GiB read + 1 GiB written")

    def one():
        return nuri.topk_cliques(G, args.k, nuri.SCORE_SIZE, profile=True, stream=stream)

    ref = None
    for i in range(args.warmup):
        r = one()
        ref = r.items
        _log(f"warmup {i}: {r.stats['wall_ns'] / 1e6:.1f} ms, children {r.stats['children']}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for i in range(args.steps):
        results.append(one())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    for i, r in enumerate(results):
        _log(f"step {i}: {r.stats['wall_ns'] / 1e6:.1f} ms, children {r.stats['children']}, "
             f"expand {r.stats['expand_ns'] / 1e6:.1f} ms in {r.stats['expand_launches']} launches")
        if ref is not None and r.items != ref:
            raise SystemExit("result changed between runs")
    children = sum(r.stats["children"] for r in results)
    lbytes = sum(r.stats["logical_bytes"] for r in results)
    ens = sum(r.stats["expand_ns"] for r in results)
    launches = sum(r.stats["expand_launches"] for r in results)
    achieved = (lbytes / launches) / (ens / launches) if ens else 0.0  # bytes/ns == GB/s
    line = {
        "metric": "expanded subgraphs/s (top-k query)",
        "value": children / elapsed,
        "unit": "subgraphs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "n": g.n, "m": g.m, "k": args.k,
                   "max_clique": results[-1].items[0][0] if results[-1].items else 0,
                   "children_per_query": children // args.steps,
                   "preprocess_ms": info["preprocess_ns"] / 1e6},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_expand", "avg_launch_us": ens / launches / 1e3 if launches else 0,
                     "launches_per_query": launches // args.steps},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(g, args.k, args.cpu_seconds)
    print(json.dumps(line), flush=True)
    G.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
