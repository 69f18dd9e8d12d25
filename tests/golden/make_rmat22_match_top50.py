"""Writes rmat22_match_top50.txt: for each of the 128 patterns of the
labelled-matching workload (R-MAT scale 22, vertex and edge weights, 16
Zipf labels; synth.random_pattern(0..127); top-50 each, the benchmark's
batch), the CPU oracle's result summarised as its length, its best score
and the SHA-256 of its canonical text (repr of the list of (score, tuple)
pairs, as the oracle and the GPU binding both return it).

A hash keeps the fixture small (the lists are ~300 KB); a test that finds a
different hash can recompute that one pattern with the oracle to see the
difference.  The oracle takes from a few seconds to about a minute per
pattern on this graph; the patterns are shared out over worker processes.

Run from anywhere: python tests/golden/make_rmat22_match_top50.py [workers]
[deadline seconds] [--resume].  With a deadline, patterns the oracle has not
finished by then are written as "unfinished" and the tests skip them.  With
--resume, the rows already in the file are kept and only the unfinished
patterns are run.  The file is rewritten after every finished pattern, so an
interrupted run keeps what it finished.
"""
import hashlib
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402
from tests.golden_lists import result_sha256, workload_sha256  # noqa: E402

SCALE, N_PATTERNS, K = 22, 128, 50
OUT = os.path.join(HERE, "rmat22_match_top50.txt")


def workload():
    g = synth.rmat(SCALE)
    synth.add_vertex_weights(g)
    synth.add_edge_weights(g)
    synth.add_zipf_labels(g)
    return g


_g = None


def _one(i):
    global _g
    if _g is None:
        _g = workload()
    p = synth.random_pattern(i)
    t = time.time()
    res, _ = oracle.topk_match(_g, p.labels, p.edges, K)
    return i, len(res), (res[0][0] if res else 0), result_sha256(res), time.time() - t


def _read_rows():
    rows = {}
    if not os.path.exists(OUT):
        return rows
    with open(OUT) as f:
        for line in f:
            parts = line.split()
            if len(parts) == 5 and parts[0] == "pattern":
                rows[int(parts[1])] = (int(parts[2]), int(parts[3]), parts[4])
    return rows


def _write(sha, rows):
    tmp = OUT + ".tmp"
    with open(tmp, "w") as f:
        f.write("# Top-50 labelled matches of the 128 patterns of the R-MAT scale-22\n"
                "# matching workload, from the CPU oracle; written by\n"
                "# make_rmat22_match_top50.py.  pattern <i> <count> <best score> <sha256>\n")
        f.write(f"workload_sha256 {sha}\n")
        for i in range(N_PATTERNS):
            if i in rows:
                n, top, h = rows[i]
                f.write(f"pattern {i} {n} {top} {h}\n")
            else:
                f.write(f"pattern {i} unfinished\n")
    os.replace(tmp, OUT)


def main():
    args = [a for a in sys.argv[1:] if not a.startswith("--")]
    resume = "--resume" in sys.argv[1:]
    workers = int(args[0]) if args else 8
    deadline = float(args[1]) if len(args) > 1 else None
    t0 = time.time()
    sha = workload_sha256(workload())
    rows = _read_rows() if resume else {}
    todo = [i for i in range(N_PATTERNS) if i not in rows]
    # spawn, not fork: the generator runs threads, and a forked copy of a
    # threaded process can deadlock in them
    pool = mp.get_context("spawn").Pool(workers)
    it = pool.imap_unordered(_one, todo)
    try:
        for _ in range(len(todo)):
            left = None if deadline is None else max(1.0, deadline - (time.time() - t0))
            try:
                i, n, top, h, dt = it.next(timeout=left)
            except mp.TimeoutError:
                break
            rows[i] = (n, top, h)
            _write(sha, rows)
            print(f"pattern {i}: {n} results, best {top}, {dt:.1f} s "
                  f"({len(rows)}/{N_PATTERNS}, {time.time() - t0:.0f} s)", flush=True)
    finally:
        pool.terminate()
    _write(sha, rows)
    print(f"wrote {OUT} ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
