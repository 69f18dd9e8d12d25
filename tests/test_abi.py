"""The C-ABI library: it loads, exports every function include/nuri.h
declares, and rejects malformed input before touching the GPU (no GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nuri.h")


@pytest.fixture(scope="module")
def nuri():
    from paper_1807_08888_amd import nuri as N
    if not os.path.exists(N.LIB_PATH):
        from paper_1807_08888_amd import build
        build.build()
    N.lib()
    return N


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nuri_[a-z_]+)\s*\(", text)))


def test_header_declares_the_expected_entry_points():
    names = _declared_functions()
    for n in ("nuri_load_graph", "nuri_topk_cliques", "nuri_topk_match", "nuri_topk_batch",
              "nuri_server_create", "nuri_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(nuri):
    L = ctypes.CDLL(nuri.LIB_PATH)
    missing = [n for n in _declared_functions() if not hasattr(L, n)]
    assert missing == []
    assert set(_declared_functions()) == set(nuri.SIGNATURES)


def _expect_einval(nuri, rp, col, **kw):
    with pytest.raises(nuri.NuriError) as e:
        nuri.Graph(np.array(rp, np.uint64), np.array(col, np.uint32), **kw)
    assert e.value.name == "EINVAL", str(e.value)
    return str(e.value)


def test_malformed_csr_rejected(nuri):
    assert "symmetric" in _expect_einval(nuri, [0, 1, 1], [1])
    assert "self loop" in _expect_einval(nuri, [0, 1, 2], [0, 0])
    assert "increasing" in _expect_einval(nuri, [0, 2, 3, 4], [2, 1, 0, 0])
    assert "range" in _expect_einval(nuri, [0, 1, 2], [5, 0])
    assert "row_ptr" in _expect_einval(nuri, [1, 1, 2], [1, 0])
    # duplicate entry = row not strictly increasing
    assert "increasing" in _expect_einval(nuri, [0, 2, 4], [1, 1, 0, 0])


def test_bad_weights_and_labels_rejected(nuri):
    rp, col = [0, 1, 2], [1, 0]
    assert "vertex weights" in _expect_einval(nuri, rp, col, vertex_weight=np.array([0, 1]))
    assert "label" in _expect_einval(nuri, rp, col, vertex_label=np.array([0, 16]))
    assert "edge weights" in _expect_einval(nuri, rp, col, edge_weight=np.array([3, 4]))


def test_errors_are_reported_not_hidden(nuri):
    g = synth.gnp(6, 0.5, 3)
    try:
        nuri.Graph.from_synth(g)
    except nuri.NuriError as e:  # no GPU here: the device error is reported
        assert e.name in ("EDEVICE", "ENOMEM")
        assert nuri.lib().nuri_last_error()


def test_bench_traffic_is_null_unless_the_kernel_source_matches(tmp_path, monkeypatch):
    """bench.py reports counter traffic only for the kernel the counters were taken on."""
    import bench
    h = bench.kernel_source_hash()
    good = tmp_path / "summary.md"
    good.write_text(f"x\ntraffic_bytes_per_launch: 1234\nkernel_source_sha256: {h}\n")
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(good))
    assert bench.measured_traffic() == 1234.0
    stale = tmp_path / "stale.md"
    stale.write_text("traffic_bytes_per_launch: 1234\nkernel_source_sha256: " + "0" * 64 + "\n")
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(stale))
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(tmp_path / "missing.md"))
    assert bench.measured_traffic() is None


# ctypes mirror of each struct in include/nuri.h
_STRUCTS = {"nuri_csr": "_CSR", "nuri_graph_info": "_GraphInfo", "nuri_pattern": "_Pattern",
            "nuri_opts": "_Opts", "nuri_query": "_Query", "nuri_result_view": "_View",
            "nuri_stats": "_Stats"}


def test_binding_structs_match_the_header(nuri, tmp_path):
    """sizeof and every field offset of the ctypes structures equal what a C
    compiler makes of include/nuri.h, and the status and score constants
    agree (a mismatch would corrupt arguments silently)."""
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "nuri.h"', "int main(void) {"]
    want = []
    for cname, pyname in _STRUCTS.items():
        py = getattr(nuri, pyname)
        lines.append(f'  printf("%zu\\n", sizeof({cname}));')
        want.append(ctypes.sizeof(py))
        for f, _ in py._fields_:
            lines.append(f'  printf("%zu\\n", offsetof({cname}, {f}));')
            want.append(getattr(py, f).offset)
    for code, name in nuri.ERRORS.items():
        lines.append(f'  printf("%d\\n", (int)NURI_{name});')
        want.append(code)
    lines.append('  printf("%d\\n%d\\n", (int)NURI_SCORE_SIZE, (int)NURI_SCORE_VERTEX_WEIGHT);')
    want += [nuri.SCORE_SIZE, nuri.SCORE_VERTEX_WEIGHT]
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    import subprocess
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.dirname(HEADER),
                           "-o", str(exe), str(src)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert got == want


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU and says so for --gpus N > 1 (no GPU needed)."""
    import subprocess
    import sys
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert p.returncode != 0
    assert "one GPU" in p.stdout + p.stderr


def test_binding_marshals_queries_and_options(nuri):
    """Query dicts and keyword options reach the C structs unchanged (no GPU)."""
    qs, keep = nuri._queries([
        {"kind": "clique", "k": 7, "weight_fn": 1},
        {"kind": "match", "k": 11, "labels": [3, 0, 3], "edges": [(0, 1), (1, 2)]},
        {"kind": "clique", "k": 1},
    ])
    assert (qs[0].kind, qs[0].k, qs[0].wf, bool(qs[0].p)) == (0, 7, 1, False)
    assert (qs[2].kind, qs[2].k, qs[2].wf) == (0, 1, nuri.SCORE_SIZE)
    assert (qs[1].kind, qs[1].k) == (1, 11)
    p = qs[1].p.contents
    assert (p.q, p.n_edges) == (3, 2)
    assert list(ctypes.cast(p.label, ctypes.POINTER(ctypes.c_uint8))[:3]) == [3, 0, 3]
    assert list(ctypes.cast(p.edges, ctypes.POINTER(ctypes.c_uint32))[:4]) == [0, 1, 1, 2]
    o = nuri._opts(frontier_budget_bytes=1 << 30, batch_B=4096, root_batch=512, bound=2,
                   deadline_ns=5, profile=True, stream=1234)
    assert (o.frontier_budget_bytes, o.batch_B, o.root_batch, o.bound, o.deadline_ns,
            o.profile, o.hip_stream) == (1 << 30, 4096, 512, 2, 5, 1, 1234)
    d = nuri._opts()
    assert (d.frontier_budget_bytes, d.batch_B, d.root_batch, d.bound, d.deadline_ns,
            d.profile, d.hip_stream) == (0, 0, 0, 0, 0, 0, None)


def test_binding_fails_loudly_without_the_library(tmp_path, monkeypatch):
    """No CPU fallback: a missing libnuri.so is an error, not a silent detour."""
    from paper_1807_08888_amd import nuri as N
    monkeypatch.setattr(N, "_lib", None)
    monkeypatch.setattr(N, "LIB_PATH", str(tmp_path / "libnuri.so"))
    with pytest.raises(RuntimeError, match="missing"):
        N.lib()


def test_product_package_never_reaches_the_oracle():
    """The HIP path and the oracle share no code: nothing under the package
    imports, loads or names the oracle module or its library."""
    pkg = os.path.join(ROOT, "paper_1807_08888_amd")
    offenders = []
    for dirpath, _, files in os.walk(pkg):
        if "_build" in dirpath or "__pycache__" in dirpath:
            continue
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".hpp", ".cpp", ".c")):
                text = open(os.path.join(dirpath, f), errors="replace").read()
                if re.search(r"\boracle\b|liboracle", text):
                    offenders.append(os.path.join(dirpath, f))
    assert offenders == []
