"""Planted mistakes in the oracle, on the CPU (no GPU).

Each mutant below is oracle.c with one plausible mistake (a dropped term, a
wrong comparison, a missing check, a wrong index).  It is compiled on its own and run
against a battery of the oracle's pins (brute force over small graphs for
both clique scores, both bounds, and labelled matching); the battery must
fail for every mutant and pass for the real oracle, so that a mistake of
that kind in the oracle would not go unnoticed.
"""
import contextlib
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth
from tests import bruteforce
from tests.test_oracle_match_degree import _index_from_distances as index_from_distances
from tests.test_oracle_patterns import _all_dfs_codes as all_dfs_codes
from tests.test_oracle_patterns import _key as dfs_key
from tests.test_oracle_patterns import _nx_support as pattern_support_nx
from tests.test_oracle_patterns import _random_labelled_connected as random_pattern_graph

ORACLE_C = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

# (name, text in oracle.c, replacement); text and replacement may be tuples
# of the same length for a mistake made in several places
MUTANTS = [
    ("pruning at or below the k-th score (not strict)",
     "return R->n == R->k && bound < R->e[R->k - 1].score;",
     "return R->n == R->k && bound <= R->e[R->k - 1].score;"),
    ("bound without the current score",
     "  int64_t b = s->score;\n  if (bound_kind == 0) {",
     "  int64_t b = 0;\n  if (bound_kind == 0) {"),
    ("child candidates not filtered by adjacency",
     "if (is_adjacent(g, p, s->P[j])) c->P[c->np++] = s->P[j];",
     "c->P[c->np++] = s->P[j];"),
    ("earlier candidates left out of X",
     "else u = s->P[b++];",
     "else { b++; continue; }"),
    ("relevant() ignores X (non-maximal results)",
     "if (s->np == 0 && s->nx == 0) {",
     "if (s->np == 0) {"),
    ("ties broken by descending ids",
     "return lex_cmp(a, na, b, nb);",
     "return -lex_cmp(a, na, b, nb);"),
    ("colour class bound takes the lightest vertex",
     "if (w > cmax[color[i]]) cmax[color[i]] = w;",
     "if (cmax[color[i]] == 0 || w < cmax[color[i]]) cmax[color[i]] = w;"),
    ("matching ignores labels",
     "if (lab[c] != P.label[a]) continue;",
     "(void)0;"),
    ("matching not injective",
     "if (r->mu[b] == c) ok = 0;",
     "if (0) ok = 0;"),
    ("matching reports every embedding of an image",
     ("if (r->depth == q && match_is_canonical(&P, r->mu)) {",
      "if (!match_may_be_canonical(&P, ch)) { free(ch); continue; }"),
     ("if (r->depth == q) {", "(void)0;")),
    ("matching drops an edge weight from the score",
     "if (w == 0) ok = 0; else add += w;",
     "if (w == 0) ok = 0;"),
    ("matching bound too low for matched edges",
     "if (matched[a] && matched[c]) ub = edge_weight(g, r->mu[a], r->mu[c]);",
     "if (matched[a] && matched[c]) ub = 1;"),
    ("matching bound too low for unmatched edges",
     "else ub = T->pairmax[P->label[a] * T->nl + P->label[c]];",
     "else ub = 1;"),
    ("result set keeps the worse of a new result and the k-th",
     "if (rank_cmp(score, ids, len, kth->score, kth->ids, kth->len) >= 0) return 0;",
     "if (rank_cmp(score, ids, len, kth->score, kth->ids, kth->len) < 0) return 0;"),
    ("greedy colouring ignores adjacency (one colour class)",
     "if (is_adjacent(g, s->P[i], s->P[j])) used[color[j]] = 1;",
     "(void)0;"),
    ("pattern automorphisms ignore labels",
     "if (P->label[perm[a]] != P->label[a]) ok = 0;",
     "(void)0;"),
    ("matching represents an image by its largest tuple",
     ("if (x < mu[i]) return 0;\n      if (x > mu[i]) break;",
      "if (x < r->mu[i]) return 0;\n      if (x > r->mu[i]) break;"),
     ("if (x > mu[i]) return 0;\n      if (x < mu[i]) break;",
      "if (x > r->mu[i]) return 0;\n      if (x < r->mu[i]) break;")),
    ("one-endpoint matching bound looks up the matched vertex's own label",
     "else if (matched[a]) ub = T->best[(uint64_t)r->mu[a] * T->nl + P->label[c]];",
     "else if (matched[a]) ub = T->best[(uint64_t)r->mu[a] * T->nl + P->label[a]];"),
    ("multi-hop index by exact distance, not cumulative",
     "if (layer[(uint64_t)h * nl + l] > run) run = layer[(uint64_t)h * nl + l];",
     "run = layer[(uint64_t)h * nl + l];"),
    ("degree bound without the current score",
     "  int64_t b = r->score;\n  for (uint32_t u = 0; u < P->q; ++u) {",
     "  int64_t b = 0;\n  for (uint32_t u = 0; u < P->q; ++u) {"),
    ("degree bound looks every unmatched vertex up at one hop",
     "hidx[((uint64_t)(P->hop[u] - 1) * g->n + seed) * nl + P->label[u]]",
     "hidx[((uint64_t)0 * g->n + seed) * nl + P->label[u]]"),
    ("degree score adds the anchor's degree, not the candidate's",
     "if (degree) add = degree_of(g, c);",
     "if (degree) add = degree_of(g, av);"),
    ("degree score leaves out the seed",
     "r->score = S->degree ? degree_of(g, v) : 0;",
     "r->score = 0;"),
    ("pattern support takes the largest image count",
     ("if (distinct < f) f = distinct;", "if (S.count[v] < f) f = S.count[v];"),
     ("if (f == UINT64_MAX || distinct > f) f = distinct;",
      "if (f == UINT64_MAX || S.count[v] > f) f = S.count[v];")),
    ("pattern groups pruned at equal support",
     ("if (nr == k && S->f < R[k - 1].f)", "if (nr == k && C->f < R[k - 1].f)"),
     ("if (nr == k && S->f <= R[k - 1].f)", "if (nr == k && C->f <= R[k - 1].f)")),
    ("non-minimal DFS codes kept",
     "if (!pm_is_min(&C->c)) { st_nonmin++; pm_group_free(C); continue; }",
     "(void)0;"),
    ("forward extensions only from the rightmost vertex",
     "for (uint32_t q = 0; q < np; ++q) {\n        uint32_t x = path[q], dx = phi[x];",
     "for (uint32_t q = 0; q < 1; ++q) {\n        uint32_t x = path[q], dx = phi[x];"),
    ("DFS code order prefers the shallower vertex",
     "else { k[0] = 1; k[1] = -(int)e->i; k[2] = e->li; k[3] = e->lj; }",
     "else { k[0] = 1; k[1] = (int)e->i; k[2] = e->li; k[3] = e->lj; }"),
]

MATCH_PATTERNS = [
    ([0, 0], [(0, 1)]),
    ([0, 1, 0], [(0, 1), (1, 2)]),
    ([0, 0, 0], [(0, 1), (1, 2), (0, 2)]),
    ([0, 1, 1, 0], [(0, 1), (1, 2), (2, 3), (0, 2)]),
    ([0, 0, 1, 0, 1], [(0, 1), (1, 2), (2, 3), (3, 4), (0, 2)]),
]


def _battery():
    """Names of the pins that fail for the oracle currently loaded."""
    failed = []
    for n, p, seed in ((8, 0.6, 1), (11, 0.3, 2), (11, 0.6, 3), (13, 0.5, 4), (9, 0.9, 5),
                       (12, 0.45, 6)):
        g = synth.gnp(n, p, seed)
        for w_hi in (3, 100):  # many ties / few ties
            synth.add_vertex_weights(g, 1, w_hi, master=seed)
            for k in (1, 2, 5, 1000):
                want_s = bruteforce.topk_cliques(g, k)
                want_w = bruteforce.topk_cliques(g, k, weights=g.vertex_weight)
                for bound in (0, 1):
                    for xprune in (False, True):
                        got_s, _ = oracle.topk_cliques(g, k, bound=bound, xprune=xprune)
                        if got_s != want_s:
                            failed.append(f"cliques size n={n} k={k} bound={bound}")
                        for priority in (0, 1):
                            got_w, _ = oracle.topk_cliques(g, k, weighted=True, bound=bound,
                                                           priority=priority, xprune=xprune)
                            if got_w != want_w:
                                failed.append(f"cliques weight n={n} k={k} bound={bound}")
    for pi, (labels, edges) in enumerate(MATCH_PATTERNS):
        for seed, w_hi in ((1, 4), (2, 4), (3, 50)):
            g = synth.gnp(9, 0.55, 100 * seed + pi)
            synth.add_zipf_labels(g, n_labels=2, s=0.5, master=100 * seed + pi)
            synth.add_edge_weights(g, 1, w_hi, master=100 * seed + pi)
            for k in (1, 2, 5, 10000):
                want, _ = bruteforce.topk_matches(g, labels, edges, k)
                got, _ = oracle.topk_match(g, labels, edges, k, n_labels=2)
                if got != want:
                    failed.append(f"match pattern {pi} seed {seed} k={k}")
                want, _ = bruteforce.topk_matches(g, labels, edges, k, score="degree")
                got, _ = oracle.topk_match(g, labels, edges, k, n_labels=2, score="degree")
                if got != want:
                    failed.append(f"degree match pattern {pi} seed {seed} k={k}")
    for seed in (1, 2, 3):
        g = synth.gnp(11, 0.35, 80 + seed)
        synth.add_zipf_labels(g, n_labels=seed, s=0.5, master=80 + seed)
        for M in (1, 2, 3):
            want = oracle.topk_patterns_definition(g, M, 10 ** 6)
            for k in (1, 3, 10 ** 6):
                if oracle.topk_patterns(g, M, k)[0] != want[:k]:
                    failed.append(f"patterns seed {seed} M={M} k={k}")
            for f, code in want[:6]:
                if pattern_support_nx(g, code) != f:
                    failed.append(f"pattern support seed {seed} M={M}")
    for seed, M in ((13, 2), (81, 3), (135, 2)):
        g = synth.gnp(8 + seed % 5, 0.4, 1000 + seed)
        synth.add_zipf_labels(g, n_labels=1 + seed % 2, s=0.5, master=1000 + seed)
        want = oracle.topk_patterns_definition(g, M, 10 ** 6)
        for k in (1, 2, 3):
            if oracle.topk_patterns(g, M, k)[0] != want[:k]:
                failed.append(f"pattern ties seed {seed} M={M} k={k}")
    rng = np.random.default_rng(5)
    for _ in range(20):
        nv = int(rng.integers(2, 6))
        ne = int(rng.integers(nv - 1, min(nv * (nv - 1) // 2, 6) + 1))
        labels, edges = random_pattern_graph(rng, nv, ne, 3)
        codes = all_dfs_codes(labels, edges)
        if oracle.min_dfs_code(labels, edges) != min(codes, key=lambda c: [dfs_key(e) for e in c]):
            failed.append("min dfs code")
    for seed in (1, 2):
        g = synth.gnp(40, 0.08, 60 + seed)
        synth.add_zipf_labels(g, n_labels=3, s=0.5, master=60 + seed)
        if not np.array_equal(oracle.hop_index(g, 4, n_labels=3),
                              index_from_distances(g, 4, 3)):
            failed.append(f"hop index seed {seed}")
    return failed


@contextlib.contextmanager
def _oracle_from(so_path):
    saved = oracle._SO, oracle._lib
    oracle._SO, oracle._lib = so_path, None
    try:
        yield
    finally:
        oracle._SO, oracle._lib = saved


def test_real_oracle_passes_the_battery():
    assert _battery() == []


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_fails_the_battery(tmp_path, name, old, new):
    src = open(ORACLE_C).read()
    olds, news = (old, new) if isinstance(old, tuple) else ((old,), (new,))
    for o, n in zip(olds, news):
        assert o in src, f"mutation site not found: {o!r}"
        src = src.replace(o, n)  # the same mistake wherever the code occurs
    mut = tmp_path / "oracle_mutant.c"
    mut.write_text(src)
    so = tmp_path / "liboracle_mutant.so"
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", str(so), str(mut)])
    with _oracle_from(str(so)):
        failed = _battery()
    assert failed, f"no pin catches the mutant: {name}"
