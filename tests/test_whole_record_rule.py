"""The decisions the expansion kernel takes on a "whole" record, checked by
brute force on small candidate sets (no GPU).

A whole record has candidate set P and at most one candidate may be left out
(slack 1), so its subtree can only yield V + P (P a clique) or V + P - {x}
(P - {x} a clique).  For each candidate the kernel counts its misses (the
other candidates it is not adjacent to), i.e. its degree in the complement
of P, and decides from the counts alone:
  * P - {x} is a clique for some x exactly when the complement's edges form a
    star (one edge, or all edges sharing one vertex): sum of misses / 2 ==
    largest miss count;
  * two candidates with two or more misses each already rule out every x, so
    the pass over the candidates' rows may stop as soon as it has seen two.
"""
import itertools

import numpy as np
import pytest


def _complement_degrees(n, missing):
    deg = [0] * n
    for a, b in missing:
        deg[a] += 1
        deg[b] += 1
    return deg


def _some_x_leaves_a_clique(n, missing):
    return any(all(x in e for e in missing) for x in range(n))


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_star_rule_and_early_stop_over_all_small_complements(n):
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        missing = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
        deg = _complement_degrees(n, missing)
        some_x = _some_x_leaves_a_clique(n, missing)
        if missing:
            # the kernel's test once every row has been read
            assert (sum(deg) // 2 == max(deg)) == some_x, missing
        # the early stop: two candidates with two or more misses
        if sum(d >= 2 for d in deg) >= 2:
            assert not some_x and missing, missing


def test_early_stop_holds_on_any_prefix_of_the_candidates():
    """The kernel counts misses per candidate over whole rows but sees the
    candidates in rounds; stopping after any round in which two candidates
    with two or more misses have appeared is safe whatever the later rounds
    hold."""
    rng = np.random.default_rng(5)
    for _ in range(300):
        n = int(rng.integers(4, 12))
        missing = [p for p in itertools.combinations(range(n), 2) if rng.random() < 0.2]
        deg = _complement_degrees(n, missing)
        order = rng.permutation(n)
        seen = 0
        for v in order:
            seen += deg[v] >= 2
            if seen >= 2:
                assert not _some_x_leaves_a_clique(n, missing)
                break
