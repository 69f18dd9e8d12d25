"""The screening bound the expansion kernel uses for vertex weights, checked
on the CPU (no GPU).

Screening tests each child against w(V) + w(child) + an upper bound of
w(P'), computed without a walk over P''s bits: for each 64-bit word of the
candidate bitmap, the number of P' bits in that word times the heaviest
candidate of the parent's P in that word.  Children that this bound rules
out are counted as pruned before they are built, so the bound must never be
below the exact sum; it is exact when every word's candidates weigh the
same.
"""
import numpy as np


def _words(bits, W):
    out = np.zeros(W, dtype=np.uint64)
    for b in bits:
        out[b >> 6] |= np.uint64(1) << np.uint64(b & 63)
    return out


def _screen_bound(p_words, child_words, weights):
    total = 0
    for w in range(len(p_words)):
        heaviest = max((int(weights[w * 64 + b]) for b in range(64)
                        if int(p_words[w]) >> b & 1), default=0)
        total += bin(int(child_words[w])).count("1") * heaviest
    return total


def test_word_bound_is_an_upper_bound_and_exact_for_equal_weights():
    rng = np.random.default_rng(11)
    for _ in range(400):
        d = int(rng.integers(1, 300))
        W = (d + 63) // 64
        weights = rng.integers(1, 1000, size=W * 64)
        P = sorted(rng.choice(d, size=int(rng.integers(1, d + 1)), replace=False).tolist())
        child = [v for v in P if rng.random() < 0.5]  # P' is a subset of P
        exact = int(sum(int(weights[v]) for v in child))
        bound = _screen_bound(_words(P, W), _words(child, W), weights)
        assert bound >= exact
        same = np.repeat(rng.integers(1, 1000, size=W), 64)
        assert _screen_bound(_words(P, W), _words(child, W), same) == \
            int(sum(int(same[v]) for v in child))
