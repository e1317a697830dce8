"""Pins of the oracle's longest common extension (the lcp / lcs queries of the
match-completion step sketched in App. B), no GPU: against an independent
brute force (zip and count) on random position pairs in both directions, and
closed forms (a position against itself, homopolymers, the string end).
"""
import numpy as np
import pytest


def _lce_brute(a, b, forward):
    """Independent of the oracle: zip the two sides and count equal pairs up to the first
    difference (reversed prefixes for the backward direction)."""
    if not forward:
        a, b = a[::-1], b[::-1]
    n = 0
    for x, y in zip(a, b):
        if x != y:
            break
        n += 1
    return n


@pytest.mark.parametrize("backward", [False, True])
def test_lce_matches_brute_force(oracle_mod, backward):
    rng = np.random.default_rng(12)
    base = bytes(rng.choice(list(b"ACGT"), 400).astype(np.uint8))
    strings = [base, base[:200] + b"T" + base[201:], base[50:], b"A" * 300, b"A" * 120 + b"C",
               b"G", base[::-1]]
    text, off = oracle_mod.pack(strings)
    o = off.astype(np.int64)
    nq = 600
    j1 = rng.integers(0, len(strings), nq)
    j2 = rng.integers(0, len(strings), nq)
    p1 = np.array([rng.integers(0, o[j + 1] - o[j] + 1) for j in j1])
    p2 = np.array([rng.integers(0, o[j + 1] - o[j] + 1) for j in j2])
    got = oracle_mod.lce(text, off, j1, p1, j2, p2, backward)
    for q in range(nq):
        a = strings[j1[q]]
        b = strings[j2[q]]
        want = _lce_brute(a[p1[q]:], b[p2[q]:], True) if not backward else \
            _lce_brute(a[:p1[q]], b[:p2[q]], False)
        assert got[q] == want, (q, j1[q], p1[q], j2[q], p2[q])


def test_lce_closed_forms(oracle_mod):
    """A position against itself extends to the string's end (start, backward);
    two homopolymers extend to the shorter remainder."""
    strings = [b"ACGTTGCA" * 10, b"A" * 50, b"A" * 70]
    text, off = oracle_mod.pack(strings)
    n0 = len(strings[0])
    assert oracle_mod.lce(text, off, [0], [5], [0], [5]).tolist() == [n0 - 5]
    assert oracle_mod.lce(text, off, [0], [5], [0], [5], backward=True).tolist() == [5]
    assert oracle_mod.lce(text, off, [1], [10], [2], [0]).tolist() == [40]
    assert oracle_mod.lce(text, off, [1], [50], [2], [70], backward=True).tolist() == [50]
    assert oracle_mod.lce(text, off, [0], [n0], [0], [0]).tolist() == [0]
