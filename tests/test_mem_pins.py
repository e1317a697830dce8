"""Pins of the oracle's maximal exact matches through the grammar (App. B's
MEM sketch), no GPU.

The ground truth is an independent brute force on the bytes: on every
diagonal of the two strings (start in b minus start in a), the maximal runs of
equal bytes.  The oracle's answer must be exactly the runs of at least
min_len bytes that hold the first byte of an anchor -- a pair of equal symbols
of the two strings' level-l parses on that diagonal -- with the parses taken
from the exported levels by a plain substitution written here.  A wrong
extension (an off-by-one before the anchor, a missing forward part), a match
seeded on the wrong diagonal or a dropped anchor fails the comparison.  On
mutated copies of one sequence every run of 64 bytes or more holds an anchor
at level 1 (local consistency: the phrases inside a long match are parsed
alike), so there the oracle finds all the brute-force matches.
"""
import numpy as np
import pytest


def _runs(a, b, same):
    """{diagonal d: [(start in a, length), ...]} of all maximal runs of equal
    bytes a[i] == b[i + d]; the main diagonal is left out when a is b."""
    A = np.frombuffer(a, np.uint8)
    B = np.frombuffer(b, np.uint8)
    out = {}
    for d in range(-(len(A) - 1), len(B)):
        if same and d == 0:
            continue
        lo = max(0, -d)
        hi = min(len(A), len(B) - d)
        if hi <= lo:
            continue
        eq = A[lo:hi] == B[lo + d:hi + d]
        runs = []
        i = 0
        n = len(eq)
        while i < n:
            if eq[i]:
                j = i
                while j < n and eq[j]:
                    j += 1
                runs.append((lo + i, j - i))
                i = j
            else:
                i += 1
        out[d] = runs
    return out


def _parse(ex, j, level):
    """Level-`level` symbols of string j and the byte offset of each."""
    levels = ex["levels"]
    cur = [int(ex["c_sym"][j])]
    for lv in range(int(ex["c_level"][j]), level, -1):
        L = levels[lv - 1]
        cur = [int(c) for x in cur for c in L["rhs"][L["rhs_off"][x]:L["rhs_off"][x + 1]]]
    memo = {}

    def elen(lv, x):
        if lv == 0:
            return 1
        if (lv, x) not in memo:
            L = levels[lv - 1]
            memo[(lv, x)] = sum(elen(lv - 1, int(c))
                                for c in L["rhs"][L["rhs_off"][x]:L["rhs_off"][x + 1]])
        return memo[(lv, x)]

    starts = np.concatenate([[0], np.cumsum([elen(level, x) for x in cur])])
    return cur, starts


def _expected(ex, strings, a, b, level, min_len):
    A, xa = _parse(ex, a, level)
    B, xb = _parse(ex, b, level)
    runs = _runs(strings[a], strings[b], a == b)
    want = set()
    for i, s in enumerate(A):
        for j, t in enumerate(B):
            if s != t or (a == b and i == j):
                continue
            d = int(xb[j]) - int(xa[i])
            for st, n in runs.get(d, []):
                if st <= xa[i] < st + n:
                    if n >= min_len:
                        want.add((st, st + d, n))
                    break
            else:
                raise AssertionError("the anchor's first bytes differ: %d %d" % (i, j))
    return sorted(want), runs


def _collection(seed):
    rng = np.random.default_rng(seed)
    base = bytearray(rng.choice(list(b"ACGT"), 700).astype(np.uint8).tobytes())
    strings = [bytes(base)]
    for _ in range(3):
        s = bytearray(base)
        for _ in range(7):  # substitutions, about 1 %
            p = int(rng.integers(0, len(s)))
            s[p] = int(rng.choice([c for c in b"ACGT" if c != s[p]]))
        p = int(rng.integers(0, len(s) - 10))
        del s[p:p + int(rng.integers(1, 4))]  # a short deletion
        strings.append(bytes(s))
    rep = bytes(base[100:220])
    strings.append(bytes(base[:300]) + rep + b"A" * 60 + rep + bytes(base[500:]))
    strings.append(b"CA" * 40 + bytes(base[200:260]))
    return strings


@pytest.mark.parametrize("seed", [3, 4])
def test_mems_equal_anchored_brute_force_runs(oracle_mod, seed):
    strings = _collection(seed)
    text, off = oracle_mod.pack(strings)
    g = oracle_mod.build(text, off, 97 + seed)
    ex = g.export()
    top = min(int(x) for x in ex["c_level"])
    pairs = [(0, 1), (1, 2), (2, 0), (4, 4), (0, 4), (5, 3), (3, 3)]
    for a, b in pairs:
        for level in sorted({1, 2, top}):
            for min_len in (1, 12, 40):
                want, _ = _expected(ex, strings, a, b, level, min_len)
                pa, pb, ln = g.mems(text, off, a, b, level, min_len)
                got = list(zip(pa.tolist(), pb.tolist(), ln.tolist()))
                assert got == want, (a, b, level, min_len)


def test_long_matches_are_all_found_at_level_one(oracle_mod):
    strings = _collection(5)
    text, off = oracle_mod.pack(strings)
    g = oracle_mod.build(text, off, 11)
    for a, b in [(0, 1), (1, 2), (3, 0), (4, 4)]:
        runs = _runs(strings[a], strings[b], a == b)
        brute = sorted((st, st + d, n) for d, rs in runs.items() for st, n in rs if n >= 64)
        pa, pb, ln = g.mems(text, off, a, b, 1, 64)
        assert list(zip(pa.tolist(), pb.tolist(), ln.tolist())) == brute, (a, b)


def test_repeat_inside_one_string(oracle_mod):
    """X Z X against itself: the two copies of X (extended by what else agrees)
    match each other, in both orders, and nothing lies on the main diagonal."""
    rng = np.random.default_rng(8)
    x = rng.choice(list(b"ACGT"), 150).astype(np.uint8).tobytes()
    z = rng.choice(list(b"ACGT"), 70).astype(np.uint8).tobytes()
    s = x + z + x
    text, off = oracle_mod.pack([s, x])
    g = oracle_mod.build(text, off, 5)
    pa, pb, ln = g.mems(text, off, 0, 0, 1, 100)
    got = list(zip(pa.tolist(), pb.tolist(), ln.tolist()))
    assert len(got) == 2
    (p, q, n), (p2, q2, n2) = got
    assert (p, q) == (q2, p2) and n == n2 and n >= 150 and q - p == 220
    assert s[p:p + n] == s[q:q + n]
    # X against X Z X: both copies
    pa, pb, ln = g.mems(text, off, 1, 0, 1, 150)
    got = list(zip(pa.tolist(), pb.tolist(), ln.tolist()))
    assert [(t[0], t[1]) for t in got] == [(0, 0), (0, 220)]
    assert all(t[2] == 150 for t in got)


def test_no_match_is_long_enough(oracle_mod):
    strings = _collection(6)
    text, off = oracle_mod.pack(strings)
    g = oracle_mod.build(text, off, 3)
    pa, pb, ln = g.mems(text, off, 0, 5, 1, 10 ** 6)
    assert len(pa) == 0


def test_bad_arguments(oracle_mod):
    strings = _collection(7)
    text, off = oracle_mod.pack(strings)
    g = oracle_mod.build(text, off, 3)
    ex = g.export()
    with pytest.raises(ValueError):
        g.mems(text, off, 0, len(strings), 1, 1)
    with pytest.raises(ValueError):
        g.mems(text, off, 0, 1, 0, 1)
    with pytest.raises(ValueError):
        g.mems(text, off, 0, 1, int(min(ex["c_level"][0], ex["c_level"][1])) + 1, 1)
