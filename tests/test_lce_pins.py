"""Pins of the oracle's longest common extension (the lcp / lcs queries of the
match-completion step sketched in App. B), no GPU: against an independent
brute force (zip and count) on random position pairs in both directions, and
closed forms (a position against itself, homopolymers, the string end).  The
same for pairs of grammar symbols (App. B's lcp(X, Y) and lcs(X, Y)), with
the symbols expanded by a plain recursion over the exported levels; two C
entries compare like their whole strings.
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


# ---------------------------------------------------- symbol pairs (App. B)
def _expand_py(levels, lv, x, memo):
    """exp of the symbol (lv, x) from the exported level arrays, by plain recursion."""
    if lv == 0:
        return bytes([x])
    key = (lv, x)
    if key not in memo:
        L = levels[lv - 1]
        a, b = int(L["rhs_off"][x]), int(L["rhs_off"][x + 1])
        memo[key] = b"".join(_expand_py(levels, lv - 1, int(y), memo) for y in L["rhs"][a:b])
    return memo[key]


def _symbol_collection(oracle_mod):
    from paper_2411_12439_amd import datagen as D
    rng = np.random.default_rng(13)
    base = D.BASES[rng.integers(0, 4, 3000)]
    cols = [base.copy() for _ in range(4)]
    for c in cols[1:]:
        c[rng.integers(0, 3000, 8)] = D.BASES[rng.integers(0, 4, 8)]
    strings = [c.tobytes() for c in cols] + [b"A" * 500, b"AC" * 200, b"G"]
    return strings, oracle_mod.build_strings(strings, D.HASH_SEED)


@pytest.mark.parametrize("backward", [False, True])
def test_symbol_lce_matches_brute_force(oracle_mod, backward):
    """lcp / lcs of symbol expansions against a plain recursive expansion and
    the zip-and-count brute force, for pairs within a level and across levels."""
    strings, g = _symbol_collection(oracle_mod)
    levels = g.export()["levels"]
    rng = np.random.default_rng(14)
    memo = {}
    nq = 400
    lv1 = rng.integers(0, len(levels) + 1, nq)
    lv2 = np.where(rng.random(nq) < 0.6, lv1, rng.integers(0, len(levels) + 1, nq))
    size = lambda lv: 256 if lv == 0 else len(levels[lv - 1]["fp"])
    s1 = np.array([rng.integers(0, size(v)) for v in lv1])
    s2 = np.array([rng.integers(0, size(v)) for v in lv2])
    got = g.symbol_lce(lv1, s1, lv2, s2, backward)
    for q in range(nq):
        a = _expand_py(levels, int(lv1[q]), int(s1[q]), memo)
        b = _expand_py(levels, int(lv2[q]), int(s2[q]), memo)
        assert got[q] == _lce_brute(a, b, not backward), q
        assert g.expand_symbol(int(lv1[q]), int(s1[q])) == a


def test_symbol_lce_closed_forms(oracle_mod):
    """lcp(X, X) = |X|; two C entries compare like the whole strings; bytes."""
    strings, g = _symbol_collection(oracle_mod)
    e = g.export()
    levels = e["levels"]
    memo = {}
    lv = [1, 2, len(levels)]
    xs = [0, 1, 0]
    got = g.symbol_lce(lv, xs, lv, xs)
    assert got.tolist() == [len(_expand_py(levels, a, b, memo)) for a, b in zip(lv, xs)]
    k = len(strings)
    j1 = np.repeat(np.arange(k), k)
    j2 = np.tile(np.arange(k), k)
    text, off = oracle_mod.pack(strings)
    lens = np.diff(off.astype(np.int64))
    fw = g.symbol_lce(e["c_level"][j1], e["c_sym"][j1], e["c_level"][j2], e["c_sym"][j2])
    assert np.array_equal(fw, oracle_mod.lce(text, off, j1, np.zeros(k * k, np.int64), j2,
                                             np.zeros(k * k, np.int64)))
    bw = g.symbol_lce(e["c_level"][j1], e["c_sym"][j1], e["c_level"][j2], e["c_sym"][j2], True)
    assert np.array_equal(bw, oracle_mod.lce(text, off, j1, lens[j1], j2, lens[j2], True))
    assert g.symbol_lce([0, 0], [65, 65], [0, 0], [65, 67]).tolist() == [1, 0]
    with pytest.raises(ValueError):
        g.symbol_lce([len(levels) + 1], [0], [1], [0])
    with pytest.raises(ValueError):
        g.symbol_lce([1], [len(levels[0]["fp"])], [1], [0])
