"""Pins of the CPU oracle against what the paper and mathematics fix (no GPU).

Each test names the passage it follows.  A plausible slip in the oracle -- a
dropped hash term, a wrong coefficient power, a type computed from the left
neighbour, a break on the wrong side of a run, a missing remap in the merge,
a wrong expansion order -- fails at least one of these.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import brute
from paper_2411_12439_amd import canon as CN
from paper_2411_12439_amd import datagen as D

SEED = D.HASH_SEED
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_strings(rng, k, lo, hi, alphabet=b"ACGT"):
    alpha = np.frombuffer(alphabet, np.uint8)
    return [alpha[rng.integers(0, len(alpha), int(rng.integers(lo, hi + 1)))].tobytes()
            for _ in range(k)]


# ---------------------------------------------------------------- hash family
def test_hash_family_matches_independent_splitmix(oracle_mod):
    """Sec. 3.2 coefficients: both sides draw from SplitMix64, reduce mod p, skip zeros."""
    for seed in (0, 1, SEED, 2**64 - 1):
        a, b, c = oracle_mod.hash_params(seed)
        fam = brute.hash_family(seed)
        for i in range(64):
            assert (int(a[i]), int(b[i]), int(c[i])) == fam[i]
            assert 0 < fam[i][0] < brute.P and 0 < fam[i][1] < brute.P and 0 < fam[i][2] < brute.P


def test_level_fingerprints_follow_eq4(oracle_mod):
    """Eq. 4: F[X] = ((a_i sum_j F[Q_j] c_i^(j-1) + b_i) mod p) mod 2^32 for every stored rule."""
    text, off = D.make_config("tiny", scale=0.05)
    g = oracle_mod.build(text, off, SEED).export()
    fam = brute.hash_family(SEED)
    prev = [brute.h0(fam, s) for s in range(256)]
    for i, L in enumerate(g["levels"], start=1):
        offs = L["rhs_off"].astype(np.int64)
        for r in range(len(L["fp"])):
            q = L["rhs"][offs[r]:offs[r + 1]].tolist()
            assert int(L["fp"][r]) == brute.poly_key(fam, i, [prev[x] for x in q]) % 2**32
        prev = L["fp"].tolist()


def test_fingerprint_depends_only_on_expansion(oracle_mod):
    """Sec. 3.2: h^i depends on exp(X) and the parse-tree topology, not on names.

    The same string inside two different collections gets rules whose
    fingerprints coincide, although their ranks differ.
    """
    rng = np.random.default_rng(5)
    s = _rand_strings(rng, 1, 3000, 3000)[0]
    g1 = oracle_mod.build_strings([s], SEED).export()
    g2 = oracle_mod.build_strings(_rand_strings(rng, 3, 500, 2000) + [s], SEED).export()
    sub = CN.subgrammar(g2, [3])
    assert CN.canon(sub) == CN.canon(g1)
    f1 = sorted(int(x) for L in g1["levels"] for x in L["fp"])
    f2 = sorted(int(x) for L in sub["levels"] for x in L["fp"])
    assert f1 == f2


# --------------------------------------------------------- brute force (P2)
def _compare_with_brute(oracle_mod, strings, seed):
    got = oracle_mod.build_strings(strings, seed).export()
    want = brute.to_export(*brute.build(strings, seed), seed)
    assert CN.exports_equal(got, want), CN.first_difference(got, want)


def test_brute_force_exhaustive_dna_up_to_8(oracle_mod):
    """Eq. 3 + phrase rule + dedup, on every string over {A,C,G,T} of length 1..8."""
    strings = [bytes(t) for L in range(1, 9) for t in itertools.product(b"ACGT", repeat=L)]
    _compare_with_brute(oracle_mod, strings, SEED)


@pytest.mark.parametrize("seed", [1, 58, 977])
def test_brute_force_binary_alphabet(oracle_mod, seed):
    """Many equal runs: random strings over {A, C} up to length 64."""
    rng = np.random.default_rng(seed)
    _compare_with_brute(oracle_mod, _rand_strings(rng, 300, 1, 64, b"AC"), seed)


def test_brute_force_mutated_copies(oracle_mod):
    """Deep rounds with repeated phrases: mutated copies of a 600-symbol base."""
    rng = np.random.default_rng(11)
    base = _rand_strings(rng, 1, 600, 600)[0]
    strings = []
    for _ in range(6):
        b = bytearray(base)
        for p in rng.integers(0, len(b), 5):
            b[p] = b"ACGT"[int(rng.integers(0, 4))]
        strings.append(bytes(b))
    _compare_with_brute(oracle_mod, strings + [b"A" * 300, b"AC" * 200, b"ACGTTGCA" * 30], SEED)


def test_brute_force_full_byte_alphabet(oracle_mod):
    rng = np.random.default_rng(3)
    strings = [rng.integers(0, 256, int(rng.integers(1, 200)), dtype=np.uint8).tobytes()
               for _ in range(100)]
    _compare_with_brute(oracle_mod, strings, 12345)


# ------------------------------------------------------------ round trip (P1)
def test_round_trip_tiny_config(oracle_mod):
    """Straight-line grammar (Sec. 2.2): exp(C[j]) = T_j for every string."""
    text, off = D.make_config("tiny")
    g = oracle_mod.build(text, off, SEED)
    for j in range(len(off) - 1):
        assert g.expand(j) == text[off[j]:off[j + 1]].tobytes()


def test_round_trip_odd_collections(oracle_mod):
    strings = [b"A", b"AA", b"AC", b"CA", b"A" * 10000, b"ACGT" * 2500, b"T", b"GATTACA" * 77]
    g = oracle_mod.build_strings(strings, SEED)
    for j, s in enumerate(strings):
        assert g.expand(j) == s


# -------------------------------------------------------------- stability (P3)
def test_merge_equals_build_of_concatenation_every_split(oracle_mod):
    """Sec. 3.5: MergeGrams(G_a, G_b) is equivalent to BuildGram(T_a o T_b).

    Merge appends G_b's new rules in G_b's order, which keeps first-occurrence
    ranks, so the equality is exact without renaming.
    """
    rng = np.random.default_rng(7)
    base = _rand_strings(rng, 1, 2000, 2000)[0]
    strings = []
    for j in range(9):
        b = bytearray(base[int(rng.integers(0, 300)):])
        for p in rng.integers(0, len(b), 20):
            b[p] = b"ACGT"[int(rng.integers(0, 4))]
        strings.append(bytes(b) if j % 4 else _rand_strings(rng, 1, 1, 700)[0])
    whole = oracle_mod.build_strings(strings, SEED).export()
    for cut in range(1, len(strings)):
        ga = oracle_mod.build_strings(strings[:cut], SEED)
        gb = oracle_mod.build_strings(strings[cut:], SEED)
        merged = ga.merge(gb).export()
        assert CN.exports_equal(merged, whole), (cut, CN.first_difference(merged, whole))


def test_merge_of_singletons_in_any_tree_order(oracle_mod):
    """Merging per-string grammars pairwise (tree order) gives the same rule sets."""
    rng = np.random.default_rng(8)
    strings = _rand_strings(rng, 8, 100, 900)
    strings += [s[10:] + s[:10] for s in strings[:4]]
    whole = oracle_mod.build_strings(strings, SEED).export()
    gs = [oracle_mod.build_strings([s], SEED) for s in strings]
    while len(gs) > 1:
        nxt = []
        for i in range(0, len(gs), 2):
            nxt.append(gs[i].merge(gs[i + 1]) if i + 1 < len(gs) else gs[i])
        gs = nxt
    assert CN.exports_equal(gs[0].export(), whole)


def test_permutation_gives_canon_equal_rules(oracle_mod):
    rng = np.random.default_rng(9)
    strings = _rand_strings(rng, 10, 50, 500)
    perm = rng.permutation(len(strings))
    g1 = oracle_mod.build_strings(strings, SEED).export()
    g2 = oracle_mod.build_strings([strings[p] for p in perm], SEED).export()
    inv = np.argsort(perm)
    g2p = dict(g2)
    g2p["c_level"] = g2["c_level"][inv]
    g2p["c_sym"] = g2["c_sym"][inv]
    assert CN.canon(g1) == CN.canon(g2p)


def test_context_independence(oracle_mod):
    """Def. 1: the sub-grammar of T_j inside BuildGram(T) equals BuildGram({T_j})."""
    text, off = D.make_config("tiny", scale=0.1)
    whole = oracle_mod.build(text, off, SEED).export()
    for j in range(len(off) - 1):
        alone = oracle_mod.build(text[off[j]:off[j + 1]], np.array([0, off[j + 1] - off[j]],
                                                                   np.uint64), SEED).export()
        assert CN.canon(CN.subgrammar(whole, [j])) == CN.canon(alone)


# ------------------------------------------------------ worked example (P4)
def _find_seed(pred, limit=100000):
    for s in range(limit):
        fam = brute.hash_family(s, 1)
        F = {ch: brute.h0(fam, ord(ch)) for ch in "acgt"}
        if pred(F):
            return s
    raise AssertionError("no seed")


def test_worked_example_round1_parse(oracle_mod):
    """Fig. merge_gram / build_gram: round-1 phrases of T_a and T_b."""
    fx = json.load(open(os.path.join(GOLDEN, "merge_figure.json")))
    seed = _find_seed(lambda F: F["a"] < F["t"] < F["g"] and F["t"] < F["c"])
    for T, want in ((fx["T_a"], fx["round1_phrases_a"]), (fx["T_b"], fx["round1_phrases_b"])):
        brk = oracle_mod.round1_breaks(T, seed)
        starts = list(np.nonzero(brk)[0]) + [len(T)]
        got = [T[starts[i]:starts[i + 1]] for i in range(len(starts) - 1)]
        assert got == want
    # level 1 of both grammars holds exactly the figure's distinct phrases
    for T, L1 in ((fx["T_a"], fx["G_a_level1"]), (fx["T_b"], fx["G_b_level1"])):
        e = oracle_mod.build_strings([T], seed).export()["levels"][0]
        offs = e["rhs_off"].astype(np.int64)
        got = {bytes(e["rhs"][offs[r]:offs[r + 1]].astype(np.uint8)).decode()
               for r in range(len(e["fp"]))}
        assert got == set(L1)


def _level(rules):
    off = np.zeros(len(rules) + 1, np.uint64)
    off[1:] = np.cumsum([len(r) for r in rules])
    rhs = np.array([x for r in rules for x in r], np.uint32)
    return {"rhs_off": off, "rhs": rhs, "fp": np.arange(len(rules), dtype=np.uint32)}


def test_worked_example_merge(oracle_mod):
    """Fig. merge_gram caption: agg is matched, tc becomes symbol 6, and G_b's level-2
    rules 1 -> 1 1 4 3 1, 2 -> 5 2 4 become 1 -> 2 2 3 4 2, 2 -> 1 6 3."""
    fx = json.load(open(os.path.join(GOLDEN, "merge_figure.json")))
    enc = lambda words: [[ord(ch) for ch in w] for w in words]
    dec = lambda rules: [[x - 1 for x in r] for r in rules]  # 1-based -> 0-based ranks
    ga = oracle_mod.from_arrays(
        7, [_level(enc(fx["G_a_level1"])), _level(dec(fx["G_a_level2_completion"])),
            _level([[0, 1]])], np.array([3], np.uint8), np.array([0], np.uint32))
    gb = oracle_mod.from_arrays(
        7, [_level(enc(fx["G_b_level1"])), _level(dec(fx["G_b_level2_printed"])),
            _level([[0, 1]])], np.array([3], np.uint8), np.array([0], np.uint32))
    m = ga.merge(gb).export()
    L1 = m["levels"][0]
    o1 = L1["rhs_off"].astype(np.int64)
    words = [bytes(L1["rhs"][o1[r]:o1[r + 1]].astype(np.uint8)).decode() for r in range(len(L1["fp"]))]
    new = fx["new_level1_symbol_printed"]
    assert words[:5] == fx["G_a_level1"] and len(words) == 6
    assert words[new["symbol"] - 1] == new["rhs"]
    L2 = m["levels"][1]
    o2 = L2["rhs_off"].astype(np.int64)
    rules2 = [(L2["rhs"][o2[r]:o2[r + 1]] + 1).tolist() for r in range(len(L2["fp"]))]
    after = fx["G_b_level2_after_merge_printed"]
    assert rules2[0] == after[0]          # matched the existing rule of G_a
    assert rules2[2] == after[1]          # appended as a new level-2 rule
    assert len(rules2) == 3
    assert ga.expand(1) == fx["T_b"].encode()
    assert ga.expand(0) == b"".join(w.encode() for w in fx["round1_phrases_a"])


# ---------------------------------------------------- textbook case (P5)
def _sais_lms(s):
    """Classic SA-IS types (Nong, Zhang, Chan) with a sentinel smaller than every symbol."""
    n = len(s)
    t = [None] * (n + 1)
    t[n] = "S"
    for i in range(n - 1, -1, -1):
        if i == n - 1:
            t[i] = "L"
        elif s[i] < s[i + 1]:
            t[i] = "S"
        elif s[i] > s[i + 1]:
            t[i] = "L"
        else:
            t[i] = t[i + 1]
    return {i for i in range(1, n) if t[i] == "S" and t[i - 1] == "L"}


def test_round1_breaks_equal_textbook_lms_for_order_preserving_h0(oracle_mod):
    """Eq. 1 vs Eq. 3: with h^0 increasing on the alphabet, RandLMSPar's round-1
    breaks are the LMS positions of the raw bytes (sentinel dropped)."""
    seed = _find_seed(lambda F: F["a"] < F["c"] < F["g"] < F["t"])
    rng = np.random.default_rng(seed)
    for _ in range(200):
        s = bytes(b"acgt"[i] for i in rng.integers(0, 4, int(rng.integers(1, 80))))
        brk = oracle_mod.round1_breaks(s, seed)
        assert brk[0] == 1
        assert set(np.nonzero(brk[1:])[0] + 1) == _sais_lms(s)


# --------------------------------------------------------- closed forms (P6)
@pytest.mark.parametrize("n", [2, 3, 17, 10000])
def test_homopolymer_is_one_rule(oracle_mod, n):
    g = oracle_mod.build_strings([b"G" * n], SEED).export()
    assert len(g["levels"]) == 1
    assert g["levels"][0]["rhs"].tolist() == [ord("G")] * n
    assert g["c_level"].tolist() == [1] and g["c_sym"].tolist() == [0]


def test_monotone_and_two_symbol_strings_are_one_phrase(oracle_mod):
    fam = brute.hash_family(SEED, 1)
    order = sorted(range(256), key=lambda s: brute.h0(fam, s))
    inc = bytes(order[:50])
    dec = bytes(order[:50][::-1])
    for s in (inc, dec, b"AC", b"CA", b"AA"):
        g = oracle_mod.build_strings([s], SEED).export()
        assert len(g["levels"]) == 1 and len(g["levels"][0]["fp"]) == 1


def test_single_symbol_strings_stay_at_level_zero(oracle_mod):
    g = oracle_mod.build_strings([b"x", b"y", b"xy"], SEED).export()
    assert g["c_level"].tolist() == [0, 0, 1]
    assert g["c_sym"].tolist()[:2] == [ord("x"), ord("y")]


def test_rejects_empty_inputs(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.build_strings([b"ab", b""], SEED)
    with pytest.raises(ValueError):
        oracle_mod.build(np.zeros(0, np.uint8), np.zeros(1, np.uint64), SEED)
    ga = oracle_mod.build_strings([b"abc"], 1)
    gb = oracle_mod.build_strings([b"abc"], 2)
    with pytest.raises(ValueError):
        ga.merge(gb)


# ----------------------------------------------------------- invariants (P7)
def test_structural_invariants(oracle_mod):
    text, off = D.make_config("tiny", scale=0.25)
    g = oracle_mod.build(text, off, SEED)
    e = g.export()
    st = g.stats()
    lens = np.diff(off.astype(np.int64))
    # Theorem 1 proof: phrases have length >= 2 except possibly the first
    active_in = int((lens >= 2).sum())
    for r in range(len(st)):
        n_in, d, u, q, act = (int(x) for x in st[r])
        assert 2 * d <= n_in + active_in
        active_in = act
    # O(log n) rounds: at most ceil(log2 n_max) + 1
    assert len(e["levels"]) <= math.ceil(math.log2(int(lens.max()))) + 1
    prev_u = 256
    for L in e["levels"]:
        # fully balanced (Sec. 3.1): level-i rhs are over V^{i-1}
        assert int(L["rhs"].max()) < prev_u
        # rhs distinct within a level
        offs = L["rhs_off"].astype(np.int64)
        seqs = {tuple(L["rhs"][offs[r]:offs[r + 1]].tolist()) for r in range(len(L["fp"]))}
        assert len(seqs) == len(L["fp"])
        prev_u = len(L["fp"])
    # every rule is reachable from C
    sub = CN.subgrammar(e, range(len(off) - 1))
    assert [len(L["fp"]) for L in sub["levels"]] == [len(L["fp"]) for L in e["levels"]]


# ----------------------------------------------------------- statistics (P8)
def test_round1_density_iid_dna(oracle_mod):
    """LMS density for iid uniform DNA with an injective h^0: sum_v (4-v)^2/48 = 14/48."""
    rng = np.random.default_rng(2)
    s = D.BASES[rng.integers(0, 4, 1 << 20)]
    brk = oracle_mod.round1_breaks(s, SEED)
    assert abs(brk.mean() - 14 / 48) < 0.005


def _level_sequences(e, j):
    """T^{i+1}_j for i = lv .. 1 (the sequence of level-i symbols of string j),
    rebuilt from the exported grammar alone: [C[j]] at its level, each level
    expanded by the right-hand sides of the level above."""
    lv = int(e["c_level"][j])
    seqs = {}
    if lv == 0:
        return lv, seqs
    cur = np.array([int(e["c_sym"][j])], np.int64)
    for i in range(lv, 0, -1):
        seqs[i + 1] = cur
        L = e["levels"][i - 1]
        off = np.asarray(L["rhs_off"], np.int64)
        rhs = np.asarray(L["rhs"], np.int64)
        parts = [rhs[off[r]:off[r + 1]] for r in cur.tolist()]
        cur = np.concatenate(parts)
    seqs[1] = cur
    return lv, seqs


@pytest.mark.parametrize("which", ["tiny", "mixed", "runs"])
def test_round_counters_follow_from_the_grammar(oracle_mod, which):
    """The oracle's per-round counters (n_i, d_i, u_i, Q_i, strings still active)
    are not read from its own loop here: they are recomputed from the exported
    grammar.  A string whose C entry sits at level lv takes part in rounds
    1..lv; in round i it enters as T^i_j and leaves as T^{i+1}_j, the
    sequence of its level-i symbols (Sec. 3.3), so n_i and d_i are sums of
    those lengths; every rule of a level is new in a single build (u_i, Q_i =
    the level's size); and d_i = n_{i+1} + the strings that become inactive."""
    O = oracle_mod
    rng = np.random.default_rng(11)
    if which == "tiny":
        text, off = D.make_config("tiny", scale=0.1)
        strings = [text[off[j]:off[j + 1]].tobytes() for j in range(len(off) - 1)]
    elif which == "mixed":
        strings = [bytes(rng.choice(list(b"ACGT"), int(n)).tolist())
                   for n in rng.integers(1, 3000, 12)] + [b"A", b"GG", b"ACGTTGCA" * 40]
    else:
        strings = [b"A" * 700, b"AC" * 300 + b"G" * 50, b"TTTTGTTTT" * 40, b"C"]
    text, off = O.pack(strings)
    g = O.build(text, off, SEED)
    st = g.stats().astype(np.int64)
    e = g.export()
    k = len(strings)
    per = [_level_sequences(e, j) for j in range(k)]
    rounds = max(lv for lv, _ in per)
    assert st.shape[0] == rounds
    for i in range(1, rounds + 1):
        part = [seqs for lv, seqs in per if lv >= i]
        n_i = sum(len(s[i]) for s in part)
        d_i = sum(len(s[i + 1]) for s in part)
        still = sum(1 for lv, _ in per if lv > i)
        L = e["levels"][i - 1]
        assert st[i - 1, 0] == n_i, (i, "n")
        assert st[i - 1, 1] == d_i, (i, "d")
        assert st[i - 1, 2] == len(L["fp"]), (i, "u")
        assert st[i - 1, 3] == len(L["rhs"]), (i, "Q")
        assert st[i - 1, 4] == still, (i, "active")
        if i < rounds:
            became_one = sum(1 for lv, _ in per if lv == i)
            assert st[i - 1, 1] == st[i, 0] + became_one
    # the input level: T^1_j is the string itself
    for j, (lv, seqs) in enumerate(per):
        if lv:
            assert bytes(seqs[1].astype(np.uint8).tolist()) == strings[j]


def test_own_order_subgrammar_equals_the_string_built_alone(oracle_mod):
    """The renaming used for whole-genome comparisons: a string's rules inside
    a collection, renumbered in its own first-occurrence order, equal the
    oracle's grammar of that string alone, rank for rank (stability, Def. 1),
    and agree with the canonical comparison."""
    O = oracle_mod
    rng = np.random.default_rng(3)
    text, off = D.make_config("bacterial", scale=0.004)
    strings = [text[off[j]:off[j + 1]].tobytes() for j in range(len(off) - 1)]
    strings += [b"A", b"ACGT" * 50, b"G" * 300]
    t, o = O.pack(strings)
    e = O.build(t, o, SEED).export()
    for j in list(range(len(strings))):
        alone = O.build(*O.pack([strings[j]]), SEED).export()
        mine = CN.own_order_subgrammar(e, j)
        assert CN.exports_equal(mine, alone), (j, CN.first_difference(mine, alone))
        assert CN.canon(CN.subgrammar(e, [j])) == CN.canon(alone)
    # a wrong order (the collection's own ranks kept) is not accepted
    j = len(strings) - 4
    sub = CN.subgrammar(e, [j])
    alone = O.build(*O.pack([strings[j]]), SEED).export()
    assert not CN.exports_equal(sub, alone)
