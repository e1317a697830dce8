"""Pins of the oracle's post-processing, RL and Simp (Sec. 2.2, post-processing
paragraph; applied RL first, then Simp, Sec. 4).  No GPU.

What fixes the result: the hand-derived example in
``golden/postprocess_example.json``, the closed form of a homopolymer, the
round trip exp(C[j]) = T_j, RL's defining properties, Simp computed by an
independent one-rule-at-a-time fixpoint (``brute_post.py``) and the size
identity of Simp.  A dropped run, a run split at a rule boundary, a wrong
run-rule order, a rule removed although C or a run rule holds it, a missed
recursive splice or a wrong renumbering fails one of them.
"""
import json
import os

import numpy as np
import pytest

import brute_post as BP
from paper_2411_12439_amd import datagen as D

SEED = D.HASH_SEED
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
FLAGS = {"rl": (True, False), "simp": (False, True), "rl_simp": (True, True)}


def _level(rules):
    off = np.zeros(len(rules) + 1, np.uint64)
    off[1:] = np.cumsum([len(r) for r in rules])
    rhs = np.array([x for r in rules for x in r], np.uint32)
    return {"rhs_off": off, "rhs": rhs, "fp": np.arange(len(rules), dtype=np.uint32)}


def _golden_grammar(oracle_mod, fx):
    levels = [_level(rules) for rules in fx["levels"]]
    cl = np.array([lv for lv, _ in fx["c"]], np.uint8)
    cs = np.array([s for _, s in fx["c"]], np.uint32)
    return oracle_mod.from_arrays(SEED, levels, cl, cs)


@pytest.mark.parametrize("which", sorted(FLAGS))
def test_golden_example(oracle_mod, which):
    """The hand-derived example: rules, C and the size statistics."""
    fx = json.load(open(os.path.join(GOLDEN, "postprocess_example.json")))
    g = _golden_grammar(oracle_mod, fx)
    rl, simp = FLAGS[which]
    got = g.postprocess(rl=rl, simp=simp, expand=True)
    want = BP.from_rules(fx[which]["rules"], fx[which]["c"])
    assert BP.rules_of(got) == want["rules"]
    assert got["c"].tolist() == want["c"]
    assert got["stats"].tolist() == fx[which]["stats"]
    assert got["expansions"] == [s.encode() for s in fx["strings"]]


@pytest.mark.parametrize("n", [2, 3, 1000])
def test_homopolymer_closed_form(oracle_mod, n):
    """s^n is one level-1 rule X -> s^n (the build's closed form); RL turns it
    into X -> [(s, n)], and Simp keeps both (the run rule is pinned by X's rhs
    being a run rule's holder, X by C)."""
    g = oracle_mod.build_strings([b"T" * n], SEED)
    for rl, simp in FLAGS.values():
        got = g.postprocess(rl=rl, simp=simp, expand=True)
        if rl:
            assert BP.rules_of(got) == [([ord("T")], n), ([256], 1)]
            assert got["c"].tolist() == [257]
            assert got["stats"].tolist() == [1, n, 1, 2, 3, 0, 2, 3]
        else:
            assert BP.rules_of(got) == [([ord("T")] * n, 1)]
            assert got["stats"].tolist() == [1, n, 0, 1, n, 0, 1, n]
        assert got["expansions"] == [b"T" * n]


def _collections():
    rng = np.random.default_rng(11)
    out = []
    # binary alphabet: many runs at every level
    for k, lo, hi in ((3, 20, 60), (6, 2, 40)):
        out.append([bytes(rng.choice([65, 67], int(rng.integers(lo, hi + 1))).astype(np.uint8))
                    for _ in range(k)])
    # mutated copies of one DNA string, plus short and one-byte strings
    base = D.BASES[rng.integers(0, 4, 300)]
    cols = [base.copy() for _ in range(4)]
    for c in cols[1:]:
        pos = rng.integers(0, 300, 4)
        c[pos] = D.BASES[rng.integers(0, 4, 4)]
    out.append([c.tobytes() for c in cols] + [b"A", b"AC", b"GGGGGG"])
    # a tandem repeat and homopolymer runs inside random DNA
    rep = (b"ACG" * 30) + b"TTTTTTTTTTTT" + D.BASES[rng.integers(0, 4, 40)].tobytes()
    out.append([rep, rep[5:], b"ACGACGACG" * 5])
    return out


@pytest.mark.parametrize("case", range(4))
def test_rl_properties_and_simp_fixpoint(oracle_mod, case):
    """RL's output has RL's defining properties over the input grammar; Simp
    equals the one-removal-at-a-time fixpoint, with and without RL first."""
    strings = _collections()[case]
    g = oracle_mod.build_strings(strings, SEED)
    level_rules, level_c = BP.level_rules_global(g.export())
    plain = g.postprocess(rl=False, simp=False)
    assert BP.rules_of(plain) == level_rules and plain["c"].tolist() == level_c
    rl = g.postprocess(rl=True, simp=False, expand=True)
    n_runs = BP.check_rl(level_rules, BP.rules_of(rl))
    assert int(rl["stats"][2]) == n_runs
    assert rl["expansions"] == [bytes(s) for s in strings]
    for base, simp_on in ((plain, g.postprocess(rl=False, simp=True, expand=True)),
                          (rl, g.postprocess(rl=True, simp=True, expand=True))):
        want_rules, want_c = BP.simp_fixpoint(BP.rules_of(base), base["c"].tolist())
        assert BP.rules_of(simp_on) == want_rules
        assert simp_on["c"].tolist() == want_c
        assert simp_on["expansions"] == [bytes(s) for s in strings]
        st = simp_on["stats"].tolist()
        # splicing a rule of q symbols in place of its one occurrence: G drops by 1
        assert st[5] == len(base["mult"]) - len(want_rules)
        assert st[6] == st[3] - st[5] and st[7] == st[4] - st[5]
        assert st[7] == BP.grammar_size(want_rules)


def test_round_trip_tiny_and_repeats(oracle_mod):
    """exp(C[j]) = T_j after RL + Simp on genome-like collections with runs."""
    for name, scale in (("tiny", 0.1), ("repeats", 0.0002)):
        text, off = D.make_config(name, scale=scale)
        g = oracle_mod.build(text, off, SEED)
        got = g.postprocess(rl=True, simp=True, expand=True)
        offs = off.astype(np.int64)
        assert got["expansions"] == [text[offs[j]:offs[j + 1]].tobytes()
                                     for j in range(len(offs) - 1)]
        st = got["stats"].tolist()
        assert st[0] == sum(len(L["fp"]) for L in g.export()["levels"])
        rules = BP.rules_of(got)
        assert all(z < 256 + r for r, (rhs, _) in enumerate(rules) for z in rhs)
        assert st[7] == BP.grammar_size(rules)

