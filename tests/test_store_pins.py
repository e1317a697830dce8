"""Pins of the oracle's stored file of a post-processed grammar (App. A,
storing the final grammar: G log g bits for the right-hand sides, g log G
bits for the pointers, one entry per string for C).  No GPU.

What fixes the encoder and decoder: words derived by hand for small grammars
(``golden/stored_example.json``); an independent reader and writer
(``store_fmt.py``, whole sections as Python integers) that must agree with
the oracle on every collection; the size of each section in closed form from
G, g and k (pinned by the post-processing pins); the round trip through the
decoder; and the decoder's refusal of every kind of malformed file.  A
swapped section, a wrong width, a cell off by one, a run rule stored in the
wrong order or a check missing from the decoder fails one of them.
"""
import json
import math
import os

import numpy as np
import pytest

import store_fmt as SF
from paper_2411_12439_amd import datagen as D

SEED = D.HASH_SEED
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
FLAGS = {"none": (False, False), "rl": (True, False), "simp": (False, True),
         "rl_simp": (True, True)}


def _words(b):
    return [hex(int(x)) for x in np.frombuffer(b, np.uint64)]


@pytest.mark.parametrize("case", range(3))
def test_golden_words(oracle_mod, case):
    fx = json.load(open(os.path.join(GOLDEN, "stored_example.json")))["cases"][case]
    s = fx["string"]
    text = (b"T" * int(s.split("*")[1])) if "*" in s else s.encode()
    g = oracle_mod.build_strings([text], SEED)
    got = g.stored(rl=fx["rl"], simp=fx["simp"])
    assert _words(got) == fx["words"]
    back = oracle_mod.decode_stored(got, expand=True)
    assert back["expansions"] == [text]


def _collections():
    rng = np.random.default_rng(12)
    base = D.BASES[rng.integers(0, 4, 400)]
    cols = [base.copy() for _ in range(5)]
    for c in cols[1:]:
        c[rng.integers(0, 400, 5)] = D.BASES[rng.integers(0, 4, 5)]
    return [
        [c.tobytes() for c in cols] + [b"A", b"AC", b"G" * 700],
        [bytes(rng.choice([65, 67], int(rng.integers(5, 80))).astype(np.uint8)) for _ in range(9)],
        [(b"ACG" * 40) + b"T" * 300 + base[:50].tobytes(), b"ACGACG" * 7],
    ]


@pytest.mark.parametrize("which", sorted(FLAGS))
@pytest.mark.parametrize("case", range(3))
def test_reader_agrees_and_sizes(oracle_mod, case, which):
    """The independent reader finds the post-processed grammar in the file,
    the section sizes follow from G, g and k, and the file round-trips."""
    strings = _collections()[case]
    g = oracle_mod.build_strings(strings, SEED)
    rl, simp = FLAGS[which]
    pp = g.postprocess(rl=rl, simp=simp)
    data = g.stored(rl=rl, simp=simp)
    f = SF.read(data)
    assert f["rules"] == SF.rules_of(pp)
    assert f["c"] == pp["c"].tolist() and f["bounds"] == pp["bounds"].tolist()
    r, G, k = int(pp["stats"][6]), int(pp["stats"][7]), len(strings)
    assert (f["r"], f["G"], f["k"]) == (r, G, k)
    assert f["runs"] == sum(1 for _, m in f["rules"] if m >= 2)
    # widths: ceil(log2 g) bits per symbol (g = 256 + r symbols), ceil(log2 G) per pointer
    assert f["b_sym"] == math.ceil(math.log2(256 + r))
    longest = max([m for _, m in f["rules"] if m >= 2], default=0)
    assert f["b_cell"] == max(f["b_sym"], longest.bit_length())
    assert f["b_ptr"] == (max(1, math.ceil(math.log2(G))) if r else 1)
    want = [-(-G * f["b_cell"] // 64), -(-r * f["b_ptr"] // 64), -(-r // 64),
            -(-k * f["b_sym"] // 64), -(-f["nb"] // 2)]
    assert f["section_words"] == want
    assert len(data) == f["size"] == f["total"] == 64 + 8 * sum(want)
    # every rule refers to ids below its block
    B = f["bounds"]
    for x, (rhs, _) in enumerate(f["rules"]):
        blk = max(b for b in range(len(B) - 1) if B[b] <= 256 + x)
        assert all(y < B[blk] for y in rhs)
    # the independent writer gives the same bytes, and the decoder the same grammar
    assert SF.write(f["rules"], f["c"], f["bounds"]) == data
    back = oracle_mod.decode_stored(data, expand=True)
    for key in ("off", "rhs", "mult", "c", "bounds"):
        assert np.array_equal(back[key], pp[key]), key
    assert back["expansions"] == [bytes(s) for s in strings]
    assert back["stats"].tolist()[6:] == [r, G]


def test_paper_budget_on_genome_like(oracle_mod):
    """On a genome-like collection (no run longer than g) the right-hand sides
    take exactly G ceil(log g) bits and the pointers g ceil(log G), as budgeted."""
    text, off = D.make_config("tiny", scale=0.2)
    g = oracle_mod.build(text, off, SEED)
    pp = g.postprocess()
    f = SF.read(g.stored())
    r, G = int(pp["stats"][6]), int(pp["stats"][7])
    assert f["b_cell"] == f["b_sym"] == math.ceil(math.log2(256 + r))
    assert f["section_words"][0] == -(-G * math.ceil(math.log2(256 + r)) // 64)
    assert f["section_words"][1] == -(-r * math.ceil(math.log2(G)) // 64)


def test_decoder_rejects_malformed(oracle_mod):
    for name, data, frag in SF.bad_files(oracle_mod, SEED):
        with pytest.raises(ValueError) as e:
            oracle_mod.decode_stored(data)
        assert frag in str(e.value), (name, str(e.value))


def test_doubling_chain_below_limit(oracle_mod):
    """60 doublings give 2^60 bytes: accepted (lengths only, nothing expanded)."""
    rules, c, b = SF.doubling_chain(60)
    d = oracle_mod.decode_stored(SF.write(rules, c, b))
    assert len(d["mult"]) == 60 and d["stats"].tolist()[6:] == [60, 120]


def test_grammar_without_rules(oracle_mod):
    """Strings of one byte each: no rules, C holds terminals (8-bit cells), one bound."""
    g = oracle_mod.build_strings([b"A", b"C", b"A"], SEED)
    data = g.stored()
    f = SF.read(data)
    assert (f["r"], f["G"], f["k"], f["nb"], f["b_sym"]) == (0, 0, 3, 1, 8)
    assert f["c"] == [65, 67, 65] and f["bounds"] == [256]
    assert len(data) == 64 + 8 + 8
    assert oracle_mod.decode_stored(data, expand=True)["expansions"] == [b"A", b"C", b"A"]


def test_decoder_on_corrupted_files(oracle_mod):
    """Random corruptions: every file is refused with ValueError or decodes to a
    grammar whose file is the same bytes (the checks leave nothing in between)."""
    g = oracle_mod.build_strings(_collections()[0], SEED)
    accepted = 0
    for data in SF.corrupted(g.stored(), 77, 400):
        try:
            d = oracle_mod.decode_stored(data)
        except ValueError:
            continue
        accepted += 1
        assert SF.write(SF.rules_of(d), d["c"].tolist(), d["bounds"].tolist()) == data
    assert 0 < accepted < 400
