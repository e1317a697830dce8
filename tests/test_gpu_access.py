"""Random access (lcg_extract), longest common extensions (lcg_lce) and the
lcp / lcs of symbol pairs (lcg_symbol_lce).

Extraction is checked against slices of the input (the grammar derives it
exactly), byte for byte: queries hit string starts and ends, single bytes,
the maximum length, strings of length one (C at level 0) and long level-1
rules (homopolymers).  LCE answers are checked against the oracle's plain
byte comparison, in both directions, on random pairs and on pairs at the same
offset of copies of one base (long matches), including string ends.  Symbol
pairs (App. B's lcp(X, Y), lcs(X, Y)) are checked against the oracle's
expand-and-compare on random pairs within and across levels, C entries
(whole strings of copies: long common parts) and symbols against themselves.
"""
import numpy as np
import pytest

from paper_2411_12439_amd import datagen as D

pytestmark = pytest.mark.gpu
SEED = D.HASH_SEED


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2411_12439_amd import lcg
    lcg.lib()
    return lcg


def _queries(rng, off, nq, maxlen):
    lens_s = np.diff(off.astype(np.int64))
    j = rng.integers(0, len(lens_s), nq)
    ln = np.minimum(rng.integers(1, maxlen + 1, nq), lens_s[j])
    st = (rng.random(nq) * (lens_s[j] - ln + 1)).astype(np.int64)
    # boundaries: string starts, string ends, single bytes, whole short strings
    k = len(lens_s)
    j = np.concatenate([j, np.arange(k), np.arange(k), np.arange(k)])
    st = np.concatenate([st, np.zeros(k, np.int64), lens_s - np.minimum(lens_s, maxlen),
                         lens_s - 1])
    ln = np.concatenate([ln, np.minimum(lens_s, maxlen), np.minimum(lens_s, maxlen),
                         np.ones(k, np.int64)])
    return j, st, ln


def _check(L, g, text, off, j, st, ln):
    out, offs = g.extract(j, st, ln)
    got = out.cpu().numpy()
    o = offs.cpu().numpy()
    base = off.astype(np.int64)
    for q in range(len(j)):
        a = int(base[j[q]] + st[q])
        want = text[a:a + int(ln[q])]
        assert np.array_equal(got[o[q]:o[q + 1]], want), (q, int(j[q]), int(st[q]), int(ln[q]))


@pytest.mark.parametrize("config,scale", [("tiny", 1.0), ("bacterial", 0.01), ("repeats", 0.0005)])
def test_random_queries(L, config, scale):
    text, off = D.make_config(config, scale=scale)
    t, o = L.to_device(text, off)
    g = L.build(t, o, seed=SEED)
    rng = np.random.default_rng(3)
    print("extract: %s scale %g" % (config, scale), flush=True)
    _check(L, g, text, off, *_queries(rng, off, 3000, L.EXTRACT_MAX))


def test_edge_strings(L):
    from oracle import oracle as O
    rng = np.random.default_rng(4)
    dna = D.BASES[rng.integers(0, 4, 9000)].tobytes()
    strings = [b"A", b"C", b"GG", b"T" * 7000, dna, b"N" * 100 + dna[:300], b"AC" * 2000, b"x"]
    text, off = O.pack(strings)
    t, o = L.to_device(text, off)
    g = L.build(t, o, seed=SEED)
    _check(L, g, text, off, *_queries(rng, off, 2000, L.EXTRACT_MAX))
    # after a merge, and on a plain-form grammar
    half = len(strings) // 2
    ta, oa = L.to_device(*O.pack(strings[:half]))
    tb, ob = L.to_device(*O.pack(strings[half:]))
    ga = L.build(ta, oa, seed=SEED)
    ga.merge(L.build(tb, ob, seed=SEED))
    _check(L, ga, text, off, *_queries(rng, off, 500, 300))
    gp = L.build(t, o, seed=SEED, mode=L.MODE_PLAIN)
    _check(L, gp, text, off, *_queries(rng, off, 500, 64))


def test_out_of_range_queries_are_rejected(L):
    text, off = D.make_config("tiny", scale=0.05)
    t, o = L.to_device(text, off)
    g = L.build(t, o, seed=SEED)
    n0 = int(off[1] - off[0])
    for j, st, ln in ((0, n0, 1), (0, n0 - 2, 3), (len(off) - 1, 0, 1), (0, 0, 0),
                      (0, 0, L.EXTRACT_MAX + 1)):
        with pytest.raises(L.LcgError) as e:
            g.extract([j], [st], [ln])
        assert e.value.name == "LCG_EINVAL"
    # a bad query does not stop the good ones
    import torch
    j = torch.tensor([0, 0], dtype=torch.int32, device="cuda")
    st = torch.tensor([5, n0], dtype=torch.int64, device="cuda")
    ln = torch.tensor([10, 1], dtype=torch.int32, device="cuda")
    offs = torch.tensor([0, 10, 11], dtype=torch.int64, device="cuda")
    out = torch.zeros(11, dtype=torch.uint8, device="cuda")
    import ctypes
    rc = L.lib().lcg_extract(g.h, 2, ctypes.c_void_p(j.data_ptr()), ctypes.c_void_p(st.data_ptr()),
                             ctypes.c_void_p(ln.data_ptr()), ctypes.c_void_p(offs.data_ptr()),
                             ctypes.c_void_p(out.data_ptr()), None)
    assert rc == -1
    assert np.array_equal(out.cpu().numpy()[:10], text[5:15])


def test_full_bacterial_random_access(L):
    text, off = D.make_config("bacterial")
    t, o = L.to_device(text, off)
    g = L.build(t, o, seed=SEED)
    rng = np.random.default_rng(9)
    _check(L, g, text, off, *_queries(rng, off, 4000, L.EXTRACT_MAX))


# ------------------------------------------------ longest common extension
def _lce_queries(rng, off, nq, base_of=None):
    """Half random pairs, half pairs at the same offset of copies of the same base
    (long matches), plus string ends."""
    lens_s = np.diff(off.astype(np.int64))
    k = len(lens_s)
    j1 = rng.integers(0, k, nq)
    j2 = rng.integers(0, k, nq)
    if base_of is not None:
        same = np.nonzero(np.arange(nq) % 2 == 0)[0]
        for q in same:
            cands = np.nonzero(base_of == base_of[j1[q]])[0]
            j2[q] = cands[rng.integers(0, len(cands))]
    p1 = (rng.random(nq) * (lens_s[j1] + 1)).astype(np.int64)
    p2 = (rng.random(nq) * (lens_s[j2] + 1)).astype(np.int64)
    if base_of is not None:
        p2[::2] = np.minimum(p1[::2], lens_s[j2[::2]])
    j1 = np.concatenate([j1, np.arange(k), np.arange(k)])
    j2 = np.concatenate([j2, np.arange(k), (np.arange(k) + 1) % k])
    p1 = np.concatenate([p1, lens_s, np.zeros(k, np.int64)])
    p2 = np.concatenate([p2, np.zeros(k, np.int64), np.zeros(k, np.int64)])
    return j1, p1, j2, p2


@pytest.mark.parametrize("backward", [False, True])
@pytest.mark.parametrize("config,scale", [("tiny", 1.0), ("bacterial", 0.01), ("repeats", 0.0005)])
def test_lce_equals_oracle(L, config, scale, backward):
    from oracle import oracle as O
    text, off = D.make_config(config, scale=scale)
    t, o = L.to_device(text, off)
    g = L.build(t, o, seed=SEED)
    rng = np.random.default_rng(21)
    base_of = np.arange(len(off) - 1) % (4 if config == "bacterial" else 1)
    q = _lce_queries(rng, off, 4000, base_of)
    got = g.lce(*q, backward=backward).cpu().numpy()
    want = O.lce(text, off, q[0], q[1], q[2], q[3], backward).astype(np.int64)
    assert np.array_equal(got, want), int(np.nonzero(got != want)[0][0])


@pytest.mark.parametrize("backward", [False, True])
def test_lce_edge_strings(L, backward):
    from oracle import oracle as O
    rng = np.random.default_rng(22)
    dna = D.BASES[rng.integers(0, 4, 5000)].tobytes()
    strings = [b"A", b"A", b"AA", b"T" * 3000, b"T" * 2999 + b"G", dna, dna[:2500] + b"N" + dna[2501:],
               dna[7:], b"ACG" * 1000, b"ACG" * 999 + b"ACC", b"C"]
    text, off = O.pack(strings)
    t, o = L.to_device(text, off)
    for g in (L.build(t, o, seed=SEED), L.build(t, o, seed=SEED, mode=L.MODE_PLAIN)):
        q = _lce_queries(rng, off, 3000)
        got = g.lce(*q, backward=backward).cpu().numpy()
        want = O.lce(text, off, q[0], q[1], q[2], q[3], backward).astype(np.int64)
        assert np.array_equal(got, want), int(np.nonzero(got != want)[0][0])


def test_lce_rejects_out_of_range(L):
    text, off = D.make_config("tiny", scale=0.05)
    t, o = L.to_device(text, off)
    g = L.build(t, o, seed=SEED)
    n0 = int(off[1] - off[0])
    for args in (([0], [n0 + 1], [0], [0]), ([len(off) - 1], [0], [0], [0])):
        with pytest.raises(L.LcgError) as e:
            g.lce(*args)
        assert e.value.name == "LCG_EINVAL"


# --------------------------------------------- symbol pairs: lcp(X, Y), lcs(X, Y)
def _symbol_queries(rng, e, nq):
    """Pairs within a level (half) and across levels, then C entries of random
    string pairs (whole strings) and each C entry against itself."""
    levels = e["levels"]
    h = len(levels)
    size = lambda lv: 256 if lv == 0 else len(levels[lv - 1]["fp"])
    lv1 = rng.integers(0, h + 1, nq)
    lv2 = np.where(rng.random(nq) < 0.5, lv1, rng.integers(0, h + 1, nq))
    s1 = np.array([rng.integers(0, size(v)) for v in lv1])
    s2 = np.array([rng.integers(0, size(v)) for v in lv2])
    # the C entries against each other: whole strings
    k = len(e["c_sym"])
    j1 = rng.integers(0, k, nq // 4)
    j2 = rng.integers(0, k, nq // 4)
    lv1 = np.concatenate([lv1, e["c_level"][j1], e["c_level"][j1]])
    s1 = np.concatenate([s1, e["c_sym"][j1], e["c_sym"][j1]])
    lv2 = np.concatenate([lv2, e["c_level"][j2], e["c_level"][j1]])
    s2 = np.concatenate([s2, e["c_sym"][j2], e["c_sym"][j1]])
    return lv1, s1, lv2, s2


@pytest.mark.parametrize("backward", [False, True])
@pytest.mark.parametrize("config,scale", [("tiny", 0.25), ("bacterial", 0.01), ("repeats", 0.0005)])
def test_symbol_lce_equals_oracle(L, config, scale, backward):
    from oracle import oracle as O
    text, off = D.make_config(config, scale=scale)
    t, o = L.to_device(text, off)
    g = L.build(t, o, seed=SEED)
    og = O.build(text, off, SEED)
    rng = np.random.default_rng(23)
    q = _symbol_queries(rng, og.export(), 600)
    got = g.symbol_lce(*q, backward=backward).cpu().numpy()
    want = og.symbol_lce(*q, backward).astype(np.int64)
    assert np.array_equal(got, want), int(np.nonzero(got != want)[0][0])


def test_symbol_lce_edges_and_errors(L):
    from oracle import oracle as O
    strings = [b"A", b"C", b"T" * 3000, b"T" * 2999 + b"G", b"ACG" * 500, b"ACG" * 499 + b"ACC"]
    text, off = O.pack(strings)
    t, o = L.to_device(text, off)
    g = L.build(t, o, seed=SEED)
    og = O.build(text, off, SEED)
    e = og.export()
    rng = np.random.default_rng(24)
    for backward in (False, True):
        q = _symbol_queries(rng, e, 300)
        got = g.symbol_lce(*q, backward=backward).cpu().numpy()
        assert np.array_equal(got, og.symbol_lce(*q, backward).astype(np.int64))
    h = len(e["levels"])
    for args in (([h + 1], [0], [1], [0]), ([1], [len(e["levels"][0]["fp"])], [1], [0]),
                 ([0], [256], [0], [0])):
        with pytest.raises(L.LcgError) as ex:
            g.symbol_lce(*args)
        assert ex.value.name == "LCG_EINVAL"
    # a grammar of one-byte strings: only bytes exist
    ta, oa = L.to_device(*O.pack([b"A", b"C"]))
    g1 = L.build(ta, oa, seed=SEED)
    assert g1.symbol_lce([0, 0], [65, 65], [0, 0], [65, 67]).cpu().tolist() == [1, 0]
