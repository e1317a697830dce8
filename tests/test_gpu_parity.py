"""Parity of the HIP library (through the C ABI) with the CPU oracle.

Both sides number a level's new rules by first occurrence, so the comparison
is exact, rank for rank (the grammar is integer data: zero tolerance).  At
full benchmark sizes, where the oracle would take minutes, sampled strings are
checked one by one: each string's sub-grammar inside the GPU grammar must
equal the oracle's grammar of that string alone (stability, Def. 1), and its
expansion must equal the input.
"""
import itertools

import numpy as np
import pytest

from paper_2411_12439_amd import canon as CN
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


def _pack(strings):
    from oracle import oracle as O
    return O.pack(strings)


def _gpu(L, text, off, **kw):
    t, o = L.to_device(text, off)
    return L.build(t, o, seed=kw.pop("seed", SEED), **kw)


def _assert_same(got, want):
    assert CN.exports_equal(got, want), CN.first_difference(got, want)


def _oracle(text, off, seed=SEED):
    from oracle import oracle as O
    return O.build(text, off, seed)


# Round paths: tail_log2=0 (default 2^22) queues every round of these small
# inputs without host reads (tail mode); tail_log2=1 reads sizes back every
# round (the path of large rounds).
PATHS = pytest.mark.parametrize("tail", [0, 1], ids=["tail", "synced"])


# ---------------------------------------------------------------- tiny config
@PATHS
@pytest.mark.parametrize("mode", [0, 1], ids=["batched", "plain"])
def test_tiny_config_equals_oracle(L, mode, tail):
    text, off = D.make_config("tiny")
    g = _gpu(L, text, off, mode=mode, tail_log2=tail)
    _assert_same(g.export(), _oracle(text, off).export())


def test_tail_and_synced_rounds_agree(L):
    """The same grammar, rank for rank, whichever rounds run in tail mode."""
    text, off = D.make_config("tiny", scale=2.0)
    ref = _gpu(L, text, off, tail_log2=1).export()
    for tail in (8, 14, 18, 30):
        _assert_same(_gpu(L, text, off, tail_log2=tail).export(), ref)


def test_tiny_config_round_statistics(L):
    text, off = D.make_config("tiny")
    st = _gpu(L, text, off).stats()
    want = _oracle(text, off).stats()
    assert st.shape[0] == want.shape[0]
    # n_in, phrases, new rules, new rhs symbols, active strings
    assert np.array_equal(st[:, :5], want)


def test_round_trip_expand(L):
    text, off = D.make_config("tiny", scale=0.3)
    g = _gpu(L, text, off)
    for j in range(len(off) - 1):
        assert np.array_equal(g.expand(j).cpu().numpy(), text[off[j]:off[j + 1]])


def _check_expand_strings(g, text, off, j0, j1):
    out, offs = g.expand_strings(j0, j1)
    want = text[off[j0]:off[j1]]
    assert np.array_equal(out.cpu().numpy(), want)
    assert np.array_equal(offs.cpu().numpy(), (off[j0:j1 + 1] - off[j0]).astype(np.int64))


@PATHS
def test_expand_strings_round_trip(L, tail):
    """All strings expanded together (and sub-ranges) give back the input."""
    text, off = D.make_config("tiny", scale=0.3)
    g = _gpu(L, text, off, tail_log2=tail)
    k = len(off) - 1
    for j0, j1 in ((0, k), (2, 5), (k - 1, k), (3, 3)):
        _check_expand_strings(g, text, off, j0, j1)


def test_speed_options_do_not_change_results(L):
    """Every setting of the options the autotuner may change gives the same grammar."""
    text, off = D.make_config("bacterial", scale=0.02)
    ref = _gpu(L, text, off).export()
    for kw in ({"table_load_log2": 2}, {"table_load_log2": 3}, {"combine_log2": 31},
               {"combine_log2": 1}, {"combine_log2": 8, "tail_log2": 16},
               {"tail_log2": 30, "table_load_log2": 2}):
        _assert_same(_gpu(L, text, off, **kw).export(), ref)


def test_autotuner(L):
    text, off = D.make_config("tiny", scale=2.0)
    t, o = L.to_device(text, off)
    best, ms = L.tune(t, o, seed=SEED)
    assert ms > 0
    assert set(best) == set(L.TUNABLE)
    assert 1 <= best["table_load_log2"] <= 3 and 1 <= best["combine_log2"] <= 31
    _assert_same(L.build(t, o, seed=SEED, **best).export(), _oracle(text, off).export())


def test_autotuner_cache(L, tmp_path, monkeypatch):
    """A cached result is returned for the same device, shape and fixed
    options without measuring again; another shape, or another setting of a
    fixed option, is measured."""
    text, off = D.make_config("tiny", scale=0.5)
    t, o = L.to_device(text, off)
    cache = str(tmp_path / "tune.json")
    first = L.tune(t, o, seed=SEED, cache=cache)

    def no_measuring(*a, **k):
        raise AssertionError("measured again")

    monkeypatch.setattr(L, "_tune_measured", no_measuring)
    assert L.tune(t, o, seed=SEED, cache=cache) == first
    t2, o2 = L.to_device(*D.make_config("tiny", scale=0.25))
    with pytest.raises(AssertionError):
        L.tune(t2, o2, seed=SEED, cache=cache)
    with pytest.raises(AssertionError):
        L.tune(t, o, seed=SEED, cache=cache, table_min_log2=20)



def test_timing_flags(L):
    """LCG_FLAG_TIMING_INSERT records the insert's device time in the rounds
    with host reads and nothing else; neither timing flag changes the grammar
    or the counts; the rounds queued without host reads run in one cooperative
    launch (mode 3) when asked for and every phase is not timed, else as
    separate kernels (mode 2); an unknown flag bit is refused."""
    text, off = D.make_config("tiny")
    t, o = L.to_device(text, off)
    kw = dict(seed=SEED, tail_log2=14)  # rounds above 2^14 symbols read their sizes back
    sp = L.build(t, o, **kw)
    si = L.build(t, o, flags=L.FLAG_TIMING_INSERT, **kw)
    sf = L.build(t, o, flags=L.FLAG_TIMING, **kw)
    ss = L.build(t, o, flags=L.FLAG_FUSED_TAIL, **kw)
    want = _oracle(text, off).export()
    for g in (sp, si, sf, ss):
        _assert_same(g.export(), want)
    p, i, f, sp_ = sp.stats(), si.stats(), sf.stats(), ss.stats()
    # n, d, u, Q, active strings and capacity; the probe and comparison counts
    # depend on which thread claims a slot first
    det = [0, 1, 2, 3, 4, 7]
    for st in (i, f, sp_):
        assert np.array_equal(st[:, det], p[:, det])
    host = p[:, 15] < 2
    assert host.any() and (~host).any()
    for st in (p, i, f):
        assert np.array_equal(st[:, 15], p[:, 15]) and (st[~host, 15] == 2).all()
    assert np.array_equal(sp_[host, 15], p[host, 15]) and (sp_[~host, 15] == 3).all()
    assert (p[:, 8:15] == 0).all()
    assert (i[host, 11] > 0).all() and np.array_equal(i[host, 8], i[host, 11])
    assert (i[:, [9, 10, 12, 13, 14]] == 0).all() and (i[~host, 8:15] == 0).all()
    assert (f[:, 8] > 0).all() and np.array_equal(f[:, 8], f[:, 9:15].sum(axis=1))
    with pytest.raises(L.LcgError) as e:
        L.build(t, o, flags=8, **kw)
    assert e.value.name == "LCG_EINVAL"


@pytest.mark.parametrize("name,scale", [("tiny", 1.0), ("bacterial", 0.01), ("batched", 0.0005)])
def test_fused_and_split_tail_agree(L, name, scale):
    """The tail rounds in one cooperative launch and as separate kernels give
    the same grammar rank for rank (and the oracle's), also for builds that
    start in the tail (every round of these collections) and into a grammar
    that already holds rules."""
    text, off = D.make_config(name, scale=scale)
    t, o = L.to_device(text, off)
    want = _oracle(text, off).export()
    fused = L.build(t, o, seed=SEED, flags=L.FLAG_FUSED_TAIL)
    split = L.build(t, o, seed=SEED)
    _assert_same(fused.export(), want)
    _assert_same(split.export(), want)
    assert (fused.stats()[:, 15] == 3).all() and (split.stats()[:, 15] == 2).all()
    k = len(off) - 1
    h = k // 2
    ta, oa = L.to_device(text[:off[h]], off[:h + 1])
    tb, ob = L.to_device(text[off[h]:], (off[h:] - off[h]).astype(np.uint64))
    g = L.build(ta, oa, seed=SEED, flags=L.FLAG_FUSED_TAIL)
    L.build_into(g, tb, ob, flags=L.FLAG_FUSED_TAIL)
    _assert_same(g.export(), want)

def test_deterministic(L):
    text, off = D.make_config("tiny", scale=0.5)
    a = _gpu(L, text, off).export()
    b = _gpu(L, text, off).export()
    _assert_same(a, b)


# ---------------------------------------------------------------- edge cases
EDGE = {
    "single_byte": [b"A"],
    "two_bytes": [b"AB"],
    "only_singletons": [b"x", b"y", b"x"],
    "singletons_mixed": [b"A", b"ACGTACGGTCA", b"T", b"GG", b"C"],
    "homopolymer_crosses_tiles": [b"G" * 20000],
    "homopolymer_tail": [b"ACGTTGCA" * 700 + b"T" * 9000],
    "run_at_tile_edges": [b"AC" * 2047 + b"G" * 4 + b"CA" * 3000, b"T" * 4095 + b"A" + b"T" * 4097],
    "tile_sized": [bytes(np.random.default_rng(1).integers(65, 69, n, dtype=np.uint8))
                   for n in (4095, 4096, 4097, 8192, 8193)],
    "period2": [b"AC" * 6000],
    "binary_runs": [bytes(np.random.default_rng(2).choice(np.frombuffer(b"AC", np.uint8), 3000))
                    for _ in range(20)],
    "all_bytes": [bytes(np.random.default_rng(3).integers(0, 256, 5000, dtype=np.uint8)),
                  bytes(range(256)) * 3, bytes(range(255, -1, -1))],
    "tandem_repeats": [(b"ACGTTG" * 500 + b"A" * 700 + b"GATTACA" * 300) for _ in range(3)],
}


@PATHS
@pytest.mark.parametrize("case", sorted(EDGE))
@pytest.mark.parametrize("mode", [0, 1], ids=["batched", "plain"])
def test_edge_cases(L, case, mode, tail):
    text, off = _pack(EDGE[case])
    g = _gpu(L, text, off, mode=mode, tail_log2=tail)
    _assert_same(g.export(), _oracle(text, off).export())
    _check_expand_strings(g, text, off, 0, len(off) - 1)


def test_exhaustive_short_dna(L):
    strings = [bytes(t) for n in range(1, 7) for t in itertools.product(b"ACGT", repeat=n)]
    text, off = _pack(strings)
    _assert_same(_gpu(L, text, off).export(), _oracle(text, off).export())


@PATHS
@pytest.mark.parametrize("key_bits", [3, 12])
def test_truncated_keys_rely_on_full_comparison(L, key_bits, tail):
    """Keys cut to a few bits collide constantly; exact comparison must still dedup correctly."""
    text, off = D.make_config("tiny", scale=0.05)
    g = _gpu(L, text, off, key_bits=key_bits, tail_log2=tail)
    _assert_same(g.export(), _oracle(text, off).export())
    assert g.stats()[:, 6].sum() > 0  # full comparisons happened


def test_small_tables_regrow(L):
    text, off = D.make_config("tiny", scale=0.2)
    g = _gpu(L, text, off, table_min_log2=6)
    _assert_same(g.export(), _oracle(text, off).export())


# ---------------------------------------------------------------- merge / build_into
@PATHS
@pytest.mark.parametrize("cut", [1, 3, 7])
def test_merge_equals_build_of_concatenation(L, cut, tail):
    text, off = D.make_config("tiny", scale=0.1)
    ta, oa = text[:off[cut]], off[:cut + 1]
    tb, ob = text[off[cut]:], off[cut:] - off[cut]
    ga = _gpu(L, ta, oa, tail_log2=tail)
    gb = _gpu(L, tb, ob, tail_log2=tail)
    ga.merge(gb)
    _assert_same(ga.export(), _oracle(text, off).export())
    _assert_same(gb.export(), _oracle(tb, ob).export())  # b unchanged


@PATHS
def test_build_into_equals_oracle(L, tail):
    text, off = D.make_config("tiny", scale=0.1)
    g = L.new(SEED)
    for lo, hi in ((0, 2), (2, 3), (3, 8)):
        t, o = L.to_device(text[off[lo]:off[hi]], off[lo:hi + 1] - off[lo])
        first = L.build_into(g, t, o, tail_log2=tail)
        assert first == lo
    _assert_same(g.export(), _oracle(text, off).export())


def test_errors(L):
    import torch
    t, o = L.to_device(np.frombuffer(b"ABC", np.uint8), np.array([0, 2, 2, 3], np.uint64))
    with pytest.raises(L.LcgError) as e:
        L.build(t, o, seed=SEED)
    assert e.value.name == "LCG_EINVAL"
    t, o = L.to_device(np.frombuffer(b"ABCABD", np.uint8), np.array([0, 6], np.uint64))
    with pytest.raises(L.LcgError) as e:
        L.build(t, o, seed=SEED, hbm_budget=1024)
    assert e.value.name == "LCG_ENOMEM"
    ga = L.build(t, o, seed=1)
    gb = L.build(t, o, seed=2)
    with pytest.raises(L.LcgError) as e:
        ga.merge(gb)
    assert e.value.name == "LCG_ESEED"
    torch.cuda.synchronize()


def test_combining_round_equals_oracle(L):
    """4 MB of the tiny recipe: round 1 has ~10^6 phrases over a few thousand keys,
    so (run with host reads) it combines equal keys per chunk; exact equality with
    the oracle."""
    text, off = D.make_config("tiny", scale=4.0)
    g = _gpu(L, text, off, tail_log2=21)
    st = g.stats()
    assert st[0, 15] == 1, "round 1 should combine equal keys"
    _assert_same(g.export(), _oracle(text, off).export())


# ---------------------------------------------------------------- other configurations (scaled)
@pytest.mark.parametrize("name,scale", [("repeats", 0.004), ("batched", 0.001), ("bacterial", 0.01)])
def test_scaled_configs_equal_oracle(L, name, scale):
    text, off = D.make_config(name, scale=scale)
    _assert_same(_gpu(L, text, off).export(), _oracle(text, off).export())


# ---------------------------------------------------------------- full benchmark size
@pytest.fixture(scope="module")
def bacterial_full(L):
    text, off = D.make_config("bacterial")
    t, o = L.to_device(text, off)
    g = L.build(t, o, seed=SEED)
    return text, off, t, o, g


@pytest.mark.parametrize("j", [0, 17, 42, 63])
def test_full_bacterial_sampled_strings(L, bacterial_full, j):
    """Each sampled string: sub-grammar == oracle grammar of the string alone; expansion == input."""
    from oracle import oracle as O
    text, off, t, o, g = bacterial_full
    got = CN.subgrammar(g.export(), [j])
    alone = O.build(text[off[j]:off[j + 1]], np.array([0, off[j + 1] - off[j]], np.uint64), SEED)
    assert CN.canon(got) == CN.canon(alone.export())
    assert np.array_equal(g.expand(j).cpu().numpy(), text[off[j]:off[j + 1]])


def test_full_bacterial_expand_strings(L, bacterial_full):
    text, off, t, o, g = bacterial_full
    _check_expand_strings(g, text, off, 0, len(off) - 1)


def test_full_bacterial_plain_equals_batched(L, bacterial_full):
    text, off, t, o, g = bacterial_full
    gp = L.build(t, o, seed=SEED, mode=L.MODE_PLAIN)
    _assert_same(gp.export(), g.export())


def test_full_bacterial_invariants(L, bacterial_full):
    text, off, t, o, g = bacterial_full
    st = g.stats()
    active = len(off) - 1
    for n_in, d, u, q, act in st[:, :5].astype(np.int64):
        assert 2 * d <= n_in + active
        assert u <= d and q <= n_in
        active = act
    assert st[-1, 4] == 0
