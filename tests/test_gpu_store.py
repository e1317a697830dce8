"""The stored file of a post-processed grammar on the GPU (lcg_slp_encode,
lcg_slp_decode) against the oracle.

The GPU grammar equals the oracle's rank for rank, so its file must equal the
oracle's byte for byte, for every combination of RL and Simp.  Decoding the
oracle's file on the GPU gives the oracle's decoded arrays, decompresses to
the input and encodes back to the same bytes.  Every malformed file the
oracle refuses is refused by the GPU decoder too, before anything is
expanded.  Random access into the post-processed grammar (lcg_slp_extract)
gives the input's substrings, before and after the stored file.
"""
import numpy as np
import pytest

import store_fmt as SF
from paper_2411_12439_amd import datagen as D

pytestmark = pytest.mark.gpu
SEED = D.HASH_SEED
FLAGS = {"none": (False, False), "rl": (True, False), "simp": (False, True),
         "rl_simp": (True, True)}


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2411_12439_amd import lcg
    lcg.lib()
    return lcg


def _dev(data):
    import torch
    return torch.from_numpy(np.frombuffer(bytes(data), np.uint8).copy()).to("cuda")


def _check_case(L, O, text, off, which):
    rl, simp = FLAGS[which]
    t, o = L.to_device(text, off)
    g = L.build(t, o, seed=SEED)
    slp = g.postprocess(rl=rl, simp=simp)
    got = bytes(slp.encode().cpu().numpy())
    og = O.build(text, off, SEED)
    want = og.stored(rl=rl, simp=simp)
    assert len(got) == len(want)
    if got != want:
        a = np.frombuffer(got, np.uint64)
        b = np.frombuffer(want, np.uint64)
        raise AssertionError("first differing word %d" % int(np.nonzero(a != b)[0][0]))
    # decode the oracle's file on the GPU
    dec = L.decode(_dev(want))
    e = dec.export()
    od = O.decode_stored(want)
    for key in ("off", "rhs", "mult", "c"):
        assert np.array_equal(e[key], od[key]), key
    assert e["stats"].tolist()[6:] == od["stats"].tolist()[6:]
    out, _ = dec.expand_strings()
    assert np.array_equal(out.cpu().numpy(), text)
    assert bytes(dec.encode().cpu().numpy()) == want


@pytest.mark.parametrize("which", sorted(FLAGS))
@pytest.mark.parametrize("config,scale", [("tiny", 1.0), ("bacterial", 0.01), ("repeats", 0.0005)])
def test_file_equals_oracle(L, config, scale, which):
    from oracle import oracle as O
    print("stored: %s %g %s" % (config, scale, which), flush=True)
    text, off = D.make_config(config, scale=scale)
    _check_case(L, O, text, off, which)


@pytest.mark.parametrize("which", ["none", "rl_simp"])
def test_edge_collections(L, which):
    from oracle import oracle as O
    rng = np.random.default_rng(31)
    dna = D.BASES[rng.integers(0, 4, 3000)].tobytes()
    cases = [
        [b"A", b"C", b"A"],                       # no rules at all
        [b"T" * 5000],                            # a run longer than 2^b_sym
        [b"A", dna, b"G" * 3, dna[:1000] + b"N" + dna[1001:], b"AC" * 800, b"x"],
    ]
    for strings in cases:
        text, off = O.pack(strings)
        _check_case(L, O, text, off, which)


def test_malformed_files_are_refused(L):
    from oracle import oracle as O
    for name, data, frag in SF.bad_files(O, SEED):
        print("malformed:", name, flush=True)
        with pytest.raises(ValueError):
            O.decode_stored(data)
        with pytest.raises(L.LcgError) as e:
            L.decode(_dev(data))
        assert e.value.name == "LCG_EINVAL", name
        assert frag in str(e.value), (name, str(e.value))


def test_long_doubling_chain_decodes_without_expansion(L):
    """2^60 bytes from 60 rules: accepted; lengths are kept, nothing expanded."""
    rules, c, b = SF.doubling_chain(60)
    dec = L.decode(_dev(SF.write(rules, c, b)))
    assert dec.size() == (60, 120, 1)
    assert dec.stats().tolist()[6:] == [60, 120]


def test_small_buffer_and_query(L):
    import ctypes
    text, off = D.make_config("tiny", scale=0.1)
    t, o = L.to_device(text, off)
    slp = L.build(t, o, seed=SEED).postprocess()
    full = slp.encode()
    n = ctypes.c_uint64()
    small = full[:64].clone()
    rc = L.lib().lcg_slp_encode(slp.h, ctypes.c_void_p(small.data_ptr()), 64, ctypes.byref(n), None)
    assert rc == -1 and n.value == full.numel()


def test_corrupted_files_same_decision_as_oracle(L):
    """Seeded random corruptions of a good file: the GPU decoder refuses exactly
    the files the oracle refuses, and decodes the others to the oracle's arrays
    (nothing is expanded: an accepted file may derive a huge text)."""
    from oracle import oracle as O
    rng = np.random.default_rng(41)
    base = D.BASES[rng.integers(0, 4, 400)]
    strings = [base.tobytes(), base[:200].tobytes() + b"T" * 40, b"A", b"GG" * 30]
    good = O.build_strings(strings, SEED).stored()
    accepted = 0
    for i, data in enumerate(SF.corrupted(good, 78, 300)):
        print("corrupted file", i, flush=True)
        try:
            want = O.decode_stored(data)
        except ValueError:
            want = None
        if len(data) == 0:
            assert want is None
            continue
        if want is None:
            with pytest.raises(L.LcgError) as e:
                L.decode(_dev(data))
            assert e.value.name == "LCG_EINVAL"
            continue
        accepted += 1
        e = L.decode(_dev(data)).export()
        for key in ("off", "rhs", "mult", "c"):
            assert np.array_equal(e[key], want[key]), (i, key)
    assert accepted > 0


# ------------------------------------------ random access to the post-processed grammar
def _slp_queries(rng, off, nq, maxlen):
    lens_s = np.diff(off.astype(np.int64))
    k = len(lens_s)
    j = rng.integers(0, k, nq)
    ln = np.minimum(rng.integers(1, maxlen + 1, nq), lens_s[j])
    st = (rng.random(nq) * (lens_s[j] - ln + 1)).astype(np.int64)
    # string starts and ends, single bytes
    j = np.concatenate([j, np.arange(k), np.arange(k), np.arange(k)])
    st = np.concatenate([st, np.zeros(k, np.int64), lens_s - np.minimum(lens_s, maxlen), lens_s - 1])
    ln = np.concatenate([ln, np.minimum(lens_s, maxlen), np.minimum(lens_s, maxlen),
                         np.ones(k, np.int64)])
    return j, st, ln


def _check_slp_extract(slp, text, off, q):
    out, offs = slp.extract(*q)
    got = out.cpu().numpy()
    o = offs.cpu().numpy()
    base = off.astype(np.int64)
    j, st, ln = q
    for i in range(len(j)):
        a = int(base[j[i]] + st[i])
        assert np.array_equal(got[o[i]:o[i + 1]], text[a:a + int(ln[i])]), (i, int(j[i]), int(st[i]))


@pytest.mark.parametrize("which", sorted(FLAGS))
@pytest.mark.parametrize("config,scale", [("tiny", 1.0), ("bacterial", 0.01), ("repeats", 0.0005)])
def test_slp_extract(L, config, scale, which):
    """Substrings of the post-processed grammar (run rules included) equal the
    input's, also after the grammar went through its stored file."""
    rl, simp = FLAGS[which]
    text, off = D.make_config(config, scale=scale)
    t, o = L.to_device(text, off)
    slp = L.build(t, o, seed=SEED).postprocess(rl=rl, simp=simp)
    rng = np.random.default_rng(51)
    q = _slp_queries(rng, off, 1500, L.EXTRACT_MAX)
    _check_slp_extract(slp, text, off, q)
    _check_slp_extract(L.decode(slp.encode()), text, off, q)


def test_slp_extract_edges_and_errors(L):
    from oracle import oracle as O
    rng = np.random.default_rng(52)
    dna = D.BASES[rng.integers(0, 4, 4000)].tobytes()
    strings = [b"A", b"T" * 7000, b"AC" * 3000, dna, b"G" * 3 + dna[:500], b"C"]
    text, off = O.pack(strings)
    t, o = L.to_device(text, off)
    slp = L.build(t, o, seed=SEED).postprocess()
    _check_slp_extract(slp, text, off, _slp_queries(rng, off, 800, L.EXTRACT_MAX))
    n0 = int(off[1] - off[0])
    for j, st, ln in ((0, n0, 1), (1, 0, L.EXTRACT_MAX + 1), (len(strings), 0, 1), (2, 0, 0)):
        with pytest.raises(L.LcgError) as e:
            slp.extract([j], [st], [ln])
        assert e.value.name == "LCG_EINVAL"


def test_save_and_load_a_file(L, tmp_path):
    """Slp.save writes the stored file to disk and load_slp reads it back: the
    same bytes as the oracle's file, the same strings."""
    from oracle import oracle as O
    text, off = D.make_config("tiny", scale=0.5)
    t, o = L.to_device(text, off)
    slp = L.build(t, o, seed=SEED).postprocess()
    path = str(tmp_path / "collection.lcgs")
    n = slp.save(path)
    raw = open(path, "rb").read()
    assert len(raw) == n and raw == O.build(text, off, SEED).stored()
    back = L.load_slp(path)
    out, _ = back.expand_strings()
    assert np.array_equal(out.cpu().numpy(), text)


def test_merged_and_plain_grammars_store_the_same_file(L):
    """A grammar built in two halves and merged (MergeGrams), and one built in
    the plain form, equal the oracle's grammar of all the strings rank for
    rank, so their stored files are the oracle's bytes; random access works
    on them."""
    from oracle import oracle as O
    text, off = D.make_config("bacterial", scale=0.01)
    o64 = off.astype(np.int64)
    strings = [text[o64[j]:o64[j + 1]].tobytes() for j in range(len(o64) - 1)]
    half = len(strings) // 2
    want = O.build(text, off, SEED).stored()
    ta, oa = L.to_device(*O.pack(strings[:half]))
    tb, ob = L.to_device(*O.pack(strings[half:]))
    merged = L.build(ta, oa, seed=SEED)
    merged.merge(L.build(tb, ob, seed=SEED))
    t, o = L.to_device(text, off)
    plain = L.build(t, o, seed=SEED, mode=L.MODE_PLAIN)
    rng = np.random.default_rng(61)
    q = _slp_queries(rng, off, 500, 300)
    for g in (merged, plain):
        slp = g.postprocess()
        assert bytes(slp.encode().cpu().numpy()) == want
        _check_slp_extract(slp, text, off, q)
