"""The two large collections at full size: the batched one (2,000 strings,
~5 GB, more than 2^32 positions) and the repeat-heavy one (8 x 250 MB with
tandem repeats and homopolymer runs).

Checked at full size: every string expands back to the input; Theorem 1's
halving holds in every round and every string ends; chosen strings'
sub-grammars equal the oracle's grammar of each string alone, rank for rank
once renumbered in the string's own first-occurrence order (stability,
Def. 1) -- on the batched collection the string holding byte 2^32, the two
after it and the last one (the 64-bit offset paths), and the shortest and
longest strings; on the repeat-heavy collection whole 250 MB strings (the
first and the last), whose 20 kb homopolymers and tandem repeats make the
deepest equal-run cases; random substrings and longest common extensions
match the input; maximal exact matches between batched strings of one base
equal the oracle's in the two strings alone; and for the repeat-heavy
collection the RL + Simp grammar decompresses to the input, also through its
stored file, gives random substrings of the input from the decoded grammar,
and keeps Simp's size identity.
"""
import numpy as np
import pytest

from paper_2411_12439_amd import canon as CN
from paper_2411_12439_amd import datagen as D

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]
SEED = D.HASH_SEED


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2411_12439_amd import lcg
    lcg.lib()
    return lcg


def _built(L, name):
    print("generating the %s collection" % name, flush=True)
    text, off = D.make_config(name)
    t, o = L.to_device(text, off)
    print("building", flush=True)
    g = L.build(t, o, seed=SEED)
    print("exporting", flush=True)
    return text, off, t, g, g.export()


@pytest.fixture(scope="module")
def batched(L):
    return _built(L, "batched")


@pytest.fixture(scope="module")
def repeats(L):
    return _built(L, "repeats")


def _round_trip_and_invariants(g, off, t):
    import torch
    k = len(off) - 1
    st = g.stats()
    active = k
    for n_in, d, u, q, act in st[:, :5].astype(np.int64):
        assert 2 * d <= n_in + active
        assert u <= d and q <= n_in
        active = act
    assert st[-1, 4] == 0
    out, offs = g.expand_strings()
    assert out.numel() == t.numel() and torch.equal(out, t)
    assert np.array_equal(offs.cpu().numpy().astype(np.uint64), off.astype(np.uint64))


def _strings_equal_oracle(e, text, off, sample):
    from oracle import oracle as O
    for j in sample:
        a, b = int(off[j]), int(off[j + 1])
        print("oracle on string %d (%d bytes at offset %d)" % (j, b - a, a), flush=True)
        alone = O.build(text[a:b], np.array([0, b - a], np.uint64), SEED).export()
        mine = CN.own_order_subgrammar(e, j)
        assert CN.exports_equal(mine, alone), (j, CN.first_difference(mine, alone))


def _random_substrings(L, g, text, off, seed):
    rng = np.random.default_rng(seed)
    k = len(off) - 1
    lens = np.diff(off.astype(np.int64))
    jq = rng.integers(0, k, 2000)
    ln = np.minimum(rng.integers(1, L.EXTRACT_MAX + 1, 2000), lens[jq])
    sq = (rng.random(2000) * (lens[jq] - ln + 1)).astype(np.int64)
    xo, xoff = g.extract(jq, sq, ln)
    xo = xo.cpu().numpy()
    xoff = xoff.cpu().numpy()
    base = off.astype(np.int64)
    for q in range(2000):
        a = int(base[jq[q]] + sq[q])
        assert np.array_equal(xo[xoff[q]:xoff[q + 1]], text[a:a + int(ln[q])]), q


def test_full_batched_round_trip(batched):
    text, off, t, g, e = batched
    assert int(off[-1]) > (1 << 32)
    _round_trip_and_invariants(g, off, t)


def test_full_batched_strings_equal_oracle(batched):
    """The string holding byte 2^32, the two after it, the last string, and
    the shortest and longest ones, each against the oracle's build of it alone."""
    text, off, t, g, e = batched
    o = off.astype(np.int64)
    k = len(o) - 1
    j32 = int(np.searchsorted(o, 1 << 32, side="right")) - 1
    assert o[j32] < (1 << 32) < o[j32 + 1] or o[j32] == (1 << 32)
    lens = np.diff(o)
    sample = [j32, j32 + 1, j32 + 2, k - 1, int(np.argmin(lens)), int(np.argmax(lens))]
    assert all(o[j] > (1 << 32) for j in sample[1:4])
    _strings_equal_oracle(e, text, off, sample)


def test_full_batched_mems_equal_oracle(batched):
    """Maximal exact matches between strings from one base (j and j + 32): the
    string holding byte 2^32, the last string, and the first, each against the
    oracle's matches in its build of the two strings alone -- by stability
    (Def. 1) the parses, hence the matches in text positions, do not depend on
    the other strings."""
    from oracle import oracle as O
    text, off, t, g, e = batched
    o = off.astype(np.int64)
    k = len(o) - 1
    j32 = int(np.searchsorted(o, 1 << 32, side="right")) - 1
    found = 0
    for a, b in [(j32, j32 + 32), (k - 1, k - 33), (0, 32)]:
        pair = [text[o[a]:o[a + 1]], text[o[b]:o[b + 1]]]
        pt = np.concatenate(pair)
        po = np.array([0, len(pair[0]), len(pt)], np.uint64)
        print("oracle on strings %d and %d (%d + %d bytes)" % (a, b, len(pair[0]), len(pair[1])),
              flush=True)
        og = O.build(pt, po, SEED)
        for level, min_len in [(2, 32), (3, 100)]:
            pa, pb, ln = g.mems(a, b, level, min_len)
            wa, wb, wl = og.mems(pt, po, 0, 1, level, min_len)
            got = np.stack([x.cpu().numpy().astype(np.uint64) for x in (pa, pb, ln)])
            assert np.array_equal(got, np.stack([wa, wb, wl])), (a, b, level)
            found += got.shape[1]
    assert found > 0


def test_full_batched_random_access(L, batched):
    text, off, t, g, e = batched
    _random_substrings(L, g, text, off, 5)


def test_full_repeats_round_trip(repeats):
    text, off, t, g, e = repeats
    _round_trip_and_invariants(g, off, t)


def test_full_repeats_whole_strings_equal_oracle(repeats):
    """Whole 250 MB strings (homopolymers up to 20 kb, tandem repeats of
    10-10,000 copies) against the oracle's build of each alone."""
    text, off, t, g, e = repeats
    _strings_equal_oracle(e, text, off, [0, len(off) - 2])


def test_full_repeats_random_access(L, repeats):
    text, off, t, g, e = repeats
    _random_substrings(L, g, text, off, 5)


def test_full_repeats_postprocess_and_store(L, repeats):
    import torch
    text, off, t, g, e = repeats
    # RL and Simp on the deep, run-heavy grammar
    slp = g.postprocess(rl=True, simp=True)
    st = [int(x) for x in slp.stats()]
    assert st[2] > 0 and st[6] == st[3] - st[5] and st[7] == st[4] - st[5]
    out, _ = slp.expand_strings()
    assert torch.equal(out, t)
    del out
    # through the stored file and back
    dec = L.decode(slp.encode())
    out, _ = dec.expand_strings()
    assert torch.equal(out, t)
    del out
    # random substrings of the decoded grammar (run rules of long homopolymers)
    _random_substrings(L, dec, text, off, 7)
    dec.free()
    slp.free()


def test_full_repeats_lce(repeats):
    from oracle import oracle as O
    text, off, t, g, e = repeats
    # longest common extensions between the copies, against the bytes
    rng = np.random.default_rng(6)
    lens = np.diff(off.astype(np.int64))
    nq = 3000
    j1 = rng.integers(0, len(lens), nq)
    j2 = rng.integers(0, len(lens), nq)
    p1 = (rng.random(nq) * lens[j1]).astype(np.int64)
    p2 = np.minimum(p1, lens[j2])  # same offsets: long matches between the copies
    for backward in (False, True):
        got = g.lce(j1, p1, j2, p2, backward=backward).cpu().numpy()
        want = O.lce(text, off, j1, p1, j2, p2, backward).astype(np.int64)
        assert np.array_equal(got, want)
