"""The two large collections at full size: the batched one (2,000 strings,
~5 GB, more than 2^32 positions) and the repeat-heavy one (8 x 250 MB with
tandem repeats and homopolymer runs).

The oracle would take minutes on the whole input, so the checks are the ones
that hold at any size: every string expands back to the input; Theorem 1's
halving holds in every round and every string ends; sampled strings'
sub-grammars equal the oracle's grammar of each string alone (stability,
Def. 1); random substrings and longest common extensions match the input;
and for the repeat-heavy collection the RL + Simp grammar decompresses to the
input, also through its stored file, gives random substrings of the input
from the decoded grammar, and keeps Simp's size identity.
"""
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


def _common_checks(L, g, text, off, t, sample):
    import torch
    from oracle import oracle as O
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
    del out
    e = g.export()
    for j in sample:
        a, b = int(off[j]), int(off[j + 1])
        alone = O.build(text[a:b], np.array([0, b - a], np.uint64), SEED)
        assert CN.canon(CN.subgrammar(e, [j])) == CN.canon(alone.export()), j
    rng = np.random.default_rng(5)
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


def test_full_batched(L):
    print("generating the batched collection (~5 GB, about a minute)", flush=True)
    text, off = D.make_config("batched")
    assert int(off[-1]) > (1 << 32)
    t, o = L.to_device(text, off)
    print("building", flush=True)
    g = L.build(t, o, seed=SEED)
    print("checking", flush=True)
    lens = np.diff(off.astype(np.int64))
    small = [int(j) for j in np.argsort(lens)[:2]] + [int(np.argmax(lens))]
    _common_checks(L, g, text, off, t, small)


def test_full_repeats(L):
    from oracle import oracle as O
    import torch
    text, off = D.make_config("repeats")
    t, o = L.to_device(text, off)
    g = L.build(t, o, seed=SEED)
    _common_checks(L, g, text, off, t, [])
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
    rng = np.random.default_rng(7)
    lens = np.diff(off.astype(np.int64))
    jq = rng.integers(0, len(lens), 2000)
    ln = rng.integers(1, L.EXTRACT_MAX + 1, 2000)
    sq = (rng.random(2000) * (lens[jq] - ln + 1)).astype(np.int64)
    xo, xoff = dec.extract(jq, sq, ln)
    xo = xo.cpu().numpy()
    xoff = xoff.cpu().numpy()
    base = off.astype(np.int64)
    for q in range(2000):
        a = int(base[jq[q]] + sq[q])
        assert np.array_equal(xo[xoff[q]:xoff[q + 1]], text[a:a + int(ln[q])]), q
    dec.free()
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
