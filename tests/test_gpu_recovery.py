"""A failed lcg_build_into leaves the running grammar as it was.

The test hook fail_round makes the call fail when it reaches a given parsing
round, after the earlier rounds have added rules, claimed dictionary slots and
appended strings.  The grammar must come back exactly as before the call
(every level, C, the statistics), and a later call with the same strings must
give the oracle's grammar of all strings, rank for rank: no rule or claim of
the failed call survives in a dictionary (a stale claim would be found by an
exact-key probe and hand out a rank that does not exist).
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


@pytest.fixture(scope="module")
def halves():
    text, off = D.make_config("bacterial", scale=0.01)
    o = off.astype(np.int64)
    k = len(o) - 1
    h = k // 2
    a = (text[:o[h]], off[:h + 1])
    b = (text[o[h]:], (off[h:] - off[h]).astype(np.uint64))
    return a, b, (text, off)


# rounds reached with host reads (tail_log2 small) and queued without them
@pytest.mark.parametrize("tail_log2,fail_round,flags", [(8, 1, 0), (8, 2, 0), (8, 4, 0), (8, 9, 0),
                                                        (22, 1, 0), (22, 3, 0), (22, 10, 0),
                                                        (22, 3, 4), (8, 9, 4)])
def test_failed_build_into_restores_the_grammar(L, halves, tail_log2, fail_round, flags):
    from oracle import oracle as O
    (ta, oa), (tb, ob), (text, off) = halves
    da, doa = L.to_device(ta, oa)
    db, dob = L.to_device(tb, ob)
    g = L.build(da, doa, seed=SEED, tail_log2=tail_log2)
    before = g.export()
    n_stats = len(g.stats())
    with pytest.raises(L.LcgError) as e:
        L.build_into(g, db, dob, tail_log2=tail_log2, fail_round=fail_round, flags=flags)
    assert e.value.name == "LCG_ETABLE"
    after = g.export()
    assert CN.exports_equal(after, before), CN.first_difference(after, before)
    assert len(g.stats()) == n_stats
    # the same strings again, without the hook: the oracle's grammar of both halves
    first = L.build_into(g, db, dob, tail_log2=tail_log2)
    assert first == len(oa) - 1
    want = O.build(text, off, SEED).export()
    got = g.export()
    assert CN.exports_equal(got, want), CN.first_difference(got, want)
    out, _ = g.expand_strings()
    assert np.array_equal(out.cpu().numpy(), text)
    g.free()


def test_failed_build_into_on_an_empty_grammar(L, halves):
    from oracle import oracle as O
    (ta, oa), _, _ = halves
    da, doa = L.to_device(ta, oa)
    g = L.new(SEED)
    with pytest.raises(L.LcgError):
        L.build_into(g, da, doa, fail_round=2, tail_log2=8)
    assert g.info()[1:] == (0, 0)
    L.build_into(g, da, doa)
    want = O.build(ta, oa, SEED).export()
    assert CN.exports_equal(g.export(), want)
    g.free()
