"""lcg_reserve: dictionary room reserved ahead changes no result.

A running grammar built with reserved room (on an empty grammar, where the
levels do not exist yet, and on a grammar whose levels do exist, which then
grow at once) must be the oracle's grammar of all its strings, rank for rank,
exactly as without the reservation.
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
def parts():
    text, off = D.make_config("bacterial", scale=0.01)
    o = off.astype(np.int64)
    k = len(o) - 1
    cuts = [0, k // 3, 2 * k // 3, k]
    out = []
    for a, b in zip(cuts, cuts[1:]):
        out.append((text[o[a]:o[b]], (off[a:b + 1] - off[a]).astype(np.uint64)))
    return out, (text, off)


@pytest.mark.parametrize("when", ["empty", "after_first"])
@pytest.mark.parametrize("tail_log2", [8, 22])
def test_reserved_room_changes_nothing(L, parts, when, tail_log2):
    from oracle import oracle as O
    pieces, (text, off) = parts
    g = L.new(SEED)
    if when == "empty":
        g.reserve([1 << 12, 1 << 16, 1 << 16, 1 << 14, 0, 1 << 10])
    for i, (t, o) in enumerate(pieces):
        L.build_into(g, *L.to_device(t, o), tail_log2=tail_log2)
        if when == "after_first" and i == 0:
            # existing levels grow now (their rules are rehashed), later ones when created
            g.reserve([0, 1 << 18, 1 << 17, 1 << 15] + [1 << 12] * 10)
    want = O.build(text, off, SEED).export()
    got = g.export()
    assert CN.exports_equal(got, want), CN.first_difference(got, want)
    out, _ = g.expand_strings()
    assert np.array_equal(out.cpu().numpy(), text)
    g.free()


def test_reserve_errors(L):
    g = L.new(SEED)
    with pytest.raises(L.LcgError) as e:
        g.reserve([0, (1 << 30) + 1])
    assert e.value.name == "LCG_ETABLE"
    with pytest.raises(L.LcgError) as e:
        g.reserve([1] * 65)
    assert e.value.name == "LCG_EINVAL"
    g.reserve([])               # nothing to do
    g.reserve([0, 0, 0])
    assert g.info()[1:] == (0, 0)   # no level created, no string
    g.free()
