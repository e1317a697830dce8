"""Serving sessions (lcg_session_*): batches admitted between rounds of others.

Every batch's strings must come out as if compressed alone (stability, Def. 1:
each string's sub-grammar, renumbered in its own first-occurrence order,
equals the oracle's grammar of the string alone), the running grammar must
equal the oracle's grammar of all strings in C order up to a per-level
renaming (canonically), and a session whose batches never overlap must give
exactly the ranks of one build of all strings.
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


def _batches():
    """Three batches of uneven size: many rounds, a few, and tiny strings."""
    text, off = D.make_config("bacterial", scale=0.02)
    big = [text[off[j]:off[j + 1]].tobytes() for j in range(len(off) - 1)][:12]
    rng = np.random.default_rng(4)
    mid = [bytes(rng.choice(list(b"ACGT"), int(n)).tolist()) for n in (5000, 20000, 777)]
    small = [b"A", b"ACGT" * 9, b"G" * 1000, b"TTAGGG" * 30]
    return [big, mid, small]


def _check(L, g, strings):
    from oracle import oracle as O
    e = g.export()
    assert CN.canon(e) == CN.canon(O.build(*O.pack(strings), SEED).export())
    for j, s in enumerate(strings):
        alone = O.build(*O.pack([s]), SEED).export()
        mine = CN.own_order_subgrammar(e, j)
        assert CN.exports_equal(mine, alone), (j, CN.first_difference(mine, alone))
    out, _ = g.expand_strings()
    assert out.cpu().numpy().tobytes() == b"".join(strings)


@pytest.mark.parametrize("tail_log2", [8, 22])
@pytest.mark.parametrize("schedule", ["staggered", "late_small", "together"])
def test_session_batches_in_flight_together(L, tail_log2, schedule):
    batches = _batches()
    g = L.new(SEED)
    ss = L.Session(g, tail_log2=tail_log2)
    dev = [L.to_device(*D.pack([np.frombuffer(s, np.uint8) for s in b])) for b in batches]
    tickets, firsts, reported = [], [], []
    # when each batch is admitted: before the given step number
    admit_at = {"staggered": [0, 1, 3], "late_small": [0, 0, 2], "together": [0, 0, 0]}[schedule]
    step = 0
    pending = list(range(len(batches)))
    while pending or ss.active():
        while pending and admit_at[pending[0]] <= step:
            i = pending.pop(0)
            f, t = ss.admit(*dev[i])
            firsts.append(f)
            tickets.append(t)
        done, n_active = ss.step()
        reported += done
        step += 1
        assert step < 200
    assert sorted(reported) == sorted(tickets) and len(set(reported)) == len(tickets)
    assert firsts == [0, len(batches[0]), len(batches[0]) + len(batches[1])]
    strings = [s for b in batches for s in b]
    _check(L, g, strings)
    ss.free()
    g.free()


def test_session_without_overlap_gives_one_build_rank_for_rank(L):
    """Batches admitted only when the session is idle: the ranks of a single
    build of all strings (first occurrence), the oracle's exactly."""
    from oracle import oracle as O
    batches = _batches()
    g = L.new(SEED)
    ss = L.Session(g, tail_log2=8)
    for b in batches:
        ss.admit(*L.to_device(*D.pack([np.frombuffer(s, np.uint8) for s in b])))
        while ss.active():
            ss.step()
    strings = [s for b in batches for s in b]
    want = O.build(*O.pack(strings), SEED).export()
    got = g.export()
    assert CN.exports_equal(got, want), CN.first_difference(got, want)
    ss.free()
    g.free()


def test_session_budget_admission(L):
    """A batch that does not fit beside the active ones is refused (nothing
    admitted) and fits once they are done."""
    batches = _batches()
    need0 = L.build_bytes(sum(len(s) for s in batches[0]), len(batches[0]))
    need2 = L.build_bytes(sum(len(s) for s in batches[2]), len(batches[2]))
    g = L.new(SEED)
    ss = L.Session(g, hbm_budget=need0 + need2 // 2, tail_log2=8)
    d0 = L.to_device(*D.pack([np.frombuffer(s, np.uint8) for s in batches[0]]))
    d2 = L.to_device(*D.pack([np.frombuffer(s, np.uint8) for s in batches[2]]))
    ss.admit(*d0)
    with pytest.raises(L.LcgError) as e:
        ss.admit(*d2)
    assert e.value.name == "LCG_ENOMEM"
    assert g.info()[2] == len(batches[0])
    while ss.active():
        ss.step()
    ss.admit(*d2)
    while ss.active():
        ss.step()
    _check(L, g, batches[0] + batches[2])
    ss.free()
    g.free()
