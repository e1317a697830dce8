"""Maximal exact matches through the grammar (lcg_mems, App. B's MEM sketch)
against the oracle, match for match: pairs of strings from one base and from
different bases, a string against itself, every level from 1 to the strings'
top, short and long minimum lengths, a repeat inside one string, the output
capacity, and the argument errors; and the batched call (lcg_mems_batch),
pair by pair against the oracle and the single-pair call."""
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


def _both(L, text, off):
    from oracle import oracle as O
    t, o = L.to_device(text, off)
    return L.build(t, o, seed=SEED), O.build(text, off, SEED)


def _same(g, og, text, off, a, b, level, min_len):
    pa, pb, ln = g.mems(a, b, level, min_len)
    wa, wb, wl = og.mems(text, off, a, b, level, min_len)
    got = np.stack([x.cpu().numpy().astype(np.uint64) for x in (pa, pb, ln)])
    want = np.stack([wa, wb, wl])
    assert got.shape == want.shape, (a, b, level, min_len, got.shape, want.shape)
    assert np.array_equal(got, want), (a, b, level, min_len)
    return got.shape[1]


@pytest.mark.parametrize("config,scale,pairs", [
    ("tiny", 0.05, [(0, 1), (2, 7), (5, 5), (7, 0)]),
    ("bacterial", 0.01, [(0, 4), (1, 2), (9, 9), (63, 3)]),
])
def test_mems_equal_oracle(L, config, scale, pairs):
    text, off = D.make_config(config, scale=scale)
    g, og = _both(L, text, off)
    cl = g.export()["c_level"]
    total = 0
    for a, b in pairs:
        top = int(min(cl[a], cl[b]))
        for level in sorted({1, 2, 3, top}):
            if level > top:
                continue
            for min_len in (1, 24, 200):
                print("pair %d %d level %d min_len %d" % (a, b, level, min_len), flush=True)
                total += _same(g, og, text, off, a, b, level, min_len)
    assert total > 0
    g.free()


def test_mems_of_a_repeat_and_ragged_strings(L):
    rng = np.random.default_rng(21)
    x = rng.choice(list(b"ACGT"), 3000).astype(np.uint8).tobytes()
    z = rng.choice(list(b"ACGT"), 700).astype(np.uint8).tobytes()
    y = bytearray(x)
    for p in rng.integers(0, len(y), 30):
        y[p] = ord("A") if y[p] != ord("A") else ord("C")
    strings = [x + z + x, bytes(y), b"AC" * 900 + x[:500], b"T" * 2000, x[1000:1777]]
    from oracle import oracle as O
    text, off = O.pack(strings)
    g, og = _both(L, text, off)
    cl = g.export()["c_level"]
    for a, b in [(0, 0), (0, 1), (1, 0), (2, 0), (3, 3), (4, 0), (2, 2)]:
        for level in range(1, int(min(cl[a], cl[b])) + 1):
            for min_len in (1, 50):
                _same(g, og, text, off, a, b, level, min_len)
    g.free()


def test_mems_capacity(L):
    import ctypes
    import torch
    text, off = D.make_config("bacterial", scale=0.01)
    g, og = _both(L, text, off)
    wa, wb, wl = og.mems(text, off, 0, 4, 1, 10)
    assert len(wa) > 10
    lib = L.lib()
    cap = 7
    out = [torch.zeros(cap, dtype=torch.int64, device="cuda") for _ in range(3)]
    n = ctypes.c_uint64()
    rc = lib.lcg_mems(g.h, 0, 4, 1, 10, cap, *(ctypes.c_void_p(t.data_ptr()) for t in out),
                      ctypes.byref(n), None)
    assert rc == 0 and n.value == len(wa)
    assert np.array_equal(out[0].cpu().numpy().astype(np.uint64), wa[:cap])
    assert np.array_equal(out[1].cpu().numpy().astype(np.uint64), wb[:cap])
    assert np.array_equal(out[2].cpu().numpy().astype(np.uint64), wl[:cap])
    # a count only
    rc = lib.lcg_mems(g.h, 0, 4, 1, 10, 0, None, None, None, ctypes.byref(n), None)
    assert rc == 0 and n.value == len(wa)
    g.free()


def test_mems_bad_arguments(L):
    text, off = D.make_config("tiny", scale=0.05)
    g, og = _both(L, text, off)
    cl = g.export()["c_level"]
    k = len(off) - 1
    for args in [(0, k, 1, 1), (k, 0, 1, 1), (0, 1, 0, 1), (0, 1, int(min(cl[0], cl[1])) + 1, 1)]:
        with pytest.raises(L.LcgError) as e:
            g.mems(*args)
        assert e.value.name == "LCG_EINVAL"
    g.free()


def test_batch_equals_the_oracle_pair_by_pair(L):
    """One lcg_mems_batch call over pairs that share strings, repeat, and put
    one string on both sides: every pair's matches equal the oracle's, and the
    single-pair call's, in (pair, start in a, start in b) order."""
    text, off = D.make_config("bacterial", scale=0.01)
    g, og = _both(L, text, off)
    pairs = [(0, 4), (4, 0), (1, 2), (9, 9), (0, 4), (63, 3), (5, 9), (2, 1)]
    a = [p[0] for p in pairs]
    b = [p[1] for p in pairs]
    for level, min_len in [(2, 24), (3, 1), (1, 60)]:
        pr, pa, pb, ln = (x.cpu().numpy() for x in g.mems_batch(a, b, level, min_len))
        assert np.all(np.diff(pr) >= 0)
        for p, (x, y) in enumerate(pairs):
            sel = pr == p
            got = np.stack([pa[sel], pb[sel], ln[sel]]).astype(np.uint64)
            want = np.stack(og.mems(text, off, x, y, level, min_len))
            assert np.array_equal(got, want), (p, x, y, level, min_len)
            one = np.stack([t.cpu().numpy() for t in g.mems(x, y, level, min_len)]).astype(np.uint64)
            assert np.array_equal(got, one), (p, x, y, level)
    g.free()


def test_batch_capacity_and_errors(L):
    import ctypes
    import torch
    text, off = D.make_config("tiny", scale=0.05)
    g, og = _both(L, text, off)
    a = np.array([0, 1, 2], np.uint32)
    b = np.array([1, 2, 0], np.uint32)
    pr, pa, pb, ln = (x.cpu().numpy() for x in g.mems_batch(a, b, 1, 10))
    assert len(pa) > 5
    lib = L.lib()
    cap = 5
    out = [torch.zeros(cap, dtype=torch.int64, device="cuda") for _ in range(3)]
    pair = torch.zeros(cap, dtype=torch.int32, device="cuda")
    n = ctypes.c_uint64()
    rc = lib.lcg_mems_batch(g.h, 3, a.ctypes.data_as(ctypes.c_void_p),
                            b.ctypes.data_as(ctypes.c_void_p), 1, 10, cap,
                            ctypes.c_void_p(pair.data_ptr()),
                            *(ctypes.c_void_p(t.data_ptr()) for t in out), ctypes.byref(n), None)
    assert rc == 0 and n.value == len(pa)
    assert np.array_equal(pair.cpu().numpy(), pr[:cap])
    assert np.array_equal(out[0].cpu().numpy(), pa[:cap])
    assert np.array_equal(out[2].cpu().numpy(), ln[:cap])
    # no pairs: nothing, no error
    rc = lib.lcg_mems_batch(g.h, 0, None, None, 1, 10, 0, None, None, None, None, ctypes.byref(n),
                            None)
    assert rc == 0 and n.value == 0
    k = len(off) - 1
    with pytest.raises(L.LcgError) as e:
        g.mems_batch([0, k], [1, 0], 1, 10)
    assert e.value.name == "LCG_EINVAL"
    rc = lib.lcg_mems_batch(g.h, 2, None, None, 1, 10, 0, None, None, None, None, ctypes.byref(n),
                            None)
    assert rc == -1  # LCG_EINVAL: NULL pair arrays
    g.free()
