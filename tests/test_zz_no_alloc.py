"""lcg_expand_strings_noalloc (the entry point that allocates no device memory)
against lcg_expand_strings, through the C ABI.

Two calls in a row share the library's fixed scratch: the second, over a
smaller range, must not see anything of the first.  The conditions of the
entry point are checked too: a grammar whose expansion lengths are not
current is refused, and so is a range whose working set exceeds the scratch,
before anything is written to the output."""
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


def _expect(g, j0, j1):
    out, offs = g.expand_strings(j0, j1)
    return out.cpu().numpy(), offs.cpu().numpy()


@pytest.mark.parametrize("name,scale", [("tiny", 1.0), ("bacterial", 0.05)])
def test_noalloc_equals_expand_strings_twice(L, name, scale):
    import torch
    text, off = D.make_config(name, scale=scale)
    strings = [text[off[j]:off[j + 1]].tobytes() for j in range(len(off) - 1)]
    strings += [b"A", b"GG", b"T" * 3000]
    from oracle import oracle as O
    text, off = O.pack(strings)
    t, o = L.to_device(text, off)
    g = L.build(t, o, seed=SEED)
    k = len(strings)
    want_all, want_off = _expect(g, 0, k)   # also prepares the expansion lengths
    for (j0, j1) in [(0, k), (1, k - 2)]:
        want, woff = _expect(g, j0, j1)
        n = int(woff[-1])
        out = torch.full((n + 64,), 0xAB, dtype=torch.uint8, device="cuda")
        offs = torch.full((j1 - j0 + 1,), -1, dtype=torch.int64, device="cuda")
        total = g.expand_strings_noalloc(out, offs, j0, j1)
        assert total == n
        got = out.cpu().numpy()
        assert np.array_equal(got[:n], want)
        assert np.all(got[n:] == 0xAB)
        assert np.array_equal(offs.cpu().numpy(), woff)
        a, b = int(off[j0]), int(off[j1])
        assert np.array_equal(got[:n], text[a:b])
    g.free()


def test_noalloc_needs_prepared_lengths(L):
    import torch
    text, off = D.make_config("tiny", scale=0.1)
    t, o = L.to_device(text, off)
    g = L.build(t, o, seed=SEED)
    out = torch.zeros(int(off[-1]), dtype=torch.uint8, device="cuda")
    with pytest.raises(L.LcgError) as e:
        g.expand_strings_noalloc(out)
    assert e.value.name == "LCG_EINVAL"
    g.expand_strings()
    assert g.expand_strings_noalloc(out) == int(off[-1])
    assert np.array_equal(out.cpu().numpy(), text)
    # the grammar changes: the lengths are stale again
    L.build_into(g, t, o)
    with pytest.raises(L.LcgError):
        g.expand_strings_noalloc(out)
    g.free()


def test_noalloc_refuses_a_range_beyond_the_scratch(L):
    import torch
    text, off = D.make_config("bacterial")
    t, o = L.to_device(text, off)
    g = L.build(t, o, seed=SEED)
    g.expand_strings()
    n = int(off[-1])
    out = torch.full((n,), 0x5A, dtype=torch.uint8, device="cuda")
    with pytest.raises(L.LcgError) as e:
        g.expand_strings_noalloc(out)
    assert e.value.name == "LCG_EINVAL" and "scratch" in str(e.value)
    assert bool((out == 0x5A).all())
    # a range that fits works right after the refusal
    want, woff = _expect(g, 3, 5)
    m = int(woff[-1])
    assert g.expand_strings_noalloc(out, None, 3, 5) == m
    assert np.array_equal(out[:m].cpu().numpy(), want)
    g.free()
