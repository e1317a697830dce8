"""lcg_export: the whole grammar in host memory in one call, equal to the
per-level copies and to the oracle's grammar rank for rank."""
import numpy as np
import pytest

from paper_2411_12439_amd import datagen as D

pytestmark = pytest.mark.gpu
SEED = D.HASH_SEED


@pytest.mark.parametrize("config,scale", [("tiny", 1.0), ("repeats", 0.0005)])
def test_export_equals_level_copies_and_oracle(config, scale):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from oracle import oracle as O
    from paper_2411_12439_amd import lcg
    text, off = D.make_config(config, scale=scale)
    t, o = lcg.to_device(text, off)
    g = lcg.build(t, o, seed=SEED)
    a, b = g.export_host(), g.export()
    want = O.build(text, off, SEED).export()
    for got in (a, want):
        assert len(got["levels"]) == len(b["levels"])
        for la, lb in zip(got["levels"], b["levels"]):
            for key in ("rhs_off", "rhs", "fp"):
                assert np.array_equal(la[key].astype(np.uint64), lb[key].astype(np.uint64)), key
        assert np.array_equal(got["c_level"], b["c_level"])
        assert np.array_equal(got["c_sym"], b["c_sym"])
    assert a["seed"] == b["seed"] == SEED


def test_export_without_levels():
    """A new grammar (no strings) and a grammar of one-byte strings have no
    levels; lcg_export still returns them whole."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from oracle import oracle as O
    from paper_2411_12439_amd import lcg
    h = lcg.new(SEED).export_host()
    assert h["seed"] == SEED and h["levels"] == []
    assert h["c_level"].size == 0 and h["c_sym"].size == 0
    strings = [b"A", b"C", b"A", b"T"]
    t, o = lcg.to_device(*O.pack(strings))
    g = lcg.build(t, o, seed=SEED)
    a, want = g.export_host(), O.build(*O.pack(strings), SEED).export()
    assert a["levels"] == [] and len(want["levels"]) == 0
    assert np.array_equal(a["c_level"], want["c_level"])
    assert np.array_equal(a["c_sym"], want["c_sym"])
    assert a["c_sym"].tolist() == [ord(x) for x in "ACAT"]
