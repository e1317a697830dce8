"""Streaming builds from a file (lcg_build_file, and lcg_build_file_sink with
its sink in host memory and flush cycles) against the oracle's build of the
same strings.

Ranks are numbered by first occurrence (string order, then position), so
compressing the file chunk by chunk into a running grammar must give the
oracle's grammar of all of its lines in file order, rank for rank (and the
library's one-call build of them).
"""
import os
import tempfile

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


def _strings(text, off):
    o = off.astype(np.int64)
    return [text[o[j]:o[j + 1]].tobytes() for j in range(len(o) - 1)]


def _write(strings, trailing_newline=True):
    fd, path = tempfile.mkstemp(suffix=".txt")
    with os.fdopen(fd, "wb") as f:
        f.write(b"\n".join(strings))
        if trailing_newline:
            f.write(b"\n")
    return path


def _assert_same(a, b):
    assert len(a["levels"]) == len(b["levels"])
    for la, lb in zip(a["levels"], b["levels"]):
        assert np.array_equal(la["rhs_off"], lb["rhs_off"])
        assert np.array_equal(la["rhs"], lb["rhs"])
        assert np.array_equal(la["fp"], lb["fp"])
    assert np.array_equal(a["c_level"], b["c_level"])
    assert np.array_equal(a["c_sym"], b["c_sym"])


@pytest.mark.parametrize("chunk,trailing", [(300 << 10, True), (1 << 20, False), (64 << 20, True)])
def test_file_equals_one_build(L, chunk, trailing):
    from oracle import oracle as O
    text, off = D.make_config("tiny")
    strings = _strings(text, off) + [b"A", b"ACGT" * 100, b"T" * 5000]
    path = _write(strings, trailing)
    try:
        g = L.new(SEED)
        info = L.build_file(g, path, chunk_bytes=chunk)
        got = g.export()
        _assert_same(got, O.build(*O.pack(strings), SEED).export())
        t, o = L.to_device(*O.pack(strings))
        _assert_same(got, L.build(t, o, seed=SEED).export())
        assert info["strings"] == len(strings)
        assert info["bytes"] == sum(len(s) for s in strings)
        if chunk == 300 << 10:
            assert info["chunks"] > 3
    finally:
        os.unlink(path)


def test_file_into_existing_grammar(L):
    from oracle import oracle as O
    text, off = D.make_config("bacterial", scale=0.01)
    strings = _strings(text, off)
    half = len(strings) // 2
    path = _write(strings[half:])
    try:
        ta, oa = L.to_device(*O.pack(strings[:half]))
        g = L.build(ta, oa, seed=SEED)
        L.build_file(g, path, chunk_bytes=200 << 10)
        _assert_same(g.export(), O.build(*O.pack(strings), SEED).export())
        # and the whole collection expands back from the streamed grammar
        out, offs = g.expand_strings()
        assert np.array_equal(out.cpu().numpy(), O.pack(strings)[0])
    finally:
        os.unlink(path)


def test_file_errors(L):
    g = L.new(SEED)
    with pytest.raises(L.LcgError) as e:
        L.build_file(g, "/nonexistent/collection.txt")
    assert e.value.name == "LCG_EINVAL"
    path = _write([b"ACGT", b"", b"GG"])
    try:
        with pytest.raises(L.LcgError) as e:
            L.build_file(L.new(SEED), path, chunk_bytes=4096)
        assert e.value.name == "LCG_EINVAL"
    finally:
        os.unlink(path)
    path = _write([b"A" * 10000, b"C"])
    try:
        with pytest.raises(L.LcgError) as e:
            L.build_file(L.new(SEED), path, chunk_bytes=4096)
        assert e.value.name == "LCG_EINVAL"
    finally:
        os.unlink(path)
    fd, path = tempfile.mkstemp()
    os.close(fd)
    try:
        g = L.new(SEED)
        info = L.build_file(g, path, chunk_bytes=4096)
        assert info["strings"] == 0 and g.info()[2] == 0
    finally:
        os.unlink(path)


@pytest.mark.parametrize("buffer_bytes", [0, 48 << 20, 1 << 40])
def test_sink_flush_cycles_equal_the_oracle(L, buffer_bytes):
    """lcg_build_file_sink: the sink's levels wait in host memory while chunks
    go into a buffer grammar, merged into the sink whenever it holds
    buffer_bytes of device memory (0: after every chunk; a huge value: once, at
    the end).  The sink, non-empty at the start, ends with the oracle's
    grammar of all strings, rank for rank."""
    from oracle import oracle as O
    text, off = D.make_config("bacterial", scale=0.01)
    strings = _strings(text, off)
    first = len(strings) // 4
    path = _write(strings[first:])
    try:
        ta, oa = L.to_device(*O.pack(strings[:first]))
        g = L.build(ta, oa, seed=SEED)
        info = L.build_file_sink(g, path, buffer_bytes, chunk_bytes=200 << 10)
        print(info, flush=True)
        assert info["strings"] == len(strings) - first
        if buffer_bytes == 0:
            assert info["flushes"] == info["chunks"] >= 4
        elif buffer_bytes == 1 << 40:
            assert info["flushes"] == 1
        else:
            assert 1 <= info["flushes"] <= info["chunks"]
        _assert_same(g.export(), O.build(*O.pack(strings), SEED).export())
        out, offs = g.expand_strings()
        assert np.array_equal(out.cpu().numpy(), O.pack(strings)[0])
        g.free()
    finally:
        os.unlink(path)


def test_sink_errors(L):
    from oracle import oracle as O
    text, off = D.make_config("tiny", scale=0.05)
    strings = _strings(text, off)
    ta, oa = L.to_device(*O.pack(strings))
    g = L.build(ta, oa, seed=SEED)
    before = g.export()
    # refused before anything streams: the sink is untouched and usable
    with pytest.raises(L.LcgError) as e:
        L.build_file_sink(g, "/nonexistent/collection.txt", 0)
    assert e.value.name == "LCG_EINVAL"
    _assert_same(g.export(), before)
    # an empty file: no flush, nothing changes
    fd, path = tempfile.mkstemp()
    os.close(fd)
    try:
        info = L.build_file_sink(g, path, 0, chunk_bytes=4096)
        assert info["strings"] == 0 and info["flushes"] == 0
        _assert_same(g.export(), before)
    finally:
        os.unlink(path)
    # a bad line after the first flushes: the sink is refused from then on
    path = _write([b"ACGTACGTAC" * 100] * 20 + [b""] + [b"GG"])
    try:
        with pytest.raises(L.LcgError) as e:
            L.build_file_sink(g, path, 0, chunk_bytes=4096)
        assert e.value.name == "LCG_EINVAL"
        with pytest.raises(L.LcgError):
            g.export()
    finally:
        os.unlink(path)
