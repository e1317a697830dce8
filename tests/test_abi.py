"""The C-ABI library loads and exports every symbol include/lcg.h declares (no GPU calls)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lcg.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lcg_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lcgmod():
    from paper_2411_12439_amd import lcg
    if not os.path.exists(lcg.LIB_PATH):
        from paper_2411_12439_amd import build_lib
        build_lib.build()
    return lcg


def test_header_declares_the_binding_exports():
    from paper_2411_12439_amd import lcg
    assert _declared() == sorted(lcg.EXPORTS)


def test_library_exports_every_declared_symbol(lcgmod):
    L = lcgmod.lib()
    for name in _declared():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", lcgmod.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    syms = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for name in _declared():
        assert name in syms, name


def test_host_only_entry_points(lcgmod):
    """Calls that touch no device: defaults, error reporting, sizing."""
    o = lcgmod.make_opts(seed=5)
    assert o.mode == lcgmod.MODE_BATCHED and o.seed == 5
    assert lcgmod.build_bytes(1000, 2) >= 17 * 1000
    g = lcgmod.new(42)
    assert g.info() == (42, 0, 0)
    assert g.level_sizes() == []
    assert g.stats().shape == (0, lcgmod.STATS_FIELDS)
    with pytest.raises(lcgmod.LcgError) as e:
        lcgmod._check(lcgmod.lib().lcg_level_size(g.h, 1, None, None))
    assert e.value.name == "LCG_EINVAL"
    # post-processing a grammar without strings is refused before any device work
    import ctypes
    h = ctypes.c_void_p()
    assert lcgmod.lib().lcg_postprocess(g.h, 3, None, ctypes.byref(h)) == -1 and not h.value
    assert lcgmod.lib().lcg_postprocess(g.h, 8, None, ctypes.byref(h)) == -1
    # stored files: missing arguments, sizes that cannot hold a header, misalignment
    L = lcgmod.lib()
    n = ctypes.c_uint64()
    assert L.lcg_slp_encode(None, None, 0, ctypes.byref(n), None) == -1
    assert L.lcg_slp_decode(None, 64, None, ctypes.byref(h)) == -1
    for ptr, size in ((8, 40), (8, 70), (9, 64)):
        assert L.lcg_slp_decode(ctypes.c_void_p(ptr), size, None, ctypes.byref(h)) == -1
        assert not h.value
    assert b"stored grammar" in L.lcg_last_error() or b"aligned" in L.lcg_last_error()
    # an allocator needs both functions; NULL restores hipMalloc
    half = lcgmod.Allocator(lcgmod._ALLOC_FN(lambda n, c: None), lcgmod._FREE_FN(), None)
    assert L.lcg_set_allocator(ctypes.byref(half)) == -1
    assert L.lcg_set_allocator(None) == 0
    # host export: a NULL grammar is refused and leaves the result empty
    hg = lcgmod.HostGrammar()
    assert L.lcg_export(None, ctypes.byref(hg)) == -1 and hg.n_levels == 0 and not hg.levels
    L.lcg_host_free(None)
    L.lcg_host_free(ctypes.byref(hg))
    g.free()


def test_product_path_has_no_fallback():
    """The binding refuses to run without the HIP library instead of computing elsewhere."""
    import importlib
    from paper_2411_12439_amd import lcg
    src = open(lcg.__file__).read()
    assert "oracle" not in src
    mod = importlib.import_module("paper_2411_12439_amd.lcg")
    saved_path, saved_lib = mod.LIB_PATH, mod._lib
    try:
        mod.LIB_PATH = "/nonexistent/liblcg.so"
        mod._lib = None
        with pytest.raises(RuntimeError):
            mod.lib()
    finally:
        mod.LIB_PATH, mod._lib = saved_path, saved_lib
