"""Device memory from PyTorch's caching allocator (lcg_set_allocator).

With the hook installed, the library's blocks come from torch (torch's
accounting sees them), results are unchanged (the oracle's grammar, the input
back from decompression), and releasing the pool hands the blocks back to
torch; with the hook removed, hipMalloc serves again.
"""
import numpy as np
import pytest

from paper_2411_12439_amd import datagen as D

pytestmark = pytest.mark.gpu
SEED = D.HASH_SEED


@pytest.fixture
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2411_12439_amd import lcg
    lcg.lib()
    yield lcg
    lcg.use_torch_allocator(False)
    lcg.release_pool()


def _allocated():
    """torch's allocated bytes once earlier tests' garbage is gone (the suite
    shares one process)."""
    import gc
    import torch
    gc.collect()
    torch.cuda.synchronize()
    return torch.cuda.memory_allocated()


def test_torch_allocator_serves_the_library(L):
    import torch
    from oracle import oracle as O
    from paper_2411_12439_amd import canon as CN
    text, off = D.make_config("tiny")
    t, o = L.to_device(text, off)
    L.release_pool()
    L.use_torch_allocator(True)
    base = _allocated()
    g = L.build(t, o, seed=SEED)
    held = torch.cuda.memory_allocated() - base
    assert held > 0  # the grammar's levels and the pool's blocks are torch's
    assert CN.canon(g.export()) == CN.canon(O.build(text, off, SEED).export())
    out, offs = g.expand_strings()
    assert torch.equal(out, t)
    del out, offs  # torch tensors of the binding, not library blocks
    g.free()
    L.release_pool()
    assert _allocated() <= base  # every block went back to torch
    # back to hipMalloc: torch sees nothing of the next build
    L.use_torch_allocator(False)
    base2 = _allocated()
    g2 = L.build(t, o, seed=SEED)
    assert _allocated() <= base2
    assert CN.canon(g2.export()) == CN.canon(O.build(text, off, SEED).export())
    g2.free()
