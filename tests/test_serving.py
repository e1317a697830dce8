"""Serving form: ring allocator (CPU) and continuous batching into a running grammar (GPU)."""
import random

import numpy as np
import pytest

from paper_2411_12439_amd import datagen as D
from paper_2411_12439_amd.serve import RingBuffer


class _HostRing(RingBuffer):
    def __init__(self, n):  # no device buffer: allocation logic only
        self.cap = n
        self.head = self.tail = self.used = 0
        self.wrapped = False


@pytest.mark.parametrize("seed", range(6))
def test_ring_allocations_never_overlap(seed):
    r = _HostRing(100)
    live = []
    rng = random.Random(seed)
    for _ in range(20000):
        if live and rng.random() < 0.45:
            m = rng.randint(1, len(live))
            tot = sum(n for _, n in live[:m])
            live = live[m:]
            r.release(tot, live[0][0] if live else 0)
        else:
            n = rng.randint(1, 60)
            off = r.alloc(n)
            if off is not None:
                assert off + n <= 100
                for o2, n2 in live:
                    assert off + n <= o2 or o2 + n2 <= off
                live.append((off, n))
        assert r.used == sum(n for _, n in live)


def test_ring_rejects_oversized_request():
    with pytest.raises(ValueError):
        _HostRing(10).alloc(11)


@pytest.fixture(scope="module")
def served():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2411_12439_amd import serve
    src = D.ServingSource(scale=0.02, n_bases=4)
    # a high offered load so that requests queue up and batches form; a small
    # ring so that it wraps
    summary, srv, reqs = serve.run_load(src, load_gbps=5.0, seconds=30.0, max_requests=60,
                                        ring_bytes=4 << 20)
    return serve, src, summary, srv, reqs


@pytest.mark.gpu
def test_serving_completes_every_request(served):
    serve, src, summary, srv, reqs = served
    assert summary["requests"] == 60 == len(srv.completed)
    assert sum(srv.batch_sizes) == 60
    assert summary["max_batch"] >= 2, "no batch formed under load"
    assert summary["p99_ms"] >= summary["p50_ms"] > 0
    assert sorted(r.c_index for r, _ in reqs) == list(range(60))


@pytest.mark.gpu
def test_serving_warmup_is_served_but_not_measured():
    """Requests of the warm-up window are compressed like the others (every one
    completes and is in the running grammar) and only the later ones enter the
    summary."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2411_12439_amd import serve
    src = D.ServingSource(scale=0.02, n_bases=4)
    # about 80 requests per second: some 25 in each window
    summary, srv, reqs = serve.run_load(src, load_gbps=0.005, seconds=0.3, warmup_s=0.3,
                                        min_requests=10, max_requests=40)
    assert summary["warmup_requests"] > 0 and 10 <= summary["requests"] <= 40
    assert summary["requests"] + summary["warmup_requests"] == len(reqs) == len(srv.completed)
    assert sorted(r.c_index for r, _ in reqs) == list(range(len(reqs)))
    assert serve.check_alone_vs_mix(srv, src, reqs, range(len(reqs))) == len(reqs)
    srv.close()


@pytest.mark.gpu
def test_serving_alone_equals_in_the_mix(served):
    """Def. 1: each request's rules inside the running grammar == the request built alone."""
    serve, src, summary, srv, reqs = served
    assert serve.check_alone_vs_mix(srv, src, reqs, range(len(reqs))) == len(reqs)


@pytest.mark.gpu
def test_serving_round_trip(served):
    serve, src, summary, srv, reqs = served
    for req, desc in reqs[::7]:
        got = srv.g.expand(req.c_index).cpu().numpy()
        assert np.array_equal(got, src.host_bytes(desc))


@pytest.mark.gpu
def test_serving_grammar_equals_oracle_of_the_stream(served):
    """The running grammar equals (canonically) the oracle's grammar of all requests
    in completion order: incremental merging loses nothing and adds nothing."""
    from oracle import oracle as O
    from paper_2411_12439_amd import canon as CN
    serve, src, summary, srv, reqs = served
    order = sorted(reqs, key=lambda x: x[0].c_index)
    strings = [src.host_bytes(desc) for _, desc in order]
    text, off = D.pack(strings)
    want = O.build(text, off, D.HASH_SEED).export()
    got = srv.g.export()
    assert CN.canon(got) == CN.canon(want)


def test_requests_carry_their_own_divergence():
    """Each request is a window of a base copy with fresh substitutions
    (~0.9 %, every one a different base), drawn from the request id alone:
    the same descriptor gives the same bytes, two requests over the same
    window differ.  Checked on the CPU (the device uses the same recipe)."""
    src = D.ServingSource(scale=0.002, n_bases=2)
    rid, v, _, _ = src.draw()
    st = 1000
    desc = (rid, v, st, 60000)
    win = src.variants[v][st:st + 60000]
    a = src.materialize(desc, device="cpu").numpy()
    b = src.materialize(desc, device="cpu").numpy()
    c = src.materialize((rid + 1, v, st, 60000), device="cpu").numpy()
    assert np.array_equal(a, b)
    diff = a != win
    rate = diff.mean()
    assert 0.0075 < rate < 0.0105, rate
    assert set(np.unique(a[diff]).tolist()) <= set(b"ACGT")
    assert (a != c).mean() > 0.015          # fresh substitutions on both
    assert np.array_equal(a[~diff], win[~diff])


@pytest.mark.gpu
def test_serving_rotates_full_running_grammars():
    """A running grammar whose level reaches the rule limit is retired once its
    batches finish; later requests go to a new one.  Every request completes,
    and every request of the last running grammar equals itself built alone."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2411_12439_amd import serve
    src = D.ServingSource(scale=0.02, n_bases=4)
    # a 2 MB ring (requests are at most 1 MB here) admits about 1-2 MB per
    # batch, which fills a level past 3000 rules: about one batch per grammar
    summary, srv, reqs = serve.run_load(src, load_gbps=5.0, seconds=30.0, max_requests=160,
                                        ring_bytes=2 << 20, max_level_rules=3000)
    assert summary["requests"] == 160 == len(srv.completed)
    assert summary["generations"] >= 3
    last = serve.checkable(srv, reqs)
    assert last and serve.check_alone_vs_mix(srv, src, reqs, last) == len(last)
    # the last grammar's strings are its requests in C order
    assert sorted(reqs[i][0].c_index for i in last) == list(range(len(last)))
    srv.close()
