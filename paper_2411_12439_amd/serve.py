"""Serving form: continuous batching of compression requests into one running grammar.

Requests (one byte string each) arrive over time.  Each is written, on a
copy stream, into a device ring buffer as soon as it arrives (synthesized
there by the request source), overlapping the build running on the compute
stream.  Whenever the GPU is free the scheduler
admits the uploaded requests that fit the HBM budget -- a contiguous range of
the ring, so the batch needs no gather -- and compresses the whole batch into
the running grammar with one ``lcg_build_into`` call (BuildGram with a
read-first dictionary, App. A.2 of the paper): phrases already in the running
grammar are reused and new ones appended, i.e. the batch is merged
incrementally.  Requests arriving meanwhile wait for the next step.  A
request's latency runs from its arrival to the end of the step that
compressed it, when its entry of C is final.

Stability (Def. 1) makes each request's result independent of its batch and of
the running grammar: the rules reachable from its C entry equal the grammar of
the request built alone.  ``check_alone_vs_mix`` verifies that on the device.
"""
import collections
import time

import numpy as np

from . import canon as _canon
from . import datagen as _datagen
from . import lcg as _lcg


class RingBuffer:
    """Device byte ring with FIFO release; every allocation is contiguous."""

    def __init__(self, nbytes, device="cuda"):
        import torch
        self.buf = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
        self.cap = int(nbytes)
        self.head = 0          # next byte to allocate
        self.tail = 0          # first byte of the oldest live allocation
        self.used = 0          # live bytes
        self.wrapped = False   # live data is [tail, end) + [0, head) instead of [tail, head)

    def alloc(self, n):
        """Offset of n free contiguous bytes, or None when full."""
        if n > self.cap:
            raise ValueError("request of %d bytes exceeds the ring (%d)" % (n, self.cap))
        if self.used == 0:
            self.head = self.tail = 0
            self.wrapped = False
        if not self.wrapped:
            if self.cap - self.head >= n:
                off = self.head
            elif self.tail >= n:                # restart at 0, ending before tail
                off = 0
                self.wrapped = True
            else:
                return None
        elif self.tail - self.head >= n:
            off = self.head
        else:
            return None
        self.head = off + n
        self.used += n
        return off

    def release(self, n, next_tail):
        """Release the oldest n live bytes; next_tail starts the oldest remaining one."""
        self.used -= n
        if self.used == 0:
            self.head = self.tail = 0
            self.wrapped = False
            return
        if self.wrapped and next_tail < self.tail:
            self.wrapped = False
        self.tail = next_tail


class Request:
    __slots__ = ("rid", "desc", "n", "arrival", "off", "event", "done", "c_index")

    def __init__(self, rid, desc, arrival):
        self.rid = rid
        self.desc = desc          # the source's descriptor (request id, copy, start, length)
        self.n = int(desc[3])
        self.arrival = arrival
        self.off = None
        self.event = None
        self.done = None
        self.c_index = None


class Server:
    """Continuous-batching compressor around one device-resident running grammar."""

    def __init__(self, source, seed=_datagen.HASH_SEED, hbm_budget=16 << 30, ring_bytes=1 << 30,
                 device="cuda"):
        import torch
        self.torch = torch
        self.source = source
        self.seed = seed
        self.g = _lcg.new(seed)
        self.budget = int(hbm_budget)
        self.ring = RingBuffer(ring_bytes, device)
        self.copy_stream = torch.cuda.Stream()
        self.waiting = collections.deque()   # arrived; the ring had no room yet
        self.ready = collections.deque()     # uploaded (or uploading), not compressed
        self.completed = []
        self.batch_sizes = []

    def close(self):
        """Free the running grammar."""
        self.g.free()

    def submit(self, req):
        self.waiting.append(req)
        self.upload()

    def upload(self):
        """Start the uploads of waiting requests while the ring has room."""
        torch = self.torch
        while self.waiting:
            req = self.waiting[0]
            off = self.ring.alloc(req.n)
            if off is None:
                return
            self.waiting.popleft()
            req.off = off
            with torch.cuda.stream(self.copy_stream):
                self.source.materialize(req.desc, out=self.ring.buf[off:off + req.n])
                req.event = torch.cuda.Event()
                req.event.record(self.copy_stream)
            self.ready.append(req)

    def step(self):
        """Compress the admissible prefix of the uploaded requests; returns its size."""
        torch = self.torch
        if not self.ready:
            return 0
        batch = []
        total = 0
        start = self.ready[0].off
        for req in self.ready:
            if req.off != start + total:   # the ring wrapped: next step
                break
            if batch and _lcg.build_bytes(total + req.n, len(batch) + 1) > self.budget:
                break
            batch.append(req)
            total += req.n
        for _ in batch:
            self.ready.popleft()
        cur = torch.cuda.current_stream()
        for req in batch:
            cur.wait_event(req.event)
        offs = np.zeros(len(batch) + 1, np.int64)
        offs[1:] = np.cumsum([r.n for r in batch])
        d_offs = torch.from_numpy(offs).to(self.ring.buf.device)
        first = _lcg.build_into(self.g, self.ring.buf[start:start + total], d_offs,
                                seed=self.seed, hbm_budget=self.budget)
        now = time.perf_counter()
        for i, req in enumerate(batch):
            req.done = now
            req.c_index = first + i
            self.completed.append(req)
        self.ring.release(total, self.ready[0].off if self.ready else 0)
        self.batch_sizes.append(len(batch))
        self.upload()
        return len(batch)


def run_load(source, load_gbps, seconds, max_requests=None, seed=_datagen.HASH_SEED,
             hbm_budget=16 << 30, ring_bytes=1 << 30):
    """Serve a Poisson stream offering `load_gbps` GB/s for `seconds` (or max_requests).

    Returns (summary, server, requests); requests[i] = (Request, descriptor).
    """
    import torch
    srv = Server(source, seed, hbm_budget, ring_bytes)
    gaps = source.arrivals(load_gbps * 1e9, 1 << 16)
    reqs = []
    t0 = time.perf_counter()
    nxt = t0 + gaps[0]
    i = 0
    while True:
        now = time.perf_counter()
        open_ = now - t0 < seconds and (max_requests is None or i < max_requests)
        while open_ and nxt <= now:
            desc = source.draw()
            r = Request(i, desc, nxt)
            srv.submit(r)
            reqs.append((r, desc))
            i += 1
            nxt += gaps[i % len(gaps)]
            open_ = max_requests is None or i < max_requests
        if srv.ready:
            srv.step()
            continue
        if srv.waiting:
            srv.upload()
            continue
        if not open_:
            break
        time.sleep(max(0.0, min(nxt - time.perf_counter(), 0.0005)))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    done = [r for r, _ in reqs]
    lat = np.array([(r.done - r.arrival) * 1e3 for r in done]) if done else np.zeros(1)
    nbytes = sum(r.n for r in done)
    start = min((r.arrival for r in done), default=t0)
    summary = {
        "offered_gbps": load_gbps,
        "requests": len(done),
        "bytes": int(nbytes),
        "sustained_gbps": round(nbytes / max(t1 - start, 1e-9) / 1e9, 4),
        "p50_ms": round(float(np.percentile(lat, 50)), 3),
        "p99_ms": round(float(np.percentile(lat, 99)), 3),
        "steps": len(srv.batch_sizes),
        "mean_batch": round(float(np.mean(srv.batch_sizes)), 2) if srv.batch_sizes else 0.0,
        "max_batch": int(max(srv.batch_sizes)) if srv.batch_sizes else 0,
        "wall_s": round(t1 - t0, 3),
    }
    return summary, srv, reqs


def check_alone_vs_mix(srv, source, reqs, sample):
    """For the sampled requests: rules reachable from the request's C entry in the
    running grammar == the grammar of the request compressed alone (canonically)."""
    import torch
    g_all = srv.g.export()
    ok = 0
    for idx in sample:
        req, desc = reqs[idx]
        t = source.materialize(desc)
        o = torch.tensor([0, req.n], dtype=torch.int64, device=t.device)
        alone = _lcg.build(t, o, seed=srv.seed).export()
        sub = _canon.subgrammar(g_all, [req.c_index])
        if _canon.canon(sub) != _canon.canon(alone):
            raise AssertionError("request %d differs alone vs in the mix" % req.rid)
        ok += 1
    return ok


def main():
    import argparse
    import json
    ap = argparse.ArgumentParser(description="serving-form benchmark (one JSON line per load)")
    ap.add_argument("--loads", default="0.5,2,8")
    ap.add_argument("--seconds", type=float, default=10.0)
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--check", type=int, default=8, help="requests checked alone vs in the mix")
    args = ap.parse_args()
    src = _datagen.ServingSource(scale=args.scale)
    for load in (float(x) for x in args.loads.split(",")):
        summary, srv, reqs = run_load(src, load, args.seconds)
        rng = np.random.default_rng(0)
        sample = rng.choice(len(reqs), size=min(args.check, len(reqs)), replace=False)
        summary["alone_vs_mix_checked"] = check_alone_vs_mix(srv, src, reqs, sample)
        print(json.dumps(summary), flush=True)


if __name__ == "__main__":
    main()
