"""Serving form: continuous batching of compression requests into one running grammar.

Requests (one byte string each) arrive over time.  Each is written, on a copy
stream, into a device ring buffer as soon as it arrives (synthesized there by
the request source), overlapping the rounds running on the compute stream.
The scheduler loop alternates two things:

* admit: the requests already in the ring that fit the HBM budget (and the
  cap on batches in flight) become one new batch of a serving session
  (``lcg_session_admit``), starting at parsing round 1;
* step: every batch in flight advances by one parsing round
  (``lcg_session_step``); a batch whose sequence is short runs all its
  remaining rounds in that step.

So a request that arrives while a large one is deep in its rounds waits for
at most one round of the others, not for their whole builds: batches at
different rounds share the GPU, each round of each batch looking up and
extending the running grammar's dictionary of its level (BuildGram against a
grammar being extended, App. A.2 of the paper).  A request's latency runs
from its arrival to the end of the step that finished its batch, when its
entry of C is final.

Stability (Def. 1) makes each request's result independent of its batch, of
the other batches and of the running grammar: the rules reachable from its C
entry equal the grammar of the request built alone.  ``check_alone_vs_mix``
verifies that on the device.
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


class Batch:
    """Requests admitted together (a contiguous span of the ring)."""
    __slots__ = ("reqs", "start", "nbytes", "ticket", "finished")

    def __init__(self, reqs, start, nbytes, ticket):
        self.reqs = reqs
        self.start = start
        self.nbytes = nbytes
        self.ticket = ticket
        self.finished = False


class Server:
    """Continuous-batching compressor around one device-resident running grammar."""

    def __init__(self, source, seed=_datagen.HASH_SEED, hbm_budget=16 << 30, ring_bytes=1 << 30,
                 max_batches=32, device="cuda"):
        import torch
        self.torch = torch
        self.source = source
        self.seed = seed
        self.g = _lcg.new(seed)
        self.budget = int(hbm_budget)
        self.session = _lcg.Session(self.g, hbm_budget=self.budget)
        self.max_batches = max_batches
        self.ring = RingBuffer(ring_bytes, device)
        self.copy_stream = torch.cuda.Stream()
        self.waiting = collections.deque()   # arrived; the ring had no room yet
        self.ready = collections.deque()     # uploaded (or uploading), not admitted
        self.inflight = collections.deque()  # admitted batches, in admission order
        self.by_ticket = {}
        self.completed = []
        self.batch_sizes = []
        self.steps = 0

    def close(self):
        """Free the session and the running grammar."""
        self.session.free()
        self.g.free()

    def submit(self, req):
        self.waiting.append(req)
        self.upload()

    def upload(self):
        """Start writing waiting requests into the ring while it has room."""
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

    def admit(self):
        """Admit the admissible prefix of the ready requests as one batch."""
        torch = self.torch
        if not self.ready or len(self.inflight) >= self.max_batches:
            return 0
        batch = []
        total = 0
        start = self.ready[0].off
        for req in self.ready:
            if req.off != start + total:   # the ring wrapped: next batch
                break
            if self.budget and batch and \
                    _lcg.build_bytes(total + req.n, len(batch) + 1) > self.budget:
                break
            batch.append(req)
            total += req.n
        cur = torch.cuda.current_stream()
        for req in batch:
            cur.wait_event(req.event)
        offs = np.zeros(len(batch) + 1, np.int64)
        offs[1:] = np.cumsum([r.n for r in batch])
        d_offs = torch.from_numpy(offs).to(self.ring.buf.device)
        try:
            first, ticket = self.session.admit(self.ring.buf[start:start + total], d_offs)
        except _lcg.LcgError as e:
            if e.name == "LCG_ENOMEM" and self.inflight:
                return 0                   # waits for memory to free up
            raise
        for _ in batch:
            self.ready.popleft()
        for i, req in enumerate(batch):
            req.c_index = first + i
        b = Batch(batch, start, total, ticket)
        self.inflight.append(b)
        self.by_ticket[ticket] = b
        self.batch_sizes.append(len(batch))
        return len(batch)

    def step(self):
        """Admit what fits, then one round of every batch in flight; returns the
        number of requests finished."""
        self.admit()
        if not self.inflight:
            return 0
        done, _ = self.session.step()
        self.steps += 1
        now = time.perf_counter()
        n = 0
        for t in done:
            b = self.by_ticket.pop(t)
            b.finished = True
            for req in b.reqs:
                req.done = now
                self.completed.append(req)
            n += len(b.reqs)
        # the ring is released in allocation order, as far as batches are finished
        while self.inflight and self.inflight[0].finished:
            b = self.inflight.popleft()
            if self.inflight:
                nxt = self.inflight[0].start
            elif self.ready:
                nxt = self.ready[0].off
            else:
                nxt = 0
            self.ring.release(b.nbytes, nxt)
        self.upload()
        return n

    def busy(self):
        return bool(self.inflight or self.ready or self.waiting)


def run_load(source, load_gbps, seconds, max_requests=None, min_requests=0,
             seed=_datagen.HASH_SEED, hbm_budget=16 << 30, ring_bytes=1 << 30):
    """Serve a Poisson stream offering `load_gbps` GB/s (None: every request is
    there from the start, which measures the capacity) for `seconds`, or until
    max_requests have arrived; at least min_requests arrive.

    Returns (summary, server, requests); requests[i] = (Request, descriptor).
    """
    import torch
    srv = Server(source, seed, hbm_budget, ring_bytes)
    saturate = load_gbps is None
    gaps = None if saturate else source.arrivals(load_gbps * 1e9, 1 << 16)
    reqs = []
    t0 = time.perf_counter()
    nxt = t0 if saturate else t0 + gaps[0]
    i = 0
    while True:
        now = time.perf_counter()
        open_ = (now - t0 < seconds or i < min_requests) and \
            (max_requests is None or i < max_requests)
        while open_ and nxt <= now:
            desc = source.draw()
            r = Request(i, desc, time.perf_counter() if saturate else nxt)
            srv.submit(r)
            reqs.append((r, desc))
            i += 1
            if not saturate:
                nxt += gaps[i % len(gaps)]
            open_ = (max_requests is None or i < max_requests) and \
                (now - t0 < seconds or i < min_requests)
            if saturate and len(srv.waiting) > 64:
                break
        if srv.inflight or srv.ready:
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
        "offered_gbps": "saturated" if saturate else load_gbps,
        "requests": len(done),
        "bytes": int(nbytes),
        "sustained_gbps": round(nbytes / max(t1 - start, 1e-9) / 1e9, 4),
        "p50_ms": round(float(np.percentile(lat, 50)), 3),
        "p99_ms": round(float(np.percentile(lat, 99)), 3),
        "steps": srv.steps,
        "batches": len(srv.batch_sizes),
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
        sub = _canon.own_order_subgrammar(g_all, req.c_index)
        if not _canon.exports_equal(sub, alone):
            raise AssertionError("request %d differs alone vs in the mix" % req.rid)
        ok += 1
    return ok


def main():
    import argparse
    import json
    ap = argparse.ArgumentParser(description="serving-form benchmark (one JSON line per load)")
    ap.add_argument("--loads", default="0.5,2,8,max")
    ap.add_argument("--seconds", type=float, default=60.0)
    ap.add_argument("--min-requests", type=int, default=2000)
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--check", type=int, default=8, help="requests checked alone vs in the mix")
    args = ap.parse_args()
    src = _datagen.ServingSource(scale=args.scale)
    for x in args.loads.split(","):
        load = None if x == "max" else float(x)
        summary, srv, reqs = run_load(src, load, args.seconds if load else 0.0,
                                      min_requests=args.min_requests)
        rng = np.random.default_rng(0)
        sample = rng.choice(len(reqs), size=min(args.check, len(reqs)), replace=False)
        summary["alone_vs_mix_checked"] = check_alone_vs_mix(srv, src, reqs, sample)
        print(json.dumps(summary), flush=True)
        srv.close()


if __name__ == "__main__":
    main()
