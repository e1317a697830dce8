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

A running grammar keeps growing with every request's new content (each one
carries fresh divergence).  Once a level of it holds max_level_rules rules,
the server starts a new running grammar (a new generation) for the batches
admitted from then on, lets the old one finish its batches in flight, and
retires it: dictionary slots are 32-bit indices, so one grammar is bounded.

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
    __slots__ = ("rid", "desc", "n", "arrival", "off", "event", "done", "c_index", "gen")

    def __init__(self, rid, desc, arrival):
        self.rid = rid
        self.desc = desc          # the source's descriptor (request id, copy, start, length)
        self.n = int(desc[3])
        self.arrival = arrival
        self.off = None
        self.event = None
        self.done = None
        self.c_index = None
        self.gen = None           # generation of the running grammar holding it


class Batch:
    """Requests admitted together (a contiguous span of the ring)."""
    __slots__ = ("reqs", "start", "nbytes", "ticket", "gen", "finished")

    def __init__(self, reqs, start, nbytes, ticket, gen):
        self.reqs = reqs
        self.start = start
        self.nbytes = nbytes
        self.ticket = ticket
        self.gen = gen
        self.finished = False


class Generation:
    """One running grammar, its serving session and its batches in flight."""

    def __init__(self, index, seed, hbm_budget, reserve=()):
        self.index = index
        self.g = _lcg.new(seed)
        if reserve:
            self.g.reserve(reserve)
        self.session = _lcg.Session(self.g, hbm_budget=hbm_budget)
        self.inflight = 0

    def close(self):
        self.session.free()
        self.g.free()


class Server:
    """Continuous-batching compressor around one device-resident running grammar."""

    def __init__(self, source, seed=_datagen.HASH_SEED, hbm_budget=16 << 30, ring_bytes=1 << 30,
                 max_batches=32, max_level_rules=1 << 27, reserve_levels=None, device="cuda"):
        import torch
        self.torch = torch
        self.source = source
        self.seed = seed
        self.budget = int(hbm_budget)
        self.max_level_rules = int(max_level_rules)
        # with reserve_levels = (lo, hi), levels lo..hi of every running
        # grammar get dictionary room for max_level_rules rules when it
        # starts, instead of doubling (and rehashing) their dictionaries as
        # they grow, each time on some batch's clock; measured, the room's
        # fill on the first batch of each grammar cost more than the
        # doublings it saves, so it is off by default
        lo, hi = reserve_levels if reserve_levels else (1, 0)
        self.reserve = [self.max_level_rules if lo <= i + 1 <= hi else 0 for i in range(hi)]
        self.gens = {}                       # live generations by index
        self.current = None
        self.generations = 0
        self._new_generation()
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

    @property
    def g(self):
        """The current running grammar."""
        return self.current.g

    def _new_generation(self):
        gen = Generation(self.generations, self.seed, self.budget, self.reserve)
        self.generations += 1
        self.gens[gen.index] = gen
        self.current = gen

    def _rotate_if_full(self):
        """Before a batch is admitted: start a new running grammar if a level of
        the current one is full (so the newest requests always sit in the
        current one)."""
        if max((u for u, _ in self.current.g.level_sizes()), default=0) >= self.max_level_rules:
            self._new_generation()

    def _retire_drained(self):
        """Free the old running grammars whose batches have all finished."""
        for i in [i for i, gen in self.gens.items()
                  if gen is not self.current and gen.inflight == 0]:
            self.gens.pop(i).close()

    def close(self):
        """Free the sessions and the running grammars."""
        for gen in self.gens.values():
            gen.close()
        self.gens.clear()

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
        self._rotate_if_full()
        cur = torch.cuda.current_stream()
        for req in batch:
            cur.wait_event(req.event)
        offs = np.zeros(len(batch) + 1, np.int64)
        offs[1:] = np.cumsum([r.n for r in batch])
        d_offs = torch.from_numpy(offs).to(self.ring.buf.device)
        gen = self.current
        try:
            first, ticket = gen.session.admit(self.ring.buf[start:start + total], d_offs)
        except _lcg.LcgError as e:
            if e.name == "LCG_ENOMEM" and self.inflight:
                return 0                   # waits for memory to free up
            raise
        for _ in batch:
            self.ready.popleft()
        for i, req in enumerate(batch):
            req.c_index = first + i
            req.gen = gen.index
        b = Batch(batch, start, total, ticket, gen.index)
        gen.inflight += 1
        self.inflight.append(b)
        self.by_ticket[(gen.index, ticket)] = b
        self.batch_sizes.append(len(batch))
        return len(batch)

    def step(self):
        """Admit what fits, then one round of every batch in flight; returns the
        number of requests finished."""
        self.admit()
        if not self.inflight:
            return 0
        finished = []
        for gen in list(self.gens.values()):
            if gen.inflight:
                done, _ = gen.session.step()
                finished += [(gen.index, t) for t in done]
        self.steps += 1
        now = time.perf_counter()
        n = 0
        for key in finished:
            b = self.by_ticket.pop(key)
            b.finished = True
            self.gens[b.gen].inflight -= 1
            for req in b.reqs:
                req.done = now
                self.completed.append(req)
            n += len(b.reqs)
        if finished:
            self._retire_drained()
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
             seed=_datagen.HASH_SEED, hbm_budget=16 << 30, ring_bytes=1 << 30,
             max_level_rules=1 << 27, reserve_levels=None, warmup_s=0.0):
    """Serve a Poisson stream offering `load_gbps` GB/s (None: every request is
    there from the start, which measures the capacity) for `seconds`, or until
    max_requests have arrived; at least min_requests arrive.  With warmup_s
    (offered loads only) the stream starts that long before the measured
    window: those requests are served alike but left out of the summary, so
    that it shows the steady state rather than the first allocations and
    dictionary growth of a fresh server.

    Returns (summary, server, requests); requests[i] = (Request, descriptor).
    """
    import torch
    srv = Server(source, seed, hbm_budget, ring_bytes, max_level_rules=max_level_rules,
                 reserve_levels=reserve_levels)
    saturate = load_gbps is None
    gaps = None if saturate else source.arrivals(load_gbps * 1e9, 1 << 16)
    reqs = []
    t0 = time.perf_counter()
    warm = 0.0 if saturate else float(warmup_s)
    t_meas = t0 + warm                   # requests arriving from here on are measured
    nxt = t0 if saturate else t0 + gaps[0]
    i = 0
    i_meas = 0

    def still_open(now):
        return (now - t0 < warm + seconds or i_meas < min_requests) and \
            (max_requests is None or i_meas < max_requests)

    while True:
        now = time.perf_counter()
        open_ = still_open(now)
        while open_ and nxt <= now:
            desc = source.draw()
            r = Request(i, desc, time.perf_counter() if saturate else nxt)
            srv.submit(r)
            reqs.append((r, desc))
            i += 1
            i_meas += r.arrival >= t_meas
            if not saturate:
                nxt += gaps[i % len(gaps)]
            open_ = still_open(now)
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
    done = [r for r, _ in reqs if r.arrival >= t_meas]
    lat = np.array([(r.done - r.arrival) * 1e3 for r in done]) if done else np.zeros(1)
    nbytes = sum(r.n for r in done)
    start = min((r.arrival for r in done), default=t0)
    # completion of the last measured request ends the window
    end = max((r.done for r in done), default=t1)
    summary = {
        "offered_gbps": "saturated" if saturate else load_gbps,
        "requests": len(done),
        "warmup_requests": len(reqs) - len(done),
        "bytes": int(nbytes),
        "sustained_gbps": round(nbytes / max(end - start, 1e-9) / 1e9, 4),
        "p50_ms": round(float(np.percentile(lat, 50)), 3),
        "p99_ms": round(float(np.percentile(lat, 99)), 3),
        "steps": srv.steps,
        "batches": len(srv.batch_sizes),
        "generations": srv.generations,
        "mean_batch": round(float(np.mean(srv.batch_sizes)), 2) if srv.batch_sizes else 0.0,
        "max_batch": int(max(srv.batch_sizes)) if srv.batch_sizes else 0,
        "wall_s": round(t1 - t0, 3),
    }
    return summary, srv, reqs


def checkable(srv, reqs):
    """Indices of the requests held by the current running grammar."""
    return [i for i, (r, _) in enumerate(reqs) if r.gen == srv.current.index]


def check_alone_vs_mix(srv, source, reqs, sample):
    """For the sampled requests (held by the current running grammar): the rules
    reachable from the request's C entry, renumbered in the request's own
    first-occurrence order, equal the grammar of the request compressed alone,
    rank for rank."""
    import torch
    g_all = srv.g.export()
    ok = 0
    for idx in sample:
        req, desc = reqs[idx]
        if req.gen != srv.current.index:
            raise ValueError("request %d is in a retired running grammar" % req.rid)
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
        cand = checkable(srv, reqs)
        sample = [cand[i] for i in rng.choice(len(cand), size=min(args.check, len(cand)),
                                              replace=False)]
        summary["alone_vs_mix_checked"] = check_alone_vs_mix(srv, src, reqs, sample)
        print(json.dumps(summary), flush=True)
        srv.close()


if __name__ == "__main__":
    main()
