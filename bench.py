#!/usr/bin/env python3
"""Benchmark of the LCG construction on one MI355X.

A step is one complete construction of the grammar of the workload's
collection in the batched form: every parsing round (classify, fingerprint,
dictionary, rewrite) over all strings at once, the merge being implicit in the
shared per-level dictionaries.  Inputs are resident in device memory before
the timed region; nothing is skipped inside it.  The plain form (one launch
sequence per string per round, then MergeGrams of the per-string grammars) is
timed on the same collection for the batched-vs-plain ratio.

Prints one JSON line (see the keys below).  Extra fields:
  p50_gbps / p99_gbps    input GB/s over the timed steps (p99 = slowest steps)
  plain_gbps, batched_vs_plain
  alg_bytes_per_input_byte, alg_gbps, alg_frac_hbm   algorithmic-byte model of
                         the whole path (per round: symbols + fingerprints read,
                         rank written, one dictionary key per phrase, new slots
                         and rules) over the step time, against 8 TB/s
  roofline               the dominant kernel, its algorithmic bytes per launch
                         over its mean launch time (HIP events recorded by the
                         library on the stream its kernels run on, in the timed
                         builds around that kernel only); phase_ms_per_step from
                         untimed builds with every phase timed
  hbm_copy_gbps          read + write GB/s of a 1 GiB device-to-device copy: the
                         streaming ceiling measured on this GPU
  path_traffic           the build's counted traffic per build (FETCH_SIZE + WRITE_SIZE,
                         copy-calibrated, committed in profiles/) over the step time,
                         against 8 TB/s and the copy ceiling; null once the kernels
                         have changed since the counters were taken
  gather_ceiling         random 8-byte reads per second at 32-byte strides of a
                         4 GiB table (torch.take): the random-access ceiling the
                         dictionary probe of rounds >= 2 runs against; the
                         roofline object gives the insert's probes per second
                         and their fraction of it
  cpu_baseline           the CPU oracle (single-threaded) on a bounded sample
  cpu_baseline_parallel  the same oracle on up to 16 host cores: disjoint runs of
                         strings built concurrently, then merged (MergeGrams)
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "input GB/s of LCG build+merge at 1 GPU (batched vs plain), % HBM peak; p50/p99"
WORKLOADS = {
    "bacterial": "bacterial-like collection: 64 strings of ~5 MB (~320 MB) from 4 random 5 Mbp "
                 "bases, 1% subs, 0.1% indels, 0.5% inserted 1-20 kb segments, 0.01% N",
    "batched": "2,000 strings, lognormal lengths (median 2 MB, clipped 50 KB-12 MB, ~5 GB) from "
               "32 bases at 0.5-2% divergence",
    "repeats": "8 strings of 250 MB from one base with 5% tandem repeats and homopolymer runs",
    "tiny": "8 strings of 128 KiB, mutated copies of one base",
}
# Per-round algorithmic bytes (round i: n_i symbols, d_i phrases, u_i new
# rules, Q_i new right-hand-side symbols; s_i = 1 byte at round 1, else 4;
# f = 4-byte fingerprint; kappa = 8-byte dictionary key):
#   n_i s_i + [i >= 2] n_i f + d_i (4 + kappa) + u_i (kappa + 4 + f) + Q_i s_i
# split by the kernel that moves them: classify reads the order keys (bytes,
# or F), emit the symbols, insert one key probe per phrase and the claimed key
# per new rule, commit the new rule's rank, F and right-hand side, rewrite the
# rank of every phrase.
PHASES = ("classify", "emit", "insert", "rank", "commit", "segments")
ROOFLINE_KERNEL = "k_insert<unsigned int, false>"
PROFILE_DIR = os.path.join(ROOT, "profiles")
# the round kernels and the device header they include: a change to either
# makes the committed counter summaries stale
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2411_12439_amd", "csrc", f)
                  for f in ("lcg_kernels.hip", "lcg_device.h")]


def phase_alg_bytes(st):
    """dict phase -> algorithmic bytes summed over rounds (stats rows of one build)."""
    out = {p: 0.0 for p in PHASES}
    for i, row in enumerate(st, start=1):
        n, d, u, q = (float(x) for x in row[:4])
        s = 1.0 if i == 1 else 4.0
        # round 1 reads its byte stream once in the model (classify takes it
        # through the h^0 table; emit's second pass over it is not charged);
        # later rounds read the fingerprints (classify) and the ranks (emit)
        out["classify"] += n * s
        out["emit"] += 0.0 if i == 1 else n * s
        out["insert"] += d * 8.0 + u * 8.0
        out["commit"] += u * 8.0 + q * s + d * 4.0
    return out


def insert_rounds(st):
    """Rows whose insert phase is exactly one k_insert<unsigned int, false>
    launch: rounds >= 2 with one insert per phrase and host reads (mode 0)."""
    return [r for i, r in enumerate(st, start=1) if i >= 2 and int(r[15]) == 0 and r[1] > 0]


def source_digest():
    import hashlib
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def profile_value(name, field):
    """A number from a committed PMC summary (key: value lines) in profiles/,
    or None when there is none or the kernel source has changed since its
    counters were taken."""
    path = os.path.join(PROFILE_DIR, name)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != source_digest():
        return None
    try:
        return float(kv[field])
    except (KeyError, ValueError):
        return None


def profile_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed PMC summary of the
    workload (None as for profile_value)."""
    name = "%s_%s_traffic.txt" % ("".join(c if c.isalnum() else "_" for c in kernel).strip("_"),
                                  workload)
    return profile_value(name, "traffic_bytes_per_launch")


def path_alg_bytes(st):
    """Algorithmic bytes of the whole path (per round: read symbols, read fingerprints,
    write rank, one dictionary probe per phrase, new slot/rank/F per rule, new rhs)."""
    tot = 0.0
    for i, row in enumerate(st, start=1):
        n, d, u, q = (float(x) for x in row[:4])
        s = 1.0 if i == 1 else 4.0
        tot += n * s + (n * 4.0 if i >= 2 else 0.0) + d * (4 + 8) + u * (8 + 4 + 4) + q * s
    return tot


def gather_ceiling(table_log2=27, lookups=1 << 26, reps=5):
    """Random 8-byte reads per second (in G) from a table of 2^table_log2
    32-byte slots (4 GiB: the dictionary's slot size, and its capacity in the
    second round of the 5 GB collection), one read per slot visited, indices
    uniform: torch.take over a word view of the table."""
    import torch
    words = (1 << table_log2) * 4
    table = torch.empty(words, dtype=torch.int64, device="cuda").fill_(7)
    gen = torch.Generator(device="cuda").manual_seed(1)
    idx = torch.randint(0, 1 << table_log2, (lookups,), device="cuda", generator=gen) * 4
    torch.take(table, idx)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        torch.take(table, idx)
    b.record()
    torch.cuda.synchronize()
    rate = lookups * reps / (a.elapsed_time(b) * 1e-3) / 1e9
    del table, idx
    torch.cuda.empty_cache()
    return {"lookups_per_s_g": round(rate, 2), "table_bytes": (1 << table_log2) * 32,
            "slot_bytes": 32, "lookups": lookups,
            "what": "torch.take of one 8-byte word per random 32-byte slot of a 4 GiB table"}


def copy_ceiling(nbytes=1 << 30, reps=5):
    """Read + write GB/s of a device-to-device copy of 1 GiB on this GPU: the
    streaming ceiling measured beside the published 8 TB/s."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    gbps = 2.0 * nbytes * reps / (a.elapsed_time(b) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return round(gbps, 1)


def host_cpu():
    """The host's CPU model (from /proc/cpuinfo) and the logical CPUs this
    process sees, recorded beside the oracle's timings."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return "%s, %d logical CPUs visible" % (model, os.cpu_count() or 0)


def cpu_baseline(text, off, seed, n_strings):
    from oracle import oracle as O
    k = min(n_strings, len(off) - 1)
    t_sub = text[:off[k]]
    o_sub = off[:k + 1]
    t0 = time.perf_counter()
    g = O.build(t_sub, o_sub, seed)
    dt = time.perf_counter() - t0
    del g
    nb = int(o_sub[-1])
    return {"value": nb / dt / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
            "host_cpu": host_cpu(),
            "sample": "first %d of %d strings (%d bytes), one thread, build of the sample; "
                      "%.1f s" % (k, len(off) - 1, nb, dt)}


def cpu_baseline_parallel(text, off, seed, per_thread):
    """The unchanged oracle on all host cores (at most 16, the GPU's share of the
    host): disjoint runs of strings built by concurrent threads (the oracle is a
    C library; ctypes releases the GIL during its calls), then merged pairwise
    in string order with the oracle's MergeGrams, the pairs of each step
    concurrently.  Valid by stability: the merge gives the grammar of the whole
    sample."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle as O
    P = max(1, min(16, os.cpu_count() or 1))
    k = min(P * per_thread, len(off) - 1)
    P = min(P, k)
    cuts = [k * i // P for i in range(P + 1)]

    def part(i):
        a, b = cuts[i], cuts[i + 1]
        o = off[a:b + 1] - off[a]
        return O.build(text[off[a]:off[b]], o, seed)

    t0 = time.perf_counter()
    with ThreadPoolExecutor(P) as ex:
        parts = list(ex.map(part, range(P)))
        t1 = time.perf_counter()
        # merge-sort fashion (App. A.3): pairs (i, i + step) merged concurrently,
        # the left grammar absorbing the right one, so string order is kept
        step = 1
        while step < P:
            list(ex.map(lambda i: parts[i].merge(parts[i + step]),
                        range(0, P - step, 2 * step)))
            step *= 2
    dt = time.perf_counter() - t0
    nb = int(off[k])
    return {"value": nb / dt / 1e9, "unit": "GB/s", "cores": P, "kind": "oracle",
            "host_cpu": host_cpu(),
            "sample": "first %d of %d strings (%d bytes) in %d runs built by %d threads, "
                      "then merged pairwise in order; %.1f s (builds %.1f s, merges %.1f s)" % (
                          k, len(off) - 1, nb, P, P, dt, t1 - t0, dt - (t1 - t0))}


def time_builds(lcg, t, o, seed, steps, warmup, phase_builds, tuned):
    """Warm-up, timed and phase-timed batched builds of one resident collection.

    Returns (step seconds, [(insert launches, insert ns)] per timed build, the
    stats of the last phase-timed build, the summed per-phase ns, timed wall s)."""
    import torch
    # Timed builds record only the dictionary insert's events, in the rounds
    # that read their sizes back (the roofline's launches): timing every phase
    # costs about nine events per round.  The phase breakdown comes from the
    # untimed builds after.
    for i in range(warmup):
        g = lcg.build(t, o, seed=seed, flags=lcg.FLAG_TIMING_INSERT, **tuned)
        g.free()
        print("[bench] warmup %d done" % i, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    step_s = []
    ins_ns_steps = []
    t_all = time.perf_counter()
    for i in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = lcg.build(t, o, seed=seed, flags=lcg.FLAG_TIMING_INSERT, **tuned)
        torch.cuda.synchronize()
        step_s.append(time.perf_counter() - t0)
        rows = insert_rounds(g.stats())
        ins_ns_steps.append((len(rows), float(sum(r[11] for r in rows))))
        g.free()
        print("[bench] step %d: %.2f ms" % (i, step_s[-1] * 1e3), file=sys.stderr, flush=True)
    wall = time.perf_counter() - t_all
    torch.cuda.synchronize()
    phase_ns = {p: 0.0 for p in PHASES}
    stats = None
    for i in range(phase_builds):
        g = lcg.build(t, o, seed=seed, flags=lcg.FLAG_TIMING, **tuned)
        stats = g.stats()
        for j, p in enumerate(PHASES):
            phase_ns[p] += float(stats[:, 9 + j].sum())
        g.free()
    torch.cuda.synchronize()
    return np.array(step_s), ins_ns_steps, stats, phase_ns, wall


def time_plain(lcg, t, o, seed, steps):
    """Seconds of `steps` plain-form builds (after one untimed one)."""
    import torch
    g = lcg.build(t, o, seed=seed, mode=lcg.MODE_PLAIN)
    g.free()
    ps = []
    for i in range(max(1, steps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = lcg.build(t, o, seed=seed, mode=lcg.MODE_PLAIN)
        torch.cuda.synchronize()
        ps.append(time.perf_counter() - t0)
        g.free()
        print("[bench] plain step %d: %.2f ms" % (i, ps[-1] * 1e3), file=sys.stderr, flush=True)
    return np.array(ps)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--phase-builds", type=int, default=3,
                    help="untimed builds after the timed ones, with every phase timed")
    ap.add_argument("--config", default="batched", choices=sorted(WORKLOADS),
                    help="the collection the headline is measured on (default: the batched one)")
    ap.add_argument("--extra-config", default="bacterial", choices=sorted(WORKLOADS),
                    help="the collection of the secondary legs (its own batched and plain builds, "
                         "decompression, post-processing, random access, LCE, streaming)")
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--cpu-bytes", type=float, default=150e6,
                    help="bytes of the oracle's sample (whole strings from the first)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--rounds", action="store_true", help="per-round phase table on stderr")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the headline builds: no secondary collection, decompression, "
                         "post-processing, random access, LCE or streaming legs")
    ap.add_argument("--serving-seconds", type=float, default=20.0,
                    help="seconds per offered load of the serving leg (0 = skip)")
    ap.add_argument("--serving-warmup", type=float, default=2.0,
                    help="seconds of each offered load served before its measured window "
                         "(left out of the latencies: a fresh server's first allocations)")
    ap.add_argument("--serving-requests", type=int, default=2000,
                    help="at least this many requests per offered load")
    ap.add_argument("--serving-loads", default="0.5,2,8,max",
                    help="offered loads in GB/s; max = every request there from the start "
                         "(the sustained rate is then the capacity)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (lcg_tune) and time the default options")
    ap.add_argument("--options", default="", metavar="NAME=V,...",
                    help="skip the autotuner and time these speed-only options (e.g. the "
                         "ones a tuned run reported, so that a profiled run builds the same "
                         "rounds the same way)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device 3 times (calibrates rocprof "
                         "FETCH_SIZE / WRITE_SIZE against a copy of known size) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path "
              "(the collection would be split across GPUs by whole strings and the per-GPU "
              "grammars merged).", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.phase_builds < 1:
        ap.error("--steps and --phase-builds must be at least 1")

    import torch
    from paper_2411_12439_amd import datagen, lcg

    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        src = torch.randint(0, 255, (nbytes,), dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes, "copies": 3}))
        return

    seed = datagen.HASH_SEED
    t_gen = time.perf_counter()
    text, off = datagen.make_config(args.config, scale=args.scale)
    n = int(off[-1])
    k = len(off) - 1
    t, o = lcg.to_device(text, off)
    torch.cuda.synchronize()
    print("[bench] %s: %d strings, %d bytes on device (%.1f s)" % (
        args.config, k, n, time.perf_counter() - t_gen), file=sys.stderr, flush=True)

    # the autotuner picks the speed-only options for this workload (untimed)
    if args.options:
        tuned = {k: int(v) for k, v in (kv.split("=") for kv in args.options.split(","))}
        bad = set(tuned) - set(lcg.TUNABLE)
        if bad:
            raise SystemExit("--options: not a speed-only option: %s" % ", ".join(sorted(bad)))
        tuned_ms = None
    else:
        tuned, tuned_ms = ({}, None) if args.no_tune else lcg.tune(t, o, seed=seed)
    if tuned:
        print("[bench] options %s%s" % (tuned, "" if tuned_ms is None else " (tuned, %.2f ms)"
                                        % tuned_ms), file=sys.stderr, flush=True)
    step_s, ins_ns_steps, stats, phase_ns, wall = time_builds(
        lcg, t, o, seed, args.steps, args.warmup, args.phase_builds, tuned)
    if args.rounds:
        print("[bench] round      n        d        u     probes  cmp  ms: " + " ".join(PHASES),
              file=sys.stderr)
        for i, row in enumerate(stats, start=1):
            print("[bench] %2d %10d %9d %8d %10d %5d  %s" % (
                i, row[0], row[1], row[2], row[5], row[6],
                " ".join("%7.3f" % (row[9 + j] / 1e6) for j in range(len(PHASES)))),
                file=sys.stderr)

    gbps = n / step_s / 1e9
    value = n * args.steps / step_s.sum() / 1e9
    alg = path_alg_bytes(stats)
    alg_gbps = alg / step_s.mean() / 1e9

    # The roofline of the dominant kernel, k_insert<unsigned int, false>: in the
    # rounds listed by insert_rounds its phase events bracket exactly its one
    # launch, so the mean below is its mean launch duration.
    per_alg = phase_alg_bytes(stats)
    rows = insert_rounds(stats)
    launches = len(rows)
    # mean over the timed builds of the insert time per build (the same
    # rounds in every build: the counts do not change between builds)
    assert all(nr == launches for nr, _ in ins_ns_steps)
    ins_ns = float(np.mean([x for _, x in ins_ns_steps]))
    ins_alg = float(sum(r[1] * 8.0 + r[2] * 8.0 for r in rows))
    achieved = ins_alg / (ins_ns * 1e-9) / 1e9 if ins_ns else 0.0
    rounds = stats.shape[0]
    traffic = profile_traffic(ROOFLINE_KERNEL, args.config)
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                "traffic": None if traffic is None else round(traffic, 1),
                # the HBM bytes the counters saw per launch over its mean duration:
                # how close the kernel runs to the bandwidth it actually uses
                "traffic_gbps": None if traffic is None or not ins_ns else
                round(traffic / (ins_ns / max(launches, 1) * 1e-9) / 1e9, 1),
                "kernel": ROOFLINE_KERNEL, "launches_per_step": launches,
                "mean_launch_us": round(ins_ns / max(launches, 1) / 1e3, 2),
                "alg_bytes_per_launch": round(ins_alg / max(launches, 1), 1),
                # from the untimed builds with every phase timed
                "phase_ms_per_step": {p: round(phase_ns[p] / args.phase_builds / 1e6, 3)
                                      for p in PHASES},
                "phase_alg_gbps": {p: round(per_alg[p] / (phase_ns[p] / args.phase_builds * 1e-9)
                                            / 1e9, 1)
                                   for p in PHASES if phase_ns[p] and per_alg[p]}}

    out = {"metric": METRIC, "value": round(value, 4), "unit": "GB/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(float(step_s.mean()) * 1e3, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
           "config": {"workload": WORKLOADS[args.config], "name": args.config, "scale": args.scale,
                      "strings": k, "bytes": n, "form": "batched", "hash_seed": seed,
                      "data_seed": datagen.CONFIG_SEEDS[args.config], "rounds": rounds},
           "p50_gbps": round(float(np.percentile(gbps, 50)), 4),
           "p99_gbps": round(float(np.percentile(gbps, 1)), 4),
           "alg_bytes_per_input_byte": round(alg / n, 3),
           "alg_gbps": round(alg_gbps, 2),
           "alg_frac_hbm": round(alg_gbps / HBM_PEAK_GBPS, 4),
           "timed_wall_s": round(wall, 3),
           "tuned_options": tuned,
           "roofline": roofline}
    out["hbm_copy_gbps"] = copy_ceiling()
    # the build's counted traffic (committed counters of this workload) over
    # the measured step time: how busy the memory system is kept, next to the
    # algorithmic-byte model above
    pb = profile_value("path_%s_traffic.txt" % args.config, "path_bytes_per_build")
    out["path_traffic"] = None if pb is None else {
        "bytes_per_build": int(pb), "gbps": round(pb / float(step_s.mean()) / 1e9, 1),
        "frac_hbm": round(pb / float(step_s.mean()) / 1e9 / HBM_PEAK_GBPS, 4),
        "frac_copy_ceiling": round(pb / float(step_s.mean()) / 1e9 / out["hbm_copy_gbps"], 4),
        "source": "profiles/path_%s_traffic.txt" % args.config}
    out["gather_ceiling"] = gather_ceiling()
    probe_rate = float(sum(r[5] for r in rows)) / (ins_ns * 1e-9) / 1e9 if ins_ns else 0.0
    roofline["probes_per_s_g"] = round(probe_rate, 2)
    roofline["frac_of_gather_ceiling"] = round(
        probe_rate / out["gather_ceiling"]["lookups_per_s_g"], 3)

    if not args.no_extra:
        # RL + Simp of this collection's grammar, against its build time
        gh = lcg.build(t, o, seed=seed)
        gh.postprocess().free()
        hps = []
        for i in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            p = gh.postprocess()
            torch.cuda.synchronize()
            hps.append(time.perf_counter() - t0)
            hst = [int(x) for x in p.stats()]
            p.free()
        gh.free()
        h_ms = float(np.mean(hps)) * 1e3
        out["postprocess_headline"] = {
            "what": "lcg_postprocess (RL, then Simp) of this collection's grammar on the device",
            "ms": round(h_ms, 3), "rules_in": hst[0], "size_in": hst[1], "rules_out": hst[6],
            "size_out": hst[7], "vs_build_ms": round(h_ms / out["ms_per_step"], 4)}
        print("[bench] postprocess of the %s grammar: %.2f ms (%.1f %% of a build)" %
              (args.config, h_ms, 100 * h_ms / out["ms_per_step"]), file=sys.stderr, flush=True)

    if not args.no_plain:
        ps = time_plain(lcg, t, o, seed, args.plain_steps)
        plain = n / float(np.median(ps)) / 1e9
        out["plain_gbps"] = round(plain, 4)
        out["plain_steps_gbps"] = [round(n / x / 1e9, 4) for x in ps]
        out["batched_vs_plain"] = round(value / plain, 2)
    del t, o
    torch.cuda.empty_cache()

    if not args.no_extra:
        extra = args.extra_config
        xt, xoff = datagen.make_config(extra, scale=args.scale)
        xn, xk = int(xoff[-1]), len(xoff) - 1
        xdt, xdo = lcg.to_device(xt, xoff)
        xs_s, _, _, _, _ = time_builds(lcg, xdt, xdo, seed, args.steps, 1, 1, tuned)
        xv = xn * len(xs_s) / xs_s.sum() / 1e9
        sec = {"workload": WORKLOADS[extra], "name": extra, "strings": xk, "bytes": xn,
               "batched_gbps": round(xv, 4),
               "batched_ms": round(float(xs_s.mean()) * 1e3, 3)}
        if not args.no_plain:
            xps = time_plain(lcg, xdt, xdo, seed, args.plain_steps)
            sec["plain_gbps"] = round(xn / float(np.median(xps)) / 1e9, 4)
            sec["batched_vs_plain"] = round(xv / sec["plain_gbps"], 2)
        out["secondary"] = sec
        print("[bench] secondary %s" % json.dumps(sec), file=sys.stderr, flush=True)
        extra_legs(args, out, xt, xoff, xdt, xdo, xn, xk, seed)
        del xdt, xdo
        torch.cuda.empty_cache()
    serving_and_cpu(args, out, text, off, seed)


def extra_legs(args, out, text, off, t, o, n, k, seed):
    """Decompression, post-processing, random access, LCE and streaming legs."""
    import torch
    from paper_2411_12439_amd import lcg
    # decompression of the whole collection (the inverse path): all strings
    # expanded together, top-down over the levels
    g = lcg.build(t, o, seed=seed)
    out_t, offs_t = g.expand_strings()
    torch.cuda.synchronize()
    if not torch.equal(out_t, t):
        raise SystemExit("expand_strings does not give back the input")
    xs = []
    for i in range(max(1, args.steps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.expand_strings()
        torch.cuda.synchronize()
        xs.append(time.perf_counter() - t0)
    # post-processing of the same grammar: RL, then Simp (Sec. 2.2, Sec. 4),
    # with the size statistics of the paper's Table 2
    sizes = g.level_sizes()
    g.postprocess().free()
    pps = []
    for i in range(max(1, args.steps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p = g.postprocess()
        torch.cuda.synchronize()
        pps.append(time.perf_counter() - t0)
        st = [int(x) for x in p.stats()]
        g_out, q_out, k_out = p.size()
        p.free()
    # decompression of the post-processed grammar (the stored form)
    p = g.postprocess()
    sout, _ = p.expand_strings()
    torch.cuda.synchronize()
    if not torch.equal(sout, t):
        raise SystemExit("the post-processed grammar does not decompress to the input")
    del sout
    sxs = []
    for i in range(max(1, args.steps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p.expand_strings()
        torch.cuda.synchronize()
        sxs.append(time.perf_counter() - t0)
    # the stored file of the post-processed grammar (App. A's bit budget):
    # encoded, decoded (with every check and the expansion lengths) and
    # decompressed from the decoded grammar
    enc, dec = [], []
    for i in range(max(1, args.steps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f = p.encode()
        torch.cuda.synchronize()
        enc.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        d = lcg.decode(f)
        torch.cuda.synchronize()
        dec.append(time.perf_counter() - t0)
        if i + 1 < max(1, args.steps):
            d.free()
    dout, _ = d.expand_strings()
    torch.cuda.synchronize()
    if not torch.equal(dout, t):
        raise SystemExit("the decoded stored grammar does not decompress to the input")
    del dout
    d.free()
    fbytes = int(f.numel())
    g_sym = 256 + g_out
    budget_bits = (st[7] * int(np.ceil(np.log2(g_sym))) + g_out * int(np.ceil(np.log2(st[7])))
                   + k_out * int(np.ceil(np.log2(g_sym))))
    del f
    p.free()
    pp_in = sum(q * (1 if i == 0 else 4) + (u + 1) * 8 for i, (u, q) in enumerate(sizes)) + 5 * k
    pp_out = q_out * 4 + (g_out + 1) * 8 + g_out * 4 + k_out * 4
    pp_s = float(np.mean(pps))
    out["postprocess"] = {
        "what": "lcg_postprocess (RL, then Simp) of the collection's grammar on the device",
        "ms": round(pp_s * 1e3, 3),
        "alg_bytes": pp_in + pp_out,
        "alg_gbps": round((pp_in + pp_out) / pp_s / 1e9, 2),
        "rules_in": st[0], "size_in": st[1], "run_rules": st[2], "rules_out": st[6],
        "size_out": st[7],
        "rl_nonterminal_increase_pct": round(100.0 * st[2] / st[0], 4),
        "rl_size_reduction_pct": round(100.0 * (st[1] - st[4]) / st[1], 3),
        "simp_deleted_rules_pct": round(100.0 * st[5] / st[3], 3),
        "simp_size_reduction_pct": round(100.0 * (st[4] - st[7]) / st[4], 3),
        "expand_ms": round(float(np.mean(sxs)) * 1e3, 3),
        "expand_gbps": round(n / float(np.mean(sxs)) / 1e9, 3),
        "stored_bytes": fbytes,
        "stored_bits_per_input_byte": round(8.0 * fbytes / n, 4),
        "stored_vs_paper_budget": round(8.0 * fbytes / budget_bits, 5),
        "encode_ms": round(float(np.mean(enc)) * 1e3, 3),
        "decode_ms": round(float(np.mean(dec)) * 1e3, 3)}
    print("[bench] postprocess (RL + Simp): %.2f ms, %s" % (pp_s * 1e3, st), file=sys.stderr,
          flush=True)

    # random access: 100,000 substrings of 256 bytes at seeded random places
    rng = np.random.default_rng(7)
    nq, qlen = 100000, 256
    lens_s = np.diff(off.astype(np.int64))
    qj = rng.integers(0, k, nq)
    qs = (rng.random(nq) * (lens_s[qj] - qlen + 1)).astype(np.int64)
    dj = torch.tensor(qj, dtype=torch.int32, device="cuda")
    ds = torch.tensor(qs, dtype=torch.int64, device="cuda")
    dl = torch.full((nq,), qlen, dtype=torch.int32, device="cuda")
    xo, _ = g.extract(dj, ds, dl)
    want = text[(off.astype(np.int64)[qj] + qs)[:, None] + np.arange(qlen)[None, :]]
    if not np.array_equal(xo.cpu().numpy().reshape(nq, qlen), want):
        raise SystemExit("lcg_extract does not give back the input")
    xts = []
    for i in range(max(1, args.steps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.extract(dj, ds, dl)
        torch.cuda.synchronize()
        xts.append(time.perf_counter() - t0)
    x_s = float(np.mean(xts))
    out["extract"] = {"what": "lcg_extract: 100,000 random 256-byte substrings of the collection",
                      "ms": round(x_s * 1e3, 3), "queries_per_s": round(nq / x_s),
                      "gbps": round(nq * qlen / x_s / 1e9, 3)}
    print("[bench] extract: %.2f ms for %d queries" % (x_s * 1e3, nq), file=sys.stderr, flush=True)
    # the same queries on the post-processed grammar (RL + Simp)
    pg = g.postprocess()
    xo, _ = pg.extract(dj, ds, dl)  # the first call also computes the expansion lengths
    if not np.array_equal(xo.cpu().numpy().reshape(nq, qlen), want):
        raise SystemExit("lcg_slp_extract does not give back the input")
    xts = []
    for i in range(max(1, args.steps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pg.extract(dj, ds, dl)
        torch.cuda.synchronize()
        xts.append(time.perf_counter() - t0)
    pg.free()
    x_s = float(np.mean(xts))
    out["slp_extract"] = {"what": "lcg_slp_extract: the same 100,000 substrings from the RL + Simp "
                                  "grammar, every answer checked",
                          "ms": round(x_s * 1e3, 3), "queries_per_s": round(nq / x_s),
                          "gbps": round(nq * qlen / x_s / 1e9, 3)}
    print("[bench] slp extract: %.2f ms for %d queries" % (x_s * 1e3, nq), file=sys.stderr,
          flush=True)

    # longest common extensions (the match-extension query of App. B): anchors
    # are 24-mers of one copy of a base genome found in another copy of the
    # same base; each is extended forward and backward.  1,000 anchors, each
    # queried 100 times (100,000 queries per direction).
    na, rep = 1000, 100
    strs = {}
    anc = []
    while len(anc) < na:
        a = int(rng.integers(0, k))
        b = (a + 4 * int(rng.integers(1, max(2, k // 4)))) % k
        pa = int(rng.integers(0, lens_s[a] - 24))
        for x in (a, b):
            if x not in strs:
                strs[x] = text[off[x]:off[x + 1]].tobytes()
        pb = strs[b].find(strs[a][pa:pa + 24])
        if pb >= 0:
            anc.append((a, pa, b, pb))
    anc = np.array(anc * rep, dtype=np.int64)
    lj1 = torch.tensor(anc[:, 0], dtype=torch.int32, device="cuda")
    lp1 = torch.tensor(anc[:, 1], dtype=torch.int64, device="cuda")
    lj2 = torch.tensor(anc[:, 2], dtype=torch.int32, device="cuda")
    lp2 = torch.tensor(anc[:, 3], dtype=torch.int64, device="cuda")
    fwd = g.lce(lj1, lp1, lj2, lp2).cpu().numpy()
    bwd = g.lce(lj1, lp1, lj2, lp2, backward=True).cpu().numpy()
    oo = off.astype(np.int64)
    for q in range(na):  # each answer L: L equal bytes, then a difference or a string end
        a, pa, b, pb = (int(x) for x in anc[q])
        lf, lb = int(fwd[q]), int(bwd[q])
        sa, sb = strs[a], strs[b]
        ok_f = sa[pa:pa + lf] == sb[pb:pb + lf] and (
            pa + lf in (len(sa),) or pb + lf == len(sb) or sa[pa + lf] != sb[pb + lf])
        ok_b = sa[pa - lb:pa] == sb[pb - lb:pb] and (
            lb == pa or lb == pb or sa[pa - lb - 1] != sb[pb - lb - 1])
        if not (ok_f and ok_b and lf >= 24):
            raise SystemExit("lcg_lce answer %d is not the longest common extension" % q)
    lts = []
    for i in range(max(1, args.steps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.lce(lj1, lp1, lj2, lp2)
        g.lce(lj1, lp1, lj2, lp2, backward=True)
        torch.cuda.synchronize()
        lts.append(time.perf_counter() - t0)
    l_s = float(np.mean(lts))
    out["lce"] = {"what": "lcg_lce: 100,000 forward and 100,000 backward longest common "
                          "extensions from 24-mer anchors shared by two copies of a base",
                  "ms": round(l_s * 1e3, 3), "queries_per_s": round(2 * len(anc) / l_s),
                  "mean_forward_bytes": round(float(fwd.mean()), 1),
                  "mean_backward_bytes": round(float(bwd.mean()), 1),
                  "compared_gbps": round(float(fwd.sum() + bwd.sum()) / l_s / 1e9, 3)}
    print("[bench] lce: %.2f ms for %d queries (mean %.1f + %.1f bytes)" %
          (l_s * 1e3, 2 * len(anc), fwd.mean(), bwd.mean()), file=sys.stderr, flush=True)
    # App. B's lcp(X, Y) / lcs(X, Y) of grammar symbols: the C entries of string
    # pairs (whole strings, so every answer can be checked against the bytes)
    import ctypes
    cl = np.zeros(k, np.uint8)
    cs = np.zeros(k, np.uint32)
    lcg._check(lcg.lib().lcg_c_copy(g.h, cl.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                    cs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))))
    ns = 100000
    sj1 = rng.integers(0, k, ns)
    sj2 = rng.integers(0, k, ns)
    q = (torch.tensor(cl[sj1], device="cuda"), torch.tensor(cs[sj1].astype(np.int32), device="cuda"),
         torch.tensor(cl[sj2], device="cuda"), torch.tensor(cs[sj2].astype(np.int32), device="cuda"))
    sf = g.symbol_lce(*q).cpu().numpy()
    sbk = g.symbol_lce(*q, backward=True).cpu().numpy()
    def string(j):
        if j not in strs:
            strs[j] = text[off[j]:off[j + 1]].tobytes()
        return strs[j]

    for i in range(2000):
        a, b = string(int(sj1[i])), string(int(sj2[i]))
        lf, lb = int(sf[i]), int(sbk[i])
        ok_f = a[:lf] == b[:lf] and (lf == min(len(a), len(b)) or a[lf] != b[lf])
        ok_b = a[len(a) - lb:] == b[len(b) - lb:] and (
            lb == min(len(a), len(b)) or a[len(a) - lb - 1] != b[len(b) - lb - 1])
        if not (ok_f and ok_b):
            raise SystemExit("lcg_symbol_lce answer %d is not the lcp / lcs" % i)
    sts = []
    for i in range(max(1, args.steps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.symbol_lce(*q)
        g.symbol_lce(*q, backward=True)
        torch.cuda.synchronize()
        sts.append(time.perf_counter() - t0)
    s_s = float(np.mean(sts))
    out["symbol_lce"] = {"what": "lcg_symbol_lce: lcp and lcs of the C entries of 100,000 random "
                                 "string pairs (exp(C[j]) = T_j; 2,000 answers checked on the bytes)",
                         "ms": round(s_s * 1e3, 3), "queries_per_s": round(2 * ns / s_s),
                         "mean_lcp_bytes": round(float(sf.mean()), 1),
                         "mean_lcs_bytes": round(float(sbk.mean()), 1)}
    print("[bench] symbol lce: %.2f ms for %d queries" % (s_s * 1e3, 2 * ns), file=sys.stderr,
          flush=True)
    # maximal exact matches between two copies of a base through the grammar
    # (App. B): 16 string pairs, at least 32 bytes, anchors at level 3 and at
    # level 2 (more anchors: frequent short symbols pair up quadratically, and
    # more of the shorter matches are found); 13 matches per pair checked on
    # the bytes (equal, and not extendable either way)
    mpairs = [(j, (j + 4) % k) for j in range(min(16, k))]
    ma = [p[0] for p in mpairs]
    mb = [p[1] for p in mpairs]
    mmin = 32
    pair_bytes = sum(len(string(a)) + len(string(b)) for a, b in mpairs)
    mres = {}
    chk = 0
    for mlevel in (3, 2):
        pr_t, pa_t, pb_t, ln_t = g.mems_batch(ma, mb, mlevel, mmin)
        pr_h = pr_t.cpu().numpy()
        res = [(pa_t[torch.from_numpy(pr_h == p).to(pa_t.device)],
                pb_t[torch.from_numpy(pr_h == p).to(pb_t.device)],
                ln_t[torch.from_numpy(pr_h == p).to(ln_t.device)]) for p in range(len(mpairs))]
        nm = int(pa_t.numel())
        mlen_sum = int(ln_t.sum())
        # the single-pair call gives each pair's matches too
        one = g.mems(ma[0], mb[0], mlevel, mmin)
        if not all(torch.equal(x, y) for x, y in zip(one, res[0])):
            raise SystemExit("lcg_mems and lcg_mems_batch differ on pair 0")
        for (a, b), (pa_t, pb_t, ln_t) in zip(mpairs, res):
            sa, sb = string(a), string(b)
            pa_h, pb_h, ln_h = (x.cpu().numpy() for x in (pa_t, pb_t, ln_t))
            for t in np.linspace(0, len(pa_h) - 1, min(len(pa_h), 13)).astype(np.int64):
                x, y, m = int(pa_h[t]), int(pb_h[t]), int(ln_h[t])
                ok = (m >= mmin and sa[x:x + m] == sb[y:y + m]
                      and (x == 0 or y == 0 or sa[x - 1] != sb[y - 1])
                      and (x + m == len(sa) or y + m == len(sb) or sa[x + m] != sb[y + m]))
                if not ok:
                    raise SystemExit("lcg_mems match %d of pair %d, %d is not maximal" % (t, a, b))
                chk += 1
        del res
        mts, ots = [], []
        for i in range(max(1, args.steps)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.mems_batch(ma, mb, mlevel, mmin, cap=nm)
            torch.cuda.synchronize()
            mts.append(time.perf_counter() - t0)
            t0 = time.perf_counter()
            for a, b in mpairs:
                g.mems(a, b, mlevel, mmin)
            torch.cuda.synchronize()
            ots.append(time.perf_counter() - t0)
        m_s = float(np.mean(mts))
        mres[str(mlevel)] = {"ms": round(m_s * 1e3, 3), "matches": nm,
                             "mean_match_bytes": round(mlen_sum / max(nm, 1), 1),
                             "input_gbps": round(pair_bytes / m_s / 1e9, 3),
                             "one_call_per_pair_ms": round(float(np.mean(ots)) * 1e3, 3)}
        print("[bench] mems level %d: %.2f ms for %d pairs in one call (%.2f ms pair by pair), "
              "%d matches" % (mlevel, m_s * 1e3, len(mpairs), np.mean(ots) * 1e3, nm),
              file=sys.stderr, flush=True)
    out["mems"] = {"what": "lcg_mems_batch: maximal exact matches of >= 32 bytes between two "
                           "copies of a base, %d string pairs in one call, anchors at level 3 and "
                           "level 2 (%d matches checked on the bytes; the single-pair call "
                           "timed beside it)" % (len(mpairs), chk),
                   "pairs": len(mpairs), "pair_bytes": pair_bytes, "by_level": mres}
    g.free()
    del out_t, offs_t
    out["expand"] = {"what": "lcg_expand_strings of all strings (decompression), output bytes/s",
                     "gbps": round(n / float(np.mean(xs)) / 1e9, 3),
                     "ms": round(float(np.mean(xs)) * 1e3, 3)}
    print("[bench] expand all strings: %.2f ms" % (np.mean(xs) * 1e3), file=sys.stderr, flush=True)

    # streaming build from a file of one string per line (the collection
    # written to a temporary file, read back through the page cache)
    import tempfile
    fd, path = tempfile.mkstemp(suffix=".txt")
    try:
        with os.fdopen(fd, "wb") as f:
            oo = off.astype(np.int64)
            for j in range(k):
                f.write(text[oo[j]:oo[j + 1]].tobytes())
                f.write(b"\n")
        g = lcg.new(seed)
        lcg.build_file(g, path, chunk_bytes=64 << 20)
        g.free()
        sts = []
        for i in range(max(1, min(args.steps, 3))):
            g = lcg.new(seed)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = lcg.build_file(g, path, chunk_bytes=64 << 20)
            torch.cuda.synchronize()
            sts.append(time.perf_counter() - t0)
            g.free()
        st_s = float(np.mean(sts))
        out["stream"] = {"what": "lcg_build_file of the collection as a text file, one string "
                                 "per line, 64 MiB chunks (read, upload, split and build overlapped)",
                         "ms": round(st_s * 1e3, 3), "gbps": round(n / st_s / 1e9, 3),
                         "chunks": info["chunks"],
                         "read_wait_ms": round(info["read_wait_s"] * 1e3, 3),
                         "build_ms": round(info["build_s"] * 1e3, 3)}
        print("[bench] stream from file: %.2f ms (%s)" % (st_s * 1e3, info), file=sys.stderr,
              flush=True)
        # the same file with the sink in host memory and flush cycles: the
        # buffer grammar is merged into the sink whenever it holds 1 GiB of
        # device memory; the result must equal the one-call build
        ref = lcg.new(seed)
        lcg.build_file(ref, path, chunk_bytes=64 << 20)
        want = ref.export()
        ref.free()
        kts = []
        for i in range(max(1, min(args.steps, 3))):
            g = lcg.new(seed)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sinfo = lcg.build_file_sink(g, path, 1 << 30, chunk_bytes=64 << 20)
            torch.cuda.synchronize()
            kts.append(time.perf_counter() - t0)
            if i == 0:
                got = g.export()
                same = all(np.array_equal(a[f], b[f]) for a, b in zip(got["levels"], want["levels"])
                           for f in ("rhs_off", "rhs", "fp")) and \
                    len(got["levels"]) == len(want["levels"]) and \
                    np.array_equal(got["c_sym"], want["c_sym"])
                if not same:
                    raise SystemExit("lcg_build_file_sink differs from lcg_build_file")
            g.free()
        sk_s = float(np.mean(kts))
        out["stream_sink"] = {"what": "lcg_build_file_sink of the same file: the sink's levels in "
                                      "host memory while streaming, the buffer grammar merged into "
                                      "it at 1 GiB of device memory (result checked against "
                                      "lcg_build_file)",
                              "ms": round(sk_s * 1e3, 3), "gbps": round(n / sk_s / 1e9, 3),
                              "chunks": sinfo["chunks"], "flushes": sinfo["flushes"],
                              "flush_ms": round(sinfo["flush_s"] * 1e3, 3),
                              "build_ms": round(sinfo["build_s"] * 1e3, 3)}
        print("[bench] stream with a host sink: %.2f ms (%s)" % (sk_s * 1e3, sinfo),
              file=sys.stderr, flush=True)
    finally:
        os.unlink(path)



def cpu_sample_strings(off, nbytes):
    """Whole strings from the first until the sample holds at least nbytes."""
    o = off.astype(np.int64)
    return max(1, min(len(o) - 1, int(np.searchsorted(o, nbytes, side="left"))))


def serving_and_cpu(args, out, text, off, seed):
    """Serving leg and the CPU baselines; prints the JSON line."""
    from paper_2411_12439_amd import datagen
    if args.serving_seconds > 0:
        from paper_2411_12439_amd import serve
        src = datagen.ServingSource()
        rows = []
        for x in args.serving_loads.split(","):
            load = None if x.strip() == "max" else float(x)
            summary, srv, reqs = serve.run_load(src, load, args.serving_seconds if load else 0.0,
                                                min_requests=args.serving_requests,
                                                warmup_s=args.serving_warmup)
            rng = np.random.default_rng(0)
            cand = serve.checkable(srv, reqs)
            sample = [cand[i] for i in rng.choice(len(cand), size=min(8, len(cand)),
                                                  replace=False)]
            summary["alone_vs_mix_checked"] = serve.check_alone_vs_mix(srv, src, reqs, sample)
            rows.append(summary)
            print("[bench] serving %s" % json.dumps(summary), file=sys.stderr, flush=True)
            srv.close()
            del srv
        out["serving"] = rows

    if not args.no_cpu:
        ks = cpu_sample_strings(off, args.cpu_bytes)
        out["cpu_baseline"] = cpu_baseline(text, off, seed, ks)
        out["cpu_baseline_parallel"] = cpu_baseline_parallel(
            text, off, seed, max(1, ks // max(1, min(16, os.cpu_count() or 1))))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
