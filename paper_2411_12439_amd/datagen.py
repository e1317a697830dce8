"""Seeded synthetic genome-like collections.

These stand in for the paper's genome collections (AllTheBacteria, human
assemblies, SARS-CoV-2; Sec. 4), which are not available here.  The module
holds no part of the grammar construction: it only produces byte strings over
``ACGT`` (and ``N``) with the structure of those workloads -- many mutated
copies of a few base genomes -- plus the offsets array that delimits them.

All randomness comes from ``numpy.random.Generator(PCG64(seed))``.
Substitutions replace a base by a uniformly random *different* base; an indel
is, with equal probability, an insertion of random bases or a deletion, of
length uniform in the stated range.

Configurations (data seeds 1001..1005 by default):

* ``tiny``      8 copies of one 131,072 bp base; subs 0.001, indels 0.0001
                (1-10 bp); each copy truncated/padded to exactly 128 KiB.
* ``bacterial`` 4 bases of 5,000,000 bp; 64 strings, string j from base
                j mod 4 with subs 0.01, indels 0.001 (1-10 bp), random inserted
                segments of 1-20 kb totalling 0.5 % of the length, then 0.0001
                of the positions set to ``N`` (~320 MB).
* ``batched``   32 bases of 12 MB; 2,000 strings with lognormal lengths
                (median 2 MB, sigma 0.67) clipped to [50 KB, 12 MB] (~5 GB); string
                j is a random window of base j mod 32 with divergence
                U[0.5 %, 2 %], 90 % substitutions and 10 % indels (1-10 bp).
* ``repeats``   one ~237.5 MB base with tandem repeats (period 1-200, copies
                log-uniform 10-10,000) making up 5 % of its length and ~1,000
                homopolymer runs (log-uniform 20-20,000 bp); 8 copies with subs
                0.001 and indels 0.0001, each truncated/padded to 250 MB (2 GB).
* ``serving``   requests of one string each, lognormal sizes (median 1 MB,
                sigma 1.5) clipped to [10 KB, 50 MB], windows of 16 bases of
                50 MB at 1 % divergence of their own (0.1 % indels from one of
                two copies of the base, 0.9 % substitutions drawn per request),
                Poisson arrivals at a given load.

``scale`` shrinks every length by a factor (for tests on small inputs with the
same structure).
"""
import numpy as np

BASES = np.frombuffer(b"ACGT", np.uint8)
_IDX = np.zeros(256, np.uint8)
_IDX[BASES] = np.arange(4, dtype=np.uint8)

CONFIG_SEEDS = {"tiny": 1001, "bacterial": 1002, "batched": 1003, "repeats": 1004, "serving": 1005}
HASH_SEED = 0x2411124390


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def random_bases(rng, n):
    return BASES[rng.integers(0, 4, size=int(n), dtype=np.uint8)]


def substitute(rng, seq, rate):
    n = len(seq)
    k = rng.binomial(n, rate) if n else 0
    if k == 0:
        return seq
    pos = rng.integers(0, n, size=k)
    cur = seq[pos]
    isbase = np.isin(cur, BASES)
    shift = rng.integers(1, 4, size=k, dtype=np.uint8)
    seq[pos[isbase]] = BASES[(_IDX[cur[isbase]] + shift[isbase]) % 4]
    return seq


def indels(rng, seq, rate, lo=1, hi=10):
    n = len(seq)
    k = rng.binomial(n, rate) if n else 0
    if k == 0:
        return seq
    pos = np.sort(rng.integers(0, n, size=k))
    ins = rng.random(k) < 0.5
    lens = rng.integers(lo, hi + 1, size=k)
    pieces = []
    cur = 0
    for p, is_ins, L in zip(pos.tolist(), ins.tolist(), lens.tolist()):
        if p < cur:
            continue
        pieces.append(seq[cur:p])
        if is_ins:
            pieces.append(random_bases(rng, L))
            cur = p
        else:
            cur = min(n, p + L)
    pieces.append(seq[cur:])
    return np.concatenate(pieces)


def insert_segments(rng, seq, fraction, lo, hi):
    """Insert random segments (length uniform in [lo, hi]) totalling ~fraction of len."""
    target = int(len(seq) * fraction)
    segs = []
    tot = 0
    while tot < target:
        L = int(rng.integers(lo, hi + 1))
        segs.append(L)
        tot += L
    if not segs:
        return seq
    pos = np.sort(rng.integers(0, len(seq) + 1, size=len(segs)))
    pieces = []
    cur = 0
    for p, L in zip(pos.tolist(), segs):
        pieces.append(seq[cur:p])
        pieces.append(random_bases(rng, L))
        cur = p
    pieces.append(seq[cur:])
    return np.concatenate(pieces)


def set_n(rng, seq, rate):
    k = rng.binomial(len(seq), rate) if len(seq) else 0
    if k:
        seq[rng.integers(0, len(seq), size=k)] = ord("N")
    return seq


def fit_length(rng, seq, n):
    if len(seq) >= n:
        return seq[:n].copy()
    return np.concatenate([seq, random_bases(rng, n - len(seq))])


def pack(strings):
    offsets = np.zeros(len(strings) + 1, np.uint64)
    offsets[1:] = np.cumsum([len(s) for s in strings])
    text = np.concatenate(strings) if strings else np.zeros(0, np.uint8)
    return np.ascontiguousarray(text, np.uint8), offsets


def tiny(seed=CONFIG_SEEDS["tiny"], scale=1.0):
    rng = _rng(seed)
    L = max(16, int(131072 * scale))
    base = random_bases(rng, L)
    out = []
    for _ in range(8):
        s = substitute(rng, base.copy(), 0.001)
        s = indels(rng, s, 0.0001)
        out.append(fit_length(rng, s, L))
    return pack(out)


def bacterial(seed=CONFIG_SEEDS["bacterial"], scale=1.0, k=64):
    rng = _rng(seed)
    L = max(64, int(5_000_000 * scale))
    bases = [random_bases(rng, L) for _ in range(4)]
    seg_hi = max(2, int(20_000 * scale))
    out = []
    for j in range(k):
        s = substitute(rng, bases[j % 4].copy(), 0.01)
        s = indels(rng, s, 0.001)
        s = insert_segments(rng, s, 0.005, 1, seg_hi)
        s = set_n(rng, s, 0.0001)
        out.append(s)
    return pack(out)


def batched(seed=CONFIG_SEEDS["batched"], scale=1.0, k=2000):
    rng = _rng(seed)
    BL = max(64, int(12_000_000 * scale))
    bases = [random_bases(rng, BL) for _ in range(32)]
    lens = np.exp(rng.normal(np.log(2e6 * scale), 0.67, size=k))
    lens = np.clip(lens, 50_000 * scale, 12_000_000 * scale).astype(np.int64)
    lens = np.maximum(lens, 2)
    out = []
    for j in range(k):
        base = bases[j % 32]
        L = int(min(lens[j], BL))
        st = int(rng.integers(0, BL - L + 1))
        d = rng.uniform(0.005, 0.02)
        s = substitute(rng, base[st:st + L].copy(), 0.9 * d)
        s = indels(rng, s, 0.1 * d)
        out.append(s)
    return pack(out)


def repeats(seed=CONFIG_SEEDS["repeats"], scale=1.0, k=8):
    rng = _rng(seed)
    L = max(1024, int(250_000_000 * scale))
    base_len = int(L * 0.95)
    base = random_bases(rng, base_len)
    # tandem repeats up to 5 % of the final length
    ins = []
    tot = 0
    while tot < 0.05 * L:
        period = int(rng.integers(1, 201))
        copies = int(np.exp(rng.uniform(np.log(10), np.log(10_000))))
        copies = max(2, min(copies, int(max(2, 0.01 * L) // period)))
        unit = random_bases(rng, period)
        ins.append(np.tile(unit, copies))
        tot += period * copies
    # homopolymer runs (~1,000 at full scale)
    n_hp = max(1, int(1000 * scale))
    for _ in range(n_hp):
        hl = int(np.exp(rng.uniform(np.log(20), np.log(20_000))) * min(1.0, scale * 10))
        hl = max(2, hl)
        ins.append(np.full(hl, BASES[int(rng.integers(0, 4))], np.uint8))
    pos = np.sort(rng.integers(0, base_len + 1, size=len(ins)))
    order = rng.permutation(len(ins))
    pieces = []
    cur = 0
    for p, o in zip(pos.tolist(), order.tolist()):
        pieces.append(base[cur:p])
        pieces.append(ins[o])
        cur = p
    pieces.append(base[cur:])
    full = np.concatenate(pieces)
    out = []
    for _ in range(k):
        s = substitute(rng, full.copy(), 0.001)
        s = indels(rng, s, 0.0001)
        out.append(fit_length(rng, s, L))
    return pack(out)


def make_config(name, seed=None, scale=1.0, **kw):
    """(text uint8[n], offsets uint64[k+1]) of a named configuration."""
    fn = {"tiny": tiny, "bacterial": bacterial, "batched": batched, "repeats": repeats}[name]
    return fn(CONFIG_SEEDS[name] if seed is None else seed, scale=scale, **kw)


class ServingSource:
    """Request generator of the serving form.

    Bases of 50 MB (scaled); each gets `variants` copies with 0.1 % indels of
    1-10 bp, made once on the host.  A request is a random window of a random
    copy, of lognormal size (median 1 MB, sigma 1.5) clipped to [10 KB, 50 MB]
    (scaled), with its own 0.9 % substitutions: every request is synthesized
    on the device from its descriptor (request id, copy, start, length) by a
    seeded counter-based generator, so that each one carries fresh
    divergence (1 % in all) without host work per byte, and can be
    synthesized again, identically, to check it.  Inter-arrival gaps are
    exponential for a given offered load (bytes per second).
    """

    SUB_RATE = 0.009

    def __init__(self, seed=CONFIG_SEEDS["serving"], scale=1.0, n_bases=16, variants=2):
        self.seed = int(seed)
        self.rng = _rng(seed)
        self.scale = scale
        self.BL = max(1024, int(50_000_000 * scale))
        self.variants = []
        for _ in range(n_bases):
            base = random_bases(self.rng, self.BL)
            for _ in range(variants):
                self.variants.append(indels(self.rng, base.copy(), 0.001))
        self._dev = None
        self.next_id = 0

    def draw(self):
        """Descriptor (request id, variant index, start, length) of the next request."""
        s = self.scale
        L = float(np.exp(self.rng.normal(np.log(1e6 * s), 1.5)))
        L = int(np.clip(L, 10_000 * s, 50_000_000 * s))
        v = int(self.rng.integers(0, len(self.variants)))
        L = max(2, min(L, len(self.variants[v])))
        st = int(self.rng.integers(0, len(self.variants[v]) - L + 1))
        rid = self.next_id
        self.next_id += 1
        return rid, v, st, L

    def _device_variants(self, device):
        import torch
        if self._dev is None:
            self._dev = [torch.from_numpy(v).to(device) for v in self.variants]
            self._bases = torch.from_numpy(BASES.copy()).to(device)
        return self._dev

    def materialize(self, desc, out=None, device="cuda"):
        """The bytes of request `desc` as a device uint8 tensor (written into
        `out` when given), on the current stream.  Position x is substituted
        iff u_x < SUB_RATE for the request's uniform draws u (Philox, seeded
        by the request id); the new base is the old one shifted by 1, 2 or 3
        in ACGT order, chosen by which third of [0, SUB_RATE) u_x falls in."""
        import torch
        rid, v, st, L = desc
        src = self._device_variants(device)[v][st:st + L]
        g = torch.Generator(device=src.device)
        g.manual_seed((self.seed * 1_000_003 + rid) & 0x7FFFFFFFFFFFFFFF)
        u = torch.rand(L, generator=g, device=src.device)
        shift = torch.floor(u * (3.0 / self.SUB_RATE)).to(torch.uint8) + 1
        idx = ((src >> 1) ^ (src >> 2)) & 3          # A, C, G, T -> 0, 1, 2, 3
        new = self._bases[((idx + shift) & 3).long()]
        res = torch.where(u < self.SUB_RATE, new, src)
        if out is None:
            return res
        out.copy_(res)
        return out

    def host_bytes(self, desc):
        """The bytes of request `desc` on the host (through the device)."""
        return self.materialize(desc).cpu().numpy()

    def mean_size(self):
        s = self.scale
        return 1e6 * s * np.exp(1.5 ** 2 / 2)

    def arrivals(self, load_bytes_per_s, n):
        """n exponential inter-arrival gaps (seconds) for the offered load."""
        lam = load_bytes_per_s / self.mean_size()
        return self.rng.exponential(1.0 / lam, size=n)
