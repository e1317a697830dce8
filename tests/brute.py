"""Brute-force LCG construction for tiny inputs -- a pin of the oracle, not a copy of it.

Written independently of ``oracle/lcg_oracle.cpp`` from the paper's text:

* the hash family comes from its own SplitMix64 (published definition) and
  Python big integers, with the polynomial of Eq. 2 / Eq. 4 evaluated by
  Horner's rule from the right (the oracle accumulates powers from the left);
* types are Eq. 3 read literally, position by position: a position takes the
  order of its fingerprint against the first *different* fingerprint to its
  right, and is undefined when no such position exists (the trailing run) --
  no right-to-left recurrence;
* a phrase starts at position 1 and at every S-type position preceded by an
  L-type one (Sec. 3.3);
* nonterminals are numbered by first occurrence per level; C holds the symbol
  a string is reduced to, at level 0 for strings of length one.
"""

P = (1 << 61) - 1
M64 = (1 << 64) - 1


def splitmix64_stream(seed):
    state = seed & M64
    while True:
        state = (state + 0x9E3779B97F4A7C15) & M64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
        yield z ^ (z >> 31)


def hash_family(seed, levels=64):
    g = splitmix64_stream(seed)

    def draw():
        while True:
            v = next(g) % P
            if v:
                return v
    out = []
    for _ in range(levels):
        a = draw()
        b = draw()
        c = draw()
        out.append((a, b, c))
    return out


def h0(fam, s):
    a, b, _ = fam[0]
    return ((a * s + b) % P) % (1 << 32)


def poly_key(fam, level, fvals):
    """(a_i * sum_j f_j c_i^(j-1) + b_i) mod p, by Horner from the right."""
    a, b, c = fam[level]
    acc = 0
    for f in reversed(fvals):
        acc = (acc * c + f) % P
    return (a * acc + b) % P


def types_literal(f):
    """Eq. 3, literally: 'L', 'S' or None (undefined) per position."""
    n = len(f)
    out = []
    for l in range(n):
        r = l + 1
        while r < n and f[r] == f[l]:
            r += 1
        if r == n:
            out.append(None)
        else:
            out.append('L' if f[l] > f[r] else 'S')
    return out


def breaks_literal(f):
    t = types_literal(f)
    return [l == 0 or (t[l] == 'S' and t[l - 1] == 'L') for l in range(len(f))]


def phrases(seq, f):
    b = breaks_literal(f)
    starts = [l for l in range(len(seq)) if b[l]]
    ends = starts[1:] + [len(seq)]
    return [tuple(seq[s:e]) for s, e in zip(starts, ends)]


def build(strings, seed):
    """Returns (levels, c_level, c_sym); levels[i] = list of (rhs tuple, F) in rank order."""
    fam = hash_family(seed)
    k = len(strings)
    c_level = [0] * k
    c_sym = [0] * k
    cur = {}
    for j, s in enumerate(strings):
        s = list(s.encode() if isinstance(s, str) else bytes(s))
        assert len(s) >= 1
        if len(s) == 1:
            c_sym[j] = s[0]
        else:
            cur[j] = s
    levels = []
    prev_fp = None  # F of level i-1 symbols (None: terminals through h0)
    level = 0
    while cur:
        level += 1
        rules = []
        index = {}
        nxt = {}
        for j in sorted(cur):
            seq = cur[j]
            f = [h0(fam, x) if prev_fp is None else prev_fp[x] for x in seq]
            out = []
            pos = 0
            for q in phrases(seq, f):
                fq = f[pos:pos + len(q)]
                pos += len(q)
                if q not in index:
                    index[q] = len(rules)
                    rules.append((q, poly_key(fam, level, fq) % (1 << 32)))
                out.append(index[q])
            if len(out) == 1:
                c_level[j] = level
                c_sym[j] = out[0]
            else:
                nxt[j] = out
        levels.append(rules)
        prev_fp = [fp for _, fp in rules]
        cur = nxt
    return levels, c_level, c_sym


def to_export(levels, c_level, c_sym, seed):
    """Same dictionary layout as the oracle's export, for direct comparison."""
    import numpy as np
    out = []
    for rules in levels:
        off = np.zeros(len(rules) + 1, np.uint64)
        off[1:] = np.cumsum([len(q) for q, _ in rules]) if rules else []
        rhs = np.array([x for q, _ in rules for x in q], np.uint32)
        fp = np.array([f for _, f in rules], np.uint32)
        out.append({"rhs_off": off, "rhs": rhs, "fp": fp})
    return {"seed": seed, "levels": out, "c_level": np.array(c_level, np.uint8),
            "c_sym": np.array(c_sym, np.uint32)}
