"""An independent reader and writer of the stored file of a post-processed
grammar, for the tests (the format: App. A, storing the final grammar, in the
layout described above ``oracle_slp_encode``).

It shares nothing with the oracle's bit loops: every section is read or
written as one Python integer (cell i of width b is bits i*b .. i*b+b-1 of
the section's little-endian value).
"""
MAGIC = b"LCGSLP01"


def nbits(x):
    """binary digits of x, at least 1"""
    return max(1, int(x).bit_length())


def _words(cells, width):
    return (cells * width + 63) // 64


def _unpack(section, n, width):
    v = int.from_bytes(section, "little")
    mask = (1 << width) - 1
    return [(v >> (i * width)) & mask for i in range(n)]


def _pack(cells, width, nwords):
    v = 0
    for i, x in enumerate(cells):
        assert 0 <= x < (1 << width)
        v |= int(x) << (i * width)
    return v.to_bytes(nwords * 8, "little")


def read(data):
    """dict with the header fields and the decoded rules [(rhs, mult)], c, bounds."""
    data = bytes(data)
    h = [int.from_bytes(data[8 * i:8 * i + 8], "little") for i in range(8)]
    assert data[:8] == MAGIC
    r, G, k, runs, nb, widths, size = h[1:]
    b_sym, b_cell, b_ptr = widths & 0xFF, (widths >> 8) & 0xFF, (widths >> 16) & 0xFF
    sizes = [_words(G, b_cell), _words(r, b_ptr), _words(r, 1), _words(k, b_sym), _words(nb, 32)]
    at, secs = 64, []
    for w in sizes:
        secs.append(data[at:at + 8 * w])
        at += 8 * w
    R = _unpack(secs[0], G, b_cell)
    P = _unpack(secs[1], r, b_ptr) + [G]
    M = _unpack(secs[2], r, 1)
    C = _unpack(secs[3], k, b_sym)
    B = _unpack(secs[4], nb, 32)
    rules = []
    for x in range(r):
        cells = R[P[x]:P[x + 1]]
        rules.append(([cells[0]], cells[1]) if M[x] else (cells, 1))
    return {"r": r, "G": G, "k": k, "runs": runs, "nb": nb, "b_sym": b_sym, "b_cell": b_cell,
            "b_ptr": b_ptr, "size": size, "total": at, "section_words": sizes,
            "rules": rules, "c": C, "bounds": B}


def write(rules, c, bounds, b_cell=None):
    """The file of rules [(rhs, mult)] (mult >= 2: a run rule, rhs = [X]), c and bounds."""
    r, k, nb = len(rules), len(c), len(bounds)
    cells, starts, marks = [], [], []
    for rhs, mult in rules:
        starts.append(len(cells))
        if mult >= 2:
            cells += [rhs[0], mult]
        else:
            cells += list(rhs)
        marks.append(1 if mult >= 2 else 0)
    G = len(cells)
    runs = sum(marks)
    b_sym = nbits(255 + r)
    longest = max([m for _, m in rules if m >= 2], default=1)
    if b_cell is None:
        b_cell = max(b_sym, nbits(longest))
    b_ptr = nbits(G - 1) if r else 1
    sizes = [_words(G, b_cell), _words(r, b_ptr), _words(r, 1), _words(k, b_sym), _words(nb, 32)]
    total = 64 + 8 * sum(sizes)
    head = MAGIC + b"".join(int(v).to_bytes(8, "little") for v in
                            (r, G, k, runs, nb, b_sym | b_cell << 8 | b_ptr << 16, total))
    body = (_pack(cells, b_cell, sizes[0]) + _pack(starts, b_ptr, sizes[1]) +
            _pack(marks, 1, sizes[2]) + _pack(c, b_sym, sizes[3]) + _pack(bounds, 32, sizes[4]))
    return head + body


def rules_of(pp):
    """[(rhs list, mult)] of a post-processed grammar dictionary."""
    off = [int(x) for x in pp["off"]]
    rhs = [int(x) for x in pp["rhs"]]
    return [(rhs[off[r]:off[r + 1]], int(pp["mult"][r])) for r in range(len(pp["mult"]))]


def doubling_chain(levels):
    """Rules X_0 -> AA, X_i -> X_{i-1} X_{i-1}: exp(X_i) has 2^(i+1) bytes; one
    rule per block."""
    rules = [([65, 65], 1)] + [([256 + i - 1, 256 + i - 1], 1) for i in range(1, levels)]
    bounds = list(range(256, 256 + levels + 1))
    return rules, [256 + levels - 1], bounds


def run_of_one(rules, c, bounds, x):
    """The file with run rule x's length cell set to 1 (still marked a run rule)."""
    data = write(rules, c, bounds)
    f = read(data)
    cells = []
    for rhs, m in rules:
        cells += [rhs[0], m] if m >= 2 else list(rhs)
    start = sum(2 if m >= 2 else len(rhs) for rhs, m in rules[:x])
    cells[start + 1] = 1
    sec = _pack(cells, f["b_cell"], f["section_words"][0])
    return data[:64] + sec + data[64 + len(sec):]


def bad_files(oracle_mod, seed):
    """(name, bytes, fragment of the refusal's message) of malformed files,
    each made from a good file of a small grammar with run rules."""
    g = oracle_mod.build_strings([b"ACGTTTTTACGA" * 3, b"GGGACGT"], seed)
    good = g.stored()
    f = read(good)
    rules, c, B = f["rules"], f["c"], f["bounds"]
    out = [("magic", b"X" + good[1:], "magic"),
           ("truncated", good[:-8], "size"),
           ("short", good[:40], "size"),
           ("wide cells", write(rules, c, B, b_cell=33), "widths")]
    # the last rule naming its own id: a cycle would be possible
    last = len(rules) - 1
    bad = list(rules)
    bad[last] = ([256 + last] + bad[last][0][1:], bad[last][1])
    out.append(("own block", write(bad, c, B), "own block"))
    runs = [x for x, (_, m) in enumerate(rules) if m >= 2]
    out.append(("run of one", run_of_one(rules, c, B, runs[0]), "run"))
    out.append(("C beyond", write(rules, [256 + len(rules)] + c[1:], B), "C names"))
    out.append(("bounds", write(rules, c, [257] + B[1:]), "bounds"))
    ch_rules, ch_c, ch_b = doubling_chain(61)
    out.append(("lengths", write(ch_rules, ch_c, ch_b), "2^61"))
    return out


def corrupted(good, seed, count):
    """`count` seeded corruptions of a good file: one to three bit flips (header
    words included), a truncation, or a 64-bit word of random bytes."""
    import numpy as np
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        b = bytearray(good)
        kind = int(rng.integers(0, 4))
        if kind < 2:
            for _ in range(int(rng.integers(1, 4))):
                bit = int(rng.integers(0, 8 * len(b)))
                b[bit // 8] ^= 1 << (bit % 8)
        elif kind == 2:
            b = b[:8 * int(rng.integers(0, len(b) // 8))]
        else:
            w = int(rng.integers(0, len(b) // 8))
            b[8 * w:8 * w + 8] = rng.integers(0, 256, 8).astype(np.uint8).tobytes()
        out.append(bytes(b))
    return out
