"""Canonical renaming of rank-encoded grammars, for comparisons.

Sec. 3.3 leaves the order in which a level's distinct phrases receive their
nonterminals arbitrary, so two correct constructions may name the rules of a
level differently.  ``canon`` removes that freedom: level by level, the rules
are sorted by their right-hand sides written in the canonical ranks of the
level below (terminals are byte values), lexicographically with a proper
prefix first, and a rule's canonical rank is its position in that order
(well defined because the right-hand sides of one level are distinct).

``subgrammar`` keeps only the rules reachable from chosen entries of C; with
``canon`` it compares one string's grammar inside a larger one against the
grammar of that string built alone (stability, Def. 1).

Grammars use the export layout of the library::

    {"seed": int, "levels": [{"rhs_off", "rhs", "fp"}, ...], "c_level", "c_sym"}
"""
import hashlib
import struct

import numpy as np


def canon_maps(g):
    """Per level, the array old rank -> canonical rank; and the sorted rules."""
    maps = []
    prev = None
    for L in g["levels"]:
        off = np.asarray(L["rhs_off"], np.int64)
        rhs = np.asarray(L["rhs"], np.uint32)
        mapped = rhs if prev is None else prev[rhs]
        u = len(off) - 1
        seqs = [tuple(mapped[off[r]:off[r + 1]].tolist()) for r in range(u)]
        order = sorted(range(u), key=seqs.__getitem__)
        cmap = np.empty(u, np.uint32)
        cmap[np.asarray(order, np.int64)] = np.arange(u, dtype=np.uint32)
        maps.append((cmap, order, seqs))
        prev = cmap
    return maps


def canon(g):
    """Canonical serialization (bytes) of a grammar."""
    maps = canon_maps(g)
    k = len(g["c_level"])
    out = [b"LCGC", struct.pack("<QII", int(g["seed"]), k, len(maps))]
    for (cmap, order, seqs), L in zip(maps, g["levels"]):
        fp = np.asarray(L["fp"], np.uint32)
        out.append(struct.pack("<I", len(order)))
        for r in order:
            q = seqs[r]
            out.append(struct.pack("<I%dI" % len(q), len(q), *q))
        out.append(fp[np.asarray(order, np.int64)].astype("<u4").tobytes() if order else b"")
    cl = np.asarray(g["c_level"], np.uint8)
    cs = np.asarray(g["c_sym"], np.uint32)
    for j in range(k):
        lv = int(cl[j])
        s = int(cs[j]) if lv == 0 else int(maps[lv - 1][0][cs[j]])
        out.append(struct.pack("<BI", lv, s))
    return b"".join(out)


def canon_digest(g):
    return hashlib.sha256(canon(g)).hexdigest()


def subgrammar(g, js):
    """The grammar of the strings C[js], keeping only reachable rules.

    Kept rules are renumbered in their original relative order.
    """
    levels = g["levels"]
    cl = np.asarray(g["c_level"], np.uint8)[list(js)]
    cs = np.asarray(g["c_sym"], np.uint32)[list(js)]
    top = int(cl.max()) if len(cl) else 0
    need = [set() for _ in range(top + 1)]
    for lv, s in zip(cl.tolist(), cs.tolist()):
        if lv > 0:
            need[lv].add(s)
    for i in range(top, 1, -1):
        off = np.asarray(levels[i - 1]["rhs_off"], np.int64)
        rhs = np.asarray(levels[i - 1]["rhs"], np.uint32)
        for r in need[i]:
            need[i - 1].update(rhs[off[r]:off[r + 1]].tolist())
    remaps = [None] * (top + 1)
    new_levels = []
    for i in range(1, top + 1):
        L = levels[i - 1]
        idx = np.array(sorted(need[i]), np.int64)
        off = np.asarray(L["rhs_off"], np.int64)
        rhs = np.asarray(L["rhs"], np.uint32)
        parts = [rhs[off[r]:off[r + 1]] for r in idx.tolist()]
        new_off = np.zeros(len(idx) + 1, np.uint64)
        if parts:
            new_off[1:] = np.cumsum([len(p) for p in parts])
        new_rhs = np.concatenate(parts).astype(np.uint32) if parts else np.zeros(0, np.uint32)
        if i >= 2:
            new_rhs = remaps[i - 1][new_rhs]
        new_levels.append({"rhs_off": new_off, "rhs": new_rhs,
                           "fp": np.asarray(L["fp"], np.uint32)[idx]})
        remap = np.full(len(off) - 1, 0xFFFFFFFF, np.uint32)
        remap[idx] = np.arange(len(idx), dtype=np.uint32)
        remaps[i] = remap
    new_cs = [s if lv == 0 else int(remaps[lv][s]) for lv, s in zip(cl.tolist(), cs.tolist())]
    return {"seed": g["seed"], "levels": new_levels, "c_level": cl.copy(),
            "c_sym": np.array(new_cs, np.uint32)}


def _gather(off, rhs, syms):
    """Concatenated right-hand sides of the rules `syms` (int64 ranks)."""
    a = off[syms]
    lens = off[syms + 1] - a
    tot = int(lens.sum())
    if tot == 0:
        return rhs[:0].astype(np.int64), lens
    starts = np.concatenate(([0], np.cumsum(lens)[:-1]))
    idx = np.repeat(a - starts, lens) + np.arange(tot, dtype=np.int64)
    return rhs[idx].astype(np.int64), lens


def _as_i64(a):
    """int64 view (or copy) of an offsets array."""
    a = np.asarray(a)
    return a.view(np.int64) if a.dtype == np.uint64 else a.astype(np.int64)


def own_order_subgrammar(g, j):
    """String j's grammar as found inside g, in the rank order a build of that
    string alone gives.

    The rules reachable from C[j] are kept and each level is renumbered in
    order of first occurrence in the string's own sequence of that level's
    symbols (T^{i+1}_j, rebuilt top-down from C[j]); that is the order in which
    a build of T_j alone numbers its rules (first occurrence, Sec. 3.3), so
    by stability (Def. 1) the result must equal that build exactly.  Works on
    whole-genome strings: every step is a vectorised pass over one level."""
    lv = int(np.asarray(g["c_level"], np.uint8)[j])
    sym = int(np.asarray(g["c_sym"], np.uint32)[j])
    if lv == 0:
        return {"seed": g["seed"], "levels": [], "c_level": np.array([0], np.uint8),
                "c_sym": np.array([sym], np.uint32)}
    cur = np.array([sym], np.int64)      # T^{lv+1}_j
    kept = [None] * lv
    for i in range(lv, 0, -1):
        L = g["levels"][i - 1]
        off = _as_i64(L["rhs_off"])
        rhs = np.asarray(L["rhs"])
        uniq, first = np.unique(cur, return_index=True)
        order = uniq[np.argsort(first, kind="stable")]
        body, lens = _gather(off, rhs, order)
        new_off = np.zeros(len(order) + 1, np.uint64)
        new_off[1:] = np.cumsum(lens)
        kept[i - 1] = (order, new_off, body, np.asarray(L["fp"], np.uint32)[order])
        if i > 1:
            cur, _ = _gather(off, rhs, cur)
    levels = []
    prev_map = None
    for i in range(1, lv + 1):
        order, new_off, body, fp = kept[i - 1]
        if prev_map is not None:
            body = prev_map[body]
        levels.append({"rhs_off": new_off, "rhs": body.astype(np.uint32), "fp": fp})
        u_old = len(g["levels"][i - 1]["rhs_off"]) - 1
        prev_map = np.full(u_old, -1, np.int64)
        prev_map[order] = np.arange(len(order), dtype=np.int64)
    return {"seed": g["seed"], "levels": levels, "c_level": np.array([lv], np.uint8),
            "c_sym": np.array([prev_map[sym]], np.uint32)}


def exports_equal(x, y):
    """Exact (rank-for-rank) equality of two exported grammars."""
    if int(x["seed"]) != int(y["seed"]) or len(x["levels"]) != len(y["levels"]):
        return False
    for a, b in zip(x["levels"], y["levels"]):
        for key in ("rhs_off", "rhs", "fp"):
            if not np.array_equal(np.asarray(a[key], np.uint64), np.asarray(b[key], np.uint64)):
                return False
    return (np.array_equal(np.asarray(x["c_level"], np.uint8), np.asarray(y["c_level"], np.uint8))
            and np.array_equal(np.asarray(x["c_sym"], np.uint32), np.asarray(y["c_sym"], np.uint32)))


def first_difference(x, y):
    """Human-readable location of the first difference (for test messages)."""
    if int(x["seed"]) != int(y["seed"]):
        return "seed"
    if len(x["levels"]) != len(y["levels"]):
        return "levels %d vs %d" % (len(x["levels"]), len(y["levels"]))
    for i, (a, b) in enumerate(zip(x["levels"], y["levels"])):
        for key in ("rhs_off", "rhs", "fp"):
            A = np.asarray(a[key], np.uint64)
            B = np.asarray(b[key], np.uint64)
            if A.shape != B.shape:
                return "level %d %s shape %s vs %s" % (i + 1, key, A.shape, B.shape)
            d = np.nonzero(A != B)[0]
            if len(d):
                return "level %d %s at %d: %d vs %d" % (i + 1, key, d[0], A[d[0]], B[d[0]])
    for key in ("c_level", "c_sym"):
        A = np.asarray(x[key], np.uint64)
        B = np.asarray(y[key], np.uint64)
        if A.shape != B.shape:
            return "%s shape" % key
        d = np.nonzero(A != B)[0]
        if len(d):
            return "%s at %d: %d vs %d" % (key, d[0], A[d[0]], B[d[0]])
    return None
