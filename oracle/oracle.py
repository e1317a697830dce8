"""ctypes wrapper of the CPU oracle (``liblcg_oracle.so``) -- TEST INFRASTRUCTURE ONLY.

The oracle is the plain, single-threaded reference of the LCG construction
(BuildGram, Sec. 3.3-3.4 of the paper), of MergeGrams (Sec. 3.5-3.6) and of
grammar expansion.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module; the product library
never does.

Grammars are returned as plain dictionaries of numpy arrays::

    {"seed": int,
     "levels": [{"rhs_off": uint64[u+1], "rhs": uint32[Q], "fp": uint32[u]}, ...],   # level 1, 2, ...
     "c_level": uint8[k], "c_sym": uint32[k]}
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lcg_oracle.cpp")
_LIB = os.path.join(_HERE, "liblcg_oracle.so")

_lib = None


def compile_lib(force=True):
    """Compile the oracle with g++ (-O2, one thread)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            compile_lib()
        L = ctypes.CDLL(_LIB)
        vp, u8p, u32p, u64p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint8), \
            ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint64)
        L.oracle_last_error.restype = ctypes.c_char_p
        L.oracle_hash_params.argtypes = [ctypes.c_uint64, u64p, u64p, u64p]
        L.oracle_round1_breaks.argtypes = [u8p, ctypes.c_uint64, ctypes.c_uint64, u8p]
        L.oracle_build.argtypes = [u8p, u64p, ctypes.c_uint32, ctypes.c_uint64]
        L.oracle_build.restype = vp
        L.oracle_from_arrays.argtypes = [ctypes.c_uint64, ctypes.c_uint32, u32p,
                                         ctypes.POINTER(u64p), ctypes.POINTER(u32p),
                                         ctypes.POINTER(u32p), ctypes.c_uint32, u8p, u32p]
        L.oracle_from_arrays.restype = vp
        L.oracle_merge.argtypes = [vp, vp]
        L.oracle_merge.restype = ctypes.c_int
        L.oracle_expand.argtypes = [vp, ctypes.c_uint32, u8p, ctypes.c_uint64]
        L.oracle_expand.restype = ctypes.c_uint64
        L.oracle_num_levels.argtypes = [vp]
        L.oracle_num_levels.restype = ctypes.c_uint32
        L.oracle_num_strings.argtypes = [vp]
        L.oracle_num_strings.restype = ctypes.c_uint32
        L.oracle_seed.argtypes = [vp]
        L.oracle_seed.restype = ctypes.c_uint64
        L.oracle_level_size.argtypes = [vp, ctypes.c_uint32, u32p, u64p]
        L.oracle_level_copy.argtypes = [vp, ctypes.c_uint32, u64p, u32p, u32p]
        L.oracle_c_copy.argtypes = [vp, u8p, u32p]
        L.oracle_num_rounds.argtypes = [vp]
        L.oracle_num_rounds.restype = ctypes.c_uint32
        L.oracle_stats_copy.argtypes = [vp, u64p]
        L.oracle_free.argtypes = [vp]
        L.oracle_postprocess.argtypes = [vp, ctypes.c_uint32]
        L.oracle_postprocess.restype = vp
        L.oracle_slp_size.argtypes = [vp, u32p, u64p, u32p]
        L.oracle_slp_copy.argtypes = [vp, u64p, u32p, u32p, u32p, u64p]
        L.oracle_slp_expand.argtypes = [vp, ctypes.c_uint32, u8p, ctypes.c_uint64]
        L.oracle_slp_expand.restype = ctypes.c_uint64
        L.oracle_slp_free.argtypes = [vp]
        L.oracle_symbol_lce.argtypes = [vp, ctypes.c_uint32, u8p, u32p, u8p, u32p,
                                        ctypes.c_uint32, u64p]
        L.oracle_symbol_lce.restype = ctypes.c_int
        L.oracle_expand_symbol.argtypes = [vp, ctypes.c_uint32, ctypes.c_uint32, u8p,
                                           ctypes.c_uint64]
        L.oracle_expand_symbol.restype = ctypes.c_uint64
        L.oracle_slp_bounds.argtypes = [vp, u32p]
        L.oracle_slp_bounds.restype = ctypes.c_uint32
        L.oracle_slp_encode.argtypes = [vp, u8p, ctypes.c_uint64]
        L.oracle_slp_encode.restype = ctypes.c_uint64
        L.oracle_slp_decode.argtypes = [u8p, ctypes.c_uint64]
        L.oracle_slp_decode.restype = vp
        L.oracle_lce.argtypes = [u8p, u64p, ctypes.c_uint32, u32p, u64p, u32p, u64p,
                                 ctypes.c_uint32, u64p]
        L.oracle_mems.argtypes = [vp, u8p, u64p, ctypes.c_uint32, ctypes.c_uint32,
                                  ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, u64p, u64p,
                                  u64p]
        L.oracle_mems.restype = ctypes.c_uint64
        _lib = L
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def hash_params(seed):
    """(a, b, c) arrays of the 64-level hash family for ``seed``."""
    a = np.zeros(64, np.uint64)
    b = np.zeros(64, np.uint64)
    c = np.zeros(64, np.uint64)
    lib().oracle_hash_params(seed, _ptr(a, ctypes.c_uint64), _ptr(b, ctypes.c_uint64),
                             _ptr(c, ctypes.c_uint64))
    return a, b, c


def round1_breaks(s, seed):
    if isinstance(s, str):
        s = s.encode()
    if isinstance(s, (bytes, bytearray)):
        s = np.frombuffer(bytes(s), np.uint8)
    s = np.ascontiguousarray(s, dtype=np.uint8)
    out = np.zeros(len(s), np.uint8)
    if len(s):
        lib().oracle_round1_breaks(_ptr(s, ctypes.c_uint8), len(s), seed, _ptr(out, ctypes.c_uint8))
    return out


class Grammar:
    """Owning handle of an oracle grammar."""

    def __init__(self, handle):
        self.h = handle

    def __del__(self):
        if getattr(self, "h", None):
            lib().oracle_free(self.h)
            self.h = None

    def export(self):
        L = lib()
        nl = L.oracle_num_levels(self.h)
        levels = []
        for i in range(1, nl + 1):
            u = ctypes.c_uint32()
            q = ctypes.c_uint64()
            L.oracle_level_size(self.h, i, ctypes.byref(u), ctypes.byref(q))
            off = np.zeros(u.value + 1, np.uint64)
            rhs = np.zeros(max(q.value, 1), np.uint32)
            fp = np.zeros(max(u.value, 1), np.uint32)
            L.oracle_level_copy(self.h, i, _ptr(off, ctypes.c_uint64), _ptr(rhs, ctypes.c_uint32),
                                _ptr(fp, ctypes.c_uint32))
            levels.append({"rhs_off": off, "rhs": rhs[:q.value], "fp": fp[:u.value]})
        k = L.oracle_num_strings(self.h)
        cl = np.zeros(max(k, 1), np.uint8)
        cs = np.zeros(max(k, 1), np.uint32)
        L.oracle_c_copy(self.h, _ptr(cl, ctypes.c_uint8), _ptr(cs, ctypes.c_uint32))
        return {"seed": int(L.oracle_seed(self.h)), "levels": levels,
                "c_level": cl[:k], "c_sym": cs[:k]}

    def stats(self):
        """Per round: n_in, phrases, new_rules, rhs_len, active (uint64[rounds, 5])."""
        L = lib()
        r = L.oracle_num_rounds(self.h)
        out = np.zeros((max(r, 1), 5), np.uint64)
        L.oracle_stats_copy(self.h, _ptr(out, ctypes.c_uint64))
        return out[:r]

    def expand(self, j):
        L = lib()
        n = L.oracle_expand(self.h, j, None, 0)
        out = np.zeros(max(n, 1), np.uint8)
        L.oracle_expand(self.h, j, _ptr(out, ctypes.c_uint8), n)
        return out[:n].tobytes()

    def symbol_lce(self, lv1, s1, lv2, s2, backward=False):
        """lcp (or lcs with ``backward``) of exp(X), exp(Y) for symbol pairs
        given as (level, rank); level 0 is a byte.  uint64[nq]."""
        lv1 = np.ascontiguousarray(lv1, np.uint8)
        lv2 = np.ascontiguousarray(lv2, np.uint8)
        s1 = np.ascontiguousarray(s1, np.uint32)
        s2 = np.ascontiguousarray(s2, np.uint32)
        out = np.zeros(max(len(s1), 1), np.uint64)
        rc = lib().oracle_symbol_lce(self.h, len(s1), _ptr(lv1, ctypes.c_uint8),
                                     _ptr(s1, ctypes.c_uint32), _ptr(lv2, ctypes.c_uint8),
                                     _ptr(s2, ctypes.c_uint32), 1 if backward else 0,
                                     _ptr(out, ctypes.c_uint64))
        if rc != 0:
            raise ValueError(lib().oracle_last_error().decode())
        return out[:len(s1)]

    def mems(self, text, offsets, a, b, level, min_len):
        """Maximal exact matches of at least min_len bytes between strings a
        and b seeded by equal symbols of their level-``level`` parses (see
        oracle_mems); ``text``/``offsets`` are the collection this grammar was
        built from.  Returns (start in a, start in b, length) as three
        uint64 arrays sorted by start in a, then in b."""
        text = np.ascontiguousarray(text, np.uint8)
        offsets = np.ascontiguousarray(offsets, np.uint64)
        L = lib()
        z = np.zeros(1, np.uint64)
        args = (self.h, _ptr(text, ctypes.c_uint8), _ptr(offsets, ctypes.c_uint64), a, b, level,
                min_len)
        n = L.oracle_mems(*args, 0, _ptr(z, ctypes.c_uint64), _ptr(z, ctypes.c_uint64),
                          _ptr(z, ctypes.c_uint64))
        if n == 2**64 - 1:
            raise ValueError(L.oracle_last_error().decode())
        pa, pb, ln = (np.zeros(max(n, 1), np.uint64) for _ in range(3))
        L.oracle_mems(*args, n, _ptr(pa, ctypes.c_uint64), _ptr(pb, ctypes.c_uint64),
                      _ptr(ln, ctypes.c_uint64))
        return pa[:n], pb[:n], ln[:n]

    def expand_symbol(self, level, sym):
        """exp(X) of the symbol (level, rank) as bytes."""
        L = lib()
        n = L.oracle_expand_symbol(self.h, level, sym, None, 0)
        out = np.zeros(max(n, 1), np.uint8)
        L.oracle_expand_symbol(self.h, level, sym, _ptr(out, ctypes.c_uint8), n)
        return out[:n].tobytes()

    def postprocess(self, rl=True, simp=True, expand=False):
        """RL and/or Simp (Sec. 2.2): the straight-line grammar described in
        ``lcg_oracle.cpp`` as a dictionary::

            {"off": uint64[g+1], "rhs": uint32[Q], "mult": uint32[g], "c": uint32[k],
             "stats": uint64[8], "bounds": uint32[nb]}

        Rule ids are 256 + index; ids below 256 are terminals.  stats: g and G
        of the input, run rules made, g and G after RL, rules removed, g and G
        of the result.  bounds: the level blocks of rule ids (rules of block b,
        ids [bounds[b], bounds[b+1]), refer only to ids below bounds[b]).  With
        ``expand``, "expansions" lists exp(C[j]) of every string, expanded
        from the post-processed grammar.
        """
        L = lib()
        h = L.oracle_postprocess(self.h, (1 if rl else 0) | (2 if simp else 0))
        try:
            return _slp_dict(h, expand)
        finally:
            L.oracle_slp_free(h)

    def stored(self, rl=True, simp=True):
        """The stored file (bytes) of the post-processed grammar; the layout is
        described above ``oracle_slp_encode`` in ``lcg_oracle.cpp``."""
        L = lib()
        h = L.oracle_postprocess(self.h, (1 if rl else 0) | (2 if simp else 0))
        try:
            n = L.oracle_slp_encode(h, None, 0)
            buf = np.zeros(n, np.uint8)
            L.oracle_slp_encode(h, _ptr(buf, ctypes.c_uint8), n)
        finally:
            L.oracle_slp_free(h)
        return buf.tobytes()

    def merge(self, other):
        """MergeGrams(self, other): self absorbs other; other is unchanged."""
        rc = lib().oracle_merge(self.h, other.h)
        if rc != 0:
            raise ValueError(lib().oracle_last_error().decode())
        return self


def decode_stored(data, expand=False):
    """The grammar of a stored file as ``Grammar.postprocess`` returns it (stats
    hold only g and G of the result); ValueError names what is malformed."""
    L = lib()
    buf = np.frombuffer(bytes(data), np.uint8).copy()
    h = L.oracle_slp_decode(_ptr(buf, ctypes.c_uint8) if len(buf) else None, len(buf))
    if not h:
        raise ValueError(L.oracle_last_error().decode())
    try:
        return _slp_dict(h, expand)
    finally:
        L.oracle_slp_free(h)


def _slp_dict(h, expand):
    """The arrays of an oracle straight-line grammar handle."""
    L = lib()
    g = ctypes.c_uint32()
    q = ctypes.c_uint64()
    k = ctypes.c_uint32()
    L.oracle_slp_size(h, ctypes.byref(g), ctypes.byref(q), ctypes.byref(k))
    off = np.zeros(g.value + 1, np.uint64)
    rhs = np.zeros(max(q.value, 1), np.uint32)
    mult = np.zeros(max(g.value, 1), np.uint32)
    c = np.zeros(max(k.value, 1), np.uint32)
    st = np.zeros(8, np.uint64)
    L.oracle_slp_copy(h, _ptr(off, ctypes.c_uint64), _ptr(rhs, ctypes.c_uint32),
                      _ptr(mult, ctypes.c_uint32), _ptr(c, ctypes.c_uint32),
                      _ptr(st, ctypes.c_uint64))
    exps = []
    for j in range(k.value if expand else 0):
        n = L.oracle_slp_expand(h, j, None, 0)
        buf = np.zeros(max(n, 1), np.uint8)
        L.oracle_slp_expand(h, j, _ptr(buf, ctypes.c_uint8), n)
        exps.append(buf[:n].tobytes())
    nb = L.oracle_slp_bounds(h, None)
    bounds = np.zeros(nb, np.uint32)
    L.oracle_slp_bounds(h, _ptr(bounds, ctypes.c_uint32))
    return {"off": off, "rhs": rhs[:q.value], "mult": mult[:g.value], "c": c[:k.value],
            "stats": st, "bounds": bounds, "expansions": exps if expand else None}


def build(text, offsets, seed):
    """BuildGram over a collection given as one byte buffer plus k+1 offsets."""
    text = np.ascontiguousarray(text, dtype=np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    k = len(offsets) - 1
    h = lib().oracle_build(_ptr(text, ctypes.c_uint8) if len(text) else None,
                           _ptr(offsets, ctypes.c_uint64), k, seed)
    if not h:
        raise ValueError(lib().oracle_last_error().decode())
    return Grammar(h)


def build_strings(strings, seed):
    """BuildGram over a list of byte strings."""
    text, offsets = pack(strings)
    return build(text, offsets, seed)


def pack(strings):
    bs = [s.encode() if isinstance(s, str) else bytes(s) for s in strings]
    offsets = np.zeros(len(bs) + 1, np.uint64)
    offsets[1:] = np.cumsum([len(b) for b in bs]) if bs else []
    text = np.frombuffer(b"".join(bs), np.uint8) if bs else np.zeros(0, np.uint8)
    return text, offsets


def lce(text, offsets, j1, p1, j2, p2, backward=False):
    """Longest common extensions of position pairs (see oracle_lce): uint64[nq]."""
    text = np.ascontiguousarray(text, np.uint8)
    offsets = np.ascontiguousarray(offsets, np.uint64)
    j1 = np.ascontiguousarray(j1, np.uint32)
    j2 = np.ascontiguousarray(j2, np.uint32)
    p1 = np.ascontiguousarray(p1, np.uint64)
    p2 = np.ascontiguousarray(p2, np.uint64)
    out = np.zeros(len(j1), np.uint64)
    lib().oracle_lce(_ptr(text, ctypes.c_uint8), _ptr(offsets, ctypes.c_uint64), len(j1),
                     _ptr(j1, ctypes.c_uint32), _ptr(p1, ctypes.c_uint64),
                     _ptr(j2, ctypes.c_uint32), _ptr(p2, ctypes.c_uint64), 1 if backward else 0,
                     _ptr(out, ctypes.c_uint64))
    return out


def from_arrays(seed, levels, c_level, c_sym):
    """A grammar given explicitly (``levels`` as in ``Grammar.export``)."""
    nl = len(levels)
    u = np.array([len(L["fp"]) for L in levels], np.uint32)
    offs = [np.ascontiguousarray(L["rhs_off"], np.uint64) for L in levels]
    rhss = [np.ascontiguousarray(L["rhs"], np.uint32) for L in levels]
    fps = [np.ascontiguousarray(L["fp"], np.uint32) for L in levels]
    u64p, u32p = ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint32)
    off_arr = (u64p * max(nl, 1))(*[_ptr(a, ctypes.c_uint64) for a in offs])
    rhs_arr = (u32p * max(nl, 1))(*[_ptr(a, ctypes.c_uint32) for a in rhss])
    fp_arr = (u32p * max(nl, 1))(*[_ptr(a, ctypes.c_uint32) for a in fps])
    cl = np.ascontiguousarray(c_level, np.uint8)
    cs = np.ascontiguousarray(c_sym, np.uint32)
    h = lib().oracle_from_arrays(seed, nl, _ptr(u, ctypes.c_uint32), off_arr, rhs_arr, fp_arr,
                                 len(cl), _ptr(cl, ctypes.c_uint8), _ptr(cs, ctypes.c_uint32))
    return Grammar(h)
