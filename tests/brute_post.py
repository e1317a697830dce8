"""Brute-force checks of RL and Simp (Sec. 2.2, post-processing) on small grammars.

A pin of the oracle, written independently of ``oracle/lcg_oracle.cpp``:

* expansions come from memoised recursion over the rule table;
* Simp is computed as a fixpoint: remove ONE removable rule (an ordinary rule
  whose id occurs exactly once, in an ordinary rule's right-hand side, and
  nowhere in a run rule or in C), splice its right-hand side into the rule
  that holds the occurrence, count all occurrences again, repeat until no rule
  is removable, then number the survivors in id order.  The oracle counts
  once and removes every such rule together; the two agree because splicing a
  rule used once moves its children's occurrences without changing any count;
* RL is checked through the properties that define it, not recomputed.

A post-processed grammar is a dict {"off", "rhs", "mult", "c"} as returned by
the oracle: rule id 256 + r has right-hand side rhs[off[r]:off[r+1]] repeated
mult[r] times; ids below 256 are terminals.
"""
import numpy as np


def rules_of(slp):
    """[(rhs list, mult)] in id order."""
    off = [int(x) for x in slp["off"]]
    rhs = [int(x) for x in slp["rhs"]]
    return [(rhs[off[r]:off[r + 1]], int(slp["mult"][r])) for r in range(len(slp["mult"]))]


def from_rules(texts, c):
    """Grammar from strings like '97 98' (ordinary) or '97*3' (run rule)."""
    rules = []
    for t in texts:
        if "*" in t:
            x, l = t.split("*")
            rules.append(([int(x)], int(l)))
        else:
            rules.append(([int(x) for x in t.split()], 1))
    return {"rules": rules, "c": list(c)}


def expansions(rules):
    """exp(id) as bytes for every rule id (dict)."""
    memo = {}

    def exp(y):
        if y < 256:
            return bytes([y])
        if y not in memo:
            rhs, m = rules[y - 256]
            memo[y] = b"".join(exp(z) for z in rhs) * m
        return memo[y]
    for r in range(len(rules)):
        exp(256 + r)
    return memo


def grammar_size(rules):
    return sum(2 if m >= 2 else len(rhs) for rhs, m in rules)


def level_rules_global(export):
    """The level grammar of an export in the global id layout without runs:
    level i's rules follow level i-1's; C entries become ids."""
    rules = []
    base = [0]
    nxt = 256
    for i, L in enumerate(export["levels"], start=1):
        off = [int(x) for x in L["rhs_off"]]
        rhs = [int(x) for x in L["rhs"]]
        b = base[-1]
        for r in range(len(off) - 1):
            q = rhs[off[r]:off[r + 1]]
            rules.append(([x if i == 1 else b + x for x in q], 1))
        base.append(nxt)
        nxt += len(off) - 1
    c = [int(s) if int(lv) == 0 else base[int(lv)] + int(s)
         for lv, s in zip(export["c_level"], export["c_sym"])]
    return rules, c


def simp_fixpoint(rules, c):
    """Simp by one removal at a time (see the module docstring)."""
    live = {256 + r: (list(rhs), m) for r, (rhs, m) in enumerate(rules)}
    while True:
        occ, pinned, holder = {}, set(c), {}
        for y, (rhs, m) in live.items():
            for z in rhs:
                if z < 256:
                    continue
                if m >= 2:
                    pinned.add(z)
                else:
                    occ[z] = occ.get(z, 0) + 1
                    holder[z] = y
        victim = next((y for y in sorted(live) if live[y][1] == 1 and occ.get(y, 0) == 1
                       and y not in pinned), None)
        if victim is None:
            break
        parent = holder[victim]
        prhs, pm = live[parent]
        i = prhs.index(victim)
        live[parent] = (prhs[:i] + live[victim][0] + prhs[i + 1:], pm)
        del live[victim]
    order = sorted(live)
    new = {y: 256 + i for i, y in enumerate(order)}
    ren = lambda z: z if z < 256 else new[z]
    out = [([ren(z) for z in live[y][0]], live[y][1]) for y in order]
    return out, [ren(z) for z in c]


def check_rl(level_rules, rl_rules):
    """The defining properties of RL's output, given the input in global ids.

    * the ordinary rules of the output are the input rules, in order, with the
      same expansions;
    * no ordinary right-hand side holds two equal adjacent symbols;
    * run rules have length >= 2, are pairwise distinct and each is used by an
      ordinary rule of the next level up;
    * every rule refers only to smaller ids.
    """
    e_in = expansions(level_rules)
    e_out = expansions(rl_rules)
    ordinary = [256 + r for r, (_, m) in enumerate(rl_rules) if m == 1]
    assert len(ordinary) == len(level_rules)
    for j, y in enumerate(ordinary):
        assert e_out[y] == e_in[256 + j]
    runs = set()
    used = set()
    for r, (rhs, m) in enumerate(rl_rules):
        y = 256 + r
        assert all(z < y for z in rhs)
        if m >= 2:
            assert len(rhs) == 1
            assert (rhs[0], m) not in runs
            runs.add((rhs[0], m))
        else:
            assert all(rhs[t] != rhs[t + 1] for t in range(len(rhs) - 1))
            used.update(z for z in rhs if z >= 256 and rl_rules[z - 256][1] >= 2)
    assert used == {256 + r for r, (_, m) in enumerate(rl_rules) if m >= 2}
    return len(runs)


def as_arrays(rules, c):
    off = np.zeros(len(rules) + 1, np.uint64)
    off[1:] = np.cumsum([len(rhs) for rhs, _ in rules])
    rhs = np.array([z for rr, _ in rules for z in rr], np.uint32)
    mult = np.array([m for _, m in rules], np.uint32)
    return {"off": off, "rhs": rhs, "mult": mult, "c": np.array(c, np.uint32)}
