// LCG reference oracle -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, single-threaded CPU implementation of the stable locally
// consistent grammar construction (BuildGram), of MergeGrams, of grammar
// expansion, of the RL and Simp post-processing and of the stored file of its
// result, and of App. B's match queries (longest common extensions, maximal
// exact matches through the grammar), written from the paper "Efficient terabyte-scale text
// compression via stable local consistency and parallel grammar processing"
// (Diaz-Dominguez, arXiv 2411.12439).  Only the test suite, the smoke check
// and the CPU-baseline leg of the benchmark load it.  It shares no code,
// header, table or constant generator with the HIP library; the product path
// never calls it.
//
// Readings of points the paper leaves open (all fixed here, and mirrored by
// the HIP library through its own, independent code):
//   * Hash family (Sec. 2.4 and 3.2, Eq. 2 and Eq. 4): one prime
//     p = 2^61 - 1 for every level, fingerprint range m = 2^32.  The
//     coefficients (a_i, b_i, c_i) of levels i = 0..63 are drawn in that
//     order from successive outputs of the SplitMix64 generator (Steele,
//     Lea and Flood, 2014, in Vigna's formulation) seeded with the caller's
//     seed; each output is reduced mod p and a zero result is drawn again,
//     so all three lie in [1, p-1] as Sec. 3.2 asks.
//   * h^0(s) = ((a_0 s + b_0) mod p) mod 2^32 for byte values s = 0..255
//     (terminals are raw bytes).
//   * Eq. 4: F[X] = ((a_i * sum_{j=1..q} F[Q[j]] c_i^{j-1} + b_i) mod p) mod 2^32,
//     leftmost symbol unscaled.
//   * Types follow Eq. 3 on fingerprints only (collisions count as equal);
//     the trailing equal-symbol run of a string has no type and no break
//     (Sec. 3.3); position 1 always starts a phrase; there is no sentinel.
//   * Nonterminals are per-level ranks (App. A.1) assigned in order of first
//     occurrence (string order, then position).  Sec. 3.3 allows any order.
//   * A string of length one is compressed at level 0: C[j] = its byte.
//     Empty strings and empty collections are rejected.
//   * Merge is Sec. 3.6 in rank form (App. A.1): the offsets L_a, L_b only
//     convert ranks to global ids and are not materialised.

#include <algorithm>
#include <array>
#include <cstdint>
#include <cstring>
#include <cstdio>
#include <string>
#include <vector>
#include <map>
#include <memory>
#include <unordered_map>

namespace {

const uint64_t kP = (1ULL << 61) - 1;  // Mersenne prime 2^61 - 1
const int kLevels = 64;                // size of the hash family H

thread_local std::string g_err;

uint64_t mulmod(uint64_t x, uint64_t y) {
  return (uint64_t)(((unsigned __int128)x * y) % kP);
}
uint64_t addmod(uint64_t x, uint64_t y) {
  return (uint64_t)(((unsigned __int128)x + y) % kP);
}

// SplitMix64: state advances by the golden-ratio increment, the output is
// the state passed through two xor-shift-multiply rounds and a final xorshift.
struct SplitMix64 {
  uint64_t s;
  uint64_t next() {
    s += 0x9E3779B97F4A7C15ULL;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
  }
  uint64_t next_nonzero_mod_p() {
    for (;;) {
      uint64_t v = next() % kP;
      if (v != 0) return v;
    }
  }
};

struct HashFamily {
  uint64_t seed;
  uint64_t a[kLevels], b[kLevels], c[kLevels];
  explicit HashFamily(uint64_t sd) : seed(sd) {
    SplitMix64 g{sd};
    for (int i = 0; i < kLevels; ++i) {
      a[i] = g.next_nonzero_mod_p();
      b[i] = g.next_nonzero_mod_p();
      c[i] = g.next_nonzero_mod_p();
    }
  }
  // h^0 on a terminal (Sec. 2.4, universal hash; Sec. 3.2).
  uint32_t h0(uint32_t s) const {
    return (uint32_t)(addmod(mulmod(a[0], s), b[0]) & 0xFFFFFFFFULL);
  }
  // Eq. 4 before the final "mod m": (a_i * sum F[Q_j] c_i^{j-1} + b_i) mod p.
  uint64_t poly(int i, const std::vector<uint32_t>& fq) const {
    uint64_t sum = 0, pw = 1;
    for (size_t j = 0; j < fq.size(); ++j) {
      sum = addmod(sum, mulmod(fq[j], pw));
      pw = mulmod(pw, c[i]);
    }
    return addmod(mulmod(a[i], sum), b[i]);
  }
};

struct Level {
  std::vector<uint64_t> rhs_off{0};  // u + 1 offsets into rhs
  std::vector<uint32_t> rhs;         // level-(i-1) ranks (bytes at level 1)
  std::vector<uint32_t> fp;          // F^i of each rule
  uint32_t size() const { return (uint32_t)fp.size(); }
};

struct RoundStat {
  uint64_t n_in;      // total length of the active strings entering the round
  uint64_t phrases;   // phrases produced (d_i)
  uint64_t new_rules; // distinct phrases = rules of the level (u_i)
  uint64_t rhs_len;   // sum of rhs lengths of the new rules (Q_i)
  uint64_t active;    // strings still active after the round
};

struct VecHash {
  size_t operator()(const std::vector<uint32_t>& v) const {
    uint64_t h = 1469598103934665603ULL;  // FNV-1a over the symbols
    for (uint32_t x : v) {
      for (int k = 0; k < 4; ++k) {
        h ^= (x >> (8 * k)) & 0xFF;
        h *= 1099511628211ULL;
      }
    }
    return (size_t)h;
  }
};
typedef std::unordered_map<std::vector<uint32_t>, uint32_t, VecHash> Dict;

}  // namespace

struct OracleGrammar {
  HashFamily H;
  std::vector<Level> levels;       // levels[i-1] holds level i
  std::vector<uint8_t> c_level;    // level of C[j]
  std::vector<uint32_t> c_sym;     // rank (or byte at level 0) of C[j]
  std::vector<RoundStat> stats;
  explicit OracleGrammar(uint64_t seed) : H(seed) {}
};

namespace {

// Fingerprint of a level-(i-1) symbol: h^0 for bytes, stored F otherwise.
uint32_t fp_of(const OracleGrammar& g, int level, uint32_t sym) {
  if (level == 0) return g.H.h0(sym);
  return g.levels[level - 1].fp[sym];
}

// Eq. 3 types from right to left.  0 = undefined (trailing equal run),
// 1 = L, 2 = S.  LMS positions (S preceded by L) are the breaks, together
// with the first position (phrase rule of Sec. 3.3).
void parse_breaks(const std::vector<uint32_t>& f, std::vector<uint8_t>& brk) {
  size_t n = f.size();
  std::vector<uint8_t> type(n, 0);
  brk.assign(n, 0);
  if (n == 0) return;
  type[n - 1] = 0;
  for (size_t l = n - 1; l-- > 0;) {
    if (f[l] > f[l + 1]) type[l] = 1;
    else if (f[l] < f[l + 1]) type[l] = 2;
    else type[l] = type[l + 1];
  }
  brk[0] = 1;
  for (size_t l = 1; l < n; ++l)
    if (type[l] == 2 && type[l - 1] == 1) brk[l] = 1;
}

}  // namespace

extern "C" {

const char* oracle_last_error(void) { return g_err.c_str(); }

void oracle_hash_params(uint64_t seed, uint64_t* a, uint64_t* b, uint64_t* c) {
  HashFamily H(seed);
  for (int i = 0; i < kLevels; ++i) { a[i] = H.a[i]; b[i] = H.b[i]; c[i] = H.c[i]; }
}

// Round-1 breaks of one string (1 = phrase starts here), for parser pins.
void oracle_round1_breaks(const uint8_t* s, uint64_t n, uint64_t seed, uint8_t* out) {
  HashFamily H(seed);
  std::vector<uint32_t> f(n);
  for (uint64_t i = 0; i < n; ++i) f[i] = H.h0(s[i]);
  std::vector<uint8_t> brk;
  parse_breaks(f, brk);
  for (uint64_t i = 0; i < n; ++i) out[i] = brk[i];
}

// BuildGram(T, H) (Sec. 3.3): rounds of RandLMSPar over the active strings,
// one dictionary per level shared by all strings, until no string is active.
OracleGrammar* oracle_build(const uint8_t* text, const uint64_t* offsets, uint32_t k,
                            uint64_t seed) {
  if (k == 0) { g_err = "empty collection"; return nullptr; }
  OracleGrammar* g = new OracleGrammar(seed);
  g->c_level.assign(k, 0);
  g->c_sym.assign(k, 0);
  std::vector<std::vector<uint32_t>> cur(k);
  std::vector<uint8_t> active(k, 0);
  size_t n_active = 0;
  for (uint32_t j = 0; j < k; ++j) {
    if (offsets[j + 1] < offsets[j]) { g_err = "offsets decrease"; delete g; return nullptr; }
    uint64_t len = offsets[j + 1] - offsets[j];
    if (len == 0) { g_err = "empty string"; delete g; return nullptr; }
    if (len == 1) { g->c_level[j] = 0; g->c_sym[j] = text[offsets[j]]; continue; }
    cur[j].assign(text + offsets[j], text + offsets[j + 1]);
    active[j] = 1;
    ++n_active;
  }
  for (int i = 1; n_active > 0; ++i) {
    if (i >= kLevels) { g_err = "hash family exhausted"; delete g; return nullptr; }
    g->levels.emplace_back();
    Level& L = g->levels.back();
    Dict dict;
    RoundStat st{0, 0, 0, 0, 0};
    std::vector<uint32_t> f, q, fq;
    std::vector<uint8_t> brk;
    for (uint32_t j = 0; j < k; ++j) {
      if (!active[j]) continue;
      const std::vector<uint32_t>& S = cur[j];
      st.n_in += S.size();
      f.resize(S.size());
      for (size_t l = 0; l < S.size(); ++l) f[l] = fp_of(*g, i - 1, S[l]);
      parse_breaks(f, brk);
      std::vector<uint32_t> next;
      size_t start = 0;
      for (size_t l = 1; l <= S.size(); ++l) {
        if (l < S.size() && !brk[l]) continue;
        q.assign(S.begin() + start, S.begin() + l);
        auto it = dict.find(q);
        uint32_t r;
        if (it != dict.end()) {
          r = it->second;
        } else {
          r = L.size();
          dict.emplace(q, r);
          fq.assign(f.begin() + start, f.begin() + l);
          uint64_t P = g->H.poly(i, fq);
          L.fp.push_back((uint32_t)(P & 0xFFFFFFFFULL));
          L.rhs.insert(L.rhs.end(), q.begin(), q.end());
          L.rhs_off.push_back(L.rhs.size());
          st.rhs_len += q.size();
        }
        next.push_back(r);
        start = l;
      }
      st.phrases += next.size();
      cur[j].swap(next);
      if (cur[j].size() == 1) {
        g->c_level[j] = (uint8_t)i;
        g->c_sym[j] = cur[j][0];
        active[j] = 0;
        --n_active;
        std::vector<uint32_t>().swap(cur[j]);
      }
    }
    st.new_rules = L.size();
    st.active = n_active;
    g->stats.push_back(st);
  }
  return g;
}

// Build a grammar directly from arrays (used to encode the paper's worked
// merge example by hand).  rhs_off has u_i + 1 entries per level.
OracleGrammar* oracle_from_arrays(uint64_t seed, uint32_t n_levels, const uint32_t* u,
                                  const uint64_t* const* rhs_off, const uint32_t* const* rhs,
                                  const uint32_t* const* fp, uint32_t k,
                                  const uint8_t* c_level, const uint32_t* c_sym) {
  OracleGrammar* g = new OracleGrammar(seed);
  for (uint32_t i = 0; i < n_levels; ++i) {
    g->levels.emplace_back();
    Level& L = g->levels.back();
    L.rhs_off.assign(rhs_off[i], rhs_off[i] + u[i] + 1);
    L.rhs.assign(rhs[i], rhs[i] + rhs_off[i][u[i]]);
    L.fp.assign(fp[i], fp[i] + u[i]);
  }
  g->c_level.assign(c_level, c_level + k);
  g->c_sym.assign(c_sym, c_sym + k);
  return g;
}

// MergeGrams(G_a, G_b) (Sec. 3.5 and 3.6): G_a absorbs G_b level by level.
// For each level i, every rule of G_b (its rhs already renamed into G_a's
// level-(i-1) ranks) is looked up among G_a's level-i right-hand sides; a hit
// reuses G_a's rank, a miss appends the rule at the end of level i.  The
// resulting rank map M renames the next level of G_b and the entries of C_b
// at level i.  Finally C_a becomes C_a . C_b.  G_b is left unchanged.
int oracle_merge(OracleGrammar* a, const OracleGrammar* b) {
  if (a->H.seed != b->H.seed) { g_err = "hash families differ"; return -3; }
  size_t la = a->levels.size(), lb = b->levels.size();
  std::vector<std::vector<uint32_t>> M(lb + 1);  // M[i]: b-rank -> a-rank, level i
  while (a->levels.size() < lb) a->levels.emplace_back();
  (void)la;
  for (size_t i = 1; i <= lb; ++i) {
    Level& A = a->levels[i - 1];
    const Level& B = b->levels[i - 1];
    Dict H;
    for (uint32_t r = 0; r < A.size(); ++r)
      H.emplace(std::vector<uint32_t>(A.rhs.begin() + A.rhs_off[r],
                                      A.rhs.begin() + A.rhs_off[r + 1]), r);
    M[i].assign(B.size(), 0);
    std::vector<uint32_t> q;
    for (uint32_t rb = 0; rb < B.size(); ++rb) {
      q.assign(B.rhs.begin() + B.rhs_off[rb], B.rhs.begin() + B.rhs_off[rb + 1]);
      if (i >= 2)
        for (uint32_t& x : q) x = M[i - 1][x];
      auto it = H.find(q);
      if (it != H.end()) {
        M[i][rb] = it->second;
      } else {
        uint32_t r = A.size();
        M[i][rb] = r;
        A.rhs.insert(A.rhs.end(), q.begin(), q.end());
        A.rhs_off.push_back(A.rhs.size());
        A.fp.push_back(B.fp[rb]);
        H.emplace(q, r);
      }
    }
  }
  for (size_t j = 0; j < b->c_level.size(); ++j) {
    uint8_t lv = b->c_level[j];
    a->c_level.push_back(lv);
    a->c_sym.push_back(lv == 0 ? b->c_sym[j] : M[lv][b->c_sym[j]]);
  }
  return 0;
}

// exp(C[j]) by recursive substitution of right-hand sides down to level 0.
// Returns the expansion length; writes at most cap bytes.
uint64_t oracle_expand_symbol(const OracleGrammar* g, uint32_t level, uint32_t sym, uint8_t* out,
                              uint64_t cap);

uint64_t oracle_expand(const OracleGrammar* g, uint32_t j, uint8_t* out, uint64_t cap) {
  return oracle_expand_symbol(g, g->c_level[j], g->c_sym[j], out, cap);
}

// exp(X) of the level-`level` symbol X = sym (level 0: the byte sym); returns
// its length, writes at most cap bytes.
uint64_t oracle_expand_symbol(const OracleGrammar* g, uint32_t level, uint32_t sym, uint8_t* out,
                              uint64_t cap) {
  uint64_t len = 0;
  std::vector<std::pair<int, uint32_t>> stack;
  stack.push_back({(int)level, sym});
  while (!stack.empty()) {
    std::pair<int, uint32_t> t = stack.back();
    stack.pop_back();
    if (t.first == 0) {
      if (len < cap) out[len] = (uint8_t)t.second;
      ++len;
      continue;
    }
    const Level& L = g->levels[t.first - 1];
    for (uint64_t x = L.rhs_off[t.second + 1]; x-- > L.rhs_off[t.second];)
      stack.push_back({t.first - 1, L.rhs[x]});
  }
  return len;
}

// ---- accessors -------------------------------------------------------
uint32_t oracle_num_levels(const OracleGrammar* g) { return (uint32_t)g->levels.size(); }
uint32_t oracle_num_strings(const OracleGrammar* g) { return (uint32_t)g->c_level.size(); }
uint64_t oracle_seed(const OracleGrammar* g) { return g->H.seed; }
void oracle_level_size(const OracleGrammar* g, uint32_t level, uint32_t* u, uint64_t* rhs_len) {
  const Level& L = g->levels[level - 1];
  *u = L.size();
  *rhs_len = L.rhs.size();
}
void oracle_level_copy(const OracleGrammar* g, uint32_t level, uint64_t* rhs_off,
                       uint32_t* rhs, uint32_t* fp) {
  const Level& L = g->levels[level - 1];
  std::memcpy(rhs_off, L.rhs_off.data(), L.rhs_off.size() * sizeof(uint64_t));
  std::memcpy(rhs, L.rhs.data(), L.rhs.size() * sizeof(uint32_t));
  std::memcpy(fp, L.fp.data(), L.fp.size() * sizeof(uint32_t));
}
void oracle_c_copy(const OracleGrammar* g, uint8_t* lvl, uint32_t* sym) {
  std::memcpy(lvl, g->c_level.data(), g->c_level.size());
  std::memcpy(sym, g->c_sym.data(), g->c_sym.size() * sizeof(uint32_t));
}
uint32_t oracle_num_rounds(const OracleGrammar* g) { return (uint32_t)g->stats.size(); }
// Five counters per round: n_in, phrases, new_rules, rhs_len, active.
void oracle_stats_copy(const OracleGrammar* g, uint64_t* out) {
  for (size_t i = 0; i < g->stats.size(); ++i) {
    out[5 * i + 0] = g->stats[i].n_in;
    out[5 * i + 1] = g->stats[i].phrases;
    out[5 * i + 2] = g->stats[i].new_rules;
    out[5 * i + 3] = g->stats[i].rhs_len;
    out[5 * i + 4] = g->stats[i].active;
  }
}
void oracle_free(OracleGrammar* g) { delete g; }

}  // extern "C"

// ---------------------------------------------------------------------
// Post-processing (Sec. 2.2, last paragraph; applied to the output of
// PBuildGram in the order RL, then Simp, Sec. 4).
//
// The result is a straight-line grammar with one id space:
//   * ids 0..255 are the terminals (byte values);
//   * then, for level i = 1, 2, ...: first the run rules made from the runs
//     in level i's right-hand sides (their symbols are level-(i-1) symbols),
//     ordered by (symbol, run length), then level i's rules in rank order.
// Every rule therefore refers only to smaller ids.  A rule is stored as a
// right-hand side and a multiplicity: exp(X) = exp(rhs(X))^mult(X).  Rules
// with mult = 1 are ordinary rules; a run rule X' -> (X, l) is stored as
// rhs = [X], mult = l >= 2.
//
// RL: every maximal equal-symbol run X^l with l >= 2 in an ordinary rule's
// right-hand side is replaced by the id of the run rule (X, l); each distinct
// pair (X, l) of a level gets one run rule.
//
// Simp: an ordinary rule whose id occurs exactly once over all right-hand
// sides and C, that one occurrence being in an ordinary rule, is removed and
// its right-hand side takes the place of its occurrence (recursively).
// Occurrences in run rules and in C keep a rule: a run rule holds a symbol,
// not a sequence, and C holds one symbol per string.  Run rules themselves
// are never removed.  The remaining rules are renumbered in id order from 256.
//
// Grammar size G counts |rhs| for ordinary rules and 2 for a run rule.

struct OracleSlp {
  std::vector<uint64_t> off{0};
  std::vector<uint32_t> rhs;
  std::vector<uint32_t> mult;
  std::vector<uint32_t> c;
  // The level structure: rule ids [bounds[b], bounds[b+1]) form block b (per
  // input level, its run rules, then its ordinary rules; blocks may be
  // empty), and the rules of a block refer only to ids below bounds[b].
  std::vector<uint32_t> bounds{256};
  // g and G of the input, run rules made, g and G after RL, rules removed,
  // g and G of the result
  uint64_t stats[8] = {0, 0, 0, 0, 0, 0, 0, 0};
};

namespace {

uint64_t slp_size(const OracleSlp& s) {
  uint64_t G = 0;
  for (size_t r = 0; r + 1 < s.off.size(); ++r)
    G += s.mult[r] >= 2 ? 2 : s.off[r + 1] - s.off[r];
  return G;
}

// The level grammar in the global id space, with RL applied when rl is set.
OracleSlp to_global(const OracleGrammar* g, bool rl) {
  OracleSlp s;
  std::vector<uint32_t> obase(g->levels.size() + 1, 0);  // first id of level i's rules
  uint32_t next = 256;
  for (size_t i = 1; i <= g->levels.size(); ++i) {
    const Level& L = g->levels[i - 1];
    auto gid = [&](uint32_t x) { return i == 1 ? x : obase[i - 1] + x; };
    // the distinct runs (X, l >= 2) of the level, in (X, l) order
    std::map<std::pair<uint32_t, uint32_t>, uint32_t> runs;
    if (rl) {
      for (uint32_t r = 0; r < L.size(); ++r) {
        uint64_t a = L.rhs_off[r], b = L.rhs_off[r + 1];
        for (uint64_t x = a; x < b;) {
          uint64_t y = x + 1;
          while (y < b && L.rhs[y] == L.rhs[x]) ++y;
          if (y - x >= 2) runs[{L.rhs[x], (uint32_t)(y - x)}] = 0;
          x = y;
        }
      }
    }
    for (auto& kv : runs) {
      kv.second = next++;
      s.rhs.push_back(gid(kv.first.first));
      s.off.push_back(s.rhs.size());
      s.mult.push_back(kv.first.second);
    }
    obase[i] = next;
    s.bounds.push_back(next);
    next += L.size();
    s.bounds.push_back(next);
    for (uint32_t r = 0; r < L.size(); ++r) {
      uint64_t a = L.rhs_off[r], b = L.rhs_off[r + 1];
      for (uint64_t x = a; x < b;) {
        uint64_t y = x + 1;
        if (rl)
          while (y < b && L.rhs[y] == L.rhs[x]) ++y;
        if (y - x >= 2)
          s.rhs.push_back(runs.at({L.rhs[x], (uint32_t)(y - x)}));
        else
          s.rhs.push_back(gid(L.rhs[x]));
        x = y;
      }
      s.off.push_back(s.rhs.size());
      s.mult.push_back(1);
    }
  }
  for (size_t j = 0; j < g->c_level.size(); ++j)
    s.c.push_back(g->c_level[j] == 0 ? g->c_sym[j] : obase[g->c_level[j]] + g->c_sym[j]);
  return s;
}

void simp_append(const OracleSlp& s, const std::vector<uint8_t>& removed,
                 const std::vector<uint32_t>& newid, uint32_t y, std::vector<uint32_t>& out) {
  if (y < 256 || !removed[y - 256]) {
    out.push_back(y < 256 ? y : newid[y - 256]);
    return;
  }
  for (uint64_t t = s.off[y - 256]; t < s.off[y - 255]; ++t)
    simp_append(s, removed, newid, s.rhs[t], out);
}

OracleSlp simp(const OracleSlp& s) {
  size_t g = s.mult.size();
  std::vector<uint64_t> occ(g, 0);    // occurrences in ordinary right-hand sides
  std::vector<uint8_t> pinned(g, 0);  // occurs in a run rule or in C
  for (size_t r = 0; r < g; ++r)
    for (uint64_t t = s.off[r]; t < s.off[r + 1]; ++t) {
      uint32_t y = s.rhs[t];
      if (y < 256) continue;
      if (s.mult[r] >= 2) pinned[y - 256] = 1;
      else ++occ[y - 256];
    }
  for (uint32_t y : s.c)
    if (y >= 256) pinned[y - 256] = 1;
  std::vector<uint8_t> removed(g, 0);
  std::vector<uint32_t> newid(g, 0);
  uint32_t next = 256;
  for (size_t r = 0; r < g; ++r) {
    removed[r] = s.mult[r] == 1 && occ[r] == 1 && !pinned[r];
    if (!removed[r]) newid[r] = next++;
  }
  OracleSlp o;
  o.bounds.clear();
  std::vector<uint32_t> kept_below(g + 1, 0);
  for (size_t r = 0; r < g; ++r) kept_below[r + 1] = kept_below[r] + !removed[r];
  for (uint32_t b : s.bounds) o.bounds.push_back(256 + kept_below[b - 256]);  // kept rules below b
  for (size_t r = 0; r < g; ++r) {
    if (removed[r]) continue;
    for (uint64_t t = s.off[r]; t < s.off[r + 1]; ++t)
      simp_append(s, removed, newid, s.rhs[t], o.rhs);
    o.off.push_back(o.rhs.size());
    o.mult.push_back(s.mult[r]);
  }
  for (uint32_t y : s.c) o.c.push_back(y < 256 ? y : newid[y - 256]);
  return o;
}

}  // namespace

extern "C" {

// flags: 1 = RL, 2 = Simp (both: RL first).
OracleSlp* oracle_postprocess(const OracleGrammar* g, uint32_t flags) {
  OracleSlp plain = to_global(g, false);
  OracleSlp s = to_global(g, (flags & 1) != 0);
  uint64_t st0 = plain.mult.size(), st1 = slp_size(plain);
  uint64_t runs = s.mult.size() - plain.mult.size();
  uint64_t g_rl = s.mult.size(), G_rl = slp_size(s);
  if (flags & 2) s = simp(s);
  OracleSlp* out = new OracleSlp(std::move(s));
  uint64_t st[8] = {st0, st1, runs, g_rl, G_rl, g_rl - out->mult.size(), out->mult.size(),
                    slp_size(*out)};
  std::memcpy(out->stats, st, sizeof(st));
  return out;
}
void oracle_slp_size(const OracleSlp* s, uint32_t* g, uint64_t* rhs_len, uint32_t* k) {
  *g = (uint32_t)s->mult.size();
  *rhs_len = s->rhs.size();
  *k = (uint32_t)s->c.size();
}
void oracle_slp_copy(const OracleSlp* s, uint64_t* off, uint32_t* rhs, uint32_t* mult,
                     uint32_t* c, uint64_t* stats) {
  std::memcpy(off, s->off.data(), s->off.size() * sizeof(uint64_t));
  std::memcpy(rhs, s->rhs.data(), s->rhs.size() * sizeof(uint32_t));
  std::memcpy(mult, s->mult.data(), s->mult.size() * sizeof(uint32_t));
  std::memcpy(c, s->c.data(), s->c.size() * sizeof(uint32_t));
  std::memcpy(stats, s->stats, sizeof(s->stats));
}
// exp(C[j]) of the post-processed grammar; returns its length, writes at most cap bytes.
uint64_t oracle_slp_expand(const OracleSlp* s, uint32_t j, uint8_t* out, uint64_t cap) {
  uint64_t len = 0;
  std::vector<uint32_t> stack{s->c[j]};
  while (!stack.empty()) {
    uint32_t y = stack.back();
    stack.pop_back();
    if (y < 256) {
      if (len < cap) out[len] = (uint8_t)y;
      ++len;
      continue;
    }
    uint32_t r = y - 256;
    for (uint32_t m = 0; m < s->mult[r]; ++m)
      for (uint64_t t = s->off[r + 1]; t-- > s->off[r];) stack.push_back(s->rhs[t]);
  }
  return len;
}
void oracle_slp_free(OracleSlp* s) { delete s; }
// The block bounds (see OracleSlp); returns their number, writes them if out.
uint32_t oracle_slp_bounds(const OracleSlp* s, uint32_t* out) {
  if (out) std::memcpy(out, s->bounds.data(), s->bounds.size() * sizeof(uint32_t));
  return (uint32_t)s->bounds.size();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// The stored file of a post-processed grammar.  App. A (storing the final
// grammar) budgets G log g bits for the right-hand sides, g log G bits for
// the pointers to them and one entry per string for C.  The file is:
//
//   header, eight 64-bit words: magic "LCGSLP01", r (rules), G (cells), k
//     (strings), runs (run rules), nb (block bounds), the widths
//     b_sym | b_cell << 8 | b_ptr << 16, the file's size in bytes;
//   R: the right-hand sides of rules 256, 257, ... one after the other, G
//     cells of b_cell bits; a run rule X' -> (X, l) takes two cells, X then l;
//   P: the first cell of every rule in R, r cells of b_ptr bits;
//   M: one bit per rule, set for the run rules;
//   C: k cells of b_sym bits;
//   B: the nb block bounds, 32-bit cells.
//
// Every section starts on a 64-bit word (padding bits are zero); in a section
// of width b, cell i occupies the bits i*b .. i*b+b-1, bit t being bit t mod
// 64 of the little-endian word t / 64.  Widths: b_sym = bits(255 + r), the
// largest id; b_cell = max(b_sym, bits(longest run)); b_ptr = bits(G - 1),
// 1 without rules; bits(x) = the binary digits of x, at least 1.
//
// The decoder accepts exactly what the encoder can write: the header's
// counts, widths (b_cell for the longest run included) and size agree;
// padding bits are zero; the bounds rise from 256 to 256 + r; the
// pointers start at 0 and rise, run rules spanning two cells; every cell of a
// rule in block b names an id below bounds[b] (so rules refer only to smaller
// ids); run lengths are at least 2; C names ids below 256 + r; and no rule
// and no sum of the strings' lengths reaches 2^61 bytes.
namespace {

uint32_t nbits(uint64_t x) {
  uint32_t b = 1;
  while (b < 64 && (x >> b) != 0) ++b;
  return b;
}

uint64_t words_for(uint64_t cells, uint32_t width) { return (cells * width + 63) / 64; }

// one bit at a time, the slow and obvious way
void put_bits(std::vector<uint64_t>& w, uint64_t base_word, uint64_t cell, uint32_t width,
              uint64_t v) {
  for (uint32_t t = 0; t < width; ++t) {
    const uint64_t bit = cell * width + t;
    if ((v >> t) & 1) w[base_word + bit / 64] |= 1ull << (bit % 64);
  }
}

uint64_t get_bits(const std::vector<uint64_t>& w, uint64_t base_word, uint64_t cell,
                  uint32_t width) {
  uint64_t v = 0;
  for (uint32_t t = 0; t < width; ++t) {
    const uint64_t bit = cell * width + t;
    v |= ((w[base_word + bit / 64] >> (bit % 64)) & 1) << t;
  }
  return v;
}

constexpr uint64_t kStoreMagic = 0x3130504C5347434Cull;  // the bytes "LCGSLP01"
constexpr uint64_t kLenLimit = 1ull << 61;

}  // namespace

extern "C" {

// The stored file of s: returns its size in bytes and writes it to out when
// cap is at least that size.
uint64_t oracle_slp_encode(const OracleSlp* s, uint8_t* out, uint64_t cap) {
  const uint64_t r = s->mult.size(), k = s->c.size(), nb = s->bounds.size();
  uint64_t runs = 0, longest = 0;
  for (uint32_t m : s->mult)
    if (m >= 2) {
      ++runs;
      if (m > longest) longest = m;
    }
  const uint64_t G = slp_size(*s);
  const uint32_t b_sym = nbits(255 + r);
  const uint32_t b_cell = std::max(b_sym, runs ? nbits(longest) : 1u);
  const uint32_t b_ptr = r ? nbits(G - 1) : 1;
  const uint64_t wR = words_for(G, b_cell), wP = words_for(r, b_ptr), wM = words_for(r, 1),
                 wC = words_for(k, b_sym), wB = words_for(nb, 32);
  const uint64_t nwords = 8 + wR + wP + wM + wC + wB;
  if (!out || cap < nwords * 8) return nwords * 8;
  std::vector<uint64_t> w(nwords, 0);
  w[0] = kStoreMagic;
  w[1] = r;
  w[2] = G;
  w[3] = k;
  w[4] = runs;
  w[5] = nb;
  w[6] = b_sym | (uint64_t)b_cell << 8 | (uint64_t)b_ptr << 16;
  w[7] = nwords * 8;
  const uint64_t oR = 8, oP = oR + wR, oM = oP + wP, oC = oM + wM, oB = oC + wC;
  uint64_t cell = 0;
  for (uint64_t x = 0; x < r; ++x) {
    put_bits(w, oP, x, b_ptr, cell);
    if (s->mult[x] >= 2) {
      put_bits(w, oR, cell++, b_cell, s->rhs[s->off[x]]);
      put_bits(w, oR, cell++, b_cell, s->mult[x]);
      put_bits(w, oM, x, 1, 1);
    } else {
      for (uint64_t t = s->off[x]; t < s->off[x + 1]; ++t) put_bits(w, oR, cell++, b_cell, s->rhs[t]);
    }
  }
  for (uint64_t j = 0; j < k; ++j) put_bits(w, oC, j, b_sym, s->c[j]);
  for (uint64_t b = 0; b < nb; ++b) put_bits(w, oB, b, 32, s->bounds[b]);
  for (uint64_t i = 0; i < nwords; ++i)
    for (int t = 0; t < 8; ++t) out[i * 8 + t] = (uint8_t)(w[i] >> (8 * t));
  return nwords * 8;
}

// The grammar of a stored file, or NULL (oracle_last_error says why).
OracleSlp* oracle_slp_decode(const uint8_t* in, uint64_t n) {
  auto fail = [](const char* why) -> OracleSlp* {
    g_err = why;
    return nullptr;
  };
  if (n < 64 || n % 8) return fail("size is not a whole header plus words");
  std::vector<uint64_t> w(n / 8, 0);
  for (uint64_t i = 0; i < n / 8; ++i)
    for (int t = 0; t < 8; ++t) w[i] |= (uint64_t)in[i * 8 + t] << (8 * t);
  if (w[0] != kStoreMagic) return fail("bad magic");
  const uint64_t r = w[1], G = w[2], k = w[3], runs = w[4], nb = w[5];
  const uint32_t b_sym = w[6] & 0xFF, b_cell = (w[6] >> 8) & 0xFF, b_ptr = (w[6] >> 16) & 0xFF;
  if (w[6] >> 24) return fail("bad widths word");
  if (w[7] != n) return fail("size differs from the header");
  if (r > 0xFFFFFFFFull - 256 || k == 0 || k > 0xFFFFFFFFull || runs > r || G >= (1ull << 58) ||
      G < r + runs || (r == 0 && G != 0) || nb < 1 || nb > 1024)
    return fail("counts out of range");
  if (b_sym != nbits(255 + r) || b_cell < b_sym || b_cell > 32 || b_ptr != (r ? nbits(G - 1) : 1u))
    return fail("widths do not match the counts");
  const uint64_t wR = words_for(G, b_cell), wP = words_for(r, b_ptr), wM = words_for(r, 1),
                 wC = words_for(k, b_sym), wB = words_for(nb, 32);
  if ((8 + wR + wP + wM + wC + wB) * 8 != n) return fail("sections do not fill the size");
  const uint64_t oR = 8, oP = oR + wR, oM = oP + wP, oC = oM + wM, oB = oC + wC;
  // padding: the bits after a section's last cell are zero
  const uint64_t sec_cells[5][3] = {{oR, G, b_cell}, {oP, r, b_ptr}, {oM, r, 1}, {oC, k, b_sym},
                                    {oB, nb, 32}};
  for (const auto& sc : sec_cells) {
    const uint64_t bits = sc[1] * sc[2];
    if (bits % 64 && (w[sc[0] + bits / 64] >> (bits % 64)) != 0) return fail("nonzero padding");
  }
  std::unique_ptr<OracleSlp> s(new OracleSlp());
  s->bounds.clear();
  for (uint64_t b = 0; b < nb; ++b) s->bounds.push_back((uint32_t)get_bits(w, oB, b, 32));
  if (s->bounds[0] != 256 || s->bounds[nb - 1] != 256 + r) return fail("bad block bounds");
  for (uint64_t b = 1; b < nb; ++b)
    if (s->bounds[b] < s->bounds[b - 1]) return fail("bad block bounds");
  std::vector<uint64_t> start(r + 1, G);
  uint64_t nrun = 0;
  for (uint64_t x = 0; x < r; ++x) {
    start[x] = get_bits(w, oP, x, b_ptr);
    nrun += get_bits(w, oM, x, 1);
  }
  if (nrun != runs) return fail("run count differs from the header");
  if (r && start[0] != 0) return fail("bad rule pointers");
  uint32_t blk = 0;
  for (uint64_t x = 0; x < r; ++x) {
    const bool run = get_bits(w, oM, x, 1) != 0;
    if (start[x + 1] <= start[x] || start[x + 1] - start[x] > 0xFFFFFFFFull ||
        (run && start[x + 1] - start[x] != 2))
      return fail("bad rule pointers");
    while (blk + 1 < nb && s->bounds[blk + 1] <= 256 + x) ++blk;  // the block of rule x
    const uint64_t below = s->bounds[blk];
    const uint64_t a = get_bits(w, oR, start[x], b_cell);
    if (a >= below) return fail("a rule names an id of its own block or above");
    s->rhs.push_back((uint32_t)a);
    if (run) {
      const uint64_t l = get_bits(w, oR, start[x] + 1, b_cell);
      if (l < 2) return fail("a run shorter than 2");
      s->mult.push_back((uint32_t)l);
    } else {
      for (uint64_t i = start[x] + 1; i < start[x + 1]; ++i) {
        const uint64_t y = get_bits(w, oR, i, b_cell);
        if (y >= below) return fail("a rule names an id of its own block or above");
        s->rhs.push_back((uint32_t)y);
      }
      s->mult.push_back(1);
    }
    s->off.push_back(s->rhs.size());
  }
  uint64_t longest = 0;
  for (uint32_t m : s->mult) longest = std::max<uint64_t>(longest, m >= 2 ? m : 0);
  if (b_cell != std::max(b_sym, longest ? nbits(longest) : 1u))
    return fail("widths do not match the longest run");
  for (uint64_t j = 0; j < k; ++j) {
    const uint64_t y = get_bits(w, oC, j, b_sym);
    if (y >= 256 + r) return fail("C names an id beyond the rules");
    s->c.push_back((uint32_t)y);
  }
  // expansion lengths in id order (every rule refers to smaller ids only)
  std::vector<uint64_t> len(r, 0);
  auto len_of = [&](uint32_t y) -> uint64_t { return y < 256 ? 1 : len[y - 256]; };
  for (uint64_t x = 0; x < r; ++x) {
    uint64_t e = 0;
    for (uint64_t t = s->off[x]; t < s->off[x + 1]; ++t) e = std::min(e + len_of(s->rhs[t]), kLenLimit);
    e = e > kLenLimit / s->mult[x] ? kLenLimit : e * s->mult[x];
    if (e >= kLenLimit) return fail("an expansion reaches 2^61 bytes");
    len[x] = e;
  }
  uint64_t total = 0;
  for (uint32_t y : s->c) total = std::min(total + len_of(y), kLenLimit);
  if (total >= kLenLimit) return fail("the strings reach 2^61 bytes");
  const uint64_t G2 = slp_size(*s);
  s->stats[6] = r;
  s->stats[7] = G2;
  return s.release();
}

// Longest common extension of two positions of a collection (the lcp / lcs
// of the match-completion step sketched in App. B), by comparing bytes:
// forward (dir 0): the longest common prefix of T_j1[p1..] and T_j2[p2..];
// backward (dir 1): the longest common suffix of T_j1[..p1) and T_j2[..p2).
// lcp (dir 0) or lcs (dir 1) of exp(X) and exp(Y), X and Y grammar symbols
// given as (level, rank) -- the quantities App. B's MEM sketch completes
// matches with -- by expanding both and comparing bytes.  Returns 0, or -1
// (oracle_last_error) for a symbol that does not exist.
int oracle_symbol_lce(const OracleGrammar* g, uint32_t nq, const uint8_t* lv1, const uint32_t* s1,
                      const uint8_t* lv2, const uint32_t* s2, uint32_t dir, uint64_t* out) {
  auto exists = [&](uint32_t lv, uint32_t x) {
    if (lv == 0) return x < 256;
    return lv <= g->levels.size() && x < g->levels[lv - 1].size();
  };
  for (uint32_t q = 0; q < nq; ++q) {
    if (!exists(lv1[q], s1[q]) || !exists(lv2[q], s2[q])) {
      g_err = "no such symbol";
      return -1;
    }
    std::vector<uint8_t> a(oracle_expand_symbol(g, lv1[q], s1[q], nullptr, 0));
    std::vector<uint8_t> b(oracle_expand_symbol(g, lv2[q], s2[q], nullptr, 0));
    oracle_expand_symbol(g, lv1[q], s1[q], a.data(), a.size());
    oracle_expand_symbol(g, lv2[q], s2[q], b.data(), b.size());
    uint64_t l = 0;
    const uint64_t na = a.size(), nb = b.size();
    if (dir == 0) {
      while (l < na && l < nb && a[l] == b[l]) ++l;
    } else {
      while (l < na && l < nb && a[na - 1 - l] == b[nb - 1 - l]) ++l;
    }
    out[q] = l;
  }
  return 0;
}

void oracle_lce(const uint8_t* text, const uint64_t* off, uint32_t nq, const uint32_t* j1,
                const uint64_t* p1, const uint32_t* j2, const uint64_t* p2, uint32_t dir,
                uint64_t* out) {
  for (uint32_t q = 0; q < nq; ++q) {
    const uint8_t* a = text + off[j1[q]];
    const uint8_t* b = text + off[j2[q]];
    const uint64_t na = off[j1[q] + 1] - off[j1[q]], nb = off[j2[q] + 1] - off[j2[q]];
    uint64_t l = 0;
    if (dir == 0) {
      while (p1[q] + l < na && p2[q] + l < nb && a[p1[q] + l] == b[p2[q] + l]) ++l;
    } else {
      while (l < p1[q] && l < p2[q] && a[p1[q] - 1 - l] == b[p2[q] - 1 - l]) ++l;
    }
    out[q] = l;
  }
}

// Maximal exact matches between strings a and b found through the grammar
// (App. B): the level-`level` parse of each string is obtained by
// substituting right-hand sides from C[j] down to that level; every pair of
// equal symbols, one in each parse, is an anchor, and the match it seeds is
// the longest run of equal bytes on the anchor's diagonal that contains the
// anchor's first byte (the lcs before it and the lcp from it, both on the
// text).  Result: the distinct such matches of at least min_len bytes as
// (start in a, start in b, length), sorted by start in a, then in b; with
// a == b an anchor pairs two different positions of the parse.  Returns the
// number of matches and writes the first min(count, cap); on a bad argument
// returns UINT64_MAX (oracle_last_error).
uint64_t oracle_mems(const OracleGrammar* g, const uint8_t* text, const uint64_t* off, uint32_t a,
                     uint32_t b, uint32_t level, uint64_t min_len, uint64_t cap, uint64_t* pa,
                     uint64_t* pb, uint64_t* len) {
  const uint32_t k = (uint32_t)g->c_level.size();
  if (a >= k || b >= k) {
    g_err = "no such string";
    return UINT64_MAX;
  }
  if (level < 1 || level > g->c_level[a] || level > g->c_level[b]) {
    g_err = "level outside 1..min(level of C[a], level of C[b])";
    return UINT64_MAX;
  }
  auto parse = [&](uint32_t j) {
    std::vector<uint32_t> cur(1, g->c_sym[j]);
    for (uint32_t l = g->c_level[j]; l > level; --l) {
      const Level& L = g->levels[l - 1];
      std::vector<uint32_t> next;
      for (uint32_t x : cur)
        for (uint64_t t = L.rhs_off[x]; t < L.rhs_off[x + 1]; ++t) next.push_back(L.rhs[t]);
      cur.swap(next);
    }
    return cur;
  };
  std::unordered_map<uint32_t, uint64_t> elen;  // expansion length per level symbol
  auto starts = [&](const std::vector<uint32_t>& ps) {
    std::vector<uint64_t> st(ps.size());
    uint64_t p = 0;
    for (size_t i = 0; i < ps.size(); ++i) {
      st[i] = p;
      auto it = elen.find(ps[i]);
      if (it == elen.end())
        it = elen.emplace(ps[i], oracle_expand_symbol(g, level, ps[i], nullptr, 0)).first;
      p += it->second;
    }
    return st;
  };
  const std::vector<uint32_t> A = parse(a), B = parse(b);
  const std::vector<uint64_t> xa = starts(A), xb = starts(B);
  std::unordered_map<uint32_t, std::vector<uint32_t>> where;  // symbol -> its indexes in B
  for (uint32_t j = 0; j < B.size(); ++j) where[B[j]].push_back(j);
  const uint8_t* ta = text + off[a];
  const uint8_t* tb = text + off[b];
  const uint64_t na = off[a + 1] - off[a], nb = off[b + 1] - off[b];
  std::vector<std::array<uint64_t, 3>> found;
  for (uint32_t i = 0; i < A.size(); ++i) {
    auto it = where.find(A[i]);
    if (it == where.end()) continue;
    for (uint32_t j : it->second) {
      if (a == b && i == j) continue;
      const uint64_t x = xa[i], y = xb[j];
      uint64_t back = 0, fwd = 0;
      while (back < x && back < y && ta[x - 1 - back] == tb[y - 1 - back]) ++back;
      while (x + fwd < na && y + fwd < nb && ta[x + fwd] == tb[y + fwd]) ++fwd;
      if (back + fwd >= min_len) found.push_back({x - back, y - back, back + fwd});
    }
  }
  std::sort(found.begin(), found.end());
  found.erase(std::unique(found.begin(), found.end()), found.end());
  for (uint64_t q = 0; q < found.size() && q < cap; ++q) {
    pa[q] = found[q][0];
    pb[q] = found[q][1];
    len[q] = found[q][2];
  }
  return found.size();
}

}  // extern "C"
