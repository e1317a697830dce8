// Post-processing of a level grammar on the device: run-length compression
// (RL) and grammar simplification (Simp), Sec. 2.2 of the paper, applied in
// the order of Sec. 4 (RL, then Simp).  The result is a straight-line grammar
// (lcg_slp in include/lcg.h) with one id space:
//
//   ids 0..255     terminals;
//   then, for every level i = 1, 2, ... of the input: the run rules made from
//                  level i's right-hand sides, in (symbol, length) order,
//                  followed by level i's rules in rank order;
//   rule X:        exp(X) = exp(rhs(X))^mult(X); a run rule (X', l) is
//                  rhs = [X], mult = l >= 2, an ordinary rule has mult = 1.
//
// Simp removes every ordinary rule whose id occurs exactly once over all
// right-hand sides and C with that occurrence in an ordinary rule, splices its
// right-hand side in place of the occurrence, and numbers the kept rules in id
// order from 256.
//
// Everything is data-parallel: positions and rules are flagged, scanned and
// scattered, runs are deduplicated with a radix sort, and the spliced
// right-hand sides are written in one pass from prefix sums of per-position
// weights (a kept symbol weighs 1, a removed one its flattened length).
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <initializer_list>
#include <memory>

#include "lcg_host.h"

struct lcg_slp {
  uint64_t seed = 0;
  uint32_t g = 0;   // rules: ids 256 .. 256 + g - 1
  uint64_t q = 0;   // total right-hand-side length
  uint32_t k = 0;   // strings
  lcg::DBuf<uint64_t> off;   // g + 1
  lcg::DBuf<uint32_t> rhs;   // q
  lcg::DBuf<uint32_t> mult;  // g
  lcg::DBuf<uint32_t> c;     // k
  uint64_t stats[LCG_SLP_STATS] = {};
  // id blocks in dependency order (per input level: its run rules, then its
  // ordinary rules): rules of a block refer only to earlier blocks
  std::vector<uint32_t> bounds;
  // for the expansion, computed on first use: expansion length E and number of
  // nonterminals NT of every rule's right-hand side
  lcg::DBuf<uint64_t> E;
  lcg::DBuf<uint32_t> nt;
  // per right-hand-side position t of rule r (prefix sums over all positions;
  // subtract the value at off[r]): S = expansion bytes before t, N = item
  // children (nonterminals that are not leaves) before t
  lcg::DBuf<uint64_t> S, N;
  lcg::DBuf<uint8_t> meta;  // RuleMeta per rule
  // item children of the item children (the step after next), per rule
  lcg::DBuf<uint64_t> gnt;
  // per rule: E, with the top bit set for a leaf
  lcg::DBuf<uint64_t> el;
  // every leaf's expansion (mult copies of its terminals), one after the other
  lcg::DBuf<uint8_t> lbytes;
  bool lens_ready = false;
};

namespace lcg {
namespace {

constexpr int kPB = 256;

inline unsigned pgrid(uint64_t n) {
  uint64_t b = (n + kPB - 1) / kPB;
  if (b < 1) b = 1;
  if (b > 16384) b = 16384;
  return (unsigned)b;
}

#define PP_LOOP(i, n)                                                                  \
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < (uint64_t)(n); \
       i += (uint64_t)gridDim.x * blockDim.x)

#define PP_CHECK(name)                                                                 \
  do {                                                                                 \
    hipError_t e_ = hipGetLastError();                                                 \
    if (e_ != hipSuccess)                                                              \
      throw LcgError{LCG_EHIP, std::string("launch of ") + name + ": " +               \
                                   hipGetErrorString(e_)};                             \
  } while (0)

__global__ void k_pp_set(uint64_t* p, uint64_t v) { *p = v; }

// ---------------------------------------------------------------- rule groups
// Kernels that visit right-hand-side positions take groups of kGrp
// consecutive rules per block (one thread per rule of the group): the
// group's offsets go to LDS, the block reads the group's positions in tiles
// (below) and each position finds its rule by binary search in LDS.
constexpr uint32_t kGrp = 256;

#define GROUP_LOOP(grp, ngroups) for (uint64_t grp = blockIdx.x; grp < (ngroups); grp += gridDim.x)

__device__ __forceinline__ void load_offsets(const uint64_t* __restrict__ off, uint64_t r0, uint32_t n,
                                             uint64_t* s_off) {
  for (uint32_t j = threadIdx.x; j <= n; j += blockDim.x) s_off[j] = off[r0 + j];
  __syncthreads();
}

// the rule j < n of the group whose positions hold t (s_off[0] <= t < s_off[n])
__device__ __forceinline__ uint32_t owner_in(const uint64_t* s_off, uint32_t n, uint64_t t) {
  uint32_t lo = 0;
  for (uint32_t step = kGrp / 2; step; step >>= 1) {
    const uint32_t mid = lo + step;
    if (mid < n && s_off[mid] <= t) lo = mid;
  }
  return lo;
}

// A group's positions go in tiles of kTile: each thread takes kPer
// consecutive positions, loads all of them before using any (the loads of a
// tile are in flight together), and walks their owners forward from one
// binary search.  Prefix sums over a tile come from one block scan of the
// threads' totals.
constexpr int kPer = 4;
constexpr uint32_t kTile = kGrp * kPer;

// A tile's right-hand-side symbols staged through LDS: loaded coalesced
// (thread i takes base + i + kGrp * m, all kPer loads in flight), read back
// kPer consecutive ones per thread.
__device__ __forceinline__ void stage_tile(const uint32_t* __restrict__ rhs, uint64_t base,
                                           uint64_t end, uint32_t* s_buf, uint32_t* y) {
  uint32_t v[kPer];
#pragma unroll
  for (int m = 0; m < kPer; ++m) {
    const uint64_t t = base + threadIdx.x + (uint64_t)kGrp * m;
    v[m] = t < end ? rhs[t] : 0;
  }
  __syncthreads();  // the previous tile's reads are done
#pragma unroll
  for (int m = 0; m < kPer; ++m) s_buf[threadIdx.x + kGrp * m] = v[m];
  __syncthreads();
#pragma unroll
  for (int m = 0; m < kPer; ++m) y[m] = s_buf[kPer * threadIdx.x + m];
}

// the owner of t, given the owner j of t - 1 (or of t itself): rules are
// never empty, so one position crosses at most one rule start
__device__ __forceinline__ uint32_t owner_from(const uint64_t* s_off, uint32_t n, uint32_t j,
                                               uint64_t t) {
  return j + (uint32_t)(j + 1 < n && s_off[j + 1] <= t);
}

__device__ __forceinline__ uint64_t lower_bound_u64(const uint64_t* a, uint64_t n, uint64_t key) {
  uint64_t lo = 0, hi = n;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// ---------------------------------------------------------------- RL
// One input level in the global position space (all levels' right-hand sides
// one after the other).  The second half is filled once the runs are known.
struct PLevel {
  const void* rhs;       // uint8 (bytes) or uint32 symbols
  const uint64_t* off;   // u + 1 offsets
  uint64_t p0;           // global position of the level's first symbol
  uint64_t q;
  uint32_t u;
  uint32_t gpre;         // first rule group of the level
  uint32_t bytes;
  uint32_t symbase;      // id of the level's symbol 0 (0: terminals)
  uint64_t cpre;         // repeated positions in earlier levels
  uint64_t out0;         // result position of the level's first ordinary symbol
  uint32_t rlbase;       // id of its first run rule
  uint32_t obase;        // id of its rule 0
  uint32_t upre;         // its first entry in the distinct-run list
  uint32_t v;            // its run rules
};

__device__ __forceinline__ uint32_t sym_at(const PLevel& L, uint64_t t) {
  return L.bytes ? (uint32_t) static_cast<const uint8_t*>(L.rhs)[t]
                 : static_cast<const uint32_t*>(L.rhs)[t];
}

// The level table in LDS (the kernels below read it once per group).
__device__ __forceinline__ void load_tab(const PLevel* __restrict__ tab, uint32_t h,
                                         PLevel* s_tab) {
  static_assert(sizeof(PLevel) % 8 == 0, "PLevel is copied in 8-byte words");
  const uint64_t* src = reinterpret_cast<const uint64_t*>(tab);
  uint64_t* dst = reinterpret_cast<uint64_t*>(s_tab);
  for (uint32_t i = threadIdx.x; i < h * (uint32_t)(sizeof(PLevel) / 8); i += blockDim.x)
    dst[i] = src[i];
  __syncthreads();
}

// the level of group grp, from lv forward (a block's groups only increase)
__device__ __forceinline__ uint32_t level_of_group(const PLevel* s_tab, uint32_t h, uint32_t lv,
                                                  uint64_t grp) {
  while (lv + 1 < h && s_tab[lv + 1].gpre <= grp) ++lv;
  return lv;
}

__device__ __forceinline__ uint32_t level_of_pos(const PLevel* tab, uint32_t h, uint64_t x) {
  uint32_t lv = 0;
  while (lv + 1 < h && tab[lv + 1].p0 <= x) ++lv;
  return lv;
}

// A position repeats when it is not its rule's first and holds the same
// symbol as the position before it; the repeated positions, in order, are the
// list P that RL works from.

// The symbols of positions t0 - 1 .. t0 + kPer of a level (0 outside it),
// t0 = base + kPer * threadIdx.x: the tile's symbols staged through LDS
// (coalesced loads, all in flight), the two outside the tile loaded once.
__device__ __forceinline__ void load_window(const PLevel& L, uint64_t base, uint32_t* s_buf,
                                            uint32_t* x) {
  uint32_t v[kPer];
#pragma unroll
  for (int m = 0; m < kPer; ++m) {
    const uint64_t t = base + threadIdx.x + (uint64_t)kGrp * m;
    v[m] = t < L.q ? sym_at(L, t) : 0;
  }
  uint32_t edge = 0;
  if (threadIdx.x == 0) edge = base >= 1 ? sym_at(L, base - 1) : 0;
  if (threadIdx.x == kGrp - 1) edge = base + kTile < L.q ? sym_at(L, base + kTile) : 0;
  __syncthreads();  // the previous tile's reads are done
#pragma unroll
  for (int m = 0; m < kPer; ++m) s_buf[threadIdx.x + kGrp * m] = v[m];
  __syncthreads();
  const uint32_t i0 = kPer * threadIdx.x;
  x[0] = threadIdx.x ? s_buf[i0 - 1] : edge;
#pragma unroll
  for (int m = 0; m < kPer; ++m) x[m + 1] = s_buf[i0 + m];
  x[kPer + 1] = threadIdx.x + 1 < kGrp ? s_buf[i0 + kPer] : edge;
}

// repeat flags of a thread's positions of a tile; returns how many are set
__device__ __forceinline__ uint32_t tile_repeats(const uint64_t* s_off, uint32_t n, uint64_t t0,
                                                 uint64_t b, const uint32_t* x, bool* rep,
                                                 uint32_t* jj) {
  uint32_t j = t0 < b ? owner_in(s_off, n, t0) : 0, cnt = 0;
#pragma unroll
  for (int m = 0; m < kPer; ++m) {
    const uint64_t t = t0 + m;
    rep[m] = false;
    jj[m] = j;
    if (t >= b) continue;
    j = owner_from(s_off, n, j, t);
    jj[m] = j;
    rep[m] = t != s_off[j] && x[m + 1] == x[m];
    cnt += rep[m];
  }
  return cnt;
}

// repeated positions of every rule group
__global__ __launch_bounds__(kGrp) void k_pp_repcount(const PLevel* __restrict__ tab, uint32_t h,
                                                      uint64_t ngroups, uint64_t* __restrict__ gcnt) {
  __shared__ uint32_t s_y[kTile];
  __shared__ uint64_t s_off[kGrp + 1];
  __shared__ uint32_t s_w[kGrp / 64];
  __shared__ PLevel s_tab[64];
  load_tab(tab, h, s_tab);
  uint32_t lv = 0;
  GROUP_LOOP(grp, ngroups) {
    lv = level_of_group(s_tab, h, lv, grp);
    const PLevel L = s_tab[lv];
    const uint64_t r0 = (grp - L.gpre) * kGrp;
    const uint32_t n = (uint32_t)min<uint64_t>(kGrp, L.u - r0);
    load_offsets(L.off, r0, n, s_off);
    const uint64_t a = s_off[0], b = s_off[n];
    uint32_t mine = 0;
    for (uint64_t base = a; base < b; base += kTile) {
      const uint64_t t0 = base + kPer * threadIdx.x;
      uint32_t x[kPer + 2], jj[kPer];
      bool rep[kPer];
      load_window(L, base, s_y, x);
      mine += tile_repeats(s_off, n, t0, b, x, rep, jj);
    }
    uint32_t total;
    block_excl_scan<uint32_t, kGrp>(mine, s_w, &total);
    if (threadIdx.x == 0) gcnt[grp] = total;
    __syncthreads();  // s_off is rewritten by the next group
  }
}

// P[gpos[grp] + ...] = the group's repeated positions (global), in order
__global__ __launch_bounds__(kGrp) void k_pp_repwrite(const PLevel* __restrict__ tab, uint32_t h,
                                                      uint64_t ngroups, const uint64_t* __restrict__ gpos,
                                                      uint64_t* __restrict__ P) {
  __shared__ uint32_t s_y[kTile];
  __shared__ uint64_t s_off[kGrp + 1];
  __shared__ uint32_t s_w[kGrp / 64];
  __shared__ PLevel s_tab[64];
  load_tab(tab, h, s_tab);
  uint32_t lv = 0;
  GROUP_LOOP(grp, ngroups) {
    const uint64_t g0 = gpos[grp];
    if (gpos[grp + 1] == g0) continue;  // no repeats in the group (uniform)
    lv = level_of_group(s_tab, h, lv, grp);
    const PLevel L = s_tab[lv];
    const uint64_t r0 = (grp - L.gpre) * kGrp;
    const uint32_t n = (uint32_t)min<uint64_t>(kGrp, L.u - r0);
    load_offsets(L.off, r0, n, s_off);
    const uint64_t a = s_off[0], b = s_off[n];
    uint64_t done = g0;
    for (uint64_t base = a; base < b; base += kTile) {
      const uint64_t t0 = base + kPer * threadIdx.x;
      uint32_t x[kPer + 2], jj[kPer];
      bool rep[kPer];
      load_window(L, base, s_y, x);
      const uint32_t cnt = tile_repeats(s_off, n, t0, b, x, rep, jj);
      uint32_t tot;
      uint64_t o = done + block_excl_scan<uint32_t, kGrp>(cnt, s_w, &tot);
#pragma unroll
      for (int m = 0; m < kPer; ++m)
        if (rep[m]) P[o++] = L.p0 + t0 + m;
      done += tot;
    }
    __syncthreads();
  }
}

// gpos at the first group of every level, and the total (for the host)
__global__ void k_pp_level_reps(const PLevel* __restrict__ tab, uint32_t h, uint64_t ngroups,
                                const uint64_t* __restrict__ gpos, uint64_t* __restrict__ out) {
  PP_LOOP(i, h + 1) out[i] = gpos[i < h ? tab[i].gpre : ngroups];
}

// Runs from the sorted repeated positions P: a run X^l (l >= 2) starting at s
// is the group of consecutive entries s+1 .. s+l-1.  At each group's first
// entry i: rlen[i] = l, and (level, key = X << 32 | l) is appended to the run
// list; rlen is 0 at the other entries.
__global__ void k_pp_runs(const PLevel* __restrict__ tab, uint32_t h, const uint64_t* __restrict__ P,
                          uint64_t c, uint32_t* __restrict__ rlen, uint64_t* __restrict__ rkey,
                          uint32_t* __restrict__ rlvl, unsigned long long* __restrict__ rcount) {
  PP_LOOP(i, c) {
    const uint64_t x = P[i];
    if (i > 0 && P[i - 1] == x - 1) {
      rlen[i] = 0;
      continue;
    }
    // last e >= i with P[e] - x == e - i (P strictly increases, so this holds
    // exactly on a prefix)
    uint64_t lo = i, hi = c - 1;
    while (lo < hi) {
      const uint64_t mid = (lo + hi + 1) >> 1;
      if (P[mid] - x == mid - i) lo = mid; else hi = mid - 1;
    }
    const uint64_t l = lo - i + 2;  // < 2^32: a run lies inside one rule
    rlen[i] = (uint32_t)l;
    const uint64_t s = x - 1;
    const uint32_t lv = level_of_pos(tab, h, s);
    const uint32_t X = sym_at(tab[lv], s - tab[lv].p0);
    const unsigned long long at = atomicAdd(rcount, 1ull);
    rkey[at] = ((uint64_t)X << 32) | l;
    rlvl[at] = lv;
  }
}

// distinct (level, key) pairs of the sorted run list
__global__ void k_pp_uniqflag(const uint32_t* __restrict__ lvl, const uint64_t* __restrict__ key,
                              uint64_t R, uint64_t* __restrict__ flag) {
  PP_LOOP(j, R) flag[j] = (j == 0 || lvl[j] != lvl[j - 1] || key[j] != key[j - 1]) ? 1 : 0;
}

__global__ void k_pp_uniqlist(const uint32_t* __restrict__ lvl, const uint64_t* __restrict__ key,
                              const uint64_t* __restrict__ flag, const uint64_t* __restrict__ pos,
                              uint64_t R, uint32_t* __restrict__ ulvl, uint64_t* __restrict__ ukey,
                              unsigned long long* __restrict__ vcnt) {
  PP_LOOP(j, R) {
    if (!flag[j]) continue;
    ulvl[pos[j]] = lvl[j];
    ukey[pos[j]] = key[j];
    atomicAdd(&vcnt[lvl[j]], 1ull);
  }
}

// Every level's ordinary rules after RL: one symbol per maximal run (the run
// rule's id for a run of length >= 2), the rules' offsets and multiplicities.
// A group's repeated positions before a position come from gpos and the
// tile's scan of repeat flags; the first position of a run of length >= 2
// finds the run's entry in P from that count.
__global__ __launch_bounds__(kGrp) void k_pp_rl_write(const PLevel* __restrict__ tab, uint32_t h,
                                                      uint64_t ngroups, const uint64_t* __restrict__ gpos,
                                                      const uint64_t* __restrict__ P, uint64_t c,
                                                      const uint32_t* __restrict__ rlen,
                                                      const uint64_t* __restrict__ ukey,
                                                      uint32_t* __restrict__ rhs1,
                                                      uint64_t* __restrict__ off1,
                                                      uint32_t* __restrict__ mult1) {
  __shared__ uint32_t s_y[kTile];
  __shared__ uint64_t s_off[kGrp + 1];
  __shared__ uint32_t s_w[kGrp / 64];
  __shared__ PLevel s_tab[64];
  load_tab(tab, h, s_tab);
  uint32_t lv = 0;
  GROUP_LOOP(grp, ngroups) {
    lv = level_of_group(s_tab, h, lv, grp);
    const PLevel L = s_tab[lv];
    const uint64_t r0 = (grp - L.gpre) * kGrp;
    const uint32_t n = (uint32_t)min<uint64_t>(kGrp, L.u - r0);
    load_offsets(L.off, r0, n, s_off);
    const uint64_t a = s_off[0], b = s_off[n];
    const bool any = gpos[grp + 1] != gpos[grp];  // uniform
    uint64_t done = gpos[grp] - L.cpre;           // the level's repeats before the tile
    for (uint64_t base = a; base < b; base += kTile) {
      const uint64_t t0 = base + kPer * threadIdx.x;
      uint32_t x[kPer + 2], jj[kPer];
      bool rep[kPer];
      load_window(L, base, s_y, x);
      const uint32_t cnt = tile_repeats(s_off, n, t0, b, x, rep, jj);
      uint32_t before = 0, tot = 0;
      if (any) {
        before = block_excl_scan<uint32_t, kGrp>(cnt, s_w, &tot);
      } else {  // no repeats counted here (or RL is off): every position stays
#pragma unroll
        for (int m = 0; m < kPer; ++m) rep[m] = false;
      }
      uint64_t gone = done + before;
#pragma unroll
      for (int m = 0; m < kPer; ++m) {
        const uint64_t t = t0 + m;
        if (t >= b) break;
        if (rep[m]) {
          ++gone;
          continue;
        }
        const uint64_t out = L.out0 + t - gone;
        const uint32_t X = x[m + 1];
        const uint32_t j = jj[m];
        uint32_t id = L.symbase + X;
        // the next position repeats: t starts a run of length >= 2
        if (c && t + 1 < s_off[j + 1] && x[m + 2] == X) {
          // t + 1 is the next repeated position: its entry in P follows the
          // level's and the group's repeats before it
          const uint64_t key = ((uint64_t)X << 32) | rlen[L.cpre + gone];
          id = L.rlbase + (uint32_t)lower_bound_u64(ukey + L.upre, L.v, key);
        }
        rhs1[out] = id;
        if (t == s_off[j]) {
          off1[L.obase - 256 + r0 + j] = out;
          mult1[L.obase - 256 + r0 + j] = 1;
        }
      }
      done += tot;
    }
    __syncthreads();
  }
}

// the run rules: rhs = [X], mult = l, ahead of their level's ordinary rules
__global__ void k_pp_rl_rules(const PLevel* __restrict__ tab, const uint32_t* __restrict__ ulvl,
                              const uint64_t* __restrict__ ukey, uint64_t vt,
                              uint32_t* __restrict__ rhs1, uint64_t* __restrict__ off1,
                              uint32_t* __restrict__ mult1) {
  PP_LOOP(j, vt) {
    const PLevel& L = tab[ulvl[j]];
    const uint32_t jl = (uint32_t)j - L.upre;
    const uint64_t key = ukey[j];
    const uint64_t pos = L.out0 - L.v + jl;
    rhs1[pos] = L.symbase + (uint32_t)(key >> 32);
    off1[L.rlbase - 256 + jl] = pos;
    mult1[L.rlbase - 256 + jl] = (uint32_t)key;
  }
}

// C in global ids (obase[lv]: id of rule 0 of level lv)
__global__ void k_pp_c_global(const uint8_t* __restrict__ cl, const uint32_t* __restrict__ cs,
                              uint32_t k, const uint32_t* __restrict__ obase,
                              uint32_t* __restrict__ c1) {
  PP_LOOP(j, k) {
    const uint32_t lv = cl[j];
    c1[j] = lv == 0 ? cs[j] : obase[lv] + cs[j];
  }
}

// ---------------------------------------------------------------- Simp
// Occurrence counts matter only up to 2.  They are counted per rule (occ:
// +1 in an ordinary rule, +2 in a run rule or C), then folded into a 2-bit
// field per rule, 16 to a 32-bit word: bit A (the low one) for exactly one
// ordinary occurrence, bit B for a rule kept for good (two or more, a run
// rule's symbol, a C entry, or a run rule itself).  A rule is removed by Simp
// exactly when its field is A alone.  Each word is stored with the number of
// removed rules in the words before it (rk: fields in the low 32 bits, that
// count in the high ones), so a kept rule's new id is one 8-byte read of a
// small array (4 bits per rule) and a popcount.
__device__ __forceinline__ uint32_t rm_bits(uint32_t f) { return f & 0x55555555u & ~(f >> 1); }

__device__ __forceinline__ bool pp_rm(const uint64_t* __restrict__ rk, uint32_t z) {
  return (rm_bits((uint32_t)rk[z >> 4]) >> (2 * (z & 15))) & 1;
}

// 256 + the kept rules before z: the new id of a kept rule z, and for any
// z <= g1 the first new id at or after it
__device__ __forceinline__ uint32_t pp_newid(const uint64_t* __restrict__ rk, uint32_t z) {
  const uint64_t w = rk[z >> 4];
  const uint32_t below = rm_bits((uint32_t)w) & ((1u << (2 * (z & 15))) - 1);
  return 256 + z - ((uint32_t)(w >> 32) + (uint32_t)__builtin_popcount(below));
}

// Occurrences over the right-hand sides: +1 in an ordinary rule, +2 in a run
// rule (which pins the symbol).  Counts stop mattering at 2.  The first
// ordinary occurrence records its rule; it is the only one when the count
// ends at 1.  One position per thread and pass (consecutive threads,
// consecutive positions): the tiles above measured slower here.
__global__ __launch_bounds__(kGrp) void k_pp_occ(const uint64_t* __restrict__ off1,
                                                 const uint32_t* __restrict__ rhs1,
                                                 const uint32_t* __restrict__ mult1, uint32_t g1,
                                                 uint32_t* occ, uint32_t* __restrict__ par) {
  __shared__ uint64_t s_off[kGrp + 1];
  __shared__ uint8_t s_run[kGrp];
  const uint64_t ngroups = (g1 + kGrp - 1) / kGrp;
  GROUP_LOOP(grp, ngroups) {
    const uint64_t r0 = grp * kGrp;
    const uint32_t n = (uint32_t)min<uint64_t>(kGrp, g1 - r0);
    if (threadIdx.x < n) s_run[threadIdx.x] = mult1[r0 + threadIdx.x] >= 2;
    load_offsets(off1, r0, n, s_off);
    const uint64_t a = s_off[0], b = s_off[n];
    for (uint64_t t = a + threadIdx.x; t < b; t += kGrp) {
      const uint32_t y = rhs1[t];
      if (y < 256) continue;
      const uint32_t z = y - 256;
      if (__hip_atomic_load(&occ[z], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= 2) continue;
      const uint32_t j = owner_in(s_off, n, t);
      if (s_run[j]) {
        atomicAdd(&occ[z], 2u);
      } else if (atomicAdd(&occ[z], 1u) == 0) {
        par[z] = (uint32_t)(r0 + j);
      }
    }
    __syncthreads();
  }
}

__global__ void k_pp_occ_c(const uint32_t* __restrict__ c1, uint32_t k, uint32_t* occ) {
  PP_LOOP(j, k) if (c1[j] >= 256) atomicAdd(&occ[c1[j] - 256], 2u);
}

// the fields of 16 rules per word from the counts, and the removed rules per
// word, for the scan that rk stores
__global__ void k_pp_fields(const uint32_t* __restrict__ occ, const uint32_t* __restrict__ mult1,
                            uint32_t g1, uint64_t nwords, uint32_t* __restrict__ oc2,
                            uint64_t* __restrict__ cnt) {
  PP_LOOP(w, nwords) {
    uint32_t f = 0;
    for (uint32_t i = 0; i < 16; ++i) {
      const uint64_t r = w * 16 + i;
      if (r >= g1) break;
      const uint32_t o = occ[r];
      const uint32_t v = (mult1[r] >= 2 || o >= 2) ? 2u : (o == 1 ? 1u : 0u);
      f |= v << (2 * i);
    }
    oc2[w] = f;
    cnt[w] = (uint64_t)__builtin_popcount(rm_bits(f));
  }
}

// rk[w] = removed rules before word w << 32 | the word's fields (w <= nwords)
__global__ void k_pp_pack(const uint32_t* __restrict__ oc2, const uint64_t* __restrict__ pre,
                          uint64_t nwords, uint64_t* __restrict__ rk) {
  PP_LOOP(w, nwords + 1) rk[w] = (pre[w] << 32) | (w < nwords ? oc2[w] : 0u);
}

// The weights of a tile's positions (1 for a terminal or a kept symbol, the
// flattened length W of a removed one), their prefix within the group
// (carry: the tiles before), and the prefix at every rule's first position
// (s_rs).  On return
// ex[m] is the weight before position t0 + m in the group, jj[m] its rule;
// after the block barrier that follows, ex[m] - s_rs[jj[m]] is its offset
// inside the rule.
__device__ __forceinline__ void tile_prefix(const uint64_t* s_off, uint32_t n, uint64_t t0,
                                            uint64_t b, const uint64_t* w, uint64_t carry,
                                            uint64_t* s_rs, uint64_t* s_w, uint64_t* ex,
                                            uint32_t* jj, uint64_t* tot) {
  uint64_t sum = 0;
#pragma unroll
  for (int m = 0; m < kPer; ++m) sum += w[m];
  uint64_t e = carry + block_excl_scan<uint64_t, kGrp>(sum, s_w, tot);
  uint32_t j = t0 < b ? owner_in(s_off, n, t0) : 0;
#pragma unroll
  for (int m = 0; m < kPer; ++m) {
    const uint64_t t = t0 + m;
    ex[m] = e;
    jj[m] = j;
    if (t >= b) continue;
    j = owner_from(s_off, n, j, t);
    jj[m] = j;
    if (t == s_off[j]) s_rs[j] = e;
    e += w[m];
  }
}

// Flattened length W of the ordinary rules [rb, re) of one level (the levels
// below are done) and, for every removed symbol they hold, its offset inside
// the holding rule (inoff).
__global__ __launch_bounds__(kGrp) void k_pp_flat(const uint64_t* __restrict__ off1,
                                                  const uint32_t* __restrict__ rhs1,
                                                  const uint64_t* __restrict__ rk, uint32_t rb,
                                                  uint32_t re, uint64_t* W,
                                                  uint64_t* __restrict__ inoff) {
  __shared__ uint32_t s_y[kTile];
  __shared__ uint64_t s_off[kGrp + 1];
  __shared__ uint64_t s_rs[kGrp + 1];
  __shared__ uint64_t s_w[kGrp / 64];
  const uint64_t ngroups = (re - rb + kGrp - 1) / kGrp;
  GROUP_LOOP(grp, ngroups) {
    const uint64_t r0 = rb + grp * kGrp;
    const uint32_t n = (uint32_t)min<uint64_t>(kGrp, re - r0);
    load_offsets(off1, r0, n, s_off);
    const uint64_t a = s_off[0], b = s_off[n];
    uint64_t carry = 0;
    for (uint64_t base = a; base < b; base += kTile) {
      const uint64_t t0 = base + kPer * threadIdx.x;
      uint32_t y[kPer];
      stage_tile(rhs1, base, b, s_y, y);
      uint64_t w[kPer];
      bool rem[kPer];
#pragma unroll
      for (int m = 0; m < kPer; ++m) {
        const bool valid = t0 + m < b;
        rem[m] = valid && y[m] >= 256 && pp_rm(rk, y[m] - 256);
        w[m] = rem[m] ? W[y[m] - 256] : (valid ? 1 : 0);
      }
      uint64_t ex[kPer], tot;
      uint32_t jj[kPer];
      tile_prefix(s_off, n, t0, b, w, carry, s_rs, s_w, ex, jj, &tot);
      __syncthreads();  // s_rs of the rules starting in this tile
#pragma unroll
      for (int m = 0; m < kPer; ++m)
        if (rem[m]) inoff[y[m] - 256] = ex[m] - s_rs[jj[m]];
      carry += tot;
    }
    if (threadIdx.x == 0) s_rs[n] = carry;
    __syncthreads();
    if (threadIdx.x < n) W[r0 + threadIdx.x] = s_rs[threadIdx.x + 1] - s_rs[threadIdx.x];
    __syncthreads();  // s_off and s_rs are rewritten by the next group
  }
}

// output length of every rule: 0 removed, 1 for a run rule, W otherwise
__global__ void k_pp_len(const uint64_t* __restrict__ rk, const uint32_t* __restrict__ mult1,
                         const uint64_t* __restrict__ W, uint32_t g1, uint64_t* __restrict__ len) {
  PP_LOOP(r, g1) len[r] = pp_rm(rk, (uint32_t)r) ? 0 : (mult1[r] >= 2 ? 1 : W[r]);
}

// where the removed rules of [rb, re) land in the output (upper levels done):
// the output position of the holder plus the weights before the occurrence
__global__ void k_pp_base(const uint64_t* __restrict__ rk, const uint32_t* __restrict__ par,
                          const uint64_t* __restrict__ inoff, const uint64_t* __restrict__ so,
                          uint32_t rb, uint32_t re, uint64_t* base) {
  PP_LOOP(i, re - rb) {
    const uint32_t r = rb + (uint32_t)i;
    if (!pp_rm(rk, r)) continue;
    const uint32_t p = par[r];
    const uint64_t dp = pp_rm(rk, p) ? base[p] : so[p];
    base[r] = dp + inoff[r];
  }
}

// every kept symbol of every rule at its output position (the rule's, plus
// the weights before the symbol inside the rule); kept rules' offsets and
// multiplicities
__global__ __launch_bounds__(kGrp) void k_pp_write(const uint64_t* __restrict__ off1,
                                                   const uint32_t* __restrict__ rhs1,
                                                   const uint32_t* __restrict__ mult1,
                                                   const uint64_t* __restrict__ rk,
                                                   const uint64_t* __restrict__ W,
                                                   const uint64_t* __restrict__ so,
                                                   const uint64_t* __restrict__ base, uint32_t g1,
                                                   uint32_t* __restrict__ rhs2,
                                                   uint64_t* __restrict__ off2,
                                                   uint32_t* __restrict__ mult2) {
  __shared__ uint32_t s_y[kTile];
  __shared__ uint64_t s_off[kGrp + 1];
  __shared__ uint64_t s_rs[kGrp + 1];
  __shared__ uint64_t s_dest[kGrp];  // output position of the rule's first symbol
  __shared__ uint64_t s_w[kGrp / 64];
  const uint64_t ngroups = (g1 + kGrp - 1) / kGrp;
  GROUP_LOOP(grp, ngroups) {
    const uint64_t r0 = grp * kGrp;
    const uint32_t n = (uint32_t)min<uint64_t>(kGrp, g1 - r0);
    if (threadIdx.x < n) {
      const uint32_t r = (uint32_t)(r0 + threadIdx.x);
      const bool keep = !pp_rm(rk, r);
      s_dest[threadIdx.x] = keep ? so[r] : base[r];
      if (keep) {
        const uint32_t id = pp_newid(rk, r) - 256;
        off2[id] = so[r];
        mult2[id] = mult1[r];
      }
    }
    load_offsets(off1, r0, n, s_off);
    const uint64_t a = s_off[0], b = s_off[n];
    uint64_t carry = 0;
    for (uint64_t base0 = a; base0 < b; base0 += kTile) {
      const uint64_t t0 = base0 + kPer * threadIdx.x;
      uint32_t y[kPer];
      stage_tile(rhs1, base0, b, s_y, y);
      uint64_t w[kPer];
      uint32_t id[kPer];  // the new id of a kept symbol (one read of rk per position)
      bool rem[kPer];
#pragma unroll
      for (int m = 0; m < kPer; ++m) {
        const bool valid = t0 + m < b;
        id[m] = y[m];
        rem[m] = false;
        if (valid && y[m] >= 256) {
          const uint32_t z = y[m] - 256;
          const uint64_t wd = rk[z >> 4];
          const uint32_t rb = rm_bits((uint32_t)wd);
          rem[m] = (rb >> (2 * (z & 15))) & 1;
          id[m] = 256 + z - ((uint32_t)(wd >> 32) +
                             (uint32_t)__builtin_popcount(rb & ((1u << (2 * (z & 15))) - 1)));
        }
        w[m] = rem[m] ? W[y[m] - 256] : (valid ? 1 : 0);
      }
      uint64_t ex[kPer], tot;
      uint32_t jj[kPer];
      tile_prefix(s_off, n, t0, b, w, carry, s_rs, s_w, ex, jj, &tot);
      __syncthreads();  // s_rs of the rules starting in this tile
#pragma unroll
      for (int m = 0; m < kPer; ++m) {
        if (t0 + m >= b || rem[m]) continue;
        rhs2[s_dest[jj[m]] + ex[m] - s_rs[jj[m]]] = id[m];
      }
      carry += tot;
    }
    __syncthreads();
  }
}

__global__ void k_pp_c_out(const uint32_t* __restrict__ c1, uint32_t k,
                           const uint64_t* __restrict__ rk, uint32_t* __restrict__ c2) {
  PP_LOOP(j, k) c2[j] = c1[j] < 256 ? c1[j] : pp_newid(rk, c1[j] - 256);
}

// new ids of the block bounds (ids 256 .. 256 + g1 of the RL grammar)
__global__ void k_pp_bounds(const uint64_t* __restrict__ rk, const uint32_t* __restrict__ ids,
                            uint32_t n, uint32_t* __restrict__ out) {
  PP_LOOP(i, n) out[i] = pp_newid(rk, ids[i] - 256);
}

// ---------------------------------------------------------------- expansion
// Expansion lengths stop at kLenLimit: a rule that reaches it (possible only
// in a decoded file) sets *err, and the grammar is refused.
constexpr uint64_t kLenLimit = 1ull << 61;

// Right-hand sides longer than kLongRule symbols (after Simp, each string's
// root rule holds ~10^5 of them) are not summed by one thread: their
// positions go in pieces of kPiece to whole blocks, and a thread per long
// rule adds up its pieces.
constexpr uint64_t kLongRule = 1024;
constexpr uint64_t kPiece = 4096;

// E and NT of the rules [r0, r1) whose right-hand sides are not long
// (earlier blocks done)
__global__ void k_slp_lens(const uint64_t* __restrict__ off, const uint32_t* __restrict__ rhs,
                           const uint32_t* __restrict__ mult, uint32_t r0, uint32_t r1,
                           uint64_t* E, uint32_t* nt, uint32_t* __restrict__ err) {
  PP_LOOP(i, r1 - r0) {
    const uint32_t r = r0 + (uint32_t)i;
    uint64_t e = 0;
    uint32_t c = 0;
    const uint64_t b = off[r + 1];
    if (b - off[r] > kLongRule) continue;
    for (uint64_t t = off[r]; t < b; ++t) {
      const uint32_t y = rhs[t];
      if (y < 256) {
        e += 1;
      } else {
        e = min(e + E[y - 256], kLenLimit);  // both terms are at most kLenLimit
        ++c;
      }
    }
    const uint64_t m = mult[r];
    const uint64_t tot = (e >= kLenLimit || e > (kLenLimit - 1) / m) ? kLenLimit : e * m;
    if (tot >= kLenLimit) atomicOr(err, 1u);
    E[r] = tot;
    nt[r] = c;
  }
}

// the long rules (any order)
__global__ void k_slp_longlist(const uint64_t* __restrict__ off, uint32_t g,
                               uint32_t* __restrict__ ids, unsigned long long* __restrict__ cnt) {
  PP_LOOP(r, g) {
    if (off[r + 1] - off[r] > kLongRule) ids[atomicAdd(cnt, 1ull)] = (uint32_t)r;
  }
}

__global__ void k_slp_strlen(const uint32_t* __restrict__ c, uint32_t ks,
                             const uint64_t* __restrict__ E, uint64_t* __restrict__ len) {
  PP_LOOP(j, ks) len[j] = c[j] < 256 ? 1 : E[c[j] - 256];
}

// strings whose C entry is a rule become items; a terminal is written at once
__global__ void k_slp_enter(const uint32_t* __restrict__ c, uint32_t ks,
                            const uint64_t* __restrict__ str_off, uint32_t* __restrict__ sym,
                            uint64_t* __restrict__ pos, unsigned long long* __restrict__ count,
                            uint8_t* __restrict__ out) {
  PP_LOOP(j, ks) {
    const uint32_t y = c[j];
    if (y < 256) {
      out[str_off[j]] = (uint8_t)y;
      continue;
    }
    const unsigned long long at = atomicAdd(count, 1ull);
    sym[at] = y;
    pos[at] = str_off[j];
  }
}

// A leaf is a rule whose right-hand side is all terminals and whose expansion
// is at most kLeaf bytes: its parent writes those bytes itself instead of
// making it an item of the next step.
constexpr uint64_t kLeaf = 64;

struct RuleMeta {
  uint64_t a;       // first right-hand-side position
  uint64_t period;  // E / mult
  uint64_t sa, na;  // S[a], N[a]
  uint32_t q, mult;
  uint32_t ntx;     // item children per repetition
  uint32_t leaf;
};

// per position: its expansion bytes and whether it is an item child
__global__ void k_slp_posw(const uint32_t* __restrict__ rhs, uint64_t q,
                           const uint64_t* __restrict__ E, const uint32_t* __restrict__ nt,
                           uint64_t* __restrict__ we, uint64_t* __restrict__ wn) {
  PP_LOOP(t, q) {
    const uint32_t y = rhs[t];
    if (y < 256) {
      we[t] = 1;
      wn[t] = 0;
    } else {
      const uint64_t e = E[y - 256];
      we[t] = e;
      wn[t] = (nt[y - 256] == 0 && e <= kLeaf) ? 0 : 1;
    }
  }
}

__global__ void k_slp_meta(const uint64_t* __restrict__ off, const uint32_t* __restrict__ mult,
                           const uint32_t* __restrict__ nt, const uint64_t* __restrict__ E,
                           const uint64_t* __restrict__ S, const uint64_t* __restrict__ N, uint32_t g,
                           RuleMeta* __restrict__ meta) {
  PP_LOOP(r, g) {
    RuleMeta mt;
    mt.a = off[r];
    const uint64_t b = off[r + 1];
    mt.q = (uint32_t)(b - mt.a);
    mt.mult = mult[r];
    mt.period = E[r] / mt.mult;
    mt.sa = S[mt.a];
    mt.na = N[mt.a];
    mt.ntx = (uint32_t)(N[b] - mt.na);
    mt.leaf = nt[r] == 0 && E[r] <= kLeaf;
    meta[r] = mt;
  }
}

// block-wide sums of a (saturating at kLenLimit) and c
__device__ __forceinline__ void block_sums(uint64_t& a, uint64_t& c, uint64_t* s_a, uint64_t* s_c) {
  for (int d = 32; d; d >>= 1) {
    a = min(a + (uint64_t)__shfl_down(a, d), kLenLimit);
    c += (uint64_t)__shfl_down(c, d);
  }
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    s_a[wv] = a;
    s_c[wv] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (uint32_t w = 1; w < kPB / 64; ++w) {
      a = min(a + s_a[w], kLenLimit);
      c += s_c[w];
    }
  }
  __syncthreads();
}

// Per piece [pa, pb) of a long rule: mode 0, the expansion bytes (saturating)
// and the nonterminals of its positions; mode 1, the item children of its item
// children (the grandchild count).  Four positions per thread and step, their
// loads issued together.
template <int MODE>
__global__ __launch_bounds__(kPB) void k_slp_pieces_sum(const uint64_t* __restrict__ pa,
                                                        const uint64_t* __restrict__ pb,
                                                        uint64_t p0, uint64_t p1,
                                                        const uint32_t* __restrict__ rhs,
                                                        const uint64_t* __restrict__ E,
                                                        const uint64_t* __restrict__ N,
                                                        const RuleMeta* __restrict__ meta,
                                                        uint64_t* __restrict__ part_a,
                                                        uint64_t* __restrict__ part_c) {
  __shared__ uint64_t s_a[kPB / 64], s_c[kPB / 64];
  for (uint64_t pc = p0 + blockIdx.x; pc < p1; pc += gridDim.x) {
    const uint64_t a = pa[pc], b = pb[pc];
    uint64_t sa = 0, sc = 0;
    for (uint64_t t0 = a + threadIdx.x; t0 < b; t0 += 4 * kPB) {
      uint32_t y[4];
      bool in[4], child[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint64_t t = t0 + (uint64_t)k * kPB;
        in[k] = t < b;
        y[k] = in[k] ? rhs[t] : 0;
        if constexpr (MODE == 1) child[k] = in[k] && N[t + 1] != N[t];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if constexpr (MODE == 0) {
          if (!in[k]) continue;
          if (y[k] < 256) {
            sa = min(sa + 1, kLenLimit);
          } else {
            sa = min(sa + E[y[k] - 256], kLenLimit);
            ++sc;
          }
        } else {
          if (!child[k]) continue;
          const RuleMeta c = meta[y[k] - 256];
          sa += (uint64_t)c.mult * c.ntx;
        }
      }
    }
    block_sums(sa, sc, s_a, s_c);
    if (threadIdx.x == 0) {
      part_a[pc] = sa;
      part_c[pc] = sc;
    }
  }
}

// per long rule i of [i0, i1) (pieces lp0[i] .. lp0[i+1]): E and NT from
// its pieces' sums
__global__ void k_slp_long_lens(const uint32_t* __restrict__ ids, const uint64_t* __restrict__ lp0,
                                uint32_t i0, uint32_t i1, const uint64_t* __restrict__ part_a,
                                const uint64_t* __restrict__ part_c,
                                const uint32_t* __restrict__ mult, uint64_t* __restrict__ E,
                                uint32_t* __restrict__ nt, uint32_t* __restrict__ err) {
  PP_LOOP(j, i1 - i0) {
    const uint32_t i = i0 + (uint32_t)j, r = ids[i];
    uint64_t e = 0, c = 0;
    for (uint64_t pc = lp0[i]; pc < lp0[i + 1]; ++pc) {
      e = min(e + part_a[pc], kLenLimit);
      c += part_c[pc];
    }
    const uint64_t m = mult[r];
    const uint64_t tot = (e >= kLenLimit || e > (kLenLimit - 1) / m) ? kLenLimit : e * m;
    if (tot >= kLenLimit) atomicOr(err, 1u);
    E[r] = tot;
    nt[r] = (uint32_t)c;
  }
}

// per long rule: its grandchild count from its pieces' sums
__global__ void k_slp_long_gnt(const uint32_t* __restrict__ ids, const uint64_t* __restrict__ lp0,
                               uint32_t n, const uint64_t* __restrict__ part_a,
                               const RuleMeta* __restrict__ meta, uint64_t* __restrict__ gnt) {
  PP_LOOP(i, n) {
    const uint32_t r = ids[i];
    uint64_t sum = 0;
    for (uint64_t pc = lp0[i]; pc < lp0[i + 1]; ++pc) sum += part_a[pc];
    gnt[r] = sum * meta[r].mult;
  }
}

// first and end position of each listed rule
__global__ void k_slp_longoff(const uint32_t* __restrict__ ids, uint32_t n,
                              const uint64_t* __restrict__ off, uint64_t* __restrict__ a,
                              uint64_t* __restrict__ b) {
  PP_LOOP(i, n) {
    a[i] = off[ids[i]];
    b[i] = off[ids[i] + 1];
  }
}

// per rule whose right-hand side is not long: the item children of its item
// children, over all repetitions (sizes the step after next)
__global__ void k_slp_gnt(const uint64_t* __restrict__ off, const uint32_t* __restrict__ rhs,
                          const uint64_t* __restrict__ N, const RuleMeta* __restrict__ meta,
                          uint32_t g, uint64_t* __restrict__ gnt) {
  PP_LOOP(r, g) {
    const uint64_t a = off[r], b = off[r + 1];
    if (b - a > kLongRule) continue;
    uint64_t sum = 0;
    for (uint64_t t = a; t < b; ++t) {
      if (N[t + 1] == N[t]) continue;  // a terminal or a leaf
      const RuleMeta c = meta[rhs[t] - 256];
      sum += (uint64_t)c.mult * c.ntx;
    }
    gnt[r] = sum * meta[r].mult;
  }
}

// el[r]: a rule's expansion length E; for a leaf, the leaf bit, E (at most
// kLeaf, the low 7 bits) and the offset of its bytes in lbytes (bits 7..62).
constexpr uint64_t kLeafBit = 1ull << 63;
constexpr uint64_t kLeafLenMask = 127;

// An item's children [v0, v1) (v = rep * q + k): terminals and leaves are
// written to out, item children go to slots o, o+1, ... of the next step.
// The first child's position comes from S; the others follow by adding the
// children's expansion lengths.
__device__ __forceinline__ void slp_item_children(const RuleMeta& mt, uint64_t pos, uint64_t v0,
                                                  uint64_t v1, uint64_t o,
                                                  const uint32_t* __restrict__ rhs,
                                                  const uint64_t* __restrict__ S,
                                                  const uint64_t* __restrict__ el,
                                                  const uint8_t* __restrict__ lbytes,
                                                  uint32_t* __restrict__ nsym,
                                                  uint64_t* __restrict__ npos,
                                                  uint8_t* __restrict__ out) {
  uint64_t rep = v0 / mt.q, k = v0 - rep * mt.q;
  uint64_t p = pos + rep * mt.period + (k ? S[mt.a + k] - mt.sa : 0);
  for (uint64_t v = v0; v < v1; ++v) {
    const uint32_t y = rhs[mt.a + k];
    if (y < 256) {
      out[p] = (uint8_t)y;
      p += 1;
    } else {
      const uint64_t e = el[y - 256];
      if (e & kLeafBit) {  // a leaf: its stored bytes
        const uint64_t len = e & kLeafLenMask;
        const uint8_t* src = lbytes + ((e & ~kLeafBit) >> 7);
        for (uint64_t x = 0; x < len; ++x) out[p + x] = src[x];
        p += len;
      } else {
        nsym[o] = y;
        npos[o] = p;
        ++o;
        p += e;
      }
    }
    if (++k == mt.q) k = 0, ++rep;
  }
}

// per rule: its bytes if it is a leaf, else 0
__global__ void k_slp_leaflen(const uint64_t* __restrict__ E, const uint32_t* __restrict__ nt,
                              uint32_t g, uint64_t* __restrict__ w) {
  PP_LOOP(r, g) w[r] = (nt[r] == 0 && E[r] <= kLeaf) ? E[r] : 0;
}

// the leaves' expansions into lbytes at their offsets
__global__ void k_slp_leafbytes(const uint64_t* __restrict__ off, const uint32_t* __restrict__ rhs,
                                const uint32_t* __restrict__ mult, const uint64_t* __restrict__ w,
                                const uint64_t* __restrict__ lboff, uint32_t g,
                                uint8_t* __restrict__ lbytes) {
  PP_LOOP(r, g) {
    if (!w[r]) continue;
    const uint64_t a = off[r], q = off[r + 1] - a;
    uint8_t* dst = lbytes + lboff[r];
    for (uint32_t rr = 0; rr < mult[r]; ++rr)
      for (uint64_t kk = 0; kk < q; ++kk) *dst++ = (uint8_t)rhs[a + kk];
  }
}

__global__ void k_slp_el(const uint64_t* __restrict__ E, const uint32_t* __restrict__ nt,
                         const uint64_t* __restrict__ lboff, uint32_t g,
                         uint64_t* __restrict__ el) {
  PP_LOOP(r, g) {
    const bool leaf = nt[r] == 0 && E[r] <= kLeaf;
    el[r] = leaf ? kLeafBit | (lboff[r] << 7) | E[r] : E[r];
  }
}

// block-wide exclusive scan of v (s_w: kPB / 64 words); *tot gets the sum
__device__ __forceinline__ unsigned long long block_scan_u64(unsigned long long v,
                                                             unsigned long long* s_w,
                                                             unsigned long long* tot) {
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  unsigned long long incl = v;
  for (int d = 1; d < 64; d <<= 1) {
    const unsigned long long o = __shfl_up(incl, d);
    if ((int)lane >= d) incl += o;
  }
  if (lane == 63) s_w[wv] = incl;
  __syncthreads();
  unsigned long long before = 0, t = 0;
  for (uint32_t w = 0; w < kPB / 64; ++w) {
    before += w < wv ? s_w[w] : 0;
    t += s_w[w];
  }
  __syncthreads();
  *tot = t;
  return before + incl - v;
}

// One step over items (sym, pos) or over pieces of big items (vi: item
// index, v0: first child; NULL for whole items).  An item with at most kSmall
// children is handled whole by one thread; a bigger one is listed in big[]
// (whole-item pass only) and handled later in pieces of kSmall children.  Item
// children are reserved per block (scan + one atomicAdd); the step after
// next is sized on the way from GNT.
constexpr uint64_t kSmall = 64;
__global__ __launch_bounds__(kPB) void k_slp_step(
    const uint32_t* __restrict__ sym, const uint64_t* __restrict__ pos, uint64_t m,
    const uint32_t* __restrict__ vi, const uint64_t* __restrict__ v0s,
    const RuleMeta* __restrict__ meta, const uint64_t* __restrict__ gnt,
    const uint32_t* __restrict__ rhs, const uint64_t* __restrict__ S, const uint64_t* __restrict__ N,
    const uint64_t* __restrict__ el, const uint8_t* __restrict__ lbytes,
    uint32_t* __restrict__ nsym, uint64_t* __restrict__ npos, unsigned long long* ncount,
    unsigned long long* gcount, uint32_t* __restrict__ big, unsigned long long* nbig,
    uint8_t* __restrict__ out) {
  __shared__ unsigned long long s_w[kPB / 64];
  __shared__ unsigned long long s_base;
  unsigned long long gsum = 0;
  for (uint64_t b0 = blockIdx.x * (uint64_t)kPB; b0 < m; b0 += (uint64_t)gridDim.x * kPB) {
    const uint64_t j = b0 + threadIdx.x;
    RuleMeta mt{};
    uint64_t p = 0, v0 = 0, v1 = 0;
    unsigned long long ntc = 0;
    if (j < m) {
      const uint64_t i = vi ? vi[j] : j;
      mt = meta[sym[i] - 256];
      p = pos[i];
      const uint64_t cnt = (uint64_t)mt.mult * mt.q;
      if (vi) {  // a piece of a big item
        v0 = v0s[j];
        v1 = min(cnt, v0 + kSmall);
      } else if (cnt <= kSmall) {
        v1 = cnt;
        gsum += gnt[sym[i] - 256];
      } else {  // big: listed for the pieces pass
        big[atomicAdd(nbig, 1ull)] = (uint32_t)i;
      }
      // item children among [v0, v1): whole repetitions plus the partial ones
      if (v1 > v0) {
        const uint64_t q = mt.q, ntx = mt.ntx;
        const uint64_t r0 = v0 / q, r1 = v1 / q, k0 = v0 - r0 * q, k1 = v1 - r1 * q;
        // N prefixes inside the rule: items before position k
        const uint64_t n0 = N[mt.a + k0] - mt.na, n1 = N[mt.a + k1] - mt.na;
        ntc = (r1 - r0) * ntx + n1 - n0;
      }
    }
    unsigned long long tot;
    const unsigned long long excl = block_scan_u64(ntc, s_w, &tot);
    if (threadIdx.x == 0) s_base = tot ? atomicAdd(ncount, tot) : 0;
    __syncthreads();
    if (v1 > v0)
      slp_item_children(mt, p, v0, v1, s_base + excl, rhs, S, el, lbytes, nsym, npos, out);
    __syncthreads();  // s_base is rewritten by the next iteration
  }
  for (int d = 32; d; d >>= 1) gsum += __shfl_xor(gsum, d);
  if ((threadIdx.x & 63) == 0 && gsum) atomicAdd(gcount, gsum);
}

// the pieces of the big items: (item, first child) for every kSmall children;
// their GNT joins the step after next
__global__ void k_slp_pieces(const uint32_t* __restrict__ big, uint64_t nb,
                             const uint32_t* __restrict__ sym, const RuleMeta* __restrict__ meta,
                             const uint64_t* __restrict__ gnt, uint32_t* __restrict__ vi,
                             uint64_t* __restrict__ v0s, unsigned long long* npieces,
                             unsigned long long* gcount) {
  PP_LOOP(j, nb) {
    const uint32_t i = big[j];
    const uint32_t r = sym[i] - 256;
    const RuleMeta mt = meta[r];
    const uint64_t cnt = (uint64_t)mt.mult * mt.q;
    const uint64_t np = (cnt + kSmall - 1) / kSmall;
    const unsigned long long at = atomicAdd(npieces, (unsigned long long)np);
    for (uint64_t x = 0; x < np; ++x) {
      vi[at + x] = i;
      v0s[at + x] = x * kSmall;
    }
    atomicAdd(gcount, (unsigned long long)gnt[r]);
  }
}

// item children of the first step's items (*m_dev of them)
__global__ void k_slp_first(const uint64_t* __restrict__ m_dev, const uint32_t* __restrict__ sym,
                            const RuleMeta* __restrict__ meta, unsigned long long* total) {
  PP_LOOP(i, *m_dev) {
    const RuleMeta mt = meta[sym[i] - 256];
    atomicAdd(total, (unsigned long long)mt.mult * mt.ntx);
  }
}

// pieces of the big items of a step (at most this many per step)
__global__ void k_slp_npieces(const uint32_t* __restrict__ big, uint64_t nb,
                              const uint32_t* __restrict__ sym, const RuleMeta* __restrict__ meta,
                              unsigned long long* npieces) {
  PP_LOOP(j, nb) {
    const RuleMeta mt = meta[sym[big[j]] - 256];
    atomicAdd(npieces, ((uint64_t)mt.mult * mt.q + kSmall - 1) / kSmall);
  }
}

// ---------------------------------------------------------------- host
struct Scan {
  DBuf<uint64_t> tmp;
  // out[0..n] = exclusive prefix sums of in[0..n) (out[n]: the total)
  void run(const uint64_t* in, uint64_t* out, uint64_t n, hipStream_t s) {
    if (n == 0) {
      k_pp_set<<<1, 1, 0, s>>>(out, 0);
      PP_CHECK("pp_set");
      return;
    }
    tmp.need(scan_tmp_words(n), s);
    scan_exclusive(in, out, n, tmp.p, s);
  }
};

void zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes) launch_zero(p, (bytes + 3) & ~size_t(3), s);
}

template <typename T>
void read_many(std::initializer_list<std::pair<const T*, T*>> items, hipStream_t s) {
  for (auto& it : items)
    HIP_CHECK(hipMemcpyAsync(it.second, it.first, sizeof(T), hipMemcpyDeviceToHost, s));
  sync(s);
}

unsigned groups_grid(uint64_t ngroups) {
  return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(ngroups, 8192));
}

}  // namespace

static lcg_slp* postprocess_core(lcg_grammar* g, uint32_t flags, hipStream_t s) {
  const bool rl = flags & LCG_PP_RL;
  const bool simp = flags & LCG_PP_SIMP;
  const uint32_t h = (uint32_t)g->levels.size();
  if (h > 63) throw LcgError{LCG_EOVERFLOW, "more than 63 levels"};
  uint64_t g0 = 0, q0 = 0, ngroups = 0;
  std::vector<PLevel> tab(std::max<uint32_t>(h, 1));
  for (uint32_t i = 0; i < h; ++i) {
    const Level& L = g->levels[i];
    PLevel& P = tab[i];
    std::memset(&P, 0, sizeof(P));
    P.rhs = i == 0 ? (const void*)L.rhs8.p : (const void*)L.rhs32.p;
    P.off = L.off.p;
    P.p0 = q0;
    P.q = L.q;
    P.u = L.u;
    P.gpre = (uint32_t)ngroups;
    P.bytes = i == 0;
    ngroups += (L.u + kGrp - 1) / kGrp;
    g0 += L.u;
    q0 += L.q;
  }
  // capacities: RL never adds positions (runs + run rules <= q per level) and
  // makes at most q/2 run rules per level
  const uint64_t gcap = g0 + (rl ? q0 / 2 : 0);
  if (256 + gcap >= (1ull << 32)) throw LcgError{LCG_EOVERFLOW, "more than 2^32 - 256 rules"};
  DBuf<PLevel> tab_d;
  tab_d.need(tab.size(), s);
  HIP_CHECK(hipMemcpyAsync(tab_d.p, tab.data(), tab.size() * sizeof(PLevel), hipMemcpyHostToDevice, s));
  // repeated positions: per rule group, scanned, then written in order (P)
  DBuf<uint64_t> gpos, P, ukey;
  DBuf<uint32_t> rlen, ulvl;
  gpos.need(ngroups + 1, s);
  std::vector<uint64_t> hreps(h + 1, 0), hv(64, 0);
  uint64_t c = 0, vt = 0;
  if (rl && h) {
    DBuf<uint64_t> gcnt, lvreps;
    gcnt.need(std::max<uint64_t>(ngroups, 1), s);
    k_pp_repcount<<<groups_grid(ngroups), kGrp, 0, s>>>(tab_d.p, h, ngroups, gcnt.p);
    PP_CHECK("pp_repcount");
    Scan sc;
    sc.run(gcnt.p, gpos.p, ngroups, s);
    lvreps.need(h + 1, s);
    k_pp_level_reps<<<pgrid(h + 1), kPB, 0, s>>>(tab_d.p, h, ngroups, gpos.p, lvreps.p);
    PP_CHECK("pp_level_reps");
    HIP_CHECK(hipMemcpyAsync(hreps.data(), lvreps.p, (h + 1) * 8, hipMemcpyDeviceToHost, s));
    sync(s);
    c = hreps[h];
    if (c) {
      P.need(c, s);
      k_pp_repwrite<<<groups_grid(ngroups), kGrp, 0, s>>>(tab_d.p, h, ngroups, gpos.p, P.p);
      PP_CHECK("pp_repwrite");
      // cnt: [0] runs of length >= 2, [1 + i] distinct ones of level i
      DBuf<unsigned long long> cnt;
      cnt.need(65, s);
      zero(cnt.p, 65 * 8, s);
      rlen.need(c, s);
      DBuf<uint64_t> rkey, k1, k2, uflag, upos;
      DBuf<uint32_t> rlvl, l1, l2;
      rkey.need(c, s);
      rlvl.need(c, s);
      k_pp_runs<<<pgrid(c), kPB, 0, s>>>(tab_d.p, h, P.p, c, rlen.p, rkey.p, rlvl.p, cnt.p);
      PP_CHECK("pp_runs");
      const uint64_t R = read_dev(cnt.p, s);
      if (R > 0x7fffffffull) throw LcgError{LCG_EOVERFLOW, "more than 2^31 runs"};
      // sort the runs by (level, key): by key, then stably by level
      k1.need(R, s);
      l1.need(R, s);
      k2.need(R, s);
      l2.need(R, s);
      size_t tb = 0, tb2 = 0;
      HIP_CHECK(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, rkey.p, k1.p, rlvl.p, l1.p, (int)R,
                                                   0, 64, s));
      HIP_CHECK(hipcub::DeviceRadixSort::SortPairs(nullptr, tb2, l1.p, l2.p, k1.p, k2.p, (int)R, 0,
                                                   8, s));
      tb = std::max(tb, tb2);
      DBuf<uint8_t> tmp;
      tmp.need(std::max<size_t>(tb, 4), s);
      HIP_CHECK(hipcub::DeviceRadixSort::SortPairs(tmp.p, tb, rkey.p, k1.p, rlvl.p, l1.p, (int)R, 0,
                                                   64, s));
      HIP_CHECK(hipcub::DeviceRadixSort::SortPairs(tmp.p, tb, l1.p, l2.p, k1.p, k2.p, (int)R, 0, 8,
                                                   s));
      uflag.need(R, s);
      upos.need(R + 1, s);
      k_pp_uniqflag<<<pgrid(R), kPB, 0, s>>>(l2.p, k2.p, R, uflag.p);
      PP_CHECK("pp_uniqflag");
      sc.run(uflag.p, upos.p, R, s);
      vt = read_dev(upos.p + R, s);
      ukey.need(vt, s);
      ulvl.need(vt, s);
      k_pp_uniqlist<<<pgrid(R), kPB, 0, s>>>(l2.p, k2.p, uflag.p, upos.p, R, ulvl.p, ukey.p,
                                             cnt.p + 1);
      PP_CHECK("pp_uniqlist");
      HIP_CHECK(hipMemcpyAsync(hv.data(), cnt.p + 1, 64 * 8, hipMemcpyDeviceToHost, s));
      sync(s);
    }
  } else {
    zero(gpos.p, (ngroups + 1) * 8, s);
  }
  // id and position bases of every level
  std::vector<uint32_t> obase(h + 1, 0);
  uint32_t next = 256;
  uint64_t pos = 0, cpre = 0, upre = 0, runs = 0;
  for (uint32_t i = 0; i < h; ++i) {
    PLevel& L = tab[i];
    const uint64_t reps = hreps[i + 1] - hreps[i], v = hv[i];
    L.symbase = i == 0 ? 0 : obase[i];
    L.cpre = cpre;
    L.upre = (uint32_t)upre;
    L.v = (uint32_t)v;
    L.rlbase = next;
    L.obase = next + (uint32_t)v;
    L.out0 = pos + v;
    obase[i + 1] = L.obase;
    next = L.obase + L.u;
    pos += v + (L.q - reps);
    cpre += reps;
    upre += v;
    runs += v;
  }
  const uint32_t g1 = next - 256;
  const uint64_t q1 = pos;
  DBuf<uint32_t> rhs1, mult1, c1;
  DBuf<uint64_t> off1;
  rhs1.need(std::max<uint64_t>(q1, 1), s);
  off1.need(g1 + 1, s);
  mult1.need(std::max<uint32_t>(g1, 1), s);
  HIP_CHECK(hipMemcpyAsync(tab_d.p, tab.data(), tab.size() * sizeof(PLevel), hipMemcpyHostToDevice, s));
  if (h) {
    k_pp_rl_write<<<groups_grid(ngroups), kGrp, 0, s>>>(tab_d.p, h, ngroups, gpos.p, P.p, c,
                                                        rlen.p, ukey.p, rhs1.p, off1.p, mult1.p);
    PP_CHECK("pp_rl_write");
  }
  if (vt) {
    k_pp_rl_rules<<<pgrid(vt), kPB, 0, s>>>(tab_d.p, ulvl.p, ukey.p, vt, rhs1.p, off1.p, mult1.p);
    PP_CHECK("pp_rl_rules");
  }
  k_pp_set<<<1, 1, 0, s>>>(off1.p + g1, q1);
  PP_CHECK("pp_set");
  DBuf<uint32_t> obase_d;
  obase_d.need(h + 1, s);
  HIP_CHECK(hipMemcpyAsync(obase_d.p, obase.data(), (h + 1) * sizeof(uint32_t),
                           hipMemcpyHostToDevice, s));
  c1.need(std::max<uint32_t>(g->k, 1), s);
  k_pp_c_global<<<pgrid(g->k), kPB, 0, s>>>(g->c_level.p, g->c_sym.p, g->k, obase_d.p, c1.p);
  PP_CHECK("pp_c_global");

  std::unique_ptr<lcg_slp> out(new lcg_slp());
  out->seed = g->seed;
  out->k = g->k;
  uint64_t* st = out->stats;
  st[0] = g0;
  st[1] = q0;
  st[2] = runs;
  st[3] = g1;
  st[4] = q1 + runs;
  std::vector<uint32_t> bounds1;  // block bounds in the ids after RL
  bounds1.push_back(256);
  for (uint32_t i = 0; i < h; ++i) {
    bounds1.push_back(tab[i].obase);
    bounds1.push_back(tab[i].obase + tab[i].u);
  }
  if (!simp) {
    out->bounds = bounds1;
    out->g = g1;
    out->q = q1;
    out->off = std::move(off1);
    out->rhs = std::move(rhs1);
    out->mult = std::move(mult1);
    out->c = std::move(c1);
    st[5] = 0;
    st[6] = g1;
    st[7] = q1 + runs;
    sync(s);
    return out.release();
  }

  // ---- Simp
  DBuf<uint32_t> occ, oc2, par;
  DBuf<uint64_t> rk, cnt, pre, W, inoff, len, so, base;
  const uint32_t g1c = std::max<uint32_t>(g1, 1);
  const uint64_t nwords = ((uint64_t)g1 + 15) / 16;
  occ.need(g1c, s);
  zero(occ.p, (size_t)g1 * 4, s);
  par.need(g1c, s);
  const uint64_t ng1 = (g1 + kGrp - 1) / kGrp;
  if (g1) {
    k_pp_occ<<<groups_grid(ng1), kGrp, 0, s>>>(off1.p, rhs1.p, mult1.p, g1, occ.p, par.p);
    PP_CHECK("pp_occ");
  }
  k_pp_occ_c<<<pgrid(g->k), kPB, 0, s>>>(c1.p, g->k, occ.p);
  PP_CHECK("pp_occ_c");
  Scan sc;
  oc2.need(std::max<uint64_t>(nwords, 1), s);
  cnt.need(std::max<uint64_t>(nwords, 1), s);
  pre.need(nwords + 1, s);
  k_pp_fields<<<pgrid(nwords), kPB, 0, s>>>(occ.p, mult1.p, g1, nwords, oc2.p, cnt.p);
  PP_CHECK("pp_fields");
  sc.run(cnt.p, pre.p, nwords, s);
  rk.need(nwords + 1, s);
  k_pp_pack<<<pgrid(nwords + 1), kPB, 0, s>>>(oc2.p, pre.p, nwords, rk.p);
  PP_CHECK("pp_pack");
  W.need(g1c, s);
  inoff.need(g1c, s);
  for (uint32_t i = 0; i < h; ++i) {
    const uint32_t u = tab[i].u;
    if (!u) continue;
    const uint32_t rb = tab[i].obase - 256;
    k_pp_flat<<<groups_grid((u + kGrp - 1) / kGrp), kGrp, 0, s>>>(off1.p, rhs1.p, rk.p, rb, rb + u,
                                                                    W.p, inoff.p);
    PP_CHECK("pp_flat");
  }
  len.need(g1c, s);
  so.need(g1 + 1, s);
  k_pp_len<<<pgrid(g1), kPB, 0, s>>>(rk.p, mult1.p, W.p, g1, len.p);
  PP_CHECK("pp_len");
  sc.run(len.p, so.p, g1, s);
  base.need(g1c, s);
  for (uint32_t i = h; i-- > 0;) {
    const uint32_t u = tab[i].u;
    if (!u) continue;
    const uint32_t rb = tab[i].obase - 256;
    k_pp_base<<<pgrid(u), kPB, 0, s>>>(rk.p, par.p, inoff.p, so.p, rb, rb + u, base.p);
    PP_CHECK("pp_base");
  }
  uint64_t removed = 0, q2 = 0;
  read_many<uint64_t>({{pre.p + nwords, &removed}, {so.p + g1, &q2}}, s);
  const uint64_t g2 = g1 - removed;
  {  // block bounds after renumbering: the kept rules before each bound
    DBuf<uint32_t> bq, bv;
    bq.need(bounds1.size(), s);
    bv.need(bounds1.size(), s);
    HIP_CHECK(hipMemcpyAsync(bq.p, bounds1.data(), bounds1.size() * 4, hipMemcpyHostToDevice, s));
    k_pp_bounds<<<pgrid(bounds1.size()), kPB, 0, s>>>(rk.p, bq.p, (uint32_t)bounds1.size(), bv.p);
    PP_CHECK("pp_bounds");
    std::vector<uint32_t> hb(bounds1.size());
    HIP_CHECK(hipMemcpyAsync(hb.data(), bv.p, hb.size() * 4, hipMemcpyDeviceToHost, s));
    sync(s);
    for (uint32_t v : hb) out->bounds.push_back(v);
  }
  out->g = (uint32_t)g2;
  out->q = q2;
  out->off.need(g2 + 1, s);
  out->rhs.need(std::max<uint64_t>(q2, 1), s);
  out->mult.need(std::max<uint64_t>(g2, 1), s);
  out->c.need(std::max<uint32_t>(g->k, 1), s);
  if (g1) {
    k_pp_write<<<groups_grid(ng1), kGrp, 0, s>>>(off1.p, rhs1.p, mult1.p, rk.p, W.p, so.p, base.p,
                                                 g1, out->rhs.p, out->off.p, out->mult.p);
    PP_CHECK("pp_write");
  }
  k_pp_set<<<1, 1, 0, s>>>(out->off.p + g2, q2);
  PP_CHECK("pp_set");
  k_pp_c_out<<<pgrid(g->k), kPB, 0, s>>>(c1.p, g->k, rk.p, out->c.p);
  PP_CHECK("pp_c_out");
  st[5] = g1 - g2;
  st[6] = g2;
  st[7] = q2 + runs;
  sync(s);
  return out.release();
}

// The long rules of p in id order and their pieces of kPiece positions: rule
// ids[i] owns the pieces lp0[i] .. lp0[i+1] (host copy in h_ids / h_lp0).
struct LongPieces {
  std::vector<uint32_t> h_ids;
  std::vector<uint64_t> h_lp0;
  DBuf<uint32_t> ids;
  DBuf<uint64_t> lp0, pa, pb, part_a, part_c;
  uint64_t pieces = 0;
};

static void long_pieces(lcg_slp* p, LongPieces& L, hipStream_t s) {
  const uint64_t cap = p->q / (kLongRule + 1) + 1;
  DBuf<unsigned long long> cnt;
  cnt.need(1, s);
  zero(cnt.p, 8, s);
  L.ids.need(cap, s);
  if (p->g) {
    k_slp_longlist<<<pgrid(p->g), kPB, 0, s>>>(p->off.p, p->g, L.ids.p, cnt.p);
    PP_CHECK("slp_longlist");
  }
  const uint64_t n = read_dev(cnt.p, s);
  if (!n) return;
  L.h_ids.resize(n);
  HIP_CHECK(hipMemcpyAsync(L.h_ids.data(), L.ids.p, n * 4, hipMemcpyDeviceToHost, s));
  sync(s);
  std::sort(L.h_ids.begin(), L.h_ids.end());
  HIP_CHECK(hipMemcpyAsync(L.ids.p, L.h_ids.data(), n * 4, hipMemcpyHostToDevice, s));
  DBuf<uint64_t> a, b;
  a.need(n, s);
  b.need(n, s);
  k_slp_longoff<<<pgrid(n), kPB, 0, s>>>(L.ids.p, (uint32_t)n, p->off.p, a.p, b.p);
  PP_CHECK("slp_longoff");
  std::vector<uint64_t> ha(n), hb(n);
  HIP_CHECK(hipMemcpyAsync(ha.data(), a.p, n * 8, hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipMemcpyAsync(hb.data(), b.p, n * 8, hipMemcpyDeviceToHost, s));
  sync(s);
  std::vector<uint64_t> hpa, hpb;
  L.h_lp0.assign(1, 0);
  for (uint64_t i = 0; i < n; ++i) {
    for (uint64_t x = ha[i]; x < hb[i]; x += kPiece) {
      hpa.push_back(x);
      hpb.push_back(std::min(hb[i], x + kPiece));
    }
    L.h_lp0.push_back(hpa.size());
  }
  L.pieces = hpa.size();
  L.lp0.need(n + 1, s);
  L.pa.need(L.pieces, s);
  L.pb.need(L.pieces, s);
  L.part_a.need(L.pieces, s);
  L.part_c.need(L.pieces, s);
  HIP_CHECK(hipMemcpyAsync(L.lp0.p, L.h_lp0.data(), (n + 1) * 8, hipMemcpyHostToDevice, s));
  HIP_CHECK(hipMemcpyAsync(L.pa.p, hpa.data(), L.pieces * 8, hipMemcpyHostToDevice, s));
  HIP_CHECK(hipMemcpyAsync(L.pb.p, hpb.data(), L.pieces * 8, hipMemcpyHostToDevice, s));
  sync(s);  // the host vectors go out of scope
}

static void slp_lens(lcg_slp* p, hipStream_t s) {
  if (p->lens_ready) return;
  const uint32_t gc = std::max<uint32_t>(p->g, 1);
  p->E.need(gc, s);
  p->nt.need(gc, s);
  DBuf<uint32_t> err;
  err.need(1, s);
  zero(err.p, 4, s);
  LongPieces lp;
  long_pieces(p, lp, s);
  for (size_t b = 0; b + 1 < p->bounds.size(); ++b) {
    const uint32_t r0 = p->bounds[b] - 256, r1 = p->bounds[b + 1] - 256;
    if (r1 <= r0) continue;
    k_slp_lens<<<pgrid(r1 - r0), kPB, 0, s>>>(p->off.p, p->rhs.p, p->mult.p, r0, r1, p->E.p,
                                              p->nt.p, err.p);
    PP_CHECK("slp_lens");
    const uint32_t i0 = (uint32_t)(std::lower_bound(lp.h_ids.begin(), lp.h_ids.end(), r0) -
                                   lp.h_ids.begin());
    const uint32_t i1 = (uint32_t)(std::lower_bound(lp.h_ids.begin(), lp.h_ids.end(), r1) -
                                   lp.h_ids.begin());
    if (i1 > i0) {  // the block's long rules, after its short ones
      const uint64_t p0 = lp.h_lp0[i0], p1 = lp.h_lp0[i1];
      k_slp_pieces_sum<0><<<(unsigned)std::min<uint64_t>(p1 - p0, 16384), kPB, 0, s>>>(
          lp.pa.p, lp.pb.p, p0, p1, p->rhs.p, p->E.p, nullptr, nullptr, lp.part_a.p, lp.part_c.p);
      PP_CHECK("slp_pieces_sum");
      k_slp_long_lens<<<pgrid(i1 - i0), kPB, 0, s>>>(lp.ids.p, lp.lp0.p, i0, i1, lp.part_a.p,
                                                     lp.part_c.p, p->mult.p, p->E.p, p->nt.p,
                                                     err.p);
      PP_CHECK("slp_long_lens");
    }
  }
  if (read_dev(err.p, s)) throw LcgError{LCG_EINVAL, "an expansion reaches 2^61 bytes"};
  p->S.need(p->q + 1, s);
  p->N.need(p->q + 1, s);
  {
    DBuf<uint64_t> we, wn;
    we.need(std::max<uint64_t>(p->q, 1), s);
    wn.need(std::max<uint64_t>(p->q, 1), s);
    k_slp_posw<<<pgrid(p->q), kPB, 0, s>>>(p->rhs.p, p->q, p->E.p, p->nt.p, we.p, wn.p);
    PP_CHECK("slp_posw");
    Scan sc;
    sc.run(we.p, p->S.p, p->q, s);
    sc.run(wn.p, p->N.p, p->q, s);
    p->meta.need(std::max<uint64_t>(p->g, 1) * sizeof(RuleMeta), s);
    k_slp_meta<<<pgrid(p->g), kPB, 0, s>>>(p->off.p, p->mult.p, p->nt.p, p->E.p, p->S.p, p->N.p,
                                           p->g, reinterpret_cast<RuleMeta*>(p->meta.p));
    PP_CHECK("slp_meta");
    p->gnt.need(std::max<uint64_t>(p->g, 1), s);
    k_slp_gnt<<<pgrid(p->g), kPB, 0, s>>>(p->off.p, p->rhs.p, p->N.p,
                                          reinterpret_cast<const RuleMeta*>(p->meta.p), p->g,
                                          p->gnt.p);
    PP_CHECK("slp_gnt");
    if (lp.pieces) {
      k_slp_pieces_sum<1><<<(unsigned)std::min<uint64_t>(lp.pieces, 16384), kPB, 0, s>>>(
          lp.pa.p, lp.pb.p, 0, lp.pieces, p->rhs.p, nullptr, p->N.p,
          reinterpret_cast<const RuleMeta*>(p->meta.p), lp.part_a.p, lp.part_c.p);
      PP_CHECK("slp_pieces_sum");
      k_slp_long_gnt<<<pgrid(lp.h_ids.size()), kPB, 0, s>>>(
          lp.ids.p, lp.lp0.p, (uint32_t)lp.h_ids.size(), lp.part_a.p,
          reinterpret_cast<const RuleMeta*>(p->meta.p), p->gnt.p);
      PP_CHECK("slp_long_gnt");
    }
    {  // the leaves' bytes, stored once
      DBuf<uint64_t> wl, lboff;
      wl.need(std::max<uint64_t>(p->g, 1), s);
      lboff.need((uint64_t)p->g + 1, s);
      k_slp_leaflen<<<pgrid(p->g), kPB, 0, s>>>(p->E.p, p->nt.p, p->g, wl.p);
      PP_CHECK("slp_leaflen");
      sc.run(wl.p, lboff.p, p->g, s);
      const uint64_t nbytes = read_dev(lboff.p + p->g, s);
      p->lbytes.need(std::max<uint64_t>(nbytes, 1), s);
      k_slp_leafbytes<<<pgrid(p->g), kPB, 0, s>>>(p->off.p, p->rhs.p, p->mult.p, wl.p, lboff.p,
                                                  p->g, p->lbytes.p);
      PP_CHECK("slp_leafbytes");
      p->el.need(std::max<uint64_t>(p->g, 1), s);
      k_slp_el<<<pgrid(p->g), kPB, 0, s>>>(p->E.p, p->nt.p, lboff.p, p->g, p->el.p);
      PP_CHECK("slp_el");
      sync(s);  // wl and lboff are released below
    }
    sync(s);
  }
  p->lens_ready = true;
}

// exp(C[j]) for j0 <= j < j1, one after the other in d_out (see lcg.h)
static void slp_expand_core(lcg_slp* p, uint32_t j0, uint32_t j1, uint8_t* d_out, uint64_t cap,
                            uint64_t* d_offsets, uint64_t* total_out, hipStream_t s) {
  if (j0 > j1 || j1 > p->k) throw LcgError{LCG_EINVAL, "string range out of bounds"};
  const uint32_t ks = j1 - j0;
  slp_lens(p, s);
  DBuf<uint64_t> len, str_off, ctr;
  Scan sc;
  len.need(std::max<uint32_t>(ks, 1), s);
  str_off.need(ks + 1, s);
  k_slp_strlen<<<pgrid(ks), kPB, 0, s>>>(p->c.p + j0, ks, p->E.p, len.p);
  PP_CHECK("slp_strlen");
  sc.run(len.p, str_off.p, ks, s);
  const uint64_t total = read_dev(str_off.p + ks, s);
  if (total_out) *total_out = total;
  if (total > cap) throw LcgError{LCG_EINVAL, "output buffer too small"};
  if (d_offsets)
    HIP_CHECK(hipMemcpyAsync(d_offsets, str_off.p, (ks + 1) * sizeof(uint64_t),
                             hipMemcpyDeviceToDevice, s));
  // the strings whose C entry is a rule are the first step's items
  ctr.need(4, s);  // [0] items written, [1] items of the step after next, [2] big items, [3] pieces
  zero(ctr.p, 32, s);
  auto* uctr = reinterpret_cast<unsigned long long*>(ctr.p);
  const RuleMeta* meta = reinterpret_cast<const RuleMeta*>(p->meta.p);
  DBuf<uint32_t> sym[2], big, vi;
  DBuf<uint64_t> pos[2], v0s;
  int cur = 0;
  sym[0].need(std::max<uint32_t>(ks, 1), s);
  pos[0].need(std::max<uint32_t>(ks, 1), s);
  k_slp_enter<<<pgrid(ks), kPB, 0, s>>>(p->c.p + j0, ks, str_off.p, sym[0].p, pos[0].p, uctr,
                                        d_out);
  PP_CHECK("slp_enter");
  // the first step's items and, from their rules, the item children they make
  k_slp_first<<<pgrid(ks), kPB, 0, s>>>(ctr.p, sym[0].p, meta, uctr + 1);
  PP_CHECK("slp_first");
  uint64_t counts[2];
  read_many<uint64_t>({{ctr.p, &counts[0]}, {ctr.p + 1, &counts[1]}}, s);
  uint64_t m = counts[0], m_next = counts[1];
  while (m) {
    sym[cur ^ 1].need(std::max<uint64_t>(m_next, 1), s);
    pos[cur ^ 1].need(std::max<uint64_t>(m_next, 1), s);
    big.need(std::max<uint64_t>(m, 1), s);
    zero(ctr.p, 32, s);
    const unsigned grid = std::min(pgrid(m), 4096u);
    k_slp_step<<<grid, kPB, 0, s>>>(sym[cur].p, pos[cur].p, m, nullptr, nullptr, meta, p->gnt.p,
                                    p->rhs.p, p->S.p, p->N.p, p->el.p, p->lbytes.p, sym[cur ^ 1].p,
                                    pos[cur ^ 1].p, uctr, uctr + 1, big.p, uctr + 2, d_out);
    PP_CHECK("slp_step");
    const uint64_t nb = read_dev(ctr.p + 2, s);
    if (nb) {  // the big items, in pieces of kSmall children
      k_slp_npieces<<<pgrid(nb), kPB, 0, s>>>(big.p, nb, sym[cur].p, meta, uctr + 3);
      PP_CHECK("slp_npieces");
      const uint64_t np = read_dev(ctr.p + 3, s);
      vi.need(np, s);
      v0s.need(np, s);
      zero(ctr.p + 3, 8, s);
      k_slp_pieces<<<pgrid(nb), kPB, 0, s>>>(big.p, nb, sym[cur].p, meta, p->gnt.p, vi.p, v0s.p,
                                             uctr + 3, uctr + 1);
      PP_CHECK("slp_pieces");
      k_slp_step<<<std::min(pgrid(np), 4096u), kPB, 0, s>>>(
          sym[cur].p, pos[cur].p, np, vi.p, v0s.p, meta, p->gnt.p, p->rhs.p, p->S.p, p->N.p,
          p->el.p, p->lbytes.p, sym[cur ^ 1].p, pos[cur ^ 1].p, uctr, uctr + 1, big.p, uctr + 2,
          d_out);
      PP_CHECK("slp_step");
    }
    const uint64_t after = read_dev(ctr.p + 1, s);
    cur ^= 1;
    m = m_next;
    m_next = after;
  }
  sync(s);
}

// ---------------------------------------------------------------- random access
// Bytes [start, start + len) of string j of a post-processed grammar, one
// wave per query (one block for queries longer than 256 bytes).  The frontier holds (symbol, offset of its expansion
// relative to the query start); each step replaces every rule by its
// children that overlap [0, len): whole repetitions of a run rule are
// skipped arithmetically, and the first overlapping child of a right-hand
// side is found by binary search over the per-position prefix sums S (a
// Simp root rule has ~10^5 children).  Terminals are written as they
// appear.  The overlapping pieces are disjoint and non-empty, so a frontier
// never holds more than len entries.
namespace {

// The children of rule r (expansion starting at `base` relative to the query
// start) that overlap [0, len): terminals are written to dst, rules pushed.
template <typename Push>
__device__ __forceinline__ void slp_overlap_children(uint32_t r, int64_t base, uint64_t len,
                                                     const uint64_t* __restrict__ off,
                                                     const uint32_t* __restrict__ rhs,
                                                     const uint32_t* __restrict__ mult,
                                                     const uint64_t* __restrict__ E,
                                                     const uint64_t* __restrict__ S,
                                                     uint8_t* __restrict__ dst, Push push) {
  const uint64_t a = off[r], b = off[r + 1];
  const uint64_t m = mult[r];
  const int64_t period = (int64_t)(E[r] / m);
  const uint64_t sa = S[a];
  uint64_t rep = base < 0 ? (uint64_t)(-base) / (uint64_t)period : 0;
  for (; rep < m; ++rep) {
    const int64_t rb = base + (int64_t)rep * period;
    if (rb >= (int64_t)len) break;
    // the child holding offset -rb (or the first child)
    uint64_t t = a;
    if (rb < 0) {
      uint64_t lo = a, hi = b - 1;  // largest t with S[t] - S[a] <= -rb
      while (lo < hi) {
        const uint64_t mid = (lo + hi + 1) >> 1;
        if (S[mid] - sa <= (uint64_t)(-rb)) lo = mid; else hi = mid - 1;
      }
      t = lo;
    }
    for (; t < b; ++t) {
      const int64_t cb = rb + (int64_t)(S[t] - sa);
      if (cb >= (int64_t)len) break;
      const uint32_t ch = rhs[t];
      if (ch < 256) {
        if (cb >= 0) dst[cb] = (uint8_t)ch;
      } else if (cb + (int64_t)E[ch - 256] > 0) {
        push(ch, cb);
      }
    }
  }
}

// C[j]'s symbol if the query is valid, else -1
__device__ __forceinline__ int64_t slp_query_root(const uint32_t* __restrict__ c, uint32_t k,
                                                  const uint64_t* __restrict__ E, uint32_t j,
                                                  uint64_t start, uint64_t len) {
  if (j >= k || len < 1 || len > LCG_EXTRACT_MAX) return -1;
  const uint32_t y = c[j];
  const uint64_t e = y < 256 ? 1 : E[y - 256];
  return start <= e && len <= e - start ? (int64_t)y : -1;
}

// Queries of at most kSXWave bytes, one wave each (the block kernel below skips them).
constexpr uint32_t kSXWave = 256;
constexpr int kSXWaves = kPB / 64;

__device__ __forceinline__ void slp_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(kPB) void k_slp_extract_wave(
    const uint64_t* __restrict__ off, const uint32_t* __restrict__ rhs,
    const uint32_t* __restrict__ mult, const uint64_t* __restrict__ E,
    const uint64_t* __restrict__ S, const uint32_t* __restrict__ c, uint32_t k, uint32_t nq,
    const uint32_t* __restrict__ qj, const uint64_t* __restrict__ qstart,
    const uint32_t* __restrict__ qlen, const uint64_t* __restrict__ qout, uint8_t* __restrict__ out,
    unsigned int* __restrict__ bad) {
  __shared__ uint32_t s_sym[kSXWaves][2][kSXWave];
  __shared__ int64_t s_pos[kSXWaves][2][kSXWave];
  __shared__ uint32_t s_n[kSXWaves][2];
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t(*sym)[kSXWave] = s_sym[wv];
  int64_t(*pos)[kSXWave] = s_pos[wv];
  uint32_t* cnt = s_n[wv];
  for (uint32_t q = blockIdx.x * kSXWaves + wv; q < nq; q += gridDim.x * kSXWaves) {
    const uint64_t len = qlen[q];
    if (len < 1 || len > kSXWave) continue;  // the block kernel's
    const int64_t root = slp_query_root(c, k, E, qj[q], qstart[q], len);
    if (root < 0) {
      if (lane == 0) atomicAdd(bad, 1u);
      continue;
    }
    uint8_t* dst = out + qout[q];
    if (root < 256) {
      if (lane == 0) dst[0] = (uint8_t)root;
      continue;
    }
    if (lane == 0) {
      sym[0][0] = (uint32_t)root;
      pos[0][0] = -(int64_t)qstart[q];
      cnt[0] = 1;
    }
    slp_wave_sync();
    int cur = 0;
    while (cnt[cur]) {
      if (lane == 0) cnt[cur ^ 1] = 0;
      slp_wave_sync();
      const uint32_t n = cnt[cur];
      auto push = [&](uint32_t ch, int64_t cb) {
        const uint32_t slot = atomicAdd(&cnt[cur ^ 1], 1u);
        if (slot < kSXWave) {  // always: the overlapping pieces are at most len
          sym[cur ^ 1][slot] = ch;
          pos[cur ^ 1][slot] = cb;
        }
      };
      for (uint32_t i = lane; i < n; i += 64)
        slp_overlap_children(sym[cur][i] - 256, pos[cur][i], len, off, rhs, mult, E, S, dst, push);
      slp_wave_sync();
      cur ^= 1;
      if (lane == 0 && cnt[cur] > kSXWave) cnt[cur] = kSXWave;
      slp_wave_sync();
    }
    slp_wave_sync();  // the frontier is rewritten by the wave's next query
  }
}

__global__ __launch_bounds__(kPB) void k_slp_extract(
    const uint64_t* __restrict__ off, const uint32_t* __restrict__ rhs,
    const uint32_t* __restrict__ mult, const uint64_t* __restrict__ E,
    const uint64_t* __restrict__ S, const uint32_t* __restrict__ c, uint32_t k, uint32_t nq,
    const uint32_t* __restrict__ qj, const uint64_t* __restrict__ qstart,
    const uint32_t* __restrict__ qlen, const uint64_t* __restrict__ qout, uint8_t* __restrict__ out,
    unsigned int* __restrict__ bad) {
  __shared__ uint32_t s_sym[2][LCG_EXTRACT_MAX];
  __shared__ int64_t s_pos[2][LCG_EXTRACT_MAX];
  __shared__ uint32_t s_n[2];
  for (uint32_t q = blockIdx.x; q < nq; q += gridDim.x) {
    const uint64_t len = qlen[q];
    if (len >= 1 && len <= kSXWave) continue;  // answered by k_slp_extract_wave
    const int64_t root = slp_query_root(c, k, E, qj[q], qstart[q], len);
    if (root < 0) {  // uniform over the block
      if (threadIdx.x == 0) atomicAdd(bad, 1u);
      continue;
    }
    uint8_t* dst = out + qout[q];
    if (threadIdx.x == 0) {
      if (root < 256) dst[0] = (uint8_t)root;
      s_sym[0][0] = (uint32_t)root;
      s_pos[0][0] = -(int64_t)qstart[q];
      s_n[0] = root < 256 ? 0 : 1;
    }
    __syncthreads();
    int cur = 0;
    while (s_n[cur]) {
      if (threadIdx.x == 0) s_n[cur ^ 1] = 0;
      __syncthreads();
      const uint32_t n = s_n[cur];
      auto push = [&](uint32_t ch, int64_t cb) {
        const uint32_t slot = atomicAdd(&s_n[cur ^ 1], 1u);
        if (slot < LCG_EXTRACT_MAX) {  // always: the overlapping pieces are at most len
          s_sym[cur ^ 1][slot] = ch;
          s_pos[cur ^ 1][slot] = cb;
        }
      };
      for (uint32_t i = threadIdx.x; i < n; i += blockDim.x)
        slp_overlap_children(s_sym[cur][i] - 256, s_pos[cur][i], len, off, rhs, mult, E, S, dst,
                             push);
      __syncthreads();
      cur ^= 1;
      if (threadIdx.x == 0 && s_n[cur] > LCG_EXTRACT_MAX) s_n[cur] = LCG_EXTRACT_MAX;
      __syncthreads();
    }
    __syncthreads();  // the frontier is rewritten by the next query
  }
}

}  // namespace

static void slp_extract_core(lcg_slp* p, uint32_t nq, const uint32_t* d_j, const uint64_t* d_start,
                             const uint32_t* d_len, const uint64_t* d_out_off, uint8_t* d_out,
                             hipStream_t s) {
  slp_lens(p, s);
  DBuf<unsigned int> bad;
  bad.need(1, s);
  zero(bad.p, 4, s);
  k_slp_extract_wave<<<std::min<uint32_t>((nq + kSXWaves - 1) / kSXWaves, 8192u), kPB, 0, s>>>(
      p->off.p, p->rhs.p, p->mult.p, p->E.p, p->S.p, p->c.p, p->k, nq, d_j, d_start, d_len,
      d_out_off, d_out, bad.p);
  PP_CHECK("slp_extract_wave");
  k_slp_extract<<<std::min<uint32_t>(nq, 8192u), kPB, 0, s>>>(
      p->off.p, p->rhs.p, p->mult.p, p->E.p, p->S.p, p->c.p, p->k, nq, d_j, d_start, d_len,
      d_out_off, d_out, bad.p);
  PP_CHECK("slp_extract");
  const unsigned int nbad = read_dev(bad.p, s);
  if (nbad)
    throw LcgError{LCG_EINVAL, std::to_string(nbad) + " quer" + (nbad == 1 ? "y" : "ies") +
                                   " out of range (string index, or start + len beyond the "
                                   "string, or len not in 1.." +
                                   std::to_string(LCG_EXTRACT_MAX) + ")"};
}

// ---------------------------------------------------------------- stored file
// The file of a post-processed grammar, with the bit budget of App. A
// (storing the final grammar): right-hand-side cells of ceil(log g) bits,
// one pointer of ceil(log G) bits per rule, one cell per string for C, plus a
// run-rule bit per rule and the level block bounds.  Layout in include/lcg.h.
// Fixed-width cells make both directions data-parallel: a 64-bit word of a
// section holds known cells, so the encoder gives each output word a thread
// and the decoder each run of cells.
namespace {

constexpr uint64_t kStoreMagic = 0x3130504C5347434Cull;  // the bytes "LCGSLP01"
constexpr uint64_t kStoreMaxBounds = 1024;
constexpr uint32_t kCellsPerThread = 16;

uint32_t store_bits(uint64_t x) {  // binary digits of x, at least 1
  uint32_t b = 1;
  while (b < 64 && (x >> b)) ++b;
  return b;
}

uint64_t store_words(uint64_t cells, uint32_t width) { return (cells * width + 63) / 64; }

struct StoreLayout {
  uint64_t r = 0, G = 0, k = 0, runs = 0, nb = 0;
  uint32_t b_sym = 0, b_cell = 0, b_ptr = 0;
  uint64_t wR = 0, wP = 0, wM = 0, wC = 0, wB = 0;  // section words
  uint64_t oR = 0, oP = 0, oM = 0, oC = 0, oB = 0;  // section starts (words)
  uint64_t bytes = 0;
  void place() {
    wR = store_words(G, b_cell);
    wP = store_words(r, b_ptr);
    wM = store_words(r, 1);
    wC = store_words(k, b_sym);
    wB = store_words(nb, 32);
    oR = 8;
    oP = oR + wR;
    oM = oP + wP;
    oC = oM + wM;
    oB = oC + wC;
    bytes = (oB + wB) * 8;
  }
};

// cell i of width b (1..64) of a section
__device__ __forceinline__ uint64_t cell_get(const uint64_t* __restrict__ w, uint64_t i, uint32_t b) {
  const uint64_t bit = i * b;
  const uint64_t q = bit >> 6;
  const uint32_t o = (uint32_t)(bit & 63);
  uint64_t v = w[q] >> o;
  if (o + b > 64) v |= w[q + 1] << (64 - o);
  return b == 64 ? v : v & ((1ull << b) - 1);
}

// number of entries of the ascending a[0..n) below key
__device__ __forceinline__ uint64_t count_below(const uint64_t* __restrict__ a, uint64_t n,
                                                uint64_t key) {
  uint64_t lo = 0, hi = n;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Word wi of a section of n cells of width b, from the cells' values get(i),
// asked in increasing i.
template <typename Get>
__device__ __forceinline__ uint64_t pack_word(uint64_t wi, uint64_t n, uint32_t b, Get& get) {
  const uint64_t lo = wi * 64;
  const uint64_t end = min(n, (lo + 64 + b - 1) / b);
  uint64_t word = 0;
  for (uint64_t i = lo / b; i < end; ++i) {
    const uint64_t v = get(i);
    const uint64_t at = i * b;
    word |= at >= lo ? v << (at - lo) : v >> (lo - at);
  }
  return word;
}

// run rules: flag per rule, the longest run
__global__ void k_st_runflags(const uint32_t* __restrict__ mult, uint64_t r,
                              uint64_t* __restrict__ fl, uint32_t* __restrict__ longest) {
  PP_LOOP(x, r) {
    const uint32_t m = mult[x];
    fl[x] = m >= 2;
    if (m >= 2) atomicMax(longest, m);
  }
}

// the run rules in id order and the cell of R that holds each one's length
__global__ void k_st_runlist(const uint32_t* __restrict__ mult, const uint64_t* __restrict__ off,
                             const uint64_t* __restrict__ rb, uint64_t r,
                             uint32_t* __restrict__ rr, uint64_t* __restrict__ lcell) {
  PP_LOOP(x, r) {
    if (mult[x] < 2) continue;
    const uint64_t j = rb[x];
    rr[j] = (uint32_t)x;
    lcell[j] = off[x] + j + 1;  // the rule's symbol cell is off[x] + j
  }
}

// R: the cells of the right-hand sides, a length cell after each run rule's symbol
struct RCells {
  const uint32_t* rhs;
  const uint32_t* mult;
  const uint32_t* rr;
  const uint64_t* lcell;
  uint64_t runs;
  uint64_t nl;  // length cells before the cell asked next
  bool started = false;
  __device__ uint64_t operator()(uint64_t i) {
    if (!started) {
      nl = count_below(lcell, runs, i);
      started = true;
    }
    if (nl < runs && lcell[nl] == i) return mult[rr[nl++]];
    return rhs[i - nl];
  }
};

__global__ void k_st_pack_r(const uint32_t* __restrict__ rhs, const uint32_t* __restrict__ mult,
                            const uint32_t* __restrict__ rr, const uint64_t* __restrict__ lcell,
                            uint64_t runs, uint64_t G, uint32_t b, uint64_t nw,
                            uint64_t* __restrict__ out) {
  PP_LOOP(wi, nw) {
    RCells get{rhs, mult, rr, lcell, runs, 0};
    out[wi] = pack_word(wi, G, b, get);
  }
}

// P: the first cell of rule x is off[x] plus the run rules before x
__global__ void k_st_pack_p(const uint64_t* __restrict__ off, const uint64_t* __restrict__ rb,
                            uint64_t r, uint32_t b, uint64_t nw, uint64_t* __restrict__ out) {
  PP_LOOP(wi, nw) {
    auto get = [&](uint64_t x) { return off[x] + rb[x]; };
    out[wi] = pack_word(wi, r, b, get);
  }
}

// M: one wave per 64 rules, one ballot per word
__global__ void k_st_pack_m(const uint32_t* __restrict__ mult, uint64_t r, uint64_t nw,
                            uint64_t* __restrict__ out) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / 64);
  for (uint64_t wi = blockIdx.x * (uint64_t)(blockDim.x / 64) + (threadIdx.x >> 6); wi < nw;
       wi += waves) {
    const uint64_t x = wi * 64 + lane;
    const uint64_t bits = __ballot(x < r && mult[x] >= 2);
    if (lane == 0) out[wi] = bits;
  }
}

__global__ void k_st_pack_c(const uint32_t* __restrict__ c, uint64_t k, uint32_t b, uint64_t nw,
                            uint64_t* __restrict__ out) {
  PP_LOOP(wi, nw) {
    auto get = [&](uint64_t j) { return (uint64_t)c[j]; };
    out[wi] = pack_word(wi, k, b, get);
  }
}

// decode: pointers and run marks
__global__ void k_st_unpack_pm(const uint64_t* __restrict__ P, const uint64_t* __restrict__ M,
                               uint64_t r, uint32_t b_ptr, uint64_t* __restrict__ S,
                               uint64_t* __restrict__ fl) {
  PP_LOOP(x, r) {
    S[x] = cell_get(P, x, b_ptr);
    fl[x] = (M[x >> 6] >> (x & 63)) & 1;
  }
}

// decode: the pointers start at 0 and rise, a rule spans at most 2^32 - 1
// cells, a run rule exactly 2 (S[r] = G)
__global__ void k_st_check_ptr(const uint64_t* __restrict__ S, const uint64_t* __restrict__ fl,
                               uint64_t r, uint32_t* __restrict__ err) {
  PP_LOOP(x, r) {
    const uint64_t a = S[x], b = S[x + 1];
    const bool bad = (x == 0 && a != 0) || b <= a || b - a > 0xFFFFFFFFull || (fl[x] && b - a != 2);
    if (bad) atomicOr(err, 1u);
  }
}

// decode: offsets, run list, placeholder multiplicities
__global__ void k_st_rules(const uint64_t* __restrict__ S, const uint64_t* __restrict__ fl,
                           const uint64_t* __restrict__ rb, uint64_t r,
                           uint64_t* __restrict__ off, uint32_t* __restrict__ mult,
                           uint32_t* __restrict__ rr, uint64_t* __restrict__ lcell) {
  PP_LOOP(x, r) {
    const uint64_t j = rb[x];
    off[x] = S[x] - j;
    mult[x] = fl[x] ? 0 : 1;
    if (fl[x]) {
      rr[j] = (uint32_t)x;
      lcell[j] = S[x] + 1;
    }
  }
}

// decode: the first cell of each block (cb[b] = S[bounds[b] - 256]; S[r] = G)
__global__ void k_st_blockcells(const uint64_t* __restrict__ S, const uint32_t* __restrict__ bounds,
                                uint32_t nb, uint64_t* __restrict__ cb) {
  PP_LOOP(b, nb) cb[b] = S[bounds[b] - 256];
}

// decode: kCellsPerThread consecutive cells of R per thread.  A length cell
// gives its run rule's multiplicity (at least 2); any other cell is the next
// right-hand-side symbol and must name an id below its block's first id.
__global__ __launch_bounds__(kPB) void k_st_cells(const uint64_t* __restrict__ R, uint64_t G,
                                                  uint32_t b, const uint64_t* __restrict__ lcell,
                                                  const uint32_t* __restrict__ rr, uint64_t runs,
                                                  const uint64_t* __restrict__ cb,
                                                  const uint32_t* __restrict__ bounds, uint32_t nb,
                                                  uint32_t* __restrict__ rhs,
                                                  uint32_t* __restrict__ mult,
                                                  uint32_t* __restrict__ longest,
                                                  uint32_t* __restrict__ err) {
  __shared__ uint64_t s_cb[kStoreMaxBounds];
  __shared__ uint32_t s_bd[kStoreMaxBounds];
  for (uint32_t i = threadIdx.x; i < nb; i += blockDim.x) {
    s_cb[i] = cb[i];
    s_bd[i] = bounds[i];
  }
  __syncthreads();
  const uint64_t chunks = (G + kCellsPerThread - 1) / kCellsPerThread;
  PP_LOOP(t, chunks) {
    const uint64_t i0 = t * kCellsPerThread;
    const uint64_t i1 = min(G, i0 + kCellsPerThread);
    uint64_t nl = count_below(lcell, runs, i0);
    uint32_t blk = 0;  // the last block whose first cell is at most i0
    for (uint32_t step = kStoreMaxBounds / 2; step; step >>= 1)
      if (blk + step < nb && s_cb[blk + step] <= i0) blk += step;
    bool bad = false;
    uint32_t lg = 0;
    for (uint64_t i = i0; i < i1; ++i) {
      while (blk + 1 < nb && s_cb[blk + 1] <= i) ++blk;
      const uint64_t v = cell_get(R, i, b);
      if (nl < runs && lcell[nl] == i) {
        bad |= v < 2;
        mult[rr[nl]] = (uint32_t)v;
        lg = max(lg, (uint32_t)v);
        ++nl;
      } else {
        bad |= v >= s_bd[blk];
        rhs[i - nl] = (uint32_t)v;
      }
    }
    if (bad) atomicOr(err, 2u);
    if (lg) atomicMax(longest, lg);
  }
}

__global__ void k_st_unpack_c(const uint64_t* __restrict__ C, uint64_t k, uint32_t b, uint64_t ids,
                              uint32_t* __restrict__ c, uint32_t* __restrict__ err) {
  PP_LOOP(j, k) {
    const uint64_t y = cell_get(C, j, b);
    if (y >= ids) atomicOr(err, 4u);
    c[j] = (uint32_t)y;
  }
}

// the strings' total expansion, stopping at kLenLimit
__global__ void k_st_total(const uint32_t* __restrict__ c, uint64_t k, const uint64_t* __restrict__ E,
                           unsigned long long* __restrict__ total) {
  uint64_t sum = 0;
  PP_LOOP(j, k) {
    const uint32_t y = c[j];
    sum = min(sum + (y < 256 ? 1 : E[y - 256]), kLenLimit);
  }
  for (int d = 32; d; d >>= 1) sum = min(sum + (uint64_t)__shfl_down(sum, d), kLenLimit);
  if ((threadIdx.x & 63) == 0 && sum) {
    unsigned long long old = *total, seen;
    do {
      seen = old;
      old = atomicCAS(total, seen, (unsigned long long)min((uint64_t)seen + sum, kLenLimit));
    } while (old != seen);
  }
}

}  // namespace

// Size of p's stored file; with d_out (cap bytes at least that size) the
// file is written there.
static uint64_t store_encode(lcg_slp* p, uint8_t* d_out, uint64_t cap, hipStream_t s) {
  StoreLayout L;
  L.r = p->g;
  L.k = p->k;
  L.nb = p->bounds.size();
  const uint64_t r = L.r;
  DBuf<uint64_t> fl, rb, lcell;
  DBuf<uint32_t> rr, longest;
  fl.need(std::max<uint64_t>(r, 1), s);
  rb.need(r + 1, s);
  longest.need(1, s);
  zero(longest.p, 4, s);
  if (r) {
    k_st_runflags<<<pgrid(r), kPB, 0, s>>>(p->mult.p, r, fl.p, longest.p);
    PP_CHECK("st_runflags");
  }
  Scan sc;
  sc.run(fl.p, rb.p, r, s);
  uint64_t runs = 0;
  uint32_t lg = 0;
  HIP_CHECK(hipMemcpyAsync(&runs, rb.p + r, 8, hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipMemcpyAsync(&lg, longest.p, 4, hipMemcpyDeviceToHost, s));
  sync(s);
  L.runs = runs;
  L.G = p->q + runs;
  L.b_sym = store_bits(255 + r);
  L.b_cell = std::max(L.b_sym, runs ? store_bits(lg) : 1u);
  L.b_ptr = r ? store_bits(L.G - 1) : 1;
  L.place();
  if (!d_out || cap < L.bytes) return L.bytes;
  if (reinterpret_cast<uintptr_t>(d_out) % 8) throw LcgError{LCG_EINVAL, "d_out is not 8-byte aligned"};
  uint64_t* w = reinterpret_cast<uint64_t*>(d_out);
  std::vector<uint64_t> head = {kStoreMagic, r, L.G, L.k, runs, L.nb,
                                L.b_sym | (uint64_t)L.b_cell << 8 | (uint64_t)L.b_ptr << 16,
                                L.bytes};
  std::vector<uint32_t> bnd(L.wB * 2, 0);
  std::copy(p->bounds.begin(), p->bounds.end(), bnd.begin());
  HIP_CHECK(hipMemcpyAsync(w, head.data(), 64, hipMemcpyHostToDevice, s));
  HIP_CHECK(hipMemcpyAsync(w + L.oB, bnd.data(), L.wB * 8, hipMemcpyHostToDevice, s));
  rr.need(std::max<uint64_t>(runs, 1), s);
  lcell.need(std::max<uint64_t>(runs, 1), s);
  if (runs) {
    k_st_runlist<<<pgrid(r), kPB, 0, s>>>(p->mult.p, p->off.p, rb.p, r, rr.p, lcell.p);
    PP_CHECK("st_runlist");
  }
  if (L.wR) {
    k_st_pack_r<<<pgrid(L.wR), kPB, 0, s>>>(p->rhs.p, p->mult.p, rr.p, lcell.p, runs, L.G, L.b_cell,
                                            L.wR, w + L.oR);
    PP_CHECK("st_pack_r");
  }
  if (L.wP) {
    k_st_pack_p<<<pgrid(L.wP), kPB, 0, s>>>(p->off.p, rb.p, r, L.b_ptr, L.wP, w + L.oP);
    PP_CHECK("st_pack_p");
    k_st_pack_m<<<pgrid(L.wM * 64), kPB, 0, s>>>(p->mult.p, r, L.wM, w + L.oM);
    PP_CHECK("st_pack_m");
  }
  k_st_pack_c<<<pgrid(L.wC), kPB, 0, s>>>(p->c.p, L.k, L.b_sym, L.wC, w + L.oC);
  PP_CHECK("st_pack_c");
  sync(s);
  return L.bytes;
}

// The grammar of a stored file (see include/lcg.h for what is checked).
static lcg_slp* store_decode(const uint8_t* d_in, uint64_t n, hipStream_t s) {
  auto bad = [](const char* why) { return LcgError{LCG_EINVAL, std::string("stored grammar: ") + why}; };
  if (n < 64 || n % 8) throw bad("size is not a whole header plus words");
  if (reinterpret_cast<uintptr_t>(d_in) % 8) throw LcgError{LCG_EINVAL, "d_in is not 8-byte aligned"};
  const uint64_t* w = reinterpret_cast<const uint64_t*>(d_in);
  uint64_t h[8];
  HIP_CHECK(hipMemcpyAsync(h, w, 64, hipMemcpyDeviceToHost, s));
  sync(s);
  if (h[0] != kStoreMagic) throw bad("bad magic");
  StoreLayout L;
  L.r = h[1];
  L.G = h[2];
  L.k = h[3];
  L.runs = h[4];
  L.nb = h[5];
  L.b_sym = h[6] & 0xFF;
  L.b_cell = (h[6] >> 8) & 0xFF;
  L.b_ptr = (h[6] >> 16) & 0xFF;
  if (h[6] >> 24) throw bad("bad widths word");
  if (h[7] != n) throw bad("size differs from the header");
  const uint64_t r = L.r, G = L.G, k = L.k, runs = L.runs;
  if (r > 0xFFFFFFFFull - 256 || k == 0 || k > 0xFFFFFFFFull || runs > r || G >= (1ull << 58) ||
      G < r + runs || (r == 0 && G != 0) || L.nb < 1 || L.nb > kStoreMaxBounds)
    throw bad("counts out of range");
  if (L.b_sym != store_bits(255 + r) || L.b_cell < L.b_sym || L.b_cell > 32 ||
      L.b_ptr != (r ? store_bits(G - 1) : 1u))
    throw bad("widths do not match the counts");
  L.place();
  if (L.bytes != n) throw bad("sections do not fill the size");
  {  // padding: the bits after a section's last cell are zero
    const uint64_t sec[5][3] = {{L.oR, G, L.b_cell}, {L.oP, r, L.b_ptr}, {L.oM, r, 1},
                                {L.oC, k, L.b_sym}, {L.oB, L.nb, 32}};
    uint64_t last[5] = {0, 0, 0, 0, 0};
    for (int i = 0; i < 5; ++i) {
      const uint64_t bits = sec[i][1] * sec[i][2];
      if (bits % 64)
        HIP_CHECK(hipMemcpyAsync(&last[i], w + sec[i][0] + bits / 64, 8, hipMemcpyDeviceToHost, s));
    }
    sync(s);
    for (int i = 0; i < 5; ++i) {
      const uint64_t bits = sec[i][1] * sec[i][2];
      if (bits % 64 && (last[i] >> (bits % 64)) != 0) throw bad("nonzero padding");
    }
  }
  std::vector<uint32_t> bnd(L.wB * 2);
  HIP_CHECK(hipMemcpyAsync(bnd.data(), w + L.oB, L.wB * 8, hipMemcpyDeviceToHost, s));
  sync(s);
  bnd.resize(L.nb);
  if (bnd[0] != 256 || bnd[L.nb - 1] != 256 + r) throw bad("bad block bounds");
  for (uint64_t b = 1; b < L.nb; ++b)
    if (bnd[b] < bnd[b - 1]) throw bad("bad block bounds");

  std::unique_ptr<lcg_slp> out(new lcg_slp());
  out->g = (uint32_t)r;
  out->q = G - runs;
  out->k = (uint32_t)k;
  out->bounds = bnd;
  out->off.need(r + 1, s);
  out->rhs.need(std::max<uint64_t>(out->q, 1), s);
  out->mult.need(std::max<uint64_t>(r, 1), s);
  out->c.need(k, s);
  DBuf<uint64_t> S, fl, rb, lcell, cb;
  DBuf<uint32_t> rr, err, bd, longest;
  S.need(r + 1, s);
  fl.need(std::max<uint64_t>(r, 1), s);
  rb.need(r + 1, s);
  err.need(1, s);
  zero(err.p, 4, s);
  longest.need(1, s);
  zero(longest.p, 4, s);
  if (r) {
    k_st_unpack_pm<<<pgrid(r), kPB, 0, s>>>(w + L.oP, w + L.oM, r, L.b_ptr, S.p, fl.p);
    PP_CHECK("st_unpack_pm");
  }
  k_pp_set<<<1, 1, 0, s>>>(S.p + r, G);
  PP_CHECK("pp_set");
  if (r) {
    k_st_check_ptr<<<pgrid(r), kPB, 0, s>>>(S.p, fl.p, r, err.p);
    PP_CHECK("st_check_ptr");
  }
  Scan sc;
  sc.run(fl.p, rb.p, r, s);
  uint64_t nruns = 0;
  uint32_t e = 0;
  HIP_CHECK(hipMemcpyAsync(&nruns, rb.p + r, 8, hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipMemcpyAsync(&e, err.p, 4, hipMemcpyDeviceToHost, s));
  sync(s);
  if (nruns != runs) throw bad("run count differs from the header");
  if (e) throw bad("bad rule pointers");
  // the pointers are sound: every length cell lies inside R and the cells
  // before cell i hold at most i of them
  rr.need(std::max<uint64_t>(runs, 1), s);
  lcell.need(std::max<uint64_t>(runs, 1), s);
  if (r) {
    k_st_rules<<<pgrid(r), kPB, 0, s>>>(S.p, fl.p, rb.p, r, out->off.p, out->mult.p, rr.p, lcell.p);
    PP_CHECK("st_rules");
  }
  k_pp_set<<<1, 1, 0, s>>>(out->off.p + r, G - runs);
  PP_CHECK("pp_set");
  bd.need(L.nb, s);
  cb.need(L.nb, s);
  HIP_CHECK(hipMemcpyAsync(bd.p, bnd.data(), L.nb * 4, hipMemcpyHostToDevice, s));
  k_st_blockcells<<<1, kPB, 0, s>>>(S.p, bd.p, (uint32_t)L.nb, cb.p);
  PP_CHECK("st_blockcells");
  if (G) {
    const uint64_t chunks = (G + kCellsPerThread - 1) / kCellsPerThread;
    k_st_cells<<<pgrid(chunks), kPB, 0, s>>>(w + L.oR, G, L.b_cell, lcell.p, rr.p, runs, cb.p, bd.p,
                                             (uint32_t)L.nb, out->rhs.p, out->mult.p, longest.p,
                                             err.p);
    PP_CHECK("st_cells");
  }
  k_st_unpack_c<<<pgrid(k), kPB, 0, s>>>(w + L.oC, k, L.b_sym, 256 + r, out->c.p, err.p);
  PP_CHECK("st_unpack_c");
  uint32_t lg = 0;
  HIP_CHECK(hipMemcpyAsync(&lg, longest.p, 4, hipMemcpyDeviceToHost, s));
  e = read_dev(err.p, s);
  if (e & 2) throw bad("a rule names an id of its own block or above, or a run is shorter than 2");
  if (e & 4) throw bad("C names an id beyond the rules");
  if (L.b_cell != std::max(L.b_sym, runs ? store_bits(lg) : 1u))
    throw bad("widths do not match the longest run");
  out->stats[6] = r;
  out->stats[7] = G;
  slp_lens(out.get(), s);
  {
    DBuf<uint64_t> tot;
    tot.need(1, s);
    zero(tot.p, 8, s);
    k_st_total<<<std::min(pgrid(k), 1024u), kPB, 0, s>>>(out->c.p, k, out->E.p,
                                                         reinterpret_cast<unsigned long long*>(tot.p));
    PP_CHECK("st_total");
    if (read_dev(tot.p, s) >= kLenLimit) throw bad("the strings reach 2^61 bytes");
  }
  return out.release();
}

}  // namespace lcg

using namespace lcg;

extern "C" {

lcg_status lcg_postprocess(lcg_grammar_t g, uint32_t flags, hipStream_t stream, lcg_slp_t* out) {
  return guard([&] {
    live(g);
    if (!out) throw LcgError{LCG_EINVAL, "out is NULL"};
    if (flags & ~uint32_t(LCG_PP_RL | LCG_PP_SIMP)) throw LcgError{LCG_EINVAL, "unknown flags"};
    if (g->k == 0) throw LcgError{LCG_EINVAL, "the grammar holds no string"};
    *out = postprocess_core(g, flags, stream);
  });
}

lcg_status lcg_slp_size(lcg_slp_t p, uint32_t* g, uint64_t* rhs_len, uint32_t* k) {
  return guard([&] {
    if (!p) throw LcgError{LCG_EINVAL, "slp is NULL"};
    if (g) *g = p->g;
    if (rhs_len) *rhs_len = p->q;
    if (k) *k = p->k;
  });
}

lcg_status lcg_slp_stats(lcg_slp_t p, uint64_t* h_stats) {
  return guard([&] {
    if (!p || !h_stats) throw LcgError{LCG_EINVAL, "slp or h_stats is NULL"};
    std::memcpy(h_stats, p->stats, sizeof(p->stats));
  });
}

lcg_status lcg_slp_device(lcg_slp_t p, const uint64_t** d_off, const uint32_t** d_rhs,
                          const uint32_t** d_mult, const uint32_t** d_c) {
  return guard([&] {
    if (!p) throw LcgError{LCG_EINVAL, "slp is NULL"};
    if (d_off) *d_off = p->off.p;
    if (d_rhs) *d_rhs = p->rhs.p;
    if (d_mult) *d_mult = p->mult.p;
    if (d_c) *d_c = p->c.p;
  });
}

lcg_status lcg_slp_copy(lcg_slp_t p, uint64_t* h_off, uint32_t* h_rhs, uint32_t* h_mult,
                        uint32_t* h_c) {
  return guard([&] {
    if (!p) throw LcgError{LCG_EINVAL, "slp is NULL"};
    if (h_off) HIP_CHECK(hipMemcpy(h_off, p->off.p, (p->g + 1ull) * 8, hipMemcpyDeviceToHost));
    if (h_rhs && p->q) HIP_CHECK(hipMemcpy(h_rhs, p->rhs.p, p->q * 4, hipMemcpyDeviceToHost));
    if (h_mult && p->g) HIP_CHECK(hipMemcpy(h_mult, p->mult.p, p->g * 4ull, hipMemcpyDeviceToHost));
    if (h_c && p->k) HIP_CHECK(hipMemcpy(h_c, p->c.p, p->k * 4ull, hipMemcpyDeviceToHost));
  });
}

lcg_status lcg_slp_extract(lcg_slp_t p, uint32_t nq, const uint32_t* d_j, const uint64_t* d_start,
                           const uint32_t* d_len, const uint64_t* d_out_off, uint8_t* d_out,
                           hipStream_t stream) {
  return guard([&] {
    if (!p) throw LcgError{LCG_EINVAL, "slp is NULL"};
    if (!nq) return;
    if (!d_j || !d_start || !d_len || !d_out_off || !d_out)
      throw LcgError{LCG_EINVAL, "NULL query or output array"};
    slp_extract_core(p, nq, d_j, d_start, d_len, d_out_off, d_out, stream);
  });
}

lcg_status lcg_slp_expand_strings(lcg_slp_t p, uint32_t j0, uint32_t j1, uint8_t* d_out,
                                  uint64_t cap, uint64_t* d_offsets, uint64_t* total,
                                  hipStream_t stream) {
  return guard([&] {
    if (!p) throw LcgError{LCG_EINVAL, "slp is NULL"};
    if (cap && !d_out) throw LcgError{LCG_EINVAL, "d_out is NULL"};
    slp_expand_core(p, j0, j1, d_out, cap, d_offsets, total, stream);
  });
}

lcg_status lcg_slp_encode(lcg_slp_t p, uint8_t* d_out, uint64_t cap, uint64_t* bytes,
                          hipStream_t stream) {
  return guard([&] {
    if (!p || !bytes) throw LcgError{LCG_EINVAL, "slp or bytes is NULL"};
    if (cap && !d_out) throw LcgError{LCG_EINVAL, "d_out is NULL"};
    *bytes = store_encode(p, d_out, cap, stream);
    if (d_out && cap < *bytes) throw LcgError{LCG_EINVAL, "output buffer too small"};
  });
}

lcg_status lcg_slp_decode(const uint8_t* d_in, uint64_t bytes, hipStream_t stream, lcg_slp_t* out) {
  return guard([&] {
    if (!d_in || !out) throw LcgError{LCG_EINVAL, "d_in or out is NULL"};
    *out = store_decode(d_in, bytes, stream);
  });
}

void lcg_slp_free(lcg_slp_t p) { delete p; }

}  // extern "C"
