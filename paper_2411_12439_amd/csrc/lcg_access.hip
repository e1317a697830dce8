// Queries on a level grammar without decompressing it: random access, the
// longest common extensions of App. B's match completion, and its maximal
// exact matches.
//
// Random access: bytes [start, start + len) of string j without expanding the
// rest of the string (the grammar's expansion lengths locate every symbol,
// Sec. 2.2's exp(X) per rule).  One wave (one block for queries longer than
// 256 bytes) answers one query: starting from C[j] it keeps, level by level,
// only the symbols whose expansion overlaps the range -- they cover disjoint
// pieces of at least one byte each, so there are never more than len of
// them -- and the level-1 symbols finally write their bytes.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <unordered_map>
#include <vector>

#include "lcg_host.h"

namespace lcg {
namespace {

constexpr int kXBlock = 256;

// Queries of at most kXWaveMax bytes are answered by one wave each (k_extract
// below skips them): a 256-entry frontier per wave keeps eight times more
// queries in flight per CU than a block with the full frontier, and each
// query is a chain of dependent reads, one level after another.
constexpr uint32_t kXWaveMax = 256;
constexpr int kXWaves = kXBlock / 64;

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(kXBlock) void k_extract_wave(
    const LevelPtrs* __restrict__ lv_ptr, const uint64_t* const* __restrict__ explen,
    const uint8_t* __restrict__ c_level, const uint32_t* __restrict__ c_sym, uint32_t k,
    uint32_t nq, const uint32_t* __restrict__ qj, const uint64_t* __restrict__ qstart,
    const uint32_t* __restrict__ qlen, const uint64_t* __restrict__ qout, uint8_t* __restrict__ out,
    unsigned int* __restrict__ bad) {
  __shared__ uint32_t s_sym[kXWaves][2][kXWaveMax];
  __shared__ int64_t s_pos[kXWaves][2][kXWaveMax];
  __shared__ uint32_t s_n[kXWaves][2];
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t(*sym)[kXWaveMax] = s_sym[wv];
  int64_t(*pos)[kXWaveMax] = s_pos[wv];
  uint32_t* cnt = s_n[wv];
  for (uint32_t q = blockIdx.x * kXWaves + wv; q < nq; q += gridDim.x * kXWaves) {
    const uint64_t len = qlen[q];
    if (len < 1 || len > kXWaveMax) continue;  // the block kernel's
    uint8_t* dst = out + qout[q];
    int level = -1;
    const uint32_t j = qj[q];
    const uint64_t start = qstart[q];
    uint32_t y = 0;
    if (j < k) {
      const uint32_t lv = c_level[j];
      y = c_sym[j];
      const uint64_t e = lv == 0 ? 1 : explen[lv - 1][y];
      if (start <= e && len <= e - start) level = (int)lv;
    }
    if (level < 0) {
      if (lane == 0) atomicAdd(bad, 1u);
      continue;
    }
    if (level == 0) {
      if (lane == 0) dst[0] = (uint8_t)y;
      continue;
    }
    if (lane == 0) {
      sym[0][0] = y;
      pos[0][0] = -(int64_t)start;
      cnt[0] = 1;
    }
    wave_sync();
    int cur = 0;
    while (level >= 2) {  // keep the children overlapping [0, len)
      if (lane == 0) cnt[cur ^ 1] = 0;
      wave_sync();
      const LevelPtrs L = lv_ptr[level - 1];
      const uint64_t* e_below = explen[level - 2];
      const uint32_t* rhs = static_cast<const uint32_t*>(L.rhs);
      const uint32_t n = cnt[cur];
      for (uint32_t i = lane; i < n; i += 64) {
        const uint32_t r = sym[cur][i];
        int64_t p = pos[cur][i];
        const uint64_t b = L.off[r + 1];
        for (uint64_t t = L.off[r]; t < b && p < (int64_t)len; ++t) {
          const uint32_t c = rhs[t];
          const int64_t e = (int64_t)e_below[c];
          if (p + e > 0) {
            const uint32_t slot = atomicAdd(&cnt[cur ^ 1], 1u);
            if (slot < kXWaveMax) {  // always: the overlapping symbols are at most len
              sym[cur ^ 1][slot] = c;
              pos[cur ^ 1][slot] = p;
            }
          }
          p += e;
        }
      }
      wave_sync();
      cur ^= 1;
      --level;
      if (lane == 0 && cnt[cur] > kXWaveMax) cnt[cur] = kXWaveMax;
      wave_sync();
    }
    {  // level 1: the bytes
      const LevelPtrs L = lv_ptr[0];
      const uint8_t* rhs = static_cast<const uint8_t*>(L.rhs);
      const uint32_t n = cnt[cur];
      for (uint32_t i = lane; i < n; i += 64) {
        const uint32_t r = sym[cur][i];
        int64_t p = pos[cur][i];
        const uint64_t a = L.off[r], b = L.off[r + 1];
        uint64_t t = a + (p < 0 ? (uint64_t)(-p) : 0);
        p = p < 0 ? 0 : p;
        for (; t < b && p < (int64_t)len; ++t, ++p) dst[p] = rhs[t];
      }
    }
    wave_sync();  // the frontier is rewritten by the wave's next query
  }
}

__global__ __launch_bounds__(kXBlock) void k_extract(
    const LevelPtrs* __restrict__ lv_ptr, const uint64_t* const* __restrict__ explen,
    const uint8_t* __restrict__ c_level, const uint32_t* __restrict__ c_sym, uint32_t k,
    uint32_t nq, const uint32_t* __restrict__ qj, const uint64_t* __restrict__ qstart,
    const uint32_t* __restrict__ qlen, const uint64_t* __restrict__ qout, uint8_t* __restrict__ out,
    unsigned int* __restrict__ bad) {
  __shared__ uint32_t s_sym[2][LCG_EXTRACT_MAX];
  __shared__ int64_t s_pos[2][LCG_EXTRACT_MAX];
  __shared__ uint32_t s_n[2];
  __shared__ int s_level;
  for (uint32_t q = blockIdx.x; q < nq; q += gridDim.x) {
    const uint64_t len = qlen[q];
    if (len >= 1 && len <= kXWaveMax) continue;  // answered by k_extract_wave
    uint8_t* dst = out + qout[q];
    if (threadIdx.x == 0) {
      int level = -1;
      const uint32_t j = qj[q];
      const uint64_t start = qstart[q];
      if (j < k && len >= 1 && len <= LCG_EXTRACT_MAX) {
        const uint32_t lv = c_level[j], y = c_sym[j];
        const uint64_t e = lv == 0 ? 1 : explen[lv - 1][y];
        if (start <= e && len <= e - start) {
          level = (int)lv;
          if (lv == 0) dst[0] = (uint8_t)y;
          s_sym[0][0] = y;
          s_pos[0][0] = -(int64_t)start;
          s_n[0] = 1;
        }
      }
      if (level < 0) atomicAdd(bad, 1u);
      s_level = level;
    }
    __syncthreads();
    int level = s_level;
    int cur = 0;
    // levels >= 2: keep the children overlapping [0, len)
    while (level >= 2) {
      if (threadIdx.x == 0) s_n[cur ^ 1] = 0;
      __syncthreads();
      const LevelPtrs L = lv_ptr[level - 1];
      const uint64_t* e_below = explen[level - 2];
      const uint32_t n = s_n[cur];
      for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const uint32_t r = s_sym[cur][i];
        int64_t p = s_pos[cur][i];
        const uint64_t b = L.off[r + 1];
        const uint32_t* rhs = static_cast<const uint32_t*>(L.rhs);
        for (uint64_t t = L.off[r]; t < b && p < (int64_t)len; ++t) {
          const uint32_t c = rhs[t];
          const int64_t e = (int64_t)e_below[c];
          if (p + e > 0) {
            const uint32_t slot = atomicAdd(&s_n[cur ^ 1], 1u);
            if (slot < LCG_EXTRACT_MAX) {  // always: the overlapping symbols are at most len
              s_sym[cur ^ 1][slot] = c;
              s_pos[cur ^ 1][slot] = p;
            }
          }
          p += e;
        }
      }
      __syncthreads();
      cur ^= 1;
      --level;
      if (threadIdx.x == 0 && s_n[cur] > LCG_EXTRACT_MAX) s_n[cur] = LCG_EXTRACT_MAX;
      __syncthreads();
    }
    if (level == 1) {
      const LevelPtrs L = lv_ptr[0];
      const uint8_t* rhs = static_cast<const uint8_t*>(L.rhs);
      const uint32_t n = s_n[cur];
      for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const uint32_t r = s_sym[cur][i];
        int64_t p = s_pos[cur][i];
        const uint64_t a = L.off[r], b = L.off[r + 1];
        uint64_t t = a + (p < 0 ? (uint64_t)(-p) : 0);
        p = p < 0 ? 0 : p;
        for (; t < b && p < (int64_t)len; ++t, ++p) dst[p] = rhs[t];
      }
    }
    __syncthreads();  // the LDS frontier is rewritten by the next query
  }
}

// ---------------------------------------------------------------- LCE
// A position of a string seen through the grammar: for every level from the
// string's top symbol down to 1, the symbol covering the position and the
// position's offset inside that symbol's expansion.
constexpr int kMaxLv = 64;

struct Cursor {
  int top;                // level of C[j] (0: a one-byte string)
  uint32_t sym[kMaxLv];   // sym[l]: level-l symbol covering the position
  uint64_t off[kMaxLv];   // offset inside exp(sym[l])
};

__device__ __forceinline__ uint64_t sym_len(const uint64_t* const* explen, int l, uint32_t y) {
  return explen[l - 1][y];
}

// recompute the levels below l from sym[l], off[l]
__device__ void cursor_descend(Cursor& c, int l, const LevelPtrs* lv_ptr,
                               const uint64_t* const* explen) {
  for (; l >= 2; --l) {
    const LevelPtrs L = lv_ptr[l - 1];
    const uint32_t* rhs = static_cast<const uint32_t*>(L.rhs);
    const uint64_t* eb = explen[l - 2];
    uint64_t o = c.off[l];
    const uint64_t tb = L.off[c.sym[l] + 1];
    // the child holding offset o (o < exp length of sym[l]: the scan ends in the rule)
    for (uint64_t t = L.off[c.sym[l]]; t < tb; ++t) {
      const uint32_t ch = rhs[t];
      const uint64_t e = eb[ch];
      c.sym[l - 1] = ch;
      c.off[l - 1] = o;
      if (o < e) break;
      o -= e;
    }
  }
}

__device__ void cursor_init(Cursor& c, int top, uint32_t y, uint64_t x, const LevelPtrs* lv_ptr,
                            const uint64_t* const* explen) {
  c.top = top;
  c.sym[top] = y;
  c.off[top] = x;
  if (top >= 1) cursor_descend(c, top, lv_ptr, explen);
}

// move by s bytes (forward, or backward with BACK), staying inside the string
template <bool BACK>
__device__ void cursor_move(Cursor& c, uint64_t s, const LevelPtrs* lv_ptr,
                            const uint64_t* const* explen) {
  int l = 1;
  for (; l < c.top; ++l) {
    if (BACK ? c.off[l] >= s : c.off[l] + s < sym_len(explen, l, c.sym[l])) break;
  }
  for (int m = l; m <= c.top; ++m) c.off[m] = BACK ? c.off[m] - s : c.off[m] + s;
  cursor_descend(c, l, lv_ptr, explen);
}

__device__ __forceinline__ uint8_t level1_byte(const LevelPtrs* lv_ptr, uint32_t r, uint64_t o) {
  const LevelPtrs L = lv_ptr[0];
  return static_cast<const uint8_t*>(L.rhs)[L.off[r] + o];
}

// The common extension of exp(y1) from offset p1 and exp(y2) from offset p2
// (level t1 and t2 symbols of expansion lengths n1, n2; level 0: a byte),
// forward or, with BACK, backward from just before p1, p2.  Two cursors walk
// the expansions together.  When both sit at the same offset of the same
// symbol at some level, the rest of that symbol (its expansion is the same)
// is skipped in one step -- the highest such level first; otherwise the bytes
// of the two level-1 symbols are compared up to a mismatch or the end of
// either symbol.
template <bool BACK>
__device__ uint64_t lce_walk(const LevelPtrs* __restrict__ lv_ptr,
                             const uint64_t* const* __restrict__ explen, int t1, uint32_t y1,
                             uint64_t p1, uint64_t n1, int t2, uint32_t y2, uint64_t p2,
                             uint64_t n2) {
  // bytes available in the walking direction
  uint64_t room1 = BACK ? p1 : n1 - p1, room2 = BACK ? p2 : n2 - p2;
  if (!room1 || !room2) return 0;
  Cursor a, b;
  cursor_init(a, t1, y1, BACK ? p1 - 1 : p1, lv_ptr, explen);
  cursor_init(b, t2, y2, BACK ? p2 - 1 : p2, lv_ptr, explen);
  uint64_t len = 0;
  for (;;) {
    uint64_t s = 0;
    for (int l = min(a.top, b.top); l >= 1; --l) {
      if (a.sym[l] == b.sym[l] && a.off[l] == b.off[l]) {
        s = BACK ? a.off[l] + 1 : sym_len(explen, l, a.sym[l]) - a.off[l];
        break;
      }
    }
    if (!s) {
      // byte by byte inside the two level-1 symbols (or the single bytes)
      uint64_t oa = a.top ? a.off[1] : 0, ob = b.top ? b.off[1] : 0;
      const uint64_t ea = a.top ? sym_len(explen, 1, a.sym[1]) : 1;
      const uint64_t eb = b.top ? sym_len(explen, 1, b.sym[1]) : 1;
      bool mismatch = false;
      for (;;) {
        const uint8_t xa = a.top ? level1_byte(lv_ptr, a.sym[1], oa) : (uint8_t)a.sym[0];
        const uint8_t xb = b.top ? level1_byte(lv_ptr, b.sym[1], ob) : (uint8_t)b.sym[0];
        if (xa != xb) {
          mismatch = true;
          break;
        }
        ++s;
        if (BACK ? (oa == 0 || ob == 0) : (oa + 1 == ea || ob + 1 == eb)) break;
        if (BACK) {
          --oa;
          --ob;
        } else {
          ++oa;
          ++ob;
        }
      }
      if (mismatch) return len + s;
    }
    len += s;
    if (s >= room1 || s >= room2) return len;  // an expansion ends
    room1 -= s;
    room2 -= s;
    cursor_move<BACK>(a, s, lv_ptr, explen);
    cursor_move<BACK>(b, s, lv_ptr, explen);
  }
}

// One thread per query: positions p1 of string j1 and p2 of string j2.
template <bool BACK>
__global__ __launch_bounds__(64) void k_lce(const LevelPtrs* __restrict__ lv_ptr,
                                            const uint64_t* const* __restrict__ explen,
                                            const uint8_t* __restrict__ c_level,
                                            const uint32_t* __restrict__ c_sym, uint32_t k,
                                            uint32_t nq, const uint32_t* __restrict__ qj1,
                                            const uint64_t* __restrict__ qp1,
                                            const uint32_t* __restrict__ qj2,
                                            const uint64_t* __restrict__ qp2,
                                            uint64_t* __restrict__ out, unsigned int* bad) {
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += gridDim.x * blockDim.x) {
    const uint32_t j1 = qj1[q], j2 = qj2[q];
    if (j1 >= k || j2 >= k) {
      atomicAdd(bad, 1u);
      continue;
    }
    const int t1 = c_level[j1], t2 = c_level[j2];
    const uint64_t n1 = t1 ? sym_len(explen, t1, c_sym[j1]) : 1;
    const uint64_t n2 = t2 ? sym_len(explen, t2, c_sym[j2]) : 1;
    const uint64_t p1 = qp1[q], p2 = qp2[q];
    if (p1 > n1 || p2 > n2) {
      atomicAdd(bad, 1u);
      continue;
    }
    out[q] = lce_walk<BACK>(lv_ptr, explen, t1, c_sym[j1], p1, n1, t2, c_sym[j2], p2, n2);
  }
}

// One thread per query: the whole expansions of the symbols (lv1, s1) and
// (lv2, s2), from their first (or, with BACK, last) byte.  lv_size[l] is the
// number of level-l symbols (256 at level 0).
template <bool BACK>
__global__ __launch_bounds__(64) void k_symbol_lce(const LevelPtrs* __restrict__ lv_ptr,
                                                   const uint64_t* const* __restrict__ explen,
                                                   const uint32_t* __restrict__ lv_size,
                                                   uint32_t levels, uint32_t nq,
                                                   const uint8_t* __restrict__ qlv1,
                                                   const uint32_t* __restrict__ qs1,
                                                   const uint8_t* __restrict__ qlv2,
                                                   const uint32_t* __restrict__ qs2,
                                                   uint64_t* __restrict__ out, unsigned int* bad) {
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += gridDim.x * blockDim.x) {
    const uint32_t t1 = qlv1[q], t2 = qlv2[q], y1 = qs1[q], y2 = qs2[q];
    if (t1 > levels || t2 > levels || y1 >= lv_size[t1] || y2 >= lv_size[t2]) {
      atomicAdd(bad, 1u);
      continue;
    }
    const uint64_t n1 = t1 ? sym_len(explen, t1, y1) : 1;
    const uint64_t n2 = t2 ? sym_len(explen, t2, y2) : 1;
    out[q] = lce_walk<BACK>(lv_ptr, explen, (int)t1, y1, BACK ? n1 : 0, n1, (int)t2, y2,
                            BACK ? n2 : 0, n2);
  }
}

// ---------------------------------------------------------------- MEMs
// Maximal exact matches between pairs of strings through the grammar
// (App. B): the level-l parses of the strings are the search space; equal
// symbols, one in each parse of a pair, are anchors, and each is completed
// into the maximal run of equal bytes on its diagonal (k_mem_extend: the lcs
// of the symbols before the anchor, the lcp of the first different symbols
// after it, with the cursor walks above).  Only the first anchor of a run of
// consecutive anchors on one diagonal (the symbols before it differ) is
// completed: the others lie inside the same match.  Many pairs go through
// one pipeline: the parses of all their strings side by side in one array
// (each string a contiguous segment), one sort of all of them by (string,
// symbol), and every later step over all pairs at once.
constexpr int kMB = 256;
constexpr uint64_t kMemMaxAnchors = 1ull << 31;  // 32-bit counts in the radix sorts

inline unsigned mem_grid(uint64_t n) {
  return (unsigned)std::min<uint64_t>((n + kMB - 1) / kMB, 16384);
}

// One pair of a batch: the C entries of its two strings and where their
// parses sit in the common array (seg_*: first symbol, n*: symbols), with the
// byte offset of each segment's first symbol in the prefix of all lengths.
struct MemPair {
  int ta, tb;
  uint32_t ya, yb;
  uint32_t sa, na, sb, nb;
  uint32_t slot_b;  // b's string slot (the high half of its sort keys)
  uint32_t same;    // a and b are one string
  uint64_t la, lb;  // byte lengths
  uint64_t ga, gb;  // byte prefix at the segments' first symbols
};

// the C entries (level, symbol) of the strings js[0..n)
__global__ __launch_bounds__(kMB) void k_mem_centries(const uint8_t* __restrict__ c_level,
                                                      const uint32_t* __restrict__ c_sym,
                                                      const uint32_t* __restrict__ js, uint32_t n,
                                                      uint32_t* __restrict__ out) {
  for (uint32_t i = blockIdx.x * kMB + threadIdx.x; i < n; i += gridDim.x * kMB) {
    out[2 * i] = c_level[js[i]];
    out[2 * i + 1] = c_sym[js[i]];
  }
}

// right-hand-side length of every symbol of a parse (levels >= 2)
__global__ __launch_bounds__(kMB) void k_mem_rhslen(const uint64_t* __restrict__ off,
                                                    const uint32_t* __restrict__ cur, uint64_t n,
                                                    uint64_t* __restrict__ cnt) {
  for (uint64_t i = blockIdx.x * (uint64_t)kMB + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * kMB) {
    const uint32_t x = cur[i];
    cnt[i] = off[x + 1] - off[x];
  }
}

// the parse one level down: every symbol's right-hand side at its place
__global__ __launch_bounds__(kMB) void k_mem_children(const uint64_t* __restrict__ off,
                                                      const uint32_t* __restrict__ rhs,
                                                      const uint32_t* __restrict__ cur, uint64_t n,
                                                      const uint64_t* __restrict__ pos,
                                                      uint32_t* __restrict__ next) {
  for (uint64_t i = blockIdx.x * (uint64_t)kMB + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * kMB) {
    const uint32_t x = cur[i];
    uint64_t p = pos[i];
    for (uint64_t t = off[x], e = off[x + 1]; t < e; ++t) next[p++] = rhs[t];
  }
}

// pos[idx[i]] for a few indexes (the segments' new starts after a step down)
__global__ __launch_bounds__(kMB) void k_mem_pick(const uint64_t* __restrict__ pos,
                                                  const uint64_t* __restrict__ idx, uint32_t n,
                                                  uint64_t* __restrict__ out) {
  for (uint32_t i = blockIdx.x * kMB + threadIdx.x; i < n; i += gridDim.x * kMB)
    out[i] = pos[idx[i]];
}

// The parse of the upper levels, while it is small, in one block per string:
// from the C entry (tops[b], ys[b]) down towards `level`, the frontier
// alternating between two global buffers of kMemTopCap entries, each thread
// holding kMemPer consecutive entries (their rule offsets loaded together, so
// a level costs one round of dependent loads); it stops at `level` or above
// the first level whose parse would not fit.  res[3b..3b+2] = {level
// reached, its parse length, 1 if the parse is in the second buffer}.
constexpr int kMPT = 1024;
constexpr int kMemPer = 8;
constexpr uint32_t kMemTopCap = kMPT * kMemPer;

__global__ __launch_bounds__(kMPT) void k_mem_parse_top(const LevelPtrs* __restrict__ lv_ptr,
                                                        const uint32_t* __restrict__ cent,
                                                        int level, uint32_t* __restrict__ buf0,
                                                        uint32_t* __restrict__ buf1,
                                                        uint32_t* __restrict__ res) {
  __shared__ uint64_t s_wave[kMPT / 64];
  const int top = (int)cent[2 * blockIdx.x];
  uint32_t* cur = buf0 + (uint64_t)blockIdx.x * kMemTopCap;
  uint32_t* nxt = buf1 + (uint64_t)blockIdx.x * kMemTopCap;
  if (threadIdx.x == 0) cur[0] = cent[2 * blockIdx.x + 1];
  __syncthreads();
  uint32_t n = 1;
  int l = top;
  while (l > level) {
    const LevelPtrs L = lv_ptr[l - 1];
    const uint32_t* rhs = static_cast<const uint32_t*>(L.rhs);
    const uint32_t i0 = threadIdx.x * kMemPer;
    uint64_t a[kMemPer], e[kMemPer];
    uint64_t part = 0;
#pragma unroll
    for (int r = 0; r < kMemPer; ++r) {
      a[r] = e[r] = 0;
      if (i0 + r < n) {
        const uint32_t x = cur[i0 + r];
        a[r] = L.off[x];
        e[r] = L.off[x + 1];
      }
      part += e[r] - a[r];
    }
    uint64_t tot;
    uint64_t p = block_excl_scan<uint64_t, kMPT>(part, s_wave, &tot);
    if (tot > kMemTopCap) break;  // the same total in every thread
#pragma unroll
    for (int r = 0; r < kMemPer; ++r)
      for (uint64_t t = a[r]; t < e[r]; ++t) nxt[p++] = rhs[t];
    __syncthreads();  // the new frontier is read by other threads next
    uint32_t* w = cur;
    cur = nxt;
    nxt = w;
    n = (uint32_t)tot;
    --l;
  }
  if (threadIdx.x == 0) {
    res[3 * blockIdx.x] = (uint32_t)l;
    res[3 * blockIdx.x + 1] = n;
    res[3 * blockIdx.x + 2] = cur != buf0 + (uint64_t)blockIdx.x * kMemTopCap;
  }
}

// The first and the last (up to) 8 bytes of every rule's expansion, level by
// level: head holds byte t of the expansion in bits 8t.., tail byte n-1-t in
// bits 8t.. (the last byte lowest); bytes past the expansion are zero.
__global__ __launch_bounds__(kMB) void k_mem_ends1(const uint64_t* __restrict__ off,
                                                   const uint8_t* __restrict__ rhs, uint32_t u,
                                                   uint64_t* __restrict__ head,
                                                   uint64_t* __restrict__ tail) {
  for (uint32_t r = blockIdx.x * kMB + threadIdx.x; r < u; r += gridDim.x * kMB) {
    const uint64_t a = off[r], n = off[r + 1] - a, k = n < 8 ? n : 8;
    uint64_t h = 0, t = 0;
    for (uint64_t i = 0; i < k; ++i) {
      h |= (uint64_t)rhs[a + i] << (8 * i);
      t |= (uint64_t)rhs[a + n - 1 - i] << (8 * i);
    }
    head[r] = h;
    tail[r] = t;
  }
}

// levels >= 2: from the children's ends and expansion lengths
__global__ __launch_bounds__(kMB) void k_mem_ends(const uint64_t* __restrict__ off,
                                                  const uint32_t* __restrict__ rhs, uint32_t u,
                                                  const uint64_t* __restrict__ elen_c,
                                                  const uint64_t* __restrict__ head_c,
                                                  const uint64_t* __restrict__ tail_c,
                                                  uint64_t* __restrict__ head,
                                                  uint64_t* __restrict__ tail) {
  for (uint32_t r = blockIdx.x * kMB + threadIdx.x; r < u; r += gridDim.x * kMB) {
    const uint64_t a = off[r], b = off[r + 1];
    uint64_t h = 0, t = 0;
    uint32_t got = 0;
    for (uint64_t x = a; x < b && got < 8; ++x) {
      const uint32_t c = rhs[x];
      const uint64_t k = min<uint64_t>(8 - got, elen_c[c]);
      h |= (head_c[c] & (k == 8 ? ~0ull : ((1ull << (8 * k)) - 1))) << (8 * got);
      got += (uint32_t)k;
    }
    got = 0;
    for (uint64_t x = b; x > a && got < 8; --x) {
      const uint32_t c = rhs[x - 1];
      const uint64_t k = min<uint64_t>(8 - got, elen_c[c]);
      t |= (tail_c[c] & (k == 8 ? ~0ull : ((1ull << (8 * k)) - 1))) << (8 * got);
      got += (uint32_t)k;
    }
    head[r] = h;
    tail[r] = t;
  }
}

// The common prefix (with BACK, suffix) of exp(X) and exp(Y), lengths nx and
// ny, from their 8-byte ends when it ends inside them: the count of equal
// bytes, or kNoEnd when the first min(8, nx, ny) bytes are all equal and both
// are longer than that (the cursor walk decides).
constexpr uint64_t kNoEnd = ~0ull;

__device__ __forceinline__ uint64_t ends_common(uint64_t ex, uint64_t ey, uint64_t nx,
                                                uint64_t ny) {
  const uint64_t km = min(min(nx, ny), (uint64_t)8);
  const uint64_t d = ex ^ ey;
  const uint64_t c = d ? (uint64_t)(__builtin_ctzll(d) >> 3) : 8;
  if (c < km) return c;
  return km == min(nx, ny) ? km : kNoEnd;
}

// expansion length of every symbol of the level-l parse
__global__ __launch_bounds__(kMB) void k_mem_elen(const uint64_t* __restrict__ explen_l,
                                                  const uint32_t* __restrict__ cur, uint64_t n,
                                                  uint64_t* __restrict__ e) {
  for (uint64_t i = blockIdx.x * (uint64_t)kMB + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * kMB)
    e[i] = explen_l[cur[i]];
}

// sort key (string slot, symbol) and index of every parse entry; segments
// (seg_start ascending, one per string slot seg_slot) cover [0, n)
__global__ __launch_bounds__(kMB) void k_mem_keys(const uint32_t* __restrict__ F, uint64_t n,
                                                  const uint32_t* __restrict__ seg_start,
                                                  const uint32_t* __restrict__ seg_slot,
                                                  uint32_t nseg, uint64_t* __restrict__ key,
                                                  uint32_t* __restrict__ idx) {
  for (uint64_t i = blockIdx.x * (uint64_t)kMB + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * kMB) {
    uint32_t lo = 0, hi = nseg;  // last segment starting at or before i
    while (hi - lo > 1) {
      const uint32_t m = (lo + hi) >> 1;
      if (seg_start[m] <= i) lo = m; else hi = m;
    }
    key[i] = ((uint64_t)seg_slot[lo] << 32) | F[i];
    idx[i] = (uint32_t)i;
  }
}

__device__ __forceinline__ uint32_t pair_of(const uint64_t* __restrict__ poff, uint32_t np,
                                            uint64_t t) {
  uint32_t lo = 0, hi = np;  // last pair whose entries start at or before t
  while (hi - lo > 1) {
    const uint32_t m = (lo + hi) >> 1;
    if (poff[m] <= t) lo = m; else hi = m;
  }
  return lo;
}

// For entry t (pair p, position i of a's parse): the range of b's entries
// with the same symbol in the sorted keys
__global__ __launch_bounds__(kMB) void k_mem_range(const MemPair* __restrict__ pairs,
                                                   const uint64_t* __restrict__ poff, uint32_t np,
                                                   uint64_t P, const uint32_t* __restrict__ F,
                                                   const uint64_t* __restrict__ keys, uint64_t n,
                                                   uint64_t* __restrict__ lo,
                                                   uint64_t* __restrict__ cnt) {
  for (uint64_t t = blockIdx.x * (uint64_t)kMB + threadIdx.x; t < P;
       t += (uint64_t)gridDim.x * kMB) {
    const uint32_t p = pair_of(poff, np, t);
    const MemPair& M = pairs[p];
    const uint64_t x = ((uint64_t)M.slot_b << 32) | F[M.sa + (t - poff[p])];
    uint64_t l = 0, h = n;
    while (l < h) {  // first key >= x
      const uint64_t m = (l + h) >> 1;
      if (keys[m] < x) l = m + 1; else h = m;
    }
    uint64_t r = l, h2 = n;
    while (r < h2) {  // first key > x
      const uint64_t m = (r + h2) >> 1;
      if (keys[m] <= x) r = m + 1; else h2 = m;
    }
    lo[t] = l;
    cnt[t] = r - l;
  }
}

// Anchors (i, j) that start a run on their diagonal; counted per entry, then
// written at the scanned positions.  With one string on both sides the pairs
// of a position with itself are not anchors.
template <bool WRITE>
__global__ __launch_bounds__(kMB) void k_mem_seeds(
    const MemPair* __restrict__ pairs, const uint64_t* __restrict__ poff, uint32_t np, uint64_t P,
    const uint32_t* __restrict__ F, const uint32_t* __restrict__ where,
    const uint64_t* __restrict__ lo, const uint64_t* __restrict__ cnt,
    uint64_t* __restrict__ nseed, const uint64_t* __restrict__ spos, uint32_t* __restrict__ sp,
    uint32_t* __restrict__ si, uint32_t* __restrict__ sj) {
  for (uint64_t t = blockIdx.x * (uint64_t)kMB + threadIdx.x; t < P;
       t += (uint64_t)gridDim.x * kMB) {
    const uint32_t p = pair_of(poff, np, t);
    const MemPair& M = pairs[p];
    const uint32_t i = M.sa + (uint32_t)(t - poff[p]);
    const uint64_t b = lo[t], e = b + cnt[t];
    const bool has_prev = i > M.sa;
    const uint32_t prev = has_prev ? F[i - 1] : 0;
    uint64_t c = WRITE ? spos[t] : 0;
    for (uint64_t u = b; u < e; ++u) {
      const uint32_t j = where[u];
      if (M.same && j == i) continue;
      if (has_prev && j > M.sb && F[j - 1] == prev) continue;
      if (WRITE) {
        sp[c] = p;
        si[c] = i;
        sj[c] = j;
      }
      ++c;
    }
    if (!WRITE) nseed[t] = c;
  }
}

// The match through each seed, completed as App. B completes a match found
// among symbols: forward, the equal symbols after the anchor in both parses
// (at most kMemRun of them), then the lcp of the first different pair; backward,
// the lcs of the two symbols before the anchor (they differ: the seed starts
// its run).  Those walks start at the symbols and go `level` levels deep.  Only
// when one expansion is a prefix (suffix) of the other does the match go on
// past it, and the rest comes from the walk over the whole strings.
constexpr int kMemRun = 64;

__global__ __launch_bounds__(64) void k_mem_extend(
    const LevelPtrs* __restrict__ lv_ptr, const uint64_t* const* __restrict__ explen, int level,
    const uint64_t* __restrict__ head, const uint64_t* __restrict__ tail,
    const MemPair* __restrict__ pairs, const uint32_t* __restrict__ F,
    const uint64_t* __restrict__ G, const uint32_t* __restrict__ sp,
    const uint32_t* __restrict__ si, const uint32_t* __restrict__ sj, uint64_t ns,
    uint64_t min_len, uint64_t* __restrict__ mpa, uint64_t* __restrict__ mpb,
    uint64_t* __restrict__ mlen, uint64_t* __restrict__ keep) {
  for (uint64_t q = blockIdx.x * (uint64_t)64 + threadIdx.x; q < ns;
       q += (uint64_t)gridDim.x * 64) {
    const MemPair& M = pairs[sp[q]];
    const uint64_t i = si[q], j = sj[q];
    const uint64_t x = G[i] - M.ga, y = G[j] - M.gb;
    uint64_t back = 0;
    if (i > M.sa && j > M.sb) {
      const uint64_t nx = G[i] - G[i - 1], ny = G[j] - G[j - 1];
      const uint32_t X = F[i - 1], Y = F[j - 1];
      back = ends_common(tail[X], tail[Y], nx, ny);
      if (back == kNoEnd) back = lce_walk<true>(lv_ptr, explen, level, X, nx, nx, level, Y, ny, ny);
      if (back == nx || back == ny)
        back += lce_walk<true>(lv_ptr, explen, M.ta, M.ya, x - back, M.la, M.tb, M.yb, y - back,
                               M.lb);
    }
    const uint64_t ea = (uint64_t)M.sa + M.na, eb = (uint64_t)M.sb + M.nb;
    uint64_t ii = i + 1, jj = j + 1;
    int run = 0;
    while (ii < ea && jj < eb && run < kMemRun && F[ii] == F[jj]) {
      ++ii;
      ++jj;
      ++run;
    }
    uint64_t fwd = G[ii] - G[i];
    if (ii < ea && jj < eb) {
      bool rest = run == kMemRun;
      if (!rest) {
        const uint64_t nx = G[ii + 1] - G[ii], ny = G[jj + 1] - G[jj];
        const uint32_t X = F[ii], Y = F[jj];
        uint64_t l1 = ends_common(head[X], head[Y], nx, ny);
        if (l1 == kNoEnd) l1 = lce_walk<false>(lv_ptr, explen, level, X, 0, nx, level, Y, 0, ny);
        fwd += l1;
        rest = l1 == nx || l1 == ny;
      }
      if (rest)
        fwd += lce_walk<false>(lv_ptr, explen, M.ta, M.ya, x + fwd, M.la, M.tb, M.yb, y + fwd,
                               M.lb);
    }
    mpa[q] = x - back;
    mpb[q] = y - back;
    mlen[q] = back + fwd;
    keep[q] = back + fwd >= min_len;
  }
}

// kept matches packed: (pair << 40 | start in a), start in b, length; sort
// values start as their index
__global__ __launch_bounds__(kMB) void k_mem_pack(
    const uint32_t* __restrict__ sp, const uint64_t* __restrict__ mpa,
    const uint64_t* __restrict__ mpb, const uint64_t* __restrict__ mlen,
    const uint64_t* __restrict__ keep, const uint64_t* __restrict__ kpos, uint64_t ns,
    uint64_t* __restrict__ pka, uint64_t* __restrict__ pb, uint64_t* __restrict__ ln,
    uint32_t* __restrict__ idx) {
  for (uint64_t q = blockIdx.x * (uint64_t)kMB + threadIdx.x; q < ns;
       q += (uint64_t)gridDim.x * kMB) {
    if (!keep[q]) continue;
    const uint64_t p = kpos[q];
    pka[p] = ((uint64_t)sp[q] << 40) | mpa[q];
    pb[p] = mpb[q];
    ln[p] = mlen[q];
    idx[p] = (uint32_t)p;
  }
}

__global__ __launch_bounds__(kMB) void k_mem_gather(const uint64_t* __restrict__ src,
                                                    const uint32_t* __restrict__ idx, uint64_t m,
                                                    uint64_t* __restrict__ dst) {
  for (uint64_t t = blockIdx.x * (uint64_t)kMB + threadIdx.x; t < m;
       t += (uint64_t)gridDim.x * kMB)
    dst[t] = src[idx[t]];
}

// after the sort by (pair, start in a, start in b): the first of equal matches
__global__ __launch_bounds__(kMB) void k_mem_first(const uint64_t* __restrict__ pka_s,
                                                   const uint64_t* __restrict__ pb,
                                                   const uint32_t* __restrict__ idx, uint64_t m,
                                                   uint64_t* __restrict__ flag) {
  for (uint64_t t = blockIdx.x * (uint64_t)kMB + threadIdx.x; t < m;
       t += (uint64_t)gridDim.x * kMB)
    flag[t] = t == 0 || pka_s[t] != pka_s[t - 1] || pb[idx[t]] != pb[idx[t - 1]];
}

__global__ __launch_bounds__(kMB) void k_mem_out(
    const uint64_t* __restrict__ pka_s, const uint64_t* __restrict__ pb,
    const uint64_t* __restrict__ ln, const uint32_t* __restrict__ idx,
    const uint64_t* __restrict__ flag, const uint64_t* __restrict__ fpos, uint64_t m, uint64_t cap,
    uint32_t* __restrict__ opair, uint64_t* __restrict__ opa, uint64_t* __restrict__ opb,
    uint64_t* __restrict__ olen) {
  for (uint64_t t = blockIdx.x * (uint64_t)kMB + threadIdx.x; t < m;
       t += (uint64_t)gridDim.x * kMB) {
    const uint64_t p = fpos[t];
    if (!flag[t] || p >= cap) continue;
    if (opair) opair[p] = (uint32_t)(pka_s[t] >> 40);
    opa[p] = pka_s[t] & ((1ull << 40) - 1);
    opb[p] = pb[idx[t]];
    olen[p] = ln[idx[t]];
  }
}

inline int bits_for(uint64_t v) {  // radix-sort key width that holds 0..v
  int b = 1;
  while (b < 64 && (v >> b)) ++b;
  return b;
}

// the 8-byte ends of levels 1..level, kept with the grammar until it changes
void ensure_ends(lcg_grammar* g, uint32_t level, hipStream_t s) {
  if (g->ends_version != g->version) {
    g->ends_first.clear();
    g->ends_last.clear();
    g->ends_version = g->version;
  }
  for (uint32_t l = (uint32_t)g->ends_first.size() + 1; l <= level; ++l) {
    const Level& L = g->levels[l - 1];
    DBuf<uint64_t> h, t;
    h.need(std::max<uint32_t>(L.u, 1), s);
    t.need(std::max<uint32_t>(L.u, 1), s);
    if (l == 1) {
      k_mem_ends1<<<mem_grid(L.u), kMB, 0, s>>>(L.off.p, L.rhs8.p, L.u, h.p, t.p);
    } else {
      k_mem_ends<<<mem_grid(L.u), kMB, 0, s>>>(L.off.p, L.rhs32.p, L.u, g->explen[l - 2].p,
                                              g->ends_first[l - 2].p, g->ends_last[l - 2].p, h.p,
                                              t.p);
    }
    HIP_CHECK(hipGetLastError());
    g->ends_first.push_back(std::move(h));
    g->ends_last.push_back(std::move(t));
  }
}

inline void scan_into(DBuf<uint64_t>& tmp, const uint64_t* in, uint64_t* out, uint64_t n,
                      hipStream_t s) {
  tmp.need(std::max<size_t>(scan_tmp_words(n), 1), s);
  scan_exclusive(in, out, n, tmp.p, s);
}

// The matches of the pairs (a[p], b[p]), p < np, at `level`: the first
// min(count, cap) written (pair index optional), *n_mems the count.
void mems_core(lcg_grammar* g, uint32_t np, const uint32_t* ha, const uint32_t* hb,
               uint32_t level, uint64_t min_len, uint64_t cap, uint32_t* d_pair, uint64_t* d_pa,
               uint64_t* d_pb, uint64_t* d_len, uint64_t* n_mems, hipStream_t s) {
  *n_mems = 0;
  if (!np) return;
  if (cap && (!d_pa || !d_pb || !d_len)) throw LcgError{LCG_EINVAL, "NULL output array"};
  if (!ha || !hb) throw LcgError{LCG_EINVAL, "NULL pair array"};
  if (np >= (1u << 23)) throw LcgError{LCG_EINVAL, "2^23 pairs or more in one call"};
  if (g->levels.size() >= (size_t)kMaxLv) throw LcgError{LCG_EOVERFLOW, "too many levels"};
  // the distinct strings of the batch: one parse each
  std::vector<uint32_t> strs, slot_a(np), slot_b(np);
  {
    std::unordered_map<uint32_t, uint32_t> at;
    for (uint32_t p = 0; p < np; ++p) {
      for (int side = 0; side < 2; ++side) {
        const uint32_t j = side ? hb[p] : ha[p];
        if (j >= g->k) throw LcgError{LCG_EINVAL, "string index beyond the grammar's"};
        auto it = at.find(j);
        if (it == at.end()) {
          it = at.emplace(j, (uint32_t)strs.size()).first;
          strs.push_back(j);
        }
        (side ? slot_b : slot_a)[p] = it->second;
      }
    }
  }
  const uint32_t ns_ = (uint32_t)strs.size();
  ensure_explen(g, s);
  DBuf<uint32_t> js, cent;
  js.need(ns_, s);
  cent.need(2 * (size_t)ns_, s);
  HIP_CHECK(hipMemcpyAsync(js.p, strs.data(), ns_ * 4, hipMemcpyHostToDevice, s));
  k_mem_centries<<<mem_grid(ns_), kMB, 0, s>>>(g->c_level.p, g->c_sym.p, js.p, ns_, cent.p);
  HIP_CHECK(hipGetLastError());
  std::vector<uint32_t> hc(2 * (size_t)ns_);
  HIP_CHECK(hipMemcpyAsync(hc.data(), cent.p, hc.size() * 4, hipMemcpyDeviceToHost, s));
  sync(s);
  for (uint32_t i = 0; i < ns_; ++i)
    if (level < 1 || level > hc[2 * i])
      throw LcgError{LCG_EINVAL, "level outside 1..min(level of C[a], level of C[b])"};
  // upper levels, one block per string
  DBuf<uint32_t> t0, t1, res;
  t0.need((size_t)ns_ * kMemTopCap, s);
  t1.need((size_t)ns_ * kMemTopCap, s);
  res.need(3 * (size_t)ns_, s);
  k_mem_parse_top<<<ns_, kMPT, 0, s>>>(g->level_ptrs.p, cent.p, (int)level, t0.p, t1.p, res.p);
  HIP_CHECK(hipGetLastError());
  std::vector<uint32_t> hr(3 * (size_t)ns_);
  HIP_CHECK(hipMemcpyAsync(hr.data(), res.p, hr.size() * 4, hipMemcpyDeviceToHost, s));
  sync(s);
  // the larger levels: the strings' frontiers side by side, each string
  // joining once the descent reaches the level its top parse stopped at
  std::vector<uint64_t> seg_start(ns_, 0), seg_len(ns_, 0);
  std::vector<uint32_t> order;  // strings in the array, in segment order
  DBuf<uint32_t> F, next;
  DBuf<uint64_t> cnt, pos, tmp, sidx, spos;
  uint64_t n = 0;
  int lmax = (int)level;
  for (uint32_t i = 0; i < ns_; ++i) lmax = std::max(lmax, (int)hr[3 * i]);
  auto join = [&](int l) {
    uint64_t add = 0;
    for (uint32_t i = 0; i < ns_; ++i)
      if ((int)hr[3 * i] == l) add += hr[3 * i + 1];
    if (!add) return;
    F.grow(n + add, n, s);
    for (uint32_t i = 0; i < ns_; ++i) {
      if ((int)hr[3 * i] != l) continue;
      const uint32_t* src = (hr[3 * i + 2] ? t1.p : t0.p) + (uint64_t)i * kMemTopCap;
      HIP_CHECK(hipMemcpyAsync(F.p + n, src, (size_t)hr[3 * i + 1] * 4, hipMemcpyDeviceToDevice,
                               s));
      seg_start[i] = n;
      seg_len[i] = hr[3 * i + 1];
      order.push_back(i);
      n += hr[3 * i + 1];
    }
  };
  for (int l = lmax; l > (int)level; --l) {
    join(l);
    if (!n) continue;
    const Level& L = g->levels[l - 1];
    cnt.need(n, s);
    k_mem_rhslen<<<mem_grid(n), kMB, 0, s>>>(L.off.p, F.p, n, cnt.p);
    HIP_CHECK(hipGetLastError());
    pos.need(n + 1, s);
    scan_into(tmp, cnt.p, pos.p, n, s);
    // the segments' new starts and the new length, in one read
    const uint32_t k = (uint32_t)order.size();
    std::vector<uint64_t> hs(k + 1);
    for (uint32_t q = 0; q < k; ++q) hs[q] = seg_start[order[q]];
    hs[k] = n;
    sidx.need(k + 1, s);
    spos.need(k + 1, s);
    HIP_CHECK(hipMemcpyAsync(sidx.p, hs.data(), (k + 1) * 8, hipMemcpyHostToDevice, s));
    k_mem_pick<<<mem_grid(k + 1), kMB, 0, s>>>(pos.p, sidx.p, k + 1, spos.p);
    HIP_CHECK(hipGetLastError());
    std::vector<uint64_t> hp(k + 1);
    HIP_CHECK(hipMemcpyAsync(hp.data(), spos.p, (k + 1) * 8, hipMemcpyDeviceToHost, s));
    sync(s);
    const uint64_t m = hp[k];
    if (m >= (1ull << 31)) throw LcgError{LCG_EOVERFLOW, "parses of 2^31 symbols or more"};
    next.need(m, s);
    k_mem_children<<<mem_grid(n), kMB, 0, s>>>(L.off.p, L.rhs32.p, F.p, n, pos.p, next.p);
    HIP_CHECK(hipGetLastError());
    std::swap(F, next);
    for (uint32_t q = 0; q < k; ++q) {
      seg_start[order[q]] = hp[q];
      seg_len[order[q]] = (q + 1 < k ? hp[q + 1] : m) - hp[q];
    }
    n = m;
  }
  join((int)level);
  if (n >= (1ull << 31)) throw LcgError{LCG_EOVERFLOW, "parses of 2^31 symbols or more"};
  // byte prefix of all symbols (G), the segments' byte bases and lengths
  DBuf<uint64_t> G;
  cnt.need(n, s);
  k_mem_elen<<<mem_grid(n), kMB, 0, s>>>(g->explen[level - 1].p, F.p, n, cnt.p);
  HIP_CHECK(hipGetLastError());
  G.need(n + 1, s);
  scan_into(tmp, cnt.p, G.p, n, s);
  std::vector<uint64_t> gidx(2 * (size_t)ns_);
  for (uint32_t i = 0; i < ns_; ++i) {
    gidx[2 * i] = seg_start[i];
    gidx[2 * i + 1] = seg_start[i] + seg_len[i];
  }
  sidx.need(gidx.size(), s);
  spos.need(gidx.size(), s);
  HIP_CHECK(hipMemcpyAsync(sidx.p, gidx.data(), gidx.size() * 8, hipMemcpyHostToDevice, s));
  k_mem_pick<<<mem_grid(gidx.size()), kMB, 0, s>>>(G.p, sidx.p, (uint32_t)gidx.size(), spos.p);
  HIP_CHECK(hipGetLastError());
  std::vector<uint64_t> gv(gidx.size());
  HIP_CHECK(hipMemcpyAsync(gv.data(), spos.p, gv.size() * 8, hipMemcpyDeviceToHost, s));
  // the sort of all parses by (string, symbol)
  std::vector<uint32_t> hseg(2 * (size_t)ns_);
  for (uint32_t q = 0; q < ns_; ++q) {
    hseg[q] = (uint32_t)seg_start[order[q]];
    hseg[ns_ + q] = order[q];
  }
  DBuf<uint32_t> segd, idx, where;
  DBuf<uint64_t> key, keys;
  segd.need(hseg.size(), s);
  HIP_CHECK(hipMemcpyAsync(segd.p, hseg.data(), hseg.size() * 4, hipMemcpyHostToDevice, s));
  key.need(n, s);
  keys.need(n, s);
  idx.need(n, s);
  where.need(n, s);
  k_mem_keys<<<mem_grid(n), kMB, 0, s>>>(F.p, n, segd.p, segd.p + ns_, ns_, key.p, idx.p);
  HIP_CHECK(hipGetLastError());
  const int kbits = 32 + bits_for(ns_);
  size_t tbytes = 0;
  HIP_CHECK(hipcub::DeviceRadixSort::SortPairs(nullptr, tbytes, key.p, keys.p, idx.p, where.p,
                                               (int)n, 0, kbits, s));
  DBuf<uint8_t> stmp;
  stmp.need(std::max<size_t>(tbytes, 4), s);
  HIP_CHECK(hipcub::DeviceRadixSort::SortPairs(stmp.p, tbytes, key.p, keys.p, idx.p, where.p,
                                               (int)n, 0, kbits, s));
  sync(s);  // gv, and hseg's copy, are complete
  // the pairs, and the entries of their a-side parses
  std::vector<MemPair> hp(np);
  std::vector<uint64_t> hpo(np + 1, 0);
  for (uint32_t p = 0; p < np; ++p) {
    const uint32_t A = slot_a[p], B = slot_b[p];
    MemPair& M = hp[p];
    M.ta = (int)hc[2 * A];
    M.ya = hc[2 * A + 1];
    M.tb = (int)hc[2 * B];
    M.yb = hc[2 * B + 1];
    M.sa = (uint32_t)seg_start[A];
    M.na = (uint32_t)seg_len[A];
    M.sb = (uint32_t)seg_start[B];
    M.nb = (uint32_t)seg_len[B];
    M.slot_b = B;
    M.same = A == B;
    M.ga = gv[2 * A];
    M.gb = gv[2 * B];
    M.la = gv[2 * A + 1] - gv[2 * A];
    M.lb = gv[2 * B + 1] - gv[2 * B];
    if (M.la >= (1ull << 40)) throw LcgError{LCG_EOVERFLOW, "a string of 2^40 bytes or more"};
    hpo[p + 1] = hpo[p] + M.na;
  }
  const uint64_t P = hpo[np];
  DBuf<MemPair> pairs;
  DBuf<uint64_t> poff, lo;
  pairs.need(np, s);
  poff.need(np + 1, s);
  HIP_CHECK(hipMemcpyAsync(pairs.p, hp.data(), np * sizeof(MemPair), hipMemcpyHostToDevice, s));
  HIP_CHECK(hipMemcpyAsync(poff.p, hpo.data(), (np + 1) * 8, hipMemcpyHostToDevice, s));
  lo.need(P, s);
  cnt.need(P, s);
  pos.need(P + 1, s);
  k_mem_range<<<mem_grid(P), kMB, 0, s>>>(pairs.p, poff.p, np, P, F.p, keys.p, n, lo.p, cnt.p);
  HIP_CHECK(hipGetLastError());
  scan_into(tmp, cnt.p, pos.p, P, s);
  const uint64_t anchors = read_dev(pos.p + P, s);
  if (anchors > kMemMaxAnchors)
    throw LcgError{LCG_EOVERFLOW, std::to_string(anchors) +
                                      " anchors at this level (at most 2^31): choose a higher "
                                      "level"};
  DBuf<uint64_t> nseed;
  nseed.need(P, s);
  k_mem_seeds<false><<<mem_grid(P), kMB, 0, s>>>(pairs.p, poff.p, np, P, F.p, where.p, lo.p,
                                                 cnt.p, nseed.p, nullptr, nullptr, nullptr,
                                                 nullptr);
  HIP_CHECK(hipGetLastError());
  scan_into(tmp, nseed.p, pos.p, P, s);
  const uint64_t ns = read_dev(pos.p + P, s);
  if (!ns) return;
  DBuf<uint32_t> sp, si, sj;
  sp.need(ns, s);
  si.need(ns, s);
  sj.need(ns, s);
  k_mem_seeds<true><<<mem_grid(P), kMB, 0, s>>>(pairs.p, poff.p, np, P, F.p, where.p, lo.p,
                                                cnt.p, nullptr, pos.p, sp.p, si.p, sj.p);
  HIP_CHECK(hipGetLastError());
  DBuf<uint64_t> mpa, mpb, mlen, keep, kpos;
  mpa.need(ns, s);
  mpb.need(ns, s);
  mlen.need(ns, s);
  keep.need(ns, s);
  ensure_ends(g, level, s);
  k_mem_extend<<<(unsigned)std::min<uint64_t>((ns + 63) / 64, 65536), 64, 0, s>>>(
      g->level_ptrs.p, g->explen_ptrs.p, (int)level, g->ends_first[level - 1].p,
      g->ends_last[level - 1].p, pairs.p, F.p, G.p, sp.p, si.p, sj.p, ns, min_len, mpa.p, mpb.p,
      mlen.p, keep.p);
  HIP_CHECK(hipGetLastError());
  kpos.need(ns + 1, s);
  scan_into(tmp, keep.p, kpos.p, ns, s);
  const uint64_t m = read_dev(kpos.p + ns, s);
  if (!m) return;
  // sort by (pair, start in a, start in b): by b, then stably by the rest
  DBuf<uint64_t> pka, pb, ln, k1, k2;
  DBuf<uint32_t> i0, i1, i2;
  pka.need(m, s);
  pb.need(m, s);
  ln.need(m, s);
  i0.need(m, s);
  k_mem_pack<<<mem_grid(ns), kMB, 0, s>>>(sp.p, mpa.p, mpb.p, mlen.p, keep.p, kpos.p, ns, pka.p,
                                         pb.p, ln.p, i0.p);
  HIP_CHECK(hipGetLastError());
  k1.need(m, s);
  k2.need(m, s);
  i1.need(m, s);
  i2.need(m, s);
  uint64_t lbmax = 0, lamax = 0;
  for (const MemPair& M : hp) {
    lbmax = std::max(lbmax, M.lb);
    lamax = std::max(lamax, M.la);
  }
  const int bb = bits_for(lbmax), ab = std::min(64, 40 + bits_for(np));
  size_t st1 = 0, st2 = 0;
  HIP_CHECK(hipcub::DeviceRadixSort::SortPairs(nullptr, st1, pb.p, k1.p, i0.p, i1.p, (int)m, 0,
                                               bb, s));
  HIP_CHECK(hipcub::DeviceRadixSort::SortPairs(nullptr, st2, k2.p, k1.p, i1.p, i2.p, (int)m, 0,
                                               ab, s));
  st1 = std::max(st1, st2);
  stmp.need(std::max<size_t>(st1, 4), s);
  HIP_CHECK(hipcub::DeviceRadixSort::SortPairs(stmp.p, st1, pb.p, k1.p, i0.p, i1.p, (int)m, 0,
                                               bb, s));
  k_mem_gather<<<mem_grid(m), kMB, 0, s>>>(pka.p, i1.p, m, k2.p);
  HIP_CHECK(hipGetLastError());
  HIP_CHECK(hipcub::DeviceRadixSort::SortPairs(stmp.p, st1, k2.p, k1.p, i1.p, i2.p, (int)m, 0,
                                               ab, s));
  // k1: (pair, start in a) in order, i2: the match each came from
  DBuf<uint64_t> flag, fpos;
  flag.need(m, s);
  fpos.need(m + 1, s);
  k_mem_first<<<mem_grid(m), kMB, 0, s>>>(k1.p, pb.p, i2.p, m, flag.p);
  HIP_CHECK(hipGetLastError());
  scan_into(tmp, flag.p, fpos.p, m, s);
  const uint64_t count = read_dev(fpos.p + m, s);
  if (cap) {
    k_mem_out<<<mem_grid(m), kMB, 0, s>>>(k1.p, pb.p, ln.p, i2.p, flag.p, fpos.p, m, cap, d_pair,
                                         d_pa, d_pb, d_len);
    HIP_CHECK(hipGetLastError());
  }
  sync(s);
  *n_mems = count;
}

}  // namespace
}  // namespace lcg

using namespace lcg;

extern "C" {

lcg_status lcg_extract(lcg_grammar_t g, uint32_t nq, const uint32_t* d_j, const uint64_t* d_start,
                       const uint32_t* d_len, const uint64_t* d_out_off, uint8_t* d_out,
                       hipStream_t stream) {
  return guard([&] {
    live(g);
    if (!nq) return;
    if (!d_j || !d_start || !d_len || !d_out_off || !d_out)
      throw LcgError{LCG_EINVAL, "NULL query or output array"};
    if (!g->k) throw LcgError{LCG_EINVAL, "the grammar holds no string"};
    ensure_explen(g, stream);
    DBuf<unsigned int> bad;
    bad.need(1, stream);
    launch_zero(bad.p, sizeof(unsigned int), stream);
    const unsigned wgrid = std::min<uint32_t>((nq + kXWaves - 1) / kXWaves, 8192u);
    k_extract_wave<<<wgrid, kXBlock, 0, stream>>>(g->level_ptrs.p, g->explen_ptrs.p, g->c_level.p,
                                                 g->c_sym.p, g->k, nq, d_j, d_start, d_len,
                                                 d_out_off, d_out, bad.p);
    HIP_CHECK(hipGetLastError());
    const unsigned grid = std::min<uint32_t>(nq, 4096u);
    k_extract<<<grid, kXBlock, 0, stream>>>(g->level_ptrs.p, g->explen_ptrs.p, g->c_level.p,
                                           g->c_sym.p, g->k, nq, d_j, d_start, d_len, d_out_off,
                                           d_out, bad.p);
    HIP_CHECK(hipGetLastError());
    const unsigned int nbad = read_dev(bad.p, stream);
    if (nbad)
      throw LcgError{LCG_EINVAL, std::to_string(nbad) + " quer" + (nbad == 1 ? "y" : "ies") +
                                     " out of range (string index, or start + len beyond the "
                                     "string, or len not in 1.." +
                                     std::to_string(LCG_EXTRACT_MAX) + ")"};
  });
}

lcg_status lcg_lce(lcg_grammar_t g, uint32_t nq, const uint32_t* d_j1, const uint64_t* d_p1,
                   const uint32_t* d_j2, const uint64_t* d_p2, uint32_t backward,
                   uint64_t* d_out, hipStream_t stream) {
  return guard([&] {
    live(g);
    if (backward > 1) throw LcgError{LCG_EINVAL, "backward must be 0 or 1"};
    if (!nq) return;
    if (!d_j1 || !d_p1 || !d_j2 || !d_p2 || !d_out)
      throw LcgError{LCG_EINVAL, "NULL query or output array"};
    if (!g->k) throw LcgError{LCG_EINVAL, "the grammar holds no string"};
    if (g->levels.size() >= (size_t)kMaxLv) throw LcgError{LCG_EOVERFLOW, "too many levels"};
    ensure_explen(g, stream);
    DBuf<unsigned int> bad;
    bad.need(1, stream);
    launch_zero(bad.p, sizeof(unsigned int), stream);
    const unsigned grid = std::min<uint32_t>((nq + 63) / 64, 16384u);
    if (backward)
      k_lce<true><<<grid, 64, 0, stream>>>(g->level_ptrs.p, g->explen_ptrs.p, g->c_level.p,
                                          g->c_sym.p, g->k, nq, d_j1, d_p1, d_j2, d_p2, d_out,
                                          bad.p);
    else
      k_lce<false><<<grid, 64, 0, stream>>>(g->level_ptrs.p, g->explen_ptrs.p, g->c_level.p,
                                           g->c_sym.p, g->k, nq, d_j1, d_p1, d_j2, d_p2, d_out,
                                           bad.p);
    HIP_CHECK(hipGetLastError());
    const unsigned int nbad = read_dev(bad.p, stream);
    if (nbad)
      throw LcgError{LCG_EINVAL, std::to_string(nbad) + " quer" + (nbad == 1 ? "y" : "ies") +
                                     " out of range (string index, or position beyond the "
                                     "string's end)"};
  });
}

lcg_status lcg_symbol_lce(lcg_grammar_t g, uint32_t nq, const uint8_t* d_lv1, const uint32_t* d_s1,
                          const uint8_t* d_lv2, const uint32_t* d_s2, uint32_t backward,
                          uint64_t* d_out, hipStream_t stream) {
  return guard([&] {
    live(g);
    if (backward > 1) throw LcgError{LCG_EINVAL, "backward must be 0 or 1"};
    if (!nq) return;
    if (!d_lv1 || !d_s1 || !d_lv2 || !d_s2 || !d_out)
      throw LcgError{LCG_EINVAL, "NULL query or output array"};
    if (g->levels.size() >= (size_t)kMaxLv) throw LcgError{LCG_EOVERFLOW, "too many levels"};
    ensure_explen(g, stream);
    const uint32_t h = (uint32_t)g->levels.size();
    std::vector<uint32_t> sizes(h + 1, 256);
    for (uint32_t l = 1; l <= h; ++l) sizes[l] = g->levels[l - 1].u;
    DBuf<uint32_t> lv_size;
    lv_size.need(h + 1, stream);
    HIP_CHECK(hipMemcpyAsync(lv_size.p, sizes.data(), (h + 1) * 4, hipMemcpyHostToDevice, stream));
    DBuf<unsigned int> bad;
    bad.need(1, stream);
    launch_zero(bad.p, sizeof(unsigned int), stream);
    const unsigned grid = std::min<uint32_t>((nq + 63) / 64, 16384u);
    if (backward)
      k_symbol_lce<true><<<grid, 64, 0, stream>>>(g->level_ptrs.p, g->explen_ptrs.p, lv_size.p, h,
                                                 nq, d_lv1, d_s1, d_lv2, d_s2, d_out, bad.p);
    else
      k_symbol_lce<false><<<grid, 64, 0, stream>>>(g->level_ptrs.p, g->explen_ptrs.p, lv_size.p, h,
                                                  nq, d_lv1, d_s1, d_lv2, d_s2, d_out, bad.p);
    HIP_CHECK(hipGetLastError());
    const unsigned int nbad = read_dev(bad.p, stream);  // also keeps `sizes` alive until the copy is done
    if (nbad)
      throw LcgError{LCG_EINVAL, std::to_string(nbad) + " quer" + (nbad == 1 ? "y names" : "ies name") +
                                     " no symbol (level beyond the grammar's, or rank beyond "
                                     "the level's rules)"};
  });
}

lcg_status lcg_mems(lcg_grammar_t g, uint32_t a, uint32_t b, uint32_t level, uint64_t min_len,
                    uint64_t cap, uint64_t* d_pa, uint64_t* d_pb, uint64_t* d_len,
                    uint64_t* n_mems, hipStream_t stream) {
  return guard([&] {
    live(g);
    if (!n_mems) throw LcgError{LCG_EINVAL, "n_mems is NULL"};
    mems_core(g, 1, &a, &b, level, min_len, cap, nullptr, d_pa, d_pb, d_len, n_mems, stream);
  });
}

lcg_status lcg_mems_batch(lcg_grammar_t g, uint32_t npairs, const uint32_t* a, const uint32_t* b,
                          uint32_t level, uint64_t min_len, uint64_t cap, uint32_t* d_pair,
                          uint64_t* d_pa, uint64_t* d_pb, uint64_t* d_len, uint64_t* n_mems,
                          hipStream_t stream) {
  return guard([&] {
    live(g);
    if (!n_mems) throw LcgError{LCG_EINVAL, "n_mems is NULL"};
    if (cap && !d_pair) throw LcgError{LCG_EINVAL, "NULL output array"};
    mems_core(g, npairs, a, b, level, min_len, cap, d_pair, d_pa, d_pb, d_len, n_mems, stream);
  });
}

}  // extern "C"
