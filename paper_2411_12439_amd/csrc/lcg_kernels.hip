// HIP kernels of liblcg for gfx950 (wave64).
//
// One parsing round of BuildGram (Sec. 3.3 of the paper) over the flat buffer
// of all active strings T^i runs as:
//   classify  Eq. 3 on fingerprints -> one break bit per position, count per tile
//   scan      exclusive prefix of the tile counts -> phrase index of each break
//   emit      per phrase: extent, Eq. 4 fingerprint (61-bit), dictionary key,
//             HyperLogLog sketch of the keys (sizes the dictionary)
//   insert    open-addressing dictionary, exact: short phrases carry their
//             content in the key, long phrases are compared in full
//   newflags  a phrase is new if it is the first occurrence of an uncommitted slot
//   scan      ranks (first-occurrence order) and right-hand-side offsets
//   commit    rewrite T^{i+1} with ranks, append the new rules and their F
//   segments  next-round offsets per string; strings reduced to one symbol
//             store it in C and become inactive (Sec. 3.3)
// MergeGrams (Sec. 3.6) reuses insert/newflags/scan/commit with G_b's rules
// as the phrases.
#include <hip/hip_cooperative_groups.h>

#include <mutex>
#include <stdexcept>
#include <string>
#include <unordered_map>

#include "lcg_kernels.h"

namespace lcg {

#define LCG_LAUNCH_CHECK(name)                                                        \
  do {                                                                                \
    hipError_t e_ = hipGetLastError();                                                \
    if (e_ != hipSuccess)                                                             \
      throw std::runtime_error(std::string("launch of " name ": ") + hipGetErrorString(e_)); \
  } while (0)

constexpr uint32_t kMaxProbe = 1u << 14;
constexpr unsigned kPersistentBlocks = 2048;  // grid of the grid-stride kernels (8 per CU)

// Blocks of `kernel` the device holds at once (occupancy x CUs, cached per
// kernel): the grid of a persistent kernel, so that no block waits for a
// whole other block to finish.
static unsigned resident_blocks(const void* kernel, int block) {
  static std::mutex mu;
  static std::unordered_map<const void*, unsigned> cache;
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find(kernel);
  if (it != cache.end()) return it->second;
  int dev = 0, per_cu = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    throw std::runtime_error("occupancy query failed");
  const unsigned v = (unsigned)(per_cu > 0 ? per_cu : 1) * (unsigned)(cus > 0 ? cus : 1);
  cache.emplace(kernel, v);
  return v;
}

static inline unsigned grid_for(uint64_t n, int block) {
  uint64_t g = (n + block - 1) / block;
  if (g == 0) g = 1;
  if (g > 0x7FFFFFFFULL) throw std::runtime_error("grid too large");
  return (unsigned)g;
}

// ------------------------------------------------------------------ helpers
// A relaxed atomic load of a word other threads update with atomics in the
// same kernel.  Workgroup scope: the load may be served by the CU's L1 and
// return an older value of the word, which only costs extra work where it is
// used (an empty slot word leads to the compare-and-swap, which returns the
// current word; a larger first occurrence to an atomicMin).  Being atomic,
// the load is never torn, merged with another or assumed unchanged by the
// compiler, which a plain load of a concurrently written word would allow.
template <typename T>
__device__ __forceinline__ T hint_load(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// largest j in [lo, hi] with off[j] <= x (requires off[lo] <= x)
__device__ __forceinline__ uint32_t seg_search(const uint64_t* off, uint32_t lo, uint32_t hi,
                                               uint64_t x) {
  while (lo < hi) {
    uint32_t mid = (lo + hi + 1) >> 1;
    if (off[mid] <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <bool BYTES>
__device__ __forceinline__ uint32_t fval(const RoundIn& in, const uint32_t* s_lut, uint64_t i) {
  if constexpr (BYTES) return s_lut[static_cast<const uint8_t*>(in.sym)[i]];
  else return in.fp[i];
}

// first break position in [pos, lim), or lim
__device__ __forceinline__ uint64_t next_break(const uint64_t* bits, uint64_t pos, uint64_t lim) {
  while (pos < lim) {
    uint64_t w = bits[pos >> 6] >> (pos & 63);
    if (w) {
      uint64_t r = pos + __builtin_ctzll(w);
      return r < lim ? r : lim;
    }
    pos = (pos | 63) + 1;
  }
  return lim;
}

// Exact dictionary key of a phrase sym[p .. p+q) if its content fits one
// (see lcg_device.h); such keys need no fingerprint.
template <bool BYTES>
__device__ __forceinline__ bool exact_key(const void* sym, uint64_t p, uint64_t q, uint64_t& k) {
  if constexpr (BYTES) {
    if (q > 7) return false;
    const uint8_t* s = static_cast<const uint8_t*>(sym) + p;
    k = q << 56;
    for (uint32_t x = 0; x < q; ++x) k |= (uint64_t)s[x] << (8 * x);
    return true;
  } else {
    if (q > 4) return false;
    const uint32_t* s = static_cast<const uint32_t*>(sym) + p;
    const int rb = rank_bits_for((uint32_t)q);
    uint64_t kk = 0;
    bool fits = true;
    for (uint32_t x = 0; x < q; ++x) {
      uint64_t r = s[x];
      if (rb < 32 && (r >> rb)) fits = false;
      kk = (kk << rb) | r;
    }
    k = (q << 58) | kk;
    return fits;
  }
}

// Content words of a wide key for the phrase sym[p .. p+q), if it has one
// (see lcg_device.h): 8..14 bytes at level 1, up to eight ranks above.
// *qcode and *bcode receive the length and width codes.
template <bool BYTES>
__device__ __forceinline__ bool wide_content(const void* sym, uint64_t p, uint64_t q,
                                             uint64_t& c0, uint64_t& c1, uint64_t& qcode,
                                             uint64_t& bcode) {
  c0 = 0;
  c1 = 0;
  bcode = 0;
  if constexpr (BYTES) {
    if (q < 8 || q > kWideMaxBytes) return false;
    const uint8_t* s = static_cast<const uint8_t*>(sym) + p;
#pragma unroll
    for (uint32_t x = 0; x < kWideMaxBytes; ++x) {
      const uint64_t b = x < q ? (uint64_t)s[x] : 0;
      if (x < 7) c0 |= b << (8 * x);
      else c1 |= b << (8 * (x - 7));
    }
    qcode = q - 8;
    return true;
  } else {
    if (q > kWideMaxRanks) return false;
    const uint32_t* s = static_cast<const uint32_t*>(sym) + p;
    uint32_t r[kWideMaxRanks];
    uint32_t m = 0;
#pragma unroll
    for (uint32_t x = 0; x < kWideMaxRanks; ++x) {
      r[x] = x < q ? s[x] : 0u;
      m |= r[x];
    }
    const uint32_t bc = m < (1u << 12) ? 0u : m < (1u << 16) ? 1u : m < (1u << 20) ? 2u
                      : m < (1u << 31) ? 3u : 4u;
    if (bc == 4 || q > 2 * wide_per_word(bc)) return false;
    const uint32_t b = wide_bits(bc), per = wide_per_word(bc);
#pragma unroll
    for (uint32_t x = 0; x < kWideMaxRanks; ++x) {
      if (x < q) {
        const uint32_t word = x >= per, at = word ? x - per : x;
        if (word) c1 |= (uint64_t)r[x] << (b * at);
        else c0 |= (uint64_t)r[x] << (b * at);
      }
    }
    qcode = q - 1;
    bcode = bc;
    return true;
  }
}

// Dictionary key of a phrase with fingerprint P; a wide key's content goes
// to wk[0..1].
template <bool BYTES>
__device__ __forceinline__ uint64_t make_key(const void* sym, uint64_t p, uint64_t q, uint64_t P,
                                             uint32_t key_bits, uint64_t* wk) {
  uint64_t k, c0, c1, qc, bc;
  if (key_bits == 0 && exact_key<BYTES>(sym, p, q, k)) return k;
  if (key_bits == 0 && wide_content<BYTES>(sym, p, q, c0, c1, qc, bc)) {
    wk[0] = c0;
    wk[1] = c1;
    return wide_key(qc, bc, c0, c1);
  }
  return long_key(P, key_bits);
}

// Length of a phrase from its key (exact and wide keys) or from plen (long keys).
template <bool BYTES>
__device__ __forceinline__ uint32_t key_len(uint64_t kk, const uint32_t* plen, uint64_t o) {
  if (is_wide(kk)) return wide_qcode(kk) + (BYTES ? 8u : 1u);
  if (kk & kLongTag) return plen[o];
  return BYTES ? (uint32_t)((kk >> 56) & 7) : (uint32_t)((kk >> 58) & 7);
}

// Symbol x of a wide key's content (kk: the key word, for the rank width).
template <bool BYTES>
__device__ __forceinline__ uint32_t wide_sym(uint64_t kk, uint64_t c0, uint64_t c1, uint32_t x) {
  if constexpr (BYTES) {
    return (uint32_t)((x < 7 ? c0 >> (8 * x) : c1 >> (8 * (x - 7))) & 0xFF);
  } else {
    const uint32_t bc = wide_bcode(kk), b = wide_bits(bc), per = wide_per_word(bc);
    const uint64_t w = x < per ? c0 : c1;
    const uint32_t at = x < per ? x : x - per;
    return (uint32_t)((w >> (b * at)) & ((1ull << b) - 1ull));
  }
}

// Symbol x of a phrase with an exact key.
template <bool BYTES>
__device__ __forceinline__ uint32_t key_sym(uint64_t kk, uint32_t x) {
  if constexpr (BYTES) {
    return (uint32_t)((kk >> (8 * x)) & 0xFF);
  } else {
    const uint32_t q = (uint32_t)((kk >> 58) & 7);
    const int rb = rank_bits_for(q);
    const uint64_t payload = kk & ((1ULL << 58) - 1);
    const uint64_t m = rb == 32 ? 0xFFFFFFFFULL : ((1ULL << rb) - 1);
    return (uint32_t)((payload >> (rb * (q - 1 - x))) & m);
  }
}

// ------------------------------------------------------------------ small kernels
__global__ void k_f0_lut(uint32_t* lut, uint64_t a0, uint64_t b0) {
  const uint64_t s = threadIdx.x;
  lut[s] = (uint32_t)(addmod61(mulmod61(a0, s), b0) & 0xFFFFFFFFULL);
}

void launch_f0_lut(uint32_t* lut, uint64_t a0, uint64_t b0, hipStream_t s) {
  k_f0_lut<<<1, 256, 0, s>>>(lut, a0, b0);
  LCG_LAUNCH_CHECK("f0_lut");
}

__global__ void k_fill_slots(Slot* t, uint64_t cap) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < cap;
       i += (uint64_t)gridDim.x * blockDim.x)
    t[i] = Slot{kEmpty, kNone, kNone, kEmpty, kEmpty};
}

void launch_fill_slots(Slot* t, uint64_t cap, hipStream_t s) {
  unsigned g = grid_for(cap, 256);
  if (g > 8192) g = 8192;
  k_fill_slots<<<g, 256, 0, s>>>(t, cap);
  LCG_LAUNCH_CHECK("fill_slots");
}

__global__ void k_zero(uint32_t* p, uint64_t words) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < words;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

void launch_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes % 4) throw std::runtime_error("launch_zero: size not a multiple of 4");
  uint64_t w = bytes / 4;
  if (!w) return;
  unsigned g = grid_for(w, 256);
  if (g > 4096) g = 4096;
  k_zero<<<g, 256, 0, s>>>(static_cast<uint32_t*>(p), w);
  LCG_LAUNCH_CHECK("zero");
}

// ------------------------------------------------------------------ classify
// Position l of segment [s, e) starts a phrase iff l == s (and e - s >= 2),
// or l is LMS-type (Eq. 3): F[l-1] > F[l] and the first position r > l with
// F[r] != F[l] lies inside the segment and has F[r] > F[l].  Positions of the
// trailing equal run never qualify: there r does not exist.
//
// The tile's fingerprints (one position to the left, kRightHalo to the right)
// are staged in LDS with wide loads; each thread then classifies 16
// consecutive positions from its 18-value window.
constexpr int kRightHalo = 64;
constexpr int kCStage = kTile + 1 + kRightHalo;  // staged position t0 - 1 + i ...
// ... lives at s_f[cpad(i)]: one padding word per 16 keeps the per-thread
// 16-position windows on distinct LDS banks
__device__ __forceinline__ uint32_t cpad(uint32_t i) { return i + (i >> 4); }
constexpr int kCStagePadded = kCStage + kCStage / 16 + 1;

// The first and last string each tile overlaps, and the offsets of the first
// (one thread per tile, so the binary searches over the offsets run side by
// side, not inside the tile's block).
__device__ __forceinline__ void tile_seg_range(const uint64_t* __restrict__ off, uint32_t k,
                                               uint64_t n, TileSeg* __restrict__ tile_seg,
                                               uint64_t tid, uint64_t nthreads) {
  const uint64_t tiles = (n + kTile - 1) / kTile;
  for (uint64_t t = tid; t < tiles; t += nthreads) {
    const uint64_t t0 = t * kTile;
    const uint64_t tl = (t0 + kTile < n ? t0 + kTile : n) - 1;
    const uint32_t lo = seg_search(off, 0, k - 1, t0);
    const uint32_t hi = seg_search(off, lo, k - 1, tl);
    TileSeg ts;
    ts.lo = lo;
    ts.hi = hi;
    ts.start = off[lo];
    ts.end = off[lo + 1];
    tile_seg[t] = ts;
  }
}

__global__ void k_tile_seg(const uint64_t* __restrict__ off, uint32_t k, uint64_t n,
                           const uint64_t* __restrict__ n_dev, TileSeg* __restrict__ tile_seg) {
  if (n_dev) n = *n_dev;
  tile_seg_range(off, k, n, tile_seg, blockIdx.x * (uint64_t)blockDim.x + threadIdx.x,
                 (uint64_t)gridDim.x * blockDim.x);
}

// A tile's raw input, held in registers from its load to its staging: 16
// bytes (level 1) or 16 fingerprints per thread, the left neighbour (thread
// 0) and one right-halo value (threads < kRightHalo).
template <bool BYTES>
struct TileRegs;
template <>
struct TileRegs<true> {
  uint4 v;
  uint32_t left, right;
};
template <>
struct TileRegs<false> {
  uint4 v[4];
  uint32_t left, right;
};

template <bool BYTES>
__device__ __forceinline__ uint32_t raw_at(const RoundIn& in, uint64_t i) {
  if constexpr (BYTES) return static_cast<const uint8_t*>(in.sym)[i];
  else return in.fp[i];
}

template <bool BYTES>
__device__ __forceinline__ void tile_load(const RoundIn& in, uint64_t t0, TileRegs<BYTES>& r) {
  const uint64_t lim = in.n - t0 < (uint64_t)kTile ? in.n - t0 : (uint64_t)kTile;
  if constexpr (BYTES) {
    const uint8_t* src = static_cast<const uint8_t*>(in.sym) + t0;
    const uint32_t i = threadIdx.x * 16;
    if ((reinterpret_cast<uintptr_t>(src) & 15) == 0 && i + 16 <= lim) {
      r.v = *reinterpret_cast<const uint4*>(src + i);
    } else {
      uint32_t w[4] = {0, 0, 0, 0};
      for (uint32_t x = 0; x < 16; ++x)
        if (i + x < lim) w[x >> 2] |= (uint32_t)src[i + x] << (8 * (x & 3));
      r.v = make_uint4(w[0], w[1], w[2], w[3]);
    }
  } else {
    const uint32_t* src = in.fp + t0;
    const bool al = (reinterpret_cast<uintptr_t>(src) & 15) == 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t i = threadIdx.x * 4 + k * kBlock * 4;
      if (al && i + 4 <= lim) {
        r.v[k] = *reinterpret_cast<const uint4*>(src + i);
      } else {
        uint32_t w[4] = {0, 0, 0, 0};
        for (uint32_t x = 0; x < 4; ++x)
          if (i + x < lim) w[x] = src[i + x];
        r.v[k] = make_uint4(w[0], w[1], w[2], w[3]);
      }
    }
  }
  r.left = threadIdx.x == 0 && t0 > 0 ? raw_at<BYTES>(in, t0 - 1) : 0u;
  const uint64_t p = t0 + kTile + threadIdx.x;
  r.right = threadIdx.x < kRightHalo && p < in.n ? raw_at<BYTES>(in, p) : 0u;
}

// registers -> s_f (fingerprints; bytes through the h^0 table).  Positions
// past the end get a value no decision reads (every break needs its run to
// end inside the string).
template <bool BYTES>
__device__ __forceinline__ void tile_store(const TileRegs<BYTES>& r, const uint32_t* s_lut,
                                           uint32_t* s_f) {
  if constexpr (BYTES) {
    const uint32_t i = threadIdx.x * 16;
    const uint32_t wv[4] = {r.v.x, r.v.y, r.v.z, r.v.w};
#pragma unroll
    for (int x = 0; x < 16; ++x) s_f[cpad(1 + i + x)] = s_lut[(wv[x >> 2] >> (8 * (x & 3))) & 0xFF];
    if (threadIdx.x == 0) s_f[0] = s_lut[r.left & 0xFF];
    if (threadIdx.x < kRightHalo) s_f[cpad(1 + kTile + threadIdx.x)] = s_lut[r.right & 0xFF];
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t i = threadIdx.x * 4 + k * kBlock * 4;
      s_f[cpad(1 + i)] = r.v[k].x;
      s_f[cpad(2 + i)] = r.v[k].y;
      s_f[cpad(3 + i)] = r.v[k].z;
      s_f[cpad(4 + i)] = r.v[k].w;
    }
    if (threadIdx.x == 0) s_f[0] = r.left;
    if (threadIdx.x < kRightHalo) s_f[cpad(1 + kTile + threadIdx.x)] = r.right;
  }
}

// For the 16 positions b .. b+15 of a thread's window when b-1 .. b+16 lie
// inside one string ending at s_end and hold no string start: bit x set iff
// the first position r > b+x with F[r] != F[b+x] exists in the string and has
// F[r] > F[b+x].  S(x) = G(x) | (E(x) & S(x+1)) with G = change to a larger
// value and E = equal neighbour is a carry chain running from high x to low
// x, i.e. the carries of an addition on the bit-reversed masks; positions
// whose equal run reaches past the window take the value found by walking
// the run (LDS, then memory), fl being its value.  Only positions in `desc`
// (F[l-1] > F[l]) use it, so the walk is skipped when none of them needs it.
template <bool BYTES>
__device__ __forceinline__ uint32_t window_first_change(uint32_t desc, uint32_t eq, uint32_t gt,
                                                        uint32_t fl, uint64_t b, uint64_t t0,
                                                        uint64_t s_end, const RoundIn& in,
                                                        const uint32_t* s_lut, const uint32_t* s_f) {
  const uint32_t full = (1u << kItems) - 1u;
  const uint32_t ne = ~eq & full;
  const uint32_t G = ne & gt;
  const uint32_t gr = __builtin_bitreverse32(G) >> (32 - kItems);
  const uint32_t pr = __builtin_bitreverse32(eq & full) >> (32 - kItems);
  const uint32_t A = gr | pr, B = gr;
  const uint32_t carries = ((A + B) ^ A ^ B) >> 1;  // carry out of reversed bit i
  uint32_t S = __builtin_bitreverse32(carries & full) >> (32 - kItems);
  // positions whose equal run reaches the end of the window
  const uint32_t tail = ne ? ~((2u << (31 - __builtin_clz(ne))) - 1u) & full : full;
  if (desc & tail) {
    uint64_t r = b + kItems + 1;
    uint32_t fr = 0;
    bool more = true;
    while (more && r < s_end) {
      const uint64_t i = r - t0 + 1;
      fr = i < (uint64_t)kCStage ? s_f[cpad((uint32_t)i)] : fval<BYTES>(in, s_lut, r);
      more = fr == fl;
      r += more ? 1 : 0;
    }
    if (r < s_end && fr > fl) S |= tail;
  }
  return S;
}

// One tile per block.  The tile's input, its entry of the tile map and the
// h^0 table are all requested before the first barrier, so the block waits
// for memory once; the map brings the offsets of the tile's first string.
// (A resident-sized grid looping over tiles measured slower: the loop form
// needs 92-116 VGPRs, half the occupancy.)
// LDS of one classified tile.
struct ClassifyLds {
  uint32_t s_lut[256];
  uint32_t s_f[kCStagePadded];
  uint32_t s_mask[kBlock];
  uint32_t s_cnt;
};

// Break bits and break count of one tile (the whole block; returns at once,
// for every thread, past the end of the sequence).
template <bool BYTES>
__device__ __forceinline__ void classify_tile(const RoundIn& in, uint64_t tile,
                                              uint64_t* __restrict__ bits,
                                              uint64_t* __restrict__ tile_cnt,
                                              const TileSeg* __restrict__ tile_seg,
                                              ClassifyLds& sh) {
  const uint64_t t0 = tile * kTile;
  if (t0 >= in.n) return;
  uint32_t* const s_lut = sh.s_lut;
  uint32_t* const s_f = sh.s_f;
  uint32_t* const s_mask = sh.s_mask;
  uint32_t& s_cnt = sh.s_cnt;
  TileRegs<BYTES> regs;
  tile_load<BYTES>(in, t0, regs);
  const TileSeg ts = tile_seg[tile];
  if constexpr (BYTES) s_lut[threadIdx.x] = in.lut[threadIdx.x];
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  tile_store<BYTES>(regs, s_lut, s_f);
  __syncthreads();
  // A tile whose windows (one position to the left, one past the tile to the
  // right) lie inside one string takes the branch-free path in every thread:
  // a block-uniform test, so the block runs that path alone, without the
  // per-thread string checks and their branches.
  const bool interior = ts.lo == ts.hi && ts.start < t0 && t0 + kTile < ts.end;
  if (interior) {
    const uint64_t b = t0 + (uint64_t)threadIdx.x * kItems;
    uint32_t fw[kItems + 2];
#pragma unroll
    for (int x = 0; x < kItems + 2; ++x) fw[x] = s_f[cpad(threadIdx.x * kItems + x)];  // position b - 1 + x
    uint32_t desc = 0, eq = 0, gt = 0;
#pragma unroll
    for (int x = 0; x < kItems; ++x) {
      desc |= (uint32_t)(fw[x] > fw[x + 1]) << x;
      eq |= (uint32_t)(fw[x + 1] == fw[x + 2]) << x;
      gt |= (uint32_t)(fw[x + 2] > fw[x + 1]) << x;
    }
    const uint32_t mask = desc & window_first_change<BYTES>(desc, eq, gt, fw[kItems + 1], b, t0,
                                                            ts.end, in, s_lut, s_f);
    s_mask[threadIdx.x] = mask;
    const uint32_t c = (uint32_t)wave_sum((unsigned long long)__builtin_popcount(mask));
    if ((threadIdx.x & 63) == 0) atomicAdd(&s_cnt, c);
  } else {
    const uint64_t b = t0 + (uint64_t)threadIdx.x * kItems;
    uint32_t mask = 0;
    if (b < in.n) {
      uint32_t fw[kItems + 2];
#pragma unroll
      for (int x = 0; x < kItems + 2; ++x) fw[x] = s_f[cpad(threadIdx.x * kItems + x)];  // position b - 1 + x
      uint32_t desc = 0, eq = 0, gt = 0;
#pragma unroll
      for (int x = 0; x < kItems; ++x) {
        desc |= (uint32_t)(fw[x] > fw[x + 1]) << x;       // F[l-1] > F[l]
        eq |= (uint32_t)(fw[x + 1] == fw[x + 2]) << x;    // F[l] == F[l+1]
        gt |= (uint32_t)(fw[x + 2] > fw[x + 1]) << x;     // F[l+1] > F[l]
      }
      uint32_t j = ts.lo;
      uint64_t s_start = ts.start, s_end = ts.end;
      if (ts.hi != ts.lo) {
        j = seg_search(in.off, ts.lo, ts.hi, b);
        s_start = in.off[j];
        s_end = in.off[j + 1];
      }
      const int xe = in.n - b < (uint64_t)kItems ? (int)(in.n - b) : kItems;
      if (s_start < b && b + kItems < s_end) {
        mask = desc & window_first_change<BYTES>(desc, eq, gt, fw[kItems + 1], b, t0, s_end, in,
                                                 s_lut, s_f);
      } else {
      for (int x = 0; x < xe; ++x) {
        const uint64_t l = b + x;
        while (l >= s_end) {
          ++j;
          s_start = in.off[j];
          s_end = in.off[j + 1];
        }
        bool brk = false;
        if (l == s_start) {
          brk = s_end - s_start >= 2;
        } else if ((desc >> x) & 1u) {
          uint32_t ne = (~eq >> x) & ((1u << (kItems - x)) - 1u);
          if (ne) {
            uint32_t y = __builtin_ctz(ne);
            uint64_t r = l + y + 1;
            brk = r < s_end && ((gt >> (x + y)) & 1u);
          } else {
            // the run continues past the window: walk it (LDS, then memory)
            // F[l] .. F[b + kItems] are all equal, the last one is fw[kItems + 1]
            const uint32_t fl = fw[kItems + 1];
            uint64_t r = b + kItems + 1;
            uint32_t fr = 0;
            bool more = true;
            while (more && r < s_end) {
              const uint64_t i = r - t0 + 1;
              fr = i < (uint64_t)kCStage ? s_f[cpad((uint32_t)i)] : fval<BYTES>(in, s_lut, r);
              more = fr == fl;
              r += more ? 1 : 0;
            }
            brk = r < s_end && fr > fl;
          }
        }
        mask |= (uint32_t)brk << x;
      }
      }
    }
    s_mask[threadIdx.x] = mask;
    atomicAdd(&s_cnt, (uint32_t)__builtin_popcount(mask));
  }
  __syncthreads();
  if (threadIdx.x < kTileWords) {
    const int t = threadIdx.x * 4;
    uint64_t w = (uint64_t)s_mask[t] | ((uint64_t)s_mask[t + 1] << 16) |
                 ((uint64_t)s_mask[t + 2] << 32) | ((uint64_t)s_mask[t + 3] << 48);
    bits[tile * kTileWords + threadIdx.x] = w;
  }
  if (threadIdx.x == 0) tile_cnt[tile] = s_cnt;
}

template <bool BYTES>
__global__ __launch_bounds__(kBlock) void k_classify(RoundIn in0, uint64_t* __restrict__ bits,
                                                     uint64_t* __restrict__ tile_cnt,
                                                     const TileSeg* __restrict__ tile_seg) {
  __shared__ ClassifyLds sh;
  RoundIn in = in0;
  if (in0.n_dev) in.n = *in0.n_dev;  // launched over a bound; the size is on the device
  classify_tile<BYTES>(in, blockIdx.x, bits, tile_cnt, tile_seg, sh);
}

void launch_classify(const RoundIn& in, uint64_t* bits, uint64_t* tile_cnt, TileSeg* tile_seg,
                     hipStream_t s) {
  static_assert(kItems == 16 && kBlock == 256, "bit packing assumes 16 positions per thread");
  unsigned tiles = grid_for(in.n, kTile);  // in.n: the size, or its bound when in.n_dev is set
  k_tile_seg<<<grid_for(tiles, 256), 256, 0, s>>>(in.off, in.k, in.n, in.n_dev, tile_seg);
  LCG_LAUNCH_CHECK("tile_seg");
  if (in.bytes) k_classify<true><<<tiles, kBlock, 0, s>>>(in, bits, tile_cnt, tile_seg);
  else k_classify<false><<<tiles, kBlock, 0, s>>>(in, bits, tile_cnt, tile_seg);
  LCG_LAUNCH_CHECK("classify");
}

// ------------------------------------------------------------------ emit
// Phrase-parallel within a tile: the block lists the tile's break positions in
// LDS (block scan of the per-thread bit counts), stages the tile and a halo
// of the input (bytes, or ranks and fingerprints) in LDS with wide loads,
// then thread j handles the j-th phrase of the tile.  A phrase ends at the
// next break or at the end of its string, whichever comes first; positions
// past the halo are read from global memory.
constexpr int kSegCache = 128;
constexpr int kHalo = 512;
constexpr int kStage = kTile + kHalo;

template <bool BYTES>
struct EmitStage;
template <>
struct EmitStage<true> {
  alignas(16) uint8_t sym[kStage + 16];  // 16 spare bytes: word reads past the last phrase
};
template <>
struct EmitStage<false> {
  uint32_t sym[kStage + 4];  // 4 spare words: fixed-length reads past the last phrase
};

template <bool BYTES>
__device__ __forceinline__ void stage_tile(const RoundIn& in, uint64_t t0, EmitStage<BYTES>& st) {
  const uint64_t lim = in.n - t0 < (uint64_t)kStage ? in.n - t0 : (uint64_t)kStage;
  if constexpr (BYTES) {
    const uint8_t* src = static_cast<const uint8_t*>(in.sym) + t0;
    if ((reinterpret_cast<uintptr_t>(src) & 15) == 0) {
      for (uint32_t i = threadIdx.x * 16; i < kStage; i += kBlock * 16) {
        if (i + 16 <= lim) {
          *reinterpret_cast<uint4*>(&st.sym[i]) = *reinterpret_cast<const uint4*>(src + i);
        } else {
          for (uint32_t x = i; x < i + 16 && x < lim; ++x) st.sym[x] = src[x];
        }
      }
    } else {
      for (uint32_t i = threadIdx.x; i < lim; i += kBlock) st.sym[i] = src[i];
    }
  } else {
    const uint32_t* ss = static_cast<const uint32_t*>(in.sym) + t0;
    if ((reinterpret_cast<uintptr_t>(ss) & 15) == 0) {
      for (uint32_t i = threadIdx.x * 4; i < kStage; i += kBlock * 4) {
        if (i + 4 <= lim) {
          *reinterpret_cast<uint4*>(&st.sym[i]) = *reinterpret_cast<const uint4*>(ss + i);
        } else {
          for (uint32_t x = i; x < i + 4 && x < lim; ++x) st.sym[x] = ss[x];
        }
      }
    } else {
      for (uint32_t i = threadIdx.x; i < lim; i += kBlock) st.sym[i] = ss[i];
    }
  }
}

// Kinds of key a phrase gets in the emit pass.
constexpr int kKeyExact = 0;  // short exact key
constexpr int kKeyWide = 1;   // wide exact key, content in c0, c1
constexpr int kKeyLong = 2;   // fingerprint key (or a phrase left to the general path)

// Content key of a staged phrase of q bytes at tile offset p (the same key as
// exact_key / wide_content build from memory): the 16 bytes from p are read
// as five aligned LDS words and byte-aligned, and the exact and wide cases
// differ only in masks, so that the lanes of a wave stay together.  Phrases
// longer than a wide key report kKeyLong.  Reads reach at most 19 bytes past
// the word holding p, inside the staged window's spare bytes.
__device__ __forceinline__ int staged_key(const uint8_t* sym, uint32_t p, uint64_t q, uint64_t& kk,
                                          uint64_t& c0, uint64_t& c1, uint64_t& qc, uint64_t& bc) {
  bc = 0;
  if (q > kWideMaxBytes) return kKeyLong;
  const uint32_t* w = reinterpret_cast<const uint32_t*>(sym) + (p >> 2);
  const uint32_t a0 = w[0], a1 = w[1], a2 = w[2], a3 = w[3], a4 = w[4];
  const uint32_t sh = p & 3u;
  const uint64_t lo = (uint64_t)__builtin_amdgcn_alignbyte(a1, a0, sh) |
                      ((uint64_t)__builtin_amdgcn_alignbyte(a2, a1, sh) << 32);
  const uint64_t hi = (uint64_t)__builtin_amdgcn_alignbyte(a3, a2, sh) |
                      ((uint64_t)__builtin_amdgcn_alignbyte(a4, a3, sh) << 32);
  const uint32_t qq = (uint32_t)q;
  if (qq <= 7) {
    kk = (lo & ((1ull << (8 * qq)) - 1ull)) | ((uint64_t)qq << 56);
    return kKeyExact;
  }
  c0 = lo & 0x00FFFFFFFFFFFFFFull;
  c1 = ((lo >> 56) | (hi << 8)) & ((1ull << (8 * (qq - 7))) - 1ull);
  qc = qq - 8;
  kk = wide_key(qc, 0, c0, c1);
  return kKeyWide;
}

// Content key of a staged phrase of q ranks at tile offset p: the ranks are
// read once (predicated on q, so nothing past the staged window's spare words)
// and give the exact key if they fit one, else the wide key, else kKeyLong.
// The same keys as exact_key / wide_content.
__device__ __forceinline__ int staged_key(const uint32_t* sym, uint32_t p, uint64_t q,
                                          uint64_t& kk, uint64_t& c0, uint64_t& c1, uint64_t& qc,
                                          uint64_t& bc) {
  if (q > kWideMaxRanks) return kKeyLong;
  uint32_t r[kWideMaxRanks];
  uint32_t m = 0;
#pragma unroll
  for (uint32_t x = 0; x < kWideMaxRanks; ++x) {
    r[x] = x < q ? sym[p + x] : 0u;
    m |= r[x];
  }
  const uint32_t qq = (uint32_t)q;
  const int rb = rank_bits_for(qq);
  if (qq <= 4 && (rb >= 32 || (m >> rb) == 0)) {
    uint64_t f = 0;
#pragma unroll
    for (uint32_t x = 0; x < 4; ++x) f = x < qq ? (f << rb) | r[x] : f;
    kk = ((uint64_t)qq << 58) | f;
    return kKeyExact;
  }
  const uint32_t b = m < (1u << 12) ? 0u : m < (1u << 16) ? 1u : m < (1u << 20) ? 2u
                   : m < (1u << 31) ? 3u : 4u;
  if (b == 4 || qq > 2 * wide_per_word(b)) return kKeyLong;
  const uint32_t bits = wide_bits(b), per = wide_per_word(b);
  c0 = 0;
  c1 = 0;
#pragma unroll
  for (uint32_t x = 0; x < kWideMaxRanks; ++x) {
    const bool second = x >= per;
    const uint64_t v = x < qq ? (uint64_t)r[x] << (bits * (second ? x - per : x)) : 0;
    if (second) c1 |= v;
    else c0 |= v;
  }
  qc = qq - 1;
  bc = b;
  kk = wide_key(qc, bc, c0, c1);
  return kKeyWide;
}

// End of the phrase starting at tile offset s_start[jj]: the next break in
// the tile, else the next break after it, but never past its string's end.
__device__ __forceinline__ uint64_t phrase_end(uint32_t jj, uint32_t c, uint64_t t0,
                                               const uint16_t* s_start, uint32_t slo, uint32_t shi,
                                               bool cached, const uint64_t* s_off,
                                               const uint64_t* off, const uint64_t* bits) {
  const uint64_t l = t0 + s_start[jj];
  uint64_t s_end;
  if (slo == shi) {
    s_end = cached ? s_off[1] : off[slo + 1];
  } else if (cached) {
    uint32_t lo = 0, hi = shi - slo;  // largest i with s_off[i] <= l
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (s_off[mid] <= l) lo = mid; else hi = mid - 1;
    }
    s_end = s_off[lo + 1];
  } else {
    s_end = off[seg_search(off, slo, shi, l) + 1];
  }
  uint64_t e = jj + 1 < c ? t0 + s_start[jj + 1] : next_break(bits, l + 1, s_end);
  return e > s_end ? s_end : e;
}

// The word a wide key's content enters the sketch as (a fold of both
// content words and the codes; hll_add mixes it).
__device__ __forceinline__ uint64_t wide_hll_word(uint64_t c0, uint64_t c1, uint64_t qc,
                                                  uint64_t bc) {
  return c0 ^ ((c1 << 29) | (c1 >> 35)) ^ (qc << 59) ^ (bc << 62) ^ 0x5bd1e9955bd1e995ULL;
}

// One key into the block's HyperLogLog registers (32-bit mix of the key:
// enough for a sizing estimate; one 32x32+64-bit multiply-add folds the two
// halves, one multiply and shifts mix the result).
__device__ __forceinline__ void hll_add(uint32_t* s_hll, uint64_t kk) {
  const uint64_t t = (uint64_t)(uint32_t)kk * 0x9E3779B1u + (kk >> 32);
  uint32_t h = (uint32_t)(t >> 32) ^ (uint32_t)t;
  h ^= h >> 16;
  h *= 0x7FEB352Du;
  h ^= h >> 15;
  const uint32_t idx = h >> (32 - kHllLog2);
  const uint32_t rest = h << kHllLog2;
  const uint32_t rho = rest ? (uint32_t)__builtin_clz(rest) + 1 : 32 - kHllLog2 + 1;
  if (s_hll[idx] < rho) atomicMax(&s_hll[idx], rho);  // frequent keys: a read, no atomic
}

// Eq. 4 of the phrase [l, e) by Horner's rule from the right:
// P = a * sum_j F[Q_j] c^(j-1) + b (mod p).  At level 1 the staged part of
// the tile is read from LDS (F through the h^0 table), the rest from memory;
// above it F is read from memory (only the long phrases need it, so the emit
// pass does not stage it).
template <bool BYTES>
__device__ __forceinline__ uint64_t phrase_fp(const RoundIn& in, const uint32_t* s_lut,
                                              const EmitStage<BYTES>& st, uint64_t t0, uint64_t l,
                                              uint64_t e, LevelHash h) {
  uint64_t S = 0;
  if constexpr (BYTES) {
    const uint64_t e_st = e < t0 + kStage ? e : t0 + kStage;  // staged part [l, e_st)
    for (uint64_t p = e; p > e_st;) {
      --p;
      S = addmod61(mulmod61(S, h.c), fval<BYTES>(in, s_lut, p));
    }
    for (uint64_t p = e_st; p > l;) {
      --p;
      S = addmod61(mulmod61(S, h.c), s_lut[st.sym[p - t0]]);
    }
  } else {
    for (uint64_t p = e; p > l;) {
      --p;
      S = addmod61(mulmod61(S, h.c), in.fp[p]);
    }
  }
  return addmod61(mulmod61(h.a, S), h.b);
}

// Key of the phrase [l, e) from memory, with its fingerprint when it needs
// one (long phrases): the general path of the emit pass, for phrases not
// keyed from the staged window.
template <bool BYTES>
__device__ __forceinline__ void emit_general(const RoundIn& in, const uint32_t* s_lut,
                                             const EmitStage<BYTES>& st, uint64_t t0, uint64_t l,
                                             uint64_t e, uint64_t o, LevelHash h,
                                             uint32_t key_bits, uint64_t* __restrict__ pstart,
                                             uint32_t* __restrict__ plen,
                                             uint64_t* __restrict__ key,
                                             uint64_t* __restrict__ wkey,
                                             uint32_t* __restrict__ fnew, uint32_t* s_hll) {
  const uint64_t q = e - l;
  uint64_t kk, c0, c1, qc, bc;
  if (key_bits == 0 && exact_key<BYTES>(in.sym, l, q, kk)) {
    key[o] = kk;
    hll_add(s_hll, kk);
  } else if (key_bits == 0 && wide_content<BYTES>(in.sym, l, q, c0, c1, qc, bc)) {
    key[o] = wide_key(qc, bc, c0, c1);
    wkey[2 * o] = c0;
    wkey[2 * o + 1] = c1;
    hll_add(s_hll, wide_hll_word(c0, c1, qc, bc));
  } else {
    const uint64_t P = phrase_fp<BYTES>(in, s_lut, st, t0, l, e, h);
    kk = long_key(P, key_bits);
    pstart[o] = l;
    plen[o] = (uint32_t)q;
    fnew[o] = (uint32_t)(P & 0xFFFFFFFFULL);
    key[o] = kk;
    hll_add(s_hll, kk);
  }
}

constexpr uint32_t kLongList = 2048;  // long phrases deferred per tile; more are done inline

// LDS of the emit pass.
template <bool BYTES>
struct EmitLds {
  uint32_t s_lut[256];
  uint16_t s_start[kTile];
  uint16_t s_long[kLongList];
  uint64_t s_off[kSegCache + 1];
  uint32_t s_seg[2];
  uint32_t s_wave[kBlock / 64];
  uint32_t s_nlong;
  uint32_t s_hll[kHll];
  EmitStage<BYTES> st;
};

// Phrases of tiles block, block + blocks, ... (the whole block); the block's
// HyperLogLog registers go to hll_part row `block` when hll_part is given.
template <bool BYTES>
__device__ __forceinline__ void emit_tiles(const RoundIn& in, uint64_t tiles, uint64_t block,
                                           uint64_t blocks, const uint64_t* __restrict__ bits,
                                           const uint64_t* __restrict__ tile_base,
                                           const TileSeg* __restrict__ tile_seg, LevelHash h,
                                           uint32_t key_bits, uint64_t* __restrict__ pstart,
                                           uint32_t* __restrict__ plen, uint64_t* __restrict__ key,
                                           uint64_t* __restrict__ wkey, uint32_t* __restrict__ fnew,
                                           uint8_t* __restrict__ hll_part, EmitLds<BYTES>& sh) {
  uint32_t* const s_lut = sh.s_lut;
  uint16_t* const s_start = sh.s_start;
  uint16_t* const s_long = sh.s_long;
  uint64_t* const s_off = sh.s_off;
  uint32_t* const s_seg = sh.s_seg;
  uint32_t* const s_wave = sh.s_wave;
  uint32_t& s_nlong = sh.s_nlong;
  uint32_t* const s_hll = sh.s_hll;
  EmitStage<BYTES>& st = sh.st;
  if constexpr (BYTES) s_lut[threadIdx.x] = in.lut[threadIdx.x];
  for (int i = threadIdx.x; i < kHll; i += kBlock) s_hll[i] = 0;
  for (uint64_t tile = block; tile < tiles; tile += blocks) {
    const uint64_t t0 = tile * kTile;
    __syncthreads();
    if (threadIdx.x == 0) {
      const TileSeg r = tile_seg[tile];
      s_seg[0] = r.lo;
      s_seg[1] = r.hi;
      s_nlong = 0;
      if (r.lo == r.hi) {  // one string: its offsets come with the map
        s_off[0] = r.start;
        s_off[1] = r.end;
      }
    }
    const uint64_t base = tile_base[tile];  // requested with the tile, used after the scan
    stage_tile<BYTES>(in, t0, st);
    uint32_t mask = (uint32_t)(bits[tile * kTileWords + threadIdx.x / 4] >> ((threadIdx.x & 3) * 16)) &
                    0xFFFFu;
    uint32_t c = 0;
    uint32_t excl = block_excl_scan<uint32_t>((uint32_t)__builtin_popcount(mask), s_wave, &c);
    while (mask) {
      const int x = __builtin_ctz(mask);
      mask &= mask - 1;
      s_start[excl++] = (uint16_t)(threadIdx.x * kItems + x);
    }
    const uint32_t slo = s_seg[0], shi = s_seg[1];
    const bool cached = shi - slo + 2 <= kSegCache + 1;
    if (cached && shi != slo)
      for (uint32_t i = threadIdx.x; i < shi - slo + 2; i += kBlock) s_off[i] = in.off[slo + i];
    __syncthreads();
    // Phrases that end inside the staged window and whose content fits an
    // exact or wide key are keyed from the window (no fingerprint: it is
    // computed once per new rule when the rule is stored).  The others (long
    // phrases, keyed by their fingerprint and compared in full, and phrases
    // running past the window) are listed and done in a second pass with full
    // waves, instead of idling the lanes of every wave that holds one.  In a
    // tile inside one string every phrase but the last ends at the next break
    // of the tile.
    const bool single = slo == shi;
    for (uint32_t jj = threadIdx.x; jj < c; jj += kBlock) {
      const uint32_t p = s_start[jj];
      const uint64_t l = t0 + p;
      const uint64_t e = single && jj + 1 < c
                             ? t0 + s_start[jj + 1]
                             : phrase_end(jj, c, t0, s_start, slo, shi, cached, s_off, in.off, bits);
      const uint64_t o = base + jj;
      uint64_t kk = 0, c0 = 0, c1 = 0, qc = 0, bc = 0;
      const int kind = key_bits == 0 && e <= t0 + kStage
                           ? staged_key(st.sym, p, e - l, kk, c0, c1, qc, bc)
                           : kKeyLong;
      if (kind != kKeyLong) {
        key[o] = kk;
        if (kind == kKeyWide) {
          wkey[2 * o] = c0;
          wkey[2 * o + 1] = c1;
          kk = wide_hll_word(c0, c1, qc, bc);
        }
        hll_add(s_hll, kk);
      } else {
        const uint32_t slot = atomicAdd(&s_nlong, 1u);
        if (slot < kLongList)
          s_long[slot] = (uint16_t)jj;
        else
          emit_general<BYTES>(in, s_lut, st, t0, l, e, o, h, key_bits, pstart, plen, key, wkey,
                              fnew, s_hll);
      }
    }
    __syncthreads();
    const uint32_t nlong = s_nlong < kLongList ? s_nlong : kLongList;
    for (uint32_t i = threadIdx.x; i < nlong; i += kBlock) {
      const uint32_t jj = s_long[i];
      const uint64_t l = t0 + s_start[jj];
      const uint64_t e = phrase_end(jj, c, t0, s_start, slo, shi, cached, s_off, in.off, bits);
      emit_general<BYTES>(in, s_lut, st, t0, l, e, base + jj, h, key_bits, pstart, plen, key, wkey,
                          fnew, s_hll);
    }
  }
  __syncthreads();
  if (hll_part)
    for (int i = threadIdx.x; i < kHll; i += kBlock)
      hll_part[block * kHll + i] = (uint8_t)s_hll[i];
}

template <bool BYTES>
__global__ __launch_bounds__(kBlock) void k_emit(RoundIn in0, const uint64_t* __restrict__ bits,
                                                 const uint64_t* __restrict__ tile_base,
                                                 const TileSeg* __restrict__ tile_seg, uint64_t tiles,
                                                 LevelHash h, uint32_t key_bits,
                                                 uint64_t* __restrict__ pstart, uint32_t* __restrict__ plen,
                                                 uint64_t* __restrict__ key, uint64_t* __restrict__ wkey,
                                                 uint32_t* __restrict__ fnew,
                                                 uint8_t* __restrict__ hll_part) {
  __shared__ EmitLds<BYTES> sh;
  RoundIn in = in0;
  if (in0.n_dev) {  // launched over a bound; the size is on the device
    in.n = *in0.n_dev;
    tiles = (in.n + kTile - 1) / kTile;
  }
  emit_tiles<BYTES>(in, tiles, blockIdx.x, gridDim.x, bits, tile_base, tile_seg, h, key_bits,
                    pstart, plen, key, wkey, fnew, hll_part, sh);
}

// register-wise maximum of the per-block HyperLogLog sketches: block i
// reduces register i over all rows
__global__ __launch_bounds__(256) void k_hll_reduce(const uint8_t* __restrict__ part,
                                                    unsigned blocks, Counters* __restrict__ ctr) {
  __shared__ uint32_t s_max;
  const uint32_t i = blockIdx.x;
  if (threadIdx.x == 0) s_max = 0;
  __syncthreads();
  uint32_t m = 0;
  for (unsigned b = threadIdx.x; b < blocks; b += blockDim.x) {
    const uint32_t v = part[(uint64_t)b * kHll + i];
    m = v > m ? v : m;
  }
  if (m) atomicMax(&s_max, m);
  __syncthreads();
  if (threadIdx.x == 0) ctr->hll[i] = s_max;
}

void launch_emit(const RoundIn& in, const uint64_t* bits, const uint64_t* tile_base,
                 const TileSeg* tile_seg, LevelHash h,
                 uint32_t key_bits, uint64_t* pstart, uint32_t* plen, uint64_t* key, uint64_t* wkey,
                 uint32_t* fnew, uint8_t* hll_part, Counters* ctr, hipStream_t s) {
  uint64_t tiles = grid_for(in.n, kTile);
  unsigned g = resident_blocks(in.bytes ? (const void*)k_emit<true> : (const void*)k_emit<false>, kBlock);
  if (g > kEmitBlocks) g = kEmitBlocks;  // rows of hll_part
  if (g > tiles) g = (unsigned)tiles;
  if (in.bytes)
    k_emit<true><<<g, kBlock, 0, s>>>(in, bits, tile_base, tile_seg, tiles, h, key_bits, pstart, plen, key,
                                      wkey, fnew, hll_part);
  else
    k_emit<false><<<g, kBlock, 0, s>>>(in, bits, tile_base, tile_seg, tiles, h, key_bits, pstart, plen, key,
                                       wkey, fnew, hll_part);
  LCG_LAUNCH_CHECK("emit");
  if (ctr) {
    k_hll_reduce<<<kHll, 256, 0, s>>>(hll_part, g, ctr);
    LCG_LAUNCH_CHECK("hll_reduce");
  }
}

// ------------------------------------------------------------------ scan
constexpr int kScanItems = 4;
constexpr int kScanPer = kBlock * kScanItems;

__global__ __launch_bounds__(kBlock) void k_scan_block(const uint64_t* __restrict__ in,
                                                       uint64_t* __restrict__ out, uint64_t n,
                                                       uint64_t* __restrict__ block_sums) {
  __shared__ uint64_t s_wave[kBlock / 64];
  const uint64_t base = (uint64_t)blockIdx.x * kScanPer + (uint64_t)threadIdx.x * kScanItems;
  uint64_t v[kScanItems];
  uint64_t sum = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < n ? in[base + i] : 0;
    sum += v[i];
  }
  uint64_t tot;
  uint64_t run = block_excl_scan<uint64_t>(sum, s_wave, &tot);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
  if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// Adds each block's offset; thread n also stores the total, offs[nb], in
// out[n].
__global__ void k_scan_add(uint64_t* __restrict__ out, uint64_t n, const uint64_t* __restrict__ offs,
                           uint64_t nb) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] += offs[i / kScanPer];
  else if (i == n) out[n] = offs[nb];
}

size_t scan_tmp_words(uint64_t n) {
  if (n <= (uint64_t)kScanPer) return 0;
  uint64_t nb = (n + kScanPer - 1) / kScanPer;
  return nb + (nb + 1) + scan_tmp_words(nb);
}

void scan_exclusive(const uint64_t* in, uint64_t* out, uint64_t n, uint64_t* tmp, hipStream_t s) {
  if (n <= (uint64_t)kScanPer) {
    k_scan_block<<<1, kBlock, 0, s>>>(in, out, n, out + n);
    LCG_LAUNCH_CHECK("scan_block");
    return;
  }
  uint64_t nb = (n + kScanPer - 1) / kScanPer;
  uint64_t* sums = tmp;
  uint64_t* offs = tmp + nb;
  k_scan_block<<<grid_for(nb * kScanPer, kScanPer), kBlock, 0, s>>>(in, out, n, sums);
  LCG_LAUNCH_CHECK("scan_block");
  scan_exclusive(sums, offs, nb, tmp + nb + nb + 1, s);
  k_scan_add<<<grid_for(n + 1, 256), 256, 0, s>>>(out, n, offs, nb);
  LCG_LAUNCH_CHECK("scan_add");
}

// Exclusive scan in one block, for short arrays whose length is on the
// device: count = ceil(*x_dev / 2^shift) (or count_host without x_dev).
// out[count] and, if given, *total receive the sum.
constexpr int kScanOneThreads = 1024;

// LDS of a one-block scan (blocks of up to kScanOneThreads threads).
struct ScanLds {
  uint64_t s_wave[kScanOneThreads / 64];
  uint64_t s_carry;
};

// Exclusive scan of in[0..count) into out[0..count] by the whole block
// (blockDim.x a multiple of 64); out[count] and *total (if given) receive
// the sum.
__device__ __forceinline__ void scan_block(const uint64_t* __restrict__ in,
                                           uint64_t* __restrict__ out, uint64_t count,
                                           uint64_t* __restrict__ total, ScanLds& sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = blockDim.x / 64;
  if (threadIdx.x == 0) sh.s_carry = 0;
  __syncthreads();
  for (uint64_t c0 = 0; c0 < count; c0 += blockDim.x) {
    const uint64_t i = c0 + threadIdx.x;
    const uint64_t v = i < count ? in[i] : 0;
    uint64_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint64_t y = __shfl_up(x, d, 64);
      if (lane >= d) x += y;
    }
    if (lane == 63) sh.s_wave[wid] = x;
    __syncthreads();
    uint64_t base = sh.s_carry, tot = 0;
    for (int w = 0; w < nw; ++w) {
      const uint64_t sw = sh.s_wave[w];
      if (w < wid) base += sw;
      tot += sw;
    }
    if (i < count) out[i] = base + x - v;
    __syncthreads();
    if (threadIdx.x == 0) sh.s_carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[count] = sh.s_carry;
    if (total) *total = sh.s_carry;
  }
}

__global__ __launch_bounds__(kScanOneThreads) void k_scan_one(const uint64_t* __restrict__ in,
                                                              uint64_t* __restrict__ out,
                                                              uint64_t count,
                                                              const uint64_t* __restrict__ x_dev,
                                                              int shift,
                                                              uint64_t* __restrict__ total) {
  __shared__ ScanLds sh;
  if (x_dev) count = (*x_dev + (1ull << shift) - 1) >> shift;
  scan_block(in, out, count, total, sh);
}

void scan_one(const uint64_t* in, uint64_t* out, uint64_t count, const uint64_t* x_dev, int shift,
              uint64_t* total, hipStream_t s) {
  k_scan_one<<<1, kScanOneThreads, 0, s>>>(in, out, count, x_dev, shift, total);
  LCG_LAUNCH_CHECK("scan_one");
}

// ------------------------------------------------------------------ insert
// Whether slot `sl`, whose key word reads w, holds the wide phrase with key
// word kk and content (c0, c1).  A slot claimed in the running pass may not
// show its content words here yet (the claimer writes them after its claim);
// its key word then carries the claiming occurrence ref < d, whose content
// words are read from the phrase arrays instead (a committed rule's content
// was written by an earlier kernel).
__device__ __forceinline__ bool wide_slot_match(const Slot* sl, uint64_t w, uint64_t kk,
                                                uint64_t c0, uint64_t c1,
                                                const uint64_t* __restrict__ wkey, uint64_t d) {
  if ((w & kHiMask) != kk) return false;
  uint64_t s0 = hint_load(&sl->c0), s1 = hint_load(&sl->c1);
  if (s0 == kEmpty || s1 == kEmpty) {
    const uint32_t ref = (uint32_t)w;
    s0 = ref < d ? wkey[2 * (uint64_t)ref] : ~c0;
    s1 = ref < d ? wkey[2 * (uint64_t)ref + 1] : ~c1;
  }
  return s0 == c0 && s1 == c1;
}

// Append the slots the active lanes won (mine != kNone) to the won list: one
// atomic per wave, the lanes' entries in lane order.
__device__ __forceinline__ void push_won(bool mine, uint32_t pos, uint32_t* won,
                                         unsigned int* won_len) {
  const uint64_t bal = __ballot(mine);
  if (!bal) return;
  const uint64_t act = __ballot(1);
  const int leader = __builtin_ctzll(act);
  const int lane = threadIdx.x & 63;
  unsigned int base = 0;
  if (lane == leader) base = atomicAdd(won_len, (unsigned int)__builtin_popcountll(bal));
  base = __shfl(base, leader, 64);
  if (mine) won[base + __builtin_popcountll(bal & ((1ull << lane) - 1ull))] = pos;
}

// Equality of two symbol sequences of length len, without an early exit and
// without a call (both forms of the probe loop around it were compiled into
// code that lost the probe result).  Eight symbols of each side per step, so
// that their loads are in flight together.
template <typename Sym>
__device__ __forceinline__ bool same_seq(const Sym* a, const Sym* b, uint32_t len) {
  uint32_t diff = 0;
  for (uint32_t i = 0; i < len; i += 8) {
#pragma unroll
    for (uint32_t k = 0; k < 8; ++k) {
      const bool in = i + k < len;
      const Sym x = in ? a[i + k] : Sym(0);
      const Sym y = in ? b[i + k] : Sym(0);
      diff |= (uint32_t)(x != y);
    }
  }
  return diff == 0;
}

// Insert-or-find every phrase.  A claimed slot keeps the claimer's key.  A
// wide phrase whose key word matches is confirmed on its two content words:
// the slot's own copy (written by the claimer right after its claim, and by
// every earlier round), or, while that copy is not visible yet, the claiming
// occurrence's (each content word is written once, from empty to its value,
// so two non-empty words are the whole content).  A long phrase whose 30
// fingerprint bits match is compared symbol by symbol against the slot's
// phrase (the claiming occurrence, or the committed rule).
//
// The claimed word of a slot never changes during the kernel, so it is read
// with a workgroup-scope atomic load (L1-cacheable): frequent short phrases
// are then served by each CU's L1 instead of one L2 line.  A stale empty word
// only sends the thread to the compare-and-swap, which returns the current
// value.
//
// One phrase per thread and iteration (batches of several measured slower on
// gfx950: they cost more in occupancy than they gain in overlap).  The probe
// loop is written out in the kernel body with a single exit: the gfx950 code
// of the same loop placed in a helper function with counters passed by
// reference lost its result.
//
// The phrases are o = begin .. end-1, or o = list[begin .. *list_len-1] when
// a list is given; d is the round's phrase count (DEV_COUNT: d = end =
// *d_dev; a separate instance, so that profiles tell the rounds queued without
// host reads from the others).
template <typename Sym, bool DEV_COUNT>
__device__ __forceinline__ void insert_phrases(uint64_t block, uint64_t blocks, uint64_t begin,
                                               uint64_t end, uint64_t d,
                                               const uint64_t* __restrict__ d_dev,
                                               const uint32_t* __restrict__ list,
                                               const uint32_t* __restrict__ list_len,
                                               const uint64_t* __restrict__ key,
                                               const uint64_t* __restrict__ wkey,
                                               const uint64_t* __restrict__ pstart,
                                               const uint32_t* __restrict__ plen,
                                               const Sym* __restrict__ content,
                                               const uint64_t* __restrict__ rule_off,
                                               const Sym* __restrict__ rule_rhs,
                                               uint32_t u_committed, Slot* table, uint64_t mask,
                                               uint32_t* __restrict__ slot_idx,
                                               uint32_t* __restrict__ won_list,
                                               uint64_t won_per_wave,
                                               uint32_t* __restrict__ won_cnt,
                                               Counters* __restrict__ ctr,
                                               unsigned long long* s_sum) {
  if (threadIdx.x < 4) s_sum[threadIdx.x] = 0;
  __syncthreads();
  unsigned long long won = 0, probes = 0, cmps = 0, fails = 0;
  const uint64_t stride = blocks * blockDim.x;
  if constexpr (DEV_COUNT) end = d = *d_dev;  // launched over a bound; the count is on the device
  const uint64_t lim = list ? (uint64_t)*list_len : end;
  // every wave walks its own phrases (the same trip count for all its lanes)
  // and lists the slots it claims in its own region of the won list
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t wave = block * (uint64_t)(blockDim.x / 64) + (threadIdx.x >> 6);
  uint32_t* const my_won = won_list ? won_list + wave * won_per_wave : nullptr;
  uint32_t nwon = 0;
  // the next iteration's phrase index and key are loaded one iteration
  // ahead, so that the key's load is not on the probe's dependency chain
  uint64_t o_next = 0, kk_next = 0;
  {
    const uint64_t i = begin + wave * 64 + lane;
    if (i < lim) {
      o_next = list ? (uint64_t)list[i] : i;
      kk_next = __builtin_nontemporal_load(&key[o_next]);  // streams past L1
    }
  }
  for (uint64_t wb = begin + wave * 64; wb < lim; wb += stride) {
    const uint64_t i = wb + lane;
    uint32_t result = kNone;
    bool claimed = false;
    const uint64_t o = o_next, kk = kk_next;
    if (i + stride < lim) {
      o_next = list ? (uint64_t)list[i + stride] : i + stride;
      kk_next = __builtin_nontemporal_load(&key[o_next]);
    }
    if (i < lim) {
    uint64_t pos = mix64(kk) & mask;
    const uint64_t home = pos;
    // the home slot's key word and (first occurrence, rank) together: most
    // phrases end at their home slot, and then the second word needs no
    // load of its own
    uint64_t w = hint_load(&table[pos].w0);
    const uint64_t mr_home = hint_load(reinterpret_cast<const uint64_t*>(&table[pos].minocc));
    const bool tagged = (kk & kLongTag) != 0;  // wide or long: the slot word carries a reference
    const bool wide = is_wide(kk);
    const bool is_long = tagged && !wide;
    const uint64_t want = tagged ? (kk | o) : kk;
    uint64_t my_pos = 0, my_c0 = 0, my_c1 = 0;
    uint32_t my_len = 0;
    if (is_long) {
      my_pos = pstart[o];
      my_len = plen[o];
    }
    if (wide) {
      my_c0 = wkey[2 * o];
      my_c1 = wkey[2 * o + 1];
    }
    for (uint32_t probe = 0; probe < kMaxProbe && result == kNone; ++probe) {
      Slot* sl = &table[pos];
      ++probes;
      if (probe) w = hint_load(&sl->w0);
      bool hit = false;
      if (w == kEmpty) {
        unsigned long long prev =
            atomicCAS(reinterpret_cast<unsigned long long*>(&sl->w0), (unsigned long long)kEmpty,
                      (unsigned long long)want);
        if (prev == kEmpty) {
          hit = true;
          claimed = true;
          ++won;
          if (wide) {  // the content beside the claim, for the phrases that follow
            __hip_atomic_store(&sl->c0, my_c0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&sl->c1, my_c1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
        } else {
          w = prev;
        }
      }
      if (!hit) {
        if (!tagged) {
          hit = w == kk;
        } else if (wide) {
          hit = wide_slot_match(sl, w, kk, my_c0, my_c1, wkey, d);
        } else if ((w & kHiMask) == kk) {
          const uint32_t rk = hint_load(&sl->rank);
          const uint32_t ref = (uint32_t)w;
          // a committed rule is compared with its stored right-hand side, a
          // slot claimed in this pass with the claiming occurrence; anything
          // else (a slot left by an interrupted call) cannot match
          const bool committed = rk != kNone && rk < u_committed;
          const bool inflight = rk == kNone && ref < d;
          uint64_t opos = 0;
          uint32_t olen = 0xFFFFFFFFu;
          const Sym* arr = content;
          if (committed) {
            opos = rule_off[rk];
            olen = (uint32_t)(rule_off[rk + 1] - opos);
            arr = rule_rhs;
          } else if (inflight) {
            opos = pstart[ref];
            olen = plen[ref];
          }
          ++cmps;
          hit = olen == my_len && same_seq<Sym>(content + my_pos, arr + opos, my_len);
        }
      }
      if (hit) result = (uint32_t)pos;
      else pos = (pos + 1) & mask;
    }
    if (result == kNone) {
      ++fails;
    } else {
      Slot* sl = &table[result];
      // (first occurrence, rank) in one load; a stale (larger) first
      // occurrence only costs an unneeded atomicMin (first occurrences only
      // decrease, and a slot's rank does not change within the pass).  The
      // claimer registers its occurrence without a look.
      const uint64_t mr = claimed ? (uint64_t)kNone << 32 | kNone
                          : result == home ? mr_home
                          : hint_load(reinterpret_cast<const uint64_t*>(&sl->minocc));
      if ((uint32_t)(mr >> 32) == kNone && (uint32_t)mr > (uint32_t)o)
        atomicMin(&sl->minocc, (uint32_t)o);
    }
    __builtin_nontemporal_store(result, &slot_idx[o]);
    }
    if (my_won) {
      const uint64_t bal = __ballot(claimed);
      if (claimed) my_won[nwon + __builtin_popcountll(bal & ((1ull << lane) - 1ull))] = result;
      nwon += (uint32_t)__builtin_popcountll(bal);
    }
  }
  if (my_won && lane == 0) won_cnt[wave] = nwon;
  // one global atomic per block and counter
  won = wave_sum(won);
  probes = wave_sum(probes);
  cmps = wave_sum(cmps);
  fails = wave_sum(fails);
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&s_sum[0], won);
    atomicAdd(&s_sum[1], probes);
    atomicAdd(&s_sum[2], cmps);
    atomicAdd(&s_sum[3], fails);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (s_sum[0]) atomicAdd(&ctr->won, s_sum[0]);
    if (s_sum[1]) atomicAdd(&ctr->probes, s_sum[1]);
    if (s_sum[2]) atomicAdd(&ctr->compares, s_sum[2]);
    if (s_sum[3]) atomicAdd(&ctr->overflow, (unsigned int)s_sum[3]);
  }
}

template <typename Sym, bool DEV_COUNT>
__global__ __launch_bounds__(256) void k_insert(uint64_t begin, uint64_t end, uint64_t d,
                                                const uint64_t* __restrict__ d_dev,
                                                const uint32_t* __restrict__ list,
                                                const uint32_t* __restrict__ list_len,
                                                const uint64_t* __restrict__ key,
                                                const uint64_t* __restrict__ wkey,
                                                const uint64_t* __restrict__ pstart,
                                                const uint32_t* __restrict__ plen,
                                                const Sym* __restrict__ content,
                                                const uint64_t* __restrict__ rule_off,
                                                const Sym* __restrict__ rule_rhs, uint32_t u_committed,
                                                Slot* table, uint64_t mask,
                                                uint32_t* __restrict__ slot_idx,
                                                uint32_t* __restrict__ won_list,
                                                uint64_t won_per_wave,
                                                uint32_t* __restrict__ won_cnt,
                                                Counters* __restrict__ ctr) {
  __shared__ unsigned long long s_sum[4];
  insert_phrases<Sym, DEV_COUNT>(blockIdx.x, gridDim.x, begin, end, d, d_dev, list, list_len, key,
                                 wkey, pstart, plen, content, rule_off, rule_rhs, u_committed,
                                 table, mask, slot_idx, won_list, won_per_wave, won_cnt, ctr, s_sum);
}

// Combining insert for rounds whose phrases repeat a few keys many times
// (round 1 of DNA-like text: ~10^8 phrases, ~10^4 distinct).  Every block
// takes a chunk of kCombChunk consecutive phrases and first builds a
// dictionary of the chunk's exact keys in LDS, with each key's first
// occurrence in the chunk; then one thread per distinct key probes the
// global dictionary once and lowers the slot's first occurrence once; then
// every phrase takes its slot from LDS.  Frequent keys thus cost one global
// access per chunk instead of one per occurrence (which, for a handful of
// keys, all land on the same few L2 lines).  Wide keys (not combined: equal
// key words need not mean equal content) are listed per chunk and probe the
// global dictionary directly, in the chunk's order; long keys, and keys that
// find no room in the LDS table or list, are appended to `rest` for k_insert.
constexpr int kCombLog2 = 11;
constexpr int kComb = 1 << kCombLog2;   // LDS dictionary entries
constexpr int kCombChunk = 4096;        // phrases per block and iteration
constexpr int kCombProbe = 32;          // LDS probe budget
constexpr int kCombItems = kCombChunk / 256;
constexpr uint16_t kCombNone = 0xFFFF;
constexpr uint16_t kCombWide = 0xFFFE;  // s_loc mark: the phrase is on the wide list
constexpr int kCombWideList = 512;      // wide phrases listed per chunk

__global__ __launch_bounds__(256) void k_insert_comb(uint64_t begin, uint64_t end, uint64_t d,
                                                     const uint64_t* __restrict__ key,
                                                     const uint64_t* __restrict__ wkey, Slot* table,
                                                     uint64_t mask, uint32_t* __restrict__ slot_idx,
                                                     uint32_t* __restrict__ rest,
                                                     uint32_t* __restrict__ rest_len,
                                                     uint32_t* __restrict__ won_list,
                                                     Counters* __restrict__ ctr) {
  __shared__ unsigned long long s_key[kComb];  // reused as the chunk's rest list
  __shared__ uint32_t s_min[kComb];
  __shared__ uint32_t s_slot[kComb];
  __shared__ uint16_t s_loc[kCombChunk];
  __shared__ uint16_t s_wide[kCombWideList];
  __shared__ unsigned long long s_sum[3];
  __shared__ uint32_t s_nrest, s_rbase, s_nwide;
  static_assert(kComb * sizeof(unsigned long long) >= kCombChunk * sizeof(uint32_t),
                "the rest list reuses the key table");
  if (threadIdx.x < 3) s_sum[threadIdx.x] = 0;
  unsigned long long won = 0, probes = 0, fails = 0;
  for (uint64_t c0 = begin + blockIdx.x * (uint64_t)kCombChunk; c0 < end;
       c0 += (uint64_t)gridDim.x * kCombChunk) {
    for (int i = threadIdx.x; i < kComb; i += blockDim.x) {
      s_key[i] = kEmpty;
      s_min[i] = kNone;
    }
    if (threadIdx.x == 0) {
      s_nrest = 0;
      s_nwide = 0;
    }
    __syncthreads();
    // 1: the chunk's exact keys into the LDS dictionary (all keys loaded first,
    // so that their loads overlap)
    uint64_t kc[kCombItems];
#pragma unroll
    for (int x = 0; x < kCombItems; ++x) {
      const uint64_t o = c0 + x * 256 + threadIdx.x;
      kc[x] = o < end ? key[o] : kLongTag;
    }
#pragma unroll
    for (int x = 0; x < kCombItems; ++x) {
      const uint32_t li = x * 256 + threadIdx.x;
      const uint64_t o = c0 + li;
      uint32_t found = kNone;
      {
        const uint64_t kk = kc[x];
        if (!(kk & kLongTag)) {
          // LDS position: the key's halves folded and one 32-bit multiply
          // (the global table's 64-bit mix is needed only once per distinct key)
          uint32_t lpos = (((uint32_t)kk ^ (uint32_t)(kk >> 32) * 0x85EBCA77u) * 0x9E3779B1u) >>
                          (32 - kCombLog2);
          for (int t = 0; t < kCombProbe && found == kNone; ++t) {
            const unsigned long long w =
                __hip_atomic_load(&s_key[lpos], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            bool hit;
            if (w == kEmpty) {
              const unsigned long long prev =
                  atomicCAS(&s_key[lpos], (unsigned long long)kEmpty, (unsigned long long)kk);
              hit = prev == kEmpty || prev == kk;
            } else {
              hit = w == kk;
            }
            if (hit) found = lpos;
            else lpos = (lpos + 1) & (kComb - 1);
          }
          // a frequent key's first occurrence is usually set already
          if (found != kNone && (uint32_t)o < __hip_atomic_load(&s_min[found], __ATOMIC_RELAXED,
                                                                __HIP_MEMORY_SCOPE_WORKGROUP))
            atomicMin(&s_min[found], (uint32_t)o);
        } else if (is_wide(kk)) {
          const uint32_t at = atomicAdd(&s_nwide, 1u);
          if (at < (uint32_t)kCombWideList) {
            s_wide[at] = (uint16_t)li;
            found = kCombWide;
          }
        }
      }
      s_loc[li] = found == kNone ? kCombNone : (uint16_t)found;
    }
    __syncthreads();
    // 2: one global insert per distinct key, with its first occurrence (the
    // home words of the thread's entries are loaded first)
    uint64_t hw[kComb / 256];
#pragma unroll
    for (int j = 0; j < kComb / 256; ++j) {
      const uint64_t kk = s_key[j * 256 + threadIdx.x];
      hw[j] = kk != kEmpty ? hint_load(&table[mix64(kk) & mask].w0) : kEmpty;
    }
#pragma unroll
    for (int j = 0; j < kComb / 256; ++j) {
      const int i = j * 256 + threadIdx.x;
      const uint64_t kk = s_key[i];
      uint32_t res = kNone;
      bool claimed = false;
      if (kk != kEmpty) {
        uint64_t pos = mix64(kk) & mask;
        for (uint32_t probe = 0; probe < kMaxProbe && res == kNone; ++probe) {
          Slot* sl = &table[pos];
          ++probes;
          uint64_t w = probe ? hint_load(&sl->w0) : hw[j];
          bool hit = false;
          if (w == kEmpty) {
            const unsigned long long prev =
                atomicCAS(reinterpret_cast<unsigned long long*>(&sl->w0),
                          (unsigned long long)kEmpty, (unsigned long long)kk);
            if (prev == kEmpty) {
              hit = true;
              claimed = true;
              ++won;
            } else {
              w = prev;
            }
          }
          if (!hit) hit = w == kk;
          if (hit) res = (uint32_t)pos;
          else pos = (pos + 1) & mask;
        }
        if (res == kNone) {
          ++fails;
        } else {
          const uint32_t m = s_min[i];
          Slot* sl = &table[res];
          const uint64_t mr = hint_load(reinterpret_cast<const uint64_t*>(&sl->minocc));
          if ((uint32_t)(mr >> 32) == kNone && (uint32_t)mr > m) atomicMin(&sl->minocc, m);
        }
      }
      s_slot[i] = res;
      push_won(claimed, res, won_list, &ctr->won_len);
    }
    // 2b: the chunk's wide phrases, each straight into the global dictionary
    // (the list's length is block-uniform, so every lane reaches push_won)
    const uint32_t nwide = s_nwide < (uint32_t)kCombWideList ? s_nwide : (uint32_t)kCombWideList;
    for (uint32_t b = 0; b < nwide; b += blockDim.x) {
      const uint32_t i = b + threadIdx.x;
      uint32_t res = kNone;
      bool claimed = false;
      if (i < nwide) {
        const uint64_t o = c0 + s_wide[i];
        const uint64_t kk = key[o];
        const uint64_t my0 = wkey[2 * o], my1 = wkey[2 * o + 1];
        uint64_t pos = mix64(kk) & mask;
        for (uint32_t probe = 0; probe < kMaxProbe && res == kNone; ++probe) {
          Slot* sl = &table[pos];
          ++probes;
          uint64_t w = hint_load(&sl->w0);
          bool hit = false;
          if (w == kEmpty) {
            const unsigned long long prev =
                atomicCAS(reinterpret_cast<unsigned long long*>(&sl->w0),
                          (unsigned long long)kEmpty, (unsigned long long)(kk | o));
            if (prev == kEmpty) {
              hit = true;
              claimed = true;
              ++won;
              __hip_atomic_store(&sl->c0, my0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              __hip_atomic_store(&sl->c1, my1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
              w = prev;
            }
          }
          if (!hit) hit = wide_slot_match(sl, w, kk, my0, my1, wkey, d);
          if (hit) res = (uint32_t)pos;
          else pos = (pos + 1) & mask;
        }
        if (res == kNone) {
          ++fails;
        } else {
          Slot* sl = &table[res];
          const uint64_t mr = claimed ? (uint64_t)kNone << 32 | kNone
                                      : hint_load(reinterpret_cast<const uint64_t*>(&sl->minocc));
          if ((uint32_t)(mr >> 32) == kNone && (uint32_t)mr > (uint32_t)o)
            atomicMin(&sl->minocc, (uint32_t)o);
        }
        slot_idx[o] = res;
      }
      push_won(claimed, res, won_list, &ctr->won_len);
    }
    __syncthreads();
    // 3: slots of the combined phrases; the others join the rest list
    uint32_t* s_list = reinterpret_cast<uint32_t*>(s_key);
    for (int x = 0; x < kCombItems; ++x) {
      const uint32_t li = x * 256 + threadIdx.x;
      const uint64_t o = c0 + li;
      if (o < end) {
        const uint16_t lr = s_loc[li];
        if (lr == kCombNone) s_list[atomicAdd(&s_nrest, 1u)] = (uint32_t)o;
        else if (lr != kCombWide) slot_idx[o] = s_slot[lr];
      }
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_nrest) s_rbase = atomicAdd(rest_len, s_nrest);
    __syncthreads();
    const uint32_t nr = s_nrest;
    for (uint32_t i = threadIdx.x; i < nr; i += blockDim.x) rest[s_rbase + i] = s_list[i];
    __syncthreads();
  }
  won = wave_sum(won);
  probes = wave_sum(probes);
  fails = wave_sum(fails);
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&s_sum[0], won);
    atomicAdd(&s_sum[1], probes);
    atomicAdd(&s_sum[2], fails);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (s_sum[0]) atomicAdd(&ctr->won, s_sum[0]);
    if (s_sum[1]) atomicAdd(&ctr->probes, s_sum[1]);
    if (s_sum[2]) atomicAdd(&ctr->overflow, (unsigned int)s_sum[2]);
  }
}

// With `combine` the phrases go through k_insert_comb in launches over
// growing ranges [0, 2^16), [2^16, 2^20), ...: a kernel boundary makes every
// slot's first occurrence visible to all CUs, so the frequent keys, whose
// first occurrences come early, find it settled in later ranges and skip the
// atomicMin (within one launch a CU may keep reading a stale first
// occurrence from its L1).  What k_insert_comb leaves (rest, count
// *rest_len, zero on entry) then goes through k_insert.  Otherwise one
// k_insert launch takes all d phrases.
WonGeom won_geometry(uint64_t d) {
  if (!d) return WonGeom{0, 0};
  uint64_t g = (d + 255) / 256;
  if (g > kPersistentBlocks) g = kPersistentBlocks;
  const uint64_t stride = g * 256;
  return WonGeom{(uint32_t)(g * 4), 64 * ((d + stride - 1) / stride)};
}

void launch_insert(bool bytes, uint64_t d, const uint64_t* d_dev, const uint64_t* key,
                   const uint64_t* wkey, const uint64_t* pstart, const uint32_t* plen,
                   const void* content, const uint64_t* rule_off, const void* rule_rhs,
                   uint32_t u_committed, Slot* table, uint64_t mask, uint32_t* slot_idx,
                   bool combine, uint32_t* rest, uint32_t* rest_len, uint32_t* won,
                   uint32_t* won_cnt, uint32_t* won2, Counters* ctr, hipStream_t s) {
  if (!d) return;
  const WonGeom geo = won_geometry(d);
  if (d_dev && combine) throw std::runtime_error("insert: combining needs the count on the host");
  const uint32_t* list = nullptr;
  const uint32_t* list_len = nullptr;
  unsigned g = grid_for(d, 256);
  if (combine) {
    const unsigned r = resident_blocks((const void*)k_insert_comb, 256);
    for (uint64_t begin = 0, end = d < (1ull << 16) ? d : (1ull << 16); begin < d;
         begin = end, end = end * 16 < d ? end * 16 : d) {
      unsigned gc = grid_for(end - begin, kCombChunk);
      if (gc > r) gc = r;
      k_insert_comb<<<gc, 256, 0, s>>>(begin, end, d, key, wkey, table, mask, slot_idx, rest,
                                       rest_len, won2, ctr);
      LCG_LAUNCH_CHECK("insert_comb");
    }
    list = rest;  // at most d phrases; the count is on the device
    list_len = rest_len;
  }
  if (g > kPersistentBlocks) g = kPersistentBlocks;
  if (g * 4 != geo.waves) throw std::runtime_error("insert: grid differs from the won geometry");
  const uint8_t* c8 = static_cast<const uint8_t*>(content);
  const uint8_t* r8 = static_cast<const uint8_t*>(rule_rhs);
  const uint32_t* c32 = static_cast<const uint32_t*>(content);
  const uint32_t* r32 = static_cast<const uint32_t*>(rule_rhs);
  if (bytes && d_dev)
    k_insert<uint8_t, true><<<g, 256, 0, s>>>(0, d, d, d_dev, list, list_len, key, wkey, pstart, plen, c8,
                                              rule_off, r8, u_committed, table, mask, slot_idx, won, geo.per_wave,
                                              won_cnt, ctr);
  else if (bytes)
    k_insert<uint8_t, false><<<g, 256, 0, s>>>(0, d, d, d_dev, list, list_len, key, wkey, pstart, plen, c8,
                                               rule_off, r8, u_committed, table, mask, slot_idx, won, geo.per_wave,
                                              won_cnt, ctr);
  else if (d_dev)
    k_insert<uint32_t, true><<<g, 256, 0, s>>>(0, d, d, d_dev, list, list_len, key, wkey, pstart,
                                               plen, c32, rule_off, r32, u_committed, table, mask,
                                               slot_idx, won, geo.per_wave, won_cnt, ctr);
  else
    k_insert<uint32_t, false><<<g, 256, 0, s>>>(0, d, d, d_dev, list, list_len, key, wkey, pstart,
                                                plen, c32, rule_off, r32, u_committed, table, mask,
                                                slot_idx, won, geo.per_wave, won_cnt, ctr);
  LCG_LAUNCH_CHECK("insert");
}

// ------------------------------------------------------------------ newflags
// Per phrase: new if it is the first occurrence of a slot claimed in this
// pass (one (first occurrence, rank) read from its slot); per flag word of 64
// phrases the new rules and their right-hand-side lengths.  For rounds where
// most phrases are new: a coalesced pass over the phrases beats one random
// flag per new rule.
// Flag words wave, wave + waves, ... (one wave per word of 64 phrases).
template <bool BYTES>
__device__ __forceinline__ void newflags_words(uint64_t d, uint64_t wave, uint64_t waves,
                                               const uint32_t* __restrict__ slot_idx,
                                               const Slot* __restrict__ table,
                                               const uint64_t* __restrict__ key,
                                               const uint32_t* __restrict__ plen,
                                               uint64_t* __restrict__ newbits,
                                               uint64_t* __restrict__ wcnt,
                                               uint64_t* __restrict__ wlen) {
  const uint32_t lane = threadIdx.x & 63;
  for (uint64_t w = wave; (w << 6) < d; w += waves) {
    const uint64_t o = (w << 6) + lane;
    bool f = false;
    unsigned long long len = 0;
    if (o < d) {
      const uint32_t sidx = slot_idx[o];
      if (sidx != kNone) {
        const uint64_t mr = *reinterpret_cast<const uint64_t*>(&table[sidx].minocc);
        f = (uint32_t)(mr >> 32) == kNone && (uint32_t)mr == (uint32_t)o;
      }
      if (f) len = key_len<BYTES>(key[o], plen, o);
    }
    const uint64_t bal = __ballot(f);
    len = wave_sum(len);
    if (lane == 0) {
      newbits[w] = bal;
      wcnt[w] = __builtin_popcountll(bal);
      wlen[w] = len;
    }
  }
}

template <bool BYTES>
__global__ __launch_bounds__(256) void k_newflags(uint64_t d, const uint64_t* __restrict__ d_dev,
                                                  const uint32_t* __restrict__ slot_idx,
                                                  const Slot* __restrict__ table,
                                                  const uint64_t* __restrict__ key,
                                                  const uint32_t* __restrict__ plen,
                                                  uint64_t* __restrict__ newbits,
                                                  uint64_t* __restrict__ wcnt,
                                                  uint64_t* __restrict__ wlen) {
  if (d_dev) d = *d_dev;
  newflags_words<BYTES>(d, blockIdx.x * (uint64_t)(blockDim.x / 64) + (threadIdx.x >> 6),
                        (uint64_t)gridDim.x * (blockDim.x / 64), slot_idx, table, key, plen,
                        newbits, wcnt, wlen);
}

void launch_newflags(bool bytes, uint64_t d, const uint64_t* d_dev, const uint32_t* slot_idx,
                     const Slot* table, const uint64_t* key, const uint32_t* plen,
                     uint64_t* newbits, uint64_t* wcnt, uint64_t* wlen, hipStream_t s) {
  if (!d) return;
  if (bytes)
    k_newflags<true><<<grid_for(d, 256), 256, 0, s>>>(d, d_dev, slot_idx, table, key, plen, newbits,
                                                      wcnt, wlen);
  else
    k_newflags<false><<<grid_for(d, 256), 256, 0, s>>>(d, d_dev, slot_idx, table, key, plen,
                                                       newbits, wcnt, wlen);
  LCG_LAUNCH_CHECK("newflags");
}

// Per flag word: its new rules and their right-hand-side lengths (the keys of
// one word's phrases lie side by side).
template <bool BYTES>
__global__ void k_word_counts(const uint64_t* __restrict__ newbits, uint64_t W,
                              const uint64_t* __restrict__ key, const uint32_t* __restrict__ plen,
                              uint64_t* __restrict__ wcnt, uint64_t* __restrict__ wlen) {
  const uint64_t w = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (w >= W) return;
  uint64_t bits = newbits[w];
  wcnt[w] = __builtin_popcountll(bits);
  uint64_t len = 0;
  while (bits) {
    const uint64_t m = w * 64 + (uint64_t)__builtin_ctzll(bits);
    bits &= bits - 1;
    len += key_len<BYTES>(key[m], plen, m);
  }
  wlen[w] = len;
}

// The first occurrence of every slot claimed in the round marks its phrase
// new (newbits zero on entry): the combining insert's list (won2, count in
// ctr->won_len), then the regions of the insert's waves (region v holds
// won_cnt[v] slots from won + v * per_wave).
__global__ __launch_bounds__(256) void k_newflags_won(const uint32_t* __restrict__ won,
                                                      const uint32_t* __restrict__ won_cnt,
                                                      uint32_t waves, uint64_t per_wave,
                                                      const uint32_t* __restrict__ won2,
                                                      const Counters* __restrict__ ctr,
                                                      const Slot* __restrict__ table,
                                                      unsigned long long* __restrict__ newbits) {
  const uint32_t n2 = ctr->won_len;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += gridDim.x * blockDim.x) {
    const uint64_t m = table[won2[i]].minocc;
    atomicOr(&newbits[m >> 6], 1ULL << (m & 63));
  }
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t nw = gridDim.x * (blockDim.x / 64);
  for (uint32_t v = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); v < waves; v += nw) {
    const uint32_t c = won_cnt[v];
    const uint32_t* r = won + (uint64_t)v * per_wave;
    for (uint32_t i = lane; i < c; i += 64) {
      const uint64_t m = table[r[i]].minocc;
      atomicOr(&newbits[m >> 6], 1ULL << (m & 63));
    }
  }
}

void launch_newflags_won(bool bytes, uint64_t d, const uint32_t* won, const uint32_t* won_cnt,
                         const uint32_t* won2, const Counters* ctr, const Slot* table, uint64_t W,
                         const uint64_t* key, const uint32_t* plen, uint64_t* newbits,
                         uint64_t* wcnt, uint64_t* wlen, hipStream_t s) {
  if (!W || !d) return;
  const WonGeom geo = won_geometry(d);
  launch_zero(newbits, W * 8, s);
  unsigned g = (geo.waves + 3) / 4;
  if (g > 2048) g = 2048;
  k_newflags_won<<<g, 256, 0, s>>>(won, won_cnt, geo.waves, geo.per_wave, won2, ctr, table,
                                   reinterpret_cast<unsigned long long*>(newbits));
  LCG_LAUNCH_CHECK("newflags_won");
  if (bytes)
    k_word_counts<true><<<grid_for(W, 256), 256, 0, s>>>(newbits, W, key, plen, wcnt, wlen);
  else
    k_word_counts<false><<<grid_for(W, 256), 256, 0, s>>>(newbits, W, key, plen, wcnt, wlen);
  LCG_LAUNCH_CHECK("word_counts");
}

// ------------------------------------------------------------------ commit
__device__ __forceinline__ unsigned long long wave_excl_scan(unsigned long long v) {
  const int lane = threadIdx.x & 63;
  unsigned long long x = v;
#pragma unroll
  for (int k = 1; k < 64; k <<= 1) {
    unsigned long long y = __shfl_up(x, k, 64);
    if (lane >= k) x += y;
  }
  return x - v;
}

// New rules: the first occurrence of every new phrase appends the rule.  One
// wave per 64-phrase flag word (a word without a new phrase ends at once), so
// the offset of a rule's right-hand side is the word's scanned length plus a
// wave scan.  A rule with an exact key gets its fingerprint here (Eq. 4 over
// the F values of its symbols, fprev), a long one brings it from emit (fnew).
// The slot then holds the rank and F side by side: one 8-byte load gives a
// later occurrence both.
// Commit the new phrase o as rule r (right-hand side at q): its content
// (from the phrase for a long key, from the key itself for an exact one),
// its F (Eq. 4 from the symbols' F, once per rule, for exact keys) and
// (F, rank) into its slot.
template <typename Sym>
__device__ __forceinline__ void commit_one(uint64_t o, uint32_t r, uint64_t q, uint64_t kk,
                                           uint32_t L, uint32_t sidx, Slot* table,
                                           const uint64_t* __restrict__ wkey,
                                           const uint64_t* __restrict__ pstart,
                                           const Sym* __restrict__ content,
                                           const uint32_t* fnew,
                                           const uint32_t* __restrict__ fprev, LevelHash h,
                                           uint64_t* __restrict__ rule_off,
                                           Sym* __restrict__ rule_rhs,
                                           uint32_t* __restrict__ rule_fp, uint32_t* sym_next,
                                           uint32_t* fnext) {
  constexpr bool kBytes = sizeof(Sym) == 1;
  uint32_t F;
  if (is_wide(kk)) {
    // at most 14 symbols (4 above level 1) from the content words, then Horner
    constexpr uint32_t kMaxWide = kBytes ? kWideMaxBytes : kWideMaxRanks;
    const uint64_t c0 = wkey[2 * o], c1 = wkey[2 * o + 1];
    uint32_t v[kMaxWide], f[kMaxWide];
#pragma unroll
    for (uint32_t x = 0; x < kMaxWide; ++x) {
      v[x] = x < L ? wide_sym<kBytes>(kk, c0, c1, x) : 0u;
      f[x] = x < L ? fprev[v[x]] : 0u;
    }
    uint64_t S = 0;
#pragma unroll
    for (int x = kMaxWide - 1; x >= 0; --x) {
      if ((uint32_t)x < L) {
        rule_rhs[q + x] = (Sym)v[x];
        S = addmod61(mulmod61(S, h.c), f[x]);
      }
    }
    F = (uint32_t)(addmod61(mulmod61(h.a, S), h.b) & 0xFFFFFFFFULL);
  } else if (kk & kLongTag) {
    // eight symbols per step, so that their loads are in flight together
    const Sym* src = content + pstart[o];
    for (uint32_t i = 0; i < L; i += 8) {
      Sym v[8];
#pragma unroll
      for (uint32_t x = 0; x < 8; ++x) v[x] = i + x < L ? src[i + x] : Sym(0);
#pragma unroll
      for (uint32_t x = 0; x < 8; ++x)
        if (i + x < L) rule_rhs[q + i + x] = v[x];
    }
    F = fnew[o];
  } else {
    // at most 7 symbols (4 above level 1): gather their F first, then Horner
    constexpr uint32_t kMaxExact = kBytes ? 7 : 4;
    uint32_t v[kMaxExact], f[kMaxExact];
#pragma unroll
    for (uint32_t x = 0; x < kMaxExact; ++x) {
      v[x] = x < L ? key_sym<kBytes>(kk, x) : 0u;
      f[x] = x < L ? fprev[v[x]] : 0u;
    }
    uint64_t S = 0;
#pragma unroll
    for (int x = kMaxExact - 1; x >= 0; --x) {
      if ((uint32_t)x < L) {
        rule_rhs[q + x] = (Sym)v[x];
        S = addmod61(mulmod61(S, h.c), f[x]);
      }
    }
    F = (uint32_t)(addmod61(mulmod61(h.a, S), h.b) & 0xFFFFFFFFULL);
  }
  rule_off[r + 1] = q + L;
  rule_fp[r] = F;
  Slot* sl = &table[sidx];
  *reinterpret_cast<uint64_t*>(&sl->minocc) = (uint64_t)F | ((uint64_t)r << 32);
  // a long key's slot word switches from the claiming occurrence to the rank
  if (kk & kLongTag) sl->w0 = (kk & kHiMask) | r;
  // the new phrase's own symbol and F of T^{i+1}: the rewrite need not read
  // them back from the slot
  if (sym_next) {
    sym_next[o] = r;
    if (fnext) fnext[o] = F;
  }
}

// one wave per flag word of 64 phrases: ranks from the word's count base and
// the wave's ballot prefix, right-hand-side offsets from the word's length
// base and a wave scan.  Words wave, wave + waves, ...
template <typename Sym>
__device__ __forceinline__ void commit_words(uint64_t d, uint64_t wave, uint64_t waves,
                                             const uint32_t* __restrict__ slot_idx, Slot* table,
                                             const uint64_t* __restrict__ newbits,
                                             const uint64_t* __restrict__ wcnt_base,
                                             const uint64_t* __restrict__ wlen_base,
                                             const uint64_t* __restrict__ key,
                                             const uint64_t* __restrict__ wkey,
                                             const uint64_t* __restrict__ pstart,
                                             const uint32_t* __restrict__ plen,
                                             const Sym* __restrict__ content,
                                             const uint32_t* fnew,
                                             const uint32_t* __restrict__ fprev, LevelHash h,
                                             uint32_t u_prev, uint64_t q_prev,
                                             uint64_t* __restrict__ rule_off,
                                             Sym* __restrict__ rule_rhs,
                                             uint32_t* __restrict__ rule_fp, uint32_t* sym_next,
                                             uint32_t* fnext) {
  constexpr bool kBytes = sizeof(Sym) == 1;
  const uint64_t W = (d + 63) / 64;
  const uint32_t lane = threadIdx.x & 63;
  for (uint64_t wd = wave; wd < W; wd += waves) {
    const uint64_t fw = newbits[wd];
    if (!fw) continue;  // uniform in the wave
    const uint64_t o = wd * 64 + lane;
    const bool isnew = (fw >> lane) & 1ULL;
    const uint64_t kk = isnew ? key[o] : 0;
    const uint32_t L = isnew ? key_len<kBytes>(kk, plen, o) : 0;
    const unsigned long long excl = wave_excl_scan(L);
    if (isnew) {
      const uint32_t r = u_prev + (uint32_t)(wcnt_base[wd] +
                                             __builtin_popcountll(fw & ((1ULL << lane) - 1ULL)));
      const uint64_t q = q_prev + wlen_base[wd] + excl;
      commit_one<Sym>(o, r, q, kk, L, slot_idx[o], table, wkey, pstart, content, fnew, fprev, h,
                      rule_off, rule_rhs, rule_fp, sym_next, fnext);
    }
  }
}

template <typename Sym>
__global__ __launch_bounds__(256) void k_commit_new(uint64_t d, const uint64_t* __restrict__ d_dev,
                                                    const uint32_t* __restrict__ slot_idx,
                                                    Slot* table, const uint64_t* __restrict__ newbits,
                                                    const uint64_t* __restrict__ wcnt_base,
                                                    const uint64_t* __restrict__ wlen_base,
                                                    const uint64_t* __restrict__ key,
                                                    const uint64_t* __restrict__ wkey,
                                                    const uint64_t* __restrict__ pstart,
                                                    const uint32_t* __restrict__ plen,
                                                    const Sym* __restrict__ content,
                                                    const uint32_t* fnew,
                                                    const uint32_t* __restrict__ fprev, LevelHash h,
                                                    uint32_t u_prev, uint64_t q_prev,
                                                    uint64_t* __restrict__ rule_off,
                                                    Sym* __restrict__ rule_rhs,
                                                    uint32_t* __restrict__ rule_fp,
                                                    uint32_t* sym_next, uint32_t* fnext) {
  if (d_dev) d = *d_dev;
  commit_words<Sym>(d, blockIdx.x * (uint64_t)(blockDim.x / 64) + (threadIdx.x >> 6),
                    (uint64_t)gridDim.x * (blockDim.x / 64), slot_idx, table, newbits, wcnt_base,
                    wlen_base, key, wkey, pstart, plen, content, fnew, fprev, h, u_prev, q_prev,
                    rule_off, rule_rhs, rule_fp, sym_next, fnext);
}

// When few phrases are new, one wave per word leaves most lanes idle: the new
// phrases are first listed in rank order (one thread per word walks its set
// bits, keeping a running right-hand-side offset) and then committed one
// thread per rule.
template <bool BYTES>
__global__ void k_new_list(uint64_t W, const uint64_t* __restrict__ newbits,
                           const uint64_t* __restrict__ wcnt_base,
                           const uint64_t* __restrict__ wlen_base, const uint64_t* __restrict__ key,
                           const uint32_t* __restrict__ plen, uint32_t* __restrict__ list,
                           uint64_t* __restrict__ qoff) {
  for (uint64_t w = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; w < W;
       w += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t bits = newbits[w];
    if (!bits) continue;
    uint64_t idx = wcnt_base[w], run = wlen_base[w];
    while (bits) {
      const uint64_t o = w * 64 + __builtin_ctzll(bits);
      bits &= bits - 1;
      list[idx] = (uint32_t)o;
      qoff[idx] = run;
      run += key_len<BYTES>(key[o], plen, o);
      ++idx;
    }
  }
}

template <typename Sym>
__global__ __launch_bounds__(256) void k_commit_list(uint64_t u_new, const uint32_t* __restrict__ list,
                                                     const uint64_t* __restrict__ qoff,
                                                     const uint32_t* __restrict__ slot_idx,
                                                     Slot* table, const uint64_t* __restrict__ key,
                                                     const uint64_t* __restrict__ wkey,
                                                     const uint64_t* __restrict__ pstart,
                                                     const uint32_t* __restrict__ plen,
                                                     const Sym* __restrict__ content,
                                                     const uint32_t* fnew,
                                                     const uint32_t* __restrict__ fprev, LevelHash h,
                                                     uint32_t u_prev, uint64_t q_prev,
                                                     uint64_t* __restrict__ rule_off,
                                                     Sym* __restrict__ rule_rhs,
                                                     uint32_t* __restrict__ rule_fp,
                                                     uint32_t* sym_next, uint32_t* fnext) {
  constexpr bool kBytes = sizeof(Sym) == 1;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < u_new;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t o = list[i];
    const uint64_t kk = key[o];
    commit_one<Sym>(o, u_prev + (uint32_t)i, q_prev + qoff[i], kk, key_len<kBytes>(kk, plen, o),
                    slot_idx[o], table, wkey, pstart, content, fnew, fprev, h, rule_off, rule_rhs,
                    rule_fp, sym_next, fnext);
  }
}

// T^{i+1}: every phrase takes the (now committed) rank of its slot, and its
// fingerprint when the next round needs it (fnext).  Four consecutive phrases
// per thread: 16-byte loads and stores, four table reads in flight.
constexpr int kRewriteItems = 4;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint64_t rank_and_fp(const Slot* __restrict__ table, uint32_t sidx) {
  // kNone only after an overflow (the round is redone)
  return sidx == kNone ? 0 : *reinterpret_cast<const uint64_t*>(&table[sidx].minocc);
}

// Phrases of the groups of four g = tid, tid + nthreads, ...  With newbits,
// the phrases flagged new were written by the commit (their rank and F are
// known there): their slots are not read; a group with some of them merges
// what the commit wrote, a group of four new ones is left as it is.
__device__ __forceinline__ void rewrite_range(uint64_t d, uint64_t tid, uint64_t nthreads,
                                              const uint32_t* __restrict__ slot_idx,
                                              const Slot* __restrict__ table,
                                              const uint64_t* __restrict__ newbits,
                                              uint32_t* sym_next, uint32_t* fnext) {
  for (uint64_t o = tid * kRewriteItems; o < d; o += nthreads * kRewriteItems) {
  const uint32_t nw =
      newbits ? (uint32_t)(newbits[o >> 6] >> (o & 63)) & ((1u << kRewriteItems) - 1u) : 0u;
  if (o + kRewriteItems <= d) {
    if (nw == (1u << kRewriteItems) - 1u) continue;
    // the phrase arrays stream past (non-temporal), the table lines stay cached
    const u32x4 si = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(slot_idx + o));
    const uint64_t f0 = nw & 1u ? 0 : rank_and_fp(table, si.x),
                   f1 = nw & 2u ? 0 : rank_and_fp(table, si.y),
                   f2 = nw & 4u ? 0 : rank_and_fp(table, si.z),
                   f3 = nw & 8u ? 0 : rank_and_fp(table, si.w);
    u32x4 sv = {(uint32_t)(f0 >> 32), (uint32_t)(f1 >> 32), (uint32_t)(f2 >> 32),
                (uint32_t)(f3 >> 32)};
    u32x4 fv = {(uint32_t)f0, (uint32_t)f1, (uint32_t)f2, (uint32_t)f3};
    if (nw) {
      const u32x4 sc = *reinterpret_cast<const u32x4*>(sym_next + o);
      sv.x = nw & 1u ? sc.x : sv.x;
      sv.y = nw & 2u ? sc.y : sv.y;
      sv.z = nw & 4u ? sc.z : sv.z;
      sv.w = nw & 8u ? sc.w : sv.w;
      if (fnext) {
        const u32x4 fc = *reinterpret_cast<const u32x4*>(fnext + o);
        fv.x = nw & 1u ? fc.x : fv.x;
        fv.y = nw & 2u ? fc.y : fv.y;
        fv.z = nw & 4u ? fc.z : fv.z;
        fv.w = nw & 8u ? fc.w : fv.w;
      }
    }
    __builtin_nontemporal_store(sv, reinterpret_cast<u32x4*>(sym_next + o));
    if (fnext) __builtin_nontemporal_store(fv, reinterpret_cast<u32x4*>(fnext + o));
  } else {
    for (uint64_t x = o; x < d; ++x) {
      if ((nw >> (x - o)) & 1u) continue;
      const uint64_t fr = rank_and_fp(table, slot_idx[x]);
      sym_next[x] = (uint32_t)(fr >> 32);
      if (fnext) fnext[x] = (uint32_t)fr;
    }
  }
  }
}

__global__ __launch_bounds__(256) void k_rewrite(uint64_t d, const uint64_t* __restrict__ d_dev,
                                                 const uint32_t* __restrict__ slot_idx,
                                                 const Slot* __restrict__ table,
                                                 const uint64_t* __restrict__ newbits,
                                                 uint32_t* sym_next, uint32_t* fnext) {
  if (d_dev) d = *d_dev;
  rewrite_range(d, blockIdx.x * (uint64_t)blockDim.x + threadIdx.x,
                (uint64_t)gridDim.x * blockDim.x, slot_idx, table, newbits, sym_next, fnext);
}

void launch_commit(bool bytes, uint64_t d, const uint64_t* d_dev, const uint32_t* slot_idx, Slot* table,
                   const uint64_t* newbits, const uint64_t* wcnt_base, const uint64_t* wlen_base,
                   const uint64_t* key, const uint64_t* wkey, const uint64_t* pstart,
                   const uint32_t* plen,
                   const void* content, const uint32_t* fnew, const uint32_t* fprev, LevelHash h,
                   uint32_t u_prev, uint64_t q_prev, uint64_t* rule_off, void* rule_rhs,
                   uint32_t* rule_fp, uint32_t* sym_next, uint32_t* fnext, uint64_t u_new,
                   uint32_t* nlist, uint64_t* nqoff, hipStream_t s) {
  if (!d) return;
  const unsigned g = grid_for((d + 63) / 64, 4);  // one wave per flag word
  // Where many phrases are new, the per-word commit also writes each new
  // phrase's own symbol and F of T^{i+1} (coalesced within its word) and the
  // rewrite skips their slots; the listed commit of rounds where few are new
  // would write them scattered, which costs more than the slot reads saved.
  if (!d_dev && nlist && nqoff && u_new * kCommitListRatio < d) {
    const uint64_t W = (d + 63) / 64;
    unsigned gw = grid_for(W, 256);
    if (gw > kPersistentBlocks) gw = kPersistentBlocks;
    unsigned gu = grid_for(u_new, 256);
    if (gu > kPersistentBlocks * 4) gu = kPersistentBlocks * 4;
    if (bytes) {
      k_new_list<true><<<gw, 256, 0, s>>>(W, newbits, wcnt_base, wlen_base, key, plen, nlist, nqoff);
      if (u_new)
        k_commit_list<uint8_t><<<gu, 256, 0, s>>>(
            u_new, nlist, nqoff, slot_idx, table, key, wkey, pstart, plen,
            static_cast<const uint8_t*>(content), fnew, fprev, h, u_prev, q_prev, rule_off,
            static_cast<uint8_t*>(rule_rhs), rule_fp, nullptr, nullptr);
    } else {
      k_new_list<false><<<gw, 256, 0, s>>>(W, newbits, wcnt_base, wlen_base, key, plen, nlist,
                                           nqoff);
      if (u_new)
        k_commit_list<uint32_t><<<gu, 256, 0, s>>>(
            u_new, nlist, nqoff, slot_idx, table, key, wkey, pstart, plen,
            static_cast<const uint32_t*>(content), fnew, fprev, h, u_prev, q_prev, rule_off,
            static_cast<uint32_t*>(rule_rhs), rule_fp, nullptr, nullptr);
    }
    LCG_LAUNCH_CHECK("commit_list");
    newbits = nullptr;  // the rewrite reads every phrase's slot
  } else if (bytes)
    k_commit_new<uint8_t><<<g, 256, 0, s>>>(
        d, d_dev, slot_idx, table, newbits, wcnt_base, wlen_base, key, wkey, pstart, plen,
        static_cast<const uint8_t*>(content), fnew, fprev, h, u_prev, q_prev, rule_off,
        static_cast<uint8_t*>(rule_rhs), rule_fp, sym_next, fnext);
  else
    k_commit_new<uint32_t><<<g, 256, 0, s>>>(
        d, d_dev, slot_idx, table, newbits, wcnt_base, wlen_base, key, wkey, pstart, plen,
        static_cast<const uint32_t*>(content), fnew, fprev, h, u_prev, q_prev, rule_off,
        static_cast<uint32_t*>(rule_rhs), rule_fp, sym_next, fnext);
  LCG_LAUNCH_CHECK("commit_new");
  if ((reinterpret_cast<uintptr_t>(slot_idx) | reinterpret_cast<uintptr_t>(sym_next) |
       reinterpret_cast<uintptr_t>(fnext)) & 15)
    throw std::runtime_error("rewrite arrays are not 16-byte aligned");
  k_rewrite<<<grid_for((d + kRewriteItems - 1) / kRewriteItems, 256), 256, 0, s>>>(
      d, d_dev, slot_idx, table, newbits, sym_next, fnext);
  LCG_LAUNCH_CHECK("rewrite");
}

// ------------------------------------------------------------------ rehash
// Committed rules with rank < rank_limit move to the new table; claims that
// were never committed (rank kNone) and rules at or above the limit are
// dropped.
__global__ void k_rehash(const Slot* __restrict__ old_t, uint64_t old_cap, Slot* new_t,
                         uint64_t mask, uint32_t rank_limit, Counters* ctr) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < old_cap;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const Slot sl = old_t[i];
    if (sl.w0 == kEmpty || sl.rank == kNone || sl.rank >= rank_limit) continue;
    uint64_t pos = mix64(probe_key(sl.w0)) & mask;
    bool done = false;
    for (uint64_t t = 0; t <= mask && !done; ++t) {
      unsigned long long prev = atomicCAS(reinterpret_cast<unsigned long long*>(&new_t[pos].w0),
                                          (unsigned long long)kEmpty, (unsigned long long)sl.w0);
      done = prev == kEmpty;
      if (done) {
        new_t[pos].minocc = sl.minocc;  // the committed rule's F
        new_t[pos].rank = sl.rank;
        new_t[pos].c0 = sl.c0;
        new_t[pos].c1 = sl.c1;
      }
      else pos = (pos + 1) & mask;
    }
    if (!done) atomicOr(&ctr->overflow, 1u);
  }
}

void launch_rehash(const Slot* old_t, uint64_t old_cap, Slot* new_t, uint64_t new_mask,
                   uint32_t rank_limit, Counters* ctr, hipStream_t s) {
  if (!old_cap) return;
  unsigned g = grid_for(old_cap, 256);
  if (g > 8192) g = 8192;
  k_rehash<<<g, 256, 0, s>>>(old_t, old_cap, new_t, new_mask, rank_limit, ctr);
  LCG_LAUNCH_CHECK("rehash");
}

// ------------------------------------------------------------------ strings
__global__ void k_c_init(const uint8_t* __restrict__ text, const uint64_t* __restrict__ off,
                         uint32_t k, uint8_t* __restrict__ c_level, uint32_t* __restrict__ c_sym) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  if (off[j + 1] - off[j] == 1) {
    c_level[j] = 0;
    c_sym[j] = text[off[j]];
  } else {
    c_level[j] = 0xFF;
    c_sym[j] = kNone;
  }
}

void launch_c_init(const uint8_t* text, const uint64_t* off, uint32_t k, uint8_t* c_level,
                   uint32_t* c_sym, hipStream_t s) {
  k_c_init<<<grid_for(k, 256), 256, 0, s>>>(text, off, k, c_level, c_sym);
  LCG_LAUNCH_CHECK("c_init");
}

// Next-round offsets: the phrases of string j start at the number of breaks
// before its first position (tile prefix + popcount inside the tile).
// Next-round offsets of strings j = tid, tid + nthreads, ... <= k.
__device__ __forceinline__ void segments_range(const uint64_t* __restrict__ off, uint32_t k,
                                               const uint64_t* __restrict__ bits,
                                               const uint64_t* __restrict__ tile_base, uint64_t d,
                                               uint64_t* __restrict__ new_off, uint64_t tid,
                                               uint64_t nthreads) {
  for (uint64_t j = tid; j <= k; j += nthreads) {
    if (j == k) {
      new_off[k] = d;
      continue;
    }
    const uint64_t x = off[j];
    const uint64_t tile = x / kTile;
    uint64_t r = tile_base[tile];
    for (uint64_t wd = tile * kTileWords; wd < (x >> 6); ++wd) r += __builtin_popcountll(bits[wd]);
    if (x & 63) r += __builtin_popcountll(bits[x >> 6] & ((1ULL << (x & 63)) - 1ULL));
    new_off[j] = r;
  }
}

__global__ void k_segments(const uint64_t* __restrict__ off, uint32_t k,
                           const uint64_t* __restrict__ bits, const uint64_t* __restrict__ tile_base,
                           uint64_t d, const uint64_t* __restrict__ d_dev,
                           uint64_t* __restrict__ new_off) {
  segments_range(off, k, bits, tile_base, d_dev ? *d_dev : d, new_off,
                 blockIdx.x * (uint64_t)blockDim.x + threadIdx.x, (uint64_t)gridDim.x * blockDim.x);
}

void launch_segments(const uint64_t* off, uint32_t k, const uint64_t* bits,
                     const uint64_t* tile_base, uint64_t d, const uint64_t* d_dev,
                     uint64_t* new_off, hipStream_t s) {
  k_segments<<<grid_for((uint64_t)k + 1, 256), 256, 0, s>>>(off, k, bits, tile_base, d, d_dev,
                                                             new_off);
  LCG_LAUNCH_CHECK("segments");
}

// Strings of the waves' groups of 64 (wave, wave + waves, ...): a string
// reduced to one symbol stores it in C; the others are counted as active.
__device__ __forceinline__ void finish_range(const uint64_t* __restrict__ off,
                                             const uint64_t* __restrict__ new_off, uint32_t k,
                                             const uint32_t* __restrict__ sym_next,
                                             uint32_t level, uint8_t* __restrict__ c_level,
                                             uint32_t* __restrict__ c_sym,
                                             Counters* __restrict__ ctr, uint64_t wave,
                                             uint64_t waves) {
  for (uint64_t w = wave; (w << 6) < k; w += waves) {
    const uint64_t j = (w << 6) + (threadIdx.x & 63);
    unsigned long long act = 0, act_len = 0;
    if (j < k) {
      const uint64_t lo = off[j + 1] - off[j];
      const uint64_t ln = new_off[j + 1] - new_off[j];
      if (lo >= 2 && ln == 1) {
        c_level[j] = (uint8_t)level;
        c_sym[j] = sym_next[new_off[j]];
      }
      act = ln >= 2;
      act_len = ln >= 2 ? ln : 0;
    }
    act = wave_sum(act);
    act_len = wave_sum(act_len);
    if ((threadIdx.x & 63) == 0 && act) {
      atomicAdd(&ctr->active, (unsigned int)act);
      atomicAdd(&ctr->active_len, act_len);
    }
  }
}

__global__ void k_finish(const uint64_t* __restrict__ off, const uint64_t* __restrict__ new_off,
                         uint32_t k, const uint32_t* __restrict__ sym_next, uint32_t level,
                         uint8_t* __restrict__ c_level, uint32_t* __restrict__ c_sym,
                         Counters* __restrict__ ctr) {
  finish_range(off, new_off, k, sym_next, level, c_level, c_sym, ctr,
               blockIdx.x * (uint64_t)(blockDim.x / 64) + (threadIdx.x >> 6),
               (uint64_t)gridDim.x * (blockDim.x / 64));
}

void launch_finish(const uint64_t* off, const uint64_t* new_off, uint32_t k,
                   const uint32_t* sym_next, uint32_t level, uint8_t* c_level, uint32_t* c_sym,
                   Counters* ctr, hipStream_t s) {
  k_finish<<<grid_for(k, 256), 256, 0, s>>>(off, new_off, k, sym_next, level, c_level, c_sym, ctr);
  LCG_LAUNCH_CHECK("finish");
}

// ------------------------------------------------------------------ merge
template <typename Sym>
__global__ void k_merge_prepare(uint32_t u_b, const uint64_t* __restrict__ b_off,
                                const Sym* __restrict__ b_rhs, const uint32_t* __restrict__ remap_prev,
                                const uint32_t* __restrict__ f_prev, LevelHash h, uint32_t key_bits,
                                Sym* __restrict__ content, uint64_t* __restrict__ pstart,
                                uint32_t* __restrict__ plen, uint64_t* __restrict__ key,
                                uint64_t* __restrict__ wkey) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= u_b) return;
  const uint64_t p0 = b_off[r], p1 = b_off[r + 1];
  for (uint64_t x = p0; x < p1; ++x) {
    Sym v = b_rhs[x];
    if (remap_prev) v = (Sym)remap_prev[v];
    content[x] = v;
  }
  uint64_t S = 0;
  for (uint64_t x = p1; x-- > p0;) S = addmod61(mulmod61(S, h.c), f_prev[content[x]]);
  const uint64_t P = addmod61(mulmod61(h.a, S), h.b);
  pstart[r] = p0;
  plen[r] = (uint32_t)(p1 - p0);
  key[r] = make_key<sizeof(Sym) == 1>(content, p0, p1 - p0, P, key_bits, wkey + 2 * (uint64_t)r);
}

void launch_merge_prepare(bool bytes, uint32_t u_b, const uint64_t* b_off, const void* b_rhs,
                          const uint32_t* remap_prev, const uint32_t* f_prev, LevelHash h,
                          uint32_t key_bits, void* content, uint64_t* pstart, uint32_t* plen,
                          uint64_t* key, uint64_t* wkey, hipStream_t s) {
  if (!u_b) return;
  if (bytes)
    k_merge_prepare<uint8_t><<<grid_for(u_b, 256), 256, 0, s>>>(
        u_b, b_off, static_cast<const uint8_t*>(b_rhs), nullptr, f_prev, h, key_bits,
        static_cast<uint8_t*>(content), pstart, plen, key, wkey);
  else
    k_merge_prepare<uint32_t><<<grid_for(u_b, 256), 256, 0, s>>>(
        u_b, b_off, static_cast<const uint32_t*>(b_rhs), remap_prev, f_prev, h, key_bits,
        static_cast<uint32_t*>(content), pstart, plen, key, wkey);
  LCG_LAUNCH_CHECK("merge_prepare");
}

__global__ void k_c_merge(const uint8_t* __restrict__ b_level, const uint32_t* __restrict__ b_sym,
                          uint32_t kb, uint32_t level, const uint32_t* __restrict__ remap,
                          uint8_t* __restrict__ out_level, uint32_t* __restrict__ out_sym) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= kb) return;
  const uint8_t L = b_level[j];
  if (level == 0) {
    out_level[j] = L;
    if (L == 0) out_sym[j] = b_sym[j];
  } else if (L == level) {
    out_sym[j] = remap[b_sym[j]];
  }
}

void launch_c_merge(const uint8_t* b_level, const uint32_t* b_sym, uint32_t kb, uint32_t level,
                    const uint32_t* remap, uint8_t* out_level, uint32_t* out_sym, hipStream_t s) {
  if (!kb) return;
  k_c_merge<<<grid_for(kb, 256), 256, 0, s>>>(b_level, b_sym, kb, level, remap, out_level, out_sym);
  LCG_LAUNCH_CHECK("c_merge");
}

// ------------------------------------------------------------------ expand
__global__ void k_expand_lens(const uint32_t* __restrict__ cur, uint64_t m,
                              const uint64_t* __restrict__ rule_off, uint64_t* __restrict__ lens) {
  const uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (x >= m) return;
  const uint32_t r = cur[x];
  lens[x] = rule_off[r + 1] - rule_off[r];
}

void launch_expand_lens(const uint32_t* cur, uint64_t m, const uint64_t* rule_off, uint64_t* lens,
                        hipStream_t s) {
  if (!m) return;
  k_expand_lens<<<grid_for(m, 256), 256, 0, s>>>(cur, m, rule_off, lens);
  LCG_LAUNCH_CHECK("expand_lens");
}

template <typename Sym>
__global__ void k_expand_emit(const uint32_t* __restrict__ cur, uint64_t m,
                              const uint64_t* __restrict__ rule_off, const Sym* __restrict__ rule_rhs,
                              const uint64_t* __restrict__ pos, Sym* __restrict__ next) {
  const uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (x >= m) return;
  const uint32_t r = cur[x];
  const uint64_t p0 = rule_off[r], p1 = rule_off[r + 1];
  const uint64_t dst = pos[x];
  for (uint64_t t = p0; t < p1; ++t) next[dst + (t - p0)] = rule_rhs[t];
}

void launch_expand_emit(bool bytes, const uint32_t* cur, uint64_t m, const uint64_t* rule_off,
                        const void* rule_rhs, const uint64_t* pos, void* next, hipStream_t s) {
  if (!m) return;
  if (bytes)
    k_expand_emit<uint8_t><<<grid_for(m, 256), 256, 0, s>>>(
        cur, m, rule_off, static_cast<const uint8_t*>(rule_rhs), pos, static_cast<uint8_t*>(next));
  else
    k_expand_emit<uint32_t><<<grid_for(m, 256), 256, 0, s>>>(
        cur, m, rule_off, static_cast<const uint32_t*>(rule_rhs), pos, static_cast<uint32_t*>(next));
  LCG_LAUNCH_CHECK("expand_emit");
}

// ------------------------------------------------------------------ expand many strings
// Expansion of a range of strings at once, top-down, by byte positions.
// Every rule's expansion length in bytes (E, per level, bottom-up) lets each
// symbol carry the byte position of its expansion; a level's symbols become
// their right-hand sides (symbol, position) in any order, so no scan is
// needed, and the level-1 symbols write their bytes at their positions.

// E of the level's rules: E_1[r] = |rhs(r)|, E_L[r] = sum of E_{L-1} over rhs(r)
__global__ void k_explen(const uint64_t* __restrict__ rule_off, const uint32_t* __restrict__ rhs,
                         const uint64_t* __restrict__ e_below, uint32_t u,
                         uint64_t* __restrict__ e) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= u) return;
  const uint64_t p0 = rule_off[r], p1 = rule_off[r + 1];
  if (!e_below) {
    e[r] = p1 - p0;
    return;
  }
  uint64_t sum = 0;
  for (uint64_t t = p0; t < p1; ++t) sum += e_below[rhs[t]];
  e[r] = sum;
}

void launch_explen(const uint64_t* rule_off, const uint32_t* rhs, const uint64_t* e_below,
                   uint32_t u, uint64_t* e, hipStream_t s) {
  if (!u) return;
  k_explen<<<grid_for(u, 256), 256, 0, s>>>(rule_off, rhs, e_below, u, e);
  LCG_LAUNCH_CHECK("explen");
}

// byte length of each string of the range (from its C entry)
__global__ void k_xs_strlen(const uint8_t* __restrict__ c_level, const uint32_t* __restrict__ c_sym,
                            uint32_t ks, const uint64_t* const* __restrict__ e_levels,
                            uint64_t* __restrict__ len) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ks) return;
  const uint32_t lv = c_level[s];
  len[s] = lv == 0 ? 1 : e_levels[lv - 1][c_sym[s]];
}

// strings whose C entry is at `level` join the level's items (level >= 1),
// or write their byte (level 0)
__global__ void k_xs_enter(const uint8_t* __restrict__ c_level, const uint32_t* __restrict__ c_sym,
                           uint32_t ks, uint32_t level, const uint64_t* __restrict__ str_off,
                           uint32_t* __restrict__ sym, uint64_t* __restrict__ pos,
                           unsigned long long* __restrict__ count, uint8_t* __restrict__ out) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ks || c_level[s] != level) return;
  if (level == 0) {
    out[str_off[s]] = (uint8_t)c_sym[s];
    return;
  }
  const unsigned long long at = atomicAdd(count, 1ULL);
  sym[at] = c_sym[s];
  pos[at] = str_off[s];
}

// children count of the level's items (sum of right-hand-side lengths)
__global__ __launch_bounds__(256) void k_xs_count(const uint32_t* __restrict__ sym, uint64_t m,
                                                  const uint64_t* __restrict__ rule_off,
                                                  unsigned long long* __restrict__ total) {
  unsigned long long c = 0;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < m;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t r = sym[i];
    c += rule_off[r + 1] - rule_off[r];
  }
  c = wave_sum(c);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(total, c);
}

// the level's items -> their children (TO_BYTES: level 1 -> bytes at their
// positions).  One thread per item: a block scan of the items' right-hand-side
// lengths and one atomicAdd per block reserve the children, which each thread
// then writes in order with their positions (the item's position plus the
// expansion lengths of the siblings before).  The grandchildren are counted
// on the way into *gcount from gc_rule (per rule: the right-hand-side lengths
// of its children summed; NULL when the children are level-1 rules).
template <bool TO_BYTES>
__global__ __launch_bounds__(kBlock) void k_xs_expand(const uint32_t* __restrict__ sym,
                                                      const uint64_t* __restrict__ pos, uint64_t m,
                                                      const uint64_t* __restrict__ rule_off,
                                                      const void* __restrict__ rule_rhs,
                                                      const uint64_t* __restrict__ e_below,
                                                      const uint64_t* __restrict__ gc_rule,
                                                      uint32_t* __restrict__ nsym,
                                                      uint64_t* __restrict__ npos,
                                                      unsigned long long* __restrict__ ncount,
                                                      unsigned long long* __restrict__ gcount,
                                                      uint8_t* __restrict__ out) {
  __shared__ unsigned long long s_wave[kBlock / 64];
  __shared__ unsigned long long s_base;
  unsigned long long gc = 0;
  for (uint64_t b0 = blockIdx.x * (uint64_t)kBlock; b0 < m; b0 += (uint64_t)gridDim.x * kBlock) {
    const uint64_t i = b0 + threadIdx.x;
    uint64_t a = 0, q = 0, p = 0;
    uint32_t r = 0;
    if (i < m) {
      r = sym[i];
      p = pos[i];
      a = rule_off[r];
      q = rule_off[r + 1] - a;
    }
    if constexpr (TO_BYTES) {
      const uint8_t* rhs = static_cast<const uint8_t*>(rule_rhs) + a;
      for (uint64_t k = 0; k < q; ++k) out[p + k] = rhs[k];
    } else {
      if (i < m && gc_rule) gc += gc_rule[r];
      unsigned long long tot = 0;
      const unsigned long long excl = block_excl_scan<unsigned long long>(q, s_wave, &tot);
      if (threadIdx.x == 0) s_base = atomicAdd(ncount, tot);
      __syncthreads();
      const uint64_t o = s_base + excl;
      const uint32_t* rhs = static_cast<const uint32_t*>(rule_rhs) + a;
      uint64_t pp = p;
      for (uint64_t k = 0; k < q; ++k) {
        const uint32_t ch = rhs[k];
        nsym[o + k] = ch;
        npos[o + k] = pp;
        pp += e_below[ch];
      }
      __syncthreads();  // s_base is rewritten by the next iteration
    }
  }
  if constexpr (!TO_BYTES) {
    gc = wave_sum(gc);
    if ((threadIdx.x & 63) == 0 && gc && gcount) atomicAdd(gcount, gc);
  }
}

// level-2 items -> bytes: each child (a level-1 rule) has its bytes copied in
// place, so the level-1 occurrences are never materialised as items
__global__ __launch_bounds__(kBlock) void k_xs_bytes2(const uint32_t* __restrict__ sym,
                                                      const uint64_t* __restrict__ pos, uint64_t m,
                                                      const uint64_t* __restrict__ off2,
                                                      const uint32_t* __restrict__ rhs2,
                                                      const uint64_t* __restrict__ off1,
                                                      const uint8_t* __restrict__ rhs1,
                                                      uint8_t* __restrict__ out) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < m;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t r = sym[i];
    uint64_t p = pos[i];
    const uint64_t b = off2[r + 1];
    for (uint64_t t = off2[r]; t < b; ++t) {
      const uint32_t c = rhs2[t];
      const uint64_t b1 = off1[c + 1];
      for (uint64_t x = off1[c]; x < b1; ++x) out[p++] = rhs1[x];
    }
  }
}

void launch_xs_bytes2(const uint32_t* sym, const uint64_t* pos, uint64_t m, const uint64_t* off2,
                      const uint32_t* rhs2, const uint64_t* off1, const uint8_t* rhs1, uint8_t* out,
                      hipStream_t s) {
  if (!m) return;
  unsigned g = grid_for(m, kBlock);
  const unsigned r = resident_blocks((const void*)k_xs_bytes2, kBlock);
  if (g > r) g = r;
  k_xs_bytes2<<<g, kBlock, 0, s>>>(sym, pos, m, off2, rhs2, off1, rhs1, out);
  LCG_LAUNCH_CHECK("xs_bytes2");
}

// per rule of a level L >= 2: the summed right-hand-side lengths of its
// children (rules of level L-1, offsets off_below)
__global__ void k_gc(const uint64_t* __restrict__ rule_off, const uint32_t* __restrict__ rhs,
                     const uint64_t* __restrict__ off_below, uint32_t u, uint64_t* __restrict__ gc) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= u) return;
  uint64_t sum = 0;
  for (uint64_t t = rule_off[r]; t < rule_off[r + 1]; ++t) {
    const uint32_t c = rhs[t];
    sum += off_below[c + 1] - off_below[c];
  }
  gc[r] = sum;
}

void launch_gc(const uint64_t* rule_off, const uint32_t* rhs, const uint64_t* off_below, uint32_t u,
               uint64_t* gc, hipStream_t s) {
  if (!u) return;
  k_gc<<<grid_for(u, 256), 256, 0, s>>>(rule_off, rhs, off_below, u, gc);
  LCG_LAUNCH_CHECK("gc");
}

void launch_xs_strlen(const uint8_t* c_level, const uint32_t* c_sym, uint32_t ks,
                      const uint64_t* const* e_levels, uint64_t* len, hipStream_t s) {
  if (!ks) return;
  k_xs_strlen<<<grid_for(ks, 256), 256, 0, s>>>(c_level, c_sym, ks, e_levels, len);
  LCG_LAUNCH_CHECK("xs_strlen");
}

void launch_xs_enter(const uint8_t* c_level, const uint32_t* c_sym, uint32_t ks, uint32_t level,
                     const uint64_t* str_off, uint32_t* sym, uint64_t* pos, uint64_t* count,
                     uint8_t* out, hipStream_t s) {
  if (!ks) return;
  k_xs_enter<<<grid_for(ks, 256), 256, 0, s>>>(c_level, c_sym, ks, level, str_off, sym, pos,
                                               reinterpret_cast<unsigned long long*>(count), out);
  LCG_LAUNCH_CHECK("xs_enter");
}

void launch_xs_count(const uint32_t* sym, uint64_t m, const uint64_t* rule_off, uint64_t* total,
                     hipStream_t s) {
  if (!m) return;
  unsigned g = grid_for(m, 256);
  if (g > kPersistentBlocks) g = kPersistentBlocks;
  k_xs_count<<<g, 256, 0, s>>>(sym, m, rule_off, reinterpret_cast<unsigned long long*>(total));
  LCG_LAUNCH_CHECK("xs_count");
}

void launch_xs_expand(bool to_bytes, const uint32_t* sym, const uint64_t* pos, uint64_t m,
                      const uint64_t* rule_off, const void* rule_rhs, const uint64_t* e_below,
                      const uint64_t* gc_rule, uint32_t* nsym, uint64_t* npos,
                      uint64_t* ncount, uint64_t* gcount, uint8_t* out, hipStream_t s) {
  if (!m) return;
  unsigned g = grid_for(m, kBlock);
  const unsigned r = resident_blocks(to_bytes ? (const void*)k_xs_expand<true>
                                              : (const void*)k_xs_expand<false>, kBlock);
  if (g > r) g = r;
  auto nc = reinterpret_cast<unsigned long long*>(ncount);
  auto gc = reinterpret_cast<unsigned long long*>(gcount);
  if (to_bytes)
    k_xs_expand<true><<<g, kBlock, 0, s>>>(sym, pos, m, rule_off, rule_rhs, e_below,
                                           gc_rule, nsym, npos, nc, gc, out);
  else
    k_xs_expand<false><<<g, kBlock, 0, s>>>(sym, pos, m, rule_off, rule_rhs, e_below,
                                            gc_rule, nsym, npos, nc, gc, out);
  LCG_LAUNCH_CHECK("xs_expand");
}

// ------------------------------------------------------------------ fused tail
// The short rounds (the tail) in one cooperative launch: the phases of a
// round (tile map, classify, tile scan, emit, insert, first-occurrence flags,
// rank scans, commit, rewrite and segments, finish) run one after another
// over the whole grid, separated by grid-wide barriers, with the same device
// functions as the separate kernels.  After each round every block reads the
// count of strings still active and the loop stops, uniformly, at zero.
//
// Blocks on different XCDs do not share an L2: the grid barrier's own
// agent-scope fences (one thread per block, after a block barrier) write the
// block's L2 back before it arrives and invalidate its caches after it
// leaves, so that reads after the barrier see what other blocks wrote.
union TailLds {
  ClassifyLds classify;
  EmitLds<true> emit_bytes;
  EmitLds<false> emit_ranks;
  ScanLds scan;
  unsigned long long sum[4];
};

__device__ __forceinline__ void grid_barrier(cooperative_groups::grid_group& grid) {
  grid.sync();
}

template <bool BYTES>
__device__ __forceinline__ void tail_round(const TailArgs& a, const TailRound& R,
                                           const uint64_t* cur_off, uint64_t n, int cur,
                                           cooperative_groups::grid_group& grid, TailLds& sh) {
  using Sym = typename std::conditional<BYTES, uint8_t, uint32_t>::type;
  const uint64_t B = gridDim.x, bid = blockIdx.x;
  const uint64_t T = B * blockDim.x, tid = bid * blockDim.x + threadIdx.x;
  const uint64_t NW = B * (blockDim.x / 64), wid = bid * (blockDim.x / 64) + (threadIdx.x >> 6);
  RoundIn in;
  in.sym = BYTES ? (const void*)a.text : (const void*)a.sym[cur ^ 1];
  in.fp = BYTES ? nullptr : a.fpv[cur ^ 1];
  in.lut = a.lut;
  in.off = cur_off;
  in.k = a.k;
  in.n = n;
  in.n_dev = nullptr;
  in.bytes = BYTES;
  const Sym* content = static_cast<const Sym*>(in.sym);
  const uint64_t tiles = (n + kTile - 1) / kTile;
  // tile map, then break bits and counts per tile
  tile_seg_range(cur_off, a.k, n, a.tile_seg, tid, T);
  grid_barrier(grid);
  for (uint64_t t = bid; t < tiles; t += B) {
    __syncthreads();
    classify_tile<BYTES>(in, t, a.bits, a.tile_cnt, a.tile_seg, sh.classify);
  }
  grid_barrier(grid);
  if (bid == 0) scan_block(a.tile_cnt, a.tile_base, tiles, &R.rec->d, sh.scan);
  grid_barrier(grid);
  const uint64_t d = R.rec->d;
  // phrases: keys, fingerprints of long ones
  if constexpr (BYTES)
    emit_tiles<true>(in, tiles, bid, B, a.bits, a.tile_base, a.tile_seg, R.h, a.key_bits, a.pstart,
                     a.plen, a.key, a.wkey, a.fpv[cur], nullptr, sh.emit_bytes);
  else
    emit_tiles<false>(in, tiles, bid, B, a.bits, a.tile_base, a.tile_seg, R.h, a.key_bits,
                      a.pstart, a.plen, a.key, a.wkey, a.fpv[cur], nullptr, sh.emit_ranks);
  grid_barrier(grid);
  insert_phrases<Sym, false>(bid, B, 0, d, d, nullptr, nullptr, nullptr, a.key, a.wkey, a.pstart,
                             a.plen, content, R.rule_off, static_cast<const Sym*>(R.rule_rhs),
                             R.u0, R.table, R.mask, a.slot_idx, nullptr, 0, nullptr, &R.rec->ctr,
                             sh.sum);
  grid_barrier(grid);
  newflags_words<BYTES>(d, wid, NW, a.slot_idx, R.table, a.key, a.plen, a.newbits, a.wcnt, a.wlen);
  grid_barrier(grid);
  const uint64_t W = (d + 63) / 64;
  if (bid == 0) scan_block(a.wcnt, a.wcnt_base, W, &R.rec->u, sh.scan);
  if (bid == (B > 1 ? 1 : 0)) {
    __syncthreads();
    scan_block(a.wlen, a.wlen_base, W, &R.rec->q, sh.scan);
  }
  grid_barrier(grid);
  commit_words<Sym>(d, wid, NW, a.slot_idx, R.table, a.newbits, a.wcnt_base, a.wlen_base, a.key,
                    a.wkey, a.pstart, a.plen, content, a.fpv[cur], R.fprev, R.h, R.u0, R.q0,
                    R.rule_off, static_cast<Sym*>(R.rule_rhs), R.rule_fp, nullptr, nullptr);
  grid_barrier(grid);
  rewrite_range(d, tid, T, a.slot_idx, R.table, nullptr, a.sym[cur], a.fpv[cur]);
  segments_range(cur_off, a.k, a.bits, a.tile_base, d, a.off[cur], tid, T);
  grid_barrier(grid);
  finish_range(cur_off, a.off[cur], a.k, a.sym[cur], R.level, a.c_level, a.c_sym, &R.rec->fin,
               wid, NW);
  grid_barrier(grid);
}

__global__ __launch_bounds__(kBlock) void k_tail(TailArgs a) {
  __shared__ TailLds sh;
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  const uint64_t* cur_off = a.off0;
  uint64_t n = a.n0;
  int cur = a.cur0;
  uint32_t r = 0;
  while (r < a.nrounds) {
    const TailRound& R = a.rounds[r];
    if (r == 0 && a.first_bytes) tail_round<true>(a, R, cur_off, n, cur, grid, sh);
    else tail_round<false>(a, R, cur_off, n, cur, grid, sh);
    ++r;
    // the same values for every block: written before the last barrier
    const uint32_t still = R.rec->fin.active;
    n = R.rec->d;
    cur_off = a.off[cur];
    cur ^= 1;
    if (!still) break;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *a.rounds_run = r;
}

unsigned tail_grid() {
  return resident_blocks((const void*)k_tail, kBlock);
}

void launch_tail(const TailArgs& a, unsigned grid, hipStream_t s) {
  if (!grid || grid > tail_grid()) throw std::runtime_error("fused tail: grid not co-resident");
  TailArgs args = a;
  void* kargs[] = {&args};
  const hipError_t e = hipLaunchCooperativeKernel((const void*)k_tail, dim3(grid), dim3(kBlock),
                                                  kargs, 0, s);
  if (e != hipSuccess)
    throw std::runtime_error(std::string("launch of the fused tail: ") + hipGetErrorString(e));
}

}  // namespace lcg
