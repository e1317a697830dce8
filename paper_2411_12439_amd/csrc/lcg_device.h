// Device-side building blocks of liblcg: Mersenne-61 arithmetic for the
// level fingerprints (Eq. 2 and Eq. 4 of the paper), the 64-bit dictionary
// keys, and the dictionary slot layout.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lcg {

constexpr uint64_t kP61 = (1ULL << 61) - 1;  // p_i of every level
constexpr uint64_t kEmpty = ~0ULL;           // free dictionary slot
constexpr uint32_t kNone = 0xFFFFFFFFu;      // no rank / no occurrence
constexpr uint64_t kLongTag = 1ULL << 63;    // key bit 63: not a short exact key
constexpr uint64_t kWideTag = 1ULL << 62;    // with bit 63: wide exact key (content in the slot)
constexpr uint64_t kHiMask = 0xFFFFFFFF00000000ULL;

// One dictionary slot (32 bytes).  w0 is the claimed word:
//   short phrase : exact key (bit 63 = 0), never equal to kEmpty;
//   wide phrase  : kLongTag | kWideTag | qcode << 59 | bcode << 57 | h25 << 32
//                  | ref, the content in c0, c1 (see wide keys below);
//   long phrase  : kLongTag | h30 << 32 | ref, where h30 is 30 bits of the
//                  phrase fingerprint;
// ref is the phrase occurrence that claimed the slot while the round runs,
// or the rule's rank once committed.
// While the rule is uncommitted (rank == kNone), minocc is the smallest
// occurrence index holding the phrase in the running round (its first
// occurrence); once committed, the same word holds the rule's fingerprint F,
// so that (F, rank) is one 8-byte load.  c0, c1 hold a wide phrase's content
// (kEmpty until its claimer has written them); other slots leave them empty.
struct Slot {
  uint64_t w0;
  uint32_t minocc;
  uint32_t rank;
  uint64_t c0, c1;
};
static_assert(sizeof(Slot) == 32, "slot layout");

// Coefficients of one level of the hash family.
struct LevelHash {
  uint64_t a, b, c;
};

// x * y mod 2^61-1 for x, y < 2^61: the 122-bit product is folded with
// 2^61 = 1 (mod p).
__device__ __forceinline__ uint64_t mulmod61(uint64_t x, uint64_t y) {
  uint64_t lo = x * y;
  uint64_t hi = __umul64hi(x, y);
  uint64_t r = (lo & kP61) + ((lo >> 61) | (hi << 3));
  r = (r & kP61) + (r >> 61);
  return r >= kP61 ? r - kP61 : r;
}

__device__ __forceinline__ uint64_t addmod61(uint64_t x, uint64_t y) {
  uint64_t r = x + y;
  return r >= kP61 ? r - kP61 : r;
}

// MurmurHash3's 64-bit finaliser (Appleby), used to place keys in the table.
__host__ __device__ __forceinline__ uint64_t mix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdULL;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ULL;
  k ^= k >> 33;
  return k;
}

// The part of w0 that decides where a key lives and what a probe compares.
__host__ __device__ __forceinline__ uint64_t probe_key(uint64_t w0) {
  return (w0 & kLongTag) ? (w0 & kHiMask) : w0;
}

// Exact keys.  Level 1 (bytes): up to 7 bytes, q in bits 56..58.  Levels >= 2
// (ranks): q in bits 58..60 and the ranks packed in 58 bits when they fit
// (q = 1 any rank; q = 2 ranks < 2^29; q = 3 ranks < 2^19; q = 4 ranks < 2^14).
// The encoding is injective per level, so equal keys mean equal phrases.
__device__ __forceinline__ int rank_bits_for(uint32_t q) {
  return q == 1 ? 32 : q == 2 ? 29 : q == 3 ? 19 : q == 4 ? 14 : 0;
}

// The long-phrase key: tag plus 30 bits of the 61-bit fingerprint P
// (optionally truncated by the key_bits test hook).
__device__ __forceinline__ uint64_t long_key(uint64_t P, uint32_t key_bits) {
  uint64_t h = (P >> 29) & 0x3FFFFFFFULL;
  if (key_bits) h &= (1ULL << key_bits) - 1;
  return kLongTag | (h << 32);
}

// Wide exact keys: phrases too long for a short key but whose content fits
// two 62-bit words c0, c1 (bit 63 of both stays clear, so a valid word never
// equals kEmpty).  Level 1: 8..14 bytes, seven in each word (qcode = q - 8).
// Levels >= 2: up to eight ranks, packed at the smallest width b of
// {12, 16, 20, 31} bits that holds every rank of the phrase (bcode 0..3),
// 5, 3, 3 or 2 ranks per word (so at most 8, 6, 6 or 4 ranks; qcode = q - 1).
// The width depends on the phrase alone, so equal phrases get equal keys and
// equal (qcode, bcode, c0, c1) means equal phrases.  The key word carries the
// tags, qcode, bcode and 25 bits of a mix of the content, which place the
// phrase in the table; a match of the key word is confirmed on c0, c1.
constexpr uint64_t kWideMaxBytes = 14;
constexpr uint32_t kWideMaxRanks = 8;
__host__ __device__ __forceinline__ uint32_t wide_bits(uint32_t bcode) {
  return bcode == 0 ? 12u : bcode == 1 ? 16u : bcode == 2 ? 20u : 31u;
}
__host__ __device__ __forceinline__ uint32_t wide_per_word(uint32_t bcode) {
  return bcode == 0 ? 5u : bcode == 3 ? 2u : 3u;
}
__host__ __device__ __forceinline__ uint64_t wide_key(uint64_t qcode, uint64_t bcode, uint64_t c0,
                                                      uint64_t c1) {
  const uint64_t h =
      mix64(c0 * 0x9E3779B97F4A7C15ULL ^ c1 ^ (qcode << 60) ^ (bcode << 56)) >> 39;  // 25 bits
  return kLongTag | kWideTag | (qcode << 59) | (bcode << 57) | (h << 32);
}
__host__ __device__ __forceinline__ bool is_wide(uint64_t kk) {
  return (kk & (kLongTag | kWideTag)) == (kLongTag | kWideTag);
}
__host__ __device__ __forceinline__ bool is_long(uint64_t kk) {
  return (kk & (kLongTag | kWideTag)) == kLongTag;
}
__host__ __device__ __forceinline__ uint32_t wide_qcode(uint64_t kk) {
  return (uint32_t)((kk >> 59) & 7);
}
__host__ __device__ __forceinline__ uint32_t wide_bcode(uint64_t kk) {
  return (uint32_t)((kk >> 57) & 3);
}

// Exclusive scan of one value per thread over a block of THREADS threads
// (a multiple of 64): wave prefix by shuffles, then the waves' totals from
// LDS (s_wave: THREADS / 64 values).  *total (if given) receives the block's
// sum.  Every thread of the block must call it.
template <typename T, int THREADS = 256>
__device__ __forceinline__ T block_excl_scan(T v, T* s_wave, T* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) s_wave[wid] = x;
  __syncthreads();
  T base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < THREADS / 64; ++w) {
    T sw = s_wave[w];
    if (w < wid) base += sw;
    tot += sw;
  }
  __syncthreads();
  if (total) *total = tot;
  return base + x - v;
}

}  // namespace lcg
