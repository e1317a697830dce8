// Host-side launchers of the liblcg HIP kernels (defined in lcg_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lcg_device.h"

namespace lcg {

constexpr int kBlock = 256;                 // threads per block of the position kernels
constexpr int kItems = 16;                  // positions per thread
constexpr int kTile = kBlock * kItems;      // positions per tile (4096)
constexpr int kTileWords = kTile / 64;      // break-bit words per tile
constexpr int kHllLog2 = 9;                 // HyperLogLog registers (512)
constexpr int kHll = 1 << kHllLog2;
constexpr unsigned kEmitBlocks = 2048;      // grid of the emit kernel (HLL partials: kEmitBlocks x kHll bytes)

// Device counters of one round.
struct Counters {
  unsigned long long won;       // slots claimed in the running insert
  unsigned long long probes;    // slots inspected
  unsigned long long compares;  // full right-hand-side comparisons
  unsigned int overflow;        // phrases whose probe sequence ran out of budget
  unsigned int active;          // strings still longer than one symbol
  unsigned long long active_len;  // their total length
  unsigned int rest_len;        // phrases left to the plain insert by the combining one
  unsigned int won_len;         // slots claimed in the running insert (entries of its won list)
  unsigned int hll[kHll];       // HyperLogLog registers of the round's phrase keys
};

// What the device records of one round run without host reads (tail mode).
struct TailRec {
  uint64_t d;    // phrases (the length of the next round's sequence)
  uint64_t u;    // new rules
  uint64_t q;    // new right-hand-side symbols
  uint64_t pad;
  Counters ctr;  // dictionary counters
  Counters fin;  // strings still longer than one symbol after the round
};

// Strings a tile of kTile positions overlaps (lo..hi) and the offsets of
// string lo.
struct TileSeg {
  uint32_t lo, hi;
  uint64_t start, end;
};

// Everything one round of the position kernels needs.
struct RoundIn {
  const void* sym;          // uint8_t (level 1) or uint32_t symbols of T^i
  const uint32_t* fp;       // F of each symbol (levels >= 2); NULL at level 1
  const uint32_t* lut;      // h^0 of the 256 byte values (level 1)
  const uint64_t* off;      // k+1 segment offsets of T^i
  uint32_t k;
  uint64_t n;               // length of T^i (a bound of it when n_dev is set)
  const uint64_t* n_dev;    // NULL, or the length of T^i in device memory
  bool bytes;               // symbols are bytes
};

void launch_f0_lut(uint32_t* lut, uint64_t a0, uint64_t b0, hipStream_t s);
void launch_fill_slots(Slot* t, uint64_t cap, hipStream_t s);
void launch_zero(void* p, size_t bytes, hipStream_t s);

void launch_classify(const RoundIn& in, uint64_t* bits, uint64_t* tile_cnt, TileSeg* tile_seg,
                     hipStream_t s);
void launch_emit(const RoundIn& in, const uint64_t* bits, const uint64_t* tile_base,
                 const TileSeg* tile_seg, LevelHash h,
                 uint32_t key_bits, uint64_t* pstart, uint32_t* plen, uint64_t* key, uint64_t* wkey,
                 uint32_t* fnew, uint8_t* hll_part, Counters* ctr, hipStream_t s);

// Exclusive scan of n uint64 values into out[0..n]; out[n] receives the total.
// tmp must hold scan_tmp_words(n) uint64.
size_t scan_tmp_words(uint64_t n);
void scan_exclusive(const uint64_t* in, uint64_t* out, uint64_t n, uint64_t* tmp, hipStream_t s);
// One-block exclusive scan of count = ceil(*x_dev / 2^shift) values (count
// itself without x_dev); out[count] and *total (if given) receive the sum.
void scan_one(const uint64_t* in, uint64_t* out, uint64_t count, const uint64_t* x_dev, int shift,
              uint64_t* total, hipStream_t s);

// combine: the rounds where few keys take most phrases (rest: d uint32 of
// scratch, its count in ctr->rest_len, zero on entry).
//
// Kernels given a device count (d_dev, in.n_dev: the size sits in device
// memory, the host passes a bound of it in d / in.n) are launched over the
// bound and stop at the count: rounds can then be queued without reading
// sizes back.
// The slots an insert over (a bound of) d phrases claims are listed per wave
// of its grid, with no atomics: wave v writes its claims from won + v *
// per_wave and their number to won_cnt[v].  won needs waves * per_wave
// entries (at most d + 256 * kInsertBlocks), won_cnt `waves`.
constexpr uint64_t kInsertBlocks = 2048;  // largest grid of the insert
struct WonGeom {
  uint32_t waves;
  uint64_t per_wave;
};
WonGeom won_geometry(uint64_t d);
// The combining insert lists its claims in won2 (room for the table's
// capacity; count in ctr->won_len, zero on entry).
void launch_insert(bool bytes, uint64_t d, const uint64_t* d_dev, const uint64_t* key,
                   const uint64_t* wkey, const uint64_t* pstart, const uint32_t* plen,
                   const void* content, const uint64_t* rule_off, const void* rule_rhs,
                   uint32_t u_committed, Slot* table, uint64_t mask, uint32_t* slot_idx,
                   bool combine, uint32_t* rest, uint32_t* rest_len, uint32_t* won,
                   uint32_t* won_cnt, uint32_t* won2, Counters* ctr, hipStream_t s);
// First-occurrence flags of the new phrases, one pass over the phrases (for
// rounds where most phrases are new), with per flag word the new rules and
// their right-hand-side lengths.
void launch_newflags(bool bytes, uint64_t d, const uint64_t* d_dev, const uint32_t* slot_idx,
                     const Slot* table, const uint64_t* key, const uint32_t* plen,
                     uint64_t* newbits, uint64_t* wcnt, uint64_t* wlen, hipStream_t s);
// First-occurrence flags of the new phrases from the insert's claims (the
// first occurrence of every slot claimed in the round is new), then per flag
// word the new rules and their right-hand-side lengths.  d: the insert's
// phrase bound; W: flag words to fill (a bound of ceil(d / 64) when the
// count is on the device).
void launch_newflags_won(bool bytes, uint64_t d, const uint32_t* won, const uint32_t* won_cnt,
                         const uint32_t* won2, const Counters* ctr, const Slot* table, uint64_t W,
                         const uint64_t* key, const uint32_t* plen, uint64_t* newbits,
                         uint64_t* wcnt, uint64_t* wlen, hipStream_t s);
void launch_commit(bool bytes, uint64_t d, const uint64_t* d_dev, const uint32_t* slot_idx, Slot* table,
                   const uint64_t* newbits, const uint64_t* wcnt_base, const uint64_t* wlen_base,
                   const uint64_t* key, const uint64_t* wkey, const uint64_t* pstart,
                   const uint32_t* plen,
                   const void* content, const uint32_t* fnew, const uint32_t* fprev, LevelHash h,
                   uint32_t u_prev, uint64_t q_prev, uint64_t* rule_off, void* rule_rhs,
                   uint32_t* rule_fp, uint32_t* sym_next, uint32_t* fnext, uint64_t u_new,
                   uint32_t* nlist, uint64_t* nqoff, hipStream_t s);
// commit: when the new rules (u_new, known on the host) are fewer than
// d / kCommitListRatio, the new phrases are listed first and committed one
// thread per rule (nlist: u_new uint32, nqoff: u_new uint64 of scratch)
constexpr uint64_t kCommitListRatio = 4;
// Rules with rank < rank_limit (kNone: every committed rule) into new_t.
void launch_rehash(const Slot* old_t, uint64_t old_cap, Slot* new_t, uint64_t new_mask,
                   uint32_t rank_limit, Counters* ctr, hipStream_t s);

// ---- the short rounds fused into one cooperative launch
// One round of the fused tail, as the host prepared it: level `level`'s
// coefficients, dictionary and rule arrays (grown for the round's worst
// case), the fingerprints of the level below, and where the round's counts
// go.
struct TailRound {
  LevelHash h;
  Slot* table;
  uint64_t mask;
  uint32_t u0;            // rules of the level before the round
  uint32_t level;
  uint64_t q0;            // right-hand-side symbols of the level before the round
  uint64_t* rule_off;
  void* rule_rhs;         // bytes at level 1, ranks above
  uint32_t* rule_fp;
  const uint32_t* fprev;  // F of the level-(level-1) symbols (h^0 of the bytes at level 1)
  TailRec* rec;
};
// Everything the fused tail kernel reads besides its rounds; the work arrays
// are sized for the first round's bounds, which bound every later round's.
struct TailArgs {
  const TailRound* rounds;
  uint32_t nrounds;
  uint32_t k;
  uint64_t n0;             // length of the first round's sequence
  const uint64_t* off0;    // its segment offsets
  const uint8_t* text;     // its symbols when it is level 1
  bool first_bytes;
  int cur0;                // ping-pong index the first round writes
  uint32_t key_bits;
  const uint32_t* lut;
  uint64_t* bits;
  uint64_t* tile_cnt;
  uint64_t* tile_base;
  TileSeg* tile_seg;
  uint64_t* pstart;
  uint32_t* plen;
  uint64_t* key;
  uint64_t* wkey;
  uint32_t* slot_idx;
  uint32_t* sym[2];
  uint32_t* fpv[2];
  uint64_t* off[2];
  uint64_t* newbits;
  uint64_t* wcnt;
  uint64_t* wlen;
  uint64_t* wcnt_base;
  uint64_t* wlen_base;
  uint8_t* c_level;        // the batch's C entries
  uint32_t* c_sym;
  uint32_t* rounds_run;    // out: rounds the kernel ran
};
// Blocks of the fused tail kernel that the device holds at once (its grid
// must not exceed them: the rounds synchronise the whole grid).
unsigned tail_grid();
// All rounds of a.rounds in one cooperative launch; the kernel stops after
// the round that leaves no string active.
void launch_tail(const TailArgs& a, unsigned grid, hipStream_t s);

void launch_c_init(const uint8_t* text, const uint64_t* off, uint32_t k, uint8_t* c_level,
                   uint32_t* c_sym, hipStream_t s);
void launch_segments(const uint64_t* off, uint32_t k, const uint64_t* bits,
                     const uint64_t* tile_base, uint64_t d, const uint64_t* d_dev,
                     uint64_t* new_off, hipStream_t s);
void launch_finish(const uint64_t* off, const uint64_t* new_off, uint32_t k,
                   const uint32_t* sym_next, uint32_t level, uint8_t* c_level, uint32_t* c_sym,
                   Counters* ctr, hipStream_t s);

// Merge: prepare G_b's level-i rules as phrases over G_a's level-(i-1) ranks.
void launch_merge_prepare(bool bytes, uint32_t u_b, const uint64_t* b_off, const void* b_rhs,
                          const uint32_t* remap_prev, const uint32_t* f_prev, LevelHash h,
                          uint32_t key_bits, void* content, uint64_t* pstart, uint32_t* plen,
                          uint64_t* key, uint64_t* wkey, hipStream_t s);
void launch_c_merge(const uint8_t* b_level, const uint32_t* b_sym, uint32_t kb, uint32_t level,
                    const uint32_t* remap, uint8_t* out_level, uint32_t* out_sym, hipStream_t s);

// Expansion (top-down, one level per call).
void launch_expand_lens(const uint32_t* cur, uint64_t m, const uint64_t* rule_off, uint64_t* lens,
                        hipStream_t s);
void launch_expand_emit(bool bytes, const uint32_t* cur, uint64_t m, const uint64_t* rule_off,
                        const void* rule_rhs, const uint64_t* pos, void* next, hipStream_t s);

// Expansion of a range of ks strings at once, top-down by byte positions.
// E (per level, bytes of every rule's expansion): launch_explen, level 1 with
// e_below = NULL, level L > 1 over rhs ranks of level L-1 with e_below = E of
// level L-1.  e_levels is a device array of the per-level E pointers.
void launch_explen(const uint64_t* rule_off, const uint32_t* rhs, const uint64_t* e_below,
                   uint32_t u, uint64_t* e, hipStream_t s);
void launch_xs_strlen(const uint8_t* c_level, const uint32_t* c_sym, uint32_t ks,
                      const uint64_t* const* e_levels, uint64_t* len, hipStream_t s);
// Strings whose C entry is at `level` join the items (sym, pos; count is the
// device item counter) or, at level 0, write their byte into out.
void launch_xs_enter(const uint8_t* c_level, const uint32_t* c_sym, uint32_t ks, uint32_t level,
                     const uint64_t* str_off, uint32_t* sym, uint64_t* pos, uint64_t* count,
                     uint8_t* out, hipStream_t s);
// *total += children of the m items (must be zeroed by the caller)
void launch_xs_count(const uint32_t* sym, uint64_t m, const uint64_t* rule_off, uint64_t* total,
                     hipStream_t s);
// Items -> children (or bytes); *gcount += grandchildren (gc_rule[r] per
// item, when given).
void launch_xs_expand(bool to_bytes, const uint32_t* sym, const uint64_t* pos, uint64_t m,
                      const uint64_t* rule_off, const void* rule_rhs, const uint64_t* e_below,
                      const uint64_t* gc_rule, uint32_t* nsym, uint64_t* npos,
                      uint64_t* ncount, uint64_t* gcount, uint8_t* out, hipStream_t s);
// Level-2 items -> the bytes of their level-1 children, in place.
void launch_xs_bytes2(const uint32_t* sym, const uint64_t* pos, uint64_t m, const uint64_t* off2,
                      const uint32_t* rhs2, const uint64_t* off1, const uint8_t* rhs1, uint8_t* out,
                      hipStream_t s);
// per rule of a level >= 2: the summed right-hand-side lengths of its children
void launch_gc(const uint64_t* rule_off, const uint32_t* rhs, const uint64_t* off_below, uint32_t u,
               uint64_t* gc, hipStream_t s);

}  // namespace lcg
