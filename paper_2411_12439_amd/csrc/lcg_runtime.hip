// Host runtime and C ABI of liblcg (declared in include/lcg.h).
//
// The host plans: it validates inputs, sizes buffers from a few counters read
// back per round, grows dictionaries and launches the kernels of
// lcg_kernels.hip.  Every operation on the data runs on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/lcg.h"
#include "lcg_kernels.h"

#include "lcg_host.h"


namespace lcg {

struct Opts {
  uint64_t seed = 0;
  uint32_t mode = LCG_MODE_BATCHED;
  uint32_t flags = 0;
  uint64_t budget = 0;
  uint32_t key_bits = 0;
  uint32_t table_min_log2 = 12;
  uint32_t tail_log2 = 22;
  uint32_t table_load_log2 = 1;
  uint32_t combine_log2 = 5;  // 31: never
  uint32_t fail_round = 0;    // test hook: fail on reaching this round (0 = off)
};

static Opts read_opts(const lcg_opts* o) {
  Opts r;
  if (!o) return r;
  r.seed = o->seed;
  r.mode = o->mode;
  r.flags = o->flags;
  r.budget = o->hbm_budget;
  r.key_bits = o->key_bits;
  if (o->table_min_log2) r.table_min_log2 = o->table_min_log2;
  if (o->tail_log2) r.tail_log2 = o->tail_log2;
  if (r.tail_log2 > 40) throw LcgError{LCG_EINVAL, "tail_log2 out of range"};
  if (o->table_load_log2) r.table_load_log2 = o->table_load_log2;
  if (r.table_load_log2 > 3) throw LcgError{LCG_EINVAL, "table_load_log2 out of range"};
  if (o->combine_log2) r.combine_log2 = o->combine_log2;
  if (r.combine_log2 > 31) throw LcgError{LCG_EINVAL, "combine_log2 out of range"};
  r.fail_round = o->fail_round;
  if (r.flags & ~(uint32_t)(LCG_FLAG_TIMING | LCG_FLAG_TIMING_INSERT | LCG_FLAG_FUSED_TAIL))
    throw LcgError{LCG_EINVAL, "unknown flag"};
  if (r.mode != LCG_MODE_BATCHED && r.mode != LCG_MODE_PLAIN)
    throw LcgError{LCG_EINVAL, "unknown mode"};
  if (r.key_bits > 30) throw LcgError{LCG_EINVAL, "key_bits must be 0..30"};
  if (r.table_min_log2 < 6 || r.table_min_log2 > 34) throw LcgError{LCG_EINVAL, "table_min_log2 out of range"};
  return r;
}

static uint64_t next_pow2(uint64_t x) {
  uint64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

// HyperLogLog estimate (Flajolet et al. 2007) over 32-bit key hashes, with
// the linear-counting correction for small cardinalities and the
// hash-collision correction for large ones.
static double hll_estimate(const unsigned int* regs) {
  const double m = kHll;
  double sum = 0;
  int zeros = 0;
  for (int i = 0; i < kHll; ++i) {
    sum += std::ldexp(1.0, -(int)regs[i]);
    if (regs[i] == 0) ++zeros;
  }
  double e = (0.7213 / (1.0 + 1.079 / m)) * m * m / sum;
  const double two32 = 4294967296.0;
  if (e <= 2.5 * m && zeros) e = m * std::log(m / zeros);
  else if (e > two32 / 30.0) e = e < two32 ? -two32 * std::log(1.0 - e / two32) : two32;
  return e;
}

// Working memory of one build call besides the grammar: the phrase arrays of
// a round are sized for the worst case n/2 + k phrases (start 8 B, length 4,
// key 8, wide-key content 16, slot 4, claimed slot 4, two symbol and two
// fingerprint streams 4 each = 60 B per phrase), plus break bits, scan and
// sketch buffers.
static uint64_t build_bytes(uint64_t n, uint32_t k) {
  return 31 * n + 64ull * k + (64ull << 20);
}

// Reusable per-call scratch.
struct Work {
  DBuf<uint64_t> bits, tile_cnt, tile_base, scan_tmp;
  DBuf<uint64_t> pstart, key, wkey;  // wkey: two content words per phrase with a wide key
  DBuf<uint32_t> plen, slot_idx;
  DBuf<uint32_t> sym[2], fpv[2];
  DBuf<uint64_t> off[2];
  DBuf<uint64_t> newbits, wcnt, wlen, wcnt_base, wlen_base, nqoff;
  DBuf<uint32_t> lut, nlist;
  DBuf<Counters> ctr, fin;
  DBuf<uint8_t> content8, hll_part;
  DBuf<TileSeg> tile_seg;
  DBuf<uint32_t> content32, remap[2], rest, won, won_cnt, won2;
  DBuf<struct TailRec> tail;
  DBuf<TailRound> tail_rounds;
  DBuf<uint32_t> tail_run;
  void release_after(hipStream_t s) {
    DBuf<uint64_t>* b64[] = {&bits, &tile_cnt, &tile_base, &scan_tmp, &pstart, &key, &wkey, &off[0],
                             &off[1], &newbits, &wcnt, &wlen, &wcnt_base, &wlen_base, &nqoff};
    DBuf<uint32_t>* b32[] = {&plen, &slot_idx, &sym[0], &sym[1], &fpv[0], &fpv[1], &lut,
                             &content32, &remap[0], &remap[1], &rest, &nlist, &won, &won_cnt,
                             &won2};
    for (auto* b : b64) b->reset_after(s);
    for (auto* b : b32) b->reset_after(s);
    ctr.reset_after(s);
    fin.reset_after(s);
    tail.reset_after(s);
    tail_rounds.reset_after(s);
    tail_run.reset_after(s);
    content8.reset_after(s);
    hll_part.reset_after(s);
    tile_seg.reset_after(s);
  }
};

static void zero_counters(Counters* c, hipStream_t s) { launch_zero(c, sizeof(Counters), s); }

// Pinned host landing area of the per-round readbacks (one per host thread,
// kept for the life of the process): pageable destinations would make every
// small device-to-host copy go through a staging buffer.
struct Mailbox {
  Counters ctr;
  Counters fin;
  uint64_t d, u_new, q_new;
  uint32_t polled[HashFamily::kLevels];  // active counts of the tail rounds
};

static Mailbox* mailbox() {
  static thread_local Mailbox* mb = nullptr;
  if (!mb) {
    void* p = nullptr;
    HIP_CHECK(hipHostMalloc(&p, sizeof(Mailbox), hipHostMallocDefault));
    mb = static_cast<Mailbox*>(p);
  }
  return mb;
}

// LCG_DEBUG=1 in the environment traces the per-round planning on stderr.
static bool debug_on() {
  static const bool on = [] {
    const char* e = std::getenv("LCG_DEBUG");
    return e && *e && *e != '0';
  }();
  return on;
}

// HIP events at the phase boundaries of one round (LCG_FLAG_TIMING):
// 0 start, 1 classified and counted, 2 emit start, 8 emitted, 3 dictionary
// sized, 4 inserted, 5 ranked, 6 committed, 7 segments done.  The host work
// between phases 1 and 2 and between 8 and 3 is not counted.
// With LCG_FLAG_TIMING_INSERT only boundaries 3 and 4 are recorded, in the
// rounds that read their sizes back: each recorded event costs a few
// microseconds of stream time, about 0.7 ms per build for all of them.
struct PhaseEvents {
  static constexpr int N = 9;
  static constexpr uint32_t kAll = (1u << N) - 1;
  static constexpr uint32_t kInsert = (1u << 3) | (1u << 4);
  hipEvent_t e[N] = {};
  uint32_t mask;  // bit i: boundary i is recorded
  explicit PhaseEvents(uint32_t m) : mask(m & kAll) {
    for (int i = 0; i < N; ++i)
      if (mask >> i & 1) HIP_CHECK(hipEventCreate(&e[i]));
  }
  PhaseEvents(const PhaseEvents&) = delete;
  PhaseEvents& operator=(const PhaseEvents&) = delete;
  ~PhaseEvents() {
    for (auto x : e)
      if (x) (void)hipEventDestroy(x);
  }
  void rec(int i, hipStream_t s) {
    if (mask >> i & 1) HIP_CHECK(hipEventRecord(e[i], s));
  }
  // device time between boundaries a and b; 0 unless both are recorded
  uint64_t ns(int a, int b) {
    if (!(mask >> a & mask >> b & 1)) return 0;
    float ms = 0;
    HIP_CHECK(hipEventElapsedTime(&ms, e[a], e[b]));
    return (uint64_t)((double)ms * 1e6);
  }
};

// the boundaries a round with host reads records under these flags
static uint32_t phase_mask(uint32_t flags) {
  if (flags & LCG_FLAG_TIMING) return PhaseEvents::kAll;
  if (flags & LCG_FLAG_TIMING_INSERT) return PhaseEvents::kInsert;
  return 0;
}

// Make room in level L's dictionary for `need` committed + new keys at load
// <= 2^-table_load_log2.
static void ensure_table(Level& L, uint64_t need, const Opts& o, Work& w, hipStream_t s,
                         bool force_grow = false) {
  uint64_t want = std::max<uint64_t>(next_pow2(std::max<uint64_t>(need, 1) << o.table_load_log2),
                                     1ull << o.table_min_log2);
  if (force_grow) want = std::max<uint64_t>(want, L.tcap * 4);
  if (L.tcap >= want && L.table.p) return;
  // slot indices are uint32 and kNone is never one
  if (want > (1ull << 31)) throw LcgError{LCG_ETABLE, "dictionary capacity limit reached"};
  DBuf<Slot> nt;
  nt.need(want, s);
  launch_fill_slots(nt.p, want, s);
  if (L.tcap && L.u) {
    zero_counters(w.ctr.p, s);
    launch_rehash(L.table.p, L.tcap, nt.p, want - 1, kNone, w.ctr.p, s);
    Mailbox* mb = mailbox();
    HIP_CHECK(hipMemcpyAsync(&mb->ctr, w.ctr.p, offsetof(Counters, hll), hipMemcpyDeviceToHost, s));
    sync(s);
    if (mb->ctr.overflow) throw LcgError{LCG_ETABLE, "rehash failed"};
  }
  L.table.reset_after(s);
  L.table = std::move(nt);
  L.tcap = want;
}

// lcg_reserve's bounds: levels it takes, rules per level (2^30 at load 1/2
// fills the largest dictionary, 2^31 slots).
constexpr uint32_t kMaxReserveLevels = 64;
constexpr uint64_t kMaxReserveRules = 1ull << 30;

// The rules lcg_reserve made room for at level lv (1-based), else 0.
static uint64_t reserved(const lcg_grammar* g, uint32_t lv) {
  return lv - 1 < g->reserve.size() ? g->reserve[lv - 1] : 0;
}

// Levels up to i exist; a level created here gets room for off_cap offsets
// if it is level i (a caller that knows the level's size saves the copy of
// the first offset when the array is grown to it), else for one.
static void ensure_level(lcg_grammar* g, size_t i, hipStream_t s, size_t off_cap = 1) {
  while (g->levels.size() < i) {
    g->levels.emplace_back();
    Level& L = g->levels.back();
    L.off.need(g->levels.size() == i ? std::max<size_t>(off_cap, 1) : 1, s);
    HIP_CHECK(hipMemsetAsync(L.off.p, 0, sizeof(uint64_t), s));
  }
}


// Room for the slots an insert over (a bound of) d phrases claims: the
// per-wave regions and counts, and the combining insert's list (at most one
// entry per slot of a table of `cap` slots).
static void need_won(Work& w, uint64_t d, uint64_t cap, hipStream_t s) {
  const WonGeom geo = won_geometry(d);
  w.won.need(std::max<uint64_t>((uint64_t)geo.waves * geo.per_wave, 1), s);
  w.won_cnt.need(std::max<uint32_t>(geo.waves, 1), s);
  w.won2.need(std::max<uint64_t>(cap, 1), s);
}

// A round whose key sketch estimates at most d / kWonRatio new rules takes
// its first-occurrence flags from the insert's claims.
constexpr uint64_t kWonRatio = 4;

struct DedupResult {
  uint32_t u_new;
  uint64_t q_new;
  uint64_t probes, compares;
  bool combined;
};

// insert -> newflags -> scan -> commit for the d phrases of level `lv`
// (1-based) described by w.pstart/w.plen/w.key over `content` (bytes at level
// 1); fnew holds their F values; ranks land in sym_next.  Regrows the
// dictionary and retries if a probe sequence ran out of budget.
static DedupResult dedup_commit(lcg_grammar* g, uint32_t lv, uint64_t d, const void* content,
                                const uint32_t* fnew, uint32_t* sym_next, uint32_t* fnext,
                                uint64_t est_new, const Opts& o, Work& w, hipStream_t s,
                                PhaseEvents* pe = nullptr) {
  Level& L = g->levels[lv - 1];
  const bool bytes = lv == 1;
  ensure_table(L, std::max<uint64_t>((uint64_t)L.u + est_new, reserved(g, lv)), o, w, s);
  const uint64_t W = (d + 63) / 64;
  // few distinct keys for many phrases: combine equal keys per chunk first
  const bool combine = o.combine_log2 < 31 && (est_new << o.combine_log2) <= d;
  w.slot_idx.need(d, s);
  need_won(w, d, combine ? L.tcap : 1, s);
  if (combine) w.rest.need(d, s);
  w.newbits.need(W, s);
  w.wcnt.need(W, s);
  w.wlen.need(W, s);
  w.wcnt_base.need(W + 1, s);
  w.wlen_base.need(W + 1, s);
  w.scan_tmp.need(std::max<size_t>(scan_tmp_words(W), 1), s);
  Mailbox* mb = mailbox();
  Counters& hc = mb->ctr;
  uint64_t u_new = 0, q_new = 0;
  for (int attempt = 0;; ++attempt) {
    zero_counters(w.ctr.p, s);
    const void* rule_rhs = bytes ? (const void*)L.rhs8.p : (const void*)L.rhs32.p;
    if (pe) pe->rec(3, s);
    launch_insert(bytes, d, nullptr, w.key.p, w.wkey.p, w.pstart.p, w.plen.p, content, L.off.p,
                  rule_rhs, L.u, L.table.p, L.tcap - 1, w.slot_idx.p, combine, w.rest.p,
                  &w.ctr.p->rest_len, w.won.p, w.won_cnt.p, w.won2.p, w.ctr.p, s);
    if (pe) pe->rec(4, s);
    // first occurrences: from the slots the insert claimed (one slot read and
    // one flag per new rule) when few phrases are new, else one coalesced
    // pass over the phrases
    if (est_new * kWonRatio <= d)
      launch_newflags_won(bytes, d, w.won.p, w.won_cnt.p, w.won2.p, w.ctr.p, L.table.p, W, w.key.p,
                          w.plen.p, w.newbits.p, w.wcnt.p, w.wlen.p, s);
    else
      launch_newflags(bytes, d, nullptr, w.slot_idx.p, L.table.p, w.key.p, w.plen.p, w.newbits.p,
                      w.wcnt.p, w.wlen.p, s);
    scan_exclusive(w.wcnt.p, w.wcnt_base.p, W, w.scan_tmp.p, s);
    scan_exclusive(w.wlen.p, w.wlen_base.p, W, w.scan_tmp.p, s);
    if (pe) pe->rec(5, s);
    HIP_CHECK(hipMemcpyAsync(&hc, w.ctr.p, offsetof(Counters, hll), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipMemcpyAsync(&mb->u_new, w.wcnt_base.p + W, 8, hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipMemcpyAsync(&mb->q_new, w.wlen_base.p + W, 8, hipMemcpyDeviceToHost, s));
    sync(s);
    u_new = mb->u_new;
    q_new = mb->q_new;
    if (debug_on())
      std::fprintf(stderr, "[lcg] level %u attempt %d: d=%llu est=%llu cap=%llu won=%llu probes=%llu cmp=%llu overflow=%u\n",
                   lv, attempt, (unsigned long long)d, (unsigned long long)est_new,
                   (unsigned long long)L.tcap, hc.won, hc.probes, hc.compares, hc.overflow);
    if (!hc.overflow) break;
    if (attempt >= 6) throw LcgError{LCG_ETABLE, "dictionary overflow persists after regrowth"};
    ensure_table(L, (uint64_t)L.u + std::max<uint64_t>(est_new, hc.won), o, w, s,
                 /*force_grow=*/true);
  }
  if ((uint64_t)L.u + u_new >= kNone) throw LcgError{LCG_EOVERFLOW, "level needs 2^32 ranks"};
  L.off.grow(L.u + u_new + 1, L.u + 1, s);
  L.fp.grow(L.u + u_new, L.u, s);
  void* rule_rhs;
  if (bytes) {
    L.rhs8.grow(L.q + q_new, L.q, s);
    rule_rhs = L.rhs8.p;
  } else {
    L.rhs32.grow(L.q + q_new, L.q, s);
    rule_rhs = L.rhs32.p;
  }
  // F of the level-(lv-1) symbols: h^0 of the bytes, else the previous level's rules
  const uint32_t* fprev = bytes ? w.lut.p : g->levels[lv - 2].fp.p;
  if (u_new * kCommitListRatio < d) {
    w.nlist.need(std::max<uint64_t>(u_new, 1), s);
    w.nqoff.need(std::max<uint64_t>(u_new, 1), s);
  }
  launch_commit(bytes, d, nullptr, w.slot_idx.p, L.table.p, w.newbits.p, w.wcnt_base.p, w.wlen_base.p,
                w.key.p, w.wkey.p, w.pstart.p, w.plen.p, content, fnew, fprev, g->H.lv[lv], L.u, L.q,
                L.off.p, rule_rhs, L.fp.p, sym_next, fnext, u_new, w.nlist.p, w.nqoff.p, s);
  if (pe) pe->rec(6, s);
  L.u += (uint32_t)u_new;
  L.q += q_new;
  return DedupResult{(uint32_t)u_new, q_new, hc.probes, hc.compares, combine};
}

// Tail mode.  Once the sequence is short (n_i <= 2^tail_log2) the rounds are
// launch-bound, not memory-bound, and the two host reads per round would
// dominate.  From there on every round is queued without reading anything
// back: each kernel reads its size (n_i, d_i) from device memory and is
// launched over the worst case (d_i <= n_i/2 + k, Theorem 1's halving), the
// level's dictionary and rule arrays are sized for that worst case before
// the round is queued, and the round's counts land in a device record.  The
// host only waits, kTailLag rounds behind the queue, for a round's count of
// strings still active, to stop queueing once it is zero; the rounds queued
// after the last one find no phrase and change nothing.
constexpr uint32_t kTailLag = 2;

static hipEvent_t tail_event(uint32_t i) {
  static thread_local std::vector<hipEvent_t> ev;
  while (ev.size() <= i) {
    hipEvent_t e;
    HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    ev.push_back(e);
  }
  return ev[i];
}

static void tail_rounds(lcg_grammar* g, uint32_t lv, uint64_t n_i, uint64_t active_len,
                        const uint8_t* d_text, const uint64_t* cur_off, int cur, uint32_t k,
                        uint32_t c_base, const Opts& o, Work& w, hipStream_t s) {
  const uint32_t lv0 = lv;
  const size_t levels_before = g->levels.size();
  const uint32_t max_rounds = (uint32_t)HashFamily::kLevels - lv0;
  w.tail.need(max_rounds, s);
  launch_zero(w.tail.p, sizeof(TailRec) * max_rounds, s);
  const bool timing = (o.flags & LCG_FLAG_TIMING) != 0;
  std::vector<std::unique_ptr<PhaseEvents>> pev;
  Mailbox* mb = mailbox();
  uint64_t nb = n_i;                  // bound of the round's sequence length
  const uint64_t* n_dev = nullptr;    // its exact value on the device (none for the first)
  uint32_t r = 0;
  bool done = false;
  for (; r < max_rounds && !done; ++r, ++lv) {
    if (o.fail_round && lv == o.fail_round)
      throw LcgError{LCG_ETABLE, "test hook: failure forced at round " + std::to_string(lv) +
                                     " (queued without host reads)"};
    const bool bytes = lv == 1;
    TailRec* rec = w.tail.p + r;
    RoundIn in;
    in.sym = bytes ? (const void*)d_text : (const void*)w.sym[cur ^ 1].p;
    in.fp = bytes ? nullptr : w.fpv[cur ^ 1].p;
    in.lut = w.lut.p;
    in.off = cur_off;
    in.k = k;
    in.n = nb;
    in.n_dev = n_dev;
    in.bytes = bytes;
    const uint64_t tiles = (nb + kTile - 1) / kTile;
    const uint64_t d_b = nb / 2 + k + 1;
    const uint64_t W_b = (d_b + 63) / 64;
    w.bits.need(tiles * kTileWords, s);
    w.tile_cnt.need(tiles, s);
    w.tile_base.need(tiles + 1, s);
    w.tile_seg.need(tiles, s);
    w.pstart.need(d_b, s);
    w.plen.need(d_b, s);
    w.key.need(d_b, s);
    w.wkey.need(2 * d_b, s);
    w.slot_idx.need(d_b, s);
    need_won(w, d_b, 1, s);
    w.sym[cur].need(d_b, s);
    w.fpv[cur].need(d_b, s);
    w.off[cur].need(k + 1, s);
    w.newbits.need(W_b, s);
    w.wcnt.need(W_b, s);
    w.wlen.need(W_b, s);
    w.wcnt_base.need(W_b + 1, s);
    w.wlen_base.need(W_b + 1, s);
    ensure_level(g, lv, s, d_b + 1);
    Level& L = g->levels[lv - 1];
    ensure_table(L, std::max<uint64_t>((uint64_t)L.u + d_b, reserved(g, lv)), o, w, s);
    if ((uint64_t)L.u + d_b >= kNone) throw LcgError{LCG_EOVERFLOW, "level needs 2^32 ranks"};
    L.off.grow(L.u + d_b + 1, L.u + 1, s);
    L.fp.grow(L.u + d_b, L.u, s);
    void* rule_rhs;
    if (bytes) {
      L.rhs8.grow(L.q + nb, L.q, s);
      rule_rhs = L.rhs8.p;
    } else {
      L.rhs32.grow(L.q + nb, L.q, s);
      rule_rhs = L.rhs32.p;
    }
    PhaseEvents* pe = nullptr;
    if (timing) {
      pev.emplace_back(new PhaseEvents(PhaseEvents::kAll));
      pe = pev.back().get();
    }
    const void* content = in.sym;
    if (pe) pe->rec(0, s);
    launch_classify(in, w.bits.p, w.tile_cnt.p, w.tile_seg.p, s);
    scan_one(w.tile_cnt.p, w.tile_base.p, tiles, n_dev, 12, &rec->d, s);  // kTile = 2^12
    if (pe) pe->rec(1, s);
    if (pe) pe->rec(2, s);
    launch_emit(in, w.bits.p, w.tile_base.p, w.tile_seg.p, g->H.lv[lv], o.key_bits, w.pstart.p,
                w.plen.p, w.key.p, w.wkey.p, w.fpv[cur].p, w.hll_part.p, nullptr, s);
    if (pe) pe->rec(8, s);
    if (pe) pe->rec(3, s);
    launch_insert(bytes, d_b, &rec->d, w.key.p, w.wkey.p, w.pstart.p, w.plen.p, content, L.off.p,
                  rule_rhs, L.u, L.table.p, L.tcap - 1, w.slot_idx.p, false, nullptr, nullptr,
                  w.won.p, w.won_cnt.p, w.won2.p, &rec->ctr, s);
    if (pe) pe->rec(4, s);
    // short rounds: most phrases are new
    launch_newflags(bytes, d_b, &rec->d, w.slot_idx.p, L.table.p, w.key.p, w.plen.p, w.newbits.p,
                    w.wcnt.p, w.wlen.p, s);
    scan_one(w.wcnt.p, w.wcnt_base.p, W_b, &rec->d, 6, &rec->u, s);
    scan_one(w.wlen.p, w.wlen_base.p, W_b, &rec->d, 6, &rec->q, s);
    if (pe) pe->rec(5, s);
    const uint32_t* fprev = bytes ? w.lut.p : g->levels[lv - 2].fp.p;
    launch_commit(bytes, d_b, &rec->d, w.slot_idx.p, L.table.p, w.newbits.p, w.wcnt_base.p,
                  w.wlen_base.p, w.key.p, w.wkey.p, w.pstart.p, w.plen.p, content, w.fpv[cur].p, fprev,
                  g->H.lv[lv], L.u, L.q, L.off.p, rule_rhs, L.fp.p, w.sym[cur].p, w.fpv[cur].p,
                  0, nullptr, nullptr, s);
    if (pe) pe->rec(6, s);
    launch_segments(cur_off, k, w.bits.p, w.tile_base.p, d_b, &rec->d, w.off[cur].p, s);
    launch_finish(cur_off, w.off[cur].p, k, w.sym[cur].p, lv, g->c_level.p + c_base,
                  g->c_sym.p + c_base, &rec->fin, s);
    if (pe) pe->rec(7, s);
    HIP_CHECK(hipMemcpyAsync(&mb->polled[r], &rec->fin.active, sizeof(uint32_t),
                             hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipEventRecord(tail_event(r), s));
    if (r >= kTailLag) {
      HIP_CHECK(hipEventSynchronize(tail_event(r - kTailLag)));
      done = mb->polled[r - kTailLag] == 0;
    }
    n_dev = &rec->d;
    nb = d_b;
    cur_off = w.off[cur].p;
    cur ^= 1;
  }
  std::vector<TailRec> rec(r);
  HIP_CHECK(hipMemcpyAsync(rec.data(), w.tail.p, sizeof(TailRec) * r, hipMemcpyDeviceToHost, s));
  sync(s);
  uint32_t j = 0;
  for (; j < r && rec[j].d; ++j) {
    const TailRec& t = rec[j];
    if (t.ctr.overflow) throw LcgError{LCG_ETABLE, "dictionary overflow in a tail round"};
    Level& L = g->levels[lv0 - 1 + j];
    if ((uint64_t)L.u + t.u >= kNone) throw LcgError{LCG_EOVERFLOW, "level needs 2^32 ranks"};
    L.u += (uint32_t)t.u;
    L.q += t.q;
    Stat row{};
    row[0] = j ? rec[j - 1].fin.active_len : active_len;
    row[1] = t.d;
    row[2] = t.u;
    row[3] = t.q;
    row[4] = t.fin.active;
    row[5] = t.ctr.probes;
    row[6] = t.ctr.compares;
    row[7] = L.tcap;
    if (timing) {
      PhaseEvents& pe = *pev[j];
      row[9] = pe.ns(0, 1);
      row[10] = pe.ns(2, 8);
      row[11] = pe.ns(3, 4);
      row[12] = pe.ns(4, 5);
      row[13] = pe.ns(5, 6);
      row[14] = pe.ns(6, 7);
      row[8] = row[9] + row[10] + row[11] + row[12] + row[13] + row[14];
    }
    row[15] = 2;  // queued without host reads
    g->stats.push_back(row);
  }
  if (j == r && r == max_rounds && rec[r - 1].fin.active)
    throw LcgError{LCG_EOVERFLOW, "more than 63 rounds"};
  // levels opened for the rounds queued after the last one stay empty
  while (g->levels.size() > levels_before && g->levels.size() > lv0 - 1 + j &&
         g->levels.back().u == 0)
    g->levels.pop_back();
}

// The tail rounds in one cooperative launch (launch_tail): the host sizes
// every round it may need for the worst case (Theorem 1's halving from
// n_i: ceil(log2 n_i) + 2 rounds, each with at most n/2 + k phrases), then
// the kernel runs them back to back and stops after the round that leaves
// no string active.  Results are those of tail_rounds, rank for rank.
static void fused_tail(lcg_grammar* g, uint32_t lv, uint64_t n_i, uint64_t active_len,
                       const uint8_t* d_text, const uint64_t* cur_off, int cur, uint32_t k,
                       uint32_t c_base, const Opts& o, Work& w, hipStream_t s) {
  const size_t levels_before = g->levels.size();
  const uint32_t lv_start = lv;
  for (;;) {
    if (lv >= (uint32_t)HashFamily::kLevels) throw LcgError{LCG_EOVERFLOW, "more than 63 rounds"};
    uint32_t bits = 0;
    while (bits < 63 && (1ull << bits) < n_i) ++bits;
    uint32_t R = std::min<uint32_t>((uint32_t)HashFamily::kLevels - lv, bits + 2);
    if (o.fail_round && o.fail_round >= lv && o.fail_round < lv + R) {
      if (o.fail_round == lv)
        throw LcgError{LCG_ETABLE, "test hook: failure forced at round " + std::to_string(lv) +
                                       " (in one cooperative launch)"};
      R = o.fail_round - lv;  // the rounds before it run; the loop then stops there
    }
    const bool first_bytes = lv == 1;
    // bounds of every round: n_0 = n_i, d_r <= n_r / 2 + k + 1, n_{r+1} = d_r
    std::vector<uint64_t> nb(R), db(R);
    for (uint32_t r = 0; r < R; ++r) {
      nb[r] = r ? db[r - 1] : n_i;
      db[r] = nb[r] / 2 + k + 1;
    }
    const uint64_t tiles0 = (nb[0] + kTile - 1) / kTile;
    const uint64_t W0 = (db[0] + 63) / 64;
    uint64_t dmax = 0;
    for (uint32_t r = 0; r < R; ++r) dmax = std::max(dmax, db[r]);
    w.bits.need(tiles0 * kTileWords, s);
    w.tile_cnt.need(tiles0, s);
    w.tile_base.need(tiles0 + 1, s);
    w.tile_seg.need(tiles0, s);
    w.pstart.need(dmax, s);
    w.plen.need(dmax, s);
    w.key.need(dmax, s);
    w.wkey.need(2 * dmax, s);
    w.slot_idx.need(dmax, s);
    // T^lv (input of the first round) stays in sym / fpv [cur ^ 1] and its
    // offsets possibly in off[cur ^ 1]: grown keeping their contents
    if (first_bytes) {
      w.sym[cur ^ 1].need(dmax, s);
      w.fpv[cur ^ 1].need(dmax, s);
    } else {
      w.sym[cur ^ 1].grow(std::max<uint64_t>(dmax, n_i), n_i, s);
      w.fpv[cur ^ 1].grow(std::max<uint64_t>(dmax, n_i), n_i, s);
    }
    w.sym[cur].need(dmax, s);
    w.fpv[cur].need(dmax, s);
    w.off[cur].need(k + 1, s);
    if (cur_off == w.off[cur ^ 1].p) w.off[cur ^ 1].grow(k + 1, k + 1, s);
    else w.off[cur ^ 1].need(k + 1, s);
    w.newbits.need(W0, s);
    w.wcnt.need(W0, s);
    w.wlen.need(W0, s);
    w.wcnt_base.need(W0 + 1, s);
    w.wlen_base.need(W0 + 1, s);
    w.tail.need(R, s);
    w.tail_rounds.need(R, s);
    w.tail_run.need(1, s);
    launch_zero(w.tail.p, sizeof(TailRec) * R, s);
    std::vector<TailRound> rounds(R);
    for (uint32_t r = 0; r < R; ++r) {
      const uint32_t lr = lv + r;
      ensure_level(g, lr, s, db[r] + 1);
      Level& L = g->levels[lr - 1];
      ensure_table(L, std::max<uint64_t>((uint64_t)L.u + db[r], reserved(g, lr)), o, w, s);
      if ((uint64_t)L.u + db[r] >= kNone) throw LcgError{LCG_EOVERFLOW, "level needs 2^32 ranks"};
      L.off.grow(L.u + db[r] + 1, L.u + 1, s);
      L.fp.grow(L.u + db[r], L.u, s);
      TailRound& T = rounds[r];
      if (lr == 1) {
        L.rhs8.grow(L.q + nb[r], L.q, s);
        T.rule_rhs = L.rhs8.p;
      } else {
        L.rhs32.grow(L.q + nb[r], L.q, s);
        T.rule_rhs = L.rhs32.p;
      }
      T.h = g->H.lv[lr];
      T.table = L.table.p;
      T.mask = L.tcap - 1;
      T.u0 = L.u;
      T.level = lr;
      T.q0 = L.q;
      T.rule_off = L.off.p;
      T.rule_fp = L.fp.p;
      T.fprev = lr == 1 ? w.lut.p : g->levels[lr - 2].fp.p;
      T.rec = w.tail.p + r;
    }
    HIP_CHECK(hipMemcpyAsync(w.tail_rounds.p, rounds.data(), sizeof(TailRound) * R,
                             hipMemcpyHostToDevice, s));
    TailArgs a{};
    a.rounds = w.tail_rounds.p;
    a.nrounds = R;
    a.k = k;
    a.n0 = n_i;
    a.off0 = cur_off;
    a.text = d_text;
    a.first_bytes = first_bytes;
    a.cur0 = cur;
    a.key_bits = o.key_bits;
    a.lut = w.lut.p;
    a.bits = w.bits.p;
    a.tile_cnt = w.tile_cnt.p;
    a.tile_base = w.tile_base.p;
    a.tile_seg = w.tile_seg.p;
    a.pstart = w.pstart.p;
    a.plen = w.plen.p;
    a.key = w.key.p;
    a.wkey = w.wkey.p;
    a.slot_idx = w.slot_idx.p;
    for (int x = 0; x < 2; ++x) {
      a.sym[x] = w.sym[x].p;
      a.fpv[x] = w.fpv[x].p;
      a.off[x] = w.off[x].p;
    }
    a.newbits = w.newbits.p;
    a.wcnt = w.wcnt.p;
    a.wlen = w.wlen.p;
    a.wcnt_base = w.wcnt_base.p;
    a.wlen_base = w.wlen_base.p;
    a.c_level = g->c_level.p + c_base;
    a.c_sym = g->c_sym.p + c_base;
    a.rounds_run = w.tail_run.p;
    // a grid no larger than the device holds at once (the rounds synchronise
    // it), and no larger than the first round's work needs
    const unsigned grid = (unsigned)std::max<uint64_t>(
        1, std::min<uint64_t>({(uint64_t)tail_grid(), 512ull, (db[0] + 255) / 256}));
    launch_tail(a, grid, s);
    std::vector<TailRec> rec(R);
    uint32_t ran = 0;
    HIP_CHECK(hipMemcpyAsync(rec.data(), w.tail.p, sizeof(TailRec) * R, hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipMemcpyAsync(&ran, w.tail_run.p, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    sync(s);  // also keeps `rounds` alive until its copy is done
    if (ran == 0 || ran > R) throw LcgError{LCG_EHIP, "internal: fused tail ran no round"};
    for (uint32_t j = 0; j < ran; ++j) {
      const TailRec& t = rec[j];
      if (t.ctr.overflow) throw LcgError{LCG_ETABLE, "dictionary overflow in a tail round"};
      Level& L = g->levels[lv - 1 + j];
      if ((uint64_t)L.u + t.u >= kNone) throw LcgError{LCG_EOVERFLOW, "level needs 2^32 ranks"};
      L.u += (uint32_t)t.u;
      L.q += t.q;
      Stat row{};
      row[0] = j ? rec[j - 1].fin.active_len : active_len;
      row[1] = t.d;
      row[2] = t.u;
      row[3] = t.q;
      row[4] = t.fin.active;
      row[5] = t.ctr.probes;
      row[6] = t.ctr.compares;
      row[7] = L.tcap;
      row[15] = 3;  // in one cooperative launch with the other tail rounds
      g->stats.push_back(row);
    }
    const TailRec& last = rec[ran - 1];
    // levels opened for rounds that did not run stay empty
    while (g->levels.size() > levels_before && g->levels.size() > lv - 1 + ran &&
           g->levels.back().u == 0)
      g->levels.pop_back();
    if (!last.fin.active) return;
    // more rounds than prepared (not reached by Theorem 1's bound): go on
    active_len = last.fin.active_len;
    n_i = last.d;
    cur ^= (int)(ran & 1);
    cur_off = w.off[cur ^ 1].p;
    lv += ran;
    if (lv - lv_start > (uint32_t)HashFamily::kLevels)
      throw LcgError{LCG_EOVERFLOW, "more than 63 rounds"};
  }
}

// BuildGram of k strings into g (fresh or existing), the batched form, kept
// as the state of a build between its rounds, so that several builds into
// one grammar can advance in turns (the serving session) as well as one
// build to its end (build_core).
//
// A round with host reads synchronises up to three times: the phrase count
// after classify (sizes the phrase arrays exactly; also returns the previous
// round's count of strings still active), the key sketch after emit (sizes
// the dictionary; rounds over at most 2^20 symbols skip it and size by the
// phrase count), and the new-rule counts (sizes the level).  The round after
// the last one runs classify on strings of length <= 1 and finds no phrase;
// that is how the build learns that every string is done.
// Once the sequence is short, one step queues all remaining rounds without
// host reads (tail_rounds).
struct Cohort {
  lcg_grammar* g;
  const uint8_t* d_text;
  uint32_t k;
  uint32_t c_base;  // index in C of the first string
  Opts o;
  Work& w;
  PhaseEvents pe;
  const uint64_t* cur_off;  // segment offsets of T^lv
  uint64_t n_i;             // length of T^lv
  uint32_t lv = 1;
  int cur = 0;              // ping-pong index of T^{lv+1}
  uint32_t active = 0;      // strings longer than one symbol
  uint64_t active_len = 0;  // their total length
  bool pending = false;     // the previous round's row waits for its active count
  Stat prev{};
  bool done = false;

  Cohort(lcg_grammar* g_, const uint8_t* text, const uint64_t* d_off, uint32_t k_,
         const std::vector<uint64_t>& h_off, const Opts& o_, Work& w_, hipStream_t s)
      : g(g_), d_text(text), k(k_), c_base(g_->k), o(o_), w(w_), pe(phase_mask(o_.flags)),
        cur_off(d_off), n_i(h_off[k_]) {
    g->c_level.grow(c_base + k, c_base, s);
    g->c_sym.grow(c_base + k, c_base, s);
    launch_c_init(d_text, d_off, k, g->c_level.p + c_base, g->c_sym.p + c_base, s);
    g->k += k;
    for (uint32_t j = 0; j < k; ++j) {
      const uint64_t len = h_off[j + 1] - h_off[j];
      active += len >= 2;
      active_len += len >= 2 ? len : 0;
    }
    if (!active) {
      sync(s);
      done = true;
      return;
    }
    w.lut.need(256, s);
    w.ctr.need(1, s);
    w.fin.need(1, s);
    w.hll_part.need((size_t)kEmitBlocks * kHll, s);
    launch_f0_lut(w.lut.p, g->H.lv[0].a, g->H.lv[0].b, s);
  }

  // The previous round's row, completed with its count of strings still
  // active (read into the mailbox by the caller).
  void close_prev(const Counters& hf) {
    prev[4] = hf.active;
    prev[13] = pe.ns(5, 6);
    prev[14] = pe.ns(6, 7);
    prev[8] += prev[13] + prev[14];
    g->stats.push_back(prev);
    active = hf.active;
    active_len = hf.active_len;
  }

  // One round with host reads, or all remaining rounds queued without them.
  void step(hipStream_t s) {
    if (done) return;
    Mailbox* mb = mailbox();
    Counters& hf = mb->fin;
    if (o.fail_round && lv == o.fail_round && n_i > (1ull << o.tail_log2))
      throw LcgError{LCG_ETABLE, "test hook: failure forced at round " + std::to_string(lv)};
    if (lv >= (uint32_t)HashFamily::kLevels) {
      HIP_CHECK(hipMemcpyAsync(&hf, w.fin.p, offsetof(Counters, hll), hipMemcpyDeviceToHost, s));
      sync(s);
      close_prev(hf);
      if (hf.active) throw LcgError{LCG_EOVERFLOW, "more than 63 rounds"};
      done = true;
      return;
    }
    if (n_i <= (1ull << o.tail_log2)) {
      // the rest of the rounds run in tail mode; first the previous round's row
      if (pending) {
        HIP_CHECK(hipMemcpyAsync(&hf, w.fin.p, offsetof(Counters, hll), hipMemcpyDeviceToHost, s));
        sync(s);
        close_prev(hf);
        pending = false;
        if (!active) {
          done = true;
          return;
        }
      }
      // separate kernels per phase, or all rounds in one cooperative launch
      // when asked for (not with per-phase timing, whose events need kernel
      // boundaries)
      if ((o.flags & LCG_FLAG_FUSED_TAIL) && !(o.flags & LCG_FLAG_TIMING))
        fused_tail(g, lv, n_i, active_len, d_text, cur_off, cur, k, c_base, o, w, s);
      else
        tail_rounds(g, lv, n_i, active_len, d_text, cur_off, cur, k, c_base, o, w, s);
      done = true;
      return;
    }
    const bool bytes = lv == 1;
    RoundIn in;
    in.sym = bytes ? (const void*)d_text : (const void*)w.sym[cur ^ 1].p;
    in.fp = bytes ? nullptr : w.fpv[cur ^ 1].p;
    in.lut = w.lut.p;
    in.off = cur_off;
    in.k = k;
    in.n = n_i;
    in.n_dev = nullptr;
    in.bytes = bytes;
    const uint64_t tiles = (n_i + kTile - 1) / kTile;
    const uint64_t d_cap = n_i / 2 + k + 1;  // phrases have length >= 2 but the first
    if (d_cap >= kNone) throw LcgError{LCG_EOVERFLOW, "a round may have 2^32 phrases"};
    w.bits.need(tiles * kTileWords, s);
    w.tile_cnt.need(tiles, s);
    w.tile_base.need(tiles + 1, s);
    w.tile_seg.need(tiles, s);
    w.scan_tmp.need(std::max<size_t>(scan_tmp_words(tiles), 1), s);
    w.off[cur].need(k + 1, s);
    pe.rec(0, s);
    launch_classify(in, w.bits.p, w.tile_cnt.p, w.tile_seg.p, s);
    scan_exclusive(w.tile_cnt.p, w.tile_base.p, tiles, w.scan_tmp.p, s);
    pe.rec(1, s);
    // the phrase count sizes the phrase arrays exactly (about 0.29 n at round 1
    // of DNA, against the worst case n/2 + k)
    HIP_CHECK(hipMemcpyAsync(&mb->d, w.tile_base.p + tiles, 8, hipMemcpyDeviceToHost, s));
    if (pending)
      HIP_CHECK(hipMemcpyAsync(&hf, w.fin.p, offsetof(Counters, hll), hipMemcpyDeviceToHost, s));
    sync(s);
    const uint64_t d = mb->d;
    if (pending) {
      close_prev(hf);
      pending = false;
      if (!active) {
        if (d) throw LcgError{LCG_EHIP, "internal: phrases after the last round"};
        done = true;
        return;
      }
    }
    if (d == 0 || d >= d_cap) throw LcgError{LCG_EHIP, "internal: phrase count out of range"};
    w.pstart.need(d, s);
    w.plen.need(d, s);
    w.key.need(d, s);
    w.wkey.need(2 * d, s);
    w.sym[cur].need(d, s);
    w.fpv[cur].need(d, s);
    zero_counters(w.ctr.p, s);
    pe.rec(2, s);
    // small rounds size the dictionary by the phrase count itself
    const bool sketch = n_i > (1u << 20);
    launch_emit(in, w.bits.p, w.tile_base.p, w.tile_seg.p, g->H.lv[lv], o.key_bits, w.pstart.p,
                w.plen.p, w.key.p, w.wkey.p, w.fpv[cur].p, w.hll_part.p,
                sketch ? w.ctr.p : nullptr, s);
    pe.rec(8, s);
    if (sketch) {
      HIP_CHECK(hipMemcpyAsync(mb->ctr.hll, w.ctr.p->hll, sizeof(unsigned int) * kHll,
                               hipMemcpyDeviceToHost, s));
      sync(s);
    }
    ensure_level(g, lv, s);
    const uint64_t est =
        sketch ? std::min<uint64_t>(d, (uint64_t)(hll_estimate(mb->ctr.hll) * 1.25) + 64) : d;
    const void* content = bytes ? (const void*)d_text : (const void*)w.sym[cur ^ 1].p;
    DedupResult r = dedup_commit(g, lv, d, content, w.fpv[cur].p, w.sym[cur].p, w.fpv[cur].p, est,
                                 o, w, s, &pe);
    zero_counters(w.fin.p, s);
    launch_segments(cur_off, k, w.bits.p, w.tile_base.p, d, nullptr, w.off[cur].p, s);
    launch_finish(cur_off, w.off[cur].p, k, w.sym[cur].p, lv, g->c_level.p + c_base,
                  g->c_sym.p + c_base, w.fin.p, s);
    pe.rec(7, s);
    // dedup_commit has waited for the insert: every earlier event is complete
    const uint64_t t_classify = pe.ns(0, 1), t_emit = pe.ns(2, 8);
    const uint64_t t_insert = pe.ns(3, 4), t_rank = pe.ns(4, 5);
    prev = Stat{active_len, d, r.u_new, r.q_new, 0, r.probes, r.compares, g->levels[lv - 1].tcap,
                t_classify + t_emit + t_insert + t_rank, t_classify, t_emit, t_insert, t_rank, 0, 0,
                r.combined ? 1u : 0u};
    pending = true;
    cur_off = w.off[cur].p;
    n_i = d;
    cur ^= 1;
    ++lv;
  }
};

static void build_core(lcg_grammar* g, const uint8_t* d_text, const uint64_t* d_off, uint32_t k,
                       const std::vector<uint64_t>& h_off, const Opts& o, Work& w, hipStream_t s) {
  Cohort c(g, d_text, d_off, k, h_off, o, w, s);
  while (!c.done) c.step(s);
}

// MergeGrams(a, b): a absorbs b level by level (Sec. 3.6).
static void level_to_host(Level& L, bool bytes, hipStream_t s);
static void level_to_device(Level& L, bool bytes, hipStream_t s);

// MergeGrams (Sec. 3.6) of b into a.  With a_host, a's levels sit in pinned
// host memory and come to the device one at a time: level lv while its rules
// are merged, with level lv - 1 (whose fingerprints name lv's keys) kept until
// lv is done.
static void merge_core(lcg_grammar* a, const lcg_grammar* b, Work& w, hipStream_t s,
                       bool a_host = false) {
  ++a->version;
  if (a->seed != b->seed) throw LcgError{LCG_ESEED, "grammars use different hash families"};
  const uint32_t ka = a->k, kb = b->k;
  a->c_level.grow(ka + kb, ka, s);
  a->c_sym.grow(ka + kb, ka, s);
  launch_c_merge(b->c_level.p, b->c_sym.p, kb, 0, nullptr, a->c_level.p + ka, a->c_sym.p + ka, s);
  w.lut.need(256, s);
  w.ctr.need(1, s);
  launch_f0_lut(w.lut.p, a->H.lv[0].a, a->H.lv[0].b, s);
  Opts o;
  int cur = 0;
  const uint32_t* remap_prev = nullptr;
  for (size_t lv = 1; lv <= b->levels.size(); ++lv) {
    if (a_host && lv <= a->levels.size()) level_to_device(a->levels[lv - 1], lv == 1, s);
    ensure_level(a, lv, s);
    const Level& B = b->levels[lv - 1];
    const bool bytes = lv == 1;
    const uint32_t ub = B.u;
    w.remap[cur].need(std::max<uint32_t>(ub, 1), s);
    if (ub) {
      w.pstart.need(ub, s);
      w.plen.need(ub, s);
      w.key.need(ub, s);
      w.wkey.need(2 * (size_t)ub, s);
      const void* content;
      const uint32_t* f_prev = bytes ? w.lut.p : a->levels[lv - 2].fp.p;
      if (bytes) {
        w.content8.need(B.q, s);
        content = w.content8.p;
        launch_merge_prepare(true, ub, B.off.p, B.rhs8.p, nullptr, f_prev, a->H.lv[lv], 0,
                             w.content8.p, w.pstart.p, w.plen.p, w.key.p, w.wkey.p, s);
      } else {
        w.content32.need(B.q, s);
        content = w.content32.p;
        launch_merge_prepare(false, ub, B.off.p, B.rhs32.p, remap_prev, f_prev, a->H.lv[lv], 0,
                             w.content32.p, w.pstart.p, w.plen.p, w.key.p, w.wkey.p, s);
      }
      dedup_commit(a, (uint32_t)lv, ub, content, B.fp.p, w.remap[cur].p, nullptr, ub, o, w, s);
      launch_c_merge(b->c_level.p, b->c_sym.p, kb, (uint32_t)lv, w.remap[cur].p,
                     a->c_level.p + ka, a->c_sym.p + ka, s);
    }
    remap_prev = w.remap[cur].p;
    cur ^= 1;
    if (a_host && lv >= 2) level_to_host(a->levels[lv - 2], lv == 2, s);
  }
  if (a_host && !b->levels.empty())
    level_to_host(a->levels[b->levels.size() - 1], b->levels.size() == 1, s);
  a->k += kb;
  sync(s);
}

// a level's arrays to pinned host memory (released on the device), and back
static void level_to_host(Level& L, bool bytes, hipStream_t s) {
  if (L.on_host) return;
  const size_t rb = L.q * (bytes ? 1 : 4);
  HIP_CHECK(hipMemcpyAsync(L.h_off.need((L.u + 1) * 8ull), L.off.p, (L.u + 1) * 8ull,
                           hipMemcpyDeviceToHost, s));
  if (rb)
    HIP_CHECK(hipMemcpyAsync(L.h_rhs.need(rb), bytes ? (const void*)L.rhs8.p : (const void*)L.rhs32.p,
                             rb, hipMemcpyDeviceToHost, s));
  if (L.u)
    HIP_CHECK(hipMemcpyAsync(L.h_fp.need(L.u * 4ull), L.fp.p, L.u * 4ull, hipMemcpyDeviceToHost, s));
  if (L.tcap && L.table.p)
    HIP_CHECK(hipMemcpyAsync(L.h_table.need(L.tcap * sizeof(Slot)), L.table.p,
                             L.tcap * sizeof(Slot), hipMemcpyDeviceToHost, s));
  sync(s);
  L.off.reset();
  L.rhs8.reset();
  L.rhs32.reset();
  L.fp.reset();
  L.table.reset();
  L.on_host = true;
}

static void level_to_device(Level& L, bool bytes, hipStream_t s) {
  if (!L.on_host) return;
  const size_t rb = L.q * (bytes ? 1 : 4);
  L.off.need(L.u + 1, s);
  HIP_CHECK(hipMemcpyAsync(L.off.p, L.h_off.p, (L.u + 1) * 8ull, hipMemcpyHostToDevice, s));
  if (rb) {
    if (bytes) {
      L.rhs8.need(L.q, s);
      HIP_CHECK(hipMemcpyAsync(L.rhs8.p, L.h_rhs.p, rb, hipMemcpyHostToDevice, s));
    } else {
      L.rhs32.need(L.q, s);
      HIP_CHECK(hipMemcpyAsync(L.rhs32.p, L.h_rhs.p, rb, hipMemcpyHostToDevice, s));
    }
  }
  if (L.u) {
    L.fp.need(L.u, s);
    HIP_CHECK(hipMemcpyAsync(L.fp.p, L.h_fp.p, L.u * 4ull, hipMemcpyHostToDevice, s));
  }
  if (L.tcap && L.h_table.p) {
    L.table.need(L.tcap, s);
    HIP_CHECK(hipMemcpyAsync(L.table.p, L.h_table.p, L.tcap * sizeof(Slot), hipMemcpyHostToDevice,
                             s));
  }
  sync(s);
  L.h_off.reset();
  L.h_rhs.reset();
  L.h_fp.reset();
  L.h_table.reset();
  L.on_host = false;
}

void sink_to_host(lcg_grammar* g, hipStream_t s) {
  ++g->version;  // cached device views of the levels are stale
  for (size_t i = 0; i < g->levels.size(); ++i) level_to_host(g->levels[i], i == 0, s);
}

void sink_to_device(lcg_grammar* g, hipStream_t s) {
  ++g->version;
  for (size_t i = 0; i < g->levels.size(); ++i) level_to_device(g->levels[i], i == 0, s);
}

void sink_flush(lcg_grammar* sink, const lcg_grammar* buf, hipStream_t s) {
  Work w;
  merge_core(sink, buf, w, s, true);
}

// device memory a grammar holds in its levels and C
uint64_t device_bytes(const lcg_grammar* g) {
  uint64_t b = g->c_level.cap + 4ull * g->c_sym.cap;
  for (const Level& L : g->levels)
    b += 8ull * L.off.cap + L.rhs8.cap + 4ull * L.rhs32.cap + 4ull * L.fp.cap +
         sizeof(Slot) * L.table.cap;
  return b;
}

static std::vector<uint64_t> fetch_offsets(const uint64_t* d_off, uint32_t k, hipStream_t s) {
  if (k == 0) throw LcgError{LCG_EINVAL, "k must be >= 1"};
  if (!d_off) throw LcgError{LCG_EINVAL, "offsets are NULL"};
  std::vector<uint64_t> h(k + 1);
  HIP_CHECK(hipMemcpyAsync(h.data(), d_off, sizeof(uint64_t) * (k + 1), hipMemcpyDeviceToHost, s));
  sync(s);
  if (h[0] != 0) throw LcgError{LCG_EINVAL, "offsets[0] must be 0"};
  for (uint32_t j = 0; j < k; ++j)
    if (h[j + 1] <= h[j])
      throw LcgError{LCG_EINVAL, "string " + std::to_string(j) + " is empty or offsets decrease"};
  return h;
}

static void check_budget(const Opts& o, uint64_t n, uint32_t k) {
  if (o.budget && build_bytes(n, k) > o.budget)
    throw LcgError{LCG_ENOMEM, "input needs more than hbm_budget bytes of working memory"};
}

// What a call that extends a grammar in place (lcg_build_into, lcg_merge)
// restores if it fails part way.
struct Snapshot {
  uint32_t k;
  std::vector<std::pair<uint32_t, uint64_t>> uq;  // rules and rhs length per level
  size_t n_stats;
};

static Snapshot snapshot(const lcg_grammar* g) {
  Snapshot sn{g->k, {}, g->stats.size()};
  for (const Level& L : g->levels) sn.uq.emplace_back(L.u, L.q);
  return sn;
}

// Undo a failed in-place call: levels and strings shrink back to the
// snapshot, and every dictionary is rebuilt from the rules kept (rank below
// the level's restored count), which drops the failed call's claims and
// rules without breaking any probe sequence.  A grammar that cannot be
// restored is marked unusable.
static void rollback(lcg_grammar* g, const Snapshot& sn, hipStream_t s) noexcept {
  if (hipStreamSynchronize(s) != hipSuccess) {
    (void)hipGetLastError();
    g->poisoned = true;
    return;
  }
  try {
    pool().flush(s);
    while (g->levels.size() > sn.uq.size()) {
      g->levels.back().table.reset_after(s);
      g->levels.pop_back();
    }
    DBuf<Counters> ctr;
    ctr.need(1, s);
    for (size_t i = 0; i < g->levels.size(); ++i) {
      Level& L = g->levels[i];
      L.u = sn.uq[i].first;
      L.q = sn.uq[i].second;
      if (!L.tcap || !L.table.p) continue;
      DBuf<Slot> nt;
      nt.need(L.tcap, s);
      launch_fill_slots(nt.p, L.tcap, s);
      zero_counters(ctr.p, s);
      launch_rehash(L.table.p, L.tcap, nt.p, L.tcap - 1, L.u, ctr.p, s);
      const Counters c = read_dev(ctr.p, s);
      if (c.overflow) throw LcgError{LCG_ETABLE, "rebuild failed"};
      L.table.reset_after(s);
      L.table = std::move(nt);
    }
    g->k = sn.k;
    g->stats.resize(sn.n_stats);
    ++g->version;
    sync(s);
  } catch (...) {
    (void)hipGetLastError();
    g->poisoned = true;
  }
}

// Run f, which extends g in place; on failure restore g and rethrow.
template <typename F>
static void restoring(lcg_grammar* g, hipStream_t s, F&& f) {
  const Snapshot sn = snapshot(g);
  try {
    f();
  } catch (...) {
    rollback(g, sn, s);
    throw;
  }
}

static void build_any(lcg_grammar* g, const uint8_t* d_text, const uint64_t* d_off, uint32_t k,
                      const Opts& o, hipStream_t s) {
  ++g->version;
  std::vector<uint64_t> h_off = fetch_offsets(d_off, k, s);
  if (!d_text) throw LcgError{LCG_EINVAL, "text is NULL"};
  Work w;
  if (o.mode == LCG_MODE_BATCHED) {
    check_budget(o, h_off[k], k);
    build_core(g, d_text, d_off, k, h_off, o, w, s);
    w.release_after(s);
    sync(s);
    return;
  }
  // plain form: one grammar per string (its own launches every round), then MergeGrams
  uint64_t max_len = 0;
  for (uint32_t j = 0; j < k; ++j) max_len = std::max(max_len, h_off[j + 1] - h_off[j]);
  check_budget(o, max_len, 1);
  std::vector<uint64_t> pairs(2 * (size_t)k);
  for (uint32_t j = 0; j < k; ++j) {
    pairs[2 * j] = 0;
    pairs[2 * j + 1] = h_off[j + 1] - h_off[j];
  }
  DBuf<uint64_t> d_pairs;
  d_pairs.need(pairs.size(), s);
  HIP_CHECK(hipMemcpyAsync(d_pairs.p, pairs.data(), sizeof(uint64_t) * pairs.size(),
                           hipMemcpyHostToDevice, s));
  for (uint32_t j = 0; j < k; ++j) {
    lcg_grammar gj(g->seed);
    std::vector<uint64_t> one{0, pairs[2 * j + 1]};
    build_core(&gj, d_text + h_off[j], d_pairs.p + 2 * j, 1, one, o, w, s);
    merge_core(g, &gj, w, s);
    g->stats.insert(g->stats.end(), gj.stats.begin(), gj.stats.end());
  }
  d_pairs.reset_after(s);
  w.release_after(s);
  sync(s);
}

static void expand_core(lcg_grammar* g, uint32_t j, uint8_t* d_out, uint64_t cap, uint64_t* out_len,
                        hipStream_t s) {
  if (j >= g->k) throw LcgError{LCG_EINVAL, "string index out of range"};
  uint8_t lvl;
  uint32_t sym;
  HIP_CHECK(hipMemcpyAsync(&lvl, g->c_level.p + j, 1, hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipMemcpyAsync(&sym, g->c_sym.p + j, 4, hipMemcpyDeviceToHost, s));
  sync(s);
  if (lvl == 0) {
    if (out_len) *out_len = 1;
    if (cap < 1) throw LcgError{LCG_EINVAL, "output buffer too small"};
    HIP_CHECK(hipMemcpyAsync(d_out, &sym, 1, hipMemcpyHostToDevice, s));
    sync(s);
    return;
  }
  DBuf<uint32_t> cur, nxt;
  DBuf<uint64_t> lens, pos, tmp;
  cur.need(1, s);
  HIP_CHECK(hipMemcpyAsync(cur.p, &sym, 4, hipMemcpyHostToDevice, s));
  uint64_t m = 1;
  for (uint32_t lv = lvl; lv >= 1; --lv) {
    const Level& L = g->levels[lv - 1];
    lens.need(m, s);
    pos.need(m + 1, s);
    tmp.need(std::max<size_t>(scan_tmp_words(m), 1), s);
    launch_expand_lens(cur.p, m, L.off.p, lens.p, s);
    scan_exclusive(lens.p, pos.p, m, tmp.p, s);
    const uint64_t total = read_dev(pos.p + m, s);
    if (lv == 1) {
      if (out_len) *out_len = total;
      if (total <= cap) launch_expand_emit(true, cur.p, m, L.off.p, L.rhs8.p, pos.p, d_out, s);
      sync(s);
      if (total > cap) throw LcgError{LCG_EINVAL, "output buffer too small"};
      return;
    }
    nxt.need(total, s);
    launch_expand_emit(false, cur.p, m, L.off.p, L.rhs32.p, pos.p, nxt.p, s);
    std::swap(cur, nxt);
    m = total;
  }
}

// Expansion lengths (bytes) of every rule of g, per level, kept until g changes.
void ensure_explen(lcg_grammar* g, hipStream_t s) {
  if (g->explen_version == g->version && g->explen.size() == g->levels.size()) return;
  const size_t nl = g->levels.size();
  g->explen.resize(nl);
  g->gc.resize(nl);
  std::vector<const uint64_t*> ptrs(std::max<size_t>(nl, 1), nullptr);
  std::vector<LevelPtrs> lp(std::max<size_t>(nl, 1));
  for (size_t i = 0; i < nl; ++i) {
    lp[i].off = g->levels[i].off.p;
    lp[i].rhs = i ? (const void*)g->levels[i].rhs32.p : (const void*)g->levels[i].rhs8.p;
  }
  for (size_t i = 0; i < nl; ++i) {
    const Level& L = g->levels[i];
    g->explen[i].need(std::max<uint32_t>(L.u, 1), s);
    launch_explen(L.off.p, i ? L.rhs32.p : nullptr, i ? g->explen[i - 1].p : nullptr, L.u,
                  g->explen[i].p, s);
    ptrs[i] = g->explen[i].p;
    if (i >= 3) {  // levels >= 4: grandchildren counts for the expansion
      g->gc[i].need(std::max<uint32_t>(L.u, 1), s);
      launch_gc(L.off.p, L.rhs32.p, g->levels[i - 1].off.p, L.u, g->gc[i].p, s);
    }
  }
  g->explen_ptrs.need(ptrs.size(), s);
  HIP_CHECK(hipMemcpyAsync(g->explen_ptrs.p, ptrs.data(), ptrs.size() * sizeof(void*),
                           hipMemcpyHostToDevice, s));
  g->level_ptrs.need(lp.size(), s);
  HIP_CHECK(hipMemcpyAsync(g->level_ptrs.p, lp.data(), lp.size() * sizeof(LevelPtrs),
                           hipMemcpyHostToDevice, s));
  sync(s);  // ptrs is a host temporary
  g->explen_version = g->version;
}

// Items of a level: the children written by the expansion first, then the
// strings entering at that level.
static inline uint64_t children_before(uint64_t m_next, uint64_t entering) {
  return m_next - entering;
}

// Device scratch of expand_strings_core: `fixed` regions live for the whole
// call; `side(w, ...)` returns side w's region, replacing what that side held
// before (the items of one level live on one side while the next level's are
// written to the other).
class XsScratch {
 public:
  virtual ~XsScratch() = default;
  virtual void* fixed(size_t bytes, hipStream_t s) = 0;
  virtual void* side(int w, size_t bytes, hipStream_t s) = 0;
};

// From the library's caching pool.
class PoolXs final : public XsScratch {
 public:
  void* fixed(size_t bytes, hipStream_t s) override {
    fixed_.emplace_back();
    fixed_.back().need(std::max<size_t>(bytes, 1), s);
    return fixed_.back().p;
  }
  void* side(int w, size_t bytes, hipStream_t s) override {
    side_[w].need(std::max<size_t>(bytes, 1), s);
    return side_[w].p;
  }

 private:
  std::vector<DBuf<uint8_t>> fixed_;
  DBuf<uint8_t> side_[2];
};

// From a fixed device region (no allocation): fixed regions from the bottom
// up, side 0 above them, side 1 down from the top.  A request that does not
// fit is refused before the region is written.
class ArenaXs final : public XsScratch {
 public:
  ArenaXs(uint8_t* base, size_t cap) : base_(base), cap_(cap), lo_(0), top0_(0), bot1_(cap) {}
  void* fixed(size_t bytes, hipStream_t) override {
    if (top0_ != lo_) throw LcgError{LCG_EHIP, "internal: fixed scratch after a side region"};
    const size_t b = round(bytes);
    if (lo_ + b > bot1_) too_big();
    void* p = base_ + lo_;
    lo_ += b;
    top0_ = lo_;
    return p;
  }
  void* side(int w, size_t bytes, hipStream_t) override {
    const size_t b = round(bytes);
    if (w == 0) {
      if (lo_ + b > bot1_) too_big();
      top0_ = lo_ + b;
      return base_ + lo_;
    }
    if (b > cap_ || cap_ - b < top0_) too_big();
    bot1_ = cap_ - b;
    return base_ + bot1_;
  }

 private:
  static size_t round(size_t b) { return (std::max<size_t>(b, 1) + 255) & ~size_t(255); }
  [[noreturn]] void too_big() const {
    throw LcgError{LCG_EINVAL, "the expansion needs more than the " +
                                   std::to_string(cap_ >> 20) +
                                   " MiB of fixed scratch of lcg_expand_strings_noalloc"};
  }
  uint8_t* base_;
  size_t cap_, lo_, top0_, bot1_;
};

// Strings j0..j1-1 expanded together, top-down by byte positions (see
// launch_xs_*): every symbol carries the position of its expansion, so a
// level is one pass over its symbols, in any order.  With `prepared` the
// expansion lengths must already be current (nothing is allocated for them).
static void expand_strings_core(lcg_grammar* g, uint32_t j0, uint32_t j1, uint8_t* d_out,
                                uint64_t cap, uint64_t* d_offsets, uint64_t* total_out,
                                hipStream_t s, XsScratch& sc, bool prepared = false) {
  if (j0 > j1 || j1 > g->k) throw LcgError{LCG_EINVAL, "string range out of bounds"};
  const uint32_t ks = j1 - j0;
  std::vector<uint8_t> h_level(ks);
  if (ks) {
    HIP_CHECK(hipMemcpyAsync(h_level.data(), g->c_level.p + j0, ks, hipMemcpyDeviceToHost, s));
    sync(s);
  }
  uint32_t top = 0;
  for (uint8_t v : h_level) top = std::max<uint32_t>(top, v);
  if (top > g->levels.size()) throw LcgError{LCG_EHIP, "internal: C entry above the top level"};
  std::vector<uint64_t> entering(top + 1, 0);
  for (uint8_t v : h_level) ++entering[v];
  if (prepared) {
    if (g->explen_version != g->version || g->explen.size() != g->levels.size())
      throw LcgError{LCG_EINVAL, "the grammar's expansion lengths are not prepared (call "
                                 "lcg_expand_strings once after the grammar changes)"};
  } else {
    ensure_explen(g, s);
  }
  const uint8_t* cl = g->c_level.p + j0;
  const uint32_t* cs = g->c_sym.p + j0;
  auto fixed64 = [&](size_t n) { return static_cast<uint64_t*>(sc.fixed(n * 8, s)); };
  uint64_t* len = fixed64(std::max<uint32_t>(ks, 1));
  uint64_t* str_off = fixed64(ks + 1);
  uint64_t* ctr = fixed64(2);  // [0]: items of the next level, [1]: children count
  uint64_t* extra = fixed64(1);
  uint64_t* tmp = fixed64(std::max<size_t>(scan_tmp_words(std::max<uint32_t>(ks, 1)), 1));
  uint64_t total = 0;
  if (ks) {
    launch_xs_strlen(cl, cs, ks, g->explen_ptrs.p, len, s);
    scan_exclusive(len, str_off, ks, tmp, s);
    total = read_dev(str_off + ks, s);
  } else {
    launch_zero(str_off, sizeof(uint64_t), s);
  }
  if (total_out) *total_out = total;
  if (total > cap) throw LcgError{LCG_EINVAL, "output buffer too small"};
  // the items of a level on one side: m symbols, then their m positions
  uint32_t* sym[2] = {nullptr, nullptr};
  uint64_t* pos[2] = {nullptr, nullptr};
  auto items = [&](int w, uint64_t m) {
    const size_t n = std::max<uint64_t>(m, 1);
    uint8_t* p = static_cast<uint8_t*>(sc.side(w, n * 8 + ((n * 4 + 255) & ~size_t(255)), s));
    sym[w] = reinterpret_cast<uint32_t*>(p);
    pos[w] = reinterpret_cast<uint64_t*>(p + ((n * 4 + 255) & ~size_t(255)));
  };
  int cur = 0;
  uint64_t m = entering[top];
  uint64_t children = 0;  // children of the current level's items
  launch_zero(ctr, 2 * sizeof(uint64_t), s);
  if (top >= 1) {
    items(cur, m);
    launch_xs_enter(cl, cs, ks, top, str_off, sym[cur], pos[cur], ctr, d_out, s);
    if (top >= 3) {
      launch_xs_count(sym[cur], m, g->levels[top - 1].off.p, ctr + 1, s);
      children = read_dev(ctr + 1, s);
    }
  }
  for (uint32_t lv = top; lv >= 1; --lv) {
    const Level& L = g->levels[lv - 1];
    if (lv == 1) {
      launch_xs_expand(true, sym[cur], pos[cur], m, L.off.p, L.rhs8.p, nullptr, nullptr,
                       nullptr, nullptr, nullptr, nullptr, d_out, s);
      break;
    }
    if (lv == 2) {
      // level-2 items write the bytes of their level-1 children in place; the
      // level-1 items left are the strings entering there (their room is
      // taken first, so that a refusal comes before any byte is written)
      const uint64_t m1 = entering[1];
      items(cur ^ 1, m1);
      const Level& L1 = g->levels[0];
      launch_xs_bytes2(sym[cur], pos[cur], m, L.off.p, L.rhs32.p, L1.off.p, L1.rhs8.p, d_out, s);
      launch_zero(ctr, 2 * sizeof(uint64_t), s);
      launch_xs_enter(cl, cs, ks, 1, str_off, sym[cur ^ 1], pos[cur ^ 1], ctr, d_out, s);
      cur ^= 1;
      m = m1;
      continue;
    }
    // the children are counted by the previous pass (or above, at the top);
    // this pass counts the grandchildren, except those of entering strings
    const uint64_t m_next = children + entering[lv - 1];
    items(cur ^ 1, m_next);
    launch_zero(ctr, 2 * sizeof(uint64_t), s);
    // grandchildren are counted while they will be items (level >= 2)
    const uint64_t* off_below = lv >= 4 ? g->levels[lv - 2].off.p : nullptr;
    launch_xs_expand(false, sym[cur], pos[cur], m, L.off.p, L.rhs32.p, g->explen[lv - 2].p,
                     lv >= 4 ? g->gc[lv - 1].p : nullptr, sym[cur ^ 1], pos[cur ^ 1], ctr,
                     ctr + 1, nullptr, s);
    launch_xs_enter(cl, cs, ks, lv - 1, str_off, sym[cur ^ 1], pos[cur ^ 1], ctr, d_out, s);
    if (lv >= 4) {
      children = read_dev(ctr + 1, s);
      if (entering[lv - 1]) {
        // the entering strings' own children
        launch_zero(extra, sizeof(uint64_t), s);
        launch_xs_count(sym[cur ^ 1] + children_before(m_next, entering[lv - 1]),
                        entering[lv - 1], off_below, extra, s);
        children += read_dev(extra, s);
      }
    }
    cur ^= 1;
    m = m_next;
  }
  if (entering[0]) launch_xs_enter(cl, cs, ks, 0, str_off, nullptr, nullptr, ctr, d_out, s);
  if (d_offsets)
    HIP_CHECK(hipMemcpyAsync(d_offsets, str_off, (ks + 1) * sizeof(uint64_t),
                             hipMemcpyDeviceToDevice, s));
  sync(s);
}

// The fixed scratch of lcg_expand_strings_noalloc: one copy per device,
// reserved when the library's code object is loaded there and kept until the
// process ends.  Host code must not use the array's name as an address: its
// device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kNoAllocScratch = 64ull << 20;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratch];

static uint8_t* scratch_ptr() {
  static std::mutex mu;
  static std::unordered_map<int, uint8_t*> per_device;
  int dev = 0;
  HIP_CHECK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto it = per_device.find(dev);
  if (it != per_device.end()) return it->second;
  void* p = nullptr;
  HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) throw LcgError{LCG_EHIP, "no device address for the fixed scratch"};
  per_device.emplace(dev, static_cast<uint8_t*>(p));
  return static_cast<uint8_t*>(p);
}

// Serving session: batches admitted at any time are compressed into one
// running grammar round by round; every step advances each admitted batch by
// one round (a batch whose sequence is short runs all its remaining rounds),
// so that a batch admitted while others are deep in their rounds starts at
// round 1 at once instead of waiting for them to finish.  The batches share
// g's dictionaries: each phrase is looked up in the level's dictionary and
// added if absent (App. A.2's BuildGram against a grammar being extended).
struct Session {
  struct Entry {
    uint64_t ticket;
    uint64_t bytes;  // working-memory bound of the batch
    std::unique_ptr<Work> w;
    std::unique_ptr<Cohort> c;
  };
  lcg_grammar* g;
  Opts o;
  std::vector<Entry> active;  // in admission order
  uint64_t next_ticket = 1;
  uint64_t held = 0;          // working-memory bound of the active batches
  bool failed = false;
};

}  // namespace lcg

struct lcg_session {
  lcg::Session s;
};

using namespace lcg;

extern "C" {

void lcg_opts_init(lcg_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->mode = LCG_MODE_BATCHED;
}

lcg_status lcg_new(uint64_t seed, lcg_grammar_t* out) {
  return guard([&] {
    if (!out) throw LcgError{LCG_EINVAL, "out is NULL"};
    *out = new lcg_grammar(seed);
  });
}

lcg_status lcg_build(const uint8_t* d_text, const uint64_t* d_offsets, uint32_t k,
                     const lcg_opts* opts, hipStream_t stream, lcg_grammar_t* out) {
  return guard([&] {
    if (!out) throw LcgError{LCG_EINVAL, "out is NULL"};
    Opts o = read_opts(opts);
    lcg_grammar* g = new lcg_grammar(o.seed);
    try {
      build_any(g, d_text, d_offsets, k, o, stream);
    } catch (...) {
      (void)hipStreamSynchronize(stream);
      delete g;
      throw;
    }
    *out = g;
  });
}

lcg_status lcg_tune(const uint8_t* d_text, const uint64_t* d_offsets, uint32_t k,
                    const lcg_opts* base, hipStream_t stream, lcg_opts* best, double* best_ms) {
  return guard([&] {
    if (!best) throw LcgError{LCG_EINVAL, "best is NULL"};
    const Opts o0 = read_opts(base);
    if (o0.mode != LCG_MODE_BATCHED) throw LcgError{LCG_EINVAL, "tuning is for the batched form"};
    lcg_opts cur;
    if (base) cur = *base;
    else lcg_opts_init(&cur);
    // explicit values, so that candidates compare with the current setting
    cur.tail_log2 = o0.tail_log2;
    cur.table_load_log2 = o0.table_load_log2;
    cur.combine_log2 = o0.combine_log2;
    hipEvent_t e0, e1;
    HIP_CHECK(hipEventCreate(&e0));
    HIP_CHECK(hipEventCreate(&e1));
    auto time_build = [&](const lcg_opts& c) {
      const Opts o = read_opts(&c);
      lcg_grammar* g = new lcg_grammar(o.seed);
      float ms = 0;
      try {
        HIP_CHECK(hipEventRecord(e0, stream));
        build_any(g, d_text, d_offsets, k, o, stream);
        HIP_CHECK(hipEventRecord(e1, stream));
        HIP_CHECK(hipEventSynchronize(e1));
        HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
      } catch (...) {
        (void)hipStreamSynchronize(stream);
        delete g;
        throw;
      }
      delete g;
      return (double)ms;
    };
    struct Knob {
      uint32_t lcg_opts::*field;
      std::vector<uint32_t> values;
    };
    const Knob knobs[] = {{&lcg_opts::tail_log2, {16, 18, 20, 22, 24}},
                          {&lcg_opts::table_load_log2, {1, 2}},
                          {&lcg_opts::combine_log2, {4, 5, 6, 31}}};
    try {
      time_build(cur);  // warm-up: pool, code objects, caches
      double best_t = time_build(cur);
      for (const Knob& kn : knobs) {
        for (uint32_t v : kn.values) {
          if (cur.*(kn.field) == v) continue;
          lcg_opts c = cur;
          c.*(kn.field) = v;
          const double t = time_build(c);
          if (t < best_t * 0.98) {  // a clear gain, not noise
            cur = c;
            best_t = t;
          }
        }
      }
      *best = cur;
      if (best_ms) *best_ms = best_t;
    } catch (...) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  });
}

lcg_status lcg_build_into(lcg_grammar_t g, const uint8_t* d_text, const uint64_t* d_offsets,
                          uint32_t k, const lcg_opts* opts, hipStream_t stream,
                          uint32_t* first_index) {
  return guard([&] {
    live(g);
    Opts o = read_opts(opts);
    if (opts && o.seed != g->seed) throw LcgError{LCG_ESEED, "opts seed differs from the grammar's"};
    Opts oo = o;
    oo.mode = LCG_MODE_BATCHED;
    uint32_t first = g->k;
    restoring(g, stream, [&] { build_any(g, d_text, d_offsets, k, oo, stream); });
    if (first_index) *first_index = first;
  });
}

lcg_status lcg_reserve(lcg_grammar_t g, const uint64_t* rules, uint32_t levels,
                       hipStream_t stream) {
  return guard([&] {
    live(g);
    if (levels && !rules) throw LcgError{LCG_EINVAL, "rules is NULL"};
    if (levels > kMaxReserveLevels) throw LcgError{LCG_EINVAL, "too many levels"};
    for (uint32_t i = 0; i < levels; ++i)
      if (rules[i] > kMaxReserveRules)
        throw LcgError{LCG_ETABLE, "reservation beyond the dictionary capacity limit"};
    if (g->reserve.size() < levels) g->reserve.resize(levels, 0);
    Opts o;  // reserved room is sized at the default load
    Work w;
    w.ctr.need(1, stream);
    for (uint32_t i = 0; i < levels; ++i) {
      g->reserve[i] = rules[i];
      // an existing level grows (and rehashes) now rather than in a later build
      if (i < g->levels.size() && rules[i]) ensure_table(g->levels[i], rules[i], o, w, stream);
    }
    sync(stream);
  });
}

lcg_status lcg_merge(lcg_grammar_t a, lcg_grammar_t b, hipStream_t stream) {
  return guard([&] {
    live(a);
    live(b);
    if (a == b) throw LcgError{LCG_EINVAL, "cannot merge a grammar into itself"};
    Work w;
    restoring(a, stream, [&] { merge_core(a, b, w, stream); });
  });
}

lcg_status lcg_session_new(lcg_grammar_t g, const lcg_opts* opts, lcg_session_t* out) {
  return guard([&] {
    live(g);
    if (!out) throw LcgError{LCG_EINVAL, "out is NULL"};
    Opts o = read_opts(opts);
    if (opts && o.seed != g->seed) throw LcgError{LCG_ESEED, "opts seed differs from the grammar's"};
    o.mode = LCG_MODE_BATCHED;
    lcg_session* ss = new lcg_session();
    ss->s.g = g;
    ss->s.o = o;
    *out = ss;
  });
}

lcg_status lcg_session_admit(lcg_session_t ss, const uint8_t* d_text, const uint64_t* d_offsets,
                             uint32_t k, hipStream_t stream, uint32_t* first_index,
                             uint64_t* ticket) {
  return guard([&] {
    if (!ss) throw LcgError{LCG_EINVAL, "session is NULL"};
    Session& S = ss->s;
    if (S.failed) throw LcgError{LCG_EINVAL, "the session failed earlier"};
    lcg_grammar* g = live(S.g);
    if (!d_text) throw LcgError{LCG_EINVAL, "text is NULL"};
    std::vector<uint64_t> h_off = fetch_offsets(d_offsets, k, stream);
    const uint64_t need = build_bytes(h_off[k], k);
    if (S.o.budget && (need > S.o.budget || (!S.active.empty() && S.held + need > S.o.budget)))
      throw LcgError{LCG_ENOMEM, "the batch does not fit hbm_budget beside the active ones"};
    const uint32_t first = g->k;
    Session::Entry e{S.next_ticket, need, std::make_unique<Work>(), nullptr};
    // a failure here leaves g as it was (the batch is not admitted)
    restoring(g, stream, [&] {
      ++g->version;
      e.c = std::make_unique<Cohort>(g, d_text, d_offsets, k, h_off, S.o, *e.w, stream);
    });
    ++S.next_ticket;
    S.held += need;
    S.active.push_back(std::move(e));
    if (first_index) *first_index = first;
    if (ticket) *ticket = S.active.back().ticket;
  });
}

lcg_status lcg_session_step(lcg_session_t ss, hipStream_t stream, uint64_t* h_done, uint32_t cap,
                            uint32_t* n_done, uint32_t* n_active) {
  return guard([&] {
    if (!ss) throw LcgError{LCG_EINVAL, "session is NULL"};
    Session& S = ss->s;
    if (S.failed) throw LcgError{LCG_EINVAL, "the session failed earlier"};
    lcg_grammar* g = live(S.g);
    if (cap < S.active.size())
      throw LcgError{LCG_EINVAL, "h_done has room for fewer tickets than batches are active"};
    if (!h_done && !S.active.empty()) throw LcgError{LCG_EINVAL, "h_done is NULL"};
    uint32_t nd = 0;
    try {
      if (!S.active.empty()) ++g->version;
      for (auto& e : S.active) e.c->step(stream);
      std::vector<Session::Entry> keep;
      for (auto& e : S.active) {
        if (e.c->done) {
          h_done[nd++] = e.ticket;
          S.held -= e.bytes;
          e.c.reset();
          e.w->release_after(stream);
        } else {
          keep.push_back(std::move(e));
        }
      }
      S.active = std::move(keep);
      sync(stream);
    } catch (...) {
      // the active batches share the grammar's dictionaries, so one of them
      // cannot be taken back alone: the session and the grammar are given up
      (void)hipStreamSynchronize(stream);
      (void)hipGetLastError();
      S.failed = true;
      g->poisoned = true;
      S.active.clear();
      throw;
    }
    if (n_done) *n_done = nd;
    if (n_active) *n_active = (uint32_t)S.active.size();
  });
}

void lcg_session_free(lcg_session_t ss) {
  if (!ss) return;
  if (!ss->s.active.empty()) {
    // unfinished batches: their strings stay in C, unfinished
    ss->s.g->poisoned = true;
    (void)hipDeviceSynchronize();
  }
  delete ss;
}

lcg_status lcg_expand_strings(lcg_grammar_t g, uint32_t j0, uint32_t j1, uint8_t* d_out,
                              uint64_t cap, uint64_t* d_offsets, uint64_t* total,
                              hipStream_t stream) {
  return guard([&] {
    live(g);
    if (!d_out && cap) throw LcgError{LCG_EINVAL, "d_out is NULL"};
    PoolXs sc;
    expand_strings_core(g, j0, j1, d_out, cap, d_offsets, total, stream, sc);
  });
}

lcg_status lcg_expand_strings_noalloc(lcg_grammar_t g, uint32_t j0, uint32_t j1, uint8_t* d_out,
                                      uint64_t cap, uint64_t* d_offsets, uint64_t* total,
                                      hipStream_t stream) {
  return guard([&] {
    live(g);
    if (!d_out && cap) throw LcgError{LCG_EINVAL, "d_out is NULL"};
    ArenaXs sc(scratch_ptr(), kNoAllocScratch);
    expand_strings_core(g, j0, j1, d_out, cap, d_offsets, total, stream, sc, /*prepared=*/true);
  });
}

lcg_status lcg_expand(lcg_grammar_t g, uint32_t j, uint8_t* d_out, uint64_t cap, uint64_t* out_len,
                      hipStream_t stream) {
  return guard([&] {
    live(g);
    expand_core(g, j, d_out, cap, out_len, stream);
  });
}

lcg_status lcg_info(lcg_grammar_t g, uint64_t* seed, uint32_t* n_levels, uint32_t* k) {
  return guard([&] {
    if (!g) throw LcgError{LCG_EINVAL, "grammar is NULL"};
    if (seed) *seed = g->seed;
    if (n_levels) *n_levels = (uint32_t)g->levels.size();
    if (k) *k = g->k;
  });
}

lcg_status lcg_level_size(lcg_grammar_t g, uint32_t level, uint32_t* u, uint64_t* rhs_len) {
  return guard([&] {
    live(g);
    if (level == 0 || level > g->levels.size()) throw LcgError{LCG_EINVAL, "bad level"};
    if (u) *u = g->levels[level - 1].u;
    if (rhs_len) *rhs_len = g->levels[level - 1].q;
  });
}

lcg_status lcg_level_copy(lcg_grammar_t g, uint32_t level, uint64_t* h_rhs_off, uint32_t* h_rhs,
                          uint32_t* h_fp) {
  return guard([&] {
    live(g);
    if (level == 0 || level > g->levels.size()) throw LcgError{LCG_EINVAL, "bad level"};
    const Level& L = g->levels[level - 1];
    HIP_CHECK(hipDeviceSynchronize());
    if (h_rhs_off) HIP_CHECK(hipMemcpy(h_rhs_off, L.off.p, sizeof(uint64_t) * (L.u + 1), hipMemcpyDeviceToHost));
    if (h_fp && L.u) HIP_CHECK(hipMemcpy(h_fp, L.fp.p, sizeof(uint32_t) * L.u, hipMemcpyDeviceToHost));
    if (h_rhs && L.q) {
      if (level == 1) {
        std::vector<uint8_t> tmp(L.q);
        HIP_CHECK(hipMemcpy(tmp.data(), L.rhs8.p, L.q, hipMemcpyDeviceToHost));
        for (uint64_t i = 0; i < L.q; ++i) h_rhs[i] = tmp[i];
      } else {
        HIP_CHECK(hipMemcpy(h_rhs, L.rhs32.p, sizeof(uint32_t) * L.q, hipMemcpyDeviceToHost));
      }
    }
  });
}

lcg_status lcg_c_copy(lcg_grammar_t g, uint8_t* h_level, uint32_t* h_sym) {
  return guard([&] {
    live(g);
    HIP_CHECK(hipDeviceSynchronize());
    if (g->k && h_level) HIP_CHECK(hipMemcpy(h_level, g->c_level.p, g->k, hipMemcpyDeviceToHost));
    if (g->k && h_sym) HIP_CHECK(hipMemcpy(h_sym, g->c_sym.p, 4ull * g->k, hipMemcpyDeviceToHost));
  });
}

void lcg_host_free(lcg_host_grammar* h) {
  if (!h) return;
  for (uint32_t i = 0; h->levels && i < h->n_levels; ++i) {
    std::free(h->levels[i].rhs_off);
    std::free(h->levels[i].rhs);
    std::free(h->levels[i].fp);
  }
  std::free(h->levels);
  std::free(h->c_level);
  std::free(h->c_sym);
  std::memset(h, 0, sizeof(*h));
}

lcg_status lcg_export(lcg_grammar_t g, lcg_host_grammar* out) {
  if (out) std::memset(out, 0, sizeof(*out));
  const lcg_status st = guard([&] {
    live(g);
    if (!out) throw LcgError{LCG_EINVAL, "out is NULL"};
    auto grab = [](size_t bytes) {
      void* p = std::malloc(bytes ? bytes : 1);
      if (!p) throw LcgError{LCG_ENOMEM, "host allocation failed"};
      return p;
    };
    const uint32_t nl = (uint32_t)g->levels.size();
    out->seed = g->seed;
    out->k = g->k;
    // at least one element, so that a grammar without levels also gets a
    // non-NULL, cleared array
    const size_t nl_alloc = nl ? nl : 1;
    out->levels = static_cast<lcg_host_level*>(grab(sizeof(lcg_host_level) * nl_alloc));
    std::memset(out->levels, 0, sizeof(lcg_host_level) * nl_alloc);
    out->n_levels = nl;
    for (uint32_t i = 0; i < nl; ++i) {
      lcg_host_level& H = out->levels[i];
      H.u = g->levels[i].u;
      H.rhs_len = g->levels[i].q;
      H.rhs_off = static_cast<uint64_t*>(grab(sizeof(uint64_t) * (H.u + 1ull)));
      H.rhs = static_cast<uint32_t*>(grab(sizeof(uint32_t) * H.rhs_len));
      H.fp = static_cast<uint32_t*>(grab(sizeof(uint32_t) * H.u));
      const lcg_status s = lcg_level_copy(g, i + 1, H.rhs_off, H.rhs, H.fp);
      if (s != LCG_OK) throw LcgError{s, g_last_error};
    }
    out->c_level = static_cast<uint8_t*>(grab(g->k));
    out->c_sym = static_cast<uint32_t*>(grab(sizeof(uint32_t) * g->k));
    const lcg_status s = lcg_c_copy(g, out->c_level, out->c_sym);
    if (s != LCG_OK) throw LcgError{s, g_last_error};
  });
  if (st != LCG_OK && out) lcg_host_free(out);
  return st;
}

lcg_status lcg_stats(lcg_grammar_t g, uint64_t* h_out, uint32_t cap_rounds, uint32_t* n_rounds) {
  return guard([&] {
    live(g);
    if (n_rounds) *n_rounds = (uint32_t)g->stats.size();
    for (uint32_t r = 0; r < cap_rounds && r < g->stats.size(); ++r)
      for (int f = 0; f < LCG_STATS_FIELDS; ++f) h_out[(size_t)r * LCG_STATS_FIELDS + f] = g->stats[r][f];
  });
}

lcg_status lcg_stats_clear(lcg_grammar_t g) {
  return guard([&] {
    live(g);
    g->stats.clear();
  });
}

uint64_t lcg_build_bytes(uint64_t n, uint32_t k) { return build_bytes(n, k); }

void lcg_free(lcg_grammar_t g) { delete g; }

void lcg_release_pool(void) { pool().trim(); }

lcg_status lcg_set_allocator(const lcg_allocator* a) {
  return guard([&] {
    if (a && (!a->alloc || !a->free)) throw LcgError{LCG_EINVAL, "allocator without alloc or free"};
    pool().set_allocator(a);
  });
}

const char* lcg_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
