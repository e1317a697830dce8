/*
 * lcg.h -- C ABI of liblcg, the MI355X (gfx950) construction of stable
 * locally consistent grammars (LCG) from Diaz-Dominguez, "Efficient
 * terabyte-scale text compression via stable local consistency and parallel
 * grammar processing" (arXiv 2411.12439).
 *
 * Every operation runs as HIP kernels on the device; the host only sizes
 * buffers, launches and reads back a few counters per parsing round.
 *
 * Conventions
 *   - Pointers named d_* are HIP device memory (for instance the data_ptr()
 *     of a torch tensor on the current device).  Pointers named h_* are host
 *     memory owned by the caller.
 *   - Work is enqueued on the given stream and ordered with the caller's
 *     other work on it.  Calls that return counters (lcg_build*, lcg_merge,
 *     lcg_expand, lcg_level_size, lcg_*_copy, lcg_stats) synchronise that
 *     stream before returning.  The caller's input buffers must stay valid
 *     until the call returns.
 *   - Grammars (lcg_grammar_t) own their device memory, which comes from the
 *     library's per-device caching pool; lcg_free returns it to the pool and
 *     lcg_release_pool gives the pool back to the driver.
 *   - Every entry point returns an lcg_status; C++ exceptions never cross the
 *     ABI.  On error nothing is written to output handles and
 *     lcg_last_error() describes the failure (thread-local string).
 *   - Nonterminals are per-level ranks (App. A.1 of the paper): rule r of
 *     level i is the r-th rule of that level, its right-hand side holds ranks
 *     of level i-1 (byte values at level 1).  The library numbers the new
 *     rules of a level in order of first occurrence (string order, then
 *     position), which Sec. 3.3 allows; the CPU oracle does the same, so the
 *     two agree rank for rank.
 *   - Terminals are raw byte values 0..255.  Strings must be non-empty; a
 *     string of length one is compressed at level 0 (C[j] is its byte).
 */
#ifndef LCG_H
#define LCG_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lcg_grammar* lcg_grammar_t;

typedef enum {
  LCG_OK = 0,
  LCG_EINVAL = -1,    /* bad argument: k = 0, empty string, offsets not increasing, bad level */
  LCG_ENOMEM = -2,    /* device allocation failed or hbm_budget exceeded */
  LCG_ESEED = -3,     /* merging grammars built with different hash families */
  LCG_EOVERFLOW = -4, /* a round needs >= 2^32 phrases, or more than 63 rounds */
  LCG_ETABLE = -5,    /* dictionary still overflowing after the allowed regrowths */
  LCG_EHIP = -6       /* a HIP runtime call failed (message in lcg_last_error) */
} lcg_status;

enum {
  LCG_MODE_BATCHED = 0, /* one launch sequence per round over all strings, shared dictionaries */
  LCG_MODE_PLAIN = 1    /* one launch sequence per string per round, then MergeGrams */
};

enum {
  LCG_FLAG_TIMING = 1u,        /* record per-round device time in the round statistics */
  LCG_FLAG_TIMING_INSERT = 2u, /* record only the dictionary insert's device time, and only
                                  in rounds that read their sizes back (not in rounds queued
                                  without host reads, see tail_log2); every other time field
                                  is 0.  Two events per such round instead of about nine per
                                  round: timing every phase slows a build by a few percent */
  LCG_FLAG_FUSED_TAIL = 4u     /* run all rounds queued without host reads (tail_log2) in one
                                  cooperative launch, their phases separated by grid-wide
                                  barriers, instead of separate kernels per phase (ignored
                                  with LCG_FLAG_TIMING).  Results do not depend on it; it is
                                  slower on gfx950, where a grid-wide barrier must write back
                                  and invalidate the L2 of every XCD */
};

typedef struct {
  uint64_t seed;       /* selects the hash family H = {h^0..h^63}; grammars merge only if equal */
  uint32_t mode;       /* LCG_MODE_BATCHED or LCG_MODE_PLAIN */
  uint32_t flags;      /* LCG_FLAG_* (other bits: LCG_EINVAL) */
  uint64_t hbm_budget; /* bytes of device working memory a call may hold; 0 = unlimited */
  uint32_t key_bits;   /* test hook: if 1..30, every phrase is keyed by only this many
                          fingerprint bits, so that dictionary lookups rely on the full
                          right-hand-side comparison; 0 = normal keys */
  uint32_t table_min_log2; /* smallest dictionary capacity, log2 (6..34; 0 = 12) */
  uint32_t tail_log2;  /* rounds over at most 2^tail_log2 symbols are queued without reading
                          sizes back to the host (dictionaries are sized for the worst
                          case): separate kernels that read their sizes from device
                          memory, or, with LCG_FLAG_FUSED_TAIL, one cooperative launch;
                          1..40, 0 = 22.  Results do not depend on it. */
  uint32_t table_load_log2; /* dictionaries are sized for a load of at most 2^-table_load_log2
                               of their capacity; 1..3, 0 = 1.  Results do not depend on it. */
  uint32_t combine_log2;    /* a round whose key sketch estimates at most d / 2^combine_log2
                               new keys for its d phrases combines equal keys per chunk of
                               phrases before the dictionary; 1..30, 0 = 5, 31 = never.
                               Results do not depend on it. */
  uint32_t fail_round; /* test hook: if nonzero, the call fails with LCG_ETABLE when it
                          reaches parsing round fail_round (after the earlier rounds have
                          changed the grammar), to exercise the recovery described at
                          lcg_build_into; 0 = off */
} lcg_opts;

/* Fill *o with the defaults (seed 0, batched mode, unlimited budget). */
void lcg_opts_init(lcg_opts* o);

/*
 * BuildGram(T, H) = G (Sec. 3.3, with the fingerprint array of Sec. 3.4).
 *   d_text     device bytes of all strings, concatenated
 *   d_offsets  device uint64[k+1]; string j is d_text[offsets[j] .. offsets[j+1]),
 *              offsets[0] = 0, strictly increasing (every string non-empty)
 *   k          number of strings, >= 1
 *   opts       NULL for defaults
 *   out        receives a new grammar; free it with lcg_free
 * Rounds of RandLMSPar (Eq. 3) parse every active string, phrases are
 * fingerprinted with Eq. 4, deduplicated exactly (full right-hand-side
 * comparison behind a 64-bit key) into the level's nonterminals, and the
 * strings are rewritten for the next round until every string has length
 * one.  Errors: LCG_EINVAL, LCG_ENOMEM, LCG_EOVERFLOW, LCG_ETABLE, LCG_EHIP.
 */
lcg_status lcg_build(const uint8_t* d_text, const uint64_t* d_offsets, uint32_t k,
                     const lcg_opts* opts, hipStream_t stream, lcg_grammar_t* out);

/*
 * BuildGram(T, H, G_a, G_b) = G_a with G_a = G_b = g (App. A.2): compress a
 * new batch of strings into an existing grammar.  Each phrase is first looked
 * up in g's level dictionaries and only phrases absent from g become new
 * rules, appended to g's levels; the batch's strings are appended to C.
 * The result equals MergeGrams(g, BuildGram(batch)).
 *   first_index  receives the index in C of the batch's first string (may be NULL)
 * Same input conventions and errors as lcg_build, plus LCG_ESEED if
 * opts->seed differs from g's seed.
 * On any error g is restored to its state before the call (its string count,
 * every level's rules, and dictionaries rebuilt from the rules kept, so that
 * no entry of the failed call can be found later) and stays usable.  If the
 * restoration itself fails (for instance after an asynchronous HIP fault), g
 * is marked unusable: every later call on it except lcg_free and lcg_info
 * returns LCG_EINVAL.
 */
lcg_status lcg_build_into(lcg_grammar_t g, const uint8_t* d_text, const uint64_t* d_offsets,
                          uint32_t k, const lcg_opts* opts, hipStream_t stream,
                          uint32_t* first_index);

/*
 * Serving session (continuous batching into one running grammar, the serving
 * form of BuildGram against a grammar being extended, App. A.2): batches of
 * strings are admitted at any time and compressed into g round by round.
 * Each lcg_session_step advances every admitted batch by one parsing round
 * (a batch whose sequence has become short, at most 2^tail_log2 symbols, runs
 * all its remaining rounds in that step), so a batch admitted while others
 * are deep in their rounds starts at round 1 at the next step instead of
 * waiting for them.  Batches share g's per-level dictionaries (a phrase is
 * looked up and added if absent), so every string's rules inside g are those
 * of the string compressed alone (stability, Def. 1), and g equals, up to a
 * renaming of each level's ranks, the grammar of all admitted strings built
 * in C order; for a given sequence of calls the ranks are always the same.
 * One thread at a time may use a session.
 */
typedef struct lcg_session* lcg_session_t;

/* A session over g (which it does not own; g must outlive it).  opts as for
 * lcg_build_into (NULL: defaults; hbm_budget bounds the working memory the
 * active batches may hold together, 0 = unlimited).  Errors: LCG_EINVAL,
 * LCG_ESEED. */
lcg_status lcg_session_new(lcg_grammar_t g, const lcg_opts* opts, lcg_session_t* out);

/* Admit k strings (the input conventions of lcg_build) as one batch.  Their
 * C indices are *first_index .. *first_index + k - 1 at once; their entries
 * are final once *ticket has been reported done by lcg_session_step.  d_text
 * and d_offsets must stay valid and unchanged until then.  Errors: LCG_EINVAL
 * (bad input, or a failed session), LCG_ENOMEM (the batch's working-memory
 * bound, lcg_build_bytes, does not fit hbm_budget beside the active batches:
 * nothing is admitted, retry after a step), LCG_EHIP. */
lcg_status lcg_session_admit(lcg_session_t s, const uint8_t* d_text, const uint64_t* d_offsets,
                             uint32_t k, hipStream_t stream, uint32_t* first_index,
                             uint64_t* ticket);

/* One round of every active batch, in admission order; synchronises the
 * stream.  h_done (host, cap entries, cap >= the number of active batches)
 * receives the tickets of the batches that finished, *n_done their number
 * and *n_active (may be NULL) the batches still active.  Errors: LCG_EINVAL
 * (cap too small, a failed session); any failure of a round (LCG_ENOMEM,
 * LCG_ETABLE, LCG_EOVERFLOW, LCG_EHIP) fails the session and leaves g unusable,
 * since the active batches share its dictionaries. */
lcg_status lcg_session_step(lcg_session_t s, hipStream_t stream, uint64_t* h_done, uint32_t cap,
                            uint32_t* n_done, uint32_t* n_active);

/* Free the session (not g).  Freeing it while batches are active leaves
 * their strings unfinished and g unusable. */
void lcg_session_free(lcg_session_t s);

/*
 * Reserve dictionary room in g: rules (host, `levels` counts) gives, for
 * each level i = 1..levels, the number of rules the level's dictionary H^i
 * (Sec. 3.3, App. A.1) is to hold without growing; 0 leaves a level as it
 * is.  A dictionary that grows rehashes every rule it holds, in whichever
 * call crosses its capacity: for a running grammar fed batch after batch
 * (lcg_build_into, sessions) that is a latency spike on one batch, which a
 * reservation moves to the call that first creates the level (or to this
 * call, for levels that already exist).  Room costs 64 device bytes per
 * reserved rule (32-byte slots at load <= 1/2).  Results never depend on it.
 * Errors: LCG_EINVAL (g NULL or unusable, rules NULL with levels > 0, more
 * than 64 levels), LCG_ETABLE (more than 2^30 rules at a level), LCG_ENOMEM,
 * LCG_EHIP.
 */
lcg_status lcg_reserve(lcg_grammar_t g, const uint64_t* rules, uint32_t levels,
                       hipStream_t stream);

/*
 * MergeGrams(G_a, G_b) (Sec. 3.5-3.6), in the rank encoding of App. A.1:
 * level by level, every rule of b (right-hand side renamed into a's ranks of
 * the level below) is looked up in a's dictionary of that level; a hit reuses
 * a's rank, a miss appends the rule to a.  C_a becomes C_a . C_b.  a is
 * modified in place, b is left unchanged.  Errors: LCG_ESEED, LCG_ENOMEM,
 * LCG_EOVERFLOW, LCG_EHIP; on error a is restored as after a failed
 * lcg_build_into.
 */
lcg_status lcg_merge(lcg_grammar_t a, lcg_grammar_t b, hipStream_t stream);

/*
 * exp(C[j]) (Sec. 2.2): expand string j top-down, level by level, into
 * d_out (device, cap bytes).  *out_len receives the expansion length; if it
 * exceeds cap nothing is written and LCG_EINVAL is returned.
 */
lcg_status lcg_expand(lcg_grammar_t g, uint32_t j, uint8_t* d_out, uint64_t cap,
                      uint64_t* out_len, hipStream_t stream);

/* Expansion of strings j0..j1-1 (j0 <= j1 <= k) one after the other into
 * d_out (device, cap bytes), top-down over the levels for all of them at once
 * (the inverse of lcg_build over that range).  d_offsets (device, j1-j0+1
 * uint64, may be NULL) receives the strings' offsets in d_out; *total (host,
 * may be NULL) the total length.  If the total exceeds cap, nothing is
 * written to d_out, *total is set and LCG_EINVAL is returned (call with
 * cap = 0 to learn the size).  The stream is synchronised before returning. */
lcg_status lcg_expand_strings(lcg_grammar_t g, uint32_t j0, uint32_t j1, uint8_t* d_out,
                              uint64_t cap, uint64_t* d_offsets, uint64_t* total,
                              hipStream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * expansion as lcg_expand_strings (same arguments, results and errors), with
 * every device buffer of the call taken from a fixed scratch region of
 * 64 MiB that the library reserves once per device when it is loaded there
 * and keeps until the process ends.  It calls no hipMalloc, hipFree or other
 * allocating routine.  Limits and conditions:
 *   - the expansion lengths of g must be current: computed by an earlier
 *     lcg_expand_strings (or lcg_extract, lcg_lce, lcg_symbol_lce) call after
 *     g last changed; otherwise LCG_EINVAL;
 *   - a range whose per-level working set (16 bytes per symbol of a level
 *     being expanded, two levels at a time, plus 40 bytes per string) does not
 *     fit the 64 MiB is refused with LCG_EINVAL before anything is written to
 *     d_out (lcg_expand_strings handles it);
 *   - every call on one GPU shares that GPU's scratch: calls that overlap on
 *     one device (on different streams or threads) race and must not be made.
 */
lcg_status lcg_expand_strings_noalloc(lcg_grammar_t g, uint32_t j0, uint32_t j1, uint8_t* d_out,
                                      uint64_t cap, uint64_t* d_offsets, uint64_t* total,
                                      hipStream_t stream);

/* Autotuner: times complete builds of the given strings (which it builds,
 * and frees, several times) under candidate values of the options that do not
 * change results (tail_log2, table_load_log2, combine_log2), one option at a
 * time starting from `base`, and writes the fastest setting found to *best
 * (the other fields copied from base) and its build time in milliseconds to
 * *best_ms (may be NULL).  Times are device times between HIP events on
 * `stream`.  Arguments as for lcg_build; base->mode must be
 * LCG_MODE_BATCHED. */
lcg_status lcg_tune(const uint8_t* d_text, const uint64_t* d_offsets, uint32_t k,
                    const lcg_opts* base, hipStream_t stream, lcg_opts* best, double* best_ms);

/*
 * Streaming build from a file (App. A.3's buffered BuildGram on one device):
 * the file holds one non-empty string per line ('\n'-terminated; the last
 * line may lack it).  It is read in chunks of whole lines of at most
 * chunk_bytes (4 KiB .. 64 GiB; a longer line is LCG_EINVAL) by host threads
 * into pinned buffers, uploaded on a copy stream while the previous chunk is
 * compressed, split into strings on the device and compressed into g with
 * lcg_build_into, so device memory is bounded by the chunk size and the
 * grammar, not by the file.  The strings are appended to C in file order;
 * the result equals lcg_build_into of the whole file at once.
 *   opts    as for lcg_build_into (NULL: defaults); its seed is taken from g
 *   h_info  NULL or uint64[6]: string bytes, strings, chunks, wall ns, ns the
 *           builder waited for the reader, ns in lcg_build_into
 * Errors: LCG_EINVAL (NULL arguments, unreadable file, empty line, line
 * longer than a chunk), and those of lcg_build_into.
 */
lcg_status lcg_build_file(lcg_grammar_t g, const char* path, uint64_t chunk_bytes,
                          const lcg_opts* opts, hipStream_t stream, uint64_t* h_info);
/*
 * Streaming build with a sink outside device memory (App. A.3's flush
 * cycle on one device): the file is read and split as for lcg_build_file,
 * but while it streams, the levels of `sink` (the running grammar, possibly
 * non-empty) sit in pinned host memory.  Chunks are compressed into a buffer
 * grammar on the device; once the buffer holds buffer_bytes of device memory
 * or more (0: after every chunk), and at the end, it is merged into the sink
 * (MergeGrams, one level of the sink on the device at a time, with the level
 * below it) and freed.  Device memory while streaming is thus bounded by the
 * buffer, one chunk's working memory and two of the sink's levels.  At the
 * end the sink returns to the device; the result equals lcg_build_into of
 * the whole file at once.  The buffer does not consult the sink while it
 * compresses (it may relearn rules the sink has; the merge drops them).  The
 * sink's round statistics do not cover the streamed strings.
 *   h_info  NULL or uint64[8]: as for lcg_build_file, then the number of
 *           flushes and the ns spent in them
 * Errors: those of lcg_build_file; LCG_ENOMEM also for pinned host memory.
 * A call that fails after its first flush leaves the sink refused by later
 * calls (it may hold part of the file).
 */
lcg_status lcg_build_file_sink(lcg_grammar_t sink, const char* path, uint64_t chunk_bytes,
                               uint64_t buffer_bytes, const lcg_opts* opts, hipStream_t stream,
                               uint64_t* h_info);

/*
 * Random access (the inverse path without expanding whole strings): for every
 * query q < nq, bytes [d_start[q], d_start[q] + d_len[q]) of string d_j[q]
 * are written to d_out + d_out_off[q].  Query arrays are device memory
 * (uint32 j, uint64 start, uint32 len, uint64 output offset); 1 <= len <=
 * LCG_EXTRACT_MAX.  One block per query descends from C[j] keeping only the
 * symbols whose expansion overlaps the range (at most len of them per level).
 * Synchronises the stream.  Errors: LCG_EINVAL for NULL arrays, a grammar
 * without strings, or any query out of range (its output is not written;
 * the other queries are).
 */
#define LCG_EXTRACT_MAX 2048
lcg_status lcg_extract(lcg_grammar_t g, uint32_t nq, const uint32_t* d_j, const uint64_t* d_start,
                       const uint32_t* d_len, const uint64_t* d_out_off, uint8_t* d_out,
                       hipStream_t stream);

/*
 * Longest common extension through the grammar: the lcp / lcs queries with
 * which the match-completion step sketched in App. B extends a match found
 * among right-hand sides.  For every query q (device arrays: uint32 j1, j2,
 * uint64 p1, p2; positions 0 <= p <= |T_j|):
 *   backward = 0: d_out[q] = length of the longest common prefix of
 *                 T_j1[p1..] and T_j2[p2..];
 *   backward = 1: length of the longest common suffix of T_j1[..p1) and
 *                 T_j2[..p2).
 * Two cursors (the symbol covering the position at every level) walk the
 * strings; whenever both sit at the same offset of the same symbol, the rest
 * of that symbol is skipped at once.  Synchronises the stream.  Errors:
 * LCG_EINVAL (NULL arrays, backward > 1, a grammar without strings, a query
 * out of range: its output is not written, the others are).
 */
lcg_status lcg_lce(lcg_grammar_t g, uint32_t nq, const uint32_t* d_j1, const uint64_t* d_p1,
                   const uint32_t* d_j2, const uint64_t* d_p2, uint32_t backward,
                   uint64_t* d_out, hipStream_t stream);
/*
 * App. B's lcp(X, Y) and lcs(X, Y): the longest common prefix (backward = 0)
 * or suffix (backward = 1) of exp(X) and exp(Y) for grammar symbols X and Y,
 * the quantities that complete a match found among right-hand sides.  Query
 * q names X = (d_lv1[q], d_s1[q]) and Y = (d_lv2[q], d_s2[q]) (device arrays:
 * uint8 levels, uint32 ranks); level 0 is a terminal (the byte s), level
 * i >= 1 the rank-s rule of level i.  d_out (uint64[nq]) receives the
 * lengths.  The same cursor walk as lcg_lce, started at the symbols' first or
 * last byte.  Synchronises the stream.  Errors: LCG_EINVAL (NULL arrays,
 * backward > 1, a query naming no symbol: its output is not written, the
 * others are), LCG_EOVERFLOW (64 levels or more).
 */
lcg_status lcg_symbol_lce(lcg_grammar_t g, uint32_t nq, const uint8_t* d_lv1, const uint32_t* d_s1,
                          const uint8_t* d_lv2, const uint32_t* d_s2, uint32_t backward,
                          uint64_t* d_out, hipStream_t stream);
/*
 * Maximal exact matches between strings a and b through the grammar (the
 * MEM example of App. B, on the level-`level` parses of the two strings
 * rather than on right-hand sides, so that matches come out in text
 * positions).  The parse of string j at level l is what substituting
 * right-hand sides from C[j] down to level l gives.  Every pair of equal
 * symbols, one in each parse, is an anchor (with a == b, two different
 * positions of the parse); the match it seeds is the maximal run of equal
 * bytes T_a[pa + t] == T_b[pb + t] on the anchor's diagonal that contains its
 * first byte, completed by the lcs before the anchor and the lcp from it
 * (the cursor walk of lcg_lce).  A match holding no anchor is not reported:
 * a lower level finds more of the short ones, at the cost of more anchors;
 * matches that cover a whole level-1 phrase alike in both strings are found
 * at level 1.
 * Output: the distinct matches of at least min_len bytes, sorted by start in
 * a, then start in b: d_pa[t], d_pb[t] (starts) and d_len[t] (uint64 device
 * arrays of `cap` entries; the first min(count, cap) are written).  *n_mems
 * (host) receives the count, which may exceed cap: call again with a larger
 * cap for all of them.  Synchronises the stream.  Errors: LCG_EINVAL (NULL
 * n_mems, NULL arrays with cap > 0, a string index beyond the grammar's,
 * level outside 1..min(level of C[a], level of C[b])), LCG_EOVERFLOW (a parse
 * of 2^31 symbols or more, more than 2^31 symbol pairs at this level --
 * choose a higher one --, 64 levels or more), LCG_ENOMEM.
 */
lcg_status lcg_mems(lcg_grammar_t g, uint32_t a, uint32_t b, uint32_t level, uint64_t min_len,
                    uint64_t cap, uint64_t* d_pa, uint64_t* d_pb, uint64_t* d_len,
                    uint64_t* n_mems, hipStream_t stream);
/*
 * lcg_mems for many pairs in one call: pair p is (a[p], b[p]) (host arrays
 * of npairs string indexes; a pair may repeat, and a string may appear in
 * several pairs and on both sides).  Each pair's matches are exactly what
 * lcg_mems gives for it; all of them come out sorted by (pair, start in a,
 * start in b), with d_pair[t] (uint32 device array) naming the pair.  The
 * parses of all the strings are made together and every later step runs
 * over all pairs at once, so a batch costs little more than its largest pair.
 * cap, *n_mems and the errors as for lcg_mems; also LCG_EINVAL for NULL pair
 * arrays or 2^23 pairs or more.
 */
lcg_status lcg_mems_batch(lcg_grammar_t g, uint32_t npairs, const uint32_t* a, const uint32_t* b,
                          uint32_t level, uint64_t min_len, uint64_t cap, uint32_t* d_pair,
                          uint64_t* d_pa, uint64_t* d_pb, uint64_t* d_len, uint64_t* n_mems,
                          hipStream_t stream);

/* An empty grammar with hash family `seed` (no levels, no strings). */
lcg_status lcg_new(uint64_t seed, lcg_grammar_t* out);

/* ---- inspection (host copies) ------------------------------------------- */
lcg_status lcg_info(lcg_grammar_t g, uint64_t* seed, uint32_t* n_levels, uint32_t* k);
/* u = number of rules of level (1..n_levels), rhs_len = sum of their lengths. */
lcg_status lcg_level_size(lcg_grammar_t g, uint32_t level, uint32_t* u, uint64_t* rhs_len);
/* h_rhs_off: uint64[u+1]; h_rhs: uint32[rhs_len] (bytes widened at level 1); h_fp: uint32[u]. */
lcg_status lcg_level_copy(lcg_grammar_t g, uint32_t level, uint64_t* h_rhs_off, uint32_t* h_rhs,
                          uint32_t* h_fp);
/* h_level: uint8[k] level of C[j]; h_sym: uint32[k] rank (byte value at level 0). */
lcg_status lcg_c_copy(lcg_grammar_t g, uint8_t* h_level, uint32_t* h_sym);

/* The whole grammar in host memory (the encoding of App. A.1: per level the
 * rules' right-hand sides as ranks of the level below and their
 * fingerprints F^i; C as (level, rank) pairs). */
typedef struct {
  uint32_t u;         /* rules of the level */
  uint64_t rhs_len;   /* total right-hand-side length */
  uint64_t* rhs_off;  /* u + 1 offsets into rhs */
  uint32_t* rhs;      /* rhs_len symbols: bytes at level 1 (widened), ranks above */
  uint32_t* fp;       /* u fingerprints */
} lcg_host_level;
typedef struct {
  uint64_t seed;
  uint32_t n_levels;
  uint32_t k;
  lcg_host_level* levels; /* n_levels entries, level 1 first */
  uint8_t* c_level;       /* k: level of C[j] (0 = a byte) */
  uint32_t* c_sym;        /* k: rank (the byte at level 0) */
} lcg_host_grammar;
/* Host copies of every level and of C into *out (arrays allocated by the
 * library; release them with lcg_host_free).  Synchronises the device.
 * Errors: LCG_EINVAL (NULL argument), LCG_ENOMEM (host allocation), LCG_EHIP;
 * on error *out is left empty. */
lcg_status lcg_export(lcg_grammar_t g, lcg_host_grammar* out);
/* Frees the arrays of an exported grammar and empties *h (NULL is ignored). */
void lcg_host_free(lcg_host_grammar* h);

/*
 * Per-round statistics of the builds that produced g, LCG_STATS_FIELDS
 * uint64 per round, in this order: total active length n_i, phrases d_i, new
 * rules u_i, new right-hand-side symbols Q_i, strings still active after the
 * round, dictionary probes, full right-hand-side comparisons, dictionary
 * capacity, then device nanoseconds (0 without LCG_FLAG_TIMING; with
 * LCG_FLAG_TIMING_INSERT only the insert's, in rounds with host reads) of the round's
 * kernels (sum of the following), of classify + tile scan, of emit, of
 * insert, of rank (new flags + scans), of commit, and of the segment update;
 * last, the mode of the round (0: one insert per phrase, 1: equal keys
 * combined per chunk of phrases first, chosen when the round's key sketch
 * estimates few distinct keys per phrase; 2: one insert per phrase, the round
 * queued without host reads, see lcg_opts.tail_log2).
 * Rounds of later builds (lcg_build_into, the per-string builds of the plain
 * form) are appended.
 */
#define LCG_STATS_FIELDS 16
lcg_status lcg_stats(lcg_grammar_t g, uint64_t* h_out, uint32_t cap_rounds, uint32_t* n_rounds);
/* Reset the statistics of g. */
lcg_status lcg_stats_clear(lcg_grammar_t g);

/* Upper bound of the device working memory (bytes) one lcg_build call over n
 * bytes in k strings may hold besides the grammar itself (worst case: every
 * phrase of length two).  hbm_budget is checked against it. */
uint64_t lcg_build_bytes(uint64_t n, uint32_t k);

void lcg_free(lcg_grammar_t g);

/* ---- post-processing: RL and Simp ------------------------------------------
 *
 * Run-length compression (RL) and grammar simplification (Simp), the two
 * post-processing steps of Sec. 2.2 that the paper applies to the output of
 * PBuildGram, RL first (Sec. 4).  The result is a straight-line grammar
 * (lcg_slp_t) that owns its device memory, with one id space:
 *   - ids 0..255 are the terminals (byte values);
 *   - then, for every level i = 1, 2, ... of the input grammar: first the run
 *     rules made from the runs in level i's right-hand sides, ordered by
 *     (symbol, run length), then level i's rules in rank order.  Every rule
 *     refers only to smaller ids.
 * Rule 256 + r has right-hand side rhs[off[r] .. off[r+1]) and multiplicity
 * mult[r]: exp = exp(rhs)^mult.  An ordinary rule has mult = 1; the run rule
 * X' -> (X, l) of a maximal equal-symbol run X^l (l >= 2) is rhs = [X],
 * mult = l.  C[j] is the id string j derives from.
 *   RL:   every maximal run X^l, l >= 2, in an ordinary right-hand side is
 *         replaced by the id of its run rule; each distinct (X, l) of a level
 *         gets one run rule.
 *   Simp: every ordinary rule whose id occurs exactly once over all
 *         right-hand sides and C, that occurrence being in an ordinary rule,
 *         is removed and its right-hand side spliced in place of the
 *         occurrence (recursively).  Occurrences in run rules and in C keep a
 *         rule; run rules are never removed.  Kept rules are renumbered in id
 *         order from 256.
 * Grammar size G counts |rhs| for ordinary rules and 2 for a run rule.
 */
typedef struct lcg_slp* lcg_slp_t;

enum {
  LCG_PP_RL = 1u,   /* run-length compression */
  LCG_PP_SIMP = 2u  /* simplification (after RL when both are set) */
};

/* Statistics of a post-processing call, in this order: rules g and size G of
 * the input, run rules made, g and G after RL, rules removed by Simp, g and G
 * of the result. */
#define LCG_SLP_STATS 8

/*
 * Post-process g (left unchanged) on `stream` into *out (free with
 * lcg_slp_free).  flags: LCG_PP_RL and/or LCG_PP_SIMP; 0 gives g itself in the
 * id layout above.  Synchronises the stream.  Errors: LCG_EINVAL (NULL
 * argument, unknown flag, a grammar without strings), LCG_EOVERFLOW (2^32 -
 * 256 rules or more, or more than 2^31 runs in a level), LCG_ENOMEM, LCG_EHIP.
 */
lcg_status lcg_postprocess(lcg_grammar_t g, uint32_t flags, hipStream_t stream, lcg_slp_t* out);
/* g = rules (ids 256 .. 256+g-1), rhs_len = total right-hand-side length, k = strings. */
lcg_status lcg_slp_size(lcg_slp_t p, uint32_t* g, uint64_t* rhs_len, uint32_t* k);
/* h_stats: uint64[LCG_SLP_STATS]. */
lcg_status lcg_slp_stats(lcg_slp_t p, uint64_t* h_stats);
/* Device arrays owned by p (valid until lcg_slp_free): off uint64[g+1],
 * rhs uint32[rhs_len], mult uint32[g], C uint32[k].  Any pointer may be NULL. */
lcg_status lcg_slp_device(lcg_slp_t p, const uint64_t** d_off, const uint32_t** d_rhs,
                          const uint32_t** d_mult, const uint32_t** d_c);
/* Host copies of the same arrays (caller-sized; any pointer may be NULL). */
lcg_status lcg_slp_copy(lcg_slp_t p, uint64_t* h_off, uint32_t* h_rhs, uint32_t* h_mult,
                        uint32_t* h_c);
/*
 * Decompression of the post-processed grammar: exp(C[j]) for j0 <= j < j1,
 * one after the other in d_out (device, cap bytes); d_offsets (device
 * uint64[j1-j0+1], may be NULL) receives where each string starts and the
 * total; *total the number of bytes.  With cap smaller than the total the
 * call returns LCG_EINVAL after setting *total (query with d_out = NULL,
 * cap = 0).  The rules' expansion lengths are computed on the first call and
 * kept with p.  Synchronises the stream.
 */
lcg_status lcg_slp_expand_strings(lcg_slp_t p, uint32_t j0, uint32_t j1, uint8_t* d_out,
                                  uint64_t cap, uint64_t* d_offsets, uint64_t* total,
                                  hipStream_t stream);
/*
 * Random access into the post-processed grammar, with the contract of
 * lcg_extract: query q writes bytes [start[q], start[q] + len[q]) of string
 * j[q] (1 <= len <= LCG_EXTRACT_MAX) to d_out + out_off[q].  One wave per
 * query (one block above 256 bytes) replaces, step by step from C[j], each
 * rule by its children that
 * overlap the range (whole repetitions of a run rule skipped at once, the
 * first overlapping child found by binary search over the rule's prefix sums
 * of expansion lengths).  The first call computes and keeps the expansion
 * lengths, like lcg_slp_expand_strings.  Synchronises the stream.  Errors:
 * LCG_EINVAL (NULL arrays; queries out of range: their output is not
 * written, the others are).
 */
lcg_status lcg_slp_extract(lcg_slp_t p, uint32_t nq, const uint32_t* d_j, const uint64_t* d_start,
                           const uint32_t* d_len, const uint64_t* d_out_off, uint8_t* d_out,
                           hipStream_t stream);
void lcg_slp_free(lcg_slp_t p);

/* ---- the stored file of a post-processed grammar ----------------------------
 *
 * App. A (storing the final grammar) budgets G log g bits for the
 * right-hand sides, g log G bits for the pointers to them and one entry per
 * string for C.  The file (little-endian) is:
 *   header, eight 64-bit words: the bytes "LCGSLP01", r (rules), G (cells),
 *     k (strings), runs (run rules), nb (block bounds), the widths
 *     b_sym | b_cell << 8 | b_ptr << 16, the file's size in bytes;
 *   R: the right-hand sides of rules 256, 257, ... one after the other, G
 *     cells of b_cell bits; a run rule X' -> (X, l) takes two cells, X and l;
 *   P: the first cell of every rule in R, r cells of b_ptr bits;
 *   M: one bit per rule, set for run rules;
 *   C: k cells of b_sym bits;
 *   B: the nb block bounds, 32-bit cells: ids [B[b], B[b+1]) form block b
 *     (per level of the input, its run rules, then its ordinary rules), whose
 *     rules name only ids below B[b].
 * Each section starts on a 64-bit word, padding bits are zero; cell i of a
 * section of width b holds the bits i*b .. i*b+b-1, bit t being bit t % 64 of
 * word t / 64.  b_sym = bits(255 + r) (the largest id, i.e. ceil(log2 g) for
 * g = 256 + r symbols), b_cell = max(b_sym, bits(longest run)), b_ptr =
 * bits(G - 1) (1 without rules), bits(x) = the binary digits of x, at least 1.
 */
/*
 * Write p's stored file to d_out (device, 8-byte aligned, cap bytes) on
 * `stream`; *bytes receives its size.  With cap smaller than the size the
 * call returns LCG_EINVAL after setting *bytes (query with d_out = NULL,
 * cap = 0).  Synchronises the stream.  Errors: LCG_EINVAL, LCG_ENOMEM, LCG_EHIP.
 */
lcg_status lcg_slp_encode(lcg_slp_t p, uint8_t* d_out, uint64_t cap, uint64_t* bytes,
                          hipStream_t stream);
/*
 * The grammar of the stored file d_in (device, 8-byte aligned, `bytes` long)
 * into *out (free with lcg_slp_free).  The caller keeps d_in.  Everything is
 * checked before anything is expanded; LCG_EINVAL (with lcg_last_error
 * naming the fault) unless: the header's counts, widths (b_cell that of the
 * longest run) and size agree; padding bits are zero; the bounds rise from
 * 256 to 256 + r (1 to 1024 of them); the pointers start at 0 and rise, a run
 * rule spanning two cells; every cell of a rule of block b names an id below
 * B[b]; run lengths are at least 2; C names ids below 256 + r; no rule and no
 * sum of the strings' lengths reaches 2^61 bytes.  So every accepted file is
 * the one lcg_slp_encode writes for the decoded grammar.
 * The result's statistics hold only its g and G (entries 6 and 7).
 * Synchronises the stream.  Errors: LCG_EINVAL, LCG_ENOMEM, LCG_EHIP.
 */
lcg_status lcg_slp_decode(const uint8_t* d_in, uint64_t bytes, hipStream_t stream, lcg_slp_t* out);

/* Return the library's cached free device blocks to where they came from
 * (hipFree, or the allocator that made them). */
void lcg_release_pool(void);

/*
 * Device memory from the caller's allocator, e.g. PyTorch's caching
 * allocator, so that the library and the caller share one pool.  alloc
 * returns `bytes` of device memory, 256-byte aligned, or NULL when it has
 * none; free takes back a block alloc returned.  Both may be called from any
 * library call made after this one, on the calling thread, and must not call
 * into the library.  Process-wide: every block the library allocates from
 * now on comes from *a (a is copied; NULL returns to hipMalloc).  Blocks
 * already held keep their origin and go back to it when released by
 * lcg_release_pool.  Call it while no other library call is running.
 * Errors: LCG_EINVAL (alloc or free missing); an allocation failure in a
 * later call gives LCG_ENOMEM.
 */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* block, void* ctx);
  void* ctx;
} lcg_allocator;
lcg_status lcg_set_allocator(const lcg_allocator* a);
/* Thread-local description of the last failure. */
const char* lcg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LCG_H */
