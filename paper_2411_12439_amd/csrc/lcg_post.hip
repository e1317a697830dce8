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

// ---------------------------------------------------------------- RL
// head[off[r]] = 1 for every rule r of the level
__global__ void k_pp_heads(const uint64_t* __restrict__ off, uint32_t u, uint8_t* __restrict__ head) {
  PP_LOOP(r, u) head[off[r]] = 1;
}

// a run starts at a rule's first position and wherever the symbol changes
template <typename Sym>
__global__ void k_pp_runflag(const Sym* __restrict__ rhs, uint64_t q, const uint8_t* __restrict__ head,
                             uint64_t* __restrict__ flag) {
  PP_LOOP(x, q) flag[x] = (x == 0 || head[x] || rhs[x] != rhs[x - 1]) ? 1 : 0;
}

// start[j] = position of run j; start[m] = q
__global__ void k_pp_runlist(const uint64_t* __restrict__ flag, const uint64_t* __restrict__ ns,
                             uint64_t q, uint64_t* __restrict__ start) {
  PP_LOOP(x, q) {
    if (flag[x]) start[ns[x]] = x;
    if (x == 0) start[ns[q]] = q;
  }
}

__global__ void k_pp_longflag(const uint64_t* __restrict__ start, uint64_t m,
                              uint64_t* __restrict__ lflag) {
  PP_LOOP(j, m) lflag[j] = (start[j + 1] - start[j] >= 2) ? 1 : 0;
}

// key of a run of length >= 2: symbol << 32 | length
template <typename Sym>
__global__ void k_pp_longkeys(const Sym* __restrict__ rhs, const uint64_t* __restrict__ start,
                              const uint64_t* __restrict__ lflag, const uint64_t* __restrict__ lpos,
                              uint64_t m, uint64_t* __restrict__ keys) {
  PP_LOOP(j, m) {
    if (!lflag[j]) continue;
    const uint64_t x = start[j];
    keys[lpos[j]] = ((uint64_t)(uint32_t)rhs[x] << 32) | (start[j + 1] - x);
  }
}

__global__ void k_pp_uniqflag(const uint64_t* __restrict__ sorted, uint64_t c,
                              uint64_t* __restrict__ uflag) {
  PP_LOOP(j, c) uflag[j] = (j == 0 || sorted[j] != sorted[j - 1]) ? 1 : 0;
}

__global__ void k_pp_uniqlist(const uint64_t* __restrict__ sorted, const uint64_t* __restrict__ uflag,
                              const uint64_t* __restrict__ upos, uint64_t c,
                              uint64_t* __restrict__ uniq) {
  PP_LOOP(j, c) if (uflag[j]) uniq[upos[j]] = sorted[j];
}

// the level's right-hand sides after RL: one symbol per run
template <typename Sym>
__global__ void k_pp_rl_rhs(const Sym* __restrict__ rhs, const uint64_t* __restrict__ start, uint64_t m,
                            const uint64_t* __restrict__ uniq, uint64_t v, uint32_t symbase,
                            uint32_t rlbase, uint32_t* __restrict__ out) {
  PP_LOOP(j, m) {
    const uint64_t x = start[j];
    const uint64_t l = start[j + 1] - x;
    const uint32_t s = (uint32_t)rhs[x];
    if (l < 2) {
      out[j] = symbase + s;
      continue;
    }
    const uint64_t key = ((uint64_t)s << 32) | l;
    uint64_t lo = 0, hi = v;  // first uniq[] >= key (present by construction)
    while (lo < hi) {
      const uint64_t mid = (lo + hi) >> 1;
      if (uniq[mid] < key) lo = mid + 1; else hi = mid;
    }
    out[j] = rlbase + (uint32_t)lo;
  }
}

// run rules of the level: rhs = [symbol], mult = length
__global__ void k_pp_rl_rules(const uint64_t* __restrict__ uniq, uint64_t v, uint32_t symbase,
                              uint64_t pos0, uint32_t rule0, uint32_t* __restrict__ rhs1,
                              uint64_t* __restrict__ off1, uint32_t* __restrict__ mult1) {
  PP_LOOP(j, v) {
    const uint64_t key = uniq[j];
    rhs1[pos0 + j] = symbase + (uint32_t)(key >> 32);
    off1[rule0 + j] = pos0 + j;
    mult1[rule0 + j] = (uint32_t)key;
  }
}

// offsets of the level's ordinary rules (ns: run index of each position, or
// NULL when runs are kept as they are)
__global__ void k_pp_ord_off(const uint64_t* __restrict__ off, const uint64_t* __restrict__ ns,
                             uint32_t u, uint64_t pos0, uint32_t rule0, uint64_t* __restrict__ off1,
                             uint32_t* __restrict__ mult1) {
  PP_LOOP(r, u) {
    const uint64_t x = off[r];
    off1[rule0 + r] = pos0 + (ns ? ns[x] : x);
    mult1[rule0 + r] = 1;
  }
}

template <typename Sym>
__global__ void k_pp_copy_rhs(const Sym* __restrict__ rhs, uint64_t q, uint32_t symbase,
                              uint32_t* __restrict__ out) {
  PP_LOOP(x, q) out[x] = symbase + (uint32_t)rhs[x];
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
__device__ __forceinline__ bool pp_removed(const uint32_t* mult1, const uint32_t* occ, uint32_t z) {
  return mult1[z] == 1 && occ[z] == 1;
}

// Occurrences: +1 in an ordinary rule, +2 in a run rule (which pins the
// symbol).  The first ordinary occurrence records its rule and position; it
// is the only one when the count ends at 1.
__global__ void k_pp_occ(const uint64_t* __restrict__ off1, const uint32_t* __restrict__ rhs1,
                         const uint32_t* __restrict__ mult1, uint32_t g1, uint32_t* occ,
                         uint32_t* __restrict__ par, uint64_t* __restrict__ at) {
  PP_LOOP(r, g1) {
    const bool run = mult1[r] >= 2;
    const uint64_t b = off1[r + 1];
    for (uint64_t t = off1[r]; t < b; ++t) {
      const uint32_t y = rhs1[t];
      if (y < 256) continue;
      const uint32_t z = y - 256;
      if (run) {
        atomicAdd(&occ[z], 2u);
        continue;
      }
      if (__hip_atomic_load(&occ[z], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= 2) continue;
      if (atomicAdd(&occ[z], 1u) == 0) {
        par[z] = (uint32_t)r;
        at[z] = t;
      }
    }
  }
}

__global__ void k_pp_occ_c(const uint32_t* __restrict__ c1, uint32_t k, uint32_t* occ) {
  PP_LOOP(j, k) if (c1[j] >= 256) atomicAdd(&occ[c1[j] - 256], 2u);
}

// flattened length of the ordinary rules [r0, r1) (lower levels done)
__global__ void k_pp_flat(const uint64_t* __restrict__ off1, const uint32_t* __restrict__ rhs1,
                          const uint32_t* __restrict__ mult1, const uint32_t* __restrict__ occ,
                          uint32_t r0, uint32_t r1, uint64_t* W) {
  PP_LOOP(i, r1 - r0) {
    const uint32_t r = r0 + (uint32_t)i;
    uint64_t w = 0;
    const uint64_t b = off1[r + 1];
    for (uint64_t t = off1[r]; t < b; ++t) {
      const uint32_t y = rhs1[t];
      w += (y >= 256 && pp_removed(mult1, occ, y - 256)) ? W[y - 256] : 1;
    }
    W[r] = w;
  }
}

// kept flag and output length of every rule
__global__ void k_pp_keep(const uint32_t* __restrict__ mult1, const uint32_t* __restrict__ occ,
                          const uint64_t* __restrict__ W, uint32_t g1, uint64_t* __restrict__ kf,
                          uint64_t* __restrict__ len) {
  PP_LOOP(r, g1) {
    const bool run = mult1[r] >= 2;
    const bool keep = !pp_removed(mult1, occ, (uint32_t)r);
    kf[r] = keep ? 1 : 0;
    len[r] = keep ? (run ? 1 : W[r]) : 0;
  }
}

// weight of every position: 1 for a kept symbol, the flattened length of a removed one
__global__ void k_pp_weights(const uint32_t* __restrict__ rhs1, uint64_t q1,
                             const uint32_t* __restrict__ mult1, const uint32_t* __restrict__ occ,
                             const uint64_t* __restrict__ W, uint64_t* __restrict__ wg) {
  PP_LOOP(t, q1) {
    const uint32_t y = rhs1[t];
    wg[t] = (y >= 256 && pp_removed(mult1, occ, y - 256)) ? W[y - 256] : 1;
  }
}

// where the removed rules of [r0, r1) land in the output (upper levels done)
__global__ void k_pp_base(const uint64_t* __restrict__ off1, const uint32_t* __restrict__ mult1,
                          const uint32_t* __restrict__ occ, const uint32_t* __restrict__ par,
                          const uint64_t* __restrict__ at, const uint64_t* __restrict__ sw,
                          const uint64_t* __restrict__ so, uint32_t r0, uint32_t r1, uint64_t* base) {
  PP_LOOP(i, r1 - r0) {
    const uint32_t r = r0 + (uint32_t)i;
    if (!pp_removed(mult1, occ, r)) continue;
    const uint32_t p = par[r];
    const uint64_t dp = pp_removed(mult1, occ, p) ? base[p] : so[p];
    base[r] = dp + sw[at[r]] - sw[off1[p]];
  }
}

// every kept symbol of every rule at its output position; kept rules' offsets
// and multiplicities
__global__ void k_pp_write(const uint64_t* __restrict__ off1, const uint32_t* __restrict__ rhs1,
                           const uint32_t* __restrict__ mult1, const uint32_t* __restrict__ occ,
                           const uint64_t* __restrict__ nidx, const uint64_t* __restrict__ so,
                           const uint64_t* __restrict__ base, const uint64_t* __restrict__ sw,
                           uint32_t g1, uint32_t* __restrict__ rhs2, uint64_t* __restrict__ off2,
                           uint32_t* __restrict__ mult2) {
  PP_LOOP(r, g1) {
    const bool keep = !pp_removed(mult1, occ, (uint32_t)r);
    const uint64_t dest = keep ? so[r] : base[r];
    const uint64_t a = off1[r], b = off1[r + 1];
    const uint64_t s0 = sw[a];
    for (uint64_t t = a; t < b; ++t) {
      const uint32_t y = rhs1[t];
      if (y < 256) {
        rhs2[dest + sw[t] - s0] = y;
      } else if (!pp_removed(mult1, occ, y - 256)) {
        rhs2[dest + sw[t] - s0] = 256 + (uint32_t)nidx[y - 256];
      }
    }
    if (keep) {
      off2[nidx[r]] = so[r];
      mult2[nidx[r]] = mult1[r];
    }
    if (r == 0) off2[nidx[g1]] = so[g1];
  }
}

__global__ void k_pp_c_out(const uint32_t* __restrict__ c1, uint32_t k,
                           const uint64_t* __restrict__ nidx, uint32_t* __restrict__ c2) {
  PP_LOOP(j, k) c2[j] = c1[j] < 256 ? c1[j] : 256 + (uint32_t)nidx[c1[j] - 256];
}

// ---------------------------------------------------------------- host
struct Scan {
  DBuf<uint64_t> tmp;
  // out[0..n] = exclusive prefix sums of in[0..n); returns the total
  uint64_t run(const uint64_t* in, uint64_t* out, uint64_t n, hipStream_t s, bool read = true) {
    if (n == 0) {
      k_pp_set<<<1, 1, 0, s>>>(out, 0);
      PP_CHECK("pp_set");
      return 0;
    }
    tmp.need(scan_tmp_words(n), s);
    scan_exclusive(in, out, n, tmp.p, s);
    return read ? read_dev(out + n, s) : 0;
  }
};

void zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes) launch_zero(p, (bytes + 3) & ~size_t(3), s);
}

}  // namespace

// RL of one level into the global arrays.  Returns (runs m, run rules v).
template <typename Sym>
static std::pair<uint64_t, uint64_t> rl_level(const Level& L, const Sym* rhs, uint32_t symbase,
                                              uint64_t pos0, uint32_t rlbase0, Scan& sc,
                                              DBuf<uint32_t>& rhs1, DBuf<uint64_t>& off1,
                                              DBuf<uint32_t>& mult1, hipStream_t s) {
  const uint64_t q = L.q;
  const uint32_t u = L.u;
  DBuf<uint8_t> head;
  DBuf<uint64_t> flag, ns, start;
  head.need((q + 3) & ~uint64_t(3), s);
  zero(head.p, q, s);
  k_pp_heads<<<pgrid(u), kPB, 0, s>>>(L.off.p, u, head.p);
  PP_CHECK("pp_heads");
  flag.need(q, s);
  ns.need(q + 1, s);
  k_pp_runflag<Sym><<<pgrid(q), kPB, 0, s>>>(rhs, q, head.p, flag.p);
  PP_CHECK("pp_runflag");
  const uint64_t m = sc.run(flag.p, ns.p, q, s);
  start.need(m + 1, s);
  k_pp_runlist<<<pgrid(q), kPB, 0, s>>>(flag.p, ns.p, q, start.p);
  PP_CHECK("pp_runlist");
  // the distinct runs of length >= 2, sorted
  DBuf<uint64_t> lflag, lpos;
  lflag.need(m, s);
  lpos.need(m + 1, s);
  k_pp_longflag<<<pgrid(m), kPB, 0, s>>>(start.p, m, lflag.p);
  PP_CHECK("pp_longflag");
  const uint64_t c = sc.run(lflag.p, lpos.p, m, s);
  uint64_t v = 0;
  DBuf<uint64_t> uniq;
  if (c > 0x7fffffffull) throw LcgError{LCG_EOVERFLOW, "more than 2^31 runs in one level"};
  if (c) {
    DBuf<uint64_t> keys, sorted, uflag, upos;
    keys.need(c, s);
    sorted.need(c, s);
    k_pp_longkeys<Sym><<<pgrid(m), kPB, 0, s>>>(rhs, start.p, lflag.p, lpos.p, m, keys.p);
    PP_CHECK("pp_longkeys");
    size_t tbytes = 0;
    HIP_CHECK(hipcub::DeviceRadixSort::SortKeys(nullptr, tbytes, keys.p, sorted.p, (int)c, 0, 64, s));
    DBuf<uint8_t> tmp;
    tmp.need(std::max<size_t>(tbytes, 4), s);
    HIP_CHECK(hipcub::DeviceRadixSort::SortKeys(tmp.p, tbytes, keys.p, sorted.p, (int)c, 0, 64, s));
    uflag.need(c, s);
    upos.need(c + 1, s);
    k_pp_uniqflag<<<pgrid(c), kPB, 0, s>>>(sorted.p, c, uflag.p);
    PP_CHECK("pp_uniqflag");
    v = sc.run(uflag.p, upos.p, c, s);
    uniq.need(v, s);
    k_pp_uniqlist<<<pgrid(c), kPB, 0, s>>>(sorted.p, uflag.p, upos.p, c, uniq.p);
    PP_CHECK("pp_uniqlist");
    k_pp_rl_rules<<<pgrid(v), kPB, 0, s>>>(uniq.p, v, symbase, pos0, rlbase0 - 256, rhs1.p, off1.p,
                                           mult1.p);
    PP_CHECK("pp_rl_rules");
    keys.reset_after(s);
    sorted.reset_after(s);
    uflag.reset_after(s);
    upos.reset_after(s);
    tmp.reset_after(s);
  }
  const uint32_t obase = rlbase0 + (uint32_t)v;
  k_pp_rl_rhs<Sym><<<pgrid(m), kPB, 0, s>>>(rhs, start.p, m, uniq.p, v, symbase, rlbase0,
                                            rhs1.p + pos0 + v);
  PP_CHECK("pp_rl_rhs");
  k_pp_ord_off<<<pgrid(u), kPB, 0, s>>>(L.off.p, ns.p, u, pos0 + v, obase - 256, off1.p, mult1.p);
  PP_CHECK("pp_ord_off");
  head.reset_after(s);
  flag.reset_after(s);
  ns.reset_after(s);
  start.reset_after(s);
  lflag.reset_after(s);
  lpos.reset_after(s);
  uniq.reset_after(s);
  return {m, v};
}

static lcg_slp* postprocess_core(lcg_grammar* g, uint32_t flags, hipStream_t s) {
  const bool rl = flags & LCG_PP_RL;
  const bool simp = flags & LCG_PP_SIMP;
  const size_t h = g->levels.size();
  uint64_t g0 = 0, q0 = 0;
  for (const Level& L : g->levels) {
    g0 += L.u;
    q0 += L.q;
  }
  // capacities: RL never adds positions (m + v <= q per level) and adds at
  // most q/2 run rules per level
  const uint64_t gcap = g0 + (rl ? q0 / 2 : 0);
  if (256 + gcap >= (1ull << 32)) throw LcgError{LCG_EOVERFLOW, "more than 2^32 - 256 rules"};
  DBuf<uint32_t> rhs1, mult1, c1;
  DBuf<uint64_t> off1;
  rhs1.need(std::max<uint64_t>(q0, 1), s);
  off1.need(gcap + 1, s);
  mult1.need(std::max<uint64_t>(gcap, 1), s);
  Scan sc;
  std::vector<uint32_t> obase(h + 1, 0);
  uint64_t pos = 0;
  uint32_t next = 256;
  uint64_t runs = 0;
  for (size_t i = 1; i <= h; ++i) {
    const Level& L = g->levels[i - 1];
    const uint32_t symbase = i == 1 ? 0 : obase[i - 1];
    if (L.u == 0) {
      obase[i] = next;
      continue;
    }
    uint64_t m = L.q, v = 0;
    if (rl) {
      auto mv = i == 1 ? rl_level<uint8_t>(L, L.rhs8.p, symbase, pos, next, sc, rhs1, off1, mult1, s)
                       : rl_level<uint32_t>(L, L.rhs32.p, symbase, pos, next, sc, rhs1, off1, mult1, s);
      m = mv.first;
      v = mv.second;
    } else {
      if (i == 1)
        k_pp_copy_rhs<uint8_t><<<pgrid(L.q), kPB, 0, s>>>(L.rhs8.p, L.q, symbase, rhs1.p + pos);
      else
        k_pp_copy_rhs<uint32_t><<<pgrid(L.q), kPB, 0, s>>>(L.rhs32.p, L.q, symbase, rhs1.p + pos);
      PP_CHECK("pp_copy_rhs");
      k_pp_ord_off<<<pgrid(L.u), kPB, 0, s>>>(L.off.p, nullptr, L.u, pos, next - 256, off1.p,
                                               mult1.p);
      PP_CHECK("pp_ord_off");
    }
    obase[i] = next + (uint32_t)v;
    next = obase[i] + L.u;
    pos += m + v;
    runs += v;
  }
  const uint32_t g1 = next - 256;
  const uint64_t q1 = pos;
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
  if (!simp) {
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
  DBuf<uint32_t> occ, par;
  DBuf<uint64_t> at, W, kf, nidx, len, so, wg, sw, base;
  occ.need(std::max<uint32_t>(g1, 1), s);
  zero(occ.p, (size_t)g1 * 4, s);
  par.need(std::max<uint32_t>(g1, 1), s);
  at.need(std::max<uint32_t>(g1, 1), s);
  k_pp_occ<<<pgrid(g1), kPB, 0, s>>>(off1.p, rhs1.p, mult1.p, g1, occ.p, par.p, at.p);
  PP_CHECK("pp_occ");
  k_pp_occ_c<<<pgrid(g->k), kPB, 0, s>>>(c1.p, g->k, occ.p);
  PP_CHECK("pp_occ_c");
  W.need(std::max<uint32_t>(g1, 1), s);
  for (size_t i = 1; i <= h; ++i) {
    const uint32_t u = g->levels[i - 1].u;
    if (!u) continue;
    k_pp_flat<<<pgrid(u), kPB, 0, s>>>(off1.p, rhs1.p, mult1.p, occ.p, obase[i] - 256,
                                        obase[i] - 256 + u, W.p);
    PP_CHECK("pp_flat");
  }
  kf.need(std::max<uint32_t>(g1, 1), s);
  len.need(std::max<uint32_t>(g1, 1), s);
  nidx.need(g1 + 1, s);
  so.need(g1 + 1, s);
  k_pp_keep<<<pgrid(g1), kPB, 0, s>>>(mult1.p, occ.p, W.p, g1, kf.p, len.p);
  PP_CHECK("pp_keep");
  const uint32_t g2 = (uint32_t)sc.run(kf.p, nidx.p, g1, s);
  const uint64_t q2 = sc.run(len.p, so.p, g1, s);
  wg.need(std::max<uint64_t>(q1, 1), s);
  sw.need(q1 + 1, s);
  k_pp_weights<<<pgrid(q1), kPB, 0, s>>>(rhs1.p, q1, mult1.p, occ.p, W.p, wg.p);
  PP_CHECK("pp_weights");
  sc.run(wg.p, sw.p, q1, s, false);
  base.need(std::max<uint32_t>(g1, 1), s);
  for (size_t i = h; i >= 1; --i) {
    const uint32_t u = g->levels[i - 1].u;
    if (!u) continue;
    k_pp_base<<<pgrid(u), kPB, 0, s>>>(off1.p, mult1.p, occ.p, par.p, at.p, sw.p, so.p,
                                        obase[i] - 256, obase[i] - 256 + u, base.p);
    PP_CHECK("pp_base");
  }
  out->g = g2;
  out->q = q2;
  out->off.need(g2 + 1, s);
  out->rhs.need(std::max<uint64_t>(q2, 1), s);
  out->mult.need(std::max<uint32_t>(g2, 1), s);
  out->c.need(std::max<uint32_t>(g->k, 1), s);
  k_pp_write<<<pgrid(g1), kPB, 0, s>>>(off1.p, rhs1.p, mult1.p, occ.p, nidx.p, so.p, base.p, sw.p,
                                        g1, out->rhs.p, out->off.p, out->mult.p);
  PP_CHECK("pp_write");
  if (g1 == 0) k_pp_set<<<1, 1, 0, s>>>(out->off.p, 0);
  k_pp_c_out<<<pgrid(g->k), kPB, 0, s>>>(c1.p, g->k, nidx.p, out->c.p);
  PP_CHECK("pp_c_out");
  st[5] = g1 - g2;
  st[6] = g2;
  st[7] = q2 + runs;
  sync(s);
  return out.release();
}

}  // namespace lcg

using namespace lcg;

extern "C" {

lcg_status lcg_postprocess(lcg_grammar_t g, uint32_t flags, hipStream_t stream, lcg_slp_t* out) {
  return guard([&] {
    if (!g || !out) throw LcgError{LCG_EINVAL, "grammar or out is NULL"};
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

void lcg_slp_free(lcg_slp_t p) { delete p; }

}  // extern "C"
