// Random access into a level grammar: bytes [start, start + len) of string j
// without expanding the rest of the string (the grammar's expansion lengths
// locate every symbol, Sec. 2.2's exp(X) per rule).  One block answers one
// query: starting from C[j] it keeps, level by level, only the symbols whose
// expansion overlaps the range -- they cover disjoint pieces of at least one
// byte each, so there are never more than len of them -- and the level-1
// symbols finally write their bytes.
#include <hip/hip_runtime.h>

#include "lcg_host.h"

namespace lcg {
namespace {

constexpr int kXBlock = 256;

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

}  // namespace
}  // namespace lcg

using namespace lcg;

extern "C" {

lcg_status lcg_extract(lcg_grammar_t g, uint32_t nq, const uint32_t* d_j, const uint64_t* d_start,
                       const uint32_t* d_len, const uint64_t* d_out_off, uint8_t* d_out,
                       hipStream_t stream) {
  return guard([&] {
    if (!g) throw LcgError{LCG_EINVAL, "grammar is NULL"};
    if (!nq) return;
    if (!d_j || !d_start || !d_len || !d_out_off || !d_out)
      throw LcgError{LCG_EINVAL, "NULL query or output array"};
    if (!g->k) throw LcgError{LCG_EINVAL, "the grammar holds no string"};
    ensure_explen(g, stream);
    DBuf<unsigned int> bad;
    bad.need(1, stream);
    launch_zero(bad.p, sizeof(unsigned int), stream);
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

}  // extern "C"
