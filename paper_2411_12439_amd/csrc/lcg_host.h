// Host-side internals shared by the library's translation units: errors,
// the device block pool, device buffers, the grammar object and the guard
// that turns exceptions into lcg_status at the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/lcg.h"
#include "lcg_kernels.h"

namespace lcg {

// ------------------------------------------------------------------ errors
struct LcgError {
  lcg_status status;
  std::string msg;
};

inline thread_local std::string g_last_error;

#define HIP_CHECK(x)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess)                                                              \
      throw LcgError{LCG_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)};        \
  } while (0)

// ------------------------------------------------------------------ hash family
// Coefficients (a_i, b_i, c_i) of levels 0..63 in [1, p-1], drawn in that
// order from SplitMix64 (Steele, Lea, Flood 2014; Vigna's constants) seeded
// with the grammar seed, each output reduced mod 2^61-1, zeros redrawn.
struct HashFamily {
  static constexpr int kLevels = 64;
  LevelHash lv[kLevels];
  explicit HashFamily(uint64_t seed) {
    uint64_t state = seed;
    auto draw = [&state]() {
      for (;;) {
        state += 0x9E3779B97F4A7C15ULL;
        uint64_t z = state;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        z ^= z >> 31;
        uint64_t v = z % kP61;
        if (v) return v;
      }
    };
    for (int i = 0; i < kLevels; ++i) {
      lv[i].a = draw();
      lv[i].b = draw();
      lv[i].c = draw();
    }
  }
};

// ------------------------------------------------------------------ device pool
// Caching pool of device blocks: calls reuse blocks instead of paying for
// hipMalloc/hipFree (which synchronise the device) every round.  New blocks
// come from hipMalloc, or from the caller's allocator once lcg_set_allocator
// installed one; every block remembers where it came from and goes back
// there when the pool is trimmed.
class Pool {
 public:
  Pool() { sources_.push_back(lcg_allocator{nullptr, nullptr, nullptr}); }  // 0: hipMalloc
  void set_allocator(const lcg_allocator* a) {
    std::lock_guard<std::mutex> lk(mu_);
    if (!a) {
      current_ = 0;
      return;
    }
    sources_.push_back(*a);
    current_ = sources_.size() - 1;
  }
  void* alloc(size_t bytes) {
    size_t sz = round_size(bytes);
    size_t src = 0;
    {
      std::lock_guard<std::mutex> lk(mu_);
      auto it = free_.lower_bound(sz);
      if (it != free_.end() && it->first <= sz + sz / 2) {
        const Block b = it->second;
        free_.erase(it);
        used_[b.p] = b;
        return b.p;
      }
      src = current_;
    }
    void* p = fresh(src, sz);
    if (!p) {
      trim();
      p = fresh(src, sz);
      if (!p)
        throw LcgError{LCG_ENOMEM, "device allocation of " + std::to_string(sz) + " bytes failed"};
    }
    std::lock_guard<std::mutex> lk(mu_);
    used_[p] = Block{p, sz, src};
    return p;
  }
  size_t size_of(void* p) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = used_.find(p);
    return it == used_.end() ? 0 : it->second.size;
  }
  void release(void* p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu_);
    auto it = used_.find(p);
    if (it == used_.end()) return;
    free_.insert({it->second.size, it->second});
    used_.erase(it);
  }
  // release once work already enqueued on `s` has finished (see flush)
  void release_after(void* p, hipStream_t s) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu_);
    pending_.push_back({p, s});
  }
  // `s` has been synchronised: its pending blocks become reusable
  void flush(hipStream_t s) {
    std::vector<void*> done;
    {
      std::lock_guard<std::mutex> lk(mu_);
      for (size_t i = 0; i < pending_.size();) {
        if (pending_[i].second == s) {
          done.push_back(pending_[i].first);
          pending_[i] = pending_.back();
          pending_.pop_back();
        } else {
          ++i;
        }
      }
    }
    for (void* p : done) release(p);
  }
  // the idle blocks go back to where they came from
  void trim() {
    std::lock_guard<std::mutex> lk(mu_);
    for (auto& kv : free_) {
      const Block& b = kv.second;
      if (b.src == 0) (void)hipFree(b.p);
      else sources_[b.src].free(b.p, sources_[b.src].ctx);
    }
    free_.clear();
  }

 private:
  struct Block {
    void* p;
    size_t size;
    size_t src;  // index into sources_
  };
  void* fresh(size_t src, size_t sz) {
    void* p = nullptr;
    if (src == 0) {
      if (hipMalloc(&p, sz) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
      }
      return p;
    }
    lcg_allocator a;
    {
      std::lock_guard<std::mutex> lk(mu_);
      a = sources_[src];
    }
    p = a.alloc(sz, a.ctx);
    if (p && (reinterpret_cast<uintptr_t>(p) & 255)) {  // the kernels rely on 256-byte blocks
      a.free(p, a.ctx);
      throw LcgError{LCG_EINVAL, "the installed allocator returned a block not 256-byte aligned"};
    }
    return p;
  }
  static size_t round_size(size_t b) {
    if (b < 256) b = 256;
    if (b <= (1u << 20)) {
      size_t p = 256;
      while (p < b) p <<= 1;
      return p;
    }
    const size_t g = 2u << 20;
    return (b + g - 1) / g * g;
  }
  std::mutex mu_;
  std::vector<lcg_allocator> sources_;  // never shrinks: blocks keep their index
  size_t current_ = 0;
  std::vector<std::pair<void*, hipStream_t>> pending_;
  std::multimap<size_t, Block> free_;
  std::unordered_map<void*, Block> used_;
};

inline Pool& pool() {
  static Pool* p = new Pool();  // never destroyed: blocks may outlive static destructors
  return *p;
}

template <typename T>
struct DBuf {
  T* p = nullptr;
  size_t cap = 0;  // elements
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), cap(o.cap) { o.p = nullptr; o.cap = 0; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) { reset(); p = o.p; cap = o.cap; o.p = nullptr; o.cap = 0; }
    return *this;
  }
  ~DBuf() { reset(); }
  // release now (no work in flight may use the block)
  void reset() {
    if (p) pool().release(p);
    p = nullptr;
    cap = 0;
  }
  // release once the work already enqueued on s is done
  void reset_after(hipStream_t s) {
    if (p) pool().release_after(p, s);
    p = nullptr;
    cap = 0;
  }
  // capacity >= n, old contents discarded; the old block is released after
  // the work enqueued on s
  void need(size_t n, hipStream_t s) {
    if (n <= cap && p) return;
    reset_after(s);
    size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
    p = static_cast<T*>(pool().alloc(bytes));
    cap = pool().size_of(p) / sizeof(T);
  }
  // capacity >= n, first `used` elements kept (copied on s)
  void grow(size_t n, size_t used, hipStream_t s) {
    if (n <= cap && p) return;
    size_t want = std::max<size_t>(n, cap + cap / 2);
    T* np = static_cast<T*>(pool().alloc(std::max<size_t>(want, 1) * sizeof(T)));
    if (used) HIP_CHECK(hipMemcpyAsync(np, p, used * sizeof(T), hipMemcpyDeviceToDevice, s));
    reset_after(s);
    p = np;
    cap = pool().size_of(np) / sizeof(T);
  }
};

// ------------------------------------------------------------------ grammar
// Pinned host memory holding a level moved out of device memory.
struct HostCopy {
  void* p = nullptr;
  HostCopy() = default;
  HostCopy(const HostCopy&) = delete;
  HostCopy& operator=(const HostCopy&) = delete;
  HostCopy(HostCopy&& o) noexcept : p(o.p) { o.p = nullptr; }
  HostCopy& operator=(HostCopy&& o) noexcept {
    if (this != &o) { reset(); p = o.p; o.p = nullptr; }
    return *this;
  }
  ~HostCopy() { reset(); }
  void reset() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
  }
  void* need(size_t bytes) {
    reset();
    if (hipHostMalloc(&p, std::max<size_t>(bytes, 64), hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      throw LcgError{LCG_ENOMEM, "pinned host allocation failed"};
    }
    return p;
  }
};

struct Level {
  uint32_t u = 0;      // rules
  uint64_t q = 0;      // total rhs length
  DBuf<uint64_t> off;  // u + 1 offsets
  DBuf<uint8_t> rhs8;  // level 1: bytes
  DBuf<uint32_t> rhs32;
  DBuf<uint32_t> fp;   // F^i of each rule
  DBuf<Slot> table;    // dictionary H^i: every committed rule holds one slot
  uint64_t tcap = 0;
  // while on_host the arrays above are released and their contents sit in
  // pinned host memory (a sink grammar between flushes of a streaming build)
  bool on_host = false;
  HostCopy h_off, h_rhs, h_fp, h_table;
};

using Stat = std::array<uint64_t, LCG_STATS_FIELDS>;

// device view of one level: its rule offsets and right-hand sides (uint8 at
// level 1, uint32 above)
struct LevelPtrs {
  const uint64_t* off;
  const void* rhs;
};

}  // namespace lcg

struct lcg_grammar {
  uint64_t seed;
  lcg::HashFamily H;
  std::vector<lcg::Level> levels;  // levels[i-1] = level i
  uint32_t k = 0;
  lcg::DBuf<uint8_t> c_level;
  lcg::DBuf<uint32_t> c_sym;
  std::vector<lcg::Stat> stats;
  uint64_t version = 0;  // changes whenever the grammar does
  // expansion lengths in bytes of every rule, per level (for lcg_expand_strings)
  std::vector<lcg::DBuf<uint64_t>> explen;
  // per rule of levels >= 3: the summed right-hand-side lengths of its children
  std::vector<lcg::DBuf<uint64_t>> gc;
  lcg::DBuf<const uint64_t*> explen_ptrs;
  lcg::DBuf<lcg::LevelPtrs> level_ptrs;  // per level: offsets and right-hand sides
  uint64_t explen_version = ~0ull;
  // per rule of levels 1..ends_first.size(): the first and the last (up to)
  // 8 bytes of its expansion (for lcg_mems); valid while ends_version == version
  std::vector<lcg::DBuf<uint64_t>> ends_first, ends_last;
  uint64_t ends_version = ~0ull;
  // set when a failed call could not restore the grammar: later calls refuse it
  bool poisoned = false;
  // reserve[i]: the rules lcg_reserve made dictionary room for at level i+1
  // (a level's dictionary is never sized below it)
  std::vector<uint64_t> reserve;
  explicit lcg_grammar(uint64_t s) : seed(s), H(s) {}
};

namespace lcg {

// g, checked: not NULL and not left unusable by a failed call.
inline lcg_grammar* live(lcg_grammar* g) {
  if (!g) throw LcgError{LCG_EINVAL, "grammar is NULL"};
  if (g->poisoned)
    throw LcgError{LCG_EINVAL, "grammar is unusable: an earlier call failed and could not restore it"};
  return g;
}

// Synchronise s; blocks whose release waited for it become reusable.
inline void sync(hipStream_t s) {
  HIP_CHECK(hipStreamSynchronize(s));
  pool().flush(s);
}

template <typename T>
inline T read_dev(const T* p, hipStream_t s) {
  T v;
  HIP_CHECK(hipMemcpyAsync(&v, p, sizeof(T), hipMemcpyDeviceToHost, s));
  sync(s);
  return v;
}

// expansion lengths (and the per-level device tables) of g, computed once
// per version of the grammar
void ensure_explen(lcg_grammar* g, hipStream_t s);
// A sink grammar (App. A.3): its levels moved to pinned host memory and back,
// and the merge of a buffer grammar into it one level at a time.
void sink_to_host(lcg_grammar* g, hipStream_t s);
void sink_to_device(lcg_grammar* g, hipStream_t s);
void sink_flush(lcg_grammar* sink, const lcg_grammar* buf, hipStream_t s);
uint64_t device_bytes(const lcg_grammar* g);

template <typename F>
lcg_status guard(F&& f) {
  try {
    f();
    return LCG_OK;
  } catch (const LcgError& e) {
    g_last_error = e.msg;
    return e.status;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return LCG_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return LCG_EHIP;
  }
}

}  // namespace lcg
