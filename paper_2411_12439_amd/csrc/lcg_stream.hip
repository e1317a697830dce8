// Streaming builds from a file: a collection of any size (one string per
// line) is compressed chunk by chunk into a running grammar, the way App. A.3
// feeds buffers to BuildGram with the growing grammar as dictionary.  Device
// memory holds two raw chunks, one split chunk and the grammar; nothing is
// proportional to the file.
//
// Pipeline: reader threads fill pinned host buffers with whole lines (parallel
// pread, cut after the chunk's last newline); the main thread uploads chunk
// i+1 on a copy stream while chunk i is split into strings on the device
// (newlines removed, offsets from a scan of per-tile newline counts) and
// compressed with lcg_build_into.
#include <hip/hip_runtime.h>

#include <fcntl.h>
#include <sys/stat.h>
#include <unistd.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>

#include "lcg_host.h"

namespace lcg {
namespace {

constexpr int kSBlock = 256;
constexpr int kSItems = 16;
constexpr uint64_t kSTile = kSBlock * kSItems;  // bytes per tile

// newlines per tile
__global__ __launch_bounds__(kSBlock) void k_nl_count(const uint8_t* __restrict__ raw, uint64_t n,
                                                      uint64_t* __restrict__ cnt) {
  __shared__ uint32_t s_w[kSBlock / 64];
  const uint64_t base = blockIdx.x * kSTile + (uint64_t)threadIdx.x * kSItems;
  uint32_t c = 0;
  for (int i = 0; i < kSItems; ++i) c += (base + i < n && raw[base + i] == '\n') ? 1 : 0;
  uint32_t tot;
  block_excl_scan<uint32_t, kSBlock>(c, s_w, &tot);
  if (threadIdx.x == 0) cnt[blockIdx.x] = tot;
}

// text without newlines; off[l + 1] = end of line l (lbase: lines before the tile)
__global__ __launch_bounds__(kSBlock) void k_nl_split(const uint8_t* __restrict__ raw, uint64_t n,
                                                      const uint64_t* __restrict__ lbase,
                                                      uint8_t* __restrict__ text,
                                                      uint64_t* __restrict__ off) {
  __shared__ uint32_t s_w[kSBlock / 64];
  const uint64_t base = blockIdx.x * kSTile + (uint64_t)threadIdx.x * kSItems;
  uint8_t b[kSItems];
  uint32_t c = 0;
  for (int i = 0; i < kSItems; ++i) {
    b[i] = base + i < n ? raw[base + i] : 0;
    c += (base + i < n && b[i] == '\n') ? 1 : 0;
  }
  uint32_t tot;
  uint64_t l = lbase[blockIdx.x] + block_excl_scan<uint32_t, kSBlock>(c, s_w, &tot);  // newlines before base
  for (int i = 0; i < kSItems; ++i) {
    const uint64_t x = base + i;
    if (x >= n) break;
    if (b[i] == '\n') {
      off[l + 1] = x - l;
      ++l;
    } else {
      text[x - l] = b[i];
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) off[0] = 0;
}

__global__ void k_set_u64(uint64_t* p, uint64_t v) { *p = v; }

// ---------------------------------------------------------------- host side
struct HostChunk {
  uint8_t* raw = nullptr;  // pinned
  uint64_t n = 0;          // bytes, whole lines (the last one may lack its newline at EOF)
  bool eof = false;
};

class Reader {
 public:
  Reader(const char* path, uint64_t cap, int nthreads) : cap_(cap), nthreads_(nthreads) {
    fd_ = ::open(path, O_RDONLY);
    if (fd_ < 0) throw LcgError{LCG_EINVAL, std::string("cannot open ") + path};
    struct stat st;
    if (fstat(fd_, &st) != 0) throw LcgError{LCG_EINVAL, std::string("cannot stat ") + path};
    size_ = (uint64_t)st.st_size;
  }
  ~Reader() {
    if (fd_ >= 0) ::close(fd_);
  }
  uint64_t size() const { return size_; }
  // the next chunk of whole lines into c.raw (capacity cap_)
  void fill(HostChunk& c) {
    const uint64_t want = std::min<uint64_t>(cap_, size_ - pos_);
    read_range(c.raw, pos_, want);
    uint64_t n = want;
    const bool eof = pos_ + want == size_;
    if (!eof) {
      const void* nl = memrchr(c.raw, '\n', want);
      if (!nl) throw LcgError{LCG_EINVAL, "a line is longer than the chunk size"};
      n = (uint64_t)((const uint8_t*)nl - c.raw) + 1;
    }
    pos_ += n;
    c.n = n;
    c.eof = pos_ == size_;
  }

 private:
  void read_range(uint8_t* dst, uint64_t at, uint64_t len) {
    const uint64_t per = (len + nthreads_ - 1) / nthreads_;
    std::vector<std::thread> th;
    std::vector<int> bad(nthreads_, 0);
    for (int t = 0; t < nthreads_; ++t) {
      const uint64_t a = std::min(len, t * per), b = std::min(len, a + per);
      if (a >= b) break;
      th.emplace_back([=, &bad] {
        uint64_t done = a;
        while (done < b) {
          const ssize_t r = ::pread(fd_, dst + done, b - done, (off_t)(at + done));
          if (r <= 0) {
            bad[t] = 1;
            return;
          }
          done += (uint64_t)r;
        }
      });
    }
    for (auto& x : th) x.join();
    for (int v : bad)
      if (v) throw LcgError{LCG_EINVAL, "read error"};
  }
  int fd_ = -1;
  uint64_t size_ = 0, pos_ = 0, cap_;
  int nthreads_;
};

// Chunks handed from the reader thread to the builder, and back.
class Pipe {
 public:
  void put_full(HostChunk* c) {
    std::lock_guard<std::mutex> lk(mu_);
    full_.push_back(c);
    cv_.notify_all();
  }
  void put_free(HostChunk* c) {
    std::lock_guard<std::mutex> lk(mu_);
    free_.push_back(c);
    cv_.notify_all();
  }
  HostChunk* get_full() {
    std::unique_lock<std::mutex> lk(mu_);
    cv_.wait(lk, [&] { return !full_.empty() || failed_; });
    if (failed_ && full_.empty()) return nullptr;
    HostChunk* c = full_.front();
    full_.pop_front();
    return c;
  }
  HostChunk* get_free() {
    std::unique_lock<std::mutex> lk(mu_);
    cv_.wait(lk, [&] { return !free_.empty() || stop_; });
    if (stop_) return nullptr;
    HostChunk* c = free_.front();
    free_.pop_front();
    return c;
  }
  void fail(const LcgError& e) {
    std::lock_guard<std::mutex> lk(mu_);
    failed_ = true;
    err_ = e;
    cv_.notify_all();
  }
  void stop() {
    std::lock_guard<std::mutex> lk(mu_);
    stop_ = true;
    cv_.notify_all();
  }
  bool failed(LcgError* e) {
    std::lock_guard<std::mutex> lk(mu_);
    if (failed_ && e) *e = err_;
    return failed_;
  }

 private:
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<HostChunk*> full_, free_;
  bool failed_ = false, stop_ = false;
  LcgError err_{LCG_OK, ""};
};

struct Pinned {
  void* p = nullptr;
  explicit Pinned(size_t bytes) {
    if (hipHostMalloc(&p, std::max<size_t>(bytes, 64), hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      throw LcgError{LCG_ENOMEM, "pinned host allocation failed"};
    }
  }
  ~Pinned() {
    if (p) (void)hipHostFree(p);
  }
};

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace
}  // namespace lcg

using namespace lcg;

namespace {

// The streaming build.  With sink, g is the sink of App. A.3: its levels stay
// in pinned host memory while the chunks are compressed into a buffer
// grammar on the device, which is merged into the sink (one level of the sink
// on the device at a time) whenever the buffer holds buffer_bytes of device
// memory or more, and at the end; then the sink returns to the device.
void build_file(lcg_grammar* g, const char* path, uint64_t chunk_bytes, const lcg_opts* opts,
                hipStream_t stream, uint64_t* h_info, bool sink, uint64_t buffer_bytes) {
  {
    if (!path) throw LcgError{LCG_EINVAL, "path is NULL"};
    if (chunk_bytes < 4096 || chunk_bytes > (1ull << 36))
      throw LcgError{LCG_EINVAL, "chunk_bytes must be in 4 KiB .. 64 GiB"};
    lcg_opts o;
    if (opts) o = *opts; else lcg_opts_init(&o);
    o.seed = g->seed;
    const double t0 = now_s();
    Reader rd(path, chunk_bytes, 8);
    constexpr int kHost = 3;
    std::vector<std::unique_ptr<Pinned>> mem;
    HostChunk hc[kHost];
    Pipe pipe;
    for (int i = 0; i < kHost; ++i) {
      mem.emplace_back(new Pinned(chunk_bytes));
      hc[i].raw = static_cast<uint8_t*>(mem.back()->p);
      pipe.put_free(&hc[i]);
    }
    std::thread reader([&] {
      try {
        for (;;) {
          HostChunk* c = pipe.get_free();
          if (!c) return;
          rd.fill(*c);
          pipe.put_full(c);
          if (c->eof) return;
        }
      } catch (const LcgError& e) {
        pipe.fail(e);
      }
    });
    hipStream_t copy_s = nullptr;
    hipEvent_t copied[2] = {nullptr, nullptr};
    uint64_t strings = 0, bytes = 0, chunks = 0, flushes = 0;
    double wait_s = 0, build_s = 0, flush_s = 0;
    lcg_grammar_t buf = nullptr;  // the buffer grammar (sink mode)
    bool touched = false;         // a flush has started: the sink holds part of the stream
    auto new_buffer = [&] {
      const lcg_status st = lcg_new(g->seed, &buf);
      if (st != LCG_OK) throw LcgError{st, std::string("buffer grammar: ") + lcg_last_error()};
    };
    auto flush = [&] {
      const double tf = now_s();
      touched = true;
      sink_flush(g, buf, stream);
      lcg_free(buf);
      buf = nullptr;
      ++flushes;
      flush_s += now_s() - tf;
    };
    auto finish = [&] {
      pipe.stop();
      reader.join();
      if (buf) lcg_free(buf);
      buf = nullptr;
      for (auto& e : copied)
        if (e) (void)hipEventDestroy(e);
      if (copy_s) (void)hipStreamDestroy(copy_s);
    };
    try {
      if (sink) sink_to_host(g, stream);
      HIP_CHECK(hipStreamCreateWithFlags(&copy_s, hipStreamNonBlocking));
      for (auto& e : copied) HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      DBuf<uint8_t> raw[2], text;
      DBuf<uint64_t> off, tcnt, tbase, stmp;
      auto upload = [&](HostChunk* c, int slot) {
        raw[slot].need(std::max<uint64_t>(c->n, 1), copy_s);
        if (c->n)
          HIP_CHECK(hipMemcpyAsync(raw[slot].p, c->raw, c->n, hipMemcpyHostToDevice, copy_s));
        HIP_CHECK(hipEventRecord(copied[slot], copy_s));
      };
      double tw = now_s();
      HostChunk* cur = pipe.get_full();
      wait_s += now_s() - tw;
      if (!cur) {
        LcgError e{LCG_EINVAL, ""};
        pipe.failed(&e);
        throw e;
      }
      upload(cur, 0);
      int slot = 0;
      while (cur) {
        HostChunk* next = nullptr;
        if (!cur->eof) {
          tw = now_s();
          next = pipe.get_full();
          wait_s += now_s() - tw;
          if (!next) {
            LcgError e{LCG_EINVAL, ""};
            pipe.failed(&e);
            throw e;
          }
          upload(next, slot ^ 1);
        }
        // split chunk `cur` into strings on the device and compress it
        HIP_CHECK(hipStreamWaitEvent(stream, copied[slot], 0));
        const uint64_t n = cur->n;
        if (n) {
          const uint64_t tiles = (n + kSTile - 1) / kSTile;
          tcnt.need(tiles, stream);
          tbase.need(tiles + 1, stream);
          k_nl_count<<<(unsigned)tiles, kSBlock, 0, stream>>>(raw[slot].p, n, tcnt.p);
          HIP_CHECK(hipGetLastError());
          stmp.need(std::max<size_t>(scan_tmp_words(tiles), 1), stream);
          scan_exclusive(tcnt.p, tbase.p, tiles, stmp.p, stream);
          const uint64_t nl = read_dev(tbase.p + tiles, stream);
          const bool tail = cur->raw[n - 1] != '\n';  // the file's last line, unterminated
          const uint64_t k = nl + (tail ? 1 : 0);
          if (k > 0xffffffffull) throw LcgError{LCG_EOVERFLOW, "more than 2^32 lines in a chunk"};
          text.need(std::max<uint64_t>(n - nl, 1), stream);
          off.need(k + 1, stream);
          k_nl_split<<<(unsigned)tiles, kSBlock, 0, stream>>>(raw[slot].p, n, tbase.p, text.p,
                                                               off.p);
          HIP_CHECK(hipGetLastError());
          if (tail) k_set_u64<<<1, 1, 0, stream>>>(off.p + k, n - nl);
          if (k) {
            const double tb = now_s();
            if (sink && !buf) new_buffer();
            const lcg_status st =
                lcg_build_into(sink ? buf : g, text.p, off.p, (uint32_t)k, &o, stream, nullptr);
            build_s += now_s() - tb;
            if (st != LCG_OK) throw LcgError{st, std::string("chunk ") + std::to_string(chunks) +
                                                     ": " + lcg_last_error()};
            if (sink && device_bytes(buf) >= buffer_bytes) flush();
          }
          strings += k;
          bytes += n - nl;
        }
        ++chunks;
        sync(stream);  // the chunk's host buffer and raw slot are free again
        pipe.put_free(cur);
        cur = next;
        slot ^= 1;
      }
      sync(copy_s);
      if (sink) {
        if (buf) flush();
        sink_to_device(g, stream);
      }
    } catch (...) {
      finish();
      if (sink) {
        if (touched) g->poisoned = true;  // it may hold part of the stream: refused from now on
        try {
          sink_to_device(g, stream);
        } catch (...) {
          g->poisoned = true;
        }
      }
      throw;
    }
    finish();
    if (h_info) {
      h_info[0] = bytes;
      h_info[1] = strings;
      h_info[2] = chunks;
      h_info[3] = (uint64_t)((now_s() - t0) * 1e9);
      h_info[4] = (uint64_t)(wait_s * 1e9);
      h_info[5] = (uint64_t)(build_s * 1e9);
      if (sink) {
        h_info[6] = flushes;
        h_info[7] = (uint64_t)(flush_s * 1e9);
      }
    }
  }
}

}  // namespace

extern "C" {

lcg_status lcg_build_file(lcg_grammar_t g, const char* path, uint64_t chunk_bytes,
                          const lcg_opts* opts, hipStream_t stream, uint64_t* h_info) {
  return guard([&] {
    live(g);
    build_file(g, path, chunk_bytes, opts, stream, h_info, false, 0);
  });
}

lcg_status lcg_build_file_sink(lcg_grammar_t sink, const char* path, uint64_t chunk_bytes,
                               uint64_t buffer_bytes, const lcg_opts* opts, hipStream_t stream,
                               uint64_t* h_info) {
  return guard([&] {
    live(sink);
    build_file(sink, path, chunk_bytes, opts, stream, h_info, true, buffer_bytes);
  });
}

}  // extern "C"
