#include "copy_pool.hpp"

#include <emmintrin.h>
#include <sys/resource.h>
#include <sys/syscall.h>
#include <unistd.h>

#include <chrono>
#include <cstdlib>
#include <cstring>

namespace gvm {

namespace {
constexpr size_t kChunk = size_t(4) << 20;
constexpr size_t kStreamMin = size_t(256) << 10;  // smaller copies may stay in cache
constexpr int kWorkerNice = 4;

uint64_t mono_ns() {
  return static_cast<uint64_t>(
      std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch()).count());
}

// Copy with non-temporal 16-byte stores: the destination (pinned staging
// read next by a DMA engine, or a rank's result area) is not read back by
// this core, so the stores skip the read-for-ownership of every line and
// leave the caches to the ranks.  Head and tail up to 16-byte alignment of
// the destination go through memcpy.
void stream_copy(char* dst, const char* src, size_t bytes) {
  size_t head = (16 - (reinterpret_cast<uintptr_t>(dst) & 15)) & 15;
  if (head > bytes) head = bytes;
  memcpy(dst, src, head);
  dst += head;
  src += head;
  bytes -= head;
  const size_t body = bytes & ~size_t(63);
  for (size_t i = 0; i < body; i += 64) {
    const __m128i a = _mm_loadu_si128(reinterpret_cast<const __m128i*>(src + i));
    const __m128i b = _mm_loadu_si128(reinterpret_cast<const __m128i*>(src + i + 16));
    const __m128i c = _mm_loadu_si128(reinterpret_cast<const __m128i*>(src + i + 32));
    const __m128i d = _mm_loadu_si128(reinterpret_cast<const __m128i*>(src + i + 48));
    _mm_stream_si128(reinterpret_cast<__m128i*>(dst + i), a);
    _mm_stream_si128(reinterpret_cast<__m128i*>(dst + i + 16), b);
    _mm_stream_si128(reinterpret_cast<__m128i*>(dst + i + 32), c);
    _mm_stream_si128(reinterpret_cast<__m128i*>(dst + i + 48), d);
  }
  _mm_sfence();  // the streamed lines are globally visible before the chunk is reported done
  memcpy(dst + body, src + body, bytes - body);
}

bool stream_enabled() {
  static const bool on = [] {
    const char* e = getenv("GVM_COPY_NT");
    return !(e && e[0] == '0');
  }();
  return on;
}
}  // namespace

void CopyEngine::copy(char* dst, const char* src, size_t bytes) {
  const uint64_t t0 = mono_ns();
  if (bytes >= kStreamMin && stream_enabled())
    stream_copy(dst, src, bytes);
  else
    memcpy(dst, src, bytes);
  busy_ns_.fetch_add(mono_ns() - t0, std::memory_order_relaxed);
  bytes_.fetch_add(bytes, std::memory_order_relaxed);
}

void CopyEngine::start(int nthreads) {
  stop();
  {
    std::lock_guard<std::mutex> lk(mu_);
    stopping_ = false;
  }
  for (int i = 0; i < nthreads; ++i) threads_.emplace_back([this] { worker(); });
}

void CopyEngine::stop() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    stopping_ = true;
  }
  cv_.notify_all();
  for (auto& t : threads_) t.join();
  threads_.clear();
  // anything still queued is copied here so that no waiter is left behind
  for (auto* q : {&urgent_, &queue_}) {
    for (Chunk& c : *q) {
      copy(c.dst, c.src, c.bytes);
      c.pending->fetch_sub(1, std::memory_order_acq_rel);
    }
    q->clear();
  }
}

void CopyEngine::worker() {
  // A lower scheduling weight than the service thread: when the host is
  // oversubscribed the copies give way to the thread that drains the rings
  // and launches work (raising a thread's nice value needs no privilege).
  (void)setpriority(PRIO_PROCESS, static_cast<id_t>(syscall(SYS_gettid)), kWorkerNice);
  for (;;) {
    Chunk c;
    {
      std::unique_lock<std::mutex> lk(mu_);
      cv_.wait(lk, [&] { return stopping_ || !queue_.empty() || !urgent_.empty(); });
      std::deque<Chunk>& q = urgent_.empty() ? queue_ : urgent_;
      if (q.empty()) return;  // stopping and drained
      c = q.front();
      q.pop_front();
    }
    copy(c.dst, c.src, c.bytes);
    c.pending->fetch_sub(1, std::memory_order_acq_rel);
  }
}

void CopyEngine::submit(void* dst, const void* src, size_t bytes, std::atomic<int>* pending, bool urgent) {
  if (bytes == 0) return;
  if (threads_.empty()) {
    copy(static_cast<char*>(dst), static_cast<const char*>(src), bytes);
    return;
  }
  const size_t n = (bytes + kChunk - 1) / kChunk;
  pending->fetch_add(static_cast<int>(n), std::memory_order_acq_rel);
  {
    std::lock_guard<std::mutex> lk(mu_);
    std::deque<Chunk>& q = urgent ? urgent_ : queue_;
    for (size_t i = 0; i < n; ++i) {
      const size_t off = i * kChunk;
      const size_t len = (off + kChunk <= bytes) ? kChunk : bytes - off;
      q.push_back(Chunk{static_cast<char*>(dst) + off, static_cast<const char*>(src) + off, len, pending});
    }
    if (queue_.size() + urgent_.size() > max_queue_) max_queue_ = queue_.size() + urgent_.size();
  }
  if (n == 1) cv_.notify_one(); else cv_.notify_all();
}

CopyEngine::Stats CopyEngine::stats() {
  Stats s;
  s.bytes = bytes_.load(std::memory_order_relaxed);
  s.busy_ns = busy_ns_.load(std::memory_order_relaxed);
  std::lock_guard<std::mutex> lk(mu_);
  s.max_queue = max_queue_;
  return s;
}

void CopyEngine::reset_stats() {
  bytes_.store(0, std::memory_order_relaxed);
  busy_ns_.store(0, std::memory_order_relaxed);
  std::lock_guard<std::mutex> lk(mu_);
  max_queue_ = 0;
}

}  // namespace gvm
