#include "copy_pool.hpp"

#include <cstring>

namespace gvm {

namespace {
constexpr size_t kChunk = size_t(4) << 20;
}  // namespace

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
  for (Chunk& c : queue_) {
    memcpy(c.dst, c.src, c.bytes);
    c.pending->fetch_sub(1, std::memory_order_acq_rel);
  }
  queue_.clear();
}

void CopyEngine::worker() {
  for (;;) {
    Chunk c;
    {
      std::unique_lock<std::mutex> lk(mu_);
      cv_.wait(lk, [&] { return stopping_ || !queue_.empty(); });
      if (queue_.empty()) return;  // stopping and drained
      c = queue_.front();
      queue_.pop_front();
    }
    memcpy(c.dst, c.src, c.bytes);
    c.pending->fetch_sub(1, std::memory_order_acq_rel);
  }
}

void CopyEngine::submit(void* dst, const void* src, size_t bytes, std::atomic<int>* pending) {
  if (bytes == 0) return;
  if (threads_.empty()) {
    memcpy(dst, src, bytes);
    return;
  }
  const size_t n = (bytes + kChunk - 1) / kChunk;
  pending->fetch_add(static_cast<int>(n), std::memory_order_acq_rel);
  {
    std::lock_guard<std::mutex> lk(mu_);
    for (size_t i = 0; i < n; ++i) {
      const size_t off = i * kChunk;
      const size_t len = (off + kChunk <= bytes) ? kChunk : bytes - off;
      queue_.push_back(Chunk{static_cast<char*>(dst) + off, static_cast<const char*>(src) + off, len, pending});
    }
  }
  if (n == 1) cv_.notify_one(); else cv_.notify_all();
}

}  // namespace gvm
