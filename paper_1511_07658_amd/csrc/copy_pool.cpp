#include "copy_pool.hpp"

#include <immintrin.h>

#include <cstring>

namespace gvm {

namespace {
constexpr size_t kSerialBytes = size_t(2) << 20;  // below this one thread is as fast
constexpr size_t kChunk = size_t(1) << 20;
}  // namespace

void CopyPool::start(int nthreads) {
  stop();
  {
    std::lock_guard<std::mutex> lk(mu_);
    stopping_ = false;
  }
  for (int i = 0; i < nthreads; ++i) threads_.emplace_back([this] { worker(); });
}

void CopyPool::stop() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    stopping_ = true;
  }
  cv_.notify_all();
  for (auto& t : threads_) t.join();
  threads_.clear();
}

void CopyPool::run_chunks(const Job& j) {
  uint64_t cur = cursor_.load(std::memory_order_acquire);
  for (;;) {
    if ((cur >> 32) != j.gen || (cur & 0xffffffffull) >= j.nchunks) return;
    if (!cursor_.compare_exchange_weak(cur, cur + 1, std::memory_order_acq_rel)) continue;
    const size_t c = static_cast<size_t>(cur & 0xffffffffull);
    const size_t off = c * kChunk;
    const size_t len = (off + kChunk <= j.bytes) ? kChunk : j.bytes - off;
    memcpy(j.dst + off, j.src + off, len);
    done_.fetch_add(1, std::memory_order_acq_rel);
    cur = cursor_.load(std::memory_order_acquire);
  }
}

void CopyPool::worker() {
  uint32_t seen = 0;
  for (;;) {
    Job j;
    {
      std::unique_lock<std::mutex> lk(mu_);
      cv_.wait(lk, [&] { return stopping_ || job_.gen != seen; });
      if (stopping_) return;
      j = job_;
      seen = j.gen;
    }
    run_chunks(j);
  }
}

void CopyPool::copy(void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return;
  if (threads_.empty() || bytes < kSerialBytes) {
    memcpy(dst, src, bytes);
    return;
  }
  Job j;
  {
    std::lock_guard<std::mutex> lk(mu_);
    j.dst = static_cast<char*>(dst);
    j.src = static_cast<const char*>(src);
    j.bytes = bytes;
    j.nchunks = (bytes + kChunk - 1) / kChunk;
    j.gen = job_.gen + 1;
    if (j.gen == 0) j.gen = 1;
    done_.store(0, std::memory_order_relaxed);
    cursor_.store(static_cast<uint64_t>(j.gen) << 32, std::memory_order_release);
    job_ = j;
  }
  cv_.notify_all();
  run_chunks(j);
  while (done_.load(std::memory_order_acquire) < j.nchunks) _mm_pause();
}

}  // namespace gvm
