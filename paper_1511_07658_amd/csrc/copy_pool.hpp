// Host memory copies between the ranks' shared-memory spaces and the
// manager's pinned staging, done asynchronously by worker threads so that
// the manager's service thread never waits for them.  One thread moves
// roughly 10 GB/s; the PCIe link takes about 57 GB/s per direction.
#pragma once

#include <atomic>
#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

namespace gvm {

class CopyEngine {
 public:
  ~CopyEngine() { stop(); }
  void start(int nthreads);
  void stop();
  // Queue a copy of `bytes` from src to dst, split into chunks that run on
  // the workers in parallel.  `pending` is incremented by the number of
  // chunks now and decremented as each chunk lands; the copy is complete
  // when it reads 0 (acquire).  Without workers the copy runs inline.
  // `urgent` chunks (a small request's) go ahead of every queued ordinary
  // chunk; each of the two queues is first-in first-out.
  void submit(void* dst, const void* src, size_t bytes, std::atomic<int>* pending, bool urgent = false);
  int threads() const { return static_cast<int>(threads_.size()); }

  // Bytes moved, summed time the workers spent copying, and the deepest
  // the chunk queue has been, since the start or the last reset.
  struct Stats {
    uint64_t bytes = 0, busy_ns = 0;
    size_t max_queue = 0;
  };
  Stats stats();
  void reset_stats();

 private:
  struct Chunk {
    char* dst;
    const char* src;
    size_t bytes;
    std::atomic<int>* pending;
  };
  void worker();
  void copy(char* dst, const char* src, size_t bytes);

  std::vector<std::thread> threads_;
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<Chunk> queue_;
  std::deque<Chunk> urgent_;
  bool stopping_ = false;
  size_t max_queue_ = 0;
  std::atomic<uint64_t> bytes_{0}, busy_ns_{0};
};

}  // namespace gvm
