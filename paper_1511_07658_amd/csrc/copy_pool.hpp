// Host memory copies between the ranks' shared-memory spaces and the
// manager's pinned staging, split over a few threads: one thread moves
// roughly 10 GB/s, the PCIe link takes about 57 GB/s per direction.
#pragma once

#include <atomic>
#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <mutex>
#include <thread>
#include <vector>

namespace gvm {

class CopyPool {
 public:
  ~CopyPool() { stop(); }
  void start(int nthreads);
  void stop();
  // Copy `bytes` from src to dst using the pool and the calling thread;
  // returns when the copy is complete.  One caller at a time.
  void copy(void* dst, const void* src, size_t bytes);

 private:
  struct Job {
    char* dst;
    const char* src;
    size_t bytes;
    size_t nchunks;
    uint32_t gen;
  };
  void worker();
  void run_chunks(const Job& j);

  std::vector<std::thread> threads_;
  std::mutex mu_;
  std::condition_variable cv_;
  Job job_{};
  bool stopping_ = false;
  // (generation << 32) | next chunk: a worker holding a stale job can never
  // claim a chunk of a newer one
  std::atomic<uint64_t> cursor_{0};
  std::atomic<uint64_t> done_{0};
};

}  // namespace gvm
