// The GPU virtualization manager (GVM) run-time of Section 5: owns the only
// device context, the per-rank shared-memory spaces and request/response
// rings, and serves the ranks' requests on the device.
#pragma once

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <future>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "copy_pool.hpp"
#include "device.hpp"
#include "shm.hpp"

namespace gvm {

// First-fit allocator of offsets inside the device arena (the HBM budget).
class Arena {
 public:
  void init(uint64_t bytes);
  bool alloc(uint64_t bytes, uint64_t* off);
  void release(uint64_t off, uint64_t bytes);
  uint64_t total() const { return total_; }
  uint64_t used() const { return used_; }
  // the peak is also read by statistics readers on other threads
  uint64_t peak() const { return peak_.load(std::memory_order_relaxed); }
  void reset_peak() { peak_.store(used_, std::memory_order_relaxed); }
  static uint64_t round(uint64_t bytes) { return (bytes + 4095) / 4096 * 4096; }

 private:
  std::map<uint64_t, uint64_t> free_;  // offset -> bytes
  uint64_t total_ = 0, used_ = 0;
  std::atomic<uint64_t> peak_{0};
};

class Manager {
 public:
  int init(const gvm_config& cfg);
  int shutdown();
  int stats_json(std::string* out);
  void reset_stats();
  // Per-request trace (the last kTraceMax requests since the start or the
  // last reset) as a Chrome trace-event JSON file.
  int trace_dump(const char* path);
  bool running() const { return started_; }

 private:
  struct Queued {
    uint64_t seq;
    uint64_t t_arrive_ns;
    int status;  // GVM_OK, or an error to report when it reaches the head
    Request req;
  };
  struct RankRt {
    bool attached = false;
    int32_t pid = 0;
    std::deque<Queued> queue;
    std::deque<Job*> running;   // on the device or in its copies, in admission order
    bool has_slot = false;
    uint64_t slot_off = 0;
    uint64_t slot_size = 0;
    bool res_valid = false;     // the slot holds the input of (res_kernel, res_n)
    uint64_t last_ticket = 0;   // ticket of the rank's latest admitted request
    uint32_t res_kernel = 0;
    uint64_t res_n = 0;
    uint64_t last_use_ns = 0;
    bool detach_pending = false;
    uint64_t detach_ticket = 0;
  };
  enum Admit { kAdmitted, kWait, kRejected, kNotNow };
  // Requests of one rank in flight at once: one in batch mode; in serving
  // mode a second plain request (no resident flags) may be admitted while
  // the first is still in flight, so that its copy-in overlaps the first's
  // device work (Section 4.2.1, concurrency types (a) to (c), within a rank).
  static constexpr size_t kRankDepth = 2;
  // batch mode: per-rank chains enqueued per service-loop iteration
  static constexpr size_t kLaunchChunk = 4;
  size_t rank_depth_ = kRankDepth;  // GVM_RANK_DEPTH=1 keeps one request per rank (measurement)
  bool rank_can_take(const RankRt& rt) const;

  void service(std::promise<int>* ready);
  bool drain_rings();
  void on_message(int r, const Request& m);
  bool complete_jobs();
  void flush_deferred();           // retire finished batches, refresh the statistics
  bool schedule();
  bool launch_ready();
  bool launch_staged();
  bool forward_pieces(Job* j);
  bool early_idle() const;
  Admit admit(int r, std::vector<Job*>& jobs);
  void respond(int r, uint64_t ticket, uint32_t kernel_id, int status, const Job* j, uint64_t t_submit);
  void release_slot(int r);
  void reap_rank(int r);
  void check_liveness();
  bool any_request_waiting() const;
  int resolve_policy(const std::vector<Job*>& jobs) const;

  gvm_config cfg_{};
  std::string ns_;
  Segment ctl_seg_;
  CtlHeader* ctl_ = nullptr;
  std::vector<std::unique_ptr<Segment>> data_;
  std::unique_ptr<Device> dev_;
  Arena arena_;
  std::vector<RankRt> ranks_;
  CopyEngine copy_;                // shm <-> pinned staging copies
  std::vector<Job*> staged_;       // admitted, waiting for their copy-in
  // batch mode, early copy-in: admitted while a batch runs, copy-in under
  // way, held back until the next request barrier
  std::vector<Job*> early_;
  uint64_t early_oldest_ns_ = 0;   // arrivals of the oldest and the newest of them
  uint64_t early_newest_ns_ = 0;
  std::thread thread_;
  std::atomic<bool> stop_{false};
  bool started_ = false;
  uint64_t seq_ = 0;
  size_t inflight_ = 0;
  bool batch_open_ = false;        // batch mode: a batch is on the device
  uint64_t last_liveness_ns_ = 0;
  std::atomic<bool> reset_pending_{false};
  // stats_json() asks the service thread to retire finished batches first
  std::atomic<bool> flush_req_{false};
  std::mutex flush_mu_;
  std::condition_variable flush_cv_;
  uint64_t flush_done_ = 0;        // guarded by flush_mu_
  std::string open_error_;
  uint64_t spin_ns_ = 200000;      // poll before sleeping once idle
  uint64_t service_cpu_ns() const;  // CPU time of the service thread so far
  void wake_group();
  bool group_wake_ = false;        // a rank asleep on the group doorbell was answered

  // statistics (guarded by stats_mu_)
  std::mutex stats_mu_;
  uint64_t stats_t0_ns_ = 0, stats_cpu0_ns_ = 0;  // wall clock and service CPU time at the last reset
  uint64_t n_done_ = 0, n_err_ = 0, n_batches_ = 0;
  std::vector<double> lat_us_[kNumKernelIds];      // submit -> result posted, per kernel id
  std::vector<double> wait_us_;        // submit -> admitted
  std::vector<double> ring_us_;        // submit -> drained from the rank's ring
  std::vector<double> batch_lag_us_;   // batch mode: last request drained -> batch admitted
  std::vector<double> iter_us_;        // service iterations that retired or launched work
  std::vector<double> iter_done_us_;   // their complete_jobs part
  KernelStats kstats_[kNumKernelIds];
  uint64_t peak_bytes_ = 0;
  // per-request trace records, a ring of the last kTraceMax
  struct TraceRec {
    int32_t rank;
    uint32_t kernel_id;
    int32_t status;
    uint32_t pad;
    uint64_t n, ticket;
    uint64_t t_submit, t_admit, t_launch, t_device, t_done;
  };
  static constexpr size_t kTraceMax = 1u << 20;
  std::vector<TraceRec> trace_;
  size_t trace_next_ = 0;          // next slot of the ring once it is full
  uint64_t n_traced_ = 0;
  std::string timing_json_ = "{}";
};

}  // namespace gvm
