// Loopback device: runs the manager's host protocol without a GPU.
//
// It computes NO kernel.  Each job's output region receives the first
// out_bytes of the job's input bytes (zero-padded), so that host-logic tests
// can check that every rank gets its own data back through shared memory,
// staging and the "device" buffer.  It is selected only by an explicit
// GVM_BACKEND_LOOPBACK in the configuration and is never a fallback for the
// HIP backend.
#include <sys/mman.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstring>

#include "device.hpp"

namespace gvm {

void request_work(int kernel_id, uint64_t n, double* flop, double* bytes) {
  const double dn = static_cast<double>(n);
  switch (kernel_id) {
    case GVM_K_VECADD:
    case GVM_K_VECMUL:
      *flop = dn;
      *bytes = 12.0 * dn;
      return;
    case GVM_K_BLACKSCHOLES:
      *flop = 0.0;
      *bytes = 20.0 * dn;
      return;
    case GVM_K_SGEMM:
      *flop = 2.0 * dn * dn * dn;
      *bytes = 12.0 * dn * dn;
      return;
    case GVM_K_EP:
      *flop = 0.0;  // integer and transcendental work; counted in pairs by the caller
      *bytes = 16.0 + 8.0 * kEpWords;
      return;
    default:
      *flop = 0.0;
      *bytes = 0.0;
  }
}

double estimate_device_us(int kernel_id, uint64_t n) {
  if (kernel_id == GVM_K_EP) return static_cast<double>(n) / 120e9 * 1e6;
  double flop = 0.0, bytes = 0.0;
  request_work(kernel_id, n, &flop, &bytes);
  const double t_mfma = kernel_id == GVM_K_SGEMM ? flop / 110e12 : 0.0;
  return std::max(t_mfma, bytes / 5e12) * 1e6;
}

namespace {

class LoopbackDevice final : public Device {
 public:
  ~LoopbackDevice() override { close(); }

  int open(const gvm_config& cfg) override {
    cfg_ = cfg;
    arena_bytes_ = cfg.hbm_budget_bytes;
    void* p = mmap(nullptr, arena_bytes_, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
    if (p == MAP_FAILED) return fail(GVM_ENOMEM, "loopback arena of %llu bytes", (unsigned long long)arena_bytes_);
    arena_ = static_cast<uint8_t*>(p);
    staging_bytes_ = align_up((cfg.staging_bytes ? cfg.staging_bytes : cfg.shm_bytes_per_rank) + 2 * kAlign, 4096);
    staging_.assign(cfg.nranks, nullptr);
    return GVM_OK;
  }

  uint8_t* arena() override { return arena_; }

  uint8_t* staging(int rank) override {
    if (rank < 0 || rank >= static_cast<int>(staging_.size())) return nullptr;
    if (!staging_[rank]) {
      void* p = mmap(nullptr, staging_bytes_, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
      if (p == MAP_FAILED) return nullptr;
      staging_[rank] = static_cast<uint8_t*>(p);
    }
    return staging_[rank];
  }

  int launch(std::vector<Job*>& jobs, int policy) override {
    if (policy >= 0 && policy < 4) policy_launches_[policy].fetch_add(1, std::memory_order_relaxed);
    const uint64_t t_batch = now_ns();
    for (Job* j : jobs) {
      j->t_launch_ns = now_ns();
      if (j->copy_in && !j->pieces) timed_copy(0, j->slot, j->pin, j->lay.in_bytes);
      const uint64_t o = slot_out_offset(j->lay);
      const uint64_t keep = j->lay.in_bytes < j->lay.out_bytes ? j->lay.in_bytes : j->lay.out_bytes;
      memmove(j->slot + o, j->slot, keep);
      memset(j->slot + o + keep, 0, j->lay.out_bytes - keep);
      if (j->copy_out) timed_copy(1, j->pin + o, j->slot + o, j->lay.out_bytes);
      KernelStats& ks = stats_[j->req.kernel_id < kNumKernelIds ? j->req.kernel_id : 0];
      ks.launches += 1;
      ks.requests += 1;
      double f, b;
      request_work(static_cast<int>(j->req.kernel_id), j->req.n, &f, &b);
      ks.work_flop += f;
      ks.work_bytes += b;
    }
    if (cfg_.batch_timing) batch_us_.push_back((now_ns() - t_batch) * 1e-3);
    counted_ = true;
    return GVM_OK;
  }

  // Counters are updated at launch; report them at the next flush.
  bool flush_retired() override {
    const bool c = counted_;
    counted_ = false;
    return c;
  }

  int stream_in(Job* j, uint64_t off, uint64_t bytes) override {
    memcpy(j->slot + off, j->pin + off, bytes);
    return GVM_OK;
  }

  int out_pieces_done(Job* j) override { return static_cast<int>(j->out_pieces); }

  int query(Job* j) override {
    if (!j->t_device_ns) j->t_device_ns = now_ns();
    return 1;
  }

  void finish(Job*) override {}

  void drain() override {}

  void close() override {
    if (arena_) munmap(arena_, arena_bytes_);
    arena_ = nullptr;
    for (uint8_t* p : staging_)
      if (p) munmap(p, staging_bytes_);
    staging_.clear();
  }

  const KernelStats* kernel_stats() const override { return stats_; }
  void reset_stats() override {
    for (auto& s : stats_) s = KernelStats{};
    batch_us_.clear();
    for (int d = 0; d < 2; ++d) copy_ms_[d] = copy_bytes_[d] = 0.0, copy_n_[d] = 0;
  }
  // launch calls by the policy the manager chose (host-logic tests check it)
  std::string describe() const override {
    return "{\"backend\":\"loopback\",\"policy_launches\":{\"ps1\":" +
           std::to_string(policy_launches_[GVM_POLICY_PS1].load()) +
           ",\"ps2\":" + std::to_string(policy_launches_[GVM_POLICY_PS2].load()) +
           ",\"grouped\":" + std::to_string(policy_launches_[GVM_POLICY_GROUPED].load()) + "}}";
  }

  // Same layout as the HIP backend's, on the host clock (batch_timing).
  std::string timing_json() const override {
    if (!cfg_.batch_timing) return "{}";
    std::string s = "{\"batch_device_us\":[";
    const size_t first = batch_us_.size() > 512 ? batch_us_.size() - 512 : 0;
    for (size_t i = first; i < batch_us_.size(); ++i) {
      if (i > first) s += ",";
      s += std::to_string(batch_us_[i]);
    }
    char buf[256];
    snprintf(buf, sizeof(buf), "],\"h2d\":{\"count\":%llu,\"ms\":%.6f,\"bytes\":%.0f},\"d2h\":{\"count\":%llu,\"ms\":%.6f,\"bytes\":%.0f}}",
             (unsigned long long)copy_n_[0], copy_ms_[0], copy_bytes_[0], (unsigned long long)copy_n_[1], copy_ms_[1],
             copy_bytes_[1]);
    return s + buf;
  }

 private:
  void timed_copy(int dir, void* dst, const void* src, uint64_t bytes) {
    const uint64_t t0 = now_ns();
    memcpy(dst, src, bytes);
    if (!cfg_.batch_timing) return;
    copy_ms_[dir] += (now_ns() - t0) * 1e-6;
    copy_bytes_[dir] += static_cast<double>(bytes);
    copy_n_[dir] += 1;
  }

  gvm_config cfg_{};
  bool counted_ = false;            // counters changed since the last flush
  std::vector<double> batch_us_;
  double copy_ms_[2] = {0, 0}, copy_bytes_[2] = {0, 0};
  uint64_t copy_n_[2] = {0, 0};
  uint8_t* arena_ = nullptr;
  uint64_t arena_bytes_ = 0;
  std::vector<uint8_t*> staging_;
  uint64_t staging_bytes_ = 0;
  KernelStats stats_[kNumKernelIds];
  std::atomic<uint64_t> policy_launches_[4] = {};
};

}  // namespace

std::unique_ptr<Device> make_loopback_device() { return std::unique_ptr<Device>(new LoopbackDevice()); }

}  // namespace gvm
