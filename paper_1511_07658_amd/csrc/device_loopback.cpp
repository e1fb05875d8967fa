// Loopback device: runs the manager's host protocol without a GPU.
//
// It computes NO kernel.  Each job's output region receives the first
// out_bytes of the job's input bytes (zero-padded), so that host-logic tests
// can check that every rank gets its own data back through shared memory,
// staging and the "device" buffer.  It is selected only by an explicit
// GVM_BACKEND_LOOPBACK in the configuration and is never a fallback for the
// HIP backend.
#include <sys/mman.h>

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
    default:
      *flop = 0.0;
      *bytes = 0.0;
  }
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

  int launch(std::vector<Job*>& jobs, int /*policy*/) override {
    for (Job* j : jobs) {
      j->t_launch_ns = now_ns();
      if (j->copy_in) memcpy(j->slot, j->pin, j->lay.in_bytes);
      const uint64_t o = slot_out_offset(j->lay);
      const uint64_t keep = j->lay.in_bytes < j->lay.out_bytes ? j->lay.in_bytes : j->lay.out_bytes;
      memmove(j->slot + o, j->slot, keep);
      memset(j->slot + o + keep, 0, j->lay.out_bytes - keep);
      if (j->copy_out) memcpy(j->pin + o, j->slot + o, j->lay.out_bytes);
      KernelStats& ks = stats_[j->req.kernel_id < 5 ? j->req.kernel_id : 0];
      ks.launches += 1;
      ks.requests += 1;
      double f, b;
      request_work(static_cast<int>(j->req.kernel_id), j->req.n, &f, &b);
      ks.work_flop += f;
      ks.work_bytes += b;
    }
    return GVM_OK;
  }

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
  }
  std::string describe() const override { return "{\"backend\":\"loopback\"}"; }

 private:
  gvm_config cfg_{};
  uint8_t* arena_ = nullptr;
  uint64_t arena_bytes_ = 0;
  std::vector<uint8_t*> staging_;
  uint64_t staging_bytes_ = 0;
  KernelStats stats_[5];
};

}  // namespace

std::unique_ptr<Device> make_loopback_device() { return std::unique_ptr<Device>(new LoopbackDevice()); }

}  // namespace gvm
